// Fused bf16 transformer forward on MFMA (placeholder until the kernel lands).
#include "model.h"

namespace nqs {

bool fused_supported(const nqs_model &) { return false; }

void fused_pack(nqs_model &, hipStream_t) {
  throw Error(NQS_EUNSUPPORTED, "bf16 fused forward not available");
}

void fused_forward(nqs_model &, const uint64_t *, int64_t, double *, double *, double *, int,
                   hipStream_t) {
  throw Error(NQS_EUNSUPPORTED, "bf16 fused forward not available");
}

}  // namespace nqs
