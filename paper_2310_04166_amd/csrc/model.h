// The amplitude model handle: dimensions, parameter layout, device buffers.
#pragma once

#include <vector>

#include "common.h"

// One molecule (symmetry sector) served by a model: its token count,
// electrons, number of masked levels, optional Z2 symmetries (qubit masks) and
// where its physical-children table starts in the model's concatenated tables
// ([(n+1)^3 2^nz2] 4-bit masks each, the last index the prefix's Z2 parities).
// A sector given by general additive symmetries (general = 1) instead keeps at
// phys_off an int32 table: n + 1 level offsets, then the four children of every
// physical prefix state (the child's state index in the next level, -1 when
// the child is unphysical).
struct nqs_sector_info {
  int32_t n, na, nb, mask_levels;
  int64_t phys_off;
  int32_t nz2, general;
  uint64_t z2[4];
};

namespace nqs {
// A model that serves several molecules reads the molecule of a configuration
// word from bits 58..63 (its occupation bits stay below); a model with one
// sector uses the words as they are.
constexpr int kTagShift = 58;
constexpr uint64_t kOccMask = (uint64_t(1) << kTagShift) - 1;

struct Sectors {                      // device view handed to kernels
  const nqs_sector_info *info;
  const uint8_t *phys;
  int tagged, count;                  // count = number of sectors in info
};

// A word whose molecule index is out of range reads molecule 0's sector (its
// results are meaningless, but no access leaves the tables).
__device__ inline const nqs_sector_info &sector_of(const Sectors &S, uint64_t x) {
  const int i = S.tagged ? int(x >> kTagShift) : 0;
  return S.info[i < S.count ? i : 0];
}
__device__ inline uint64_t occupation(const Sectors &S, uint64_t x) {
  return S.tagged ? (x & kOccMask) : x;
}
// 4-bit set of physical tokens at level t after a alpha / b beta electrons;
// occ holds the occupation bits of the prefix (bits of later tokens ignored),
// whose Z2 parities select the table entry
__device__ inline int phys_mask(const Sectors &S, const nqs_sector_info &si, int t, int a, int b,
                                uint64_t occ) {
  if (si.general) {
    // the prefix's state: walk its tokens through the children table
    const int32_t *g = reinterpret_cast<const int32_t *>(S.phys + si.phys_off);
    const int32_t *kids = g + si.n + 1;
    int id = 0;
    for (int p = 0; p < t && id >= 0; ++p) id = kids[4 * (g[p] + id) + int((occ >> (2 * p)) & 3ull)];
    if (id < 0) return 0;
    const int32_t *c = kids + 4 * (g[t] + id);
    return int(c[0] >= 0) | (int(c[1] >= 0) << 1) | (int(c[2] >= 0) << 2) | (int(c[3] >= 0) << 3);
  }
  const uint64_t below = t >= 32 ? ~0ull : ((1ull << (2 * t)) - 1);
  int par = 0;
  for (int j = 0; j < si.nz2; ++j) par |= (__popcll(occ & below & si.z2[j]) & 1) << j;
  return S.phys[si.phys_off + ((int64_t(t) * (si.n + 1) + a) * (si.n + 1) + b) * (1 << si.nz2) + par];
}
}  // namespace nqs

struct nqs_model {
  int kind = 0, precision = 0, strategy = 0, dlev = 0;
  int n = 0, na = 0, nb = 0;          // tokens, sector
  int d = 0, L = 0, H = 0, F = 0, PH = 0;  // transformer
  int hid = 0;                        // MLP
  int mask_levels = 0;                // positions p < mask_levels use masked conditionals
  int64_t P = 0;                      // parameter count
  std::vector<int64_t> off;           // parameter offsets, see param_index()
  std::vector<uint8_t> phys_host;     // concatenated physical-child tables of the sectors
  std::vector<nqs_sector_info> sec_host;  // one entry, or one per molecule when tagged
  int tagged = 0;                     // configuration words carry the molecule index
  uint64_t sec_gen = 0;               // bumped whenever the sector tables are reinstalled
  std::vector<uint64_t> z2;           // Z2 symmetries of the model's own sector (qubit masks)
  std::vector<int32_t> gen_eig, gen_target;  // general additive symmetries (amp_model_set_symmetries)
  int gen_nadd = 0;
  std::vector<int64_t> nade_off;      // per-qubit ansatz: offsets of its derived blocks in packed
  uint32_t z2_target = 0;             // their parities in the target sector (bit j)
  int64_t act_budget = int64_t(1) << 30;  // bytes of activations per layer-by-layer chunk

  nqs::DevBuf master;                 // canonical parameters (double in FP64, float otherwise)
  nqs::DevBuf phys;                   // device copy of phys_host
  nqs::DevBuf sec;                    // device copy of sec_host
  nqs::DevBuf packed;                 // bf16 weight fragments of the fused kernel
  nqs::DevBuf packed_vec;             // permuted fp32 vectors of the fused kernel
  nqs::DevBuf nade_frag, nade_vec;    // per-qubit ansatz, bf16: weight fragments, fp32 vectors
  std::vector<int32_t> nade_fo;       // first fragment set of each qubit in nade_frag
  bool packed_valid = false;
  int64_t tab_M = 0;                  // TABLE: basis size
  nqs::DevBuf tab_basis, tab_tkeys, tab_order, tab_cum;  // TABLE: see table.hip
  nqs::DevBuf ws, ws2, grad_acc, part, logit_buf, la_tmp, ph_tmp;  // workspaces
  nqs::DevBuf s_pre[2], s_cnt[2], s_child, s_flag, s_off, s_cond, s_lost;  // sampler
  nqs::DevBuf s_scan;                 // sampler: tile totals of the multi-block scan
  nqs::DevBuf s_early;                // sampler: every short prefix and its conditionals
  int prefix_share = 1;               // bf16 transformer: prefix-shared evaluation of batches
  int tail_tree = 1;                  // local energy: the tree tail where the sector allows it
  int64_t tree_rows_q = 0, tree_rows_q1 = 0;  // distinct prefixes evaluated by the tree tail
  int mixed_backward = 1;             // bf16 transformer: backward on split-bf16 MFMA products
  nqs::DevBuf mx_w;                   // their weight images
  nqs::DevBuf pf_tab, pf_list, pf_logp, pf_kv, pf_scan;  // its prefix table, keys and values
  nqs::DevBuf pf3_ws, pf3_logp, pf3_kv;  // three levels: bookkeeping, middle-level entries

  bool fp64() const { return precision == NQS_FP64; }
  nqs::Sectors sectors() const {
    return {sec.as<nqs_sector_info>(), phys.as<uint8_t>(), tagged, int(sec_host.size())};
  }
  size_t elem() const { return fp64() ? 8 : 4; }
};

namespace nqs {

// Index of a named tensor in nqs_model::off (transformer layout).
enum TfParam : int {
  TF_TOK = 0, TF_POS = 1,
  // per layer l: base 2 + 12 l + k
  TF_LN1G = 0, TF_LN1B, TF_WQKV, TF_BQKV, TF_WO, TF_BO, TF_LN2G, TF_LN2B, TF_W1, TF_B1, TF_W2, TF_B2,
};
inline int tf_layer(int l, int k) { return 2 + 12 * l + k; }
// after the layers: base 2 + 12 L + k
enum TfTail : int { TF_LNFG = 0, TF_LNFB, TF_WHEAD, TF_BHEAD, TF_LBIAS, TF_PW1, TF_PB1, TF_PW2,
                    TF_PB2, TF_PW3, TF_PB3, TF_NTAIL };
inline int tf_tail(int L, int k) { return 2 + 12 * L + k; }
// MLP: per position p: 6 p + k
enum MlpParam : int { MLP_W1 = 0, MLP_B1, MLP_W2, MLP_B2, MLP_W3, MLP_B3 };

// Forward of the layer-by-layer path.  logits (optional, [B*n*4] in T) keeps
// the head outputs for the sampler; logabs / phase (optional, double).
void model_forward(nqs_model &m, const uint64_t *x, int64_t B, double *logabs, double *phase,
                   void *logits, hipStream_t s);
// Conditional logits of token p for B prefixes (tokens >= p ignored), as
// double [B*4] (host-order: node-major).
void model_cond_logits(nqs_model &m, const uint64_t *prefix, int64_t B, int p, double *out4,
                       hipStream_t s);
void model_backward(nqs_model &m, const uint64_t *x, int64_t B, const double *gl,
                    const double *gp, void *grad, hipStream_t s);
// Fused bf16 forward (tf_fused.hip).
int64_t model_chunk(const nqs_model &m, bool bwd);
// Launch shape of the fused kernel: chunks of 2 * pairs configurations per
// wave step, `blocks` blocks of four waves striding over the chunks (0 = the
// default: one chunk per wave, chunk size from the batch size).
struct FusedTile {
  int pairs = 0, blocks = 0;
};
// With `count` (a device pointer) the kernel reads the number of
// configurations from the device and B is only the capacity of x / outputs;
// such a launch has a fixed grid and can be captured in a graph.
void fused_forward(nqs_model &m, const uint64_t *x, int64_t B, double *logabs, double *phase,
                   double *cond_out, int cond_p, hipStream_t s, const int64_t *count = nullptr,
                   FusedTile tile = FusedTile{});
void fused_pack(nqs_model &m, hipStream_t s);
// per-qubit ansatz: block matrices of the complex layers from the canonical parameters
void nade_pack(nqs_model &m, hipStream_t s);
// per-qubit ansatz in bf16 (nade_fused.hip): fragments from the fp32 block
// matrices of nade_pack, and the fused forward (log|psi|, phase, or the
// sampler's token log-probabilities of token cond_p)
bool nade_fused_supported(const nqs_model &m);
void nade_fused_pack(nqs_model &m, hipStream_t s);
void nade_fused_forward(nqs_model &m, const uint64_t *x, int64_t B, double *logabs,
                        double *phase, double *cond_out, int cond_p, hipStream_t s,
                        const int64_t *count = nullptr);
// Kernel timing of the fused kernels (nqs_timing_*): whether it is on, and a
// record measured by a caller (events inside a captured graph).
bool timing_on();
void timing_add(float ms, int64_t configs, int mode = 0);
// an event recorded on s when timing is on and the launch has a host-side size
// (count == nullptr), else null; timing_end records the launch between the two
hipEvent_t timing_begin(hipStream_t s, const int64_t *count);
void timing_end(hipEvent_t start, hipStream_t s, int64_t configs, int mode = -1);
bool fused_supported(const nqs_model &m);
// Prefix-shared bf16 forward (log|psi| and phase) for 8 < n <= 16 tokens of an
// untagged model with prefix sharing on: positions 0..7 once per distinct
// 8-token prefix of x, positions 8..15 per configuration (tf_fused.hip).
bool fused_shared_supported(const nqs_model &m);
void fused_forward_shared(nqs_model &m, const uint64_t *x, int64_t B, double *logabs,
                          double *phase, hipStream_t s);
// 2 or 3 (13..16 tokens) levels of the shared forward, 0 if it does not apply.
// Three levels: positions 0..7 per 8-token prefix, 8 .. pm-1 per pm-token
// prefix, pm .. pm+3 per configuration; x must be sorted by those prefixes
// (dedupe_pairs with 2 pm bits).
int fused_shared_levels(const nqs_model &m);
// The middle split pm: n - 5 when the sector fixes the last token (14..16
// tokens; that position's conditional is then a membership test), else n - 4.
int fused_shared_pm(const nqs_model &m);
// Whether every sector masks every level and leaves at most one token at its
// last position (whose conditional is then 1 for that token).
bool last_token_fixed(const nqs_model &m);
// Three levels with the tree tail (13..15 tokens, the sector fixes the last
// token, tail_tree on): positions 8 .. n-4 once per (n-4)-token prefix, n-3
// once per (n-3)-token prefix and n-2 once per (n-2)-token prefix, three of
// the latter with their parent in a slot of four rows; x must be sorted by
// tokens (dedupe_pairs with pm = -1).
bool fused_tree(const nqs_model &m);
void fused_forward_tree(nqs_model &m, const uint64_t *x, int64_t B, double *logabs,
                        double *phase, hipStream_t s);
void fused_forward_shared3(nqs_model &m, const uint64_t *x, int64_t B, double *logabs,
                           double *phase, hipStream_t s);
// explicit psi over a basis (table.hip): install the basis (host, ascending),
// rebuild the prefix sums of |psi|^2 from the master parameters, forward,
// conditional logits of token p for the sampler, backward into double acc[2M]
void table_install(nqs_model &m, const uint64_t *basis, int64_t M);
void table_pack(nqs_model &m, hipStream_t s);
void table_forward(nqs_model &m, const uint64_t *x, int64_t B, double *logabs, double *phase,
                   hipStream_t s);
void table_cond_logits(nqs_model &m, const uint64_t *prefix, int64_t B, int p, double *out4,
                       hipStream_t s);
void table_backward(nqs_model &m, const uint64_t *x, int64_t B, const double *gl,
                    const double *gp, double *acc, hipStream_t s);

}  // namespace nqs
