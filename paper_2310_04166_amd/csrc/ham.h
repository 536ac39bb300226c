// The compiled Hamiltonian: flip-grouped Pauli tables on the host and, after
// first use, on the device.
#pragma once

#include <vector>

#include "common.h"

struct nqs_ham {
  int n = 0;        // spatial orbitals
  int N = 0;        // spin-orbitals (qubits)
  int n_alpha = 0, n_beta = 0;
  double e_core = 0.0;
  std::vector<uint64_t> flip;   // [G] ascending; flip[0] == 0 (diagonal group)
  std::vector<int64_t> off;     // [G+1]
  std::vector<uint64_t> zmask;  // [T]
  std::vector<double> coef;     // [T]

  // device copies (uploaded on first use, on the device current at that time)
  int device = -1;
  nqs::DevBuf d_flip, d_off, d_zmask, d_coef;
  // local_energy workspaces
  nqs::DevBuf w_cnt, w_off, w_xp, w_h, w_owner, w_la, w_ph, w_diag, w_lax, w_phx;
  nqs::DevBuf w_keys, w_ukeys, w_u32, w_tmp;   // distinct-x' workspaces
  nqs::DevBuf w_lp2;                           // their amplitudes as fp32 pairs (bf16 models)
  nqs::DevBuf w_scan;                          // tile totals of the multi-block scan
  int64_t last_distinct = 0;                   // distinct x' of the last local_energy call
  int64_t last_pairs = 0;                      // (x, x') pairs of the last local_energy call

  void upload();
};

namespace nqs {
// Device side of the bit work (eloc.hip).
void launch_count_pairs(const nqs_ham &H, const uint64_t *x, int64_t n, int64_t *cnt,
                        hipStream_t s);
void launch_emit_pairs(const nqs_ham &H, const uint64_t *x, int64_t n, const int64_t *off,
                       uint64_t *xp, double *hval, int32_t *owner, double *hdiag,
                       int64_t owner_base, hipStream_t s);
// Exclusive scan of n int64 into out[0..n] (out[n] = total).  The workspace
// (scan_workspace_entries(n) int64, none for n <= 8192) is either a raw device
// array or a buffer of the calling handle, grown as needed.
int64_t scan_workspace_entries(int64_t n);
void launch_exclusive_scan(const int64_t *in, int64_t *out, int64_t n, hipStream_t s,
                           int64_t *tile_ws);
void launch_exclusive_scan(const int64_t *in, int64_t *out, int64_t n, hipStream_t s,
                           DevBuf &ws);
}  // namespace nqs
