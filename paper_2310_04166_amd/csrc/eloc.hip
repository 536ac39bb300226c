// Local-energy bit work and the counts-weighted reducer (paper: "Variational
// Monte Carlo": local-energy, energy-estimator and gradient equations).
//
// One 64-lane wavefront owns one sampled configuration x and sweeps the flip
// groups of the compiled Hamiltonian 64 at a time.  For each group f the lane
// forms x' = x ^ f and keeps it when x' has the alpha and beta electron counts
// of x itself (popcounts of the even and odd bits): H conserves both, so these
// are exactly the structurally connected x' (for x in the Hamiltonian's own
// sector, that sector; for a model whose sector is defined by other additive
// quantum numbers, x's own (N_alpha, N_beta) block).  A wave ballot and a
// popcount of the lanes below give each kept pair its output slot, so pairs
// come out in group order without atomics.  Each kept group's Pauli terms,
// coef * (-1)^popcount(x & zmask), are then summed in double, in term order.
#include "ham.h"

namespace nqs {
namespace {

constexpr uint64_t kAlphaBits = 0x5555555555555555ull;
constexpr uint64_t kBetaBits = 0xAAAAAAAAAAAAAAAAull;
constexpr int kWave = 64;
constexpr int kWavesPerBlock = 4;

__device__ inline bool in_sector(uint64_t xp, int na, int nb) {
  return __popcll(xp & kAlphaBits) == na && __popcll(xp & kBetaBits) == nb;
}

// Sum of one flip group's Pauli terms in term order, four loads in flight.
__device__ inline double group_value(uint64_t x, int64_t t0, int64_t t1, const uint64_t *zmask,
                                     const double *coef) {
  double h = 0.0;
  int64_t t = t0;
  for (; t + 4 <= t1; t += 4) {
    double c[4];
    uint64_t z[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      c[u] = coef[t + u];
      z[u] = zmask[t + u];
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) h += (__popcll(x & z[u]) & 1) ? -c[u] : c[u];
  }
  for (; t < t1; ++t) {
    const double c = coef[t];
    h += (__popcll(x & zmask[t]) & 1) ? -c : c;
  }
  return h;
}

// Order visible to the other lanes of the wave (LDS list below).
__device__ inline void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

struct PendPair {
  int64_t slot;   // output slot of a kept pair
  int64_t g;      // its flip group
};

__global__ void __launch_bounds__(256) count_pairs_kernel(
    const uint64_t *__restrict__ x, int64_t n, const uint64_t *__restrict__ flip, int64_t G,
    int64_t *__restrict__ cnt) {
  const int lane = threadIdx.x % kWave;
  const int64_t i = int64_t(blockIdx.x) * kWavesPerBlock + threadIdx.x / kWave;
  if (i >= n) return;
  const uint64_t xi = x[i];
  const int na = __popcll(xi & kAlphaBits), nb = __popcll(xi & kBetaBits);
  int64_t c = 0;
  for (int64_t g0 = 1; g0 < G; g0 += kWave) {
    const int64_t g = g0 + lane;
    const bool keep = g < G && in_sector(xi ^ flip[g], na, nb);
    c += __popcll(__ballot(keep));
  }
  if (lane == 0) cnt[i] = c;
}

// Kept pairs are written (x', owner) as they are found, and their groups are
// listed in LDS; the Pauli sums are then taken 64 groups at a time with every
// lane busy (most groups fail the sector test, so summing where they are found
// would leave most lanes idle through the term loop).
__global__ void __launch_bounds__(256) emit_pairs_kernel(
    const uint64_t *__restrict__ x, int64_t n, const uint64_t *__restrict__ flip,
    const int64_t *__restrict__ goff, const uint64_t *__restrict__ zmask,
    const double *__restrict__ coef, int64_t G, const int64_t *__restrict__ off,
    uint64_t *__restrict__ xp, double *__restrict__ hval, int32_t *__restrict__ owner,
    double *__restrict__ hdiag, int64_t owner_base) {
  __shared__ PendPair pend_all[kWavesPerBlock][2 * kWave];
  const int lane = threadIdx.x % kWave;
  PendPair *pend = pend_all[threadIdx.x / kWave];
  const int64_t i = int64_t(blockIdx.x) * kWavesPerBlock + threadIdx.x / kWave;
  if (i >= n) return;   // uniform over the wave; no block barrier follows
  const uint64_t xi = x[i];
  const int na = __popcll(xi & kAlphaBits), nb = __popcll(xi & kBetaBits);
  const uint64_t below = (lane == 0) ? 0ull : (~0ull >> (kWave - lane));
  int64_t base = off[i] - off[0];
  int npend = 0;
  auto handle = [&](int count) {
    if (lane < count) {
      const PendPair e = pend[lane];
      hval[e.slot] = group_value(xi, goff[e.g], goff[e.g + 1], zmask, coef);
    }
  };
  for (int64_t g0 = 1; g0 < G; g0 += kWave) {
    const int64_t g = g0 + lane;
    const uint64_t f = (g < G) ? flip[g] : 0ull;
    const bool keep = g < G && in_sector(xi ^ f, na, nb);
    const uint64_t mask = __ballot(keep);
    const int rank = __popcll(mask & below);
    if (keep) {
      const int64_t slot = base + rank;
      if (xp) xp[slot] = xi ^ f;
      if (owner) owner[slot] = int32_t(owner_base + i);
      if (hval) pend[npend + rank] = PendPair{slot, g};
    }
    base += __popcll(mask);
    if (!hval) continue;
    npend += __popcll(mask);
    wave_sync();
    if (npend >= kWave) {
      handle(kWave);
      // move the overflow (fewer than 64 entries) to the front of the list
      PendPair tail{};
      if (lane < npend - kWave) tail = pend[kWave + lane];
      wave_sync();
      if (lane < npend - kWave) pend[lane] = tail;
      npend -= kWave;
      wave_sync();
    }
  }
  if (hval) handle(npend);
  if (hdiag) {
    // diagonal group: lanes split its terms, then a fixed-order wave reduction
    double h = 0.0;
    for (int64_t t = goff[0] + lane; t < goff[1]; t += kWave) {
      const double c = coef[t];
      h += (__popcll(xi & zmask[t]) & 1) ? -c : c;
    }
    for (int s = kWave / 2; s > 0; s >>= 1) h += __shfl_xor(h, s);
    if (lane == 0) hdiag[i] = h;
  }
}

// Exclusive scan of int64 counts; out has n+1 entries (out[n] = total).
__global__ void __launch_bounds__(1024) scan_kernel(const int64_t *__restrict__ in,
                                                    int64_t *__restrict__ out, int64_t n) {
  __shared__ int64_t warp_sums[16];
  __shared__ int64_t carry;
  if (threadIdx.x == 0) carry = 0;
  __syncthreads();
  const int lane = threadIdx.x % kWave, w = threadIdx.x / kWave;
  for (int64_t b0 = 0; b0 < n; b0 += 1024) {
    const int64_t i = b0 + threadIdx.x;
    const int64_t v = (i < n) ? in[i] : 0;
    int64_t s = v;  // inclusive scan within the wave
    for (int d = 1; d < kWave; d <<= 1) {
      const int64_t o = __shfl_up(s, d);
      if (lane >= d) s += o;
    }
    if (lane == kWave - 1) warp_sums[w] = s;
    __syncthreads();
    int64_t prefix = carry;
    for (int k = 0; k < w; ++k) prefix += warp_sums[k];
    if (i < n) out[i] = prefix + s - v;
    __syncthreads();
    if (threadIdx.x == 1023) carry = prefix + s;
    __syncthreads();
  }
  if (threadIdx.x == 0) out[n] = carry;
}

// First pass of the multi-block scan: tile t (1024 entries) scanned exclusively
// in place of out, its total in tile_sum[t].
__global__ void __launch_bounds__(1024) tile_scan_kernel(const int64_t *__restrict__ in,
                                                         int64_t *__restrict__ out, int64_t n,
                                                         int64_t *__restrict__ tile_sum) {
  __shared__ int64_t warp_sums[16];
  const int lane = threadIdx.x % kWave, w = threadIdx.x / kWave;
  const int64_t i = int64_t(blockIdx.x) * 1024 + threadIdx.x;
  const int64_t v = (i < n) ? in[i] : 0;
  int64_t s = v;
  for (int d = 1; d < kWave; d <<= 1) {
    const int64_t o = __shfl_up(s, d);
    if (lane >= d) s += o;
  }
  if (lane == kWave - 1) warp_sums[w] = s;
  __syncthreads();
  int64_t prefix = 0;
  for (int k = 0; k < w; ++k) prefix += warp_sums[k];
  if (i < n) out[i] = prefix + s - v;
  if (threadIdx.x == 1023) tile_sum[blockIdx.x] = prefix + s;
}

__global__ void copy_one_kernel(const int64_t *__restrict__ src, int64_t *__restrict__ dst) {
  if (threadIdx.x == 0) *dst = *src;
}

// Third pass: the exclusive offset of each tile added to its entries.
__global__ void __launch_bounds__(1024) tile_add_kernel(int64_t *__restrict__ out, int64_t n,
                                                        const int64_t *__restrict__ tile_off) {
  const int64_t i = int64_t(blockIdx.x) * 1024 + threadIdx.x;
  if (i < n) out[i] += tile_off[blockIdx.x];
}

// E_loc(x_i) = hdiag_i + sum_j H_ij exp((la'_j - la_i) + i (ph'_j - ph_i)), one
// wave per x over its contiguous pairs, fixed-order reduction, double.  With
// uid, the amplitudes of pair j are those of distinct configuration uid[j].
// F: the type of the amplitude ratio's exp / sincos (float in the bf16 mode:
// the log-amplitude differences are taken in double and evaluated in fp32,
// about 1e-7 relative per term; double in the FP64 and FP32 modes); the
// matrix-element products and their sums stay double.
// lp2 (optional, bf16 mode): the distinct x' log|psi| and phase as one fp32
// pair, one 8-byte gather per pair instead of two (the fused network computes
// both in fp32, so the pair holds them exactly).
template <class F>
__global__ void __launch_bounds__(256) accumulate_kernel(
    int64_t n, const int64_t *__restrict__ off, const double *__restrict__ hval,
    const uint32_t *__restrict__ uid, const double *__restrict__ la_p,
    const double *__restrict__ ph_p, const float2 *__restrict__ lp2,
    const double *__restrict__ la_x, const double *__restrict__ ph_x,
    const double *__restrict__ hdiag, double *__restrict__ eloc) {
  const int lane = threadIdx.x % kWave;
  const int64_t i = int64_t(blockIdx.x) * kWavesPerBlock + threadIdx.x / kWave;
  if (i >= n) return;
  const int64_t j0 = off[i] - off[0], j1 = off[i + 1] - off[0];
  const double lx = la_x[i], px = ph_x[i];
  double re = 0.0, im = 0.0;
  // four pairs per lane and iteration, their index and amplitude loads issued
  // before any is used; each lane still adds its pairs in order
  constexpr int Q = 4;
  for (int64_t j = j0 + lane; j < j1; j += Q * kWave) {
    int64_t u[Q];
    double hv[Q], lp[Q], pp[Q];
#pragma unroll
    for (int q = 0; q < Q; ++q) {
      const int64_t jq = j + q * kWave;
      u[q] = jq < j1 ? (uid ? int64_t(uid[jq]) : jq) : -1;
      hv[q] = jq < j1 ? hval[jq] : 0.0;
    }
    if (lp2) {
#pragma unroll
      for (int q = 0; q < Q; ++q) {
        const float2 v = u[q] >= 0 ? lp2[u[q]] : float2{0.f, 0.f};
        lp[q] = u[q] >= 0 ? double(v.x) : lx;
        pp[q] = u[q] >= 0 ? double(v.y) : px;
      }
    } else {
#pragma unroll
      for (int q = 0; q < Q; ++q) {
        lp[q] = u[q] >= 0 ? la_p[u[q]] : lx;
        pp[q] = u[q] >= 0 ? ph_p[u[q]] : px;
      }
    }
#pragma unroll
    for (int q = 0; q < Q; ++q) {
      if (u[q] < 0) continue;
      F a, s, c;
      if constexpr (sizeof(F) == 4) {
        a = expf(F(lp[q] - lx));
        sincosf(F(pp[q] - px), &s, &c);
      } else {
        a = exp(lp[q] - lx);
        sincos(pp[q] - px, &s, &c);
      }
      re += hv[q] * double(a) * double(c);
      im += hv[q] * double(a) * double(s);
    }
  }
  for (int s = kWave / 2; s > 0; s >>= 1) {
    re += __shfl_xor(re, s);
    im += __shfl_xor(im, s);
  }
  if (lane == 0) {
    eloc[2 * i] = hdiag[i] + re;
    eloc[2 * i + 1] = im;
  }
}

__global__ void pack_amp_kernel(const double *__restrict__ la, const double *__restrict__ ph,
                                int64_t n, float2 *__restrict__ out) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < n) out[i] = float2{float(la[i]), float(ph[i])};
}

// sums = {W, sum n Re E, sum n Im E, sum n |E|^2}; one block, fixed order.
__global__ void __launch_bounds__(1024) reduce_kernel(const double *__restrict__ eloc,
                                                      const uint64_t *__restrict__ counts,
                                                      int64_t n, double *__restrict__ sums) {
  __shared__ double part[4][1024];
  double a[4] = {0, 0, 0, 0};
  for (int64_t i = threadIdx.x; i < n; i += 1024) {
    const double w = counts ? double(counts[i]) : 1.0;
    const double re = eloc[2 * i], im = eloc[2 * i + 1];
    a[0] += w;
    a[1] += w * re;
    a[2] += w * im;
    a[3] += w * (re * re + im * im);
  }
  for (int k = 0; k < 4; ++k) part[k][threadIdx.x] = a[k];
  __syncthreads();
  for (int s = 512; s > 0; s >>= 1) {
    if (threadIdx.x < s)
      for (int k = 0; k < 4; ++k) part[k][threadIdx.x] += part[k][threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x < 4) sums[threadIdx.x] = part[threadIdx.x][0];
}

__global__ void weights_kernel(const double *__restrict__ eloc, const uint64_t *__restrict__ counts,
                               int64_t n, const double *__restrict__ sums,
                               double *__restrict__ gl, double *__restrict__ gp) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double W = sums[0];
  const double er = sums[1] / W, ei = sums[2] / W;
  const double w = 2.0 * (counts ? double(counts[i]) : 1.0) / W;
  gl[i] = w * (eloc[2 * i] - er);
  gp[i] = w * (eloc[2 * i + 1] - ei);
}

template <class T>
__global__ void adam_kernel(T *__restrict__ p, const T *__restrict__ g, T *__restrict__ m,
                            T *__restrict__ v, int64_t n, double lr, double b1, double b2,
                            double eps, double c1, double c2) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double gi = double(g[i]);
  const double mi = b1 * double(m[i]) + (1.0 - b1) * gi;
  const double vi = b2 * double(v[i]) + (1.0 - b2) * gi * gi;
  m[i] = T(mi);
  v[i] = T(vi);
  p[i] = T(double(p[i]) - lr * (mi / c1) / (sqrt(vi / c2) + eps));
}

}  // namespace

void launch_count_pairs(const nqs_ham &H, const uint64_t *x, int64_t n, int64_t *cnt,
                        hipStream_t s) {
  if (n <= 0) return;
  const int64_t blocks = ceil_div(n, kWavesPerBlock);
  hipLaunchKernelGGL(count_pairs_kernel, dim3(unsigned(blocks)), dim3(256), 0, s, x, n,
                     H.d_flip.as<uint64_t>(), int64_t(H.flip.size()), cnt);
  HIP_LAUNCH_OK();
}

void launch_emit_pairs(const nqs_ham &H, const uint64_t *x, int64_t n, const int64_t *off,
                       uint64_t *xp, double *hval, int32_t *owner, double *hdiag,
                       int64_t owner_base, hipStream_t s) {
  if (n <= 0) return;
  const int64_t blocks = ceil_div(n, kWavesPerBlock);
  hipLaunchKernelGGL(emit_pairs_kernel, dim3(unsigned(blocks)), dim3(256), 0, s, x, n,
                     H.d_flip.as<uint64_t>(), H.d_off.as<int64_t>(), H.d_zmask.as<uint64_t>(),
                     H.d_coef.as<double>(), int64_t(H.flip.size()), off, xp, hval, owner, hdiag,
                     owner_base);
  HIP_LAUNCH_OK();
}

// Up to 8 tiles one block scans alone; beyond, three passes (tiles, the tile
// totals with the one-block scan, offsets added back) over tile_ws, which
// holds 2 * tiles + 1 int64 (scan_workspace_entries).
int64_t scan_workspace_entries(int64_t n) {
  const int64_t tiles = ceil_div(n, 1024);
  return tiles <= 8 ? 0 : 2 * tiles + 1;
}

void launch_exclusive_scan(const int64_t *in, int64_t *out, int64_t n, hipStream_t s,
                           int64_t *tile_ws) {
  const int64_t tiles = ceil_div(n, 1024);
  if (tiles <= 8) {
    hipLaunchKernelGGL(scan_kernel, dim3(1), dim3(1024), 0, s, in, out, n);
    HIP_LAUNCH_OK();
    return;
  }
  NQS_REQUIRE(tiles < (int64_t(1) << 31), NQS_EUNSUPPORTED, "scan: too many entries");
  NQS_REQUIRE(tile_ws != nullptr, NQS_EINVAL, "scan: no workspace");
  int64_t *tile_sum = tile_ws, *tile_off = tile_ws + tiles;
  hipLaunchKernelGGL(tile_scan_kernel, dim3(unsigned(tiles)), dim3(1024), 0, s, in, out, n,
                     tile_sum);
  HIP_LAUNCH_OK();
  hipLaunchKernelGGL(scan_kernel, dim3(1), dim3(1024), 0, s, tile_sum, tile_off, tiles);
  HIP_LAUNCH_OK();
  hipLaunchKernelGGL(tile_add_kernel, dim3(unsigned(tiles)), dim3(1024), 0, s, out, n, tile_off);
  HIP_LAUNCH_OK();
  // out[n] = the total, the last entry of the tile-offset scan
  hipLaunchKernelGGL(copy_one_kernel, dim3(1), dim3(64), 0, s, tile_off + tiles, out + n);
  HIP_LAUNCH_OK();
}

// The same with the workspace in a buffer of the calling handle (grown
// outside any graph capture: no captured sequence of this library contains a
// scan), so calls through different handles on different streams do not share
// it.
void launch_exclusive_scan(const int64_t *in, int64_t *out, int64_t n, hipStream_t s,
                           DevBuf &ws) {
  const int64_t e = scan_workspace_entries(n);
  launch_exclusive_scan(in, out, n, s, e ? static_cast<int64_t *>(ws.reserve(size_t(e) * 8))
                                         : nullptr);
}

void launch_accumulate(int64_t n, const int64_t *off, const double *hval, const uint32_t *uid,
                       const double *la_p, const double *ph_p, const double *la_x,
                       const double *ph_x, const double *hdiag, double *eloc, hipStream_t s,
                       bool fp32_ratio, int64_t n_amp, float2 *lp2_ws) {
  if (n <= 0) return;
  const dim3 grid(unsigned(ceil_div(n, kWavesPerBlock)));
  if (fp32_ratio) {
    // distinct x' (uid set): their amplitudes packed as fp32 pairs first
    const bool packed = uid && lp2_ws && n_amp > 0;
    if (packed) {
      hipLaunchKernelGGL(pack_amp_kernel, dim3(unsigned(ceil_div(n_amp, 256))), dim3(256), 0, s,
                         la_p, ph_p, n_amp, lp2_ws);
      HIP_LAUNCH_OK();
    }
    hipLaunchKernelGGL(accumulate_kernel<float>, grid, dim3(256), 0, s, n, off, hval, uid, la_p,
                       ph_p, packed ? lp2_ws : nullptr, la_x, ph_x, hdiag, eloc);
  } else {
    hipLaunchKernelGGL(accumulate_kernel<double>, grid, dim3(256), 0, s, n, off, hval, uid, la_p,
                       ph_p, nullptr, la_x, ph_x, hdiag, eloc);
  }
  HIP_LAUNCH_OK();
}

void launch_reduce(const double *eloc, const uint64_t *counts, int64_t n, double *sums,
                   hipStream_t s) {
  hipLaunchKernelGGL(reduce_kernel, dim3(1), dim3(1024), 0, s, eloc, counts, n, sums);
  HIP_LAUNCH_OK();
}

void launch_weights(const double *eloc, const uint64_t *counts, int64_t n, const double *sums,
                    double *gl, double *gp, hipStream_t s) {
  if (n <= 0) return;
  hipLaunchKernelGGL(weights_kernel, dim3(unsigned(ceil_div(n, 256))), dim3(256), 0, s, eloc,
                     counts, n, sums, gl, gp);
  HIP_LAUNCH_OK();
}

void launch_adam(void *p, const void *g, void *m, void *v, int64_t n, int elem, double lr,
                 double b1, double b2, double eps, int64_t t, hipStream_t s) {
  if (n <= 0) return;
  const double c1 = 1.0 - pow(b1, double(t)), c2 = 1.0 - pow(b2, double(t));
  const dim3 grid(unsigned(ceil_div(n, 256)));
  if (elem == 8)
    hipLaunchKernelGGL(adam_kernel<double>, grid, dim3(256), 0, s, (double *)p, (const double *)g,
                       (double *)m, (double *)v, n, lr, b1, b2, eps, c1, c2);
  else
    hipLaunchKernelGGL(adam_kernel<float>, grid, dim3(256), 0, s, (float *)p, (const float *)g,
                       (float *)m, (float *)v, n, lr, b1, b2, eps, c1, c2);
  HIP_LAUNCH_OK();
}

}  // namespace nqs
