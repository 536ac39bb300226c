// Many molecules in one pass: the local-energy path of the paper ("Variational
// Monte Carlo": local-energy and energy-estimator equations) for a batch of
// molecules of different sizes that share one amplitude network.
//
// Configuration words carry the molecule index in bits 58..63.  One step of
// the batch is a fixed sequence of launches with fixed grids whose sizes
// (samples, pairs, distinct x') live in device memory:
//
//   1. clear   - empty the hash table, zero the counters (fill kernel)
//   2. pairs   - persistent waves take (molecule, sample) work items strided
//                over the grid and sweep the molecule's flip groups: x' = x ^ f,
//                sector screen by popcount, H_xx' from the Pauli terms; every
//                kept x' is inserted into an open-addressing hash table keyed by
//                (molecule, x'), whose first inserter numbers it as a distinct
//                configuration.  Pair j keeps its table slot and H value.
//   3. psi(x)  - the fused amplitude kernel on the samples (persistent)
//   4. psi(x') - the fused amplitude kernel on the distinct x' (persistent,
//                count read from the device)
//   5. E_loc   - one wave per sample over its pairs in group order, double
//   6. sums    - one block per molecule: W, sum n Re E, sum n Im E, sum n |E|^2
//
// The numbering of distinct x' depends on timing, but every amplitude is
// computed independently of its position in the batch and E_loc sums its
// pairs in a fixed order, so results are bitwise reproducible.  No library
// call and no memset is inside the sequence, so it is captured once into a
// hipGraph (per capacity and launch shape) and replayed every step.  Launch
// shapes come from a small autotuner that times candidates on the batch.
#include <algorithm>
#include <array>
#include <cmath>
#include <functional>
#include <memory>
#include <string>
#include <vector>

#include "ham.h"
#include "model.h"

namespace nqs {
namespace {

constexpr int kMaxMol = 64;
constexpr int kWave = 64;
constexpr uint64_t kAlphaBits = 0x5555555555555555ull;
constexpr uint64_t kBetaBits = 0xAAAAAAAAAAAAAAAAull;
constexpr uint64_t kEmpty = ~0ull;
constexpr uint32_t kNoSlot = 0xFFFFFFFFu;

struct MolTab {
  int64_t g0;   // first flip group of the molecule in the concatenated tables
  int64_t o0;   // first entry of its group offsets (G + 1 entries, absolute term indices)
  int64_t G;    // flip groups, the diagonal group first
  int64_t K;    // in-sector connected x' of every configuration
  int32_t na, nb, n, pad;
};

// Sizes of one step; uploaded before each launch of the sequence.
struct StepDesc {
  int64_t U, P;                    // samples, pairs
  int64_t u_off[kMaxMol + 1];      // first sample of each molecule
  int64_t p_off[kMaxMol + 1];      // first pair of each molecule
};

struct Counters {
  int64_t work;       // unused (kept for layout)
  int64_t distinct;   // distinct x' so far
  int64_t overflow;   // a configuration had more connected x' than K, or the table was full
  int64_t pad;
};

__device__ inline uint64_t mix64(uint64_t z) {
  // splitmix64 finaliser (Steele, Lea, Flood, OOPSLA 2014)
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

__global__ void clear_kernel(uint64_t *__restrict__ table, int64_t table_size,
                             Counters *__restrict__ ctr) {
  const int64_t i0 = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  const int64_t stride = int64_t(gridDim.x) * blockDim.x;
  for (int64_t i = i0; i < table_size; i += stride) table[i] = kEmpty;
  if (i0 == 0) {
    ctr->work = 0;
    ctr->distinct = 0;
    ctr->overflow = 0;
  }
}

// Longest linear probe; a longer run means the table is too full for the
// step (it is then enlarged and the step run again).
constexpr int kMaxProbe = 256;

// Inserts key; returns its slot.  The first inserter numbers the key.
__device__ inline uint32_t insert_key(uint64_t key, uint64_t tagged, uint64_t *table,
                                      uint32_t *ids, uint64_t mask, uint64_t *ukeys,
                                      Counters *ctr) {
  uint64_t h = mix64(key) & mask;
  for (int probe = 0; probe < kMaxProbe; ++probe) {
    // most keys are already present (a distinct x' has ~10 pairs): a plain
    // read settles those without an atomic, so popular keys see no contention
    const uint64_t seen = __hip_atomic_load(table + h, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (seen == key) return uint32_t(h);
    if (seen != kEmpty) {
      h = (h + 1) & mask;
      continue;
    }
    const uint64_t prev = atomicCAS(reinterpret_cast<unsigned long long *>(table + h),
                                    (unsigned long long)kEmpty, (unsigned long long)key);
    if (prev == kEmpty) {
      const int64_t id = atomicAdd(reinterpret_cast<unsigned long long *>(&ctr->distinct), 1ull);
      ids[h] = uint32_t(id);
      ukeys[id] = tagged;
      return uint32_t(h);
    }
    if (prev == key) return uint32_t(h);
    h = (h + 1) & mask;
  }
  atomicOr(reinterpret_cast<unsigned long long *>(&ctr->overflow), 2ull);
  return kNoSlot;
}

struct Pend {
  int g, r;       // flip group, output rank within the sample
  uint64_t xp;    // the connected configuration
};

__global__ void __launch_bounds__(256) pairs_kernel(
    const StepDesc *__restrict__ desc, const MolTab *__restrict__ tabs,
    const uint64_t *__restrict__ flip, const int64_t *__restrict__ goff,
    const uint64_t *__restrict__ zmask, const double *__restrict__ coef,
    const uint64_t *__restrict__ x, int n_mol, int nbits, uint64_t *__restrict__ table,
    uint32_t *__restrict__ ids, uint64_t table_mask, uint64_t *__restrict__ ukeys,
    uint32_t *__restrict__ slot, double *__restrict__ hval, double *__restrict__ hdiag,
    Counters *__restrict__ ctr) {
  const int lane = threadIdx.x % kWave;
  const uint64_t below = (lane == 0) ? 0ull : (~0ull >> (kWave - lane));
  const int64_t U = desc->U;
  __shared__ Pend pend_all[4][2 * kWave];   // per wave: kept pairs waiting to be handled
  Pend *pend = pend_all[threadIdx.x / kWave];
  // samples strided over the waves (the samples of every molecule are spread
  // over all waves); the wave index is made wave-uniform explicitly
  const int64_t wave = int64_t(blockIdx.x) * (blockDim.x / kWave) +
                       __builtin_amdgcn_readfirstlane(int(threadIdx.x / kWave));
  const int64_t n_waves = int64_t(gridDim.x) * (blockDim.x / kWave);
  for (int64_t s = wave; s < U; s += n_waves) {
    const uint64_t xw = x[s];
    const int mol = int(xw >> kTagShift);
    const uint64_t xs = xw & kOccMask;
    if (mol >= n_mol || s < desc->u_off[mol] || s >= desc->u_off[mol + 1]) {
      // the word's molecule disagrees with the offsets: no slot of it is written
      atomicOr(reinterpret_cast<unsigned long long *>(&ctr->overflow), 4ull);
      continue;
    }
    const MolTab tb = tabs[mol];
    const int64_t base = desc->p_off[mol] + (s - desc->u_off[mol]) * tb.K;
    const uint64_t tag = uint64_t(mol) << kTagShift, ktag = uint64_t(mol) << nbits;
    // Kept pairs are first listed in LDS (group, output rank, x'), then handled
    // 64 at a time with every lane busy: most flip groups fail the sector
    // screen, so handling them where they are found would leave ~70 % of the
    // lanes idle through the term loop and the table insert.
    int found = 0, npend = 0;
    auto handle = [&](int count) {
      if (lane < count) {
        const Pend e = pend[lane];
        if (e.r < tb.K) {
          // the group's terms, four loads in flight at a time, summed in order
          const int64_t t0 = goff[tb.o0 + e.g], t1 = goff[tb.o0 + e.g + 1];
          double hv = 0.0;
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
            for (int u = 0; u < 4; ++u) hv += (__popcll(xs & z[u]) & 1) ? -c[u] : c[u];
          }
          for (; t < t1; ++t) {
            const double c = coef[t];
            hv += (__popcll(xs & zmask[t]) & 1) ? -c : c;
          }
          hval[base + e.r] = hv;
          slot[base + e.r] = insert_key(ktag | e.xp, tag | e.xp, table, ids, table_mask, ukeys, ctr);
        }
      }
    };
    for (int64_t g0 = 1; g0 < tb.G; g0 += kWave) {
      const int64_t g = g0 + lane;
      const uint64_t f = (g < tb.G) ? flip[tb.g0 + g] : 0ull;
      const uint64_t xp = xs ^ f;
      const bool keep = g < tb.G && __popcll(xp & kAlphaBits) == tb.na &&
                        __popcll(xp & kBetaBits) == tb.nb;
      const uint64_t m = __ballot(keep);
      const int rank = __popcll(m & below);
      if (keep) pend[npend + rank] = Pend{int(g), found + rank, xp};
      npend += __popcll(m);
      found += __popcll(m);
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
      if (npend >= kWave) {
        handle(kWave);
        // move the overflow (fewer than 64 entries) to the front of the list
        Pend tail{};
        if (lane < npend - kWave) tail = pend[kWave + lane];
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        if (lane < npend - kWave) pend[lane] = tail;
        npend -= kWave;
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
      }
    }
    handle(npend);
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    if (found > tb.K) {
      atomicOr(reinterpret_cast<unsigned long long *>(&ctr->overflow), 1ull);
      found = tb.K;
    }
    for (int64_t r = found + lane; r < tb.K; r += kWave) {   // groups with no term
      hval[base + r] = 0.0;
      slot[base + r] = kNoSlot;
    }
    // diagonal group: lanes split its terms, then a fixed-order wave reduction
    double h = 0.0;
    for (int64_t t = goff[tb.o0] + lane; t < goff[tb.o0 + 1]; t += kWave) {
      const double c = coef[t];
      h += (__popcll(xs & zmask[t]) & 1) ? -c : c;
    }
    for (int o = kWave / 2; o > 0; o >>= 1) h += __shfl_xor(h, o);
    if (lane == 0) hdiag[s] = h;
  }
}

// E_loc(x_s) = hdiag_s + sum_j H_j exp((la'_j - la_s) + i (ph'_j - ph_s)) over the
// sample's pairs in group order; one wave per sample, fixed-order reduction.
// F: the type of the ratio's exp / sincos (float for the bf16 step: the
// log-amplitude differences in fp32; double otherwise); sums in double.
template <class F>
__global__ void __launch_bounds__(256) accumulate_kernel(
    const StepDesc *__restrict__ desc, const MolTab *__restrict__ tabs,
    const uint64_t *__restrict__ x, int n_mol, const uint32_t *__restrict__ slot,
    const uint32_t *__restrict__ ids, const double *__restrict__ hval,
    const double *__restrict__ la_p, const double *__restrict__ ph_p,
    const double *__restrict__ la_x, const double *__restrict__ ph_x,
    const double *__restrict__ hdiag, double *__restrict__ eloc) {
  const int lane = threadIdx.x % kWave;
  const int64_t U = desc->U;
  const int64_t waves = int64_t(gridDim.x) * (blockDim.x / kWave);
  const int64_t wave = int64_t(blockIdx.x) * (blockDim.x / kWave) +
                       __builtin_amdgcn_readfirstlane(int(threadIdx.x / kWave));
  for (int64_t s = wave; s < U; s += waves) {
    const int mol = int(x[s] >> kTagShift);
    if (mol >= n_mol || s < desc->u_off[mol] || s >= desc->u_off[mol + 1]) {
      if (lane == 0) {
        eloc[2 * s] = NAN;
        eloc[2 * s + 1] = NAN;
      }
      continue;
    }
    const int64_t K = tabs[mol].K;
    const int64_t j0 = desc->p_off[mol] + (s - desc->u_off[mol]) * K;
    const double lx = la_x[s], px = ph_x[s];
    double re = 0.0, im = 0.0;
    // four pairs per lane and iteration, loads issued before any is used;
    // each lane still adds its pairs in order
    constexpr int Q = 4;
    for (int64_t j = j0 + lane; j < j0 + K; j += Q * kWave) {
      uint32_t sl[Q], u[Q];
      double hv[Q], lp[Q], pp[Q];
#pragma unroll
      for (int q = 0; q < Q; ++q) {
        const int64_t jq = j + q * kWave;
        sl[q] = jq < j0 + K ? slot[jq] : kNoSlot;
        hv[q] = jq < j0 + K ? hval[jq] : 0.0;
      }
#pragma unroll
      for (int q = 0; q < Q; ++q) u[q] = sl[q] != kNoSlot ? ids[sl[q]] : 0u;
#pragma unroll
      for (int q = 0; q < Q; ++q) {
        lp[q] = sl[q] != kNoSlot ? la_p[u[q]] : lx;
        pp[q] = sl[q] != kNoSlot ? ph_p[u[q]] : px;
      }
#pragma unroll
      for (int q = 0; q < Q; ++q) {
        if (sl[q] == kNoSlot) continue;
        F a, sn, cs;
        if constexpr (sizeof(F) == 4) {
          a = expf(F(lp[q] - lx));
          sincosf(F(pp[q] - px), &sn, &cs);
        } else {
          a = exp(lp[q] - lx);
          sincos(pp[q] - px, &sn, &cs);
        }
        re += hv[q] * double(a) * double(cs);
        im += hv[q] * double(a) * double(sn);
      }
    }
    for (int o = kWave / 2; o > 0; o >>= 1) {
      re += __shfl_xor(re, o);
      im += __shfl_xor(im, o);
    }
    if (lane == 0) {
      eloc[2 * s] = hdiag[s] + re;
      eloc[2 * s + 1] = im;
    }
  }
}

// sums[i] = {W, sum n Re E, sum n Im E, sum n |E|^2} of molecule i; one block each.
__global__ void __launch_bounds__(256) reduce_kernel(const StepDesc *__restrict__ desc,
                                                     const double *__restrict__ eloc,
                                                     const uint64_t *__restrict__ counts,
                                                     double *__restrict__ sums) {
  __shared__ double part[4][256];
  const int i = blockIdx.x;
  const int64_t a0 = desc->u_off[i], a1 = desc->u_off[i + 1];
  double acc[4] = {0, 0, 0, 0};
  for (int64_t s = a0 + threadIdx.x; s < a1; s += 256) {
    const double w = double(counts[s]);
    const double re = eloc[2 * s], im = eloc[2 * s + 1];
    acc[0] += w;
    acc[1] += w * re;
    acc[2] += w * im;
    acc[3] += w * (re * re + im * im);
  }
  for (int k = 0; k < 4; ++k) part[k][threadIdx.x] = acc[k];
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (int(threadIdx.x) < o)
      for (int k = 0; k < 4; ++k) part[k][threadIdx.x] += part[k][threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x < 4) sums[4 * i + threadIdx.x] = part[threadIdx.x][0];
}

// distinct x' per molecule (from the tags of the distinct list)
__global__ void count_mol_kernel(const uint64_t *__restrict__ ukeys,
                                 const Counters *__restrict__ ctr, int n_mol,
                                 unsigned long long *__restrict__ per_mol) {
  __shared__ unsigned long long local[kMaxMol];
  if (threadIdx.x < kMaxMol) local[threadIdx.x] = 0;
  __syncthreads();
  const int64_t n = ctr->distinct;
  for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n;
       i += int64_t(gridDim.x) * blockDim.x) {
    const int m = int(ukeys[i] >> kTagShift);
    if (m < n_mol) atomicAdd(&local[m], 1ull);
  }
  __syncthreads();
  if (int(threadIdx.x) < n_mol && local[threadIdx.x]) atomicAdd(&per_mol[threadIdx.x], local[threadIdx.x]);
}

__global__ void zero_u64_kernel(unsigned long long *p, int n) {
  if (int(threadIdx.x) < n) p[threadIdx.x] = 0;
}

// Upstream weights of the summed energy of the molecules: sample s of molecule
// i gets 2 n_s / W_i (E_loc,s - E_i), split into real and imaginary parts.
__global__ void weights_kernel(const double *__restrict__ eloc, const uint64_t *__restrict__ counts,
                               const uint64_t *__restrict__ x, int64_t U, int n_mol,
                               const double *__restrict__ sums, double *__restrict__ gl,
                               double *__restrict__ gp) {
  const int64_t s = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (s >= U) return;
  const int i = int(x[s] >> kTagShift);
  if (i >= n_mol) {
    gl[s] = NAN;
    gp[s] = NAN;
    return;
  }
  const double W = sums[4 * i];
  const double w = 2.0 * double(counts[s]) / W;
  gl[s] = w * (eloc[2 * s] - sums[4 * i + 1] / W);
  gp[s] = w * (eloc[2 * s + 1] - sums[4 * i + 2] / W);
}

inline dim3 g1(int64_t n) { return dim3(unsigned(ceil_div(n, 256))); }

int64_t choose(int64_t n, int64_t k) {
  if (k < 0 || k > n) return 0;
  int64_t r = 1;
  for (int64_t i = 1; i <= k; ++i) r = r * (n - k + i) / i;
  return r;
}

}  // namespace
}  // namespace nqs

using namespace nqs;

struct nqs_batch {
  int n_mol = 0, nbits = 0;
  nqs_model *model = nullptr;
  uint64_t sec_gen = 0;            // the model's sector-table generation the graph was made for
  std::vector<MolTab> tabs_host;
  DevBuf tabs, flip, goff, zmask, coef;
  // capacities and step buffers (fixed addresses inside a captured graph)
  int64_t u_cap = 0, p_cap = 0, t_size = 0;
  DevBuf x, cnt, lax, phx, eloc, hdiag, sums, desc, ctr;
  DevBuf table, ids, ukeys, la, ph, slot, hval;
  StepDesc *desc_host = nullptr;   // pinned
  // launch shapes (autotuned) and the captured sequence
  int pairs_blocks = 1024, acc_blocks = 1024;
  FusedTile xp_tile{8, 512}, x_tile{4, 512};
  bool tuned = false, use_graph = true;
  hipStream_t cap_stream = nullptr;
  hipGraphExec_t exec = nullptr;
  hipEvent_t ev0 = nullptr, ev1 = nullptr;   // around the distinct-x' amplitude launch
  bool graph_has_psi_x = false;
  // statistics of the last step
  int64_t last_pairs = 0, last_distinct = 0, captures = 0;
  int64_t est_distinct = 0;        // raised when a step overfills the distinct-x' table
  int64_t t_override = 0;          // table size of the next step (batch_set_table), 0 = automatic
  std::vector<int64_t> distinct_per_mol;
  DevBuf per_mol;
  std::vector<double> tune_ms;     // candidate timings of the last tuning

  ~nqs_batch() {
    if (exec) (void)hipGraphExecDestroy(exec);
    if (ev0) (void)hipEventDestroy(ev0);
    if (ev1) (void)hipEventDestroy(ev1);
    if (cap_stream) (void)hipStreamDestroy(cap_stream);
    if (desc_host) (void)hipHostFree(desc_host);
  }
};

namespace nqs {
namespace {

void drop_graph(nqs_batch &b) {
  if (b.exec) HIP_OK(hipGraphExecDestroy(b.exec));
  b.exec = nullptr;
}

// Grow the step buffers to hold U samples and P pairs (with slack, so that
// small changes between steps keep the captured graph).
void reserve(nqs_batch &b, int64_t U, int64_t P) {
  bool grown = false;
  if (U > b.u_cap) {
    b.u_cap = std::max<int64_t>(U + U / 2, 1024);
    b.x.reserve(size_t(b.u_cap) * 8);
    b.cnt.reserve(size_t(b.u_cap) * 8);
    b.lax.reserve(size_t(b.u_cap) * 8);
    b.phx.reserve(size_t(b.u_cap) * 8);
    b.eloc.reserve(size_t(b.u_cap) * 16);
    b.hdiag.reserve(size_t(b.u_cap) * 8);
    grown = true;
  }
  if (P > b.p_cap) {
    b.p_cap = std::max<int64_t>(P + P / 2, 1 << 16);
    NQS_REQUIRE(b.p_cap < (int64_t(1) << 32), NQS_EUNSUPPORTED, "batch: more than 2^32 pairs");
    b.ukeys.reserve(size_t(b.p_cap) * 8);
    b.la.reserve(size_t(b.p_cap) * 8);
    b.ph.reserve(size_t(b.p_cap) * 8);
    b.slot.reserve(size_t(b.p_cap) * 4);
    b.hval.reserve(size_t(b.p_cap) * 8);
    grown = true;
  }
  // distinct-x' table: at least twice the pairs (or the enlarged estimate
  // after an overfull step).  A sparse table is measured faster than one
  // sized for the distinct x' alone: fewer keys share a cache line, so the
  // concurrent compare-and-swaps of different CUs rarely collide.
  const int64_t want = std::max<int64_t>(b.est_distinct, b.p_cap);
  int64_t t = int64_t(1) << 16;
  while (t < 2 * want) t <<= 1;
  if (b.t_override > 0) t = b.t_override;
  if (t > b.t_size || (b.t_override > 0 && t != b.t_size)) {
    b.t_size = t;
    b.table.reserve(size_t(t) * 8);
    b.ids.reserve(size_t(t) * 4);
    grown = true;
  }
  if (grown) drop_graph(b);
}

// The launch sequence of one step (steps 1..6 above) on stream s.
void enqueue(nqs_batch &b, bool psi_x, hipStream_t s) {
  nqs_model &m = *b.model;
  auto *desc = b.desc.as<StepDesc>();
  auto *ctr = b.ctr.as<Counters>();
  hipLaunchKernelGGL(clear_kernel, dim3(2048), dim3(256), 0, s, b.table.as<uint64_t>(), b.t_size,
                     ctr);
  HIP_LAUNCH_OK();
  hipLaunchKernelGGL(pairs_kernel, dim3(unsigned(b.pairs_blocks)), dim3(256), 0, s, desc,
                     b.tabs.as<MolTab>(), b.flip.as<uint64_t>(), b.goff.as<int64_t>(),
                     b.zmask.as<uint64_t>(), b.coef.as<double>(), b.x.as<uint64_t>(), b.n_mol,
                     b.nbits,
                     b.table.as<uint64_t>(), b.ids.as<uint32_t>(), uint64_t(b.t_size - 1),
                     b.ukeys.as<uint64_t>(), b.slot.as<uint32_t>(), b.hval.as<double>(),
                     b.hdiag.as<double>(), ctr);
  HIP_LAUNCH_OK();
  if (psi_x)
    fused_forward(m, b.x.as<uint64_t>(), b.u_cap, b.lax.as<double>(), b.phx.as<double>(), nullptr,
                  -1, s, &desc->U, b.x_tile);
  HIP_OK(hipEventRecord(b.ev0, s));
  fused_forward(m, b.ukeys.as<uint64_t>(), b.p_cap, b.la.as<double>(), b.ph.as<double>(), nullptr,
                -1, s, &ctr->distinct, b.xp_tile);
  HIP_OK(hipEventRecord(b.ev1, s));
  hipLaunchKernelGGL(accumulate_kernel<float>, dim3(unsigned(b.acc_blocks)), dim3(256), 0, s, desc,
                     b.tabs.as<MolTab>(), b.x.as<uint64_t>(), b.n_mol, b.slot.as<uint32_t>(),
                     b.ids.as<uint32_t>(), b.hval.as<double>(), b.la.as<double>(),
                     b.ph.as<double>(), b.lax.as<double>(), b.phx.as<double>(),
                     b.hdiag.as<double>(), b.eloc.as<double>());
  HIP_LAUNCH_OK();
  hipLaunchKernelGGL(reduce_kernel, dim3(unsigned(b.n_mol)), dim3(256), 0, s, desc,
                     b.eloc.as<double>(), b.cnt.as<uint64_t>(), b.sums.as<double>());
  HIP_LAUNCH_OK();
}

void capture(nqs_batch &b, bool psi_x) {
  drop_graph(b);
  if (!b.cap_stream) HIP_OK(hipStreamCreateWithFlags(&b.cap_stream, hipStreamNonBlocking));
  hipGraph_t g = nullptr;
  HIP_OK(hipStreamBeginCapture(b.cap_stream, hipStreamCaptureModeThreadLocal));
  try {
    enqueue(b, psi_x, b.cap_stream);
  } catch (...) {
    (void)hipStreamEndCapture(b.cap_stream, &g);
    if (g) (void)hipGraphDestroy(g);
    throw;
  }
  HIP_OK(hipStreamEndCapture(b.cap_stream, &g));
  hipGraphExec_t e = nullptr;
  const hipError_t st = hipGraphInstantiate(&e, g, nullptr, nullptr, 0);
  (void)hipGraphDestroy(g);
  HIP_OK(st);
  b.exec = e;
  b.graph_has_psi_x = psi_x;
  ++b.captures;
}

float time_ms(hipStream_t s, const std::function<void()> &f) {
  hipEvent_t e0, e1;
  HIP_OK(hipEventCreate(&e0));
  HIP_OK(hipEventCreate(&e1));
  HIP_OK(hipEventRecord(e0, s));
  f();
  HIP_OK(hipEventRecord(e1, s));
  HIP_OK(hipEventSynchronize(e1));
  float ms = 0.f;
  HIP_OK(hipEventElapsedTime(&ms, e0, e1));
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  return ms;
}

// Times candidate launch shapes on the current step's data (the buffers hold
// a complete step) and keeps the fastest.  Results do not depend on the shape.
void tune(nqs_batch &b, hipStream_t s) {
  nqs_model &m = *b.model;
  auto *ctr = b.ctr.as<Counters>();
  auto *desc = b.desc.as<StepDesc>();
  b.tune_ms.clear();
  // pairs kernel: blocks of four waves
  float best = 1e30f;
  int best_pb = b.pairs_blocks;
  for (int pb : {512, 1024, 2048, 4096}) {
    b.pairs_blocks = pb;
    float t = 1e30f;
    for (int rep = 0; rep < 2; ++rep)
      t = std::min(t, time_ms(s, [&] {
            hipLaunchKernelGGL(clear_kernel, dim3(2048), dim3(256), 0, s, b.table.as<uint64_t>(),
                               b.t_size, ctr);
            hipLaunchKernelGGL(pairs_kernel, dim3(unsigned(pb)), dim3(256), 0, s, desc,
                               b.tabs.as<MolTab>(), b.flip.as<uint64_t>(), b.goff.as<int64_t>(),
                               b.zmask.as<uint64_t>(), b.coef.as<double>(), b.x.as<uint64_t>(),
                               b.n_mol, b.nbits, b.table.as<uint64_t>(), b.ids.as<uint32_t>(),
                               uint64_t(b.t_size - 1), b.ukeys.as<uint64_t>(),
                               b.slot.as<uint32_t>(), b.hval.as<double>(), b.hdiag.as<double>(),
                               ctr);
          }));
    HIP_LAUNCH_OK();
    b.tune_ms.push_back(t);
    if (t < best) {
      best = t;
      best_pb = pb;
    }
  }
  b.pairs_blocks = best_pb;
  // the table and distinct list of the last candidate are complete: time the
  // amplitude kernel on the distinct x'
  best = 1e30f;
  FusedTile best_tile = b.xp_tile;
  for (int pairs : {2, 4, 8, 16})
    for (int blocks : {512, 1024}) {
      const FusedTile tile{pairs, blocks};
      float t = 1e30f;
      for (int rep = 0; rep < 2; ++rep)
        t = std::min(t, time_ms(s, [&] {
              fused_forward(m, b.ukeys.as<uint64_t>(), b.p_cap, b.la.as<double>(),
                            b.ph.as<double>(), nullptr, -1, s, &ctr->distinct, tile);
            }));
      b.tune_ms.push_back(t);
      if (t < best) {
        best = t;
        best_tile = tile;
      }
    }
  b.xp_tile = best_tile;
  b.tuned = true;
  drop_graph(b);
}

}  // namespace
}  // namespace nqs

extern "C" int batch_create(nqs_ham *const *hams, int n_mol, nqs_model *model, nqs_batch **out) {
  return guarded([&] {
    NQS_REQUIRE(hams && model && out, NQS_EINVAL, "batch_create: null argument");
    *out = nullptr;
    NQS_REQUIRE(n_mol >= 1 && n_mol <= kMaxMol, NQS_EINVAL, "batch_create: 1..64 molecules");
    auto b = std::make_unique<nqs_batch>();
    b->n_mol = n_mol;
    b->model = model;
    std::vector<int32_t> ns, nas, nbs;
    std::vector<uint64_t> flip, zmask;
    std::vector<int64_t> goff;
    std::vector<double> coef;
    for (int i = 0; i < n_mol; ++i) {
      const nqs_ham *H = hams[i];
      NQS_REQUIRE(H, NQS_EINVAL, "batch_create: null Hamiltonian");
      NQS_REQUIRE(H->N <= kTagShift, NQS_EUNSUPPORTED,
                  "batch_create: more than 58 spin-orbitals leave no room for the molecule index");
      const int64_t G = int64_t(H->flip.size());
      // every single and double excitation must have its own flip group, so that
      // every configuration has the same number K of connected x'
      const int64_t n = H->n, c2 = choose(n, 2);
      NQS_REQUIRE(G == 1 + 2 * c2 + 2 * choose(n, 4) + c2 * c2, NQS_EUNSUPPORTED,
                  "batch_create: a flip group of molecule " + std::to_string(i) +
                      " has no term (exactly cancelling integrals)");
      uint64_t hf = 0;
      for (int p = 0; p < H->n_alpha; ++p) hf |= uint64_t(1) << (2 * p);
      for (int p = 0; p < H->n_beta; ++p) hf |= uint64_t(1) << (2 * p + 1);
      int64_t K = 0;
      for (int64_t g = 1; g < G; ++g) {
        const uint64_t xp = hf ^ H->flip[size_t(g)];
        K += __builtin_popcountll(xp & kAlphaBits) == H->n_alpha &&
             __builtin_popcountll(xp & kBetaBits) == H->n_beta;
      }
      MolTab t{};
      t.g0 = int64_t(flip.size());
      t.o0 = int64_t(goff.size());
      t.G = G;
      t.K = K;
      t.na = H->n_alpha;
      t.nb = H->n_beta;
      t.n = H->n;
      const int64_t tbase = int64_t(coef.size());
      flip.insert(flip.end(), H->flip.begin(), H->flip.end());
      for (int64_t g = 0; g <= G; ++g) goff.push_back(tbase + H->off[size_t(g)]);
      zmask.insert(zmask.end(), H->zmask.begin(), H->zmask.end());
      coef.insert(coef.end(), H->coef.begin(), H->coef.end());
      b->tabs_host.push_back(t);
      b->nbits = std::max(b->nbits, H->N);
      ns.push_back(H->n);
      nas.push_back(H->n_alpha);
      nbs.push_back(H->n_beta);
    }
    NQS_REQUIRE(b->nbits + 7 <= 64, NQS_EUNSUPPORTED, "batch_create: keys need N + 7 bits");
    const int st = amp_model_set_sectors(model, n_mol, ns.data(), nas.data(), nbs.data());
    if (st != NQS_OK) throw Error(st, std::string("batch_create: ") + nqs_last_error());
    b->sec_gen = model->sec_gen;
    NQS_REQUIRE(model->precision != NQS_BF16 || fused_supported(*model), NQS_EUNSUPPORTED,
                "batch_create: model shape not supported by the fused kernel");
    auto up = [](DevBuf &d, const void *src, size_t bytes) {
      HIP_OK(hipMemcpy(d.reserve(bytes), src, bytes, hipMemcpyHostToDevice));
    };
    up(b->tabs, b->tabs_host.data(), b->tabs_host.size() * sizeof(MolTab));
    up(b->flip, flip.data(), flip.size() * 8);
    up(b->goff, goff.data(), goff.size() * 8);
    up(b->zmask, zmask.data(), std::max<size_t>(zmask.size(), 1) * 8);
    up(b->coef, coef.data(), std::max<size_t>(coef.size(), 1) * 8);
    b->sums.reserve(size_t(n_mol) * 32);
    b->desc.reserve(sizeof(StepDesc));
    b->ctr.reserve(sizeof(Counters));
    HIP_OK(hipHostMalloc(reinterpret_cast<void **>(&b->desc_host), sizeof(StepDesc),
                         hipHostMallocDefault));
    HIP_OK(hipEventCreate(&b->ev0));
    HIP_OK(hipEventCreate(&b->ev1));
    *out = b.release();
  });
}

extern "C" void batch_destroy(nqs_batch *b) { delete b; }

extern "C" int batch_info(const nqs_batch *b, int64_t *k_per_config, int64_t *n_groups) {
  return guarded([&] {
    NQS_REQUIRE(b, NQS_EINVAL, "batch_info: null handle");
    for (int i = 0; i < b->n_mol; ++i) {
      if (k_per_config) k_per_config[i] = b->tabs_host[size_t(i)].K;
      if (n_groups) n_groups[i] = b->tabs_host[size_t(i)].G;
    }
  });
}

extern "C" int batch_set_mode(nqs_batch *b, int use_graph, int retune) {
  return guarded([&] {
    NQS_REQUIRE(b, NQS_EINVAL, "batch_set_mode: null handle");
    b->use_graph = use_graph != 0;
    if (retune) b->tuned = false;
    drop_graph(*b);
  });
}

extern "C" int batch_set_tile(nqs_batch *b, int pairs_blocks, int fused_pairs, int fused_blocks) {
  return guarded([&] {
    NQS_REQUIRE(b, NQS_EINVAL, "batch_set_tile: null handle");
    NQS_REQUIRE(pairs_blocks >= 1 && fused_pairs >= 1 && fused_pairs <= 16 && fused_blocks >= 1,
                NQS_EINVAL, "batch_set_tile: blocks >= 1, 1 <= pairs <= 16");
    b->pairs_blocks = pairs_blocks;
    b->xp_tile = FusedTile{fused_pairs, fused_blocks};
    b->tuned = true;
    drop_graph(*b);
  });
}

extern "C" int batch_set_table(nqs_batch *b, int64_t slots) {
  return guarded([&] {
    NQS_REQUIRE(b, NQS_EINVAL, "batch_set_table: null handle");
    NQS_REQUIRE(slots == 0 || (slots >= 1024 && slots <= (int64_t(1) << 31) &&
                               (slots & (slots - 1)) == 0),
                NQS_EINVAL, "batch_set_table: 0 or a power of two in 1024 .. 2^31");
    b->t_override = slots;
    if (slots == 0) b->t_size = 0;   // automatic size again at the next call
  });
}

extern "C" int batch_local_energy(nqs_batch *b, const uint64_t *x, const uint64_t *counts,
                                  const int64_t *offsets, const double *logabs_x,
                                  const double *phase_x, double *eloc, double *sums,
                                  int64_t *n_pairs, nqs_stream stream) {
  return guarded([&] {
    NQS_REQUIRE(b && offsets && sums, NQS_EINVAL, "batch_local_energy: null argument");
    NQS_REQUIRE((logabs_x == nullptr) == (phase_x == nullptr), NQS_EINVAL,
                "batch_local_energy: give both or neither of logabs_x, phase_x");
    nqs_model &m = *b->model;
    NQS_REQUIRE(m.tagged && int(m.sec_host.size()) == b->n_mol, NQS_EINVAL,
                "batch_local_energy: the model no longer serves this batch's molecules");
    if (m.sec_gen != b->sec_gen) {
      // the model's sector tables were reinstalled (another batch_create or
      // amp_model_set_sectors): they must still be this batch's molecules, and
      // the captured sequence, which holds the old tables' addresses, is dropped
      for (int i = 0; i < b->n_mol; ++i) {
        const nqs_sector_info &si = m.sec_host[size_t(i)];
        const MolTab &t = b->tabs_host[size_t(i)];
        NQS_REQUIRE(si.n == t.n && si.na == t.na && si.nb == t.nb, NQS_EINVAL,
                    "batch_local_energy: the model's sectors are now another batch's molecules");
      }
      drop_graph(*b);
      b->sec_gen = m.sec_gen;
    }
    hipStream_t s = as_stream(stream);
    StepDesc &d = *b->desc_host;
    HIP_OK(hipStreamSynchronize(s));   // the pinned descriptor of the previous call is free
    NQS_REQUIRE(offsets[0] == 0, NQS_EINVAL, "batch_local_energy: offsets[0] != 0");
    int64_t P = 0;
    for (int i = 0; i < b->n_mol; ++i) {
      NQS_REQUIRE(offsets[i + 1] >= offsets[i], NQS_EINVAL,
                  "batch_local_energy: offsets not ascending");
      d.u_off[i] = offsets[i];
      d.p_off[i] = P;
      P += (offsets[i + 1] - offsets[i]) * b->tabs_host[size_t(i)].K;
    }
    const int64_t U = offsets[b->n_mol];
    d.u_off[b->n_mol] = U;
    d.p_off[b->n_mol] = P;
    d.U = U;
    d.P = P;
    if (n_pairs) *n_pairs = P;
    b->last_pairs = P;
    NQS_REQUIRE(U == 0 || (x && counts && eloc), NQS_EINVAL, "batch_local_energy: null array");
    for (int attempt = 0;; ++attempt) {
    reserve(*b, std::max<int64_t>(U, 1), std::max<int64_t>(P, 1));
    HIP_OK(hipMemcpyAsync(b->desc.ptr, &d, sizeof(StepDesc), hipMemcpyHostToDevice, s));
    if (U > 0) {
      HIP_OK(hipMemcpyAsync(b->x.ptr, x, size_t(U) * 8, hipMemcpyDeviceToDevice, s));
      HIP_OK(hipMemcpyAsync(b->cnt.ptr, counts, size_t(U) * 8, hipMemcpyDeviceToDevice, s));
    }
    const bool psi_x = logabs_x == nullptr;
    if (!psi_x && U > 0) {
      HIP_OK(hipMemcpyAsync(b->lax.ptr, logabs_x, size_t(U) * 8, hipMemcpyDeviceToDevice, s));
      HIP_OK(hipMemcpyAsync(b->phx.ptr, phase_x, size_t(U) * 8, hipMemcpyDeviceToDevice, s));
    }
    if (m.precision == NQS_BF16) {
      if (!b->tuned && U > 0) {
        enqueue(*b, psi_x, s);     // fills the buffers the tuner times on
        tune(*b, s);
      }
      if (b->use_graph) {
        if (!b->exec || b->graph_has_psi_x != psi_x) capture(*b, psi_x);
        HIP_OK(hipGraphLaunch(b->exec, s));
      } else {
        enqueue(*b, psi_x, s);
      }
    } else {
      // FP32 / FP64 models: the layer-by-layer network needs host-side sizes
      auto *desc = b->desc.as<StepDesc>();
      auto *ctr = b->ctr.as<Counters>();
      hipLaunchKernelGGL(clear_kernel, dim3(2048), dim3(256), 0, s, b->table.as<uint64_t>(),
                         b->t_size, ctr);
      HIP_LAUNCH_OK();
      hipLaunchKernelGGL(pairs_kernel, dim3(unsigned(b->pairs_blocks)), dim3(256), 0, s, desc,
                         b->tabs.as<MolTab>(), b->flip.as<uint64_t>(), b->goff.as<int64_t>(),
                         b->zmask.as<uint64_t>(), b->coef.as<double>(), b->x.as<uint64_t>(),
                         b->n_mol, b->nbits, b->table.as<uint64_t>(), b->ids.as<uint32_t>(),
                         uint64_t(b->t_size - 1), b->ukeys.as<uint64_t>(), b->slot.as<uint32_t>(),
                         b->hval.as<double>(), b->hdiag.as<double>(), ctr);
      HIP_LAUNCH_OK();
      Counters c{};
      HIP_OK(hipMemcpyAsync(&c, ctr, sizeof(Counters), hipMemcpyDeviceToHost, s));
      HIP_OK(hipStreamSynchronize(s));
      if (psi_x && U > 0)
        model_forward(m, b->x.as<uint64_t>(), U, b->lax.as<double>(), b->phx.as<double>(),
                      nullptr, s);
      if (c.distinct > 0)
        model_forward(m, b->ukeys.as<uint64_t>(), c.distinct, b->la.as<double>(),
                      b->ph.as<double>(), nullptr, s);
      hipLaunchKernelGGL(accumulate_kernel<double>, dim3(unsigned(b->acc_blocks)), dim3(256), 0, s,
                         desc,
                         b->tabs.as<MolTab>(), b->x.as<uint64_t>(), b->n_mol,
                         b->slot.as<uint32_t>(),
                         b->ids.as<uint32_t>(), b->hval.as<double>(), b->la.as<double>(),
                         b->ph.as<double>(), b->lax.as<double>(), b->phx.as<double>(),
                         b->hdiag.as<double>(), b->eloc.as<double>());
      HIP_LAUNCH_OK();
      hipLaunchKernelGGL(reduce_kernel, dim3(unsigned(b->n_mol)), dim3(256), 0, s, desc,
                         b->eloc.as<double>(), b->cnt.as<uint64_t>(), b->sums.as<double>());
      HIP_LAUNCH_OK();
    }
    auto *per_mol = static_cast<unsigned long long *>(b->per_mol.reserve(kMaxMol * 8));
    hipLaunchKernelGGL(zero_u64_kernel, dim3(1), dim3(kMaxMol), 0, s, per_mol, kMaxMol);
    HIP_LAUNCH_OK();
    hipLaunchKernelGGL(count_mol_kernel, dim3(256), dim3(256), 0, s, b->ukeys.as<uint64_t>(),
                       b->ctr.as<Counters>(), b->n_mol, per_mol);
    HIP_LAUNCH_OK();
    b->distinct_per_mol.assign(size_t(b->n_mol), 0);
    HIP_OK(hipMemcpyAsync(b->distinct_per_mol.data(), per_mol, size_t(b->n_mol) * 8,
                          hipMemcpyDeviceToHost, s));
    Counters c{};
    HIP_OK(hipMemcpyAsync(&c, b->ctr.ptr, sizeof(Counters), hipMemcpyDeviceToHost, s));
    HIP_OK(hipStreamSynchronize(s));
    if ((c.overflow & 2) && attempt < 3) {
      // the table was too small for this step's distinct x': enlarge, run again
      b->est_distinct = std::max<int64_t>(4 * b->est_distinct, c.distinct * 2 + 1);
      b->t_override = 0;
      continue;
    }
    if (U > 0)
      HIP_OK(hipMemcpyAsync(eloc, b->eloc.ptr, size_t(U) * 16, hipMemcpyDeviceToDevice, s));
    HIP_OK(hipMemcpyAsync(sums, b->sums.ptr, size_t(b->n_mol) * 32, hipMemcpyDeviceToDevice, s));
    HIP_OK(hipStreamSynchronize(s));
    b->last_distinct = c.distinct;
    if (m.precision == NQS_BF16 && U > 0 && timing_on()) {
      float ms = 0.f;
      HIP_OK(hipEventElapsedTime(&ms, b->ev0, b->ev1));
      timing_add(ms, c.distinct);
    }
    NQS_REQUIRE(c.overflow == 0, NQS_EINVAL,
                "batch_local_energy: a configuration's molecule disagrees with the offsets, or it "
                "had more connected x' than its molecule's K, or the distinct-x' table overflowed");
    break;
    }
  });
}

extern "C" int batch_stats(const nqs_batch *b, int64_t *n_pairs, int64_t *n_distinct,
                           int64_t *distinct_per_mol, int64_t *captures, int32_t *tile,
                           double *tune_ms, int n_tune) {
  return guarded([&] {
    NQS_REQUIRE(b, NQS_EINVAL, "batch_stats: null handle");
    if (distinct_per_mol)
      for (int i = 0; i < b->n_mol; ++i)
        distinct_per_mol[i] = size_t(i) < b->distinct_per_mol.size() ? b->distinct_per_mol[size_t(i)] : 0;
    if (n_pairs) *n_pairs = b->last_pairs;
    if (n_distinct) *n_distinct = b->last_distinct;
    if (captures) *captures = b->captures;
    if (tile) {
      tile[0] = b->pairs_blocks;
      tile[1] = b->xp_tile.pairs;
      tile[2] = b->xp_tile.blocks;
    }
    if (tune_ms)
      for (int i = 0; i < n_tune && i < int(b->tune_ms.size()); ++i) tune_ms[i] = b->tune_ms[size_t(i)];
  });
}

extern "C" int vmc_weights_batch(const double *eloc, const uint64_t *counts, const uint64_t *x,
                                 int64_t n, const double *sums, int n_mol, double *g_logabs,
                                 double *g_phase, nqs_stream stream) {
  return guarded([&] {
    NQS_REQUIRE(n >= 0, NQS_EINVAL, "vmc_weights_batch: negative n");
    if (n == 0) return;
    NQS_REQUIRE(eloc && counts && x && sums && g_logabs && g_phase, NQS_EINVAL,
                "vmc_weights_batch: null pointer");
    NQS_REQUIRE(n_mol >= 1 && n_mol <= kMaxMol, NQS_EINVAL, "vmc_weights_batch: 1..64 molecules");
    hipLaunchKernelGGL(weights_kernel, g1(n), dim3(256), 0, as_stream(stream), eloc, counts, x, n,
                       n_mol, sums, g_logabs, g_phase);
    HIP_LAUNCH_OK();
  });
}
