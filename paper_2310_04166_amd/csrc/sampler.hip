// Autoregressive statistics sampling with symmetry pruning (paper:
// "Autoregressive statistics sampling"; "Pruning strategies"; Algorithm 1 for
// the physicality table).
//
// The whole tree walk stays on the GPU: per level, the model gives the four
// logits of every frontier node, one thread per node splits the node's samples
// over its children with sequential conditional binomials, and a scan
// compacts the children that received samples into the next frontier (children
// of node i in order k = 0..3, so the frontier stays in tree order).
//
// Random numbers are Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11) keyed
// by the 64-bit seed with counter (prefix lo32, prefix hi32, level + 64 j,
// block), j being which of the node's three binomials is drawn.  Binomials:
// inversion by sequential search for n p < 10, otherwise BTRS (W. Hormann,
// J. Statist. Comput. Simul. 46, 1993).  All of this is double precision
// without contraction, so a draw depends only on (seed, node, logits).
#include <cmath>
#include <vector>

#include "ham.h"
#include "model.h"

#pragma clang fp contract(off)

namespace nqs {
namespace {

constexpr uint32_t kM0 = 0xD2511F53u, kM1 = 0xCD9E8D57u;
constexpr uint32_t kW0 = 0x9E3779B9u, kW1 = 0xBB67AE85u;
constexpr uint64_t kAlphaBits = 0x5555555555555555ull;
constexpr uint64_t kBetaBits = 0xAAAAAAAAAAAAAAAAull;

struct Uniforms {
  uint32_t c0, c1, c2, c3, k0, k1;
  double buf[2];
  int nbuf;

  __device__ Uniforms(uint64_t seed, uint64_t prefix, int level, int j)
      : c0(uint32_t(prefix)), c1(uint32_t(prefix >> 32)), c2(uint32_t(level + 64 * j)), c3(0),
        k0(uint32_t(seed)), k1(uint32_t(seed >> 32)), nbuf(0) {}

  __device__ static double unit(uint32_t hi, uint32_t lo) {
    return ((double(hi >> 6) * 67108864.0 + double(lo >> 6)) + 0.5) * (1.0 / 4503599627370496.0);
  }

  __device__ double operator()() {
    if (nbuf == 0) {
      uint32_t x0 = c0, x1 = c1, x2 = c2, x3 = c3, a = k0, b = k1;
      for (int r = 0; r < 10; ++r) {
        if (r) {
          a += kW0;
          b += kW1;
        }
        const uint64_t p0 = uint64_t(kM0) * x0, p1 = uint64_t(kM1) * x2;
        const uint32_t y0 = uint32_t(p1 >> 32) ^ x1 ^ a, y1 = uint32_t(p1);
        const uint32_t y2 = uint32_t(p0 >> 32) ^ x3 ^ b, y3 = uint32_t(p0);
        x0 = y0; x1 = y1; x2 = y2; x3 = y3;
      }
      ++c3;
      buf[0] = unit(x2, x3);  // second draw of the block
      buf[1] = unit(x0, x1);  // first draw of the block
      nbuf = 2;
    }
    return buf[--nbuf];
  }
};

__device__ double log_factorial(int64_t k) {
  if (k < 10) {
    double f = 1.0;
    for (int64_t i = 2; i <= k; ++i) f *= double(i);
    return log(f);
  }
  const double k1 = double(k) + 1.0;
  const double r = 1.0 / (k1 * k1);
  return (((double(k) + 0.5) * log(k1) - k1) + 0.5 * log(2.0 * 3.141592653589793)) +
         (1.0 / 12.0 - (1.0 / 360.0 - (1.0 / 1260.0) * r) * r) / k1;
}

__device__ int64_t binomial_inversion(int64_t n, double p, Uniforms &uni) {
  const double q = 1.0 - p;
  const double s = p / q;
  const double a = double(n + 1) * s;
  const double r0 = pow(q, double(n));
  while (true) {
    double r = r0;
    double u = uni();
    int64_t k = 0;
    while (u >= r) {
      u -= r;
      ++k;
      if (k > n) break;
      r *= a / double(k) - s;
    }
    if (k <= n) return k;
  }
}

__device__ int64_t binomial_btrs(int64_t n, double p, Uniforms &uni) {
  const double q = 1.0 - p;
  const double spq = sqrt((double(n) * p) * q);
  const double b = 1.15 + 2.53 * spq;
  const double a = (-0.0873 + 0.0248 * b) + 0.01 * p;
  const double c = double(n) * p + 0.5;
  const double vr = 0.92 - 4.2 / b;
  const double alpha = (2.83 + 5.1 / b) * spq;
  const double lpq = log(p / q);
  const int64_t m = int64_t(floor(double(n + 1) * p));
  const double h = log_factorial(m) + log_factorial(n - m);
  while (true) {
    const double u = uni() - 0.5;
    double v = uni();
    const double us = 0.5 - fabs(u);
    const double kf = floor(((2.0 * a) / us + b) * u + c);
    if (kf < 0.0 || kf > double(n)) continue;
    const int64_t k = int64_t(kf);
    if (us >= 0.07 && v <= vr) return k;
    v = log((v * alpha) / (a / (us * us) + b));
    if (v <= ((h - log_factorial(k)) - log_factorial(n - k)) + double(k - m) * lpq) return k;
  }
}

__device__ int64_t binomial(int64_t n, double p, Uniforms &uni) {
  if (n == 0 || p <= 0.0) return 0;
  if (p >= 1.0) return n;
  const bool flip = p > 0.5;
  const double pp = flip ? 1.0 - p : p;
  const int64_t k = (double(n) * pp < 10.0) ? binomial_inversion(n, pp, uni)
                                            : binomial_btrs(n, pp, uni);
  return flip ? n - k : k;
}

// One thread per frontier node: split its samples over the four tokens.  A
// node whose molecule has no token at level p (a smaller molecule of a batch)
// passes all its samples to child 0, which is the same configuration word.
// With `count` (device) the frontier holds *count nodes of capacity B, and
// the threads past them clear their children so that the scan over the
// capacity sees zeros.
__global__ void split_kernel(const uint64_t *__restrict__ prefix, const uint64_t *__restrict__ cnt,
                             const double *__restrict__ logits, int64_t B,
                             const int64_t *__restrict__ count, int p, Sectors S,
                             uint64_t seed, uint64_t *__restrict__ child,
                             uint64_t *__restrict__ flag, unsigned long long *__restrict__ lost) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= B) return;
  if (count && i >= *count) {
    for (int k = 0; k < 4; ++k) {
      child[4 * i + k] = 0;
      flag[4 * i + k] = 0;
    }
    return;
  }
  const uint64_t x = prefix[i];
  const nqs_sector_info si = sector_of(S, x);
  if (p >= si.n) {
    for (int k = 0; k < 4; ++k) {
      child[4 * i + k] = k == 0 ? cnt[i] : 0;
      flag[4 * i + k] = k == 0 ? 1 : 0;
    }
    return;
  }
  const uint64_t occ = occupation(S, x);
  const int a = __popcll(occ & kAlphaBits), b = __popcll(occ & kBetaBits);
  const int ph = phys_mask(S, si, p, a, b, occ);
  const int allow = p < si.mask_levels ? ph : 0xF;
  const double *l = logits + 4 * i;
  double mx = -INFINITY;
  for (int k = 0; k < 4; ++k)
    if ((allow >> k) & 1) mx = fmax(mx, l[k]);
  double e[4];
  for (int k = 0; k < 4; ++k) e[k] = ((allow >> k) & 1) ? exp(l[k] - mx) : 0.0;
  int64_t out[4] = {0, 0, 0, 0};
  int64_t rest = int64_t(cnt[i]);
  for (int k = 0; k < 3; ++k) {
    if (rest == 0) break;
    double tail = e[k];
    for (int j = k + 1; j < 4; ++j) tail = tail + e[j];
    if (e[k] == tail) {
      out[k] = rest;
    } else {
      Uniforms uni(seed, x, p, k);
      out[k] = binomial(rest, e[k] / tail, uni);
    }
    rest -= out[k];
  }
  out[3] += rest;
  unsigned long long dropped = 0;
  for (int k = 0; k < 4; ++k) {
    if (!((ph >> k) & 1)) {
      dropped += uint64_t(out[k]);
      out[k] = 0;
    }
    child[4 * i + k] = uint64_t(out[k]);
    flag[4 * i + k] = out[k] > 0 ? 1 : 0;
  }
  if (dropped) atomicAdd(lost, dropped);
}

// (next_count, optional: the number of children, off[B4], for the next level)
__global__ void compact_kernel(const uint64_t *__restrict__ prefix,
                               const uint64_t *__restrict__ child, const int64_t *__restrict__ off,
                               int64_t B4, int p, uint64_t *__restrict__ npre,
                               uint64_t *__restrict__ ncnt, int64_t *__restrict__ next_count) {
  const int64_t j = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (next_count && j == 0) *next_count = off[B4];
  if (j >= B4) return;
  const uint64_t c = child[j];
  if (c == 0) return;
  const int k = int(j & 3);
  const int64_t o = off[j];
  npre[o] = prefix[j >> 2] | (uint64_t(k) << (2 * p));
  ncnt[o] = c;
}

__global__ void init_kernel(unsigned long long *lost) { *lost = 0; }
__global__ void zero_f64_kernel(double *__restrict__ p, int64_t n) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0.0;
}
// The conditional logits of level p.  At the last level of a sector that
// leaves one token there (every level masked) the split sends all counts to
// that token whatever the logits, so the network is not evaluated: finite
// zeros stand in for them.
bool level_is_fixed(const nqs_model &m, int p) { return p == m.n - 1 && last_token_fixed(m); }

// The first levels: row p of a configuration depends on its tokens 0..p-1
// only, so one evaluation of every (P-1)-token prefix (P = 7: 4,096 words)
// gives the conditionals of levels 0..P-1 for every node there, each level
// then a lookup instead of a network pass of its own (the same arithmetic per
// row, so the same logits).  Fused bf16 transformers of one molecule.
int early_levels(const nqs_model &m) {
  return m.kind == NQS_MODEL_TRANSFORMER && m.precision == NQS_BF16 && !m.tagged &&
                 fused_supported(m)
             ? std::min(7, m.n - 1)
             : 0;
}
__global__ void iota_u64_kernel(uint64_t *__restrict__ w, int64_t n) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < n) w[i] = uint64_t(i);
}
// cond of level p < P for the frontier: the node's word holds tokens 0..p-1
// and zeros beyond, so it is its own index among the (P-1)-token prefixes
__global__ void early_cond_kernel(const uint64_t *__restrict__ pre, int64_t B,
                                  const int64_t *__restrict__ count,
                                  const double *__restrict__ early, int P, int p, uint64_t mask,
                                  double *__restrict__ cond) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= B || (count && i >= *count)) return;
  const int64_t idx = int64_t(pre[i] & mask);
  for (int k = 0; k < 4; ++k) cond[4 * i + k] = early[(idx * P + p) * 4 + k];
}
void zero_logits(double *cond, int64_t B, hipStream_t s) {
  hipLaunchKernelGGL(zero_f64_kernel, dim3(unsigned(ceil_div(4 * B, 256))), dim3(256), 0, s, cond,
                     4 * B);
  HIP_LAUNCH_OK();
}

// offsets[i] = first leaf of molecule i (leaves are grouped by molecule in
// ascending order); offsets[n_mol] = B.
__global__ void mol_offsets_kernel(const uint64_t *__restrict__ leaves, int64_t B, int n_mol,
                                   int64_t *__restrict__ offsets) {
  const int i = int(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i > n_mol) return;
  int64_t lo = 0, hi = B;
  while (lo < hi) {
    const int64_t mid = (lo + hi) / 2;
    if (int(leaves[mid] >> kTagShift) < i) lo = mid + 1;
    else hi = mid;
  }
  offsets[i] = lo;
}

// Expands the trees whose roots (configuration word, samples) are given, all
// levels together; returns the number of leaves, left in m.s_pre/s_cnt[cur].
int64_t walk_trees(nqs_model &m, const std::vector<uint64_t> &root_pre,
                   const std::vector<uint64_t> &root_cnt, uint64_t seed, int &cur,
                   uint64_t &lost_out, hipStream_t s) {
  int64_t B = int64_t(root_pre.size());
  auto *lost_d = static_cast<unsigned long long *>(m.s_lost.reserve(8));
  cur = 0;
  m.s_pre[0].reserve(size_t(B > 0 ? B : 1) * 8);
  m.s_cnt[0].reserve(size_t(B > 0 ? B : 1) * 8);
  hipLaunchKernelGGL(init_kernel, dim3(1), dim3(1), 0, s, lost_d);
  HIP_LAUNCH_OK();
  if (B > 0) {
    HIP_OK(hipMemcpyAsync(m.s_pre[0].ptr, root_pre.data(), size_t(B) * 8, hipMemcpyHostToDevice, s));
    HIP_OK(hipMemcpyAsync(m.s_cnt[0].ptr, root_cnt.data(), size_t(B) * 8, hipMemcpyHostToDevice, s));
  }
  for (int p = 0; p < m.n && B > 0; ++p) {
    double *cond = static_cast<double *>(m.s_cond.reserve(size_t(B) * 4 * 8));
    if (level_is_fixed(m, p)) zero_logits(cond, B, s);
    else model_cond_logits(m, m.s_pre[cur].as<uint64_t>(), B, p, cond, s);
    auto *child = static_cast<uint64_t *>(m.s_child.reserve(size_t(B) * 4 * 8));
    auto *flag = static_cast<int64_t *>(m.s_flag.reserve(size_t(B) * 4 * 8));
    auto *off = static_cast<int64_t *>(m.s_off.reserve(size_t(B * 4 + 1) * 8));
    hipLaunchKernelGGL(split_kernel, dim3(unsigned(ceil_div(B, 256))), dim3(256), 0, s,
                       m.s_pre[cur].as<uint64_t>(), m.s_cnt[cur].as<uint64_t>(), cond, B,
                       nullptr, p, m.sectors(), seed, child, reinterpret_cast<uint64_t *>(flag),
                       lost_d);
    HIP_LAUNCH_OK();
    launch_exclusive_scan(flag, off, B * 4, s, m.s_scan);
    int64_t nb = 0;
    HIP_OK(hipMemcpyAsync(&nb, off + B * 4, 8, hipMemcpyDeviceToHost, s));
    HIP_OK(hipStreamSynchronize(s));
    const int nxt = 1 - cur;
    m.s_pre[nxt].reserve(size_t(nb > 0 ? nb : 1) * 8);
    m.s_cnt[nxt].reserve(size_t(nb > 0 ? nb : 1) * 8);
    hipLaunchKernelGGL(compact_kernel, dim3(unsigned(ceil_div(B * 4, 256))), dim3(256), 0, s,
                       m.s_pre[cur].as<uint64_t>(), child, off, B * 4, p,
                       m.s_pre[nxt].as<uint64_t>(), m.s_cnt[nxt].as<uint64_t>(), nullptr);
    HIP_LAUNCH_OK();
    cur = nxt;
    B = nb;
  }
  uint64_t lost_h = 0;
  HIP_OK(hipMemcpyAsync(&lost_h, lost_d, 8, hipMemcpyDeviceToHost, s));
  HIP_OK(hipStreamSynchronize(s));
  lost_out = lost_h;
  return B;
}

// The same walk with the frontier sizes kept on the device: every level's
// arrays are sized by a bound (four children per node, at most one node per
// sample) and its kernels read the node count from the device, so the host
// waits once, after the last level, instead of once per level.  For models
// whose conditionals take a device count (the fused bf16 kernels); results are
// those of walk_trees (the random numbers are keyed by node, not by position).
constexpr int64_t kDeviceWalkMax = int64_t(1) << 24;   // frontier bound (nodes)
bool g_device_walk = true;                             // nqs_sampler_device_walk

bool device_walk_ok(const nqs_model &m, uint64_t total) {
  return g_device_walk && m.precision == NQS_BF16 &&
         (fused_supported(m) || nade_fused_supported(m)) && total <= uint64_t(kDeviceWalkMax);
}

int64_t walk_trees_device(nqs_model &m, const std::vector<uint64_t> &root_pre,
                          const std::vector<uint64_t> &root_cnt, uint64_t seed, int &cur,
                          uint64_t &lost_out, hipStream_t s) {
  const int64_t B0 = int64_t(root_pre.size());
  uint64_t total = 0;
  for (uint64_t c : root_cnt) total += c;
  // frontier bounds per level
  std::vector<int64_t> cap(size_t(m.n) + 1);
  cap[0] = B0;
  int64_t cmax = std::max<int64_t>(B0, 1);
  for (int p = 0; p < m.n; ++p) {
    cap[size_t(p + 1)] = std::min<int64_t>(4 * cap[size_t(p)], int64_t(total));
    cmax = std::max(cmax, cap[size_t(p + 1)]);
  }
  auto *lost_d = static_cast<unsigned long long *>(m.s_lost.reserve(8 + 8 * size_t(m.n + 1)));
  int64_t *nb_d = reinterpret_cast<int64_t *>(lost_d + 1);   // node count of each level
  cur = 0;
  for (int k = 0; k < 2; ++k) {
    m.s_pre[k].reserve(size_t(cmax) * 8);
    m.s_cnt[k].reserve(size_t(cmax) * 8);
  }
  auto *cond = static_cast<double *>(m.s_cond.reserve(size_t(cmax) * 4 * 8));
  auto *child = static_cast<uint64_t *>(m.s_child.reserve(size_t(cmax) * 4 * 8));
  auto *flag = static_cast<int64_t *>(m.s_flag.reserve(size_t(cmax) * 4 * 8));
  auto *off = static_cast<int64_t *>(m.s_off.reserve(size_t(cmax * 4 + 1) * 8));
  hipLaunchKernelGGL(init_kernel, dim3(1), dim3(1), 0, s, lost_d);
  HIP_LAUNCH_OK();
  if (B0 > 0) {
    HIP_OK(hipMemcpyAsync(m.s_pre[0].ptr, root_pre.data(), size_t(B0) * 8, hipMemcpyHostToDevice, s));
    HIP_OK(hipMemcpyAsync(m.s_cnt[0].ptr, root_cnt.data(), size_t(B0) * 8, hipMemcpyHostToDevice, s));
  }
  // the conditionals of levels 0..P-1 for every prefix of P-1 tokens
  const int P = early_levels(m);
  const int64_t n_early = P > 0 ? int64_t(1) << (2 * (P - 1)) : 0;
  double *early = nullptr;
  if (P > 0) {
    auto *words = static_cast<uint64_t *>(
        m.s_early.reserve(size_t(n_early) * 8 + size_t(n_early) * size_t(P) * 4 * 8));
    early = reinterpret_cast<double *>(words + n_early);
    hipLaunchKernelGGL(iota_u64_kernel, dim3(unsigned(ceil_div(n_early, 256))), dim3(256), 0, s,
                       words, n_early);
    HIP_LAUNCH_OK();
    fused_forward(m, words, n_early, nullptr, nullptr, early, -P, s, nullptr);
  }
  int64_t last = 0;   // level whose count is the result
  for (int p = 0; p < m.n && cap[size_t(p)] > 0; ++p) {
    const int64_t B = cap[size_t(p)];
    const int64_t *count = p == 0 ? nullptr : nb_d + p;   // level 0: B0 nodes (host)
    if (level_is_fixed(m, p)) {
      zero_logits(cond, B, s);
    } else if (p < P) {
      hipLaunchKernelGGL(early_cond_kernel, dim3(unsigned(ceil_div(B, 256))), dim3(256), 0, s,
                         m.s_pre[cur].as<uint64_t>(), B, count, early, P, p,
                         (uint64_t(1) << (2 * (P - 1))) - 1, cond);
      HIP_LAUNCH_OK();
    } else {
      fused_forward(m, m.s_pre[cur].as<uint64_t>(), B, nullptr, nullptr, cond, p, s, count);
    }
    hipLaunchKernelGGL(split_kernel, dim3(unsigned(ceil_div(B, 256))), dim3(256), 0, s,
                       m.s_pre[cur].as<uint64_t>(), m.s_cnt[cur].as<uint64_t>(), cond, B, count,
                       p, m.sectors(), seed, child, reinterpret_cast<uint64_t *>(flag), lost_d);
    HIP_LAUNCH_OK();
    launch_exclusive_scan(flag, off, B * 4, s, m.s_scan);
    const int nxt = 1 - cur;
    hipLaunchKernelGGL(compact_kernel, dim3(unsigned(ceil_div(B * 4, 256))), dim3(256), 0, s,
                       m.s_pre[cur].as<uint64_t>(), child, off, B * 4, p,
                       m.s_pre[nxt].as<uint64_t>(), m.s_cnt[nxt].as<uint64_t>(), nb_d + p + 1);
    HIP_LAUNCH_OK();
    cur = nxt;
    last = p + 1;
  }
  uint64_t host[2] = {0, 0};
  HIP_OK(hipMemcpyAsync(&host[0], lost_d, 8, hipMemcpyDeviceToHost, s));
  if (last > 0) HIP_OK(hipMemcpyAsync(&host[1], nb_d + last, 8, hipMemcpyDeviceToHost, s));
  HIP_OK(hipStreamSynchronize(s));
  lost_out = host[0];
  return last > 0 ? int64_t(host[1]) : B0;
}

void copy_leaves(nqs_model &m, int cur, int64_t B, int64_t capacity, uint64_t *configs,
                 uint64_t *counts, hipStream_t s) {
  NQS_REQUIRE(B <= capacity, NQS_ECAPACITY, "sampler: capacity too small");
  NQS_REQUIRE(B == 0 || (configs && counts), NQS_EINVAL, "sampler: null output");
  if (B > 0) {
    HIP_OK(hipMemcpyAsync(configs, m.s_pre[cur].ptr, size_t(B) * 8, hipMemcpyDeviceToDevice, s));
    HIP_OK(hipMemcpyAsync(counts, m.s_cnt[cur].ptr, size_t(B) * 8, hipMemcpyDeviceToDevice, s));
  }
}

}  // namespace
}  // namespace nqs

using namespace nqs;

extern "C" int nqs_sampler_device_walk(int on) {
  return guarded([&] { g_device_walk = on != 0; });
}

extern "C" int sample_unique(nqs_model *m, uint64_t n_samples, uint64_t seed, uint64_t *configs,
                             uint64_t *counts, int64_t capacity, int64_t *n_unique, uint64_t *lost,
                             nqs_stream stream) {
  return guarded([&] {
    NQS_REQUIRE(m && n_unique, NQS_EINVAL, "sample_unique: null argument");
    NQS_REQUIRE(capacity >= 0, NQS_EINVAL, "sample_unique: negative capacity");
    NQS_REQUIRE(!m->tagged, NQS_EINVAL,
                "sample_unique: the model serves several molecules (use sample_unique_batch)");
    hipStream_t s = as_stream(stream);
    std::vector<uint64_t> pre, cnt;
    if (n_samples > 0) {
      pre.push_back(0);
      cnt.push_back(n_samples);
    }
    int cur = 0;
    uint64_t lost_h = 0;
    const int64_t B = device_walk_ok(*m, n_samples)
                          ? walk_trees_device(*m, pre, cnt, seed, cur, lost_h, s)
                          : walk_trees(*m, pre, cnt, seed, cur, lost_h, s);
    if (lost) *lost = lost_h;
    *n_unique = B;
    copy_leaves(*m, cur, B, capacity, configs, counts, s);
  });
}

extern "C" int sample_unique_batch(nqs_model *m, int n_mol, const uint64_t *n_samples,
                                   uint64_t seed, uint64_t *configs, uint64_t *counts,
                                   int64_t capacity, int64_t *n_unique, int64_t *offsets,
                                   uint64_t *lost, nqs_stream stream) {
  return guarded([&] {
    NQS_REQUIRE(m && n_unique && n_samples && offsets, NQS_EINVAL,
                "sample_unique_batch: null argument");
    NQS_REQUIRE(capacity >= 0, NQS_EINVAL, "sample_unique_batch: negative capacity");
    NQS_REQUIRE(m->tagged && n_mol == int(m->sec_host.size()), NQS_EINVAL,
                "sample_unique_batch: n_mol differs from the model's molecules");
    hipStream_t s = as_stream(stream);
    std::vector<uint64_t> pre, cnt;
    for (int i = 0; i < n_mol; ++i)
      if (n_samples[i] > 0) {
        pre.push_back(uint64_t(i) << kTagShift);
        cnt.push_back(n_samples[i]);
      }
    int cur = 0;
    uint64_t lost_h = 0;
    uint64_t total = 0;
    for (uint64_t c : cnt) total += c;
    const int64_t B = device_walk_ok(*m, total)
                          ? walk_trees_device(*m, pre, cnt, seed, cur, lost_h, s)
                          : walk_trees(*m, pre, cnt, seed, cur, lost_h, s);
    if (lost) *lost = lost_h;
    *n_unique = B;
    int64_t *off_d = static_cast<int64_t *>(m->s_off.reserve(size_t(n_mol + 1) * 8));
    hipLaunchKernelGGL(mol_offsets_kernel, dim3(unsigned(ceil_div(n_mol + 1, 64))), dim3(64), 0,
                       s, m->s_pre[cur].as<uint64_t>(), B, n_mol, off_d);
    HIP_LAUNCH_OK();
    HIP_OK(hipMemcpyAsync(offsets, off_d, size_t(n_mol + 1) * 8, hipMemcpyDeviceToHost, s));
    HIP_OK(hipStreamSynchronize(s));
    copy_leaves(*m, cur, B, capacity, configs, counts, s);
  });
}
