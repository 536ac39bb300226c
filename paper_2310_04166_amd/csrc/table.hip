// The network-free amplitude: psi(x) given explicitly on a basis of
// configurations (paper: "Variational Monte Carlo", local-energy equation --
// with psi the exact ground vector, E_loc(x) = E_0 for every x, the
// zero-variance property).  Parameters are log|psi| and phi of every basis
// configuration; any configuration outside the basis has psi = 0.
//
//   amp_forward  binary search of x in the basis sorted by uint64 value;
//   sampler      the conditional of token p after a prefix is the Born mass of
//                the basis configurations that continue prefix + token,
//                divided by the prefix's mass (the product rule written for an
//                explicit psi); masses are differences of prefix sums of
//                |psi|^2 over the basis sorted in tree order (token 0 most
//                significant), so each is two binary searches;
//   backward     d log|psi(x_l)| / d logabs_i = [x_l = basis_i], the same for
//                the phase: the upstream weights are added to the entry of x_l.
#include <algorithm>
#include <cmath>
#include <vector>

#include "model.h"
#include "ops.h"

namespace nqs {
namespace {

// tree key: tokens in reverse order, so that token 0 is the most significant
// 2-bit digit of a 2n-bit number (lexicographic in tokens = numeric)
__host__ __device__ inline uint64_t tree_key(uint64_t x, int n) {
  uint64_t k = 0;
  for (int p = 0; p < n; ++p) k |= ((x >> (2 * p)) & 3ull) << (2 * (n - 1 - p));
  return k;
}

// first index in a[0..M) with a[i] >= v
__device__ inline int64_t lower_bound(const uint64_t *a, int64_t M, uint64_t v) {
  int64_t lo = 0, hi = M;
  while (lo < hi) {
    const int64_t mid = lo + (hi - lo) / 2;
    if (a[mid] < v) lo = mid + 1;
    else hi = mid;
  }
  return lo;
}

__global__ void table_forward_kernel(const uint64_t *__restrict__ basis, int64_t M,
                                     const double *__restrict__ P, const uint64_t *__restrict__ x,
                                     int64_t B, double *__restrict__ logabs,
                                     double *__restrict__ phase) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= B) return;
  const uint64_t v = x[i];
  const int64_t j = lower_bound(basis, M, v);
  const bool hit = j < M && basis[j] == v;
  if (logabs) logabs[i] = hit ? P[j] : -INFINITY;
  if (phase) phase[i] = hit ? P[M + j] : 0.0;
}

// cum[0] = 0, cum[k+1] = sum_{j <= k} exp(2 (logabs[idx[j]] - max)): one block,
// each thread a contiguous chunk, fixed order; cum[M + 1] = max.
__global__ void __launch_bounds__(1024) table_cum_kernel(const double *__restrict__ P,
                                                         const int64_t *__restrict__ idx,
                                                         int64_t M, double *__restrict__ cum) {
  __shared__ double part[1024];
  const int t = threadIdx.x;
  double mx = -INFINITY;
  for (int64_t j = t; j < M; j += 1024) mx = fmax(mx, P[j]);
  part[t] = mx;
  __syncthreads();
  for (int s = 512; s > 0; s >>= 1) {
    if (t < s) part[t] = fmax(part[t], part[t + s]);
    __syncthreads();
  }
  mx = part[0];
  __syncthreads();
  const int64_t chunk = (M + 1023) / 1024, j0 = t * chunk, j1 = j0 + chunk < M ? j0 + chunk : M;
  double s = 0.0;
  for (int64_t j = j0; j < j1; ++j) s += exp(2.0 * (P[idx[j]] - mx));
  part[t] = s;
  __syncthreads();
  double base = 0.0;
  for (int k = 0; k < t; ++k) base += part[k];
  for (int64_t j = j0; j < j1; ++j) {
    base += exp(2.0 * (P[idx[j]] - mx));
    cum[j + 1] = base;
  }
  if (t == 0) {
    cum[0] = 0.0;
    cum[M + 1] = mx;
  }
}

// log of the Born mass of prefix (tokens 0..p-1 of x) followed by token k, for
// k = 0..3 (-inf for an empty range)
__global__ void table_cond_kernel(const uint64_t *__restrict__ tkeys, const double *__restrict__ cum,
                                  int64_t M, int n, const uint64_t *__restrict__ prefix, int64_t B,
                                  int p, double *__restrict__ out4) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= B * 4) return;
  const int64_t b = i / 4;
  const int k = int(i % 4);
  const uint64_t below = p == 0 ? 0ull : (~0ull >> (64 - 2 * p));
  const uint64_t head = tree_key((prefix[b] & below) | (uint64_t(k) << (2 * p)), n);
  const int shift = 2 * (n - 1 - p);           // digits of the tokens after p
  const uint64_t lo_key = head, hi_key = head + (1ull << shift);
  const int64_t lo = lower_bound(tkeys, M, lo_key);
  // at 64 qubits the range of the largest prefix ends at 2^64 (the sum wraps)
  const int64_t hi = hi_key < lo_key ? M : lower_bound(tkeys, M, hi_key);
  const double mass = cum[hi] - cum[lo];
  out4[i] = mass > 0.0 ? log(mass) : -INFINITY;
}

__global__ void table_backward_kernel(const uint64_t *__restrict__ basis, int64_t M,
                                      const uint64_t *__restrict__ x, int64_t B,
                                      const double *__restrict__ gl, const double *__restrict__ gp,
                                      double *__restrict__ acc) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= B) return;
  const uint64_t v = x[i];
  const int64_t j = lower_bound(basis, M, v);
  if (j < M && basis[j] == v) {
    atomicAdd(acc + j, gl[i]);
    atomicAdd(acc + M + j, gp[i]);
  }
}

inline dim3 grid1(int64_t n) { return dim3(unsigned(ceil_div(n, 256))); }

}  // namespace

void table_install(nqs_model &m, const uint64_t *basis, int64_t M) {
  NQS_REQUIRE(M >= 1, NQS_EINVAL, "table: empty basis");
  const uint64_t occ = m.n >= 32 ? ~0ull : ((1ull << (2 * m.n)) - 1);
  for (int64_t j = 0; j < M; ++j) {
    NQS_REQUIRE(j == 0 || basis[j] > basis[j - 1], NQS_EINVAL,
                "table: basis not strictly ascending");
    NQS_REQUIRE((basis[j] & ~occ) == 0, NQS_EINVAL, "table: configuration beyond the qubits");
  }
  std::vector<uint64_t> keys(size_t(M), 0);
  std::vector<int64_t> order(size_t(M), 0);
  for (int64_t j = 0; j < M; ++j) {
    keys[size_t(j)] = tree_key(basis[j], m.n);
    order[size_t(j)] = j;
  }
  std::sort(order.begin(), order.end(),
            [&](int64_t a, int64_t b) { return keys[size_t(a)] < keys[size_t(b)]; });
  std::vector<uint64_t> tkeys(static_cast<size_t>(M));
  for (int64_t j = 0; j < M; ++j) tkeys[size_t(j)] = keys[size_t(order[size_t(j)])];
  m.tab_M = M;
  HIP_OK(hipMemcpy(m.tab_basis.reserve(size_t(M) * 8), basis, size_t(M) * 8, hipMemcpyHostToDevice));
  HIP_OK(hipMemcpy(m.tab_tkeys.reserve(size_t(M) * 8), tkeys.data(), size_t(M) * 8,
                   hipMemcpyHostToDevice));
  HIP_OK(hipMemcpy(m.tab_order.reserve(size_t(M) * 8), order.data(), size_t(M) * 8,
                   hipMemcpyHostToDevice));
}

void table_pack(nqs_model &m, hipStream_t s) {
  double *cum = static_cast<double *>(m.tab_cum.reserve(size_t(m.tab_M + 2) * 8));
  hipLaunchKernelGGL(table_cum_kernel, dim3(1), dim3(1024), 0, s, m.master.as<double>(),
                     m.tab_order.as<int64_t>(), m.tab_M, cum);
  HIP_LAUNCH_OK();
}

void table_forward(nqs_model &m, const uint64_t *x, int64_t B, double *logabs, double *phase,
                   hipStream_t s) {
  if (B <= 0) return;
  hipLaunchKernelGGL(table_forward_kernel, grid1(B), dim3(256), 0, s, m.tab_basis.as<uint64_t>(),
                     m.tab_M, m.master.as<double>(), x, B, logabs, phase);
  HIP_LAUNCH_OK();
}

void table_cond_logits(nqs_model &m, const uint64_t *prefix, int64_t B, int p, double *out4,
                       hipStream_t s) {
  if (B <= 0) return;
  hipLaunchKernelGGL(table_cond_kernel, grid1(B * 4), dim3(256), 0, s, m.tab_tkeys.as<uint64_t>(),
                     m.tab_cum.as<double>(), m.tab_M, m.n, prefix, B, p, out4);
  HIP_LAUNCH_OK();
}

void table_backward(nqs_model &m, const uint64_t *x, int64_t B, const double *gl,
                    const double *gp, double *acc, hipStream_t s) {
  if (B <= 0) return;
  hipLaunchKernelGGL(table_backward_kernel, grid1(B), dim3(256), 0, s, m.tab_basis.as<uint64_t>(),
                     m.tab_M, x, B, gl, gp, acc);
  HIP_LAUNCH_OK();
}

}  // namespace nqs
