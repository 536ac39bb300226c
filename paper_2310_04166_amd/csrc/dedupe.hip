// Distinct connected configurations of a slice of (x, x') pairs.  Many sampled
// x share connected x' (they cluster around the dominant determinants), and
// psi(x') does not depend on which x it is connected to, so the amplitude
// network runs once per distinct x' (the local-energy sum itself is unchanged).
//
// keys = x' of every pair; radix sort (key, pair index) over the 2n used bits;
// a head flag marks the first of each run of equal keys; an inclusive scan of
// the flags numbers the runs; run heads write the distinct keys in ascending
// order and every pair learns its run number through the sorted pair index.
// Optionally (pm >= 16) the bits are reordered before sorting - bits 0..15
// most significant, then bits 16 .. pm-1, then the rest - and restored in the
// output, so that the distinct x' come out grouped by their first 8 tokens and
// within those by their first pm / 2 tokens (the prefix-shared forward reads
// one prefix's keys and values for consecutive configurations); pm = -1 orders
// tokens 8, 9, ... lexicographically after the first 8, so that the x' sharing
// any prefix of 8 or more tokens are consecutive.
#include <algorithm>

#include <hipcub/hipcub.hpp>

#include "common.h"

namespace nqs {
namespace {

__global__ void iota_kernel(uint32_t *v, int64_t n) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < n) v[i] = uint32_t(i);
}

__host__ __device__ inline uint64_t low_bits(int b) { return b >= 64 ? ~0ull : (1ull << b) - 1; }
// x' -> sort key (fields [0,16), [16,pm), [pm,N) to [N-16,N), [N-pm,N-16), [0,N-pm))
__device__ inline uint64_t prefix_key(uint64_t v, int N, int pm) {
  return ((v & 0xFFFFull) << (N - 16)) | (((v >> 16) & low_bits(pm - 16)) << (N - pm)) | (v >> pm);
}
__device__ inline uint64_t prefix_key_inverse(uint64_t k, int N, int pm) {
  return (k >> (N - 16)) | (((k >> (N - pm)) & low_bits(pm - 16)) << 16) |
         ((k & low_bits(N - pm)) << pm);
}
// the w 2-bit tokens of v in reverse order (an involution)
__device__ inline uint64_t reverse_tokens(uint64_t v, int w) {
  uint64_t r = 0;
  for (int i = 0; i < w; ++i) r |= ((v >> (2 * i)) & 3ull) << (2 * (w - 1 - i));
  return r;
}
// pm = -1: bits 0..15 most significant, then token 8, token 9, ... in that
// order of significance, so every prefix of 8 or more tokens is contiguous
__device__ inline uint64_t token_key(uint64_t v, int N) {
  return ((v & 0xFFFFull) << (N - 16)) | reverse_tokens(v >> 16, (N - 16) / 2);
}
__device__ inline uint64_t token_key_inverse(uint64_t k, int N) {
  return (k >> (N - 16)) | (reverse_tokens(k & low_bits(N - 16), (N - 16) / 2) << 16);
}
__device__ inline uint64_t sort_key(uint64_t v, int N, int pm) {
  return pm > 0 ? prefix_key(v, N, pm) : pm < 0 ? token_key(v, N) : v;
}
__device__ inline uint64_t sort_key_inverse(uint64_t k, int N, int pm) {
  return pm > 0 ? prefix_key_inverse(k, N, pm) : pm < 0 ? token_key_inverse(k, N) : k;
}
__global__ void prefix_key_kernel(uint64_t *__restrict__ k, int64_t n, int key_bits, int pm) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < n) k[i] = sort_key(k[i], key_bits, pm);
}

// keys of at most 32 bits: the (reordered) key of every pair as uint32
__global__ void narrow_key_kernel(const uint64_t *__restrict__ xp, int64_t n, int key_bits, int pm,
                                  uint32_t *__restrict__ k) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < n) k[i] = uint32_t(sort_key(xp[i], key_bits, pm));
}

template <class K>
__global__ void head_kernel(const K *__restrict__ keys, int64_t n, uint32_t *__restrict__ head) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < n) head[i] = (i == 0 || keys[i] != keys[i - 1]) ? 1u : 0u;
}

template <class K>
__global__ void scatter_kernel(const K *__restrict__ keys, const uint32_t *__restrict__ vals,
                               const uint32_t *__restrict__ head, const uint32_t *__restrict__ run,
                               int64_t n, int key_bits, int pm, uint64_t *__restrict__ ukeys,
                               uint32_t *__restrict__ pair_uid) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const uint32_t id = run[i] - 1u;
  if (head[i]) ukeys[id] = sort_key_inverse(uint64_t(keys[i]), key_bits, pm);
  pair_uid[vals[i]] = id;
}

inline dim3 g1(int64_t n) { return dim3(unsigned(ceil_div(n, 256))); }

}  // namespace

// Returns the number of distinct keys U; ukeys[0..U) ascending (in the
// reordered key when pm > 0), pair_uid[p] = index of xp[p] in ukeys.  All
// buffers are caller-provided workspaces sized for n pairs; tmp is grown as
// needed.  Keys of at most 32 bits are sorted as uint32 (in the two halves of
// keys_sorted; xp is left as it is), wider keys as uint64 (xp reordered in
// place when pm > 0).
int64_t dedupe_pairs(uint64_t *xp, int64_t n, int key_bits, int pm, uint64_t *keys_sorted,
                     uint32_t *vals_in, uint32_t *vals_sorted, uint32_t *head, uint32_t *run,
                     uint64_t *ukeys, uint32_t *pair_uid, DevBuf &tmp, hipStream_t s) {
  if (n <= 0) return 0;
  NQS_REQUIRE(n < (int64_t(1) << 31), NQS_EUNSUPPORTED, "dedupe: slice too large");
  NQS_REQUIRE(pm == 0 || (pm >= 16 && pm < key_bits) || (pm == -1 && key_bits > 16 && key_bits % 2 == 0),
              NQS_EINVAL, "dedupe: prefix fields");
  const int ni = int(n);
  hipLaunchKernelGGL(iota_kernel, g1(n), dim3(256), 0, s, vals_in, n);
  HIP_LAUNCH_OK();
  size_t sort_bytes = 0, scan_bytes = 0;
  if (key_bits <= 32) {
    uint32_t *k_in = reinterpret_cast<uint32_t *>(keys_sorted), *k_out = k_in + n;
    hipLaunchKernelGGL(narrow_key_kernel, g1(n), dim3(256), 0, s, xp, n, key_bits, pm, k_in);
    HIP_LAUNCH_OK();
    HIP_OK(hipcub::DeviceRadixSort::SortPairs(nullptr, sort_bytes, k_in, k_out, vals_in,
                                              vals_sorted, ni, 0, key_bits, s));
    HIP_OK(hipcub::DeviceScan::InclusiveSum(nullptr, scan_bytes, head, run, ni, s));
    void *t = tmp.reserve(std::max(sort_bytes, scan_bytes) + 256);
    HIP_OK(hipcub::DeviceRadixSort::SortPairs(t, sort_bytes, k_in, k_out, vals_in, vals_sorted,
                                              ni, 0, key_bits, s));
    hipLaunchKernelGGL(head_kernel<uint32_t>, g1(n), dim3(256), 0, s, k_out, n, head);
    HIP_LAUNCH_OK();
    HIP_OK(hipcub::DeviceScan::InclusiveSum(t, scan_bytes, head, run, ni, s));
    hipLaunchKernelGGL(scatter_kernel<uint32_t>, g1(n), dim3(256), 0, s, k_out, vals_sorted, head,
                       run, n, key_bits, pm, ukeys, pair_uid);
    HIP_LAUNCH_OK();
    uint32_t u = 0;
    HIP_OK(hipMemcpyAsync(&u, run + (n - 1), 4, hipMemcpyDeviceToHost, s));
    HIP_OK(hipStreamSynchronize(s));
    return int64_t(u);
  }
  if (pm != 0) {
    hipLaunchKernelGGL(prefix_key_kernel, g1(n), dim3(256), 0, s, xp, n, key_bits, pm);
    HIP_LAUNCH_OK();
  }
  HIP_OK(hipcub::DeviceRadixSort::SortPairs(nullptr, sort_bytes, xp, keys_sorted, vals_in,
                                            vals_sorted, ni, 0, key_bits, s));
  HIP_OK(hipcub::DeviceScan::InclusiveSum(nullptr, scan_bytes, head, run, ni, s));
  void *t = tmp.reserve(std::max(sort_bytes, scan_bytes) + 256);
  HIP_OK(hipcub::DeviceRadixSort::SortPairs(t, sort_bytes, xp, keys_sorted, vals_in, vals_sorted,
                                            ni, 0, key_bits, s));
  hipLaunchKernelGGL(head_kernel<uint64_t>, g1(n), dim3(256), 0, s, keys_sorted, n, head);
  HIP_LAUNCH_OK();
  HIP_OK(hipcub::DeviceScan::InclusiveSum(t, scan_bytes, head, run, ni, s));
  hipLaunchKernelGGL(scatter_kernel<uint64_t>, g1(n), dim3(256), 0, s, keys_sorted, vals_sorted,
                     head, run, n, key_bits, pm, ukeys, pair_uid);
  HIP_LAUNCH_OK();
  uint32_t u = 0;
  HIP_OK(hipMemcpyAsync(&u, run + (n - 1), 4, hipMemcpyDeviceToHost, s));
  HIP_OK(hipStreamSynchronize(s));
  return int64_t(u);
}

}  // namespace nqs
