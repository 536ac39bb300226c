// Layer-by-layer building blocks (see ops.h).  These kernels favour clarity:
// they serve the FP64 and FP32 forward modes, every backward pass and the
// sampler's conditionals in those modes; the bf16 forward has its own fused
// kernel.
#include "ops.h"

#include "act.h"

#include <hipblaslt/hipblaslt.h>
#include <rocblas/rocblas.h>

#include <array>
#include <type_traits>
#include <functional>
#include <map>

namespace nqs {
namespace {

// Epilogue of the library GEMM: bias and activation, in place on C (M x N, ldc).
template <class T>
__global__ void epilogue_kernel(T *C, int64_t M, int64_t N, int64_t ldc, const T *bias, T *aux,
                                int epi) {
  const int64_t idx = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (idx >= M * N) return;
  const int64_t i = idx / N, j = idx % N;
  T *c = C + i * ldc + j;
  const T v = *c + (bias ? bias[j] : T(0));
  switch (epi) {
    case EPI_GELU: aux[i * ldc + j] = v; *c = gelu_tanh(v); break;
    case EPI_TANH: *c = tanh(v); break;
    case EPI_LRELU: aux[i * ldc + j] = v; *c = v >= T(0) ? v : T(0.01) * v; break;
    default: *c = v;
  }
}

template <class T>
__global__ void add_into_kernel(const T *src, int64_t n, double *dst) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < n) dst[i] += double(src[i]);
}

template <class T>
__global__ void fill_kernel(T *dst, int64_t n, T v) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < n) dst[i] = v;
}

#define BLAS_OK(expr)                                                                   \
  do {                                                                                  \
    rocblas_status st_ = (expr);                                                        \
    if (st_ != rocblas_status_success)                                                  \
      throw Error(NQS_EHIP, std::string(#expr " failed: ") + rocblas_status_to_string(st_)); \
  } while (0)

rocblas_handle blas(hipStream_t s) {
  static rocblas_handle handles[64] = {};
  int dev = 0;
  HIP_OK(hipGetDevice(&dev));
  NQS_REQUIRE(dev >= 0 && dev < 64, NQS_EHIP, "device index out of range");
  if (!handles[dev]) BLAS_OK(rocblas_create_handle(&handles[dev]));
  BLAS_OK(rocblas_set_stream(handles[dev], s));
  return handles[dev];
}

// FP32 GEMMs: rocBLAS or hipBLASLt (FP32 compute), whichever is faster for the
// call's shape.  On the first call of a shape bucket both are timed (rocBLAS and
// up to eight hipBLASLt algorithms from its heuristic, each once after a warm-up,
// into a scratch output) and the fastest is kept for the bucket; hipBLASLt's kernels for the
// backward's weight-gradient shapes (reductions over ~1e5 token rows) are
// several times faster than rocBLAS's, its first heuristic choice for narrow
// outputs is several times slower.
struct GemmChoice {
  bool lt = false;
  hipblasLtMatmulDesc_t desc = nullptr;
  hipblasLtMatrixLayout_t la = nullptr, lb = nullptr, lc = nullptr;
  hipblasLtMatmulAlgo_t algo{};
};

struct LtState {
  hipblasLtHandle_t handle = nullptr;
  DevBuf ws, scratch;
  std::map<std::array<int, 9>, GemmChoice> plans;   // exact shapes
  // timing decisions per shape bucket (dimensions rounded up to powers of two, so
  // the ragged last chunk of a step reuses them): -1 = rocBLAS, r = hipBLASLt's
  // r-th heuristic algorithm
  std::map<std::array<int, 9>, int> decisions;
};

int pow2_ceil(int v) {
  int p = 1;
  while (p < v) p <<= 1;
  return p;
}

constexpr size_t kLtWorkspace = size_t(64) << 20;

LtState &lt_state() {
  static LtState states[64];
  int dev = 0;
  HIP_OK(hipGetDevice(&dev));
  NQS_REQUIRE(dev >= 0 && dev < 64, NQS_EHIP, "device index out of range");
  LtState &st = states[dev];
  if (!st.handle) {
    if (hipblasLtCreate(&st.handle) != HIPBLAS_STATUS_SUCCESS)
      throw Error(NQS_EHIP, "hipblasLtCreate failed");
    st.ws.reserve(kLtWorkspace);
  }
  return st;
}

float time_call(hipStream_t s, const std::function<bool()> &f) {
  hipEvent_t e0, e1;
  HIP_OK(hipEventCreate(&e0));
  HIP_OK(hipEventCreate(&e1));
  float ms = -1.f;
  if (f()) {                       // warm-up; also checks the call is accepted
    HIP_OK(hipEventRecord(e0, s));
    const bool ok = f();
    HIP_OK(hipEventRecord(e1, s));
    HIP_OK(hipEventSynchronize(e1));
    if (ok) HIP_OK(hipEventElapsedTime(&ms, e0, e1));
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  return ms;
}

const GemmChoice &choose_gemm(LtState &st, rocblas_handle h, rocblas_operation ta,
                              rocblas_operation tb, int m, int n, int k, const float *A, int lda,
                              const float *B, int ldb, float beta, int ldc, hipStream_t s) {
  const bool tA = ta == rocblas_operation_transpose, tB = tb == rocblas_operation_transpose;
  const std::array<int, 9> key{int(tA), int(tB), m, n, k, lda, ldb, ldc, int(beta != 0.f)};
  auto it = st.plans.find(key);
  if (it != st.plans.end()) return it->second;
  const std::array<int, 9> bucket{int(tA), int(tB), pow2_ceil(m), pow2_ceil(n), pow2_ceil(k),
                                  tA ? pow2_ceil(lda) : lda, tB ? pow2_ceil(ldb) : ldb, ldc,
                                  int(beta != 0.f)};
  auto dit = st.decisions.find(bucket);
  const int decided = dit == st.decisions.end() ? -2 : dit->second;
  GemmChoice c;
  float *C = static_cast<float *>(st.scratch.reserve(size_t(ldc) * size_t(n) * 4));
  const float alpha = 1.f;
  int best_rank = -1;
  float best = 1e30f;
  if (decided == -2) {
    best = time_call(s, [&] {
      return rocblas_sgemm(h, ta, tb, m, n, k, &alpha, A, lda, B, ldb, &beta, C, ldc) ==
             rocblas_status_success;
    });
    if (best < 0.f) best = 1e30f;
  }
  const hipblasOperation_t opa = tA ? HIPBLAS_OP_T : HIPBLAS_OP_N, opb = tB ? HIPBLAS_OP_T : HIPBLAS_OP_N;
  bool good = hipblasLtMatmulDescCreate(&c.desc, HIPBLAS_COMPUTE_32F, HIP_R_32F) == HIPBLAS_STATUS_SUCCESS &&
              hipblasLtMatmulDescSetAttribute(c.desc, HIPBLASLT_MATMUL_DESC_TRANSA, &opa, sizeof(opa)) == HIPBLAS_STATUS_SUCCESS &&
              hipblasLtMatmulDescSetAttribute(c.desc, HIPBLASLT_MATMUL_DESC_TRANSB, &opb, sizeof(opb)) == HIPBLAS_STATUS_SUCCESS &&
              hipblasLtMatrixLayoutCreate(&c.la, HIP_R_32F, tA ? k : m, tA ? m : k, lda) == HIPBLAS_STATUS_SUCCESS &&
              hipblasLtMatrixLayoutCreate(&c.lb, HIP_R_32F, tB ? n : k, tB ? k : n, ldb) == HIPBLAS_STATUS_SUCCESS &&
              hipblasLtMatrixLayoutCreate(&c.lc, HIP_R_32F, m, n, ldc) == HIPBLAS_STATUS_SUCCESS;
  if (good) {
    hipblasLtMatmulPreference_t pref = nullptr;
    size_t wsb = kLtWorkspace;
    hipblasLtMatmulHeuristicResult_t res[8] = {};
    int got = 0;
    if (hipblasLtMatmulPreferenceCreate(&pref) == HIPBLAS_STATUS_SUCCESS &&
        hipblasLtMatmulPreferenceSetAttribute(pref, HIPBLASLT_MATMUL_PREF_MAX_WORKSPACE_BYTES, &wsb,
                                              sizeof(wsb)) == HIPBLAS_STATUS_SUCCESS &&
        hipblasLtMatmulAlgoGetHeuristic(st.handle, c.desc, c.la, c.lb, c.lc, c.lc, pref, 8, res,
                                        &got) == HIPBLAS_STATUS_SUCCESS) {
      if (decided >= 0 && decided < got) {
        c.lt = true;
        c.algo = res[decided].algo;
      } else if (decided == -2) {
        for (int a = 0; a < got; ++a) {
          const float ms = time_call(s, [&] {
            return hipblasLtMatmul(st.handle, c.desc, &alpha, A, c.la, B, c.lb, &beta, C, c.lc,
                                   C, c.lc, &res[a].algo, st.ws.ptr, kLtWorkspace, s) ==
                   HIPBLAS_STATUS_SUCCESS;
          });
          if (ms >= 0.f && ms < best) {
            best = ms;
            best_rank = a;
            c.lt = true;
            c.algo = res[a].algo;
          }
        }
      }
    }
    if (pref) hipblasLtMatmulPreferenceDestroy(pref);
  }
  if (decided == -2) st.decisions.emplace(bucket, best_rank);
  return st.plans.emplace(key, c).first->second;
}

void blas_gemm(rocblas_handle h, rocblas_operation ta, rocblas_operation tb, int m, int n, int k,
               float alpha, const float *A, int lda, const float *B, int ldb, float beta,
               float *C, int ldc, hipStream_t s) {
  // the library's kernels may assume 16-byte aligned operands
  const bool aligned = ((reinterpret_cast<uintptr_t>(A) | reinterpret_cast<uintptr_t>(B) |
                         reinterpret_cast<uintptr_t>(C)) & 15) == 0;
  if (aligned && alpha == 1.f) {
    LtState &st = lt_state();
    const GemmChoice &c = choose_gemm(st, h, ta, tb, m, n, k, A, lda, B, ldb, beta, ldc, s);
    if (c.lt) {
      if (hipblasLtMatmul(st.handle, c.desc, &alpha, A, c.la, B, c.lb, &beta, C, c.lc, C, c.lc,
                          &c.algo, st.ws.ptr, kLtWorkspace, s) != HIPBLAS_STATUS_SUCCESS)
        throw Error(NQS_EHIP, "hipblasLtMatmul failed");
      return;
    }
  }
  BLAS_OK(rocblas_sgemm(h, ta, tb, m, n, k, &alpha, A, lda, B, ldb, &beta, C, ldc));
}
void blas_gemm(rocblas_handle h, rocblas_operation ta, rocblas_operation tb, int m, int n, int k,
               double alpha, const double *A, int lda, const double *B, int ldb, double beta,
               double *C, int ldc, hipStream_t) {
  BLAS_OK(rocblas_dgemm(h, ta, tb, m, n, k, &alpha, A, lda, B, ldb, &beta, C, ldc));
}

// partial[y][j] = sum over rows of slice y of Y[r, j]; 64 columns x 4 row lanes
// per block, eight loads in flight per lane, a fixed summation order
template <class T>
__global__ void __launch_bounds__(256) colsum_kernel(const T *Y, int64_t R, int64_t N, int64_t ld,
                                                     int64_t rows_per, double *partial) {
  __shared__ double red[4][64];
  const int c = threadIdx.x % 64, q = threadIdx.x / 64;
  const int64_t j = int64_t(blockIdx.x) * 64 + c;
  const int64_t r0 = int64_t(blockIdx.y) * rows_per;
  const int64_t r1 = r0 + rows_per < R ? r0 + rows_per : R;
  double a = 0.0;
  if (j < N) {
    int64_t r = r0 + q;
    for (; r + 28 < r1; r += 32) {
      T v[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) v[u] = Y[(r + 4 * u) * ld + j];
#pragma unroll
      for (int u = 0; u < 8; ++u) a += double(v[u]);
    }
    for (; r < r1; r += 4) a += double(Y[r * ld + j]);
  }
  red[q][c] = a;
  __syncthreads();
  if (q == 0 && j < N)
    partial[int64_t(blockIdx.y) * N + j] = ((red[0][c] + red[1][c]) + red[2][c]) + red[3][c];
}

// First level of a slice reduction: out[g][i] = sum of part[z][i] over the
// slices z of group g (groups of zs consecutive slices); 64 elements x 4 slice
// lanes per block, a fixed summation order.
template <class P>
__global__ void __launch_bounds__(256) sum_slices_kernel(const P *part, int64_t nslices,
                                                         int64_t len, int64_t zs, double *out) {
  __shared__ double red[4][64];
  const int c = threadIdx.x % 64, q = threadIdx.x / 64;
  const int64_t i = int64_t(blockIdx.x) * 64 + c;
  const int64_t z0 = int64_t(blockIdx.y) * zs;
  const int64_t z1 = z0 + zs < nslices ? z0 + zs : nslices;
  double a = 0.0;
  if (i < len) {
    int64_t z = z0 + q;
    for (; z + 12 < z1; z += 16) {
      P v[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) v[u] = part[(z + 4 * u) * len + i];
#pragma unroll
      for (int u = 0; u < 4; ++u) a += double(v[u]);
    }
    for (; z < z1; z += 4) a += double(part[z * len + i]);
  }
  red[q][c] = a;
  __syncthreads();
  if (q == 0 && i < len)
    out[int64_t(blockIdx.y) * len + i] = ((red[0][c] + red[1][c]) + red[2][c]) + red[3][c];
}

// acc[i] += sum over slices z of part[z][i], in slice order
template <class P>
__global__ void slices_acc_kernel(const P *part, int64_t nslices, int64_t len, double *acc) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= len) return;
  double a = 0.0;
  int64_t z = 0;
  for (; z + 8 <= nslices; z += 8) {
    P v[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) v[u] = part[(z + u) * len + i];
#pragma unroll
    for (int u = 0; u < 8; ++u) a += double(v[u]);
  }
  for (; z < nslices; ++z) a += double(part[z * len + i]);
  acc[i] += a;
}

typedef __attribute__((ext_vector_type(16))) float f32x16;

// Weight-gradient partial sums on fp32 MFMA (32x32x2):
//     part[z][i][j] = sum over the rows r of slice z of X[r][i] * dY[r][j].
// One block per (128 x 128 output tile, row slice); wave w owns the 64 x 64
// quarter (w / 2, w % 2) as 2 x 2 accumulator blocks.  For a pair of rows the
// lane l supplies X[r + l/32][i0 + l%32] (A operand, k = l/32) and
// dY[r + l/32][j0 + l%32] (B operand); accumulator element v of lane l is
// (i0 + (v/4)*8 + (l/32)*4 + v%4, j0 + l%32).
// The slice's rows are read through buffer resources that end at the slice's
// last row, so rows past it read as zeros; columns outside the matrices read a
// clamped valid column, which only feeds accumulator rows / columns that are
// never stored.  The host keeps a slice under 2 GiB of either matrix.
__global__ void __launch_bounds__(256) wgrad_f32_kernel(const float *__restrict__ X, int64_t ldx,
                                                        const float *__restrict__ dY, int64_t ldy,
                                                        int64_t R, int M, int N, int64_t rows_per,
                                                        int tiles_n, float *__restrict__ part) {
  const int lane = threadIdx.x % 64, w = threadIdx.x / 64;
  const int tm = int(blockIdx.x) / tiles_n, tn = int(blockIdx.x) % tiles_n;
  const int i0 = tm * 128 + (w / 2) * 64, j0 = tn * 128 + (w % 2) * 64;
  const int64_t r0 = int64_t(blockIdx.y) * rows_per;
  const int64_t r1 = r0 + rows_per < R ? r0 + rows_per : R;
  const int rows = int(r1 - r0);
  const int kk = lane / 32, c = lane % 32;
  const int ia = i0 + c, ib = i0 + 32 + c, ja = j0 + c, jb = j0 + 32 + c;
  const auto rx = __builtin_amdgcn_make_buffer_rsrc(const_cast<float *>(X + r0 * ldx), 0,
                                                    int(int64_t(rows) * ldx * 4), 0x00020000);
  const auto ry = __builtin_amdgcn_make_buffer_rsrc(const_cast<float *>(dY + r0 * ldy), 0,
                                                    int(int64_t(rows) * ldy * 4), 0x00020000);
  const int lx = int(ldx) * 4, ly = int(ldy) * 4;   // bytes per row
  const int oxa = kk * lx + (ia < M ? ia : M - 1) * 4, oxb = kk * lx + (ib < M ? ib : M - 1) * 4;
  const int oya = kk * ly + (ja < N ? ja : N - 1) * 4, oyb = kk * ly + (jb < N ? jb : N - 1) * 4;
  f32x16 acc[2][2] = {};
  constexpr int U = 8;   // row pairs per batch of loads
  struct Batch {
    float a0[U], a1[U], b0[U], b1[U];
  };
  auto load = [&](int r, Batch &q) {   // rows r .. r + 2U - 1 of the slice
#pragma unroll
    for (int u = 0; u < U; ++u) {
      // row offsets in unsigned 32-bit arithmetic: a batch may run past the slice
      const int sx = int(uint32_t(r + 2 * u) * uint32_t(lx));
      const int sy = int(uint32_t(r + 2 * u) * uint32_t(ly));
      q.a0[u] = __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(rx, oxa, sx, 0));
      q.a1[u] = __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(rx, oxb, sx, 0));
      q.b0[u] = __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(ry, oya, sy, 0));
      q.b1[u] = __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(ry, oyb, sy, 0));
    }
  };
  auto multiply = [&](const Batch &q) {
#pragma unroll
    for (int u = 0; u < U; ++u) {
      acc[0][0] = __builtin_amdgcn_mfma_f32_32x32x2f32(q.a0[u], q.b0[u], acc[0][0], 0, 0, 0);
      acc[0][1] = __builtin_amdgcn_mfma_f32_32x32x2f32(q.a0[u], q.b1[u], acc[0][1], 0, 0, 0);
      acc[1][0] = __builtin_amdgcn_mfma_f32_32x32x2f32(q.a1[u], q.b0[u], acc[1][0], 0, 0, 0);
      acc[1][1] = __builtin_amdgcn_mfma_f32_32x32x2f32(q.a1[u], q.b1[u], acc[1][1], 0, 0, 0);
    }
  };
  // two batches in flight: the next batch loads while the current one
  // multiplies (a batch past the slice reads zeros and is never multiplied)
  const int nb = (rows + 2 * U - 1) / (2 * U);
  Batch p0, p1;
  load(0, p0);
  int bt = 0;
  for (; bt + 2 <= nb; bt += 2) {
    load((bt + 1) * 2 * U, p1);
    multiply(p0);
    load((bt + 2) * 2 * U, p0);
    multiply(p1);
  }
  if (bt < nb) multiply(p0);
  float *pz = part + int64_t(blockIdx.y) * M * N;
#pragma unroll
  for (int bi = 0; bi < 2; ++bi)
#pragma unroll
    for (int bj = 0; bj < 2; ++bj) {
      const int j = j0 + 32 * bj + c;
      if (j >= N) continue;
#pragma unroll
      for (int v = 0; v < 16; ++v) {
        const int i = i0 + 32 * bi + (v / 4) * 8 + kk * 4 + v % 4;
        if (i < M) pz[int64_t(i) * N + j] = acc[bi][bj][v];
      }
    }
}

// one wave per row
template <class T>
__global__ void __launch_bounds__(256) layernorm_kernel(const T *x, int64_t R, int d, const T *g,
                                                        const T *b, T *y, T *mean, T *rstd) {
  const int lane = threadIdx.x % 64;
  const int64_t r = int64_t(blockIdx.x) * 4 + threadIdx.x / 64;
  if (r >= R) return;
  const T *xr = x + r * d;
  T s = 0;
  for (int j = lane; j < d; j += 64) s += xr[j];
  for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o);
  const T mu = s / T(d);
  T v = 0;
  for (int j = lane; j < d; j += 64) v += (xr[j] - mu) * (xr[j] - mu);
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  const T rs = T(1) / sqrt(v / T(d) + T(1e-5));
  for (int j = lane; j < d; j += 64) y[r * d + j] = (xr[j] - mu) * rs * g[j] + b[j];
  if (lane == 0) {
    if (mean) mean[r] = mu;
    if (rstd) rstd[r] = rs;
  }
}

// d = 64 CPL: a wave normalises RPW consecutive rows, all their loads issued
// before the first reduction (lane: columns lane + 64 k); the same arithmetic
// as layernorm_kernel per row.
template <class T, int CPL, int RPW>
__global__ void __launch_bounds__(256) layernorm_rows_kernel(const T *__restrict__ x, int64_t R,
                                                             const T *__restrict__ g,
                                                             const T *__restrict__ b,
                                                             T *__restrict__ y, T *__restrict__ mean,
                                                             T *__restrict__ rstd) {
  constexpr int d = 64 * CPL;
  const int lane = threadIdx.x % 64;
  const int64_t r0 = (int64_t(blockIdx.x) * 4 + threadIdx.x / 64) * RPW;
  if (r0 >= R) return;
  T v[RPW][CPL];
#pragma unroll
  for (int q = 0; q < RPW; ++q)
#pragma unroll
    for (int k = 0; k < CPL; ++k) v[q][k] = r0 + q < R ? x[(r0 + q) * d + lane + 64 * k] : T(0);
#pragma unroll
  for (int q = 0; q < RPW; ++q) {
    if (r0 + q >= R) break;
    T sum = 0;
#pragma unroll
    for (int k = 0; k < CPL; ++k) sum += v[q][k];
    for (int o = 32; o > 0; o >>= 1) sum += __shfl_xor(sum, o);
    const T mu = sum / T(d);
    T var = 0;
#pragma unroll
    for (int k = 0; k < CPL; ++k) var += (v[q][k] - mu) * (v[q][k] - mu);
    for (int o = 32; o > 0; o >>= 1) var += __shfl_xor(var, o);
    const T rs = T(1) / sqrt(var / T(d) + T(1e-5));
#pragma unroll
    for (int k = 0; k < CPL; ++k) {
      const int j = lane + 64 * k;
      y[(r0 + q) * d + j] = (v[q][k] - mu) * rs * g[j] + b[j];
    }
    if (lane == 0) {
      if (mean) mean[r0 + q] = mu;
      if (rstd) rstd[r0 + q] = rs;
    }
  }
}

template <class T>
__global__ void __launch_bounds__(256) layernorm_bwd_kernel(const T *x, const T *mean,
                                                            const T *rstd, int64_t R, int d,
                                                            const T *g, const T *dy, T *dx,
                                                            bool accumulate, T *dyxh) {
  const int lane = threadIdx.x % 64;
  const int64_t r = int64_t(blockIdx.x) * 4 + threadIdx.x / 64;
  if (r >= R) return;
  const T mu = mean[r], rs = rstd[r];
  T s1 = 0, s2 = 0;
  for (int j = lane; j < d; j += 64) {
    const T xh = (x[r * d + j] - mu) * rs;
    const T gy = dy[r * d + j] * g[j];
    s1 += gy;
    s2 += gy * xh;
    if (dyxh) dyxh[r * d + j] = dy[r * d + j] * xh;
  }
  for (int o = 32; o > 0; o >>= 1) {
    s1 += __shfl_xor(s1, o);
    s2 += __shfl_xor(s2, o);
  }
  s1 /= T(d);
  s2 /= T(d);
  for (int j = lane; j < d; j += 64) {
    const T xh = (x[r * d + j] - mu) * rs;
    const T v = rs * (dy[r * d + j] * g[j] - s1 - xh * s2);
    dx[r * d + j] = accumulate ? dx[r * d + j] + v : v;
  }
}

// The layer-norm backward with its parameters' gradients: rows of a block's
// contiguous range taken by its four waves in turn (wave w: rows w, w + 4, ..,
// two at a time),
// each lane owning columns lane + 64 k (k < CPL); per-lane double sums of
// dy * xhat (gain) and dy (bias) over the rows, combined over the waves in
// order into gpart[block][j], bpart[block][j].
template <class T, int CPL>
__global__ void __launch_bounds__(256) layernorm_bwd_acc_kernel(
    const T *__restrict__ x, const T *__restrict__ mean, const T *__restrict__ rstd, int64_t R,
    int64_t rows_per, const T *__restrict__ g, const T *__restrict__ dy, T *__restrict__ dx,
    bool accumulate, double *__restrict__ gpart, double *__restrict__ bpart) {
  constexpr int d = 64 * CPL;
  __shared__ double red[2][4][d];
  const int lane = threadIdx.x % 64, w = threadIdx.x / 64;
  const int64_t r0 = int64_t(blockIdx.x) * rows_per;
  const int64_t r1 = r0 + rows_per < R ? r0 + rows_per : R;
  double ga[CPL], ba[CPL];
  T gj[CPL];
#pragma unroll
  for (int k = 0; k < CPL; ++k) {
    ga[k] = ba[k] = 0.0;
    gj[k] = g[lane + 64 * k];
  }
  // two rows (r, r + 4) per iteration, every load of both issued first
  for (int64_t r = r0 + w; r < r1; r += 8) {
    constexpr int RW = 2;
    T xv[RW][CPL], dyv[RW][CPL], dxo[RW][CPL], mu[RW], rs[RW];
    bool in[RW];
#pragma unroll
    for (int q = 0; q < RW; ++q) {
      const int64_t rq = r + 4 * q;
      in[q] = rq < r1;
      mu[q] = in[q] ? mean[rq] : T(0);
      rs[q] = in[q] ? rstd[rq] : T(0);
#pragma unroll
      for (int k = 0; k < CPL; ++k) {
        const int64_t e = rq * d + lane + 64 * k;
        xv[q][k] = in[q] ? x[e] : T(0);
        dyv[q][k] = in[q] ? dy[e] : T(0);
        dxo[q][k] = in[q] && accumulate ? dx[e] : T(0);
      }
    }
#pragma unroll
    for (int q = 0; q < RW; ++q) {
      if (!in[q]) continue;
      const int64_t rq = r + 4 * q;
      T xh[CPL], s1 = 0, s2 = 0;
#pragma unroll
      for (int k = 0; k < CPL; ++k) {
        xh[k] = (xv[q][k] - mu[q]) * rs[q];
        const T gy = dyv[q][k] * gj[k];
        s1 += gy;
        s2 += gy * xh[k];
        ga[k] += double(dyv[q][k] * xh[k]);
        ba[k] += double(dyv[q][k]);
      }
      for (int o = 32; o > 0; o >>= 1) {
        s1 += __shfl_xor(s1, o);
        s2 += __shfl_xor(s2, o);
      }
      s1 /= T(d);
      s2 /= T(d);
#pragma unroll
      for (int k = 0; k < CPL; ++k) {
        const T v = rs[q] * (dyv[q][k] * gj[k] - s1 - xh[k] * s2);
        dx[rq * d + lane + 64 * k] = accumulate ? dxo[q][k] + v : v;
      }
    }
  }
#pragma unroll
  for (int k = 0; k < CPL; ++k) {
    red[0][w][lane + 64 * k] = ga[k];
    red[1][w][lane + 64 * k] = ba[k];
  }
  __syncthreads();
  for (int j = threadIdx.x; j < d; j += 256) {
    gpart[int64_t(blockIdx.x) * d + j] = ((red[0][0][j] + red[0][1][j]) + red[0][2][j]) + red[0][3][j];
    bpart[int64_t(blockIdx.x) * d + j] = ((red[1][0][j] + red[1][1][j]) + red[1][2][j]) + red[1][3][j];
  }
}

// One 64-lane block per (sequence, head); T_ <= 32, dh <= 64.
template <class T>
__global__ void __launch_bounds__(64) attention_fwd_kernel(const T *qkv, int T_, int d, int H,
                                                           T *o, T *probs) {
  const int64_t b = blockIdx.x / H;
  const int h = blockIdx.x % H, dh = d / H;
  __shared__ T q[32][65], k[32][65], v[32][65];
  const T *base = qkv + b * T_ * 3 * d;
  for (int idx = threadIdx.x; idx < T_ * dh; idx += 64) {
    const int t = idx / dh, j = idx % dh;
    q[t][j] = base[t * 3 * d + h * dh + j];
    k[t][j] = base[t * 3 * d + d + h * dh + j];
    v[t][j] = base[t * 3 * d + 2 * d + h * dh + j];
  }
  __syncthreads();
  const int t = threadIdx.x;
  if (t >= T_) return;
  const T scale = T(1) / sqrt(T(dh));
  T sc[32];
  T mx = T(-1e300);
  for (int s = 0; s <= t; ++s) {
    T a = 0;
    for (int j = 0; j < dh; ++j) a += q[t][j] * k[s][j];
    sc[s] = a * scale;
    mx = sc[s] > mx ? sc[s] : mx;
  }
  T z = 0;
  for (int s = 0; s <= t; ++s) {
    sc[s] = exp(sc[s] - mx);
    z += sc[s];
  }
  for (int s = 0; s <= t; ++s) sc[s] /= z;
  if (probs) {
    T *pr = probs + ((b * H + h) * T_ + t) * T_;
    for (int s = 0; s < T_; ++s) pr[s] = s <= t ? sc[s] : T(0);
  }
  T *orow = o + (b * T_ + t) * d + h * dh;
  for (int j = 0; j < dh; ++j) {
    T a = 0;
    for (int s = 0; s <= t; ++s) a += sc[s] * v[s][j];
    orow[j] = a;
  }
}

template <class T>
__global__ void __launch_bounds__(64) attention_bwd_kernel(const T *qkv, const T *probs,
                                                           const T *dout, int T_, int d, int H,
                                                           T *dqkv) {
  const int64_t b = blockIdx.x / H;
  const int h = blockIdx.x % H, dh = d / H;
  __shared__ T q[32][65], k[32][65], v[32][65], dO[32][65];
  __shared__ T P[32][33], dS[32][33];
  const T *base = qkv + b * T_ * 3 * d;
  for (int idx = threadIdx.x; idx < T_ * dh; idx += 64) {
    const int t = idx / dh, j = idx % dh;
    q[t][j] = base[t * 3 * d + h * dh + j];
    k[t][j] = base[t * 3 * d + d + h * dh + j];
    v[t][j] = base[t * 3 * d + 2 * d + h * dh + j];
    dO[t][j] = dout[(b * T_ + t) * d + h * dh + j];
  }
  for (int idx = threadIdx.x; idx < T_ * T_; idx += 64)
    P[idx / T_][idx % T_] = probs[(b * H + h) * T_ * T_ + idx];
  __syncthreads();
  const T scale = T(1) / sqrt(T(dh));
  const int t = threadIdx.x;
  if (t < T_) {
    T dp[32];
    T rowdot = 0;
    for (int s = 0; s <= t; ++s) {
      T a = 0;
      for (int j = 0; j < dh; ++j) a += dO[t][j] * v[s][j];
      dp[s] = a;
      rowdot += a * P[t][s];
    }
    for (int s = 0; s < T_; ++s) dS[t][s] = s <= t ? P[t][s] * (dp[s] - rowdot) : T(0);
  }
  __syncthreads();
  T *drow = dqkv + b * T_ * 3 * d;
  if (t < T_) {
    for (int j = 0; j < dh; ++j) {
      T aq = 0, ak = 0, av = 0;
      for (int s = 0; s < T_; ++s) {
        aq += dS[t][s] * k[s][j];   // dQ[t] = sum_s dS[t,s] K[s]
        ak += dS[s][t] * q[s][j];   // dK[t] = sum_s dS[s,t] Q[s]
        av += P[s][t] * dO[s][j];   // dV[t] = sum_s P[s,t] dO[s]
      }
      drow[t * 3 * d + h * dh + j] = aq * scale;
      drow[t * 3 * d + d + h * dh + j] = ak * scale;
      drow[t * 3 * d + 2 * d + h * dh + j] = av;
    }
  }
}

// Short sequences (T <= 16 positions, head dim <= 16): sixteen lanes per
// (sequence, head) item, lane t owns query / key position t, so nearly every
// lane works; the item's K, V (and for the backward Q, dO, P, dS) rows sit in
// LDS.  IPB items per block.  Loops run over all 16 slots with masks, so the
// per-lane arrays stay in registers.
template <class T, int IPB>
__global__ void __launch_bounds__(IPB * 16) attention_fwd16_kernel(const T *qkv, int64_t n_items,
                                                                   int T_, int d, int H, T *o,
                                                                   T *probs) {
  __shared__ T kk[IPB][16][17], vv[IPB][16][17];
  const int g = threadIdx.x / 16, t = threadIdx.x % 16;
  const int64_t item = int64_t(blockIdx.x) * IPB + g;
  const bool ok = item < n_items && t < T_;
  const int dh = d / H;
  const int64_t b = item / H;
  const int h = int(item % H);
  const T *row = qkv + (b * T_ + t) * 3 * d + h * dh;
  T q[16];
#pragma unroll
  for (int j = 0; j < 16; ++j) {
    const bool in = ok && j < dh;
    q[j] = in ? row[j] : T(0);
    kk[g][t][j] = in ? row[d + j] : T(0);
    vv[g][t][j] = in ? row[2 * d + j] : T(0);
  }
  __syncthreads();
  if (!ok) return;
  const T scale = T(1) / sqrt(T(dh));
  T sc[16];
  T mx = T(-1e300);
#pragma unroll
  for (int u = 0; u < 16; ++u) {
    T a = 0;
#pragma unroll
    for (int j = 0; j < 16; ++j) a += q[j] * kk[g][u][j];
    sc[u] = a * scale;
    if (u <= t) mx = sc[u] > mx ? sc[u] : mx;
  }
  T z = 0;
#pragma unroll
  for (int u = 0; u < 16; ++u) {
    sc[u] = u <= t ? exp(sc[u] - mx) : T(0);
    z += sc[u];
  }
  const T iz = T(1) / z;
#pragma unroll
  for (int u = 0; u < 16; ++u) sc[u] *= iz;
  if (probs) {
    T *pr = probs + (item * T_ + t) * T_;
#pragma unroll
    for (int u = 0; u < 16; ++u)
      if (u < T_) pr[u] = sc[u];
  }
  T *orow = o + (b * T_ + t) * d + h * dh;
#pragma unroll
  for (int j = 0; j < 16; ++j) {
    T a = 0;
#pragma unroll
    for (int u = 0; u < 16; ++u) a += sc[u] * vv[g][u][j];
    if (j < dh) orow[j] = a;
  }
}

template <class T, int IPB>
__global__ void __launch_bounds__(IPB * 16) attention_bwd16_kernel(const T *qkv, const T *probs,
                                                                   const T *dout, int64_t n_items,
                                                                   int T_, int d, int H, T *dqkv) {
  __shared__ T qq[IPB][16][17], kk[IPB][16][17], vv[IPB][16][17], dO[IPB][16][17];
  __shared__ T P[IPB][16][17], dS[IPB][16][17];
  const int g = threadIdx.x / 16, t = threadIdx.x % 16;
  const int64_t item = int64_t(blockIdx.x) * IPB + g;
  const bool ok = item < n_items && t < T_;
  const int dh = d / H;
  const int64_t b = item / H;
  const int h = int(item % H);
  const T *row = qkv + (b * T_ + t) * 3 * d + h * dh;
  const T *drow = dout + (b * T_ + t) * d + h * dh;
  const T *pr = probs + (item * T_ + t) * T_;
#pragma unroll
  for (int j = 0; j < 16; ++j) {
    const bool in = ok && j < dh;
    qq[g][t][j] = in ? row[j] : T(0);
    kk[g][t][j] = in ? row[d + j] : T(0);
    vv[g][t][j] = in ? row[2 * d + j] : T(0);
    dO[g][t][j] = in ? drow[j] : T(0);
    P[g][t][j] = (ok && j < T_) ? pr[j] : T(0);
  }
  __syncthreads();
  {
    // dS[t][u] = P[t][u] (dO[t] . V[u] - sum_w P[t][w] dO[t] . V[w]); P = 0 above the diagonal
    T dp[16];
    T rowdot = 0;
#pragma unroll
    for (int u = 0; u < 16; ++u) {
      T a = 0;
#pragma unroll
      for (int j = 0; j < 16; ++j) a += dO[g][t][j] * vv[g][u][j];
      dp[u] = a;
      rowdot += a * P[g][t][u];
    }
#pragma unroll
    for (int u = 0; u < 16; ++u) dS[g][t][u] = P[g][t][u] * (dp[u] - rowdot);
  }
  __syncthreads();
  if (!ok) return;
  const T scale = T(1) / sqrt(T(dh));
  T *out = dqkv + (b * T_ + t) * 3 * d + h * dh;
#pragma unroll
  for (int j = 0; j < 16; ++j) {
    T aq = 0, ak = 0, av = 0;
#pragma unroll
    for (int u = 0; u < 16; ++u) {
      aq += dS[g][t][u] * kk[g][u][j];   // dQ[t] = sum_u dS[t,u] K[u]
      ak += dS[g][u][t] * qq[g][u][j];   // dK[t] = sum_u dS[u,t] Q[u]
      av += P[g][u][t] * dO[g][u][j];    // dV[t] = sum_u P[u,t] dO[u]
    }
    if (j < dh) {
      out[j] = aq * scale;
      out[d + j] = ak * scale;
      out[2 * d + j] = av;
    }
  }
}

// Short sequences with head dimension 16 (T <= 16 positions): one block per
// S whole sequences and all H heads.  A sequence's rows are contiguous, so the
// block's q, k, v rows (and, for the backward, dO rows) are one contiguous
// range, loaded into LDS with 16-byte loads; lane (sequence s, head h,
// position t) then works from LDS (the 16 lanes of a head read the same key
// row at a time), and the outputs go back through LDS to 16-byte stores.
// The backward recomputes the probabilities from q and k with the forward's
// arithmetic, so no probability array is kept.
typedef __attribute__((ext_vector_type(4))) float f4;
constexpr int kSeqPad = 4;   // LDS row padding (elements), rows stay 16-byte aligned

template <class T>
struct Vec16 {
  typedef __attribute__((ext_vector_type(16 / sizeof(T)))) T type;
};

// n elements (a multiple of the vector width) between global and LDS rows of
// w elements (LDS row stride ld)
template <class T, bool TO_LDS>
__device__ inline void seq_copy(T *sm, int ld, T *g, int64_t n, int w) {
  typedef typename Vec16<T>::type V;
  constexpr int VW = 16 / sizeof(T);
  for (int64_t i = threadIdx.x; i * VW < n; i += blockDim.x) {
    const int64_t e = i * VW;
    const int row = int(e / w), col = int(e % w);
    V *l = reinterpret_cast<V *>(sm + row * ld + col);
    V *q = reinterpret_cast<V *>(g + e);
    if (TO_LDS) *l = *q;
    else *q = *l;
  }
}

// scores of query row t against key rows u <= t, softmax; p[u] = 0 above t
template <class T>
__device__ inline void seq_probs(const T (&q)[16], const T *krow0, int ld, int t, T scale,
                                 T (&p)[16]) {
  T mx = T(-1e300);
#pragma unroll
  for (int u = 0; u < 16; ++u) {
    T a = 0;
    if (u <= t) {
      const T *k = krow0 + u * ld;
#pragma unroll
      for (int j = 0; j < 16; ++j) a += q[j] * k[j];
    }
    p[u] = a * scale;
    if (u <= t) mx = p[u] > mx ? p[u] : mx;
  }
  T z = 0;
#pragma unroll
  for (int u = 0; u < 16; ++u) {
    p[u] = u <= t ? exp(p[u] - mx) : T(0);
    z += p[u];
  }
  const T iz = T(1) / z;
#pragma unroll
  for (int u = 0; u < 16; ++u) p[u] *= iz;
}

template <class T>
__global__ void __launch_bounds__(256) attention_fwd_seq_kernel(const T *__restrict__ qkv,
                                                                int64_t B, int T_, int d, int H,
                                                                int S, T *__restrict__ o) {
  extern __shared__ __attribute__((aligned(16))) char seq_smem[];
  T *sm = reinterpret_cast<T *>(seq_smem);
  const int ld = 3 * d + kSeqPad;
  const int64_t b0 = int64_t(blockIdx.x) * S;
  const int nseq = B - b0 < S ? int(B - b0) : S;
  seq_copy<T, true>(sm, ld, const_cast<T *>(qkv) + b0 * T_ * 3 * d, int64_t(nseq) * T_ * 3 * d,
                    3 * d);
  __syncthreads();
  const int sq = int(threadIdx.x) / (H * 16), h = (int(threadIdx.x) / 16) % H,
            t = int(threadIdx.x) % 16;
  const bool ok = sq < nseq && t < T_;
  T acc[16];
  if (ok) {
    const T *base = sm + (sq * T_) * ld + h * 16;
    T q[16], p[16];
#pragma unroll
    for (int j = 0; j < 16; ++j) q[j] = base[t * ld + j];
    seq_probs<T>(q, base + d, ld, t, T(0.25), p);   // 1 / sqrt(16)
#pragma unroll
    for (int j = 0; j < 16; ++j) acc[j] = 0;
#pragma unroll
    for (int u = 0; u < 16; ++u) {
      if (u > t) continue;
      const T *v = base + u * ld + 2 * d;
#pragma unroll
      for (int j = 0; j < 16; ++j) acc[j] += p[u] * v[j];
    }
  }
  __syncthreads();   // every lane has read the q rows
  if (ok) {
    T *dst = sm + (sq * T_ + t) * ld + h * 16;   // the lane's own q slot
#pragma unroll
    for (int j = 0; j < 16; ++j) dst[j] = acc[j];
  }
  __syncthreads();
  seq_copy<T, false>(sm, ld, o + b0 * T_ * d, int64_t(nseq) * T_ * d, d);
}

// LDS: rows of q, k, v (3d) and dO (d), then per (sequence, head) the 16 x 17
// probabilities and score gradients
template <class T>
__global__ void __launch_bounds__(256) attention_bwd_seq_kernel(const T *__restrict__ qkv,
                                                                const T *__restrict__ dout,
                                                                int64_t B, int T_, int d, int H,
                                                                int S, T *__restrict__ dqkv) {
  extern __shared__ __attribute__((aligned(16))) char seq_smem[];
  T *sm = reinterpret_cast<T *>(seq_smem);
  const int ld = 3 * d + kSeqPad, ldo = d + kSeqPad;
  T *so = sm + S * 16 * ld;                    // dO rows
  T *sp = so + S * 16 * ldo;                   // [S][H][16][17] probabilities
  T *sd = sp + S * H * 16 * 17;                // [S][H][16][17] score gradients
  const int64_t b0 = int64_t(blockIdx.x) * S;
  const int nseq = B - b0 < S ? int(B - b0) : S;
  seq_copy<T, true>(sm, ld, const_cast<T *>(qkv) + b0 * T_ * 3 * d, int64_t(nseq) * T_ * 3 * d,
                    3 * d);
  seq_copy<T, true>(so, ldo, const_cast<T *>(dout) + b0 * T_ * d, int64_t(nseq) * T_ * d, d);
  __syncthreads();
  const int sq = int(threadIdx.x) / (H * 16), h = (int(threadIdx.x) / 16) % H,
            t = int(threadIdx.x) % 16;
  const bool ok = sq < nseq && t < T_;
  const T *base = sm + (sq * T_) * ld + h * 16;    // q of position 0, head h
  const T *obase = so + (sq * T_) * ldo + h * 16;  // dO of position 0, head h
  T *P = sp + (sq * H + h) * 16 * 17, *dS = sd + (sq * H + h) * 16 * 17;
  const T scale = T(0.25);
  T gq[16];
  if (ok) {
    T q[16], p[16], dO[16];
#pragma unroll
    for (int j = 0; j < 16; ++j) {
      q[j] = base[t * ld + j];
      dO[j] = obase[t * ldo + j];
    }
    seq_probs<T>(q, base + d, ld, t, scale, p);
    // dS[t][u] = P[t][u] (dO[t] . V[u] - sum_w P[t][w] dO[t] . V[w])
    T dp[16], rowdot = 0;
#pragma unroll
    for (int u = 0; u < 16; ++u) {
      T a = 0;
      if (u <= t) {
        const T *v = base + u * ld + 2 * d;
#pragma unroll
        for (int j = 0; j < 16; ++j) a += dO[j] * v[j];
      }
      dp[u] = a;
      rowdot += a * p[u];
    }
#pragma unroll
    for (int j = 0; j < 16; ++j) gq[j] = 0;
#pragma unroll
    for (int u = 0; u < 16; ++u) {
      const T ds = p[u] * (dp[u] - rowdot);
      P[t * 17 + u] = p[u];
      dS[t * 17 + u] = ds;
      if (u > t) continue;
      const T *k = base + u * ld + d;
#pragma unroll
      for (int j = 0; j < 16; ++j) gq[j] += ds * k[j];   // dQ[t] = sum_u dS[t,u] K[u]
    }
  }
  __syncthreads();
  T gk[16], gv[16];
  if (ok) {
#pragma unroll
    for (int j = 0; j < 16; ++j) gk[j] = gv[j] = 0;
#pragma unroll
    for (int u = 0; u < 16; ++u) {
      if (u < t || u >= T_) continue;
      const T ds = dS[u * 17 + t], pu = P[u * 17 + t];
      const T *q = base + u * ld, *dO = obase + u * ldo;
#pragma unroll
      for (int j = 0; j < 16; ++j) {
        gk[j] += ds * q[j];    // dK[t] = sum_u dS[u,t] Q[u]
        gv[j] += pu * dO[j];   // dV[t] = sum_u P[u,t] dO[u]
      }
    }
  }
  __syncthreads();   // every lane has read the q, k, v rows
  if (ok) {
    T *dst = sm + (sq * T_ + t) * ld + h * 16;
#pragma unroll
    for (int j = 0; j < 16; ++j) {
      dst[j] = gq[j] * scale;
      dst[d + j] = gk[j] * scale;
      dst[2 * d + j] = gv[j];
    }
  }
  __syncthreads();
  seq_copy<T, false>(sm, ld, dqkv + b0 * T_ * 3 * d, int64_t(nseq) * T_ * 3 * d, 3 * d);
}

// fp32, head dimension 16, T <= 16: one 16-lane row of the wave per
// (sequence, head), lane t holding position t's q, k, v (and dO) in registers;
// position u's values reach the row's other lanes by the row broadcast of DPP
// (row_newbcast:u), so no LDS is used.  The backward rebuilds the
// probabilities and score gradients of column t (P[u][t], dS[u][t], u >= t)
// from broadcasts of row u's q, dO and its softmax statistics.
// row_newbcast writes every lane from a lane of its own row, so the DPP's
// "old" operand never reaches the result; passing the running sum there ties
// each broadcast to the sum it feeds, which keeps the compiler from hoisting
// all 256 broadcasts of a loop (and spilling them)
template <int U>
__device__ inline float row_bcast(float v, float dep = 0.f) {
  return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(__builtin_bit_cast(int, dep),
                                                               __builtin_bit_cast(int, v),
                                                               0x150 + U, 0xF, 0xF, false));
}

// f(u) for u = 0..15 as constants, one u at a time (a scheduling barrier
// between them keeps the broadcasts of one u live, not all 256)
template <int U, class F>
__device__ inline void for_u(F &&f) {
  f(std::integral_constant<int, U>{});
  if constexpr (U + 1 < 16) for_u<U + 1>(f);
}

__device__ inline void load16(const float *p, bool ok, float (&v)[16]) {
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const f4 w = ok ? *reinterpret_cast<const f4 *>(p + 4 * q) : f4{0.f, 0.f, 0.f, 0.f};
    v[4 * q] = w[0];
    v[4 * q + 1] = w[1];
    v[4 * q + 2] = w[2];
    v[4 * q + 3] = w[3];
  }
}
__device__ inline void store16(float *p, const float (&v)[16]) {
#pragma unroll
  for (int q = 0; q < 4; ++q)
    *reinterpret_cast<f4 *>(p + 4 * q) = f4{v[4 * q], v[4 * q + 1], v[4 * q + 2], v[4 * q + 3]};
}

// row t's probabilities over u <= t, and the softmax statistics (max, sum)
__device__ inline void row_probs(const float (&q)[16], const float (&k)[16], int t,
                                 float (&p)[16], float &mx, float &z) {
  for_u<0>([&](auto U) {
    float a = 0.f;
#pragma unroll
    for (int j = 0; j < 16; ++j) a += q[j] * row_bcast<U>(k[j], a);
    p[U] = a * 0.25f;   // 1 / sqrt(16)
  });
  mx = -INFINITY;
#pragma unroll
  for (int u = 0; u < 16; ++u)
    if (u <= t) mx = p[u] > mx ? p[u] : mx;
  z = 0.f;
#pragma unroll
  for (int u = 0; u < 16; ++u) {
    p[u] = u <= t ? expf(p[u] - mx) : 0.f;
    z += p[u];
  }
  const float iz = 1.f / z;
#pragma unroll
  for (int u = 0; u < 16; ++u) p[u] *= iz;
}

__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4)))
attention_fwd_dpp_kernel(const float *__restrict__ qkv,
                                                                int64_t n_items, int T_, int d,
                                                                int H, float *__restrict__ o) {
  const int t = int(threadIdx.x) % 16;
  const int64_t item = int64_t(blockIdx.x) * 16 + threadIdx.x / 16;
  const bool ok = item < n_items && t < T_;
  const int64_t b = item / H;
  const int h = int(item % H);
  const float *row = qkv + (b * T_ + t) * 3 * d + h * 16;
  float q[16], k[16], v[16], p[16], mx, z;
  load16(row, ok, q);
  load16(row + d, ok, k);
  load16(row + 2 * d, ok, v);
  row_probs(q, k, t, p, mx, z);
  float acc[16];
#pragma unroll
  for (int j = 0; j < 16; ++j) acc[j] = 0.f;
  for_u<0>([&](auto U) {
#pragma unroll
    for (int j = 0; j < 16; ++j) acc[j] += p[U] * row_bcast<U>(v[j], acc[j]);
  });
  if (ok) store16(o + (b * T_ + t) * d + h * 16, acc);
}

__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(3)))
attention_bwd_dpp_kernel(const float *__restrict__ qkv,
                                                                const float *__restrict__ dout,
                                                                int64_t n_items, int T_, int d,
                                                                int H, float *__restrict__ dqkv) {
  const int t = int(threadIdx.x) % 16;
  const int64_t item = int64_t(blockIdx.x) * 16 + threadIdx.x / 16;
  const bool ok = item < n_items && t < T_;
  const int64_t b = item / H;
  const int h = int(item % H);
  const float *row = qkv + (b * T_ + t) * 3 * d + h * 16;
  float q[16], k[16], v[16], dO[16], p[16], mx, z;
  load16(row, ok, q);
  load16(row + d, ok, k);
  load16(row + 2 * d, ok, v);
  load16(dout + (b * T_ + t) * d + h * 16, ok, dO);
  row_probs(q, k, t, p, mx, z);
  // row t: dS[t][u] = P[t][u] (dO[t] . V[u] - sum_w P[t][w] dO[t] . V[w]), dQ[t] = sum_u dS[t,u] K[u]
  float ds[16], rowdot = 0.f;
  for_u<0>([&](auto U) {
    float a = 0.f;
#pragma unroll
    for (int j = 0; j < 16; ++j) a += dO[j] * row_bcast<U>(v[j], a);
    ds[U] = a;
    rowdot += a * p[U];
  });
#pragma unroll
  for (int u = 0; u < 16; ++u) ds[u] = p[u] * (ds[u] - rowdot);
  float *out = dqkv + (b * T_ + t) * 3 * d + h * 16;
  {
    float gq[16];
#pragma unroll
    for (int j = 0; j < 16; ++j) gq[j] = 0.f;
    for_u<0>([&](auto U) {
#pragma unroll
      for (int j = 0; j < 16; ++j) gq[j] += ds[U] * row_bcast<U>(k[j], gq[j]);
    });
#pragma unroll
    for (int j = 0; j < 16; ++j) gq[j] *= 0.25f;
    if (ok) store16(out, gq);
  }
  float gk[16], gv[16];
#pragma unroll
  for (int j = 0; j < 16; ++j) gk[j] = gv[j] = 0.f;
  // column t: P[u][t] and dS[u][t] for t <= u < T from row u's broadcasts;
  // dK[t] = sum_u dS[u,t] Q[u], dV[t] = sum_u P[u,t] dO[u]
  for_u<0>([&](auto U) {
    float qb[16], ob[16], sc = 0.f, dp = 0.f;
#pragma unroll
    for (int j = 0; j < 16; ++j) {
      // each broadcast waits for the previous u's accumulation into the same
      // feature (one u's broadcasts live at a time)
      qb[j] = row_bcast<U>(q[j], gk[j]);
      ob[j] = row_bcast<U>(dO[j], gv[j]);
      sc += qb[j] * k[j];
      dp += ob[j] * v[j];
    }
    const float mu = row_bcast<U>(mx, sc), zu = row_bcast<U>(z, sc), ru = row_bcast<U>(rowdot, dp);
    const bool in = t <= U && U < T_;
    const float put = in ? expf(sc * 0.25f - mu) / zu : 0.f;
    const float dsut = in ? put * (dp - ru) : 0.f;
#pragma unroll
    for (int j = 0; j < 16; ++j) {
      gk[j] += dsut * qb[j];
      gv[j] += put * ob[j];
    }
  });
  if (ok) {
#pragma unroll
    for (int j = 0; j < 16; ++j) gk[j] *= 0.25f;
    store16(out + d, gk);
    store16(out + 2 * d, gv);
  }
}

// sequences per block of the seq kernels: all heads of S sequences in at most
// 256 lanes and 64 KiB of LDS (0: the shape does not fit them)
template <class T>
int seq_per_block(int T_, int d, int H, bool bwd) {
  if (T_ > 16 || d != 16 * H || (3 * d * int(sizeof(T))) % 16 != 0) return 0;
  const size_t per = size_t(16) * (3 * d + kSeqPad) * sizeof(T) +
                     (bwd ? size_t(16) * (d + kSeqPad) * sizeof(T) + size_t(2) * H * 16 * 17 * sizeof(T)
                          : 0);
  int S = 256 / (16 * H);
  while (S > 1 && per * S > 64 * 1024) --S;
  return per * S <= 64 * 1024 && S >= 1 ? S : 0;
}
template <class T>
size_t seq_lds_bytes(int T_, int d, int H, bool bwd, int S) {
  (void)T_;
  return size_t(S) * (size_t(16) * (3 * d + kSeqPad) * sizeof(T) +
                      (bwd ? size_t(16) * (d + kSeqPad) * sizeof(T) +
                                 size_t(2) * H * 16 * 17 * sizeof(T)
                           : 0));
}

template <class T>
__global__ void gelu_bwd_kernel(const T *pre, T *dy, int64_t n) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < n) dy[i] *= gelu_tanh_grad(pre[i]);
}
template <class T>
__global__ void tanh_bwd_kernel(const T *y, T *dy, int64_t n) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < n) dy[i] *= T(1) - y[i] * y[i];
}
template <class T>
__global__ void lrelu_bwd_kernel(const T *pre, T *dy, int64_t n) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < n) dy[i] *= pre[i] >= T(0) ? T(1) : T(0.01);
}
template <class TS, class TD>
__global__ void convert_kernel(const TS *src, TD *dst, int64_t n) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < n) dst[i] = TD(src[i]);
}
__global__ void zero_kernel(uint32_t *p, int64_t n) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0u;
}

inline dim3 grid1(int64_t n, int b = 256) { return dim3(unsigned(ceil_div(n, b))); }

}  // namespace

template <class T, bool TA, bool TB>
void gemm(int64_t M, int64_t N, int64_t K, const T *A, int64_t lda, const T *B, int64_t ldb, T *C,
          int64_t ldc, const T *bias, T *aux, int epi, hipStream_t s) {
  if (M <= 0 || N <= 0) return;
  NQS_REQUIRE(M < (int64_t(1) << 31) && N < (int64_t(1) << 31) && K < (int64_t(1) << 31),
              NQS_EUNSUPPORTED, "gemm: dimension too large");
  // row-major C = op(A) op(B) is column-major C^T = op(B)^T op(A)^T
  blas_gemm(blas(s), TB ? rocblas_operation_transpose : rocblas_operation_none,
            TA ? rocblas_operation_transpose : rocblas_operation_none, int(N), int(M), int(K),
            T(1), B, int(ldb), A, int(lda), epi == EPI_ADD ? T(1) : T(0), C, int(ldc), s);
  if (bias || (epi != EPI_STORE && epi != EPI_ADD)) {
    hipLaunchKernelGGL(epilogue_kernel<T>, grid1(M * N), dim3(256), 0, s, C, M, N, ldc, bias, aux,
                       epi);
    HIP_LAUNCH_OK();
  }
}

void blas_gemm_batched(rocblas_handle h, rocblas_operation ta, rocblas_operation tb, int m, int n,
                       int k, float alpha, const float *A, int lda, int64_t sa, const float *B,
                       int ldb, int64_t sb, float beta, float *C, int ldc, int64_t sc, int batch) {
  BLAS_OK(rocblas_sgemm_strided_batched(h, ta, tb, m, n, k, &alpha, A, lda, sa, B, ldb, sb, &beta,
                                        C, ldc, sc, batch));
}
void blas_gemm_batched(rocblas_handle h, rocblas_operation ta, rocblas_operation tb, int m, int n,
                       int k, double alpha, const double *A, int lda, int64_t sa, const double *B,
                       int ldb, int64_t sb, double beta, double *C, int ldc, int64_t sc,
                       int batch) {
  BLAS_OK(rocblas_dgemm_strided_batched(h, ta, tb, m, n, k, &alpha, A, lda, sa, B, ldb, sb, &beta,
                                        C, ldc, sc, batch));
}

template <class T, bool TA, bool TB>
void gemm_batched(int64_t M, int64_t N, int64_t K, const T *A, int64_t lda, int64_t sa,
                  const T *B, int64_t ldb, int64_t sb, T *C, int64_t ldc, int64_t sc,
                  int64_t batch, bool accumulate, hipStream_t s) {
  if (M <= 0 || N <= 0 || batch <= 0) return;
  NQS_REQUIRE(M < (int64_t(1) << 31) && N < (int64_t(1) << 31) && K < (int64_t(1) << 31) &&
                  batch < (int64_t(1) << 31),
              NQS_EUNSUPPORTED, "gemm_batched: dimension too large");
  // row-major C = op(A) op(B) is column-major C^T = op(B)^T op(A)^T
  blas_gemm_batched(blas(s), TB ? rocblas_operation_transpose : rocblas_operation_none,
                    TA ? rocblas_operation_transpose : rocblas_operation_none, int(N), int(M),
                    int(K), T(1), B, int(ldb), sb, A, int(lda), sa, accumulate ? T(1) : T(0), C,
                    int(ldc), sc, int(batch));
}

template <class T>
void add_into(const T *src, int64_t n, double *dst, hipStream_t s) {
  if (n <= 0) return;
  hipLaunchKernelGGL(add_into_kernel<T>, grid1(n), dim3(256), 0, s, src, n, dst);
  HIP_LAUNCH_OK();
}

template <class T>
void fill_ones(T *dst, int64_t n, hipStream_t s) {
  if (n <= 0) return;
  hipLaunchKernelGGL(fill_kernel<T>, grid1(n), dim3(256), 0, s, dst, n, T(1));
  HIP_LAUNCH_OK();
}

namespace {
// Second-level scratch of a slice reduction: at most kLevelElems doubles.
constexpr int64_t kLevelElems = int64_t(1) << 17;

// acc[i] += sum_z part[z*len + i] in a fixed order: slices are summed in
// groups by sum_slices_kernel (enough blocks to fill the chip), then the group
// sums in order by slices_acc_kernel.  lvl holds kLevelElems doubles.
template <class P>
void reduce_slices(const P *part, int64_t nslices, int64_t len, double *acc, double *lvl,
                   hipStream_t s) {
  if (len <= 0 || nslices <= 0) return;
  const int64_t col_blocks = ceil_div(len, int64_t(64));
  int64_t groups = std::min(ceil_div(int64_t(2048), col_blocks), ceil_div(nslices, int64_t(8)));
  groups = std::min(groups, kLevelElems / len);
  if (groups <= 1) {
    hipLaunchKernelGGL(slices_acc_kernel<P>, grid1(len), dim3(256), 0, s, part, nslices, len, acc);
    HIP_LAUNCH_OK();
    return;
  }
  const int64_t zs = ceil_div(nslices, groups);
  groups = ceil_div(nslices, zs);
  hipLaunchKernelGGL(sum_slices_kernel<P>, dim3(unsigned(col_blocks), unsigned(groups)), dim3(256),
                     0, s, part, nslices, len, zs, lvl);
  HIP_LAUNCH_OK();
  hipLaunchKernelGGL(slices_acc_kernel<double>, grid1(len), dim3(256), 0, s,
                     static_cast<const double *>(lvl), groups, len, acc);
  HIP_LAUNCH_OK();
}

// row slices of a column sum: enough blocks to fill the chip, >= 256 rows each
int64_t colsum_slices(int64_t R, int64_t N) {
  const int64_t z = std::min(ceil_div(int64_t(2048), ceil_div(N, int64_t(64))),
                             ceil_div(R, int64_t(256)));
  return std::max<int64_t>(z, 1);
}
}  // namespace

size_t colsum_scratch_bytes(int64_t R, int64_t N) {
  return size_t(colsum_slices(R, N) * N + kLevelElems) * sizeof(double);
}

template <class T>
void colsum_acc(const T *Y, int64_t R, int64_t N, int64_t ld, double *acc, double *scratch,
                hipStream_t s) {
  if (R <= 0 || N <= 0) return;
  const int64_t slices = colsum_slices(R, N);
  const int64_t rows_per = ceil_div(R, slices);
  const int64_t used = ceil_div(R, rows_per);
  hipLaunchKernelGGL(colsum_kernel<T>, dim3(unsigned(ceil_div(N, 64)), unsigned(used)), dim3(256),
                     0, s, Y, R, N, ld, rows_per, scratch);
  HIP_LAUNCH_OK();
  reduce_slices<double>(scratch, used, N, acc, scratch + slices * N, s);
}

void slices_acc(const double *part, int64_t nslices, int64_t len, double *acc, hipStream_t s) {
  if (len <= 0) return;
  hipLaunchKernelGGL(slices_acc_kernel<double>, grid1(len), dim3(256), 0, s, part, nslices, len,
                     acc);
  HIP_LAUNCH_OK();
}

namespace {
// row slices of the weight-gradient reduction: enough blocks to fill the chip,
// at least 128 rows per slice, partial sums within the scratch budget
constexpr size_t kWgradScratch = size_t(64) << 20;
int64_t wgrad_slices(int64_t R, int64_t M, int64_t N) {
  const int64_t tiles = ceil_div(M, 128) * ceil_div(N, 128);
  int64_t z = ceil_div(int64_t(1024), tiles);
  z = std::min<int64_t>(z, ceil_div(R, int64_t(128)));
  z = std::min<int64_t>(z, int64_t(kWgradScratch / size_t(4 * M * N)));
  return std::max<int64_t>(z, 1);
}
// a slice of either matrix must stay under 2 GiB (32-bit buffer offsets; rows
// are at most 1 MiB, so a batch reaching 16 rows past the slice cannot wrap)
int64_t wgrad_slices(int64_t R, int64_t M, int64_t N, int64_t ld) {
  const int64_t z = wgrad_slices(R, M, N);
  return std::max<int64_t>(z, ceil_div(R * ld * 4, int64_t(1) << 30) + 1);
}
}  // namespace

size_t wgrad_scratch_bytes(int64_t R, int64_t M, int64_t N, int64_t ld, size_t elem) {
  if (elem == sizeof(double)) return size_t(M * N) * sizeof(double);
  // float partials, the second level of the reduction (8-byte aligned), then
  // the mixed kernel's column sums (double)
  const int64_t z = wgrad_slices(R, M, N, ld);
  return size_t(ceil_div(z * M * N, int64_t(2))) * 8 + size_t(kLevelElems) * sizeof(double) +
         size_t(z * N) * sizeof(double);
}

void wgrad_acc(const float *X, int64_t ldx, const float *dY, int64_t ldy, int64_t R,
                      int64_t M, int64_t N, double *acc, void *scratch, hipStream_t s, bool mixed,
                      double *bias_acc) {
  if (M <= 0 || N <= 0) return;
  NQS_REQUIRE(M < (int64_t(1) << 24) && N < (int64_t(1) << 24), NQS_EUNSUPPORTED,
              "weight gradient: dimension too large");
  if (R <= 0) return;
  const int64_t ld = std::max(ldx, ldy);
  NQS_REQUIRE(ld * 4 <= (int64_t(1) << 20), NQS_EUNSUPPORTED, "weight gradient: row too long");
  const int64_t z = wgrad_slices(R, M, N, ld), rows_per = ceil_div(R, z);
  const int tiles_n = int(ceil_div(N, int64_t(128)));
  const int64_t tiles = ceil_div(M, int64_t(128)) * tiles_n;
  const dim3 grid = dim3(unsigned(tiles), unsigned(ceil_div(R, rows_per)));
  float *part = static_cast<float *>(scratch);
  double *lvl = static_cast<double *>(scratch) + ceil_div(z * M * N, int64_t(2));
  double *bpart = lvl + kLevelElems;
  NQS_REQUIRE(!bias_acc || mixed, NQS_EINVAL, "weight gradient: bias sums need the mixed kernel");
  if (mixed) {
    mx_wgrad_partials(X, ldx, dY, ldy, R, M, N, rows_per, part, bias_acc ? bpart : nullptr, s);
  } else {
    hipLaunchKernelGGL(wgrad_f32_kernel, grid, dim3(256), 0, s, X, ldx, dY, ldy, R, int(M), int(N),
                       rows_per, tiles_n, part);
    HIP_LAUNCH_OK();
  }
  reduce_slices<float>(part, int64_t(grid.y), M * N, acc, lvl, s);
  if (bias_acc) reduce_slices<double>(bpart, int64_t(grid.y), N, bias_acc, lvl, s);
}

void wgrad_acc(const double *X, int64_t ldx, const double *dY, int64_t ldy, int64_t R,
                       int64_t M, int64_t N, double *acc, void *scratch, hipStream_t s) {
  if (M <= 0 || N <= 0 || R <= 0) return;
  double *part = static_cast<double *>(scratch);
  gemm<double, true, false>(M, N, R, X, ldx, dY, ldy, part, N, nullptr, nullptr, EPI_STORE, s);
  add_into<double>(part, M * N, acc, s);
}

template <class T>
void layernorm(const T *x, int64_t R, int d, const T *g, const T *b, T *y, T *mean, T *rstd,
               hipStream_t s) {
  if (R <= 0) return;
  constexpr int RPW = 4;
  if (d == 64 || d == 128) {
    const dim3 grid = grid1(ceil_div(R, RPW), 4);
    if (d == 64)
      hipLaunchKernelGGL((layernorm_rows_kernel<T, 1, RPW>), grid, dim3(256), 0, s, x, R, g, b, y,
                         mean, rstd);
    else
      hipLaunchKernelGGL((layernorm_rows_kernel<T, 2, RPW>), grid, dim3(256), 0, s, x, R, g, b, y,
                         mean, rstd);
    HIP_LAUNCH_OK();
    return;
  }
  hipLaunchKernelGGL(layernorm_kernel<T>, grid1(R, 4), dim3(256), 0, s, x, R, d, g, b, y, mean, rstd);
  HIP_LAUNCH_OK();
}

template <class T>
void layernorm_bwd(const T *x, const T *mean, const T *rstd, int64_t R, int d, const T *g,
                   const T *dy, T *dx, bool accumulate, T *dyxh, hipStream_t s) {
  if (R <= 0) return;
  hipLaunchKernelGGL(layernorm_bwd_kernel<T>, grid1(R, 4), dim3(256), 0, s, x, mean, rstd, R, d, g,
                     dy, dx, accumulate, dyxh);
  HIP_LAUNCH_OK();
}

namespace {
constexpr int64_t kLnBlocks = 1024;   // row ranges of the layer-norm backward's sums
}

bool layernorm_bwd_acc_supported(int d) { return d == 64 || d == 128; }

size_t layernorm_bwd_acc_scratch_bytes(int d) {
  return size_t(2 * kLnBlocks * d + kLevelElems) * sizeof(double);
}

template <class T>
void layernorm_bwd_acc(const T *x, const T *mean, const T *rstd, int64_t R, int d, const T *g,
                       const T *dy, T *dx, bool accumulate, double *gacc, double *bacc,
                       double *scratch, hipStream_t s) {
  if (R <= 0) return;
  NQS_REQUIRE(layernorm_bwd_acc_supported(d), NQS_EUNSUPPORTED, "layer norm backward: d");
  const int64_t rows_per = ceil_div(R, kLnBlocks), blocks = ceil_div(R, rows_per);
  double *gpart = scratch, *bpart = scratch + kLnBlocks * d, *lvl = scratch + 2 * kLnBlocks * d;
  if (d == 64)
    hipLaunchKernelGGL((layernorm_bwd_acc_kernel<T, 1>), dim3(unsigned(blocks)), dim3(256), 0, s, x,
                       mean, rstd, R, rows_per, g, dy, dx, accumulate, gpart, bpart);
  else
    hipLaunchKernelGGL((layernorm_bwd_acc_kernel<T, 2>), dim3(unsigned(blocks)), dim3(256), 0, s, x,
                       mean, rstd, R, rows_per, g, dy, dx, accumulate, gpart, bpart);
  HIP_LAUNCH_OK();
  reduce_slices<double>(gpart, blocks, d, gacc, lvl, s);
  reduce_slices<double>(bpart, blocks, d, bacc, lvl, s);
}

template <class T>
void attention_fwd(const T *qkv, int64_t B, int T_, int d, int H, T *o, T *probs, hipStream_t s) {
  if (B <= 0) return;
  if (std::is_same<T, float>::value && T_ <= 16 && d == 16 * H) {
    // fp32: the DPP kernels (the backward recomputes the probabilities)
    hipLaunchKernelGGL(attention_fwd_dpp_kernel, dim3(unsigned(ceil_div(B * H, 16))), dim3(256), 0,
                       s, reinterpret_cast<const float *>(qkv), B * H, T_, d, H,
                       reinterpret_cast<float *>(o));
    HIP_LAUNCH_OK();
    return;
  }
  // the seq kernels only where the backward fits them too: it recomputes the
  // probabilities the seq forward does not write
  if (seq_per_block<T>(T_, d, H, true) > 0) {
    const int S = seq_per_block<T>(T_, d, H, false);
    hipLaunchKernelGGL(attention_fwd_seq_kernel<T>, dim3(unsigned(ceil_div(B, S))),
                       dim3(unsigned(S * H * 16)), seq_lds_bytes<T>(T_, d, H, false, S), s, qkv, B,
                       T_, d, H, S, o);
    HIP_LAUNCH_OK();
    return;
  }
  if (T_ <= 16 && d / H <= 16) {
    constexpr int IPB = sizeof(T) == 8 ? 8 : 16;
    hipLaunchKernelGGL((attention_fwd16_kernel<T, IPB>), dim3(unsigned(ceil_div(B * H, IPB))),
                       dim3(IPB * 16), 0, s, qkv, B * H, T_, d, H, o, probs);
    HIP_LAUNCH_OK();
    return;
  }
  NQS_REQUIRE(T_ <= 32 && d / H <= 64, NQS_EUNSUPPORTED, "attention: sequence > 32 or head dim > 64");
  hipLaunchKernelGGL(attention_fwd_kernel<T>, dim3(unsigned(B * H)), dim3(64), 0, s, qkv, T_, d, H,
                     o, probs);
  HIP_LAUNCH_OK();
}

template <class T>
void attention_bwd(const T *qkv, const T *probs, const T *dout, int64_t B, int T_, int d, int H,
                   T *dqkv, hipStream_t s) {
  if (B <= 0) return;
  if (std::is_same<T, float>::value && T_ <= 16 && d == 16 * H) {
    hipLaunchKernelGGL(attention_bwd_dpp_kernel, dim3(unsigned(ceil_div(B * H, 16))), dim3(256), 0,
                       s, reinterpret_cast<const float *>(qkv), reinterpret_cast<const float *>(dout),
                       B * H, T_, d, H, reinterpret_cast<float *>(dqkv));
    HIP_LAUNCH_OK();
    return;
  }
  if (const int S = seq_per_block<T>(T_, d, H, true)) {
    hipLaunchKernelGGL(attention_bwd_seq_kernel<T>, dim3(unsigned(ceil_div(B, S))),
                       dim3(unsigned(S * H * 16)), seq_lds_bytes<T>(T_, d, H, true, S), s, qkv,
                       dout, B, T_, d, H, S, dqkv);
    HIP_LAUNCH_OK();
    return;
  }
  if (T_ <= 16 && d / H <= 16) {
    constexpr int IPB = sizeof(T) == 8 ? 4 : 8;
    hipLaunchKernelGGL((attention_bwd16_kernel<T, IPB>), dim3(unsigned(ceil_div(B * H, IPB))),
                       dim3(IPB * 16), 0, s, qkv, probs, dout, B * H, T_, d, H, dqkv);
    HIP_LAUNCH_OK();
    return;
  }
  NQS_REQUIRE(T_ <= 32 && d / H <= 64, NQS_EUNSUPPORTED, "attention: sequence > 32 or head dim > 64");
  hipLaunchKernelGGL(attention_bwd_kernel<T>, dim3(unsigned(B * H)), dim3(64), 0, s, qkv, probs,
                     dout, T_, d, H, dqkv);
  HIP_LAUNCH_OK();
}

template <class T>
void gelu_bwd(const T *pre, T *dy, int64_t n, hipStream_t s) {
  if (n <= 0) return;
  hipLaunchKernelGGL(gelu_bwd_kernel<T>, grid1(n), dim3(256), 0, s, pre, dy, n);
  HIP_LAUNCH_OK();
}
template <class T>
void tanh_bwd(const T *y, T *dy, int64_t n, hipStream_t s) {
  if (n <= 0) return;
  hipLaunchKernelGGL(tanh_bwd_kernel<T>, grid1(n), dim3(256), 0, s, y, dy, n);
  HIP_LAUNCH_OK();
}
template <class T>
void lrelu_bwd(const T *pre, T *dy, int64_t n, hipStream_t s) {
  if (n <= 0) return;
  hipLaunchKernelGGL(lrelu_bwd_kernel<T>, grid1(n), dim3(256), 0, s, pre, dy, n);
  HIP_LAUNCH_OK();
}
template <class TS, class TD>
void convert(const TS *src, TD *dst, int64_t n, hipStream_t s) {
  if (n <= 0) return;
  hipLaunchKernelGGL((convert_kernel<TS, TD>), grid1(n), dim3(256), 0, s, src, dst, n);
  HIP_LAUNCH_OK();
}
void zero_async(void *p, size_t bytes, hipStream_t s) {
  // a fill kernel rather than a memset node, so that graph capture stays safe
  const int64_t words = int64_t((bytes + 3) / 4);
  if (words <= 0) return;
  hipLaunchKernelGGL(zero_kernel, grid1(words), dim3(256), 0, s, static_cast<uint32_t *>(p), words);
  HIP_LAUNCH_OK();
}

#define INST_T(T)                                                                               \
  template void colsum_acc<T>(const T *, int64_t, int64_t, int64_t, double *, double *,         \
                              hipStream_t);                                                      \
  template void layernorm<T>(const T *, int64_t, int, const T *, const T *, T *, T *, T *,      \
                             hipStream_t);                                                       \
  template void layernorm_bwd<T>(const T *, const T *, const T *, int64_t, int, const T *,      \
                                 const T *, T *, bool, T *, hipStream_t);                        \
  template void layernorm_bwd_acc<T>(const T *, const T *, const T *, int64_t, int, const T *,  \
                                     const T *, T *, bool, double *, double *, double *,          \
                                     hipStream_t);                                                \
  template void attention_fwd<T>(const T *, int64_t, int, int, int, T *, T *, hipStream_t);     \
  template void attention_bwd<T>(const T *, const T *, const T *, int64_t, int, int, int, T *,  \
                                 hipStream_t);                                                   \
  template void gelu_bwd<T>(const T *, T *, int64_t, hipStream_t);                              \
  template void tanh_bwd<T>(const T *, T *, int64_t, hipStream_t);                              \
  template void lrelu_bwd<T>(const T *, T *, int64_t, hipStream_t);                             \
  template void gemm<T, false, false>(int64_t, int64_t, int64_t, const T *, int64_t, const T *, \
                                      int64_t, T *, int64_t, const T *, T *, int, hipStream_t);  \
  template void gemm<T, false, true>(int64_t, int64_t, int64_t, const T *, int64_t, const T *,  \
                                     int64_t, T *, int64_t, const T *, T *, int, hipStream_t);   \
  template void gemm<T, true, false>(int64_t, int64_t, int64_t, const T *, int64_t, const T *,  \
                                     int64_t, T *, int64_t, const T *, T *, int, hipStream_t);   \
  template void gemm_batched<T, false, false>(int64_t, int64_t, int64_t, const T *, int64_t,     \
                                              int64_t, const T *, int64_t, int64_t, T *, int64_t, \
                                              int64_t, int64_t, bool, hipStream_t);               \
  template void gemm_batched<T, false, true>(int64_t, int64_t, int64_t, const T *, int64_t,      \
                                             int64_t, const T *, int64_t, int64_t, T *, int64_t,  \
                                             int64_t, int64_t, bool, hipStream_t);                \
  template void gemm_batched<T, true, false>(int64_t, int64_t, int64_t, const T *, int64_t,      \
                                             int64_t, const T *, int64_t, int64_t, T *, int64_t,  \
                                             int64_t, int64_t, bool, hipStream_t);                \
  template void add_into<T>(const T *, int64_t, double *, hipStream_t);                         \
  template void fill_ones<T>(T *, int64_t, hipStream_t);

INST_T(float)
INST_T(double)
template void convert<double, float>(const double *, float *, int64_t, hipStream_t);
template void convert<float, double>(const float *, double *, int64_t, hipStream_t);
template void convert<double, double>(const double *, double *, int64_t, hipStream_t);

}  // namespace nqs
