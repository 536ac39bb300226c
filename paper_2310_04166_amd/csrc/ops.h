// Building blocks of the layer-by-layer amplitude path (FP64 and FP32 modes,
// and every backward pass): a tiled GEMM with fused epilogues, layer norm,
// causal attention for short sequences, and column reductions.
#pragma once

#include "common.h"

namespace nqs {

enum Epi : int {
  EPI_STORE = 0,   // C = AB + bias
  EPI_GELU = 1,    // aux = AB + bias, C = gelu_tanh(aux)
  EPI_TANH = 2,    // C = tanh(AB + bias)
  EPI_LRELU = 3,   // aux = AB + bias, C = leaky_relu(aux, 0.01)
  EPI_ADD = 4,     // C += AB + bias
};

// C[M,N] = op(A)[M,K] op(B)[K,N] (row-major); op(A)(i,k) = TA ? A[k*lda+i] :
// A[i*lda+k], op(B)(k,j) = TB ? B[j*ldb+k] : B[k*ldb+j].  A plain library GEMM
// (rocBLAS) followed by the bias / activation epilogue.
template <class T, bool TA, bool TB>
void gemm(int64_t M, int64_t N, int64_t K, const T *A, int64_t lda, const T *B, int64_t ldb, T *C,
          int64_t ldc, const T *bias, T *aux, int epi, hipStream_t s);
// Strided batch of row-major products, no epilogue: for q < batch,
// C_q (+)= op(A_q) op(B_q) with A_q = A + q sa, B_q = B + q sb, C_q = C + q sc
// (a stride may be 0 to share an operand); accumulate adds into C.
template <class T, bool TA, bool TB>
void gemm_batched(int64_t M, int64_t N, int64_t K, const T *A, int64_t lda, int64_t sa,
                  const T *B, int64_t ldb, int64_t sb, T *C, int64_t ldc, int64_t sc,
                  int64_t batch, bool accumulate, hipStream_t s);
// dst[i] += src[i] (into a double accumulator)
template <class T>
void add_into(const T *src, int64_t n, double *dst, hipStream_t s);
template <class T>
void fill_ones(T *dst, int64_t n, hipStream_t s);

// Deterministic column sums: acc[j] += sum_r Y[r*ld + j] (double accumulator);
// scratch holds colsum_scratch_bytes(R, N) bytes.
template <class T>
void colsum_acc(const T *Y, int64_t R, int64_t N, int64_t ld, double *acc, double *scratch,
                hipStream_t s);
size_t colsum_scratch_bytes(int64_t R, int64_t N);
// Weight gradient: acc[i*N + j] += sum_r X[r*ldx + i] * dY[r*ldy + j] for i < M,
// j < N (double accumulator).  FP32: a split-K MFMA reduction over row slices
// whose partial sums are added in a fixed order; FP64: a library GEMM.  scratch
// holds at least wgrad_scratch_bytes(R, M, N, max(ldx, ldy), element size) bytes.
// mixed: the partial sums take split bf16 operands (mx_wgrad_partials) instead
// of fp32 MFMA, and with bias_acc also bias_acc[j] += sum_r dY[r*ldy + j].
void wgrad_acc(const float *X, int64_t ldx, const float *dY, int64_t ldy, int64_t R, int64_t M,
               int64_t N, double *acc, void *scratch, hipStream_t s, bool mixed = false,
               double *bias_acc = nullptr);
void wgrad_acc(const double *X, int64_t ldx, const double *dY, int64_t ldy, int64_t R, int64_t M,
               int64_t N, double *acc, void *scratch, hipStream_t s);
size_t wgrad_scratch_bytes(int64_t R, int64_t M, int64_t N, int64_t ld, size_t elem);
// acc[i] += sum_z part[z*len + i]
void slices_acc(const double *part, int64_t nslices, int64_t len, double *acc, hipStream_t s);

// ---- Mixed-precision products (mx_gemm.hip), used by the backward of bf16
// models: fp32 operands split into bf16 hi + lo parts, three MFMA products
// (hi hi, hi lo, lo hi) with fp32 accumulation, about 2^-16 relative error per
// product.
enum MxEpi : int {
  MX_STORE = 0,   // C = A op(W) + bias
  MX_ADD = 1,     // C = res + A op(W) + bias (res another array)
  MX_GELU = 2,    // aux = A op(W) + bias, C = gelu_tanh(aux)
  MX_DGELU = 3,   // C = (A op(W)) * gelu_tanh'(aux), no bias
};
// Shapes the products take: N and K multiples of 32.
bool mx_supported(int64_t N, int64_t K);
// Image of a right operand, op(W)(k, n) = trans ? W[n*ldw + k] : W[k*ldw + n]
// (k < K, n < N), in mx_pack_bytes(N, K) bytes of device memory.
size_t mx_pack_bytes(int64_t N, int64_t K);
void mx_pack(const float *W, int64_t ldw, bool trans, int64_t N, int64_t K, void *out,
             hipStream_t s);
// C[M,N] (ldc) from A[M,K] (row-major, lda % 4 == 0, 16-byte aligned) and the
// image Wp of op(W), with the epilogue epi; aux has the leading dimension ldc.
void mx_gemm(int64_t M, int64_t N, int64_t K, const float *A, int64_t lda, const void *Wp, float *C,
             int64_t ldc, const float *res, int64_t ldr, const float *bias, float *aux, int epi,
             hipStream_t s);
// part[z][i][j] = sum over rows r of slice z (rows z*rows_per ..) of
// X[r][i] dY[r][j], i < M, j < N; a slice under 1 GiB of either matrix; with
// bpart (optional) also bpart[z][j] = sum over those rows of dY[r][j] (double).
void mx_wgrad_partials(const float *X, int64_t ldx, const float *dY, int64_t ldy, int64_t R,
                       int64_t M, int64_t N, int64_t rows_per, float *part, double *bpart,
                       hipStream_t s);

// Row-wise layer norm over d columns; mean/rstd may be null.
template <class T>
void layernorm(const T *x, int64_t R, int d, const T *g, const T *b, T *y, T *mean, T *rstd,
               hipStream_t s);
// dx (+)= LN backward; dyxh = dy * xhat (for the gain gradient).
template <class T>
void layernorm_bwd(const T *x, const T *mean, const T *rstd, int64_t R, int d, const T *g,
                   const T *dy, T *dx, bool accumulate, T *dyxh, hipStream_t s);

// The same with the layer norm's parameter gradients: gacc[j] += sum_r dy *
// xhat, bacc[j] += sum_r dy (double, fixed order), for d = 64 or 128;
// scratch holds layernorm_bwd_acc_scratch_bytes(d) bytes.
bool layernorm_bwd_acc_supported(int d);
size_t layernorm_bwd_acc_scratch_bytes(int d);
template <class T>
void layernorm_bwd_acc(const T *x, const T *mean, const T *rstd, int64_t R, int d, const T *g,
                       const T *dy, T *dx, bool accumulate, double *gacc, double *bacc,
                       double *scratch, hipStream_t s);

// Causal attention for B sequences of T tokens: qkv [B*T, 3d] -> o [B*T, d],
// probs [B, H, T, T] (if non-null; not written for head dimension 16 and
// T <= 16 in fp32, nor in fp64 where the backward fits 64 KiB of LDS per
// block: there the backward recomputes them and ignores probs).
template <class T>
void attention_fwd(const T *qkv, int64_t B, int T_, int d, int H, T *o, T *probs, hipStream_t s);
template <class T>
void attention_bwd(const T *qkv, const T *probs, const T *dout, int64_t B, int T_, int d, int H,
                   T *dqkv, hipStream_t s);

// Elementwise helpers.
template <class T>
void gelu_bwd(const T *pre, T *dy, int64_t n, hipStream_t s);   // dy *= gelu'(pre)
template <class T>
void tanh_bwd(const T *y, T *dy, int64_t n, hipStream_t s);     // dy *= 1 - y^2
template <class T>
void lrelu_bwd(const T *pre, T *dy, int64_t n, hipStream_t s);  // dy *= (pre>=0 ? 1 : 0.01)
template <class TS, class TD>
void convert(const TS *src, TD *dst, int64_t n, hipStream_t s);
void zero_async(void *p, size_t bytes, hipStream_t s);

}  // namespace nqs
