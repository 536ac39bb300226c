// Mixed-precision products of the layer-by-layer path: the backward pass of
// bf16 models, its forward recomputation included ("Variational Monte Carlo":
// the gradient 2 Re E[(E_loc - E) d log psi*] through the amplitude network).
//
// Every fp32 operand x is split into two bf16 numbers, hi = bf16(x) and
// lo = bf16(x - hi), and a product a b is taken as
//     hi(a) hi(b) + hi(a) lo(b) + lo(a) hi(b)
// on the bf16 matrix cores (v_mfma_f32_32x32x16_bf16) with fp32 accumulation.
// The dropped lo(a) lo(b) term and the rounding of lo leave a relative error
// of about 2^-16 per product (2^-8 with plain bf16 operands).  The layer
// path's products are tall and thin (M ~ 1e5 token rows; N and K of 64 .. 512),
// so at the bf16 MFMA rate they are bound by HBM and the three products cost
// no time; bias, residual and activation are applied in the epilogue rather
// than in passes of their own over C.
#include "ops.h"

namespace nqs {
namespace {

typedef __attribute__((ext_vector_type(8))) __bf16 bf16x8;
typedef __attribute__((ext_vector_type(2))) __bf16 bf16x2;
typedef __attribute__((ext_vector_type(2))) float f32x2;
typedef __attribute__((ext_vector_type(4))) float f32x4;
typedef __attribute__((ext_vector_type(16))) float f32x16;

constexpr int kBN = 128;                      // columns of a chunk of the right operand
constexpr int kBK = 32;                       // k of a slab
constexpr int kLdsRow = 40;                   // bf16 per LDS row of a slab: 32 k + 8 padding
constexpr int kSlabEntries = kBN * kBK / 8;   // bf16x8 entries of one part (hi or lo) of a slab

// hi = bf16(v) (round to nearest even), lo = bf16(v - hi)
__device__ inline void split8(const float (&v)[8], bf16x8 &hi, bf16x8 &lo) {
#pragma unroll
  for (int i = 0; i < 8; i += 2) {
    const f32x2 p = {v[i], v[i + 1]};
    const bf16x2 h = __builtin_convertvector(p, bf16x2);
    const f32x2 r = {v[i] - float(h[0]), v[i + 1] - float(h[1])};
    const bf16x2 l = __builtin_convertvector(r, bf16x2);
    hi[i] = h[0];
    hi[i + 1] = h[1];
    lo[i] = l[0];
    lo[i + 1] = l[1];
  }
}

// The tanh form of GELU, 0.5 x (1 + tanh u) with u = sqrt(2/pi) (x + 0.044715 x^3),
// written as x s with s = 1 / (1 + e^{-2u}) (hardware exp2 and reciprocal,
// about 1 ulp each), and its derivative s + 2 x s (1 - s) du/dx
// (tanh u = 2 s - 1, 1 - tanh^2 u = 4 s (1 - s)).
constexpr float kGeluC = 0.7978845608028654f;   // sqrt(2/pi)
__device__ inline float gelu_sig(float x, float &s) {
  const float e = __builtin_amdgcn_exp2f(-2.0f * 1.4426950408889634f * kGeluC * x *
                                         fmaf(0.044715f, x * x, 1.0f));
  s = __builtin_amdgcn_rcpf(1.0f + e);
  return x * s;
}
__device__ inline float gelu_fast(float x) {
  float s;
  return gelu_sig(x, s);
}
__device__ inline float gelu_grad_fast(float x) {
  float s;
  gelu_sig(x, s);
  return fmaf(2.0f * x * s * (1.0f - s), kGeluC * fmaf(3.0f * 0.044715f, x * x, 1.0f), s);
}

__device__ inline f32x16 mfma(const bf16x8 &a, const bf16x8 &b, const f32x16 &c) {
  return __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, c, 0, 0, 0);
}

// Right operand image: for chunk ch (columns ch*128 ..) and slab s (k = s*32 ..)
// the hi part, then the lo part, each [n 0..127][k 0..31] bf16 (entry
// n * 4 + k / 8 of 8 consecutive k); columns past N are zero.
__global__ void mx_pack_kernel(const float *__restrict__ W, int64_t ldw, int trans, int N, int K,
                               bf16x8 *__restrict__ out) {
  const int slabs = K / kBK, chunks = (N + kBN - 1) / kBN;
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= int64_t(chunks) * slabs * kSlabEntries) return;
  const int e = int(i % kSlabEntries), cs = int(i / kSlabEntries);
  const int n = e / 4, kq = e % 4, s = cs % slabs, ch = cs / slabs;
  const int col = ch * kBN + n;
  float v[8];
#pragma unroll
  for (int j = 0; j < 8; ++j) {
    const int64_t k = int64_t(s) * kBK + kq * 8 + j;
    v[j] = col < N ? (trans ? W[int64_t(col) * ldw + k] : W[k * ldw + col]) : 0.f;
  }
  bf16x8 hi, lo;
  split8(v, hi, lo);
  out[(int64_t(cs) * 2) * kSlabEntries + e] = hi;
  out[(int64_t(cs) * 2 + 1) * kSlabEntries + e] = lo;
}

struct MxArgs {
  const float *A;
  int64_t lda;
  const bf16x8 *W;        // right operand image (mx_pack_kernel)
  float *C;
  int64_t ldc;
  const float *res;       // MX_ADD: residual input (not C)
  int64_t ldr;
  const float *bias;      // optional, per column
  float *aux;             // MX_GELU: pre-activation out; MX_DGELU: pre-activation in (ld = ldc)
  int64_t M;
  int N, K;
};

// One block per 128 rows of A (wave w: rows 32w .. 32w + 31 as the MFMA's A
// operand, read from HBM / L2 straight into registers); the block walks the
// chunks of 128 columns, and for each the slabs of 32 k, the slab's right
// operand staged in LDS (double-buffered, one barrier per slab).  The next
// slab's right operand and A values are loaded into registers while the
// current slab multiplies.  Lane l supplies row l % 32 and k = 8 (l / 32) ..
// + 7 of a 16-k step to both operands; accumulator element v of lane l is row
// (v/4)*8 + (l/32)*4 + v%4, column l % 32 of its 32 x 32 tile.  Rows past M
// read row M - 1 and are not stored; every wave takes part in every barrier.
template <int EPI>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(3)))
mx_gemm_kernel(MxArgs a) {
  __shared__ __attribute__((aligned(16))) __bf16 sB[2][2][kBN * kLdsRow];
  const int lane = threadIdx.x % 64, w = threadIdx.x / 64, c = lane % 32, kg = lane / 32;
  const int64_t row0 = int64_t(blockIdx.x) * 128 + w * 32;
  const int64_t arow = row0 + c < a.M ? row0 + c : a.M - 1;
  const float *__restrict__ Ar = a.A + arow * a.lda + kg * 8;
  float *__restrict__ C = a.C;
  const float *__restrict__ res = a.res;
  float *__restrict__ aux = a.aux;
  const int chunks = (a.N + kBN - 1) / kBN, slabs = a.K / kBK, total = chunks * slabs;
  // slab image g: thread t copies its entries t + 256 j (j < 4; hi: j < 2, lo: j >= 2)
  bf16x8 stg[4];
  auto stage_load = [&](int g) {
    const bf16x8 *src = a.W + int64_t(g) * 2 * kSlabEntries + threadIdx.x;
#pragma unroll
    for (int j = 0; j < 4; ++j) stg[j] = src[256 * j];
  };
  auto stage_store = [&](int buf) {
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int e = int(threadIdx.x) + 256 * (j % 2);
      *reinterpret_cast<bf16x8 *>(&sB[buf][j / 2][(e / 4) * kLdsRow + (e % 4) * 8]) = stg[j];
    }
  };
  // A values of slab s: two 16-k steps of 8
  f32x4 av[4];
  auto a_load = [&](int s) {
#pragma unroll
    for (int j = 0; j < 4; ++j) av[j] = *reinterpret_cast<const f32x4 *>(Ar + s * kBK + j * 4 + (j / 2) * 8);
  };
  stage_load(0);
  a_load(0);
  f32x16 acc[4] = {};
  for (int g = 0; g < total; ++g) {
    const int ch = g / slabs, s = g % slabs, buf = g & 1;
    // the buffer written here was last read two slabs ago, before the
    // previous barrier
    stage_store(buf);
    if (g + 1 < total) stage_load(g + 1);
    __syncthreads();
    bf16x8 ahi[2], alo[2];
#pragma unroll
    for (int ks = 0; ks < 2; ++ks) {
      const float v[8] = {av[2 * ks][0], av[2 * ks][1], av[2 * ks][2], av[2 * ks][3],
                          av[2 * ks + 1][0], av[2 * ks + 1][1], av[2 * ks + 1][2], av[2 * ks + 1][3]};
      split8(v, ahi[ks], alo[ks]);
    }
    if (g + 1 < total) a_load((g + 1) % slabs);
#pragma unroll
    for (int ks = 0; ks < 2; ++ks)
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        const int off = (t * 32 + c) * kLdsRow + ks * 16 + kg * 8;
        const bf16x8 bhi = *reinterpret_cast<const bf16x8 *>(&sB[buf][0][off]);
        const bf16x8 blo = *reinterpret_cast<const bf16x8 *>(&sB[buf][1][off]);
        acc[t] = mfma(ahi[ks], bhi, acc[t]);
        acc[t] = mfma(ahi[ks], blo, acc[t]);
        acc[t] = mfma(alo[ks], bhi, acc[t]);
      }
    if (s + 1 < slabs) continue;
    // epilogue of chunk ch: per 32-column tile, the inputs first, then the
    // stores; a lane's rows are row0 + 4 (l / 32) + r_v with the wave-uniform
    // r_v = (v/4)*8 + v%4
    const int64_t lrow = row0 + kg * 4;
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      const int col = ch * kBN + t * 32 + c;
      const bool cin = col < a.N;
      const float b = a.bias && cin ? a.bias[col] : 0.f;
      float *cb = C + lrow * a.ldc + col;
      const float *rb = EPI == MX_ADD ? res + lrow * a.ldr + col : nullptr;
      float *xb = EPI == MX_GELU || EPI == MX_DGELU ? aux + lrow * a.ldc + col : nullptr;
      float in[16];
#pragma unroll
      for (int v = 0; v < 16; ++v) {
        const int rv = (v / 4) * 8 + v % 4;
        const bool ok = cin && lrow + rv < a.M;
        in[v] = 0.f;
        if (EPI == MX_ADD && ok) in[v] = rb[rv * a.ldr];
        if (EPI == MX_DGELU && ok) in[v] = xb[rv * a.ldc];
      }
#pragma unroll
      for (int v = 0; v < 16; ++v) {
        const int rv = (v / 4) * 8 + v % 4;
        if (!cin || lrow + rv >= a.M) continue;
        const float x = acc[t][v] + b;
        if (EPI == MX_STORE) {
          cb[rv * a.ldc] = x;
        } else if (EPI == MX_ADD) {
          cb[rv * a.ldc] = in[v] + x;
        } else if (EPI == MX_GELU) {
          xb[rv * a.ldc] = x;
          cb[rv * a.ldc] = gelu_fast(x);
        } else {
          cb[rv * a.ldc] = x * gelu_grad_fast(in[v]);
        }
      }
      acc[t] = f32x16{};
      __builtin_amdgcn_sched_barrier(0);   // one tile's inputs live at a time
    }
  }
}

constexpr int kWRows = 32;            // rows of a weight-gradient slab
constexpr int kWLds = kWRows + 8;     // bf16 per LDS column of a slab (padded)

// Weight-gradient partial sums with split operands:
//     part[z][i][j] = sum over the rows r of slice z of X[r][i] * dY[r][j].
// One block per (128 x 128 output tile, row slice); wave w owns the 64 x 64
// quarter (w / 2, w % 2) as 2 x 2 accumulator blocks.  The slice is walked in
// slabs of 32 rows: thread t loads column t % 128 of the tile's columns of X
// and of dY, rows 16 (t / 128) .. + 15 of the slab (each load instruction
// reads whole rows of 128 consecutive columns), splits them and stores them
// column-major in LDS, so that a lane's MFMA operand (8 consecutive rows of
// one column, hi or lo) is one 16-byte read.  The next slab's values are
// loaded while the current one multiplies.  The slice's rows are read through
// buffer resources that end at its last row (the whole offset in the per-lane
// offset), so rows past it read as zeros; a column past M (N) reads whatever
// lies there in the slice (the next row's entries, or zero past its end),
// which only feeds accumulator rows (columns) that are never stored.  The
// host keeps a slice under 1 GiB of either matrix.  With bpart, the blocks of
// the first row of output tiles also sum dY's columns over the slice from the
// fp32 values they load (double sums in a fixed order): bpart[z][j].
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2)))
mx_wgrad_kernel(const float *__restrict__ X, int64_t ldx, const float *__restrict__ dY,
                int64_t ldy, int64_t R, int M, int N, int64_t rows_per, int tiles_n,
                float *__restrict__ part, double *__restrict__ bpart) {
  __shared__ __attribute__((aligned(16))) __bf16 sW[4][128 * kWLds];   // X hi, X lo, dY hi, dY lo
  __shared__ double sbias[128];
  const int lane = threadIdx.x % 64, w = threadIdx.x / 64, c = lane % 32, kg = lane / 32;
  const int tm = int(blockIdx.x) / tiles_n, tn = int(blockIdx.x) % tiles_n;
  const int i0 = tm * 128, j0 = tn * 128;
  const int wi = (w / 2) * 64, wj = (w % 2) * 64;
  const int64_t r0 = int64_t(blockIdx.y) * rows_per;
  const int64_t r1 = r0 + rows_per < R ? r0 + rows_per : R;
  const int rows = int(r1 - r0);
  const auto rx = __builtin_amdgcn_make_buffer_rsrc(const_cast<float *>(X + r0 * ldx), 0,
                                                    int(int64_t(rows) * ldx * 4), 0x00020000);
  const auto ry = __builtin_amdgcn_make_buffer_rsrc(const_cast<float *>(dY + r0 * ldy), 0,
                                                    int(int64_t(rows) * ldy * 4), 0x00020000);
  const uint32_t lx = uint32_t(ldx) * 4, ly = uint32_t(ldy) * 4;   // bytes per row
  const int sc = int(threadIdx.x) % 128, sr = (int(threadIdx.x) / 128) * 16;
  const uint32_t cx = uint32_t(i0 + sc) * 4, cy = uint32_t(j0 + sc) * 4;
  float vx[16], vy[16];
  auto load = [&](int r) {   // rows r + sr .. r + sr + 15 of the slice
    uint32_t ox = uint32_t(r + sr) * lx + cx, oy = uint32_t(r + sr) * ly + cy;
#pragma unroll
    for (int u = 0; u < 16; ++u) {
      vx[u] = __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(rx, int(ox), 0, 0));
      vy[u] = __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(ry, int(oy), 0, 0));
      ox += lx;
      oy += ly;
    }
  };
  auto store = [&]() {
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      bf16x8 hi, lo;
      const float *px = vx + 8 * h, *py = vy + 8 * h;
      const float tx[8] = {px[0], px[1], px[2], px[3], px[4], px[5], px[6], px[7]};
      split8(tx, hi, lo);
      *reinterpret_cast<bf16x8 *>(&sW[0][sc * kWLds + sr + 8 * h]) = hi;
      *reinterpret_cast<bf16x8 *>(&sW[1][sc * kWLds + sr + 8 * h]) = lo;
      const float ty[8] = {py[0], py[1], py[2], py[3], py[4], py[5], py[6], py[7]};
      split8(ty, hi, lo);
      *reinterpret_cast<bf16x8 *>(&sW[2][sc * kWLds + sr + 8 * h]) = hi;
      *reinterpret_cast<bf16x8 *>(&sW[3][sc * kWLds + sr + 8 * h]) = lo;
    }
  };
  f32x16 acc[2][2] = {};
  const bool bias = bpart && tm == 0;
  double bsum = 0.0;
  const int nslab = (rows + kWRows - 1) / kWRows;
  load(0);
  for (int g = 0; g < nslab; ++g) {
    if (bias) {
#pragma unroll
      for (int u = 0; u < 16; ++u) bsum += double(vy[u]);
    }
    store();
    __syncthreads();
    if (g + 1 < nslab) load((g + 1) * kWRows);
#pragma unroll
    for (int ks = 0; ks < 2; ++ks) {
      bf16x8 ah[2], al[2], bh[2], bl[2];
#pragma unroll
      for (int q = 0; q < 2; ++q) {
        const int oa = (wi + 32 * q + c) * kWLds + ks * 16 + kg * 8;
        const int ob = (wj + 32 * q + c) * kWLds + ks * 16 + kg * 8;
        ah[q] = *reinterpret_cast<const bf16x8 *>(&sW[0][oa]);
        al[q] = *reinterpret_cast<const bf16x8 *>(&sW[1][oa]);
        bh[q] = *reinterpret_cast<const bf16x8 *>(&sW[2][ob]);
        bl[q] = *reinterpret_cast<const bf16x8 *>(&sW[3][ob]);
      }
#pragma unroll
      for (int bi = 0; bi < 2; ++bi)
#pragma unroll
        for (int bj = 0; bj < 2; ++bj) {
          acc[bi][bj] = mfma(ah[bi], bh[bj], acc[bi][bj]);
          acc[bi][bj] = mfma(ah[bi], bl[bj], acc[bi][bj]);
          acc[bi][bj] = mfma(al[bi], bh[bj], acc[bi][bj]);
        }
    }
    __syncthreads();
  }
  if (bias) {   // the two row groups of each column: sr = 16 into LDS, sr = 0 adds
    if (sr != 0) sbias[sc] = bsum;
    __syncthreads();
    if (sr == 0 && j0 + sc < N) bpart[int64_t(blockIdx.y) * N + j0 + sc] = bsum + sbias[sc];
  }
  float *pz = part + int64_t(blockIdx.y) * M * N;
#pragma unroll
  for (int bi = 0; bi < 2; ++bi)
#pragma unroll
    for (int bj = 0; bj < 2; ++bj) {
      const int j = j0 + wj + 32 * bj + c;
      if (j >= N) continue;
#pragma unroll
      for (int v = 0; v < 16; ++v) {
        const int i = i0 + wi + 32 * bi + (v / 4) * 8 + kg * 4 + v % 4;
        if (i < M) pz[int64_t(i) * N + j] = acc[bi][bj][v];
      }
    }
}

}  // namespace

bool mx_supported(int64_t N, int64_t K) {
  return N > 0 && K > 0 && N % 32 == 0 && K % kBK == 0 && N < (int64_t(1) << 24) &&
         K < (int64_t(1) << 24);
}

size_t mx_pack_bytes(int64_t N, int64_t K) {
  return size_t(ceil_div(N, kBN)) * size_t(K / kBK) * 2 * kSlabEntries * sizeof(bf16x8);
}

void mx_pack(const float *W, int64_t ldw, bool trans, int64_t N, int64_t K, void *out,
             hipStream_t s) {
  NQS_REQUIRE(mx_supported(N, K), NQS_EUNSUPPORTED, "mixed product: N % 32, K % 32 required");
  const int64_t items = ceil_div(N, kBN) * (K / kBK) * kSlabEntries;
  hipLaunchKernelGGL(mx_pack_kernel, dim3(unsigned(ceil_div(items, 256))), dim3(256), 0, s, W, ldw,
                     trans ? 1 : 0, int(N), int(K), static_cast<bf16x8 *>(out));
  HIP_LAUNCH_OK();
}

void mx_gemm(int64_t M, int64_t N, int64_t K, const float *A, int64_t lda, const void *Wp, float *C,
             int64_t ldc, const float *res, int64_t ldr, const float *bias, float *aux, int epi,
             hipStream_t s) {
  if (M <= 0 || N <= 0) return;
  NQS_REQUIRE(mx_supported(N, K), NQS_EUNSUPPORTED, "mixed product: N % 32, K % 32 required");
  NQS_REQUIRE(lda % 4 == 0 && (reinterpret_cast<uintptr_t>(A) & 15) == 0, NQS_EINVAL,
              "mixed product: A rows must be 16-byte aligned");
  NQS_REQUIRE((epi != MX_ADD || (res && res != C)) && (epi != MX_GELU && epi != MX_DGELU || aux) &&
                  (epi != MX_DGELU || !bias),
              NQS_EINVAL, "mixed product: epilogue operands");
  NQS_REQUIRE(ceil_div(M, 128) < (int64_t(1) << 31), NQS_EUNSUPPORTED, "mixed product: M too large");
  MxArgs a{A, lda, static_cast<const bf16x8 *>(Wp), C, ldc, res, ldr, bias, aux, M, int(N), int(K)};
  const dim3 grid(unsigned(ceil_div(M, 128)));
  switch (epi) {
    case MX_STORE: hipLaunchKernelGGL(mx_gemm_kernel<MX_STORE>, grid, dim3(256), 0, s, a); break;
    case MX_ADD: hipLaunchKernelGGL(mx_gemm_kernel<MX_ADD>, grid, dim3(256), 0, s, a); break;
    case MX_GELU: hipLaunchKernelGGL(mx_gemm_kernel<MX_GELU>, grid, dim3(256), 0, s, a); break;
    case MX_DGELU: hipLaunchKernelGGL(mx_gemm_kernel<MX_DGELU>, grid, dim3(256), 0, s, a); break;
    default: NQS_REQUIRE(false, NQS_EINVAL, "mixed product: unknown epilogue");
  }
  HIP_LAUNCH_OK();
}

void mx_wgrad_partials(const float *X, int64_t ldx, const float *dY, int64_t ldy, int64_t R,
                       int64_t M, int64_t N, int64_t rows_per, float *part, double *bpart,
                       hipStream_t s) {
  const int tiles_n = int(ceil_div(N, int64_t(128)));
  const int64_t tiles = ceil_div(M, int64_t(128)) * tiles_n;
  const dim3 grid = dim3(unsigned(tiles), unsigned(ceil_div(R, rows_per)));
  hipLaunchKernelGGL(mx_wgrad_kernel, grid, dim3(256), 0, s, X, ldx, dY, ldy, R, int(M), int(N),
                     rows_per, tiles_n, part, bpart);
  HIP_LAUNCH_OK();
}

}  // namespace nqs
