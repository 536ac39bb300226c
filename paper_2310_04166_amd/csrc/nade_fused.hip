// Fused bf16 forward of the paper's per-qubit complex-weight ansatz on MFMA
// (gfx950): log|psi| and phase of a batch of configurations.  Paper: Appendix
// "ANQS architecture" (one MLP per qubit, complex tanh, split leaky ReLU,
// LogSumExp normaliser) and "Pruning strategies" (Mask-Unphysical per qubit).
//
// Design.  One 64-lane wave owns 32 configurations and walks all 2n qubits in
// registers; nothing but the configurations, the weights and the two outputs
// touches memory.  Per qubit i the three complex layers are real GEMMs with
// the block matrices of nade_pack ([Re h, Im h] times [[Re W, Im W], [-Im W,
// Re W]]), run as v_mfma_f32_32x32x16_bf16 with the weights as the A operand
// (rows = output features) and the activations as the B operand (columns =
// the 32 configurations).  An accumulator block then holds 32 features x 32
// configurations, lane l owning configuration l%32 and, for j = 0..15,
// feature (j/4)*8 + (l/32)*4 + j%4 of the block; converted to bf16 it is the
// B operand of the next GEMM when the k index inside each 16-wide step is
// permuted the same way in the packed weights (as in the transformer kernel).
//   layer 1: 128 features (64 Re | 64 Im) from the i prefix bits; the bits
//            are the B operand (exact in bf16), W1 rows >= i are zero;
//   tanh:    feature f and 64 + f sit in the same lane and row, so the
//            complex tanh is lane-local: with r = e^{-2|a|},
//            tanh(a + ib) = (sgn(a)(1 - r^2) + 2i r sin 2b) / (1 + 2r cos 2b + r^2);
//   layer 2: 128 x 128 block matrix, 32 MFMAs; split leaky ReLU (slope 0.01);
//   layer 3: the 4 outputs (Re z0, Re z1, Im z0, Im z1) as rows 0..3 of one
//            32-row block (the other weight rows are zero and not loaded);
//   combine: lanes 0..31 hold z of their configuration: Mask-Unphysical on
//            the qubit's two values, log psi_i(v) = z_v - LSE(2 Re z)/2,
//            log|psi| and phase accumulated in double.
// The inputs of layers 2 and 3 (tanh and leaky-ReLU outputs) enter as bf16
// pairs hi + lo (lo = the rounding error of hi, two MFMAs per product): with
// single bf16 operands the local energy of the dominant samples of the
// 30-qubit system was 6.7e-4 Ha off the FP64 oracle (7e-7 Ha with the pairs),
// the per-sample local energies 8e-3 Ha on average (1e-5 Ha).
// Per qubit and wave: 4 ceil(i/16) + 64 + 16 MFMAs and 2048 complex tanh; the
// tanh (four transcendentals each) bounds the kernel, not HBM (8 bytes in and
// 16 bytes out per configuration).
#include <cmath>
#include <vector>

#include "model.h"

namespace nqs {
namespace {

typedef __attribute__((ext_vector_type(8))) __bf16 bf16x8;
typedef __attribute__((ext_vector_type(2))) __bf16 bf16x2;
typedef __attribute__((ext_vector_type(16))) float f32x16;
typedef __attribute__((ext_vector_type(2))) float f32x2;
typedef __attribute__((ext_vector_type(4))) float f32x4;
typedef __attribute__((ext_vector_type(4))) uint32_t u32x4;

constexpr int kHid = 64;                 // complex hidden width (128 real features)
constexpr int kFeat = 2 * kHid;
constexpr int kVec = 2 * kFeat + 4;      // per-qubit fp32 vectors: b1, b2 (permuted), b3
constexpr int kMaxQubits = 64;
constexpr int kWaves = 4;                // waves per block, 32 configurations each

struct NadeArgs {
  const bf16x8 *frag;                    // weight fragments, 64 per fragment set
  const float *vec;                      // kVec floats per qubit
  int32_t fo[kMaxQubits];                // first fragment set of qubit i
  Sectors sec;
  const uint64_t *x;
  int64_t B;                             // configurations (capacity when `count` is given)
  const int64_t *count;                  // optional device-side count
  int N;                                 // qubits (2n)
  int cond_p;                            // token of the conditional mode
  double *logabs, *phase;                // forward mode (either may be null)
  double *cond;                          // conditional mode: [B x 4] token log-probabilities
};

__device__ __host__ inline int feat_of(int h, int j) { return (j / 4) * 8 + h * 4 + (j % 4); }

__device__ inline f32x16 mfma(const bf16x8 &a, const bf16x8 &b, const f32x16 &c) {
  return __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, c, 0, 0, 0);
}

__device__ inline f32x16 load16(const float *p) {
  const f32x4 *q = reinterpret_cast<const f32x4 *>(p);
  const f32x4 a = q[0], b = q[1], c = q[2], d = q[3];
  f32x16 r;
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    r[i] = a[i];
    r[4 + i] = b[i];
    r[8 + i] = c[i];
    r[12 + i] = d[i];
  }
  return r;
}

__device__ inline bf16x8 pack8(const float (&v)[8]) {
  bf16x8 r;
#pragma unroll
  for (int i = 0; i < 8; i += 2) {
    const f32x2 p = {v[i], v[i + 1]};
    const bf16x2 q = __builtin_convertvector(p, bf16x2);
    r[i] = q[0];
    r[i + 1] = q[1];
  }
  return r;
}

// v = hi + lo, both bf16 (lo is the rounding error of hi)
__device__ inline void pack8_hilo(const float (&v)[8], bf16x8 &hi, bf16x8 &lo) {
  hi = pack8(v);
  float r[8];
#pragma unroll
  for (int i = 0; i < 8; ++i) r[i] = v[i] - float(hi[i]);
  lo = pack8(r);
}

// bits first .. first+7 of occ as bf16 0.0 / 1.0 (0x3F80), in natural order
__device__ inline bf16x8 bits_frag(uint64_t occ, int first) {
  const uint32_t byte = uint32_t(occ >> first) & 0xFFu;
  u32x4 w;
#pragma unroll
  for (int m = 0; m < 4; ++m)
    w[m] = ((byte >> (2 * m)) & 1u) * 0x3F80u | ((byte >> (2 * m + 1)) & 1u) * 0x3F800000u;
  return __builtin_bit_cast(bf16x8, w);
}

// complex tanh from hardware exp2 / sin / cos / reciprocal (about 1 ulp each in
// fp32, far below the bf16 rounding of the result); v_sin / v_cos take
// revolutions, reduced to [0, 1) first
__device__ inline void ctanh(float a, float b, float &re, float &im) {
  constexpr float kM2Log2e = -2.0f * 1.4426950408889634f;
  constexpr float kInvPi = 0.3183098861837907f;     // 2b radians = b / pi revolutions
  const float r = __builtin_amdgcn_exp2f(fabsf(a) * kM2Log2e);
  const float u = __builtin_amdgcn_fractf(b * kInvPi);
  const float sn = __builtin_amdgcn_sinf(u), cs = __builtin_amdgcn_cosf(u);
  const float r2 = r * r, tr = r + r;
  const float inv = __builtin_amdgcn_rcpf(fmaf(tr, cs, 1.0f + r2));
  re = copysignf((1.0f - r2) * inv, a);
  im = tr * sn * inv;
}

// (Re z0, Re z1, Im z0, Im z1) of qubit i for the wave's 32 configurations,
// whose bits below i are those of occ; valid in lanes 0..31 (lane = column)
__device__ inline f32x4 qubit_z(const NadeArgs &a, int i, uint64_t occ, int lane) {
  const int h = lane >> 5, col = lane & 31;
  const bf16x8 *W = a.frag + int64_t(a.fo[i]) * 64 + lane;
  const float *V = a.vec + int64_t(i) * kVec;
  const int ks = (i + 15) >> 4;
  // layer 1 and the complex tanh, one pair of blocks (Re features 32b.., Im
  // features 64 + 32b..) at a time, so that at most 32 accumulators are live;
  // the tanh outputs as hi (hf) + lo (hl)
  bf16x8 hf[8], hl[8];
#pragma unroll
  for (int b = 0; b < 2; ++b) {
    f32x16 ar = load16(V + (2 * b + h) * 16), ai = load16(V + (2 * (b + 2) + h) * 16);
    for (int k = 0; k < ks; ++k) {
      const bf16x8 xb = bits_frag(occ, 16 * k + 8 * h);
      ar = mfma(W[(b * ks + k) * 64], xb, ar);
      ai = mfma(W[((b + 2) * ks + k) * 64], xb, ai);
    }
#pragma unroll
    for (int u = 0; u < 2; ++u) {
      float re[8], im[8];
#pragma unroll
      for (int e = 0; e < 8; ++e) ctanh(ar[8 * u + e], ai[8 * u + e], re[e], im[e]);
      pack8_hilo(re, hf[2 * b + u], hl[2 * b + u]);
      pack8_hilo(im, hf[4 + 2 * b + u], hl[4 + 2 * b + u]);
    }
  }
  W += 4 * ks * 64;
  // layer 2 one output block at a time, leaky ReLU applied at once; its
  // outputs (as hi + lo) enter layer 3 right away, whose input k-step 2t + u is
  // half u of layer 2's output block t, so no layer-3 operand is kept
  const bf16x8 *W3 = W + 32 * 64;
  f32x16 z = {};
  const bf16x8 zero = {};
#pragma unroll
  for (int t = 0; t < 4; ++t) {
    f32x16 c = load16(V + kFeat + (2 * t + h) * 16);
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      const bf16x8 w = W[(t * 8 + k) * 64];
      c = mfma(w, hl[k], mfma(w, hf[k], c));
    }
#pragma unroll
    for (int u = 0; u < 2; ++u) {
      float v[8];
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        const float y = c[8 * u + e];
        v[e] = fmaxf(y, 0.01f * y);
      }
      bf16x8 g, gl;
      pack8_hilo(v, g, gl);
      const bf16x8 w3 = col < 4 ? W3[(2 * t + u) * 64] : zero;
      z = mfma(w3, gl, mfma(w3, g, z));
    }
  }
  const float *b3 = V + 2 * kFeat;
  return f32x4{z[0] + b3[0], z[1] + b3[1], z[2] + b3[2], z[3] + b3[3]};
}

// log psi_i(0), log psi_i(1) (real parts) under Mask-Unphysical: the network's
// normalised conditionals when unmasked or both values are physical, else 0
// for the physical value and -inf for the other
__device__ inline void qubit_logp(const f32x4 &z, bool masked, bool ok0, bool ok1, float &l0,
                                  float &l1) {
  if (!masked || (ok0 && ok1)) {
    constexpr float kLog2e = 1.4426950408889634f, kLn2 = 0.6931471805599453f;
    const float r0 = 2.0f * z[0], r1 = 2.0f * z[1], mx = fmaxf(r0, r1);
    const float lse = mx + kLn2 * __builtin_amdgcn_logf(__builtin_amdgcn_exp2f((r0 - mx) * kLog2e) +
                                                        __builtin_amdgcn_exp2f((r1 - mx) * kLog2e));
    l0 = z[0] - 0.5f * lse;
    l1 = z[1] - 0.5f * lse;
  } else {
    l0 = ok0 ? 0.0f : -INFINITY;
    l1 = ok1 ? 0.0f : -INFINITY;
  }
}

// kCond: the sampler's conditional mode (its own kernel, so that the three
// evaluations it keeps do not raise the forward's register allocation)
template <bool kCond>
__device__ inline void nade_body(const NadeArgs &a) {
  const int lane = threadIdx.x & 63, h = lane >> 5, col = lane & 31;
  const int64_t B = a.count ? (*a.count < a.B ? *a.count : a.B) : a.B;
  const int64_t c0 = (int64_t(blockIdx.x) * kWaves + (threadIdx.x >> 6)) * 32;
  if (c0 >= B) return;                   // whole waves only: no block-level barrier follows
  const int64_t cfg = c0 + col;
  const bool valid = cfg < B;
  const uint64_t xw = a.x[valid ? cfg : c0];
  const nqs_sector_info &si = sector_of(a.sec, xw);
  const uint64_t occ = occupation(a.sec, xw);
  const int mask_levels = si.mask_levels;
  if (kCond) {
    // token p of the four-way sampler: qubit 2p on the prefix, qubit 2p + 1
    // on the prefix extended by a = 0 and a = 1; outputs the token
    // log-probabilities 2 (log|psi_2p(a)| + log|psi_2p+1(b | a)|), k = a + 2b
    const int p = a.cond_p;
    const uint64_t below = p == 0 ? 0ull : (~0ull >> (64 - 2 * p));
    const uint64_t pre = occ & below;
    const f32x4 zA = qubit_z(a, 2 * p, pre, lane);
    const f32x4 zB0 = qubit_z(a, 2 * p + 1, pre, lane);
    const f32x4 zB1 = qubit_z(a, 2 * p + 1, pre | (1ull << (2 * p)), lane);
    const bool masked = p < mask_levels;
    const int phys = masked ? phys_mask(a.sec, si, p, __popcll(pre & 0x5555555555555555ull),
                                        __popcll(pre & 0xAAAAAAAAAAAAAAAAull), pre)
                            : 0xF;
    float lA[2], lB[2][2];
    qubit_logp(zA, masked, (phys & 5) != 0, (phys & 10) != 0, lA[0], lA[1]);
    qubit_logp(zB0, masked, (phys & 1) != 0, (phys & 4) != 0, lB[0][0], lB[0][1]);
    qubit_logp(zB1, masked, (phys & 2) != 0, (phys & 8) != 0, lB[1][0], lB[1][1]);
    if (h == 0 && valid) {
#pragma unroll
      for (int k = 0; k < 4; ++k)
        a.cond[cfg * 4 + k] = 2.0 * (double(lA[k & 1]) + double(lB[k & 1][k >> 1]));
    }
    return;
  }
  double la = 0.0, ph = 0.0;
  int na = 0, nb = 0, phys = 0xF;
  for (int i = 0; i < a.N; ++i) {
    const f32x4 z = qubit_z(a, i, occ, lane);
    // Mask-Unphysical on the qubit's two values; lanes 0..31 hold its z
    const int p = i >> 1, v = int((occ >> i) & 1);
    const bool masked = p < mask_levels;
    if ((i & 1) == 0 && masked) phys = phys_mask(a.sec, si, p, na, nb, occ);
    bool ok0, ok1;
    if ((i & 1) == 0) {
      ok0 = (phys & 5) != 0;
      ok1 = (phys & 10) != 0;
    } else {
      const int al = int((occ >> (i - 1)) & 1);
      ok0 = ((phys >> al) & 1) != 0;
      ok1 = ((phys >> (al + 2)) & 1) != 0;
    }
    float l0, l1;
    qubit_logp(z, masked, ok0, ok1, l0, l1);
    la += double(v ? l1 : l0);
    if (!masked || (ok0 && ok1)) ph += double(v ? z[3] : z[2]);
    if (i & 1) {
      na += int((occ >> (i - 1)) & 1);
      nb += v;
    }
  }
  if (h == 0 && valid) {
    if (a.logabs) a.logabs[cfg] = la;
    if (a.phase) a.phase[cfg] = ph;
  }
}

// three waves per SIMD (163 registers): the kernel is latency-bound and more
// waves help, but at four the hi / lo operands spill (36 bytes per lane, 5 %
// slower than three)
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(3, 3)))
nade_fused_kernel(NadeArgs a) {
  nade_body<false>(a);
}

__global__ void __launch_bounds__(256) nade_cond_kernel(NadeArgs a) { nade_body<true>(a); }

// Fragment order: (block ob, k-step s, lane l, slot e) <- W[krow][32 ob + l%32]
// with krow = 16 s + 8 (l/32) + e (natural, for the bit input) or
// 16 s + feat_of(l/32, e) (permuted, for accumulator inputs); rows >= rows and
// columns >= cols read zero.  W row-major with leading dimension ld.
__device__ inline __bf16 frag_value(const float *W, int rows, int ld, int cols, int n_ks,
                                    bool natural, int64_t e) {
  const int slot = int(e % 8), l = int((e / 8) % 64);
  const int s = int((e / 512) % n_ks), ob = int(e / (512 * int64_t(n_ks)));
  const int hh = l / 32;
  const int krow = 16 * s + (natural ? 8 * hh + slot : feat_of(hh, slot));
  const int c = 32 * ob + l % 32;
  return __bf16(krow < rows && c < cols ? W[int64_t(krow) * ld + c] : 0.0f);
}

// one qubit: its W1 (natural, i rows), W2 and W3 (permuted) fragments and its
// vectors b1, b2 in accumulator order, b3 as is
__global__ void nade_frag_kernel(const float *W1, const float *B1, const float *W2,
                                 const float *B2, const float *W3, const float *B3, int i, int ks,
                                 __bf16 *frag, float *vec) {
  const int64_t e = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  const int64_t n1 = int64_t(4) * ks * 512, n2 = int64_t(32) * 512, n3 = int64_t(8) * 512;
  if (e < n1) {
    frag[e] = frag_value(W1, i, kFeat, kFeat, ks, true, e);
  } else if (e < n1 + n2) {
    frag[e] = frag_value(W2, kFeat, kFeat, kFeat, 8, false, e - n1);
  } else if (e < n1 + n2 + n3) {
    frag[e] = frag_value(W3, kFeat, 4, 4, 8, false, e - n1 - n2);
  } else if (e < n1 + n2 + n3 + kVec) {
    const int c = int(e - n1 - n2 - n3);
    if (c < 2 * kFeat) {
      const float *src = c < kFeat ? B1 : B2;
      const int cc = c % kFeat, j = cc % 16, hh = (cc / 16) % 2, b = cc / 32;
      vec[c] = src[32 * b + feat_of(hh, j)];
    } else {
      vec[c] = B3[c - 2 * kFeat];
    }
  }
}

inline int qubit_sets(int i) { return 4 * ((i + 15) / 16) + 32 + 8; }

}  // namespace

bool nade_fused_supported(const nqs_model &m) {
  return m.kind == NQS_MODEL_NADE && m.hid == kHid && 2 * m.n <= kMaxQubits;
}

void nade_fused_pack(nqs_model &m, hipStream_t s) {
  NQS_REQUIRE(nade_fused_supported(m), NQS_EUNSUPPORTED,
              "fused forward: the per-qubit ansatz needs hidden width 64 and at most 64 qubits");
  NQS_REQUIRE(!m.fp64() && m.nade_off.size() == size_t(2 * m.n) * 6, NQS_EINVAL,
              "fused forward: fp32 block matrices are not packed");
  const int N = 2 * m.n;
  m.nade_fo.assign(size_t(N), 0);
  int64_t sets = 0;
  for (int i = 0; i < N; ++i) {
    m.nade_fo[size_t(i)] = int32_t(sets);
    sets += qubit_sets(i);
  }
  auto *frag = static_cast<__bf16 *>(m.nade_frag.reserve(size_t(sets) * 1024));
  auto *vec = static_cast<float *>(m.nade_vec.reserve(size_t(N) * kVec * 4));
  const float *P = m.packed.as<float>();
  for (int i = 0; i < N; ++i) {
    auto blk = [&](int k) { return P + m.nade_off[size_t(i) * 6 + k]; };
    const int ks = (i + 15) / 16;
    const int64_t work = int64_t(qubit_sets(i)) * 512 + kVec;
    hipLaunchKernelGGL(nade_frag_kernel, dim3(unsigned(ceil_div(work, 256))), dim3(256), 0, s,
                       blk(0), blk(1), blk(2), blk(3), blk(4), blk(5), i, ks,
                       frag + int64_t(m.nade_fo[size_t(i)]) * 512, vec + int64_t(i) * kVec);
    HIP_LAUNCH_OK();
  }
}

void nade_fused_forward(nqs_model &m, const uint64_t *x, int64_t B, double *logabs,
                        double *phase, double *cond_out, int cond_p, hipStream_t s,
                        const int64_t *count) {
  NQS_REQUIRE(m.nade_fo.size() == size_t(2 * m.n), NQS_EINVAL,
              "fused forward: weights not packed");
  if (B <= 0) return;
  NadeArgs a{};
  a.frag = m.nade_frag.as<bf16x8>();
  a.vec = m.nade_vec.as<float>();
  for (int i = 0; i < 2 * m.n; ++i) a.fo[i] = m.nade_fo[size_t(i)];
  a.sec = m.sectors();
  a.x = x;
  a.B = B;
  a.count = count;
  a.N = 2 * m.n;
  a.logabs = logabs;
  a.phase = phase;
  a.cond = cond_out;
  a.cond_p = cond_p;
  NQS_REQUIRE(!cond_out || (cond_p >= 0 && cond_p < m.n), NQS_EINVAL,
              "fused forward: conditional token out of range");
  const int64_t blocks = ceil_div(B, int64_t(32) * kWaves);
  NQS_REQUIRE(blocks <= int64_t(0x7FFFFFFF), NQS_EUNSUPPORTED, "fused forward: batch too large");
  hipEvent_t e0 = cond_out ? nullptr : timing_begin(s, count);
  if (cond_out)
    hipLaunchKernelGGL(nade_cond_kernel, dim3(unsigned(blocks)), dim3(64 * kWaves), 0, s, a);
  else
    hipLaunchKernelGGL(nade_fused_kernel, dim3(unsigned(blocks)), dim3(64 * kWaves), 0, s, a);
  HIP_LAUNCH_OK();
  timing_end(e0, s, B);
}

}  // namespace nqs
