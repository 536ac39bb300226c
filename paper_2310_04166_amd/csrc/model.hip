// Amplitude networks, layer-by-layer path (FP64 and FP32 modes, all backward
// passes).  Paper: the ANQS product rule psi(x) = prod_p psi_p(x_p | x_<p);
// Mask-Unphysical conditionals ("Pruning strategies"); Appendix B for the
// per-token MLP.  The physicality of a prefix comes from Algorithm 1, filled
// bottom-up into a (position, n_alpha, n_beta) table when the model is made.
#include <algorithm>
#include <type_traits>
#include <cmath>

#include "model.h"
#include "ops.h"

using nqs::DevBuf;

namespace nqs {
namespace {

__device__ inline int tok_of(uint64_t x, int t) { return int((x >> (2 * t)) & 3ull); }

template <class T>
__device__ inline T gelu_t(T x) {
  const T c = T(0.7978845608028654);
  return T(0.5) * x * (T(1) + tanh(c * (x + T(0.044715) * x * x * x)));
}

inline dim3 g1(int64_t n, int b = 256) { return dim3(unsigned(ceil_div(n, b))); }

// ---------------------------------------------------------------- kernels ---

template <class T>
__global__ void embed_kernel(const uint64_t *x, int64_t B, int n, int d, const T *tok,
                             const T *pos, T *h) {
  const int64_t idx = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (idx >= B * n * d) return;
  const int j = int(idx % d);
  const int64_t r = idx / d;
  const int t = int(r % n);
  const int in = t == 0 ? 4 : tok_of(x[r / n], t - 1);
  h[idx] = tok[in * d + j] + pos[t * d + j];
}

// final layer norm + head (d -> 4) + bias + per-position logit bias; wave per row
template <class T>
__global__ void __launch_bounds__(256) head_kernel(const T *h, int64_t R, int n, int d, const T *g,
                                                   const T *bb, const T *W, const T *bh,
                                                   const T *lb, T *hf, T *mean, T *rstd,
                                                   T *logits) {
  const int lane = threadIdx.x % 64;
  const int64_t r = int64_t(blockIdx.x) * 4 + threadIdx.x / 64;
  if (r >= R) return;
  const T *hr = h + r * d;
  T s = 0;
  for (int j = lane; j < d; j += 64) s += hr[j];
  for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o);
  const T mu = s / T(d);
  T v = 0;
  for (int j = lane; j < d; j += 64) v += (hr[j] - mu) * (hr[j] - mu);
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  const T rs = T(1) / sqrt(v / T(d) + T(1e-5));
  T acc[4] = {0, 0, 0, 0};
  for (int j = lane; j < d; j += 64) {
    const T y = (hr[j] - mu) * rs * g[j] + bb[j];
    if (hf) hf[r * d + j] = y;
#pragma unroll
    for (int k = 0; k < 4; ++k) acc[k] += y * W[j * 4 + k];
  }
#pragma unroll
  for (int k = 0; k < 4; ++k)
    for (int o = 32; o > 0; o >>= 1) acc[k] += __shfl_xor(acc[k], o);
  if (lane == 0) {
    const int t = int(r % n);
#pragma unroll
    for (int k = 0; k < 4; ++k) logits[r * 4 + k] = acc[k] + bh[k] + lb[t * 4 + k];
    if (mean) mean[r] = mu;
    if (rstd) rstd[r] = rs;
  }
}

// log|psi| = 1/2 sum_t log softmax over allowed tokens; one thread per configuration.
// Rows hold T positions; the configuration's own molecule has n <= T tokens.
// stride selects the 4 logits of position t inside a row of `stride` values.
template <class T>
__global__ void logabs_kernel(const uint64_t *x, int64_t B, int Tn, const T *logits, int stride,
                              Sectors S, double *logabs) {
  const int64_t b = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (b >= B) return;
  const uint64_t xb = x[b];
  const nqs_sector_info si = sector_of(S, xb);
  int a = 0, c = 0;
  double s = 0.0;
  for (int t = 0; t < si.n; ++t) {
    const int tk = tok_of(xb, t);
    const int allow = t < si.mask_levels ? phys_mask(S, si, t, a, c, occupation(S, xb)) : 0xF;
    if (!((allow >> tk) & 1)) { s = -INFINITY; break; }
    const T *l = logits + (b * Tn + t) * stride;
    double mx = -INFINITY;
    for (int k = 0; k < 4; ++k)
      if ((allow >> k) & 1) mx = fmax(mx, double(l[k]));
    double z = 0.0;
    for (int k = 0; k < 4; ++k)
      if ((allow >> k) & 1) z += exp(double(l[k]) - mx);
    s += double(l[tk]) - mx - log(z);
    a += tk & 1;
    c += tk >> 1;
  }
  logabs[b] = 0.5 * s;
}

// d(sum_b g_b log|psi_b|)/d logits; zero for masked tokens and absent positions
template <class T>
__global__ void dlogits_kernel(const uint64_t *x, int64_t B, int Tn, const T *logits, int stride,
                               Sectors S, const double *gl, T *dlog, int dstride) {
  const int64_t b = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (b >= B) return;
  const uint64_t xb = x[b];
  const nqs_sector_info si = sector_of(S, xb);
  int a = 0, c = 0;
  bool ok = true;
  for (int t = 0; t < Tn; ++t) {
    T *dl = dlog + (b * Tn + t) * dstride;
    if (t >= si.n) {
      for (int k = 0; k < 4; ++k) dl[k] = T(0);
      continue;
    }
    const int tk = tok_of(xb, t);
    const int allow = t < si.mask_levels ? phys_mask(S, si, t, a, c, occupation(S, xb)) : 0xF;
    if (!((allow >> tk) & 1)) ok = false;
    const T *l = logits + (b * Tn + t) * stride;
    double mx = -INFINITY;
    for (int k = 0; k < 4; ++k)
      if ((allow >> k) & 1) mx = fmax(mx, double(l[k]));
    double z = 0.0;
    for (int k = 0; k < 4; ++k)
      if ((allow >> k) & 1) z += exp(double(l[k]) - mx);
    for (int k = 0; k < 4; ++k) {
      double v = 0.0;
      if (ok && ((allow >> k) & 1))
        v = 0.5 * gl[b] * ((k == tk ? 1.0 : 0.0) - exp(double(l[k]) - mx) / z);
      dl[k] = T(v);
    }
    a += tk & 1;
    c += tk >> 1;
  }
}

template <class T>
__global__ void cond_extract_kernel(const T *logits, int64_t B, int n, int stride, int p,
                                    double *out) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= B * 4) return;
  out[i] = double(logits[((i / 4) * n + p) * stride + (i % 4)]);
}

// phase-MLP first layer over the one-hot code of the configuration's own tokens
template <class T>
__global__ void phase_in_kernel(const uint64_t *x, int64_t B, Sectors S, int PH, const T *W1,
                                const T *b1, T *pre, T *out) {
  const int64_t idx = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (idx >= B * PH) return;
  const int j = int(idx % PH);
  const uint64_t xb = x[idx / PH];
  const int n = sector_of(S, xb).n;
  T a = b1[j];
  for (int t = 0; t < n; ++t) a += W1[(4 * t + tok_of(xb, t)) * PH + j];
  pre[idx] = a;
  out[idx] = gelu_t(a);
}

template <class T>
__global__ void __launch_bounds__(256) phase_out_kernel(const T *z, int64_t B, int PH, const T *w3,
                                                        const T *b3, double *phase) {
  const int lane = threadIdx.x % 64;
  const int64_t b = int64_t(blockIdx.x) * 4 + threadIdx.x / 64;
  if (b >= B) return;
  T a = 0;
  for (int j = lane; j < PH; j += 64) a += z[b * PH + j] * w3[j];
  for (int o = 32; o > 0; o >>= 1) a += __shfl_xor(a, o);
  if (lane == 0) phase[b] = double(a + b3[0]);
}

// MLP: phase = sum_p out[b, p, 4 + x_p]
template <class T>
__global__ void mlp_phase_kernel(const uint64_t *x, int64_t B, int n, const T *out8,
                                 double *phase) {
  const int64_t b = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (b >= B) return;
  double s = 0.0;
  for (int t = 0; t < n; ++t) s += double(out8[(b * n + t) * 8 + 4 + tok_of(x[b], t)]);
  phase[b] = s;
}

// one-hot code of tokens 0..p-1, [B, 4p]; positions beyond the configuration's
// own molecule are zero
template <class T>
__global__ void onehot_kernel(const uint64_t *x, int64_t B, int p, Sectors S, T *X) {
  const int64_t idx = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (idx >= B * 4 * p) return;
  const int col = int(idx % (4 * p));
  const uint64_t xb = x[idx / (4 * p)];
  X[idx] = (col / 4 < sector_of(S, xb).n && tok_of(xb, col / 4) == (col % 4)) ? T(1) : T(0);
}

// scatter rows [B, w] into positions of [B, n, w]
template <class T>
__global__ void scatter_pos_kernel(const T *src, int64_t B, int n, int w, int p, T *dst) {
  const int64_t idx = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (idx >= B * w) return;
  dst[((idx / w) * n + p) * w + idx % w] = src[idx];
}
template <class T>
__global__ void gather_pos_kernel(const T *src, int64_t B, int n, int w, int p, T *dst) {
  const int64_t idx = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (idx >= B * w) return;
  dst[idx] = src[((idx / w) * n + p) * w + idx % w];
}

// MLP phase gradient into the phase outputs: d out[b,p,4+x_p] = g_phase[b]
template <class T>
__global__ void mlp_dphase_kernel(const uint64_t *x, int64_t B, int n, const double *gp, T *d8) {
  const int64_t idx = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (idx >= B * n * 4) return;
  const int k = int(idx % 4);
  const int64_t r = idx / 4;
  const int t = int(r % n);
  const int64_t b = r / n;
  d8[r * 8 + 4 + k] = tok_of(x[b], t) == k ? T(gp[b]) : T(0);
}

// one-hot input class of every row (BOS = class 4 at position 0), [B*n, 5]
template <class T>
__global__ void in_class_kernel(const uint64_t *x, int64_t B, int n, T *E) {
  const int64_t idx = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (idx >= B * n * 5) return;
  const int c = int(idx % 5);
  const int64_t r = idx / 5;
  const int t = int(r % n);
  const int in = t == 0 ? 4 : tok_of(x[r / n], t - 1);
  E[idx] = in == c ? T(1) : T(0);
}

template <class T>
__global__ void phase_dz_kernel(const double *gp, int64_t B, int PH, const T *w3, T *dz, T *gpt) {
  const int64_t idx = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (idx >= B * PH) return;
  const int64_t b = idx / PH;
  dz[idx] = T(gp[b]) * w3[idx % PH];
  if (idx % PH == 0) gpt[b] = T(gp[b]);
}

// ------------------------------------------------------------- workspace ---

struct Carver {
  char *base;
  size_t used = 0;
  template <class T>
  T *take(int64_t count) {
    const size_t bytes = (size_t(count) * sizeof(T) + 255) & ~size_t(255);
    T *p = base ? reinterpret_cast<T *>(base + used) : nullptr;
    used += bytes;
    return p;
  }
};

template <class T>
struct Layer {
  T *h_in, *a1, *m1, *r1, *qkv, *probs, *o, *h_mid, *a2, *m2, *r2, *fpre, *f;
};

template <class T>
struct TfAct {
  std::vector<Layer<T>> layer;
  T *h_out, *mf, *rf, *hf, *logits, *z1pre, *z1, *z2pre, *z2;
};

template <class T>
void carve_tf(const nqs_model &m, int64_t B, bool save, Carver &c, TfAct<T> &A) {
  const int64_t R = B * m.n;
  const int d = m.d, F = m.F;
  A.layer.resize(m.L);
  for (int l = 0; l < m.L; ++l) {
    Layer<T> &y = A.layer[l];
    if (l == 0 || save) {
      y.h_in = c.take<T>(R * d);
      y.a1 = c.take<T>(R * d);
      y.m1 = c.take<T>(R);
      y.r1 = c.take<T>(R);
      y.qkv = c.take<T>(R * 3 * d);
      y.probs = save ? c.take<T>(B * m.H * m.n * m.n) : nullptr;
      y.o = c.take<T>(R * d);
      y.h_mid = save ? c.take<T>(R * d) : y.h_in;
      y.a2 = c.take<T>(R * d);
      y.m2 = c.take<T>(R);
      y.r2 = c.take<T>(R);
      y.fpre = c.take<T>(R * F);
      y.f = c.take<T>(R * F);
    } else {
      y = A.layer[0];
    }
  }
  A.h_out = save ? c.take<T>(R * d) : A.layer[0].h_in;
  A.mf = c.take<T>(R);
  A.rf = c.take<T>(R);
  A.hf = save ? c.take<T>(R * d) : nullptr;
  A.logits = c.take<T>(R * 4);
  A.z1pre = c.take<T>(B * m.PH);
  A.z1 = c.take<T>(B * m.PH);
  A.z2pre = c.take<T>(B * m.PH);
  A.z2 = c.take<T>(B * m.PH);
}

template <class T>
const T *P(const nqs_model &m, int idx) {
  return m.master.as<T>() + m.off[idx];
}

// ----------------------------------------------------------- transformer ---

// Split bf16 images of the transformer's weights for the backward of bf16
// models (mixed-precision products, mx_gemm): per layer the right operands of
// the forward products (QKV, O, W1, W2) and of the input gradients (their
// transposes), and the phase MLP's W2 both ways.
struct MxPack {
  struct Layer {
    const void *qkv, *o, *w1, *w2, *qkvT, *oT, *w1T, *w2T;
  };
  std::vector<Layer> layer;
  const void *pw2 = nullptr, *pw2T = nullptr;
};

bool mx_backward_ok(const nqs_model &m) {
  const int64_t d = m.d, F = m.F, PH = m.PH;
  return m.precision == NQS_BF16 && m.kind == NQS_MODEL_TRANSFORMER && mx_supported(3 * d, d) &&
         mx_supported(d, 3 * d) && mx_supported(d, d) && mx_supported(F, d) &&
         mx_supported(d, F) && mx_supported(PH, PH);
}

MxPack mx_pack_model(nqs_model &m, hipStream_t s) {
  const int64_t d = m.d, F = m.F, PH = m.PH;
  struct Item {
    const float *W;
    int64_t ldw;
    bool trans;
    int64_t N, K;
    const void **dst;
  };
  MxPack pk;
  pk.layer.resize(size_t(m.L));
  std::vector<Item> items;
  for (int l = 0; l < m.L; ++l) {
    auto W = [&](int k) { return P<float>(m, tf_layer(l, k)); };
    MxPack::Layer &y = pk.layer[size_t(l)];
    items.push_back({W(TF_WQKV), 3 * d, false, 3 * d, d, &y.qkv});
    items.push_back({W(TF_WO), d, false, d, d, &y.o});
    items.push_back({W(TF_W1), F, false, F, d, &y.w1});
    items.push_back({W(TF_W2), d, false, d, F, &y.w2});
    items.push_back({W(TF_WQKV), 3 * d, true, d, 3 * d, &y.qkvT});
    items.push_back({W(TF_WO), d, true, d, d, &y.oT});
    items.push_back({W(TF_W1), F, true, d, F, &y.w1T});
    items.push_back({W(TF_W2), d, true, F, d, &y.w2T});
  }
  const float *pw2 = P<float>(m, tf_tail(m.L, TF_PW2));
  items.push_back({pw2, PH, false, PH, PH, &pk.pw2});
  items.push_back({pw2, PH, true, PH, PH, &pk.pw2T});
  size_t total = 0;
  for (const Item &it : items) total += (mx_pack_bytes(it.N, it.K) + 255) & ~size_t(255);
  char *base = static_cast<char *>(m.mx_w.reserve(total));
  size_t off = 0;
  for (const Item &it : items) {
    mx_pack(it.W, it.ldw, it.trans, it.N, it.K, base + off, s);
    *it.dst = base + off;
    off += (mx_pack_bytes(it.N, it.K) + 255) & ~size_t(255);
  }
  return pk;
}

// mx_gemm for fp32 activations (the mixed path exists for them only)
template <class T>
void mxg(int64_t M, int64_t N, int64_t K, const T *A, int64_t lda, const void *Wp, T *C,
         int64_t ldc, const T *res, int64_t ldr, const T *bias, T *aux, int epi, hipStream_t s) {
  if constexpr (std::is_same<T, float>::value)
    mx_gemm(M, N, K, A, lda, Wp, C, ldc, res, ldr, bias, aux, epi, s);
  else
    NQS_REQUIRE(false, NQS_EINVAL, "mixed products take fp32 activations");
}

// mx: the weights' split images (bf16 models' backward), else library products
template <class T>
void tf_forward_chunk(nqs_model &m, const uint64_t *x, int64_t B, bool save, TfAct<T> &A,
                      double *logabs, double *phase, hipStream_t s, const MxPack *mx = nullptr) {
  const int n = m.n, d = m.d, F = m.F, H = m.H, L = m.L, PH = m.PH;
  const int64_t R = B * n;
  hipLaunchKernelGGL(embed_kernel<T>, g1(R * d), dim3(256), 0, s, x, B, n, d, P<T>(m, TF_TOK),
                     P<T>(m, TF_POS), A.layer[0].h_in);
  HIP_LAUNCH_OK();
  for (int l = 0; l < L; ++l) {
    Layer<T> &y = A.layer[l];
    auto W = [&](int k) { return P<T>(m, tf_layer(l, k)); };
    layernorm<T>(y.h_in, R, d, W(TF_LN1G), W(TF_LN1B), y.a1, y.m1, y.r1, s);
    T *h_next = (l + 1 < L) ? A.layer[l + 1].h_in : A.h_out;
    if (mx) {
      // residuals read from the previous stream position, no copies
      const MxPack::Layer &p = mx->layer[size_t(l)];
      mxg<T>(R, 3 * d, d, y.a1, d, p.qkv, y.qkv, 3 * d, nullptr, 0, W(TF_BQKV), nullptr, MX_STORE,
             s);
      attention_fwd<T>(y.qkv, B, n, d, H, y.o, y.probs, s);
      mxg<T>(R, d, d, y.o, d, p.o, y.h_mid, d, y.h_in, d, W(TF_BO), nullptr, MX_ADD, s);
      layernorm<T>(y.h_mid, R, d, W(TF_LN2G), W(TF_LN2B), y.a2, y.m2, y.r2, s);
      mxg<T>(R, F, d, y.a2, d, p.w1, y.f, F, nullptr, 0, W(TF_B1), y.fpre, MX_GELU, s);
      mxg<T>(R, d, F, y.f, F, p.w2, h_next, d, y.h_mid, d, W(TF_B2), nullptr, MX_ADD, s);
      continue;
    }
    gemm<T, false, false>(R, 3 * d, d, y.a1, d, W(TF_WQKV), 3 * d, y.qkv, 3 * d, W(TF_BQKV),
                             nullptr, EPI_STORE, s);
    attention_fwd<T>(y.qkv, B, n, d, H, y.o, y.probs, s);
    if (y.h_mid != y.h_in)
      HIP_OK(hipMemcpyAsync(y.h_mid, y.h_in, R * d * sizeof(T), hipMemcpyDeviceToDevice, s));
    gemm<T, false, false>(R, d, d, y.o, d, W(TF_WO), d, y.h_mid, d, W(TF_BO), nullptr, EPI_ADD,
                             s);
    layernorm<T>(y.h_mid, R, d, W(TF_LN2G), W(TF_LN2B), y.a2, y.m2, y.r2, s);
    gemm<T, false, false>(R, F, d, y.a2, d, W(TF_W1), F, y.f, F, W(TF_B1), y.fpre, EPI_GELU, s);
    if (h_next != y.h_mid)
      HIP_OK(hipMemcpyAsync(h_next, y.h_mid, R * d * sizeof(T), hipMemcpyDeviceToDevice, s));
    gemm<T, false, false>(R, d, F, y.f, F, W(TF_W2), d, h_next, d, W(TF_B2), nullptr, EPI_ADD,
                             s);
  }
  hipLaunchKernelGGL(head_kernel<T>, g1(R, 4), dim3(256), 0, s, A.h_out, R, n, d,
                     P<T>(m, tf_tail(L, TF_LNFG)), P<T>(m, tf_tail(L, TF_LNFB)),
                     P<T>(m, tf_tail(L, TF_WHEAD)), P<T>(m, tf_tail(L, TF_BHEAD)),
                     P<T>(m, tf_tail(L, TF_LBIAS)), A.hf, A.mf, A.rf, A.logits);
  HIP_LAUNCH_OK();
  if (logabs) {
    hipLaunchKernelGGL(logabs_kernel<T>, g1(B), dim3(256), 0, s, x, B, n, A.logits, 4,
                       m.sectors(), logabs);
    HIP_LAUNCH_OK();
  }
  if (phase || save) {
    hipLaunchKernelGGL(phase_in_kernel<T>, g1(B * PH), dim3(256), 0, s, x, B, m.sectors(), PH,
                       P<T>(m, tf_tail(L, TF_PW1)), P<T>(m, tf_tail(L, TF_PB1)), A.z1pre, A.z1);
    HIP_LAUNCH_OK();
    if (mx)
      mxg<T>(B, PH, PH, A.z1, PH, mx->pw2, A.z2, PH, nullptr, 0, P<T>(m, tf_tail(L, TF_PB2)),
             A.z2pre, MX_GELU, s);
    else
      gemm<T, false, false>(B, PH, PH, A.z1, PH, P<T>(m, tf_tail(L, TF_PW2)), PH, A.z2, PH,
                               P<T>(m, tf_tail(L, TF_PB2)), A.z2pre, EPI_GELU, s);
    if (phase) {
      hipLaunchKernelGGL(phase_out_kernel<T>, g1(B, 4), dim3(256), 0, s, A.z2, B, PH,
                         P<T>(m, tf_tail(L, TF_PW3)), P<T>(m, tf_tail(L, TF_PB3)), phase);
      HIP_LAUNCH_OK();
    }
  }
}

// dW += X^T dY reduced over the R rows, accumulated in double at the parameter's offset
// (mixed: split bf16 operands).
template <class T>
void wgrad(nqs_model &m, int64_t Mi, int64_t No, int64_t R, const T *X, int64_t ldx, const T *dY,
           int64_t ldy, int pidx, hipStream_t s, bool mixed = false) {
  void *part = m.part.reserve(wgrad_scratch_bytes(R, Mi, No, std::max(ldx, ldy), sizeof(T)));
  if constexpr (std::is_same<T, float>::value)
    wgrad_acc(X, ldx, dY, ldy, R, Mi, No, m.grad_acc.as<double>() + m.off[pidx], part, s, mixed);
  else
    wgrad_acc(X, ldx, dY, ldy, R, Mi, No, m.grad_acc.as<double>() + m.off[pidx], part, s);
}

// db += column sums of dY (fixed-order, double)
template <class T>
void bgrad(nqs_model &m, const T *dY, int64_t R, int64_t N, int64_t ld, int pidx, hipStream_t s) {
  double *part = static_cast<double *>(m.part.reserve(colsum_scratch_bytes(R, N)));
  colsum_acc<T>(dY, R, N, ld, m.grad_acc.as<double>() + m.off[pidx], part, s);
}

// layer-norm backward into dx with its gain and bias gradients (one kernel
// where the width allows; else the row kernel, dy * xhat into tmp and two
// column sums)
template <class T>
void lnbgrad(nqs_model &m, const T *x, const T *mean, const T *rstd, int64_t R, int d, const T *g,
             const T *dy, T *dx, bool accumulate, T *tmp, int gidx, int bidx, hipStream_t s) {
  if (layernorm_bwd_acc_supported(d)) {
    double *scratch = static_cast<double *>(m.part.reserve(layernorm_bwd_acc_scratch_bytes(d)));
    double *acc = m.grad_acc.as<double>();
    layernorm_bwd_acc<T>(x, mean, rstd, R, d, g, dy, dx, accumulate, acc + m.off[gidx],
                         acc + m.off[bidx], scratch, s);
    return;
  }
  layernorm_bwd<T>(x, mean, rstd, R, d, g, dy, dx, accumulate, tmp, s);
  bgrad<T>(m, tmp, R, d, d, gidx, s);
  bgrad<T>(m, dy, R, d, d, bidx, s);
}

// a linear layer's dW += X^T dY and db += column sums of dY (mixed: in one kernel)
template <class T>
void wbgrad(nqs_model &m, int64_t Mi, int64_t No, int64_t R, const T *X, int64_t ldx, const T *dY,
            int64_t ldy, int widx, int bidx, hipStream_t s, bool mixed) {
  if constexpr (std::is_same<T, float>::value) {
    if (mixed) {
      void *part = m.part.reserve(wgrad_scratch_bytes(R, Mi, No, std::max(ldx, ldy), sizeof(T)));
      double *acc = m.grad_acc.as<double>();
      wgrad_acc(X, ldx, dY, ldy, R, Mi, No, acc + m.off[widx], part, s, true, acc + m.off[bidx]);
      return;
    }
  }
  wgrad<T>(m, Mi, No, R, X, ldx, dY, ldy, widx, s, mixed);
  bgrad<T>(m, dY, R, No, ldy, bidx, s);
}

// mx: the weights' split images (bf16 models), else library products
template <class T>
void tf_backward_chunk(nqs_model &m, const uint64_t *x, int64_t B, const double *gl,
                       const double *gp, hipStream_t s, const MxPack *mx = nullptr) {
  const int n = m.n, d = m.d, F = m.F, H = m.H, L = m.L, PH = m.PH;
  const int64_t R = B * n;
  Carver c0{nullptr};
  TfAct<T> A;
  carve_tf<T>(m, B, true, c0, A);
  // backward temporaries
  const size_t act_bytes = c0.used;
  auto carve_bwd = [&](Carver &c, T *&dh, T *&dl, T *&da, T *&df, T *&dq, T *&tmp, T *&dz,
                       T *&gpt) {
    dh = c.take<T>(R * d);
    dl = c.take<T>(R * 4);
    da = c.take<T>(R * d);
    df = c.take<T>(R * F);
    dq = c.take<T>(R * 3 * d);
    tmp = c.take<T>(R * d);
    dz = c.take<T>(B * PH * 2);
    gpt = c.take<T>(B);
  };
  T *dh, *dl, *da, *df, *dq, *tmp, *dz, *gpt;
  Carver c1{nullptr};
  c1.used = act_bytes;
  carve_bwd(c1, dh, dl, da, df, dq, tmp, dz, gpt);
  char *base = static_cast<char *>(m.ws.reserve(c1.used));
  Carver c2{base};
  carve_tf<T>(m, B, true, c2, A);
  carve_bwd(c2, dh, dl, da, df, dq, tmp, dz, gpt);

  tf_forward_chunk<T>(m, x, B, true, A, nullptr, nullptr, s, mx);
  const bool mixed = mx != nullptr;

  // head and masked log-softmax
  hipLaunchKernelGGL(dlogits_kernel<T>, g1(B), dim3(256), 0, s, x, B, n, A.logits, 4,
                     m.sectors(), gl, dl, 4);
  HIP_LAUNCH_OK();
  wbgrad<T>(m, d, 4, R, A.hf, d, dl, 4, tf_tail(L, TF_WHEAD), tf_tail(L, TF_BHEAD), s, mixed);
  bgrad<T>(m, dl, B, int64_t(n) * 4, int64_t(n) * 4, tf_tail(L, TF_LBIAS), s);
  gemm<T, false, true>(R, d, 4, dl, 4, P<T>(m, tf_tail(L, TF_WHEAD)), 4, da, d, nullptr,
                          nullptr, EPI_STORE, s);
  lnbgrad<T>(m, A.h_out, A.mf, A.rf, R, d, P<T>(m, tf_tail(L, TF_LNFG)), da, dh, false, tmp,
             tf_tail(L, TF_LNFG), tf_tail(L, TF_LNFB), s);

  for (int l = L - 1; l >= 0; --l) {
    Layer<T> &y = A.layer[l];
    auto W = [&](int k) { return P<T>(m, tf_layer(l, k)); };
    const MxPack::Layer *p = mixed ? &mx->layer[size_t(l)] : nullptr;
    // h_out = h_mid + gelu(a2 W1 + b1) W2 + b2
    wbgrad<T>(m, F, d, R, y.f, F, dh, d, tf_layer(l, TF_W2), tf_layer(l, TF_B2), s, mixed);
    if (p) {
      mxg<T>(R, F, d, dh, d, p->w2T, df, F, nullptr, 0, nullptr, y.fpre, MX_DGELU, s);
    } else {
      gemm<T, false, true>(R, F, d, dh, d, W(TF_W2), d, df, F, nullptr, nullptr, EPI_STORE, s);
      gelu_bwd<T>(y.fpre, df, R * F, s);
    }
    wbgrad<T>(m, d, F, R, y.a2, d, df, F, tf_layer(l, TF_W1), tf_layer(l, TF_B1), s, mixed);
    if (p) mxg<T>(R, d, F, df, F, p->w1T, da, d, nullptr, 0, nullptr, nullptr, MX_STORE, s);
    else gemm<T, false, true>(R, d, F, df, F, W(TF_W1), F, da, d, nullptr, nullptr, EPI_STORE, s);
    lnbgrad<T>(m, y.h_mid, y.m2, y.r2, R, d, W(TF_LN2G), da, dh, true, tmp, tf_layer(l, TF_LN2G),
               tf_layer(l, TF_LN2B), s);
    // h_mid = h_in + attn(a1) Wo + bo
    wbgrad<T>(m, d, d, R, y.o, d, dh, d, tf_layer(l, TF_WO), tf_layer(l, TF_BO), s, mixed);
    if (p) mxg<T>(R, d, d, dh, d, p->oT, da, d, nullptr, 0, nullptr, nullptr, MX_STORE, s);
    else gemm<T, false, true>(R, d, d, dh, d, W(TF_WO), d, da, d, nullptr, nullptr, EPI_STORE, s);
    attention_bwd<T>(y.qkv, y.probs, da, B, n, d, H, dq, s);
    wbgrad<T>(m, d, 3 * d, R, y.a1, d, dq, 3 * d, tf_layer(l, TF_WQKV), tf_layer(l, TF_BQKV), s,
              mixed);
    if (p)
      mxg<T>(R, d, 3 * d, dq, 3 * d, p->qkvT, da, d, nullptr, 0, nullptr, nullptr, MX_STORE, s);
    else
      gemm<T, false, true>(R, d, 3 * d, dq, 3 * d, W(TF_WQKV), 3 * d, da, d, nullptr, nullptr,
                              EPI_STORE, s);
    lnbgrad<T>(m, y.h_in, y.m1, y.r1, R, d, W(TF_LN1G), da, dh, true, tmp, tf_layer(l, TF_LN1G),
               tf_layer(l, TF_LN1B), s);
  }
  // embeddings: token table through the one-hot input classes, positions by column sums
  hipLaunchKernelGGL(in_class_kernel<T>, g1(R * 5), dim3(256), 0, s, x, B, n, tmp);
  HIP_LAUNCH_OK();
  wgrad<T>(m, 5, d, R, tmp, 5, dh, d, TF_TOK, s, mixed);
  bgrad<T>(m, dh, B, int64_t(n) * d, int64_t(n) * d, TF_POS, s);

  // phase MLP: phi = gelu(gelu(onehot W1 + b1) W2 + b2) w3 + b3
  T *dz2 = dz, *dz1 = dz + B * PH;
  hipLaunchKernelGGL(phase_dz_kernel<T>, g1(B * PH), dim3(256), 0, s, gp, B, PH,
                     P<T>(m, tf_tail(L, TF_PW3)), dz2, gpt);
  HIP_LAUNCH_OK();
  wgrad<T>(m, PH, 1, B, A.z2, PH, gpt, 1, tf_tail(L, TF_PW3), s, mixed);
  bgrad<T>(m, gpt, B, 1, 1, tf_tail(L, TF_PB3), s);
  gelu_bwd<T>(A.z2pre, dz2, B * PH, s);
  wbgrad<T>(m, PH, PH, B, A.z1, PH, dz2, PH, tf_tail(L, TF_PW2), tf_tail(L, TF_PB2), s, mixed);
  if (mixed) {
    mxg<T>(B, PH, PH, dz2, PH, mx->pw2T, dz1, PH, nullptr, 0, nullptr, A.z1pre, MX_DGELU, s);
  } else {
    gemm<T, false, true>(B, PH, PH, dz2, PH, P<T>(m, tf_tail(L, TF_PW2)), PH, dz1, PH, nullptr,
                            nullptr, EPI_STORE, s);
    gelu_bwd<T>(A.z1pre, dz1, B * PH, s);
  }
  bgrad<T>(m, dz1, B, PH, PH, tf_tail(L, TF_PB1), s);
  hipLaunchKernelGGL(onehot_kernel<T>, g1(B * 4 * n), dim3(256), 0, s, x, B, n, m.sectors(), tmp);
  HIP_LAUNCH_OK();
  wgrad<T>(m, 4 * n, PH, B, tmp, 4 * n, dz1, PH, tf_tail(L, TF_PW1), s, mixed);
}

// ------------------------------------------------------------------- MLP ---

struct MlpAct {
  void *X, *h1, *pre2, *h2, *out8, *o;
};

template <class T>
void mlp_position(nqs_model &m, const uint64_t *x, int64_t B, int p, T *X, T *h1, T *pre2, T *h2,
                  T *o, hipStream_t s) {
  const int hid = m.hid;
  if (p > 0) {
    hipLaunchKernelGGL(onehot_kernel<T>, g1(B * 4 * p), dim3(256), 0, s, x, B, p, m.sectors(), X);
    HIP_LAUNCH_OK();
  }
  auto W = [&](int k) { return P<T>(m, 6 * p + k); };
  // p == 0: no input, h1 = tanh(b1)
  gemm<T, false, false>(B, hid, 4 * p, X, 4 * p > 0 ? 4 * p : 1, W(MLP_W1), hid, h1, hid,
                           W(MLP_B1), nullptr, EPI_TANH, s);
  gemm<T, false, false>(B, hid, hid, h1, hid, W(MLP_W2), hid, h2, hid, W(MLP_B2), pre2,
                           EPI_LRELU, s);
  gemm<T, false, false>(B, 8, hid, h2, hid, W(MLP_W3), 8, o, 8, W(MLP_B3), nullptr, EPI_STORE,
                           s);
}

template <class T>
size_t mlp_carve(const nqs_model &m, int64_t B, Carver &c, T *&X, T *&h1, T *&pre2, T *&h2,
                 T *&o, T *&out8) {
  X = c.take<T>(B * 4 * m.n);
  h1 = c.take<T>(B * m.hid);
  pre2 = c.take<T>(B * m.hid);
  h2 = c.take<T>(B * m.hid);
  o = c.take<T>(B * 8);
  out8 = c.take<T>(B * m.n * 8);
  return c.used;
}

template <class T>
void mlp_forward_chunk(nqs_model &m, const uint64_t *x, int64_t B, double *logabs, double *phase,
                       T *out8_keep, hipStream_t s) {
  T *X, *h1, *pre2, *h2, *o, *out8;
  Carver c0{nullptr};
  mlp_carve<T>(m, B, c0, X, h1, pre2, h2, o, out8);
  Carver c{static_cast<char *>(m.ws.reserve(c0.used))};
  mlp_carve<T>(m, B, c, X, h1, pre2, h2, o, out8);
  if (out8_keep) out8 = out8_keep;
  for (int p = 0; p < m.n; ++p) {
    mlp_position<T>(m, x, B, p, X, h1, pre2, h2, o, s);
    hipLaunchKernelGGL(scatter_pos_kernel<T>, g1(B * 8), dim3(256), 0, s, o, B, m.n, 8, p, out8);
    HIP_LAUNCH_OK();
  }
  if (logabs) {
    hipLaunchKernelGGL(logabs_kernel<T>, g1(B), dim3(256), 0, s, x, B, m.n, out8, 8,
                       m.sectors(), logabs);
    HIP_LAUNCH_OK();
  }
  if (phase) {
    hipLaunchKernelGGL(mlp_phase_kernel<T>, g1(B), dim3(256), 0, s, x, B, m.n, out8, phase);
    HIP_LAUNCH_OK();
  }
}

template <class T>
void mlp_backward_chunk(nqs_model &m, const uint64_t *x, int64_t B, const double *gl,
                        const double *gp, hipStream_t s) {
  const int n = m.n, hid = m.hid;
  T *X, *h1, *pre2, *h2, *o, *out8;
  Carver c0{nullptr};
  mlp_carve<T>(m, B, c0, X, h1, pre2, h2, o, out8);
  T *d8 = c0.take<T>(B * n * 8);
  T *dp = c0.take<T>(B * 8);
  T *dh2 = c0.take<T>(B * hid);
  T *dh1 = c0.take<T>(B * hid);
  Carver c{static_cast<char *>(m.ws.reserve(c0.used))};
  mlp_carve<T>(m, B, c, X, h1, pre2, h2, o, out8);
  d8 = c.take<T>(B * n * 8);
  dp = c.take<T>(B * 8);
  dh2 = c.take<T>(B * hid);
  dh1 = c.take<T>(B * hid);
  for (int p = 0; p < n; ++p) {
    mlp_position<T>(m, x, B, p, X, h1, pre2, h2, o, s);
    hipLaunchKernelGGL(scatter_pos_kernel<T>, g1(B * 8), dim3(256), 0, s, o, B, n, 8, p, out8);
    HIP_LAUNCH_OK();
  }
  hipLaunchKernelGGL(dlogits_kernel<T>, g1(B), dim3(256), 0, s, x, B, n, out8, 8, m.sectors(),
                     gl, d8, 8);
  HIP_LAUNCH_OK();
  hipLaunchKernelGGL(mlp_dphase_kernel<T>, g1(B * n * 4), dim3(256), 0, s, x, B, n, gp, d8);
  HIP_LAUNCH_OK();
  for (int p = 0; p < n; ++p) {
    mlp_position<T>(m, x, B, p, X, h1, pre2, h2, o, s);
    hipLaunchKernelGGL(gather_pos_kernel<T>, g1(B * 8), dim3(256), 0, s, d8, B, n, 8, p, dp);
    HIP_LAUNCH_OK();
    auto W = [&](int k) { return P<T>(m, 6 * p + k); };
    wgrad<T>(m, hid, 8, B, h2, hid, dp, 8, 6 * p + MLP_W3, s);
    bgrad<T>(m, dp, B, 8, 8, 6 * p + MLP_B3, s);
    gemm<T, false, true>(B, hid, 8, dp, 8, W(MLP_W3), 8, dh2, hid, nullptr, nullptr, EPI_STORE,
                            s);
    lrelu_bwd<T>(pre2, dh2, B * hid, s);
    wgrad<T>(m, hid, hid, B, h1, hid, dh2, hid, 6 * p + MLP_W2, s);
    bgrad<T>(m, dh2, B, hid, hid, 6 * p + MLP_B2, s);
    gemm<T, false, true>(B, hid, hid, dh2, hid, W(MLP_W2), hid, dh1, hid, nullptr, nullptr,
                            EPI_STORE, s);
    tanh_bwd<T>(h1, dh1, B * hid, s);
    if (p > 0) wgrad<T>(m, 4 * p, hid, B, X, 4 * p, dh1, hid, 6 * p + MLP_W1, s);
    bgrad<T>(m, dh1, B, hid, hid, 6 * p + MLP_B1, s);
  }
}

// ------------------------------------------------------------------ NADE ---
// The paper's per-qubit ansatz with complex weights (Appendix "ANQS
// architecture"): qubit i has an MLP reading the i previous bits, h1 =
// tanh(x W1 + b1) (complex tanh), h2 = LeReLU(Re) + i LeReLU(Im) of h1 W2 + b2,
// z = h2 W3 + b3 (two complex outputs), log psi_i(v) = z_v - 1/2 LSE(2 Re z).
// A complex layer is one real GEMM: [Re h, Im h] times the block matrix
// [[Re W, Im W], [-Im W, Re W]] gives [Re(hW), Im(hW)]; the blocks are built
// from the canonical parameters (nade_pack).  Token p of the four-way sampler
// is qubits 2p (alpha) and 2p + 1 (beta): its outputs are the token
// log-probabilities 2 Re log psi_2p(a) + 2 Re log psi_2p+1(b | a) and phases
// Im log psi_2p(a) + Im log psi_2p+1(b | a), so the MLP model's log-softmax,
// phase and gradient kernels apply to them unchanged.  Mask-Unphysical per
// qubit: with one physical value v, psi_i(v) = 1 and psi_i(1 - v) = 0.

// derived blocks of qubit i, in order: W1cat (i x 2H), b1cat (2H), W2blk
// (2H x 2H), b2cat (2H), W3blk (2H x 4, columns Re z0, Re z1, Im z0, Im z1), b3cat (4)
constexpr int kNadeBlocks = 6;

// W1 has Q rows (the qubit count): rows in .. Q-1 are zero, so that every
// qubit's block has the same shape (the batched products read all Q rows, the
// per-qubit ones the first `in`)
template <class T>
__global__ void nade_pack_kernel(const T *w1r, const T *w1i, const T *b1r, const T *b1i,
                                 const T *w2r, const T *w2i, const T *b2r, const T *b2i,
                                 const T *w3r, const T *w3i, const T *b3r, const T *b3i, int in,
                                 int Q, int H, T *W1, T *B1, T *W2, T *B2, T *W3, T *B3) {
  const int64_t idx = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  const int64_t H2 = 2 * H;
  const int64_t n1 = int64_t(Q) * H2, n2 = H2 * H2, n3 = H2 * 4;
  if (idx < n1) {
    const int64_t j = idx / H2, c = idx % H2;
    W1[idx] = j >= in ? T(0) : c < H ? w1r[j * H + c] : w1i[j * H + c - H];
  } else if (idx < n1 + H2) {
    const int64_t c = idx - n1;
    B1[c] = c < H ? b1r[c] : b1i[c - H];
  } else if (idx < n1 + H2 + n2) {
    const int64_t e = idx - n1 - H2, r = e / H2, c = e % H2;
    const int64_t rr = r % H, cc = c % H;
    W2[e] = (r < H) == (c < H) ? w2r[rr * H + cc] : (r < H ? w2i[rr * H + cc] : -w2i[rr * H + cc]);
  } else if (idx < n1 + 2 * H2 + n2) {
    const int64_t c = idx - n1 - H2 - n2;
    B2[c] = c < H ? b2r[c] : b2i[c - H];
  } else if (idx < n1 + 2 * H2 + n2 + n3) {
    const int64_t e = idx - n1 - 2 * H2 - n2, r = e / 4, c = e % 4;
    const int64_t rr = r % H, v = c % 2;
    W3[e] = (r < H) == (c < 2) ? w3r[rr * 2 + v] : (r < H ? w3i[rr * 2 + v] : -w3i[rr * 2 + v]);
  } else if (idx < n1 + 2 * H2 + n2 + n3 + 4) {
    const int64_t c = idx - n1 - 2 * H2 - n2 - n3;
    B3[c] = c < 2 ? b3r[c] : b3i[c - 2];
  }
}

// X[b][c] = bit c of x for c < 2p, X[b][2p] = a (row stride 2p + 1)
template <class T>
__global__ void nade_bits_kernel(const uint64_t *x, int64_t B, int p, int a, T *X) {
  const int w = 2 * p + 1;
  const int64_t idx = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (idx >= B * w) return;
  const int c = int(idx % w);
  X[idx] = c < 2 * p ? T((x[idx / w] >> c) & 1ull) : T(a);
}

// complex tanh in place on rows [Re(H) | Im(H)]: with r = e^{-2|a|},
// tanh(a + ib) = (sgn(a)(1 - r^2) + 2i r sin 2b) / (1 + 2r cos 2b + r^2)
template <class T>
__global__ void nade_ctanh_kernel(T *h, int64_t B, int H) {
  const int64_t idx = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (idx >= B * H) return;
  T *row = h + (idx / H) * 2 * H;
  const int64_t j = idx % H;
  const T a = row[j], b = row[H + j];
  const T r = exp(T(-2) * fabs(a));
  const T den = T(1) + T(2) * r * cos(T(2) * b) + r * r;
  row[j] = (a >= T(0) ? T(1) : T(-1)) * (T(1) - r * r) / den;
  row[H + j] = T(2) * r * sin(T(2) * b) / den;
}

// d(tanh z): with s = 1 - h^2 (complex), dz = (Re s gr + Im s gi) + i (-Im s gr + Re s gi)
template <class T>
__global__ void nade_ctanh_bwd_kernel(const T *h, T *g, int64_t B, int H) {
  const int64_t idx = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (idx >= B * H) return;
  const int64_t base = (idx / H) * 2 * H, j = idx % H;
  const T hr = h[base + j], hi = h[base + H + j];
  const T sr = T(1) - hr * hr + hi * hi, si = T(-2) * hr * hi;
  const T gr = g[base + j], gi = g[base + H + j];
  g[base + j] = sr * gr + si * gi;
  g[base + H + j] = -si * gr + sr * gi;
}

// masked log-modulus and phase of one qubit's two values from its outputs
// z = (Re z0, Re z1, Im z0, Im z1)
template <class T>
__device__ inline void nade_qubit(const T *z, bool masked, bool ok0, bool ok1, double (&la)[2],
                                  double (&ph)[2]) {
  if (!masked || (ok0 && ok1)) {
    const double r0 = 2.0 * double(z[0]), r1 = 2.0 * double(z[1]);
    const double mx = fmax(r0, r1);
    const double lse = mx + log(exp(r0 - mx) + exp(r1 - mx));
    la[0] = double(z[0]) - 0.5 * lse;
    la[1] = double(z[1]) - 0.5 * lse;
    ph[0] = double(z[2]);
    ph[1] = double(z[3]);
  } else {
    la[0] = ok0 ? 0.0 : -INFINITY;
    la[1] = ok1 ? 0.0 : -INFINITY;
    ph[0] = ph[1] = 0.0;
  }
}

// the physical tokens of token p and whether the level is masked
__device__ inline int nade_phys(uint64_t xb, int p, Sectors S, bool &masked) {
  const nqs_sector_info &si = sector_of(S, xb);
  const uint64_t occ = occupation(S, xb);
  const uint64_t below = (p == 0) ? 0ull : (~0ull >> (64 - 2 * p));
  const int na = __popcll(occ & below & 0x5555555555555555ull);
  const int nb = __popcll(occ & below & 0xAAAAAAAAAAAAAAAAull);
  masked = p < si.mask_levels;
  return masked ? phys_mask(S, si, p, na, nb, occ) : 0xF;
}

// token outputs of position p: out8[b, p, k] = 2 (la_a(a) + la_b(b | a)),
// out8[b, p, 4 + k] = ph_a(a) + ph_b(b | a), k = a + 2b
template <class T>
__global__ void nade_combine_kernel(const uint64_t *x, int64_t B, int n, int p, const T *za,
                                    const T *zb0, const T *zb1, Sectors S, T *out8) {
  const int64_t b = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (b >= B) return;
  bool masked;
  const int phys = nade_phys(x[b], p, S, masked);
  double laA[2], phA[2], laB[2][2], phB[2][2];
  nade_qubit(za + 4 * b, masked, (phys & 5) != 0, (phys & 10) != 0, laA, phA);
  for (int a = 0; a < 2; ++a)
    nade_qubit((a ? zb1 : zb0) + 4 * b, masked, ((phys >> a) & 1) != 0,
               ((phys >> (a + 2)) & 1) != 0, laB[a], phB[a]);
  T *o = out8 + (b * n + p) * 8;
  for (int k = 0; k < 4; ++k) {
    const int a = k & 1, c = k >> 1;
    o[k] = T(2.0 * (laA[a] + laB[a][c]));
    o[4 + k] = T(phA[a] + phB[a][c]);
  }
}

template <class T>
const T *nade_blk(const nqs_model &m, int i, int k) {
  return m.packed.as<T>() + m.nade_off[size_t(i) * kNadeBlocks + k];
}

template <class T>
struct NadeEval {
  T *h1, *pre2, *h2, *z;
};

// qubit i's network on B rows of X (row stride ldx, i inputs)
template <class T>
void nade_subnet(nqs_model &m, int i, int64_t B, const T *X, int ldx, const NadeEval<T> &E,
                 hipStream_t s) {
  const int H2 = 2 * m.hid;
  gemm<T, false, false>(B, H2, i, X, ldx > 0 ? ldx : 1, nade_blk<T>(m, i, 0), H2, E.h1, H2,
                        nade_blk<T>(m, i, 1), nullptr, EPI_STORE, s);
  hipLaunchKernelGGL(nade_ctanh_kernel<T>, g1(B * m.hid), dim3(256), 0, s, E.h1, B, m.hid);
  HIP_LAUNCH_OK();
  gemm<T, false, false>(B, H2, H2, E.h1, H2, nade_blk<T>(m, i, 2), H2, E.h2, H2,
                        nade_blk<T>(m, i, 3), E.pre2, EPI_LRELU, s);
  gemm<T, false, false>(B, 4, H2, E.h2, H2, nade_blk<T>(m, i, 4), 4, E.z, 4,
                        nade_blk<T>(m, i, 5), nullptr, EPI_STORE, s);
}

template <class T>
struct NadeAct {
  T *X0, *X1, *out8;
  NadeEval<T> e[3];     // alpha, beta | a = 0, beta | a = 1
};

template <class T>
size_t nade_carve(const nqs_model &m, int64_t B, Carver &c, NadeAct<T> &A) {
  const int64_t w = 2 * m.n + 1, H2 = 2 * m.hid;
  A.X0 = c.take<T>(B * w);
  A.X1 = c.take<T>(B * w);
  A.out8 = c.take<T>(B * m.n * 8);
  for (auto &e : A.e) {
    e.h1 = c.take<T>(B * H2);
    e.pre2 = c.take<T>(B * H2);
    e.h2 = c.take<T>(B * H2);
    e.z = c.take<T>(B * 4);
  }
  return c.used;
}

// the three evaluations of token p (alpha qubit; beta qubit after a = 0 and a = 1)
template <class T>
void nade_token(nqs_model &m, const uint64_t *x, int64_t B, int p, NadeAct<T> &A, hipStream_t s) {
  const int w = 2 * p + 1;
  hipLaunchKernelGGL(nade_bits_kernel<T>, g1(B * w), dim3(256), 0, s, x, B, p, 0, A.X0);
  HIP_LAUNCH_OK();
  hipLaunchKernelGGL(nade_bits_kernel<T>, g1(B * w), dim3(256), 0, s, x, B, p, 1, A.X1);
  HIP_LAUNCH_OK();
  nade_subnet<T>(m, 2 * p, B, A.X0, w, A.e[0], s);
  nade_subnet<T>(m, 2 * p + 1, B, A.X0, w, A.e[1], s);
  nade_subnet<T>(m, 2 * p + 1, B, A.X1, w, A.e[2], s);
}

template <class T>
void nade_forward_chunk(nqs_model &m, const uint64_t *x, int64_t B, double *logabs, double *phase,
                        T *out8_keep, hipStream_t s) {
  NadeAct<T> A;
  Carver c0{nullptr};
  nade_carve<T>(m, B, c0, A);
  Carver c{static_cast<char *>(m.ws.reserve(c0.used))};
  nade_carve<T>(m, B, c, A);
  if (out8_keep) A.out8 = out8_keep;
  for (int p = 0; p < m.n; ++p) {
    nade_token<T>(m, x, B, p, A, s);
    hipLaunchKernelGGL(nade_combine_kernel<T>, g1(B), dim3(256), 0, s, x, B, m.n, p, A.e[0].z,
                       A.e[1].z, A.e[2].z, m.sectors(), A.out8);
    HIP_LAUNCH_OK();
  }
  if (logabs) {
    hipLaunchKernelGGL(logabs_kernel<T>, g1(B), dim3(256), 0, s, x, B, m.n, A.out8, 8,
                       m.sectors(), logabs);
    HIP_LAUNCH_OK();
  }
  if (phase) {
    hipLaunchKernelGGL(mlp_phase_kernel<T>, g1(B), dim3(256), 0, s, x, B, m.n, A.out8, phase);
    HIP_LAUNCH_OK();
  }
}

// ---- the per-qubit ansatz with all qubits batched (amp_forward, local energy
// and the backward in FP64 / FP32).  Given x every qubit's network reads known
// bits, so the Q = 2n networks are independent: each layer is one strided batch
// of Q products (W1 padded to Q rows), activations are qubit-major [Q][B][.].

// X[b][c] = bit c of the configuration (c < Q)
template <class T>
__global__ void nade_qb_bits_kernel(const uint64_t *x, int64_t B, int Q, Sectors S, T *X) {
  const int64_t idx = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (idx >= B * Q) return;
  X[idx] = T((occupation(S, x[idx / Q]) >> (idx % Q)) & 1ull);
}

// rows [Re(H) | Im(H)] of qubit q (rows of B per qubit): add b1[q], complex tanh
template <class T>
__global__ void nade_qb_bias_ctanh_kernel(T *h, const T *b1, int64_t B, int Q, int H) {
  const int64_t idx = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (idx >= int64_t(Q) * B * H) return;
  const int64_t row = idx / H, j = idx % H, q = row / B;
  T *r = h + row * 2 * H;
  const T *bq = b1 + q * 2 * H;
  const T a = r[j] + bq[j], b = r[H + j] + bq[H + j];
  const T e = exp(T(-2) * fabs(a));
  const T den = T(1) + T(2) * e * cos(T(2) * b) + e * e;
  r[j] = (a >= T(0) ? T(1) : T(-1)) * (T(1) - e * e) / den;
  r[H + j] = T(2) * e * sin(T(2) * b) / den;
}

// pre = P + b2[q] (kept in P), Y = leaky ReLU(pre), slope 0.01
template <class T>
__global__ void nade_qb_bias_lrelu_kernel(T *P, const T *b2, int64_t B, int Q, int H2, T *Y) {
  const int64_t idx = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (idx >= int64_t(Q) * B * H2) return;
  const int64_t q = idx / (B * H2), c = idx % H2;
  const T v = P[idx] + b2[q * H2 + c];
  P[idx] = v;
  Y[idx] = v >= T(0) ? v : T(0.01) * v;
}

// Walk the qubits of configuration b with their outputs z = Z[q][b] + b3[q]:
// Mask-Unphysical per qubit, log|psi| and phase; with gl / gp, the gradient of
// gl log|psi| + gp phase with respect to every qubit's z instead (DZ[q][b]).
template <class T>
__global__ void nade_qb_combine_kernel(const uint64_t *x, int64_t B, int Q, Sectors S, const T *Z,
                                       const T *b3, double *logabs, double *phase,
                                       const double *gl, const double *gp, T *DZ) {
  const int64_t b = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (b >= B) return;
  const nqs_sector_info &si = sector_of(S, x[b]);
  const uint64_t occ = occupation(S, x[b]);
  double la = 0.0, ph = 0.0;
  int na = 0, nb = 0, phys = 0xF;
  for (int q = 0; q < Q; ++q) {
    const int p = q >> 1, v = int((occ >> q) & 1);
    const bool masked = p < si.mask_levels;
    if ((q & 1) == 0 && masked) phys = phys_mask(S, si, p, na, nb, occ);
    bool ok0, ok1;
    if ((q & 1) == 0) {
      ok0 = (phys & 5) != 0;
      ok1 = (phys & 10) != 0;
    } else {
      const int al = int((occ >> (q - 1)) & 1);
      ok0 = ((phys >> al) & 1) != 0;
      ok1 = ((phys >> (al + 2)) & 1) != 0;
    }
    const T *zq = Z + (int64_t(q) * B + b) * 4;
    double z[4];
    for (int k = 0; k < 4; ++k) z[k] = double(zq[k]) + double(b3[q * 4 + k]);
    const bool free = !masked || (ok0 && ok1);
    double dz[4] = {0.0, 0.0, 0.0, 0.0};
    if (free) {
      const double r0 = 2.0 * z[0], r1 = 2.0 * z[1], mx = fmax(r0, r1);
      const double e0 = exp(r0 - mx), e1 = exp(r1 - mx);
      la += z[v] - 0.5 * (mx + log(e0 + e1));
      ph += z[2 + v];
      if (DZ) {
        // d(z_v - LSE(2 Re z) / 2) / d Re z_w = [w == v] - softmax(2 Re z)_w
        const double w0 = e0 / (e0 + e1), w1 = e1 / (e0 + e1);
        dz[0] = gl[b] * ((v == 0 ? 1.0 : 0.0) - w0);
        dz[1] = gl[b] * ((v == 1 ? 1.0 : 0.0) - w1);
        dz[2 + v] = gp[b];
      }
    } else if (!(v ? ok1 : ok0)) {
      la = -INFINITY;
    }
    if (DZ) {
      T *d = DZ + (int64_t(q) * B + b) * 4;
      for (int k = 0; k < 4; ++k) d[k] = T(dz[k]);
    }
    if (q & 1) {
      na += int((occ >> (q - 1)) & 1);
      nb += v;
    }
  }
  if (logabs) logabs[b] = la;
  if (phase) phase[b] = ph;
}

// Canonical parameters of every qubit from the block-matrix gradients
// (G1 [Q][Q][2H], g1 [Q][2H], G2 [Q][2H][2H], g2 [Q][2H], G3 [Q][2H][4],
// g3 [Q][4]); blockIdx.y is the qubit, whose parameters start at
// H i (i - 1) + i (2H^2 + 8H + 4) in the canonical order
template <class T>
__global__ void nade_qb_fold_kernel(const T *G1, const T *g1, const T *G2, const T *g2,
                                    const T *G3, const T *g3, int Q, int H, double *acc) {
  const int i = blockIdx.y;
  const int64_t H2 = 2 * H;
  int64_t e = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  double *o = acc + int64_t(H) * i * (i - 1) + int64_t(i) * (2 * H * H + 8 * H + 4);
  const T *W1 = G1 + int64_t(i) * Q * H2, *b1 = g1 + i * H2, *W2 = G2 + int64_t(i) * H2 * H2,
          *b2 = g2 + i * H2, *W3 = G3 + int64_t(i) * H2 * 4, *b3 = g3 + i * 4;
  const int64_t n1 = int64_t(i) * H, n2 = int64_t(H) * H;
  if (e < n1) {
    const int64_t j = e / H, c = e % H;
    o[e] += double(W1[j * H2 + c]);
    o[n1 + e] += double(W1[j * H2 + H + c]);
    return;
  }
  e -= n1;
  o += 2 * n1;
  if (e < H) {
    o[e] += double(b1[e]);
    o[H + e] += double(b1[H + e]);
    return;
  }
  e -= H;
  o += 2 * H;
  if (e < n2) {
    const int64_t r = e / H, c = e % H;
    o[e] += double(W2[r * H2 + c]) + double(W2[(H + r) * H2 + H + c]);
    o[n2 + e] += double(W2[r * H2 + H + c]) - double(W2[(H + r) * H2 + c]);
    return;
  }
  e -= n2;
  o += 2 * n2;
  if (e < H) {
    o[e] += double(b2[e]);
    o[H + e] += double(b2[H + e]);
    return;
  }
  e -= H;
  o += 2 * H;
  if (e < 2 * H) {
    const int64_t r = e / 2, v = e % 2;
    o[e] += double(W3[r * 4 + v]) + double(W3[(H + r) * 4 + 2 + v]);
    o[2 * H + e] += double(W3[r * 4 + 2 + v]) - double(W3[(H + r) * 4 + v]);
    return;
  }
  e -= 2 * H;
  o += 4 * H;
  if (e < 2) {
    o[e] += double(b3[e]);
    o[2 + e] += double(b3[2 + e]);
  }
}

template <class T>
struct NadeQB {
  T *X, *H1, *P2, *Y2, *Z;       // bits [B][Q]; per qubit: tanh, pre-ReLU, ReLU, outputs
  T *DZ, *D2, *ones;             // backward only (D1 reuses Y2)
};

template <class T>
size_t nade_qb_carve(const nqs_model &m, int64_t B, bool bwd, Carver &c, NadeQB<T> &A) {
  const int64_t Q = 2 * m.n, H2 = 2 * m.hid;
  A.X = c.take<T>(B * Q);
  A.H1 = c.take<T>(Q * B * H2);
  A.P2 = c.take<T>(Q * B * H2);
  A.Y2 = c.take<T>(Q * B * H2);
  A.Z = c.take<T>(Q * B * 4);
  A.DZ = A.D2 = A.ones = nullptr;
  if (bwd) {
    A.DZ = c.take<T>(Q * B * 4);
    A.D2 = c.take<T>(Q * B * H2);
    A.ones = c.take<T>(B);
  }
  return c.used;
}

// the Q networks on B configurations: H1, P2, Y2 and Z (b3 not added)
template <class T>
void nade_qb_layers(nqs_model &m, const uint64_t *x, int64_t B, NadeQB<T> &A, hipStream_t s) {
  const int Q = 2 * m.n, H = m.hid, H2 = 2 * H;
  hipLaunchKernelGGL(nade_qb_bits_kernel<T>, g1(B * Q), dim3(256), 0, s, x, B, Q, m.sectors(), A.X);
  HIP_LAUNCH_OK();
  gemm_batched<T, false, false>(B, H2, Q, A.X, Q, 0, nade_blk<T>(m, 0, 0), H2, int64_t(Q) * H2,
                                A.H1, H2, B * H2, Q, false, s);
  hipLaunchKernelGGL(nade_qb_bias_ctanh_kernel<T>, g1(int64_t(Q) * B * H), dim3(256), 0, s, A.H1,
                     nade_blk<T>(m, 0, 1), B, Q, H);
  HIP_LAUNCH_OK();
  gemm_batched<T, false, false>(B, H2, H2, A.H1, H2, B * H2, nade_blk<T>(m, 0, 2), H2,
                                int64_t(H2) * H2, A.P2, H2, B * H2, Q, false, s);
  hipLaunchKernelGGL(nade_qb_bias_lrelu_kernel<T>, g1(int64_t(Q) * B * H2), dim3(256), 0, s, A.P2,
                     nade_blk<T>(m, 0, 3), B, Q, H2, A.Y2);
  HIP_LAUNCH_OK();
  gemm_batched<T, false, false>(B, 4, H2, A.Y2, H2, B * H2, nade_blk<T>(m, 0, 4), 4,
                                int64_t(H2) * 4, A.Z, 4, B * 4, Q, false, s);
}

template <class T>
void nade_qb_forward_chunk(nqs_model &m, const uint64_t *x, int64_t B, double *logabs,
                           double *phase, hipStream_t s) {
  NadeQB<T> A;
  Carver c0{nullptr};
  nade_qb_carve<T>(m, B, false, c0, A);
  Carver c{static_cast<char *>(m.ws.reserve(c0.used))};
  nade_qb_carve<T>(m, B, false, c, A);
  nade_qb_layers<T>(m, x, B, A, s);
  hipLaunchKernelGGL(nade_qb_combine_kernel<T>, g1(B), dim3(256), 0, s, x, B, 2 * m.n,
                     m.sectors(), A.Z, nade_blk<T>(m, 0, 5), logabs, phase, nullptr, nullptr,
                     static_cast<T *>(nullptr));
  HIP_LAUNCH_OK();
}

// Gradients of the block matrices of every qubit, accumulated over the chunks
// of the batch in T (G: the six arrays of nade_qb_fold_kernel, contiguous),
// then folded onto the canonical parameters in m.grad_acc.
template <class T>
void nade_qb_backward(nqs_model &m, const uint64_t *x, int64_t Btot, const double *gl,
                      const double *gp, int64_t ch, hipStream_t s) {
  const int Q = 2 * m.n, H = m.hid, H2 = 2 * H;
  for (int i = 0; i < Q; ++i)
    NQS_REQUIRE(m.off[size_t(12 * i)] ==
                    int64_t(H) * i * (i - 1) + int64_t(i) * (2 * H * H + 8 * H + 4),
                NQS_EINVAL, "per-qubit ansatz: unexpected parameter layout");
  const int64_t s1 = int64_t(Q) * H2, s2 = int64_t(H2) * H2, s3 = int64_t(H2) * 4;
  const int64_t gsize = Q * (s1 + H2 + s2 + H2 + s3 + 4);
  T *G1 = static_cast<T *>(m.ws2.reserve(size_t(gsize) * sizeof(T)));
  T *gb1 = G1 + Q * s1, *G2 = gb1 + Q * H2, *gb2 = G2 + Q * s2, *G3 = gb2 + Q * H2,
    *gb3 = G3 + Q * s3;
  zero_async(G1, size_t(gsize) * sizeof(T), s);
  NadeQB<T> A;
  Carver c0{nullptr};
  nade_qb_carve<T>(m, std::min(ch, Btot), true, c0, A);
  Carver c{static_cast<char *>(m.ws.reserve(c0.used))};
  for (int64_t b0 = 0; b0 < Btot; b0 += ch) {
    const int64_t B = std::min(ch, Btot - b0);
    Carver cc{c.base};
    nade_qb_carve<T>(m, B, true, cc, A);
    const uint64_t *xb = x + b0;
    nade_qb_layers<T>(m, xb, B, A, s);
    hipLaunchKernelGGL(nade_qb_combine_kernel<T>, g1(B), dim3(256), 0, s, xb, B, Q, m.sectors(),
                       A.Z, nade_blk<T>(m, 0, 5), nullptr, nullptr, gl + b0, gp + b0, A.DZ);
    HIP_LAUNCH_OK();
    fill_ones<T>(A.ones, B, s);
    // layer 3: dW3 = Y2^T DZ, db3 = 1^T DZ, dY2 = DZ W3^T
    gemm_batched<T, true, false>(H2, 4, B, A.Y2, H2, B * H2, A.DZ, 4, B * 4, G3, 4, s3, Q, true, s);
    gemm_batched<T, true, false>(1, 4, B, A.ones, 1, 0, A.DZ, 4, B * 4, gb3, 4, 4, Q, true, s);
    gemm_batched<T, false, true>(B, H2, 4, A.DZ, 4, B * 4, nade_blk<T>(m, 0, 4), 4, s3, A.D2, H2,
                                 B * H2, Q, false, s);
    // layer 2 through the leaky ReLU
    lrelu_bwd<T>(A.P2, A.D2, int64_t(Q) * B * H2, s);
    gemm_batched<T, true, false>(H2, H2, B, A.H1, H2, B * H2, A.D2, H2, B * H2, G2, H2, s2, Q,
                                 true, s);
    gemm_batched<T, true, false>(1, H2, B, A.ones, 1, 0, A.D2, H2, B * H2, gb2, H2, H2, Q, true,
                                 s);
    T *D1 = A.Y2;
    gemm_batched<T, false, true>(B, H2, H2, A.D2, H2, B * H2, nade_blk<T>(m, 0, 2), H2, s2, D1,
                                 H2, B * H2, Q, false, s);
    // layer 1 through the complex tanh; rows of W1 beyond a qubit's inputs get
    // gradients of padding, which the fold does not read
    hipLaunchKernelGGL(nade_ctanh_bwd_kernel<T>, g1(int64_t(Q) * B * H), dim3(256), 0, s, A.H1,
                       D1, int64_t(Q) * B, H);
    HIP_LAUNCH_OK();
    gemm_batched<T, true, false>(Q, H2, B, A.X, Q, 0, D1, H2, B * H2, G1, H2, s1, Q, true, s);
    gemm_batched<T, true, false>(1, H2, B, A.ones, 1, 0, D1, H2, B * H2, gb1, H2, H2, Q, true, s);
  }
  const int64_t per_max = int64_t(Q - 1) * H + 2 * H + int64_t(H) * H + 2 * H + 2;
  hipLaunchKernelGGL(nade_qb_fold_kernel<T>, dim3(unsigned(ceil_div(per_max, 256)), unsigned(Q)),
                     dim3(256), 0, s, G1, gb1, G2, gb2, G3, gb3, Q, H, m.grad_acc.as<double>());
  HIP_LAUNCH_OK();
}

template <class T>
int64_t chunk_rows(const nqs_model &m, bool bwd) {
  // configurations per chunk, sized for the model's activation budget (an
  // eighth of the device memory free at creation, 1..16 GiB): on a 288 GB
  // device a whole 2e4-sample, 15-token backward is one chunk of large GEMMs
  // (per-qubit ansatz: the qubit-batched activations, which also bound the
  // sampler's token evaluations)
  const int64_t per = m.kind == NQS_MODEL_NADE
                          ? int64_t(2 * m.n) * (4 * 2 * m.hid + 9) + 1
                      : m.kind == NQS_MODEL_MLP
                          ? int64_t(m.n) * 8 * 4 + 4 * m.n + 3 * m.hid + 8
                          : int64_t(m.n) * (bwd ? (m.L * (7 * m.d + 2 * m.F + 8) +
                                                   m.L * m.H * m.n + 14 * m.d + 3 * m.F)
                                                : (8 * m.d + 2 * m.F + 8)) + 6 * m.PH;
  int64_t c = m.act_budget / (per * int64_t(sizeof(T)));
  // at most 128k token rows: measured fastest for the library GEMMs of both transformer
  // workloads (64k and 320k rows are 5-25 % slower per step); the split-bf16
  // backward takes up to 512k rows (fewer launches)
  const bool mx = bwd && m.mixed_backward && mx_backward_ok(m);
  c = std::min<int64_t>(c, m.kind == NQS_MODEL_NADE ? 65536 : (mx ? 524288 : 131072) / m.n);
  return c < 64 ? 64 : c;
}

template <class T>
void forward_T(nqs_model &m, const uint64_t *x, int64_t B, double *logabs, double *phase,
               T *logits_keep, hipStream_t s) {
  if (m.kind == NQS_MODEL_MLP) {
    mlp_forward_chunk<T>(m, x, B, logabs, phase, logits_keep, s);
    return;
  }
  if (m.kind == NQS_MODEL_NADE) {
    // the sampler's token outputs from the token path, amplitudes batched over qubits
    if (logits_keep) nade_forward_chunk<T>(m, x, B, logabs, phase, logits_keep, s);
    else nade_qb_forward_chunk<T>(m, x, B, logabs, phase, s);
    return;
  }
  Carver c0{nullptr};
  TfAct<T> A;
  carve_tf<T>(m, B, false, c0, A);
  Carver c{static_cast<char *>(m.ws.reserve(c0.used))};
  carve_tf<T>(m, B, false, c, A);
  if (logits_keep) A.logits = logits_keep;
  tf_forward_chunk<T>(m, x, B, false, A, logabs, phase, s);
}

}  // namespace

int64_t model_chunk(const nqs_model &m, bool bwd) {
  return m.fp64() ? chunk_rows<double>(m, bwd) : chunk_rows<float>(m, bwd);
}

void model_forward(nqs_model &m, const uint64_t *x, int64_t B, double *logabs, double *phase,
                   void *logits, hipStream_t s) {
  if (m.kind == NQS_MODEL_TABLE) {
    NQS_REQUIRE(!logits, NQS_EINVAL, "table model: no per-position logits");
    table_forward(m, x, B, logabs, phase, s);
    return;
  }
  const int64_t ch = model_chunk(m, false);
  const int w = m.kind == NQS_MODEL_TRANSFORMER ? 4 : 8;
  for (int64_t b0 = 0; b0 < B; b0 += ch) {
    const int64_t nb = B - b0 < ch ? B - b0 : ch;
    const size_t lo = size_t(b0) * m.n * w;
    if (m.fp64())
      forward_T<double>(m, x + b0, nb, logabs ? logabs + b0 : nullptr, phase ? phase + b0 : nullptr,
                        logits ? static_cast<double *>(logits) + lo : nullptr, s);
    else
      forward_T<float>(m, x + b0, nb, logabs ? logabs + b0 : nullptr, phase ? phase + b0 : nullptr,
                       logits ? static_cast<float *>(logits) + lo : nullptr, s);
  }
}

void model_cond_logits(nqs_model &m, const uint64_t *prefix, int64_t B, int p, double *out4,
                       hipStream_t s) {
  if (m.kind == NQS_MODEL_TABLE) {
    table_cond_logits(m, prefix, B, p, out4, s);
    return;
  }
  if (m.precision == NQS_BF16 && (fused_supported(m) || nade_fused_supported(m))) {
    fused_forward(m, prefix, B, nullptr, nullptr, out4, p, s);
    return;
  }
  const int w = m.kind == NQS_MODEL_TRANSFORMER ? 4 : 8;
  const int64_t ch = model_chunk(m, false);
  void *buf = m.logit_buf.reserve(size_t(ch) * m.n * w * m.elem());
  for (int64_t b0 = 0; b0 < B; b0 += ch) {
    const int64_t nb = B - b0 < ch ? B - b0 : ch;
    if (m.fp64()) {
      forward_T<double>(m, prefix + b0, nb, nullptr, nullptr, static_cast<double *>(buf), s);
      hipLaunchKernelGGL(cond_extract_kernel<double>, g1(nb * 4), dim3(256), 0, s,
                         static_cast<double *>(buf), nb, m.n, w, p, out4 + 4 * b0);
    } else {
      forward_T<float>(m, prefix + b0, nb, nullptr, nullptr, static_cast<float *>(buf), s);
      hipLaunchKernelGGL(cond_extract_kernel<float>, g1(nb * 4), dim3(256), 0, s,
                         static_cast<float *>(buf), nb, m.n, w, p, out4 + 4 * b0);
    }
    HIP_LAUNCH_OK();
  }
}

// derived NADE blocks of every qubit from the canonical parameters
void nade_pack(nqs_model &m, hipStream_t s) {
  const int H = m.hid, H2 = 2 * H, Q = 2 * m.n;
  // one array per block kind, qubit-major with a uniform stride (W1 padded to
  // Q rows), so that the batched products can stride over the qubits
  const int64_t sizes[kNadeBlocks] = {int64_t(Q) * H2, H2, int64_t(H2) * H2, H2, int64_t(H2) * 4, 4};
  int64_t first[kNadeBlocks], total = 0;
  for (int k = 0; k < kNadeBlocks; ++k) {
    first[k] = total;
    total += Q * sizes[k];
  }
  m.nade_off.clear();
  for (int i = 0; i < Q; ++i)
    for (int k = 0; k < kNadeBlocks; ++k) m.nade_off.push_back(first[k] + i * sizes[k]);
  m.packed.reserve(size_t(total) * m.elem());
  for (int i = 0; i < Q; ++i) {
    const int64_t count = int64_t(Q) * H2 + 2 * H2 + int64_t(H2) * H2 + int64_t(H2) * 4 + 4;
    auto launch = [&](auto *base) {
      using T = std::remove_pointer_t<decltype(base)>;
      auto prm = [&](int k) { return base + m.off[size_t(12 * i + k)]; };
      auto blk = [&](int k) { return m.packed.as<T>() + m.nade_off[size_t(i) * kNadeBlocks + k]; };
      hipLaunchKernelGGL(nade_pack_kernel<T>, g1(count), dim3(256), 0, s, prm(0), prm(1), prm(2),
                         prm(3), prm(4), prm(5), prm(6), prm(7), prm(8), prm(9), prm(10), prm(11),
                         i, Q, H, blk(0), blk(1), blk(2), blk(3), blk(4), blk(5));
    };
    if (m.fp64())
      launch(m.master.as<double>());
    else
      launch(m.master.as<float>());
    HIP_LAUNCH_OK();
  }
}

void model_backward(nqs_model &m, const uint64_t *x, int64_t B, const double *gl,
                    const double *gp, void *grad, hipStream_t s) {
  double *acc = static_cast<double *>(m.grad_acc.reserve(size_t(m.P) * 8));
  zero_async(acc, size_t(m.P) * 8, s);
  if (m.kind == NQS_MODEL_TABLE) {
    table_backward(m, x, B, gl, gp, acc, s);
    convert<double, double>(acc, static_cast<double *>(grad), m.P, s);
    return;
  }
  const int64_t ch = model_chunk(m, true);
  if (m.kind == NQS_MODEL_NADE && B > 0) {
    if (m.fp64()) nade_qb_backward<double>(m, x, B, gl, gp, ch, s);
    else nade_qb_backward<float>(m, x, B, gl, gp, ch, s);
  }
  // bf16 transformers: split images of the weights, made once per call
  MxPack mx;
  const bool mixed = B > 0 && m.mixed_backward && mx_backward_ok(m);
  if (mixed) mx = mx_pack_model(m, s);
  for (int64_t b0 = 0; b0 < B && m.kind != NQS_MODEL_NADE; b0 += ch) {
    const int64_t nb = B - b0 < ch ? B - b0 : ch;
    if (m.kind == NQS_MODEL_MLP) {
      if (m.fp64()) mlp_backward_chunk<double>(m, x + b0, nb, gl + b0, gp + b0, s);
      else mlp_backward_chunk<float>(m, x + b0, nb, gl + b0, gp + b0, s);
    } else {
      if (m.fp64()) tf_backward_chunk<double>(m, x + b0, nb, gl + b0, gp + b0, s);
      else tf_backward_chunk<float>(m, x + b0, nb, gl + b0, gp + b0, s, mixed ? &mx : nullptr);
    }
  }
  if (m.fp64()) convert<double, double>(acc, static_cast<double *>(grad), m.P, s);
  else convert<double, float>(acc, static_cast<float *>(grad), m.P, s);
}

}  // namespace nqs
