// Amplitude networks, layer-by-layer path (FP64 and FP32 modes, all backward
// passes).  Paper: the ANQS product rule psi(x) = prod_p psi_p(x_p | x_<p);
// Mask-Unphysical conditionals ("Pruning strategies"); Appendix B for the
// per-token MLP.  The physicality of a prefix comes from Algorithm 1, filled
// bottom-up into a (position, n_alpha, n_beta) table when the model is made.
#include <algorithm>
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

template <class T>
void tf_forward_chunk(nqs_model &m, const uint64_t *x, int64_t B, bool save, TfAct<T> &A,
                      double *logabs, double *phase, hipStream_t s) {
  const int n = m.n, d = m.d, F = m.F, H = m.H, L = m.L, PH = m.PH;
  const int64_t R = B * n;
  hipLaunchKernelGGL(embed_kernel<T>, g1(R * d), dim3(256), 0, s, x, B, n, d, P<T>(m, TF_TOK),
                     P<T>(m, TF_POS), A.layer[0].h_in);
  HIP_LAUNCH_OK();
  for (int l = 0; l < L; ++l) {
    Layer<T> &y = A.layer[l];
    auto W = [&](int k) { return P<T>(m, tf_layer(l, k)); };
    layernorm<T>(y.h_in, R, d, W(TF_LN1G), W(TF_LN1B), y.a1, y.m1, y.r1, s);
    gemm<T, false, false>(R, 3 * d, d, y.a1, d, W(TF_WQKV), 3 * d, y.qkv, 3 * d, W(TF_BQKV),
                             nullptr, EPI_STORE, s);
    attention_fwd<T>(y.qkv, B, n, d, H, y.o, y.probs, s);
    if (y.h_mid != y.h_in)
      HIP_OK(hipMemcpyAsync(y.h_mid, y.h_in, R * d * sizeof(T), hipMemcpyDeviceToDevice, s));
    gemm<T, false, false>(R, d, d, y.o, d, W(TF_WO), d, y.h_mid, d, W(TF_BO), nullptr, EPI_ADD,
                             s);
    layernorm<T>(y.h_mid, R, d, W(TF_LN2G), W(TF_LN2B), y.a2, y.m2, y.r2, s);
    gemm<T, false, false>(R, F, d, y.a2, d, W(TF_W1), F, y.f, F, W(TF_B1), y.fpre, EPI_GELU, s);
    T *h_next = (l + 1 < L) ? A.layer[l + 1].h_in : A.h_out;
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
    gemm<T, false, false>(B, PH, PH, A.z1, PH, P<T>(m, tf_tail(L, TF_PW2)), PH, A.z2, PH,
                             P<T>(m, tf_tail(L, TF_PB2)), A.z2pre, EPI_GELU, s);
    if (phase) {
      hipLaunchKernelGGL(phase_out_kernel<T>, g1(B, 4), dim3(256), 0, s, A.z2, B, PH,
                         P<T>(m, tf_tail(L, TF_PW3)), P<T>(m, tf_tail(L, TF_PB3)), phase);
      HIP_LAUNCH_OK();
    }
  }
}

// dW += X^T dY reduced over the R rows, accumulated in double at the parameter's offset.
template <class T>
void wgrad(nqs_model &m, int64_t Mi, int64_t No, int64_t R, const T *X, int64_t ldx, const T *dY,
           int64_t ldy, int pidx, hipStream_t s) {
  void *part = m.part.reserve(wgrad_scratch_bytes(R, Mi, No, std::max(ldx, ldy), sizeof(T)));
  wgrad_acc(X, ldx, dY, ldy, R, Mi, No, m.grad_acc.as<double>() + m.off[pidx], part, s);
}

// db += column sums of dY (fixed-order, double)
template <class T>
void bgrad(nqs_model &m, const T *dY, int64_t R, int64_t N, int64_t ld, int pidx, hipStream_t s) {
  double *part = static_cast<double *>(m.part.reserve(colsum_scratch_bytes(R, N)));
  colsum_acc<T>(dY, R, N, ld, m.grad_acc.as<double>() + m.off[pidx], part, s);
}

template <class T>
void tf_backward_chunk(nqs_model &m, const uint64_t *x, int64_t B, const double *gl,
                       const double *gp, hipStream_t s) {
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

  tf_forward_chunk<T>(m, x, B, true, A, nullptr, nullptr, s);

  // head and masked log-softmax
  hipLaunchKernelGGL(dlogits_kernel<T>, g1(B), dim3(256), 0, s, x, B, n, A.logits, 4,
                     m.sectors(), gl, dl, 4);
  HIP_LAUNCH_OK();
  wgrad<T>(m, d, 4, R, A.hf, d, dl, 4, tf_tail(L, TF_WHEAD), s);
  bgrad<T>(m, dl, R, 4, 4, tf_tail(L, TF_BHEAD), s);
  bgrad<T>(m, dl, B, int64_t(n) * 4, int64_t(n) * 4, tf_tail(L, TF_LBIAS), s);
  gemm<T, false, true>(R, d, 4, dl, 4, P<T>(m, tf_tail(L, TF_WHEAD)), 4, da, d, nullptr,
                          nullptr, EPI_STORE, s);
  layernorm_bwd<T>(A.h_out, A.mf, A.rf, R, d, P<T>(m, tf_tail(L, TF_LNFG)), da, dh, false, tmp, s);
  bgrad<T>(m, tmp, R, d, d, tf_tail(L, TF_LNFG), s);
  bgrad<T>(m, da, R, d, d, tf_tail(L, TF_LNFB), s);

  for (int l = L - 1; l >= 0; --l) {
    Layer<T> &y = A.layer[l];
    auto W = [&](int k) { return P<T>(m, tf_layer(l, k)); };
    // h_out = h_mid + gelu(a2 W1 + b1) W2 + b2
    wgrad<T>(m, F, d, R, y.f, F, dh, d, tf_layer(l, TF_W2), s);
    bgrad<T>(m, dh, R, d, d, tf_layer(l, TF_B2), s);
    gemm<T, false, true>(R, F, d, dh, d, W(TF_W2), d, df, F, nullptr, nullptr, EPI_STORE, s);
    gelu_bwd<T>(y.fpre, df, R * F, s);
    wgrad<T>(m, d, F, R, y.a2, d, df, F, tf_layer(l, TF_W1), s);
    bgrad<T>(m, df, R, F, F, tf_layer(l, TF_B1), s);
    gemm<T, false, true>(R, d, F, df, F, W(TF_W1), F, da, d, nullptr, nullptr, EPI_STORE, s);
    layernorm_bwd<T>(y.h_mid, y.m2, y.r2, R, d, W(TF_LN2G), da, dh, true, tmp, s);
    bgrad<T>(m, tmp, R, d, d, tf_layer(l, TF_LN2G), s);
    bgrad<T>(m, da, R, d, d, tf_layer(l, TF_LN2B), s);
    // h_mid = h_in + attn(a1) Wo + bo
    wgrad<T>(m, d, d, R, y.o, d, dh, d, tf_layer(l, TF_WO), s);
    bgrad<T>(m, dh, R, d, d, tf_layer(l, TF_BO), s);
    gemm<T, false, true>(R, d, d, dh, d, W(TF_WO), d, da, d, nullptr, nullptr, EPI_STORE, s);
    attention_bwd<T>(y.qkv, y.probs, da, B, n, d, H, dq, s);
    wgrad<T>(m, d, 3 * d, R, y.a1, d, dq, 3 * d, tf_layer(l, TF_WQKV), s);
    bgrad<T>(m, dq, R, 3 * d, 3 * d, tf_layer(l, TF_BQKV), s);
    gemm<T, false, true>(R, d, 3 * d, dq, 3 * d, W(TF_WQKV), 3 * d, da, d, nullptr, nullptr,
                            EPI_STORE, s);
    layernorm_bwd<T>(y.h_in, y.m1, y.r1, R, d, W(TF_LN1G), da, dh, true, tmp, s);
    bgrad<T>(m, tmp, R, d, d, tf_layer(l, TF_LN1G), s);
    bgrad<T>(m, da, R, d, d, tf_layer(l, TF_LN1B), s);
  }
  // embeddings: token table through the one-hot input classes, positions by column sums
  hipLaunchKernelGGL(in_class_kernel<T>, g1(R * 5), dim3(256), 0, s, x, B, n, tmp);
  HIP_LAUNCH_OK();
  wgrad<T>(m, 5, d, R, tmp, 5, dh, d, TF_TOK, s);
  bgrad<T>(m, dh, B, int64_t(n) * d, int64_t(n) * d, TF_POS, s);

  // phase MLP: phi = gelu(gelu(onehot W1 + b1) W2 + b2) w3 + b3
  T *dz2 = dz, *dz1 = dz + B * PH;
  hipLaunchKernelGGL(phase_dz_kernel<T>, g1(B * PH), dim3(256), 0, s, gp, B, PH,
                     P<T>(m, tf_tail(L, TF_PW3)), dz2, gpt);
  HIP_LAUNCH_OK();
  wgrad<T>(m, PH, 1, B, A.z2, PH, gpt, 1, tf_tail(L, TF_PW3), s);
  bgrad<T>(m, gpt, B, 1, 1, tf_tail(L, TF_PB3), s);
  gelu_bwd<T>(A.z2pre, dz2, B * PH, s);
  wgrad<T>(m, PH, PH, B, A.z1, PH, dz2, PH, tf_tail(L, TF_PW2), s);
  bgrad<T>(m, dz2, B, PH, PH, tf_tail(L, TF_PB2), s);
  gemm<T, false, true>(B, PH, PH, dz2, PH, P<T>(m, tf_tail(L, TF_PW2)), PH, dz1, PH, nullptr,
                          nullptr, EPI_STORE, s);
  gelu_bwd<T>(A.z1pre, dz1, B * PH, s);
  bgrad<T>(m, dz1, B, PH, PH, tf_tail(L, TF_PB1), s);
  hipLaunchKernelGGL(onehot_kernel<T>, g1(B * 4 * n), dim3(256), 0, s, x, B, n, m.sectors(), tmp);
  HIP_LAUNCH_OK();
  wgrad<T>(m, 4 * n, PH, B, tmp, 4 * n, dz1, PH, tf_tail(L, TF_PW1), s);
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

template <class T>
int64_t chunk_rows(const nqs_model &m, bool bwd) {
  // configurations per chunk, sized for the model's activation budget (an
  // eighth of the device memory free at creation, 1..16 GiB): on a 288 GB
  // device a whole 2e4-sample, 15-token backward is one chunk of large GEMMs
  const int64_t per = m.kind == NQS_MODEL_MLP
                          ? int64_t(m.n) * 8 * 4 + 4 * m.n + 3 * m.hid + 8
                          : int64_t(m.n) * (bwd ? (m.L * (7 * m.d + 2 * m.F + 8) +
                                                   m.L * m.H * m.n + 14 * m.d + 3 * m.F)
                                                : (8 * m.d + 2 * m.F + 8)) + 6 * m.PH;
  int64_t c = m.act_budget / (per * int64_t(sizeof(T)));
  // at most 128k token rows: measured fastest for the library GEMMs of both transformer
  // workloads (64k and 320k rows are 5-25 % slower per step)
  c = std::min<int64_t>(c, 131072 / m.n);
  return c < 64 ? 64 : c;
}

template <class T>
void forward_T(nqs_model &m, const uint64_t *x, int64_t B, double *logabs, double *phase,
               T *logits_keep, hipStream_t s) {
  if (m.kind == NQS_MODEL_MLP) {
    mlp_forward_chunk<T>(m, x, B, logabs, phase, logits_keep, s);
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
  const int64_t ch = model_chunk(m, false);
  const int w = m.kind == NQS_MODEL_MLP ? 8 : 4;
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
  if (m.precision == NQS_BF16 && fused_supported(m)) {
    fused_forward(m, prefix, B, nullptr, nullptr, out4, p, s);
    return;
  }
  const int w = m.kind == NQS_MODEL_MLP ? 8 : 4;
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

void model_backward(nqs_model &m, const uint64_t *x, int64_t B, const double *gl,
                    const double *gp, void *grad, hipStream_t s) {
  double *acc = static_cast<double *>(m.grad_acc.reserve(size_t(m.P) * 8));
  zero_async(acc, size_t(m.P) * 8, s);
  const int64_t ch = model_chunk(m, true);
  for (int64_t b0 = 0; b0 < B; b0 += ch) {
    const int64_t nb = B - b0 < ch ? B - b0 : ch;
    if (m.kind == NQS_MODEL_MLP) {
      if (m.fp64()) mlp_backward_chunk<double>(m, x + b0, nb, gl + b0, gp + b0, s);
      else mlp_backward_chunk<float>(m, x + b0, nb, gl + b0, gp + b0, s);
    } else {
      if (m.fp64()) tf_backward_chunk<double>(m, x + b0, nb, gl + b0, gp + b0, s);
      else tf_backward_chunk<float>(m, x + b0, nb, gl + b0, gp + b0, s);
    }
  }
  if (m.fp64()) convert<double, double>(acc, static_cast<double *>(grad), m.P, s);
  else convert<double, float>(acc, static_cast<float *>(grad), m.P, s);
}

}  // namespace nqs
