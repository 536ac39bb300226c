// Fused bf16 transformer forward on MFMA (gfx950): log|psi|, phase, or the
// sampler's conditional logits, for a batch of configurations.  Paper: ANQS
// product rule and Mask-Unphysical conditionals ("Pruning strategies").
//
// Design.  One 64-lane wave owns 32 rows = 2 configurations x 16 positions
// (sequences are padded to 16 tokens) and carries them through every layer in
// registers; there is no LDS traffic for activations.  All GEMMs use
// v_mfma_f32_32x32x16_bf16 (bf16 operands, fp32 accumulation).  Activations
// are kept "feature-major": an accumulator block holds 32 features x 32 rows,
// lane l owning row l%32 and, for j = 0..15, feature
//     (j/4)*8 + (l/32)*4 + j%4.
// Read as an MFMA operand, lane l supplies row l%32 and 8 consecutive k-slots
// (l/32)*8 .. +7.  So the accumulator of one GEMM is, after conversion to
// bf16, already the activation operand of the next one, provided the k index
// inside every 16-wide step is permuted the same way in the weights:
//     slot i of lane-half h  <->  feature pi_h(i) = (i/4)*8 + h*4 + i%4.
// Weights are packed once into that fragment order (fused_pack).  Value and
// attention-output products are computed in the transposed orientation
// (activations as the A operand) so that no transpose is ever needed:
//     S^T = K Q^T,  P^T = softmax over keys,  O^T = V^T P^T,
// where V comes out key-major and O^T feature-major again.
//
// The attention probabilities P and the attention output O enter their
// products as bf16 pairs hi + lo (lo = the rounding error of hi, two MFMAs per
// product): their bf16 rounding dominated the error of the local energy of the
// highest-count samples (1.6e-4 Ha against the FP64 oracle on the 30-qubit
// system; 1.7e-6 Ha with the pairs, for 7 % more kernel time).
//
// The attention weight matrices are packed as two bf16 fragment sets, hi =
// bf16(W) and lo = bf16(W - hi), and their products take both (W x = hi x +
// lo x), so those weights carry about 16 significant bits.  Optimiser steps
// move the fp32 master weights off the bf16 grid; rounding them to bf16 alone
// changes the network itself, the same way for every configuration, and moved
// the energy of the 30-qubit system's dominant samples by ~1e-4 Ha (local
// energies of single samples by up to 2e-3 Ha) after steps of the size of five
// Adam steps at 1e-3, most of it from the attention matrices (NP_* below).  The
// lo set is a second step of the same kind in the weight stream (a sub-step),
// so the LDS ring and the registers are unchanged; only the MFMA count and the
// stream length grow.
//
// Per 32 rows and layer: Q, K (2 x 8 x 8), V (8 x 4), S (8), O (2 x 16),
// out-projection (2 x 32), FFN (128 + 128) MFMAs.  After 16 passes (32
// configurations) the phase MLP of those 32 configurations runs as one
// 256 x 256 GEMM with the configurations as the 32 columns.
#include <cmath>
#include <vector>

#include "ham.h"
#include "model.h"
#include "ops.h"

namespace nqs {
namespace {

typedef __attribute__((ext_vector_type(8))) __bf16 bf16x8;
typedef __attribute__((ext_vector_type(2))) __bf16 bf16x2;
typedef __attribute__((ext_vector_type(16))) float f32x16;
typedef __attribute__((ext_vector_type(2))) float f32x2;
typedef __attribute__((ext_vector_type(4))) float f32x4;
typedef __attribute__((ext_vector_type(2))) int i32x2;

struct TimingRecord {
  hipEvent_t start, stop;           // null for a record measured elsewhere (ms set)
  int64_t configs;
  float ms;
  int mode;                         // row layout of the transformer kernel, -1 for the others
};
bool g_timing = false;
std::vector<TimingRecord> g_records;

constexpr int kMaxLayers = 8;
constexpr int kSeqMax = 32;       // longest sequence (tokens)
constexpr int kTrunk = 8;         // positions of a shared prefix (TRUNK / SUFFIX)
// bytes of middle-level entries held at once (a slice; addressed by 32-bit offsets)
constexpr int64_t kMidSliceBytes = int64_t(1) << 31;

// Row layouts of a wave's 32 rows (R rows per configuration, 32 / R
// configurations per pass):
//   PLAIN   R = 16: positions 0..15 of 2 configurations (up to 16 tokens);
//   WIDE    R = 32: positions 0..31 of 1 configuration (17..32 tokens);
//   TRUNK   R = 8:  positions 0..7 of 4 distinct 8-token prefixes; the keys and
//                   values of every layer and the log-probability of the 8
//                   tokens are stored per prefix;
//   SUFFIX  R = 8:  positions 8..15 of 4 configurations, attending to the
//                   stored keys and values of their prefix.
// Positions 0..7 of a causal network see only tokens 0..6, so their hidden
// states, keys and values are the same for every configuration with the same
// first 8 tokens; distinct x' of one step share few such prefixes (at most
// 4^8), so TRUNK + SUFFIX do about half the work of PLAIN per configuration.
//   MID     R = 4:  positions 8..pm-1 (pm <= 12; rows up to 11) of 8
//                   distinct pm-token prefixes (of at most two 8-token
//                   prefixes), attending to their 8-token prefix's keys and
//                   values; stores
//                   its own keys and values and the log-probability of tokens
//                   8..pm-1 per pm-token prefix;
//   TAIL    R = 4:  positions pm..pm+3 of 8 configurations (of at most two
//                   8-token prefixes), attending to both stored levels.
// pm = n - 4 makes TAIL the last four positions.  When the sector leaves one
// token at the last position its masked conditional is 1 or 0 (a membership
// test, no network), so pm = n - 5: TAIL takes the four positions before the
// last, a small kernel applies the test, and the middle level holds
// (n-5)-token prefixes, ~2.4x fewer than (n-4)-token ones on the
// 30-spin-orbital system.
//   TREE    R = 4:  when the sector fixes the last token (q = n - 3, and
//                   pm = q - 1): each item is a slot of four rows holding
//                   subtrees of one (q-1)-token prefix: root rows (distinct
//                   q-token prefixes, position q), each followed by some of its
//                   distinct (q+1)-token extensions (position q + 1); a row
//                   attends to the 8-token prefix, the middle level and, in
//                   its slot, to its root row and itself.  Each
//                   row stores its masked conditional (4 log-probabilities) per
//                   prefix; a gather over the configurations adds them up with
//                   MID's (which also stores the conditional of its row pm) and
//                   applies the last token's membership test.
//   PHASE:          no transformer rows: the phase MLP of every configuration.
// At 15 tokens a configuration's rows 12 and 13 are shared by the ~2.1 x'
// per 12-token prefix and ~1.5 per 13-token prefix, so TREE evaluates ~3.1e6
// slots instead of TAIL's 7.7e6 configurations (MID then covers the 11-token
// prefixes, 1.4e6 instead of 5.9e5).
// MID / TAIL / TREE take their items through an index list (a.src; -1 =
// padding; TREE: four entries per slot, one per row) in which a pass of 8
// items holds at most two 8-token prefixes: the second one's keys take score
// rows 8..15 and its values the k-slots 4..7 of the prefix's value step, so
// a pass costs the same with one or two.
enum Mode : int { PLAIN = 0, WIDE = 1, TRUNK = 2, SUFFIX = 3, MID = 4, TAIL = 5, TREE = 6, PHASE = 7 };
template <int MODE>
struct Rows {
  static constexpr int R = MODE == PLAIN ? 16 : MODE == WIDE ? 32 : MODE <= SUFFIX ? 8 : 4;
  static constexpr int CPT = 32 / R;            // configurations per pass
  static constexpr int P0 = MODE == SUFFIX || MODE == MID ? kTrunk : MODE == TAIL ? 12 : 0;
  // layouts that attend to both stored levels (8-token prefix and middle)
  static constexpr bool TAILS = MODE == TAIL || MODE == TREE;
  // layouts that read the 8-token prefix's stored entry through an item list
  static constexpr bool LISTED = MODE == MID || TAILS;
  static constexpr int MAXP = 32 / CPT;         // passes per chunk of 32 configurations
};
// Fragment sets (1 = hi, 2 = hi and lo) of the attention matrices (Q, K, V,
// output projection), of the first and of the second feed-forward matrix.
// Measured on the 30-qubit model after five Adam steps at 1e-3 (energy of the
// eight highest-count samples against the FP64 oracle; kernel time per launch
// on the local-energy step): every matrix split 3.8e-5 Ha / 22.4 ms, attention
// and W2 6.5e-5 / 20.0 ms, attention only 2.4e-5 / 17.4 ms, none (weights
// rounded to bf16) ~1.8e-4 Ha in an FP64 simulation of the same rounding.  With
// the attention matrices split the remaining difference is the activations'
// rounding (the FFN weights' share simulated at 6e-6 .. 4e-5 Ha on three
// trained models), so the FFN matrices keep one set.
constexpr int NP_ATT = 2, NP_W1 = 1, NP_W2 = 1;
constexpr int NP = 2;             // layout: every layer keeps room for both sets

__device__ __host__ inline int perm_feature(int b, int h, int j) {
  return 32 * b + (j / 4) * 8 + h * 4 + (j % 4);
}

struct FusedArgs {
  const bf16x8 *pk;                 // packed weight fragments
  const float *vec;                 // permuted fp32 vectors
  int64_t q[kMaxLayers], k[kMaxLayers], v[kMaxLayers], o[kMaxLayers], w1[kMaxLayers],
      w2[kMaxLayers];               // fragment offsets (units of bf16x8)
  int64_t ln1g[kMaxLayers], ln1b[kMaxLayers], bq[kMaxLayers], bk[kMaxLayers], bv[kMaxLayers],
      bo[kMaxLayers], ln2g[kMaxLayers], ln2b[kMaxLayers], b1[kMaxLayers], b2[kMaxLayers];
  int64_t p2, p2lo;                 // phase W2 fragments (hi, lo)
  int64_t p1, p1lo;                 // phase W1 fragments (hi, lo; PHASE): rows 4t + token, then zeros
  int ks1;                          // k-steps of the phase W1 fragments (4 n rows)
  int64_t lnfg, lnfb, whead, bhead, lbias, tok, pos, pb1, pb2, pw3, pb3, pw1;  // vec offsets
  Sectors sec;                      // molecule(s) of the configurations
  const uint64_t *x;
  int64_t B;                        // configurations (capacity when `count` is given)
  const int64_t *count;             // optional device-side count (persistent launches)
  int n, L, cond_p;                 // n = positions of the model; cond_p: see the logit store
  int passes;                       // passes per chunk (32 / R configurations each; 0: from *count)
  int lds_floats;                   // vec[0 .. lds_floats) is staged in LDS (all but pw1)
  double *logabs, *phase, *cond;
  // TRUNK / SUFFIX: per prefix entry (kv_bytes each) the keys and values of
  // positions 0..7 in every layer, and the log-probability of tokens 0..7;
  // SUFFIX finds a configuration's entry at slot[x & 0xFFFF]
  uint8_t *kv;
  int64_t kv_bytes, kv_total;       // bytes per entry, of the buffer (<= 2^31)
  float *plogp;
  const int64_t *slot;
  // MID / TAIL: item -> configuration (-1 = padding); the 8- and pm-token
  // prefix entries of configuration i are pre8[i + 1] - 1 and pre12[i + 1] - 1
  // (inclusive counts of the prefixes' first occurrences in x); the pm-token
  // prefix entries (kv2_bytes each) hold keys and values of rows 8..11
  const int64_t *src, *pre8, *pre12;
  uint8_t *kv2;
  int64_t kv2_bytes, kv2_total;
  int64_t j0;                       // first pm-token prefix entry held in kv2 (a slice)
  float *plogp2;
  int pm;                           // MID covers positions 8 .. pm - 1, TAIL pm .. pm + 3
  // TREE (pm = q - 1): the masked conditionals, 4 floats per prefix: of MID's
  // row pm per pm-token prefix (lp_mid; MID stores it when set), of row q per
  // q-token prefix (lp_q) and of row q + 1 per (q+1)-token prefix (lp_q1), whose
  // indices for configuration i are preq[i + 1] - 1 and preq1[i + 1] - 1
  float *lp_mid, *lp_q, *lp_q1;
  const int64_t *preq, *preq1;
};

// A buffer store whose per-lane offset is at least the resource's size is
// discarded by the hardware's range check; lanes without an entry store there
// instead of branching around the store (buffers here are at most 2^31 bytes).
constexpr uint32_t kDropOff = 0xC0000000u;
// configuration index bits of a list entry (TREE entries carry flags above)
constexpr int64_t kSrcIndex = (int64_t(1) << 47) - 1;

// Byte offsets inside a prefix entry, layer l (NB blocks of 32 features):
//   key   (block b, head e, position t, lane half h) at kv_key_off + 32 t + 16 h:
//         16 B, the lane's 8 feature slots of head e;
//   value (block b, feature f, lane half h) at kv_val_off + 16 f + 8 h: 8 B,
//         positions 4 h .. 4 h + 3.
// The layer / block / head part is wave-uniform (a scalar offset), the lane
// part a per-lane constant.
template <int NB>
__device__ inline uint32_t kv_key_off(int l, int b, int e) {
  return uint32_t(l * NB * 1024 + b * 512 + e * 256);
}
template <int NB>
__device__ inline uint32_t kv_val_off(int l, int b) {
  return uint32_t(l * NB * 1024 + NB * 512 + b * 512);
}
// pm-token prefix entries (rows 8..11), layer l: key (block b, head e,
// position t < 4, lane half h) at mk_off + 32 t + 16 h, 16 B; value (block b,
// feature f) at mv_off + 8 f, 8 B = positions 0..3.
template <int NB>
__device__ inline uint32_t mk_off(int l, int b, int e) {
  return uint32_t(l * NB * 512 + b * 256 + e * 128);
}
template <int NB>
__device__ inline uint32_t mv_off(int l, int b) {
  return uint32_t(l * NB * 512 + NB * 256 + b * 256);
}

__device__ inline bf16x8 to_bf16(const f32x16 &c, int half) {
  bf16x8 r;
#pragma unroll
  for (int i = 0; i < 8; i += 2) {
    f32x2 p = {c[half * 8 + i], c[half * 8 + i + 1]};
    bf16x2 q = __builtin_convertvector(p, bf16x2);
    r[i] = q[0];
    r[i + 1] = q[1];
  }
  return r;
}

__device__ inline f32x16 mfma(const bf16x8 &a, const bf16x8 &b, const f32x16 &c) {
  return __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, c, 0, 0, 0);
}

__device__ inline f32x16 load16(const float *p) {
  const f32x4 *q = reinterpret_cast<const f32x4 *>(p);
  f32x4 a = q[0], b = q[1], c = q[2], d = q[3];
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

// Sum / max over the two lanes that hold the same row (l and l ^ 32).
__device__ inline float pair_sum(float v) {
  const auto r = __builtin_amdgcn_permlane32_swap(__float_as_uint(v), __float_as_uint(v), false, false);
  return __uint_as_float(r[0]) + __uint_as_float(r[1]);
}
__device__ inline float pair_max(float v) {
  const auto r = __builtin_amdgcn_permlane32_swap(__float_as_uint(v), __float_as_uint(v), false, false);
  return fmaxf(__uint_as_float(r[0]), __uint_as_float(r[1]));
}

__device__ inline float gelu(float x) {
  // 0.5 x (1 + tanh(u)) = x / (1 + exp(-2u)), u = sqrt(2/pi) (x + 0.044715 x^3);
  // hardware exp2 and reciprocal (about 1 ulp each), far below bf16 rounding
  constexpr float c1 = -2.0f * 0.7978845608028654f * 1.4426950408889634f;
  constexpr float c3 = c1 * 0.044715f;
  const float e = __builtin_amdgcn_exp2f(x * fmaf(x * x, c3, c1));
  return x * __builtin_amdgcn_rcpf(1.0f + e);
}

__device__ inline bf16x8 pack8(const float (&v)[8]) {
  bf16x8 r;
#pragma unroll
  for (int i = 0; i < 8; i += 2) {
    f32x2 p = {v[i], v[i + 1]};
    bf16x2 q = __builtin_convertvector(p, bf16x2);
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
// four values as hi (words h[0], h[1]) and lo (l[0], l[1]) bf16 pairs
__device__ inline void pack4_hilo(const float *v, uint32_t (&hw)[2], uint32_t (&lw)[2]) {
#pragma unroll
  for (int i = 0; i < 2; ++i) {
    const f32x2 p = {v[2 * i], v[2 * i + 1]};
    const bf16x2 q = __builtin_convertvector(p, bf16x2);
    const f32x2 d = {v[2 * i] - float(q[0]), v[2 * i + 1] - float(q[1])};
    hw[i] = __builtin_bit_cast(uint32_t, q);
    lw[i] = __builtin_bit_cast(uint32_t, __builtin_convertvector(d, bf16x2));
  }
}
// m ? b : a, bitwise (one v_bfi_b32; keeps a lane-dependent choice between
// vector elements from becoming a dynamically indexed vector)
__device__ inline float bsel(float a, float b, uint32_t m) {
  return __uint_as_float((__float_as_uint(b) & m) | (__float_as_uint(a) & ~m));
}
// the bf16 rounding error of to_bf16(c, half) == hi, as bf16
__device__ inline bf16x8 lo_bf16(const f32x16 &c, int half, const bf16x8 &hi) {
  float r[8];
#pragma unroll
  for (int i = 0; i < 8; ++i) r[i] = c[half * 8 + i] - float(hi[i]);
  return pack8(r);
}

// 16 consecutive floats from LDS
__device__ inline f32x16 lds16(const float *p) {
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

// Layer norm of the feature-major residual into a bf16 operand; gain and shift
// are permuted vectors in LDS at V + g_off / V + b_off (V includes the lane
// half's offset), 32 floats per accumulator block.
template <int NB>
__device__ inline void layer_norm(const f32x16 (&res)[NB], const float *V, int g_off, int b_off,
                                  bf16x8 (&X)[2 * NB]) {
  float s = 0.f, s2 = 0.f;
#pragma unroll
  for (int q = 0; q < NB; ++q)
#pragma unroll
    for (int j = 0; j < 16; ++j) {
      s += res[q][j];
      s2 = fmaf(res[q][j], res[q][j], s2);
    }
  s = pair_sum(s);
  s2 = pair_sum(s2);
  const float mu = s * (1.0f / (32 * NB));
  const float rs = rsqrtf(fmaxf(s2 * (1.0f / (32 * NB)) - mu * mu, 0.f) + 1e-5f);
#pragma unroll
  for (int q = 0; q < NB; ++q) {
    const f32x16 gg = lds16(V + g_off + q * 32), bb = lds16(V + b_off + q * 32);
    f32x16 y;
#pragma unroll
    for (int j = 0; j < 16; ++j) y[j] = fmaf((res[q][j] - mu) * rs, gg[j], bb[j]);
    X[2 * q] = to_bf16(y, 0);
    X[2 * q + 1] = to_bf16(y, 1);
  }
}

// The weight stream of one layer is a fixed sequence of steps of KS fragments
// each: for every head pair b the Q, K, V and output-projection fragments, then
// for every hidden block fb the two feed-forward fragments.  The next step is
// always loaded while the current one is multiplied.
// Every layer occupies the same-sized slice of the packed buffers, so all
// offsets inside a layer are compile-time constants (in bf16x8 entries, 64 per
// fragment, and in floats for the permuted vectors).
template <int D>
struct Shape {
  static constexpr int NB = D / 32, KS = D / 16, F = 4 * D, FB = F / 32, FKS = F / 16;
  static constexpr int STEPS = 4 * NB + 2 * FB;
  static constexpr int64_t OQ = 0, OK = int64_t(NB) * KS * 64, OV = 2 * OK, OO = 3 * OK,
                           OW1 = 4 * OK, OW2 = OW1 + int64_t(FB) * KS * 64,
                           FRAG_L = OW2 + int64_t(NB) * FKS * 64,
                           LAYER = NP * FRAG_L;   // hi set, then lo set (FRAG_L further)
  // sub-steps: step s of the stream contributes one per fragment set it uses
  static constexpr int np_of(int s) {
    return s < 4 * NB ? NP_ATT : ((s - 4 * NB) % 2 == 0 ? NP_W1 : NP_W2);
  }
  static constexpr int first_sub(int s) {      // index of step s's first sub-step
    return s <= 4 * NB ? s * NP_ATT
                       : 4 * NB * NP_ATT + ((s - 4 * NB) / 2) * (NP_W1 + NP_W2) +
                             ((s - 4 * NB) % 2 ? NP_W1 : 0);
  }
  static constexpr int USTEPS = first_sub(STEPS);  // sub-steps of the weight stream per layer
  static constexpr int step_of(int u) {        // the step of sub-step u, and its set
    return u < 4 * NB * NP_ATT ? u / NP_ATT
         : 4 * NB + 2 * ((u - 4 * NB * NP_ATT) / (NP_W1 + NP_W2)) +
               ((u - 4 * NB * NP_ATT) % (NP_W1 + NP_W2) < NP_W1 ? 0 : 1);
  }
  static constexpr int set_of(int u) { return u - first_sub(step_of(u)); }
  // Feed-forward steps in stream order j = step - 4 NB: W1(0), W1(1), then
  // W1(fb + 1), W2(fb - 1) for fb = 1 .. FB - 2, then W2(FB - 2), W2(FB - 1)
  // (the kernel evaluates the GELU of block fb between those two products).
  static constexpr bool ffn_is_w1(int j) { return j < 2 || (j < 2 * FB - 2 && j % 2 == 0); }
  static constexpr int ffn_block(int j) {
    return j < 2 ? j : j >= 2 * FB - 2 ? j - FB : (j % 2 == 0 ? j / 2 + 1 : j / 2 - 1);
  }
  static constexpr int64_t VLN1G = 0, VLN1B = D, VBQ = 2 * D, VBK = 3 * D, VBV = 4 * D,
                           VBO = 5 * D, VLN2G = 6 * D, VLN2B = 7 * D, VB1 = 8 * D,
                           VB2 = 8 * D + F, VEC_L = 9 * D + F;
};

// Per-layer weight slices are read through buffer resources: the layer's base
// goes into the resource, the lane's part of the address into a VGPR and the
// compile-time offset into the scalar offset, so no 64-bit addresses stay live.
typedef __attribute__((ext_vector_type(4))) int i32x4;
// The four waves of a block stream the same weight fragments.  Each step is
// loaded once per block into a ring of three LDS slots (one step, KS
// fragments of 1 KiB, each): wave w loads fragments w, w + 4, ... of the step
// after next into registers, stores the next step's share into its slot, and
// a block barrier publishes it.  The MFMAs read their fragments from LDS.
//
// The wave-dependent part of a fragment's address depends only on the kind
// of step, so it sits in three per-lane offsets (voff[kind]); the rest is a
// compile-time constant of (step, j).
struct StageOff {
  uint32_t v[3];   // bytes: lane * 16 + wave part for Q/K/V/W1, output projection, W2
};
template <int D>
__device__ inline StageOff stage_offsets(int lane, int wv) {
  using S = Shape<D>;
  const uint32_t l = uint32_t(lane) * 16u;
  return {{l + uint32_t(wv) * 1024u, l + uint32_t((wv / 2) * S::KS + wv % 2) * 1024u,
           l + uint32_t((wv / 2) * S::FKS + wv % 2) * 1024u}};
}
// Sub-step u of a layer's stream is step S::step_of(u) of the fragment set
// S::set_of(u).
template <int D>
__device__ inline void stage_load(bf16x8 (&st)[Shape<D>::KS / 4], __amdgpu_buffer_rsrc_t W,
                                  const StageOff &vo, int u) {
  using S = Shape<D>;
  constexpr int KS = S::KS;
  const int s = S::step_of(u);
  const int64_t set_off = int64_t(S::set_of(u)) * S::FRAG_L;
#pragma unroll
  for (int j = 0; j < KS / 4; ++j) {
    int kind;
    int64_t off;   // fragment f = wv + 4 j without the wave part
    if (s < 4 * S::NB) {
      const int b = s / 4;
      kind = s % 4 == 3 ? 1 : 0;
      off = s % 4 == 3 ? S::OO + (int64_t(2 * b) + int64_t(2 * j) * KS) * 64
          : (s % 4 == 0 ? S::OQ : s % 4 == 1 ? S::OK : S::OV) + int64_t(b) * KS * 64 + int64_t(4 * j) * 64;
    } else {
      const int fb = S::ffn_block(s - 4 * S::NB);
      const bool w1 = S::ffn_is_w1(s - 4 * S::NB);
      kind = w1 ? 0 : 2;
      off = w1 ? S::OW1 + int64_t(fb) * KS * 64 + int64_t(4 * j) * 64
               : S::OW2 + (int64_t(2 * fb) + int64_t(2 * j) * S::FKS) * 64;
    }
    const uint32_t voff = kind == 0 ? vo.v[0] : kind == 1 ? vo.v[1] : vo.v[2];
    st[j] = __builtin_bit_cast(
        bf16x8, __builtin_amdgcn_raw_buffer_load_b128(W, voff, uint32_t((off + set_off) * 16), 0));
  }
}
template <int D>
__device__ inline void stage_store(bf16x8 *slot, const bf16x8 (&st)[Shape<D>::KS / 4], int wv,
                                   int lane) {
#pragma unroll
  for (int j = 0; j < Shape<D>::KS / 4; ++j) slot[(wv + 4 * j) * 64 + lane] = st[j];
}
// fragments half * KS/2 .. half * KS/2 + KS/2 - 1 of the step in `slot`
template <int D>
__device__ inline void fetch_half(bf16x8 (&f)[Shape<D>::KS / 2], const bf16x8 *slot, int half,
                                  int lane) {
#pragma unroll
  for (int ii = 0; ii < Shape<D>::KS / 2; ++ii) f[ii] = slot[(half * (Shape<D>::KS / 2) + ii) * 64 + lane];
}

// One half step of the pipelined feed-forward block: the HS MFMAs of fragment
// half h of a W1 step (into Hn) or of a W2 step (into res, operand Hp0 / Hp1),
// each followed by PER / HS of the GELU values G0 .. G0 + PER - 1 of Hc.
template <int D, bool W1, int PER, int G0>
__device__ inline void ffn_half(const bf16x8 (&f)[Shape<D>::KS / 2], int h,
                                const bf16x8 (&X)[Shape<D>::KS], f32x16 &Hn,
                                f32x16 (&res)[Shape<D>::NB], const bf16x8 &Hp0,
                                const bf16x8 &Hp1, f32x16 &Hc) {
  constexpr int HS = Shape<D>::KS / 2, PM = PER / HS;
  static_assert(PER % HS == 0, "GELU values per MFMA");
#pragma unroll
  for (int i = 0; i < HS; ++i) {
    if (W1) {
      Hn = mfma(f[i], X[h * HS + i], Hn);
    } else {
      const int fi = h * HS + i;               // W2 fragment 2q + e
      res[fi / 2] = mfma(f[i], (fi % 2) ? Hp1 : Hp0, res[fi / 2]);
    }
#pragma unroll
    for (int k = 0; k < PM; ++k) Hc[G0 + i * PM + k] = gelu(Hc[G0 + i * PM + k]);
  }
}

template <int D, int MODE>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2, 2)))
fused_kernel(FusedArgs a) {
  using S = Shape<D>;
  constexpr int NB = S::NB, KS = S::KS, FB = S::FB, STEPS = S::STEPS;
  constexpr int R = Rows<MODE>::R, CPT = Rows<MODE>::CPT, P0 = Rows<MODE>::P0;
  const int lane = threadIdx.x % 64, h = lane / 32, r = lane % 32;
  // The permuted fp32 vectors (biases, layer-norm parameters, head, embeddings)
  // are read by every lane at the same few addresses; they are staged in LDS
  // once per block so that the vector memory path carries only the weights.
  extern __shared__ f32x4 s_vec4[];
  {
    const f32x4 *src = reinterpret_cast<const f32x4 *>(a.vec);
    for (int i = int(threadIdx.x); i < a.lds_floats / 4; i += int(blockDim.x)) s_vec4[i] = src[i];
    __syncthreads();
  }
  const float *svec = reinterpret_cast<const float *>(s_vec4);
  bf16x8 *ring = reinterpret_cast<bf16x8 *>(s_vec4 + a.lds_floats / 4);
  constexpr int RS = KS * 64;        // one ring slot, in bf16x8 entries
  // wave of the block, explicitly wave-uniform so the loops stay scalar
  const int wv = __builtin_amdgcn_readfirstlane(int(threadIdx.x / 64));
  // a persistent launch reads the number of configurations from the device;
  // with passes = 0 it also sizes its chunks from it: the fewest passes that
  // spread the count over the grid's blocks
  const int64_t B = a.count ? (*a.count < a.B ? *a.count : a.B) : a.B;
  int passes = a.passes;
  if (passes == 0) {
    const int64_t per = int64_t(4 * CPT) * gridDim.x;
    const int64_t want = (B + per - 1) / per;
    passes = want < 1 ? 1 : want > Rows<MODE>::MAXP ? Rows<MODE>::MAXP : int(want);
  }
  // All four waves of a block take part in every barrier of the weight
  // stream, so the loops are uniform over the block: a block owns chunks of
  // 4 x CPT x passes configurations (wave w the w-th quarter) and a wave whose
  // configurations run out computes on empty rows and writes nothing.
  const int64_t block_cfgs = int64_t(4 * CPT) * passes;
  // Blocks are dispatched to the chip's 8 XCDs in turn (block i on XCD i % 8),
  // each with its own L2.  When the grid has one chunk per block, the chunks
  // of one XCD are made contiguous (neighbouring configurations share a
  // prefix's keys and values), a bijection of the block indices.
  int64_t bc0 = blockIdx.x;
  {
    const int64_t G = gridDim.x;
    if (G * block_cfgs >= B && G >= 8) {
      const int64_t xcd = bc0 % 8, k = bc0 / 8, q = G / 8, rem = G % 8;
      bc0 = xcd * q + (xcd < rem ? xcd : rem) + k;
    }
  }
  if (bc0 * block_cfgs >= B) return;
  const int c = r / R;               // configuration of this lane's row within the pass
  // position of this lane's row (TREE: per slot, below)
  const int t_lane = MODE == TAIL ? a.pm + r % R : P0 + r % R;
  const int n = a.n;
  const bf16x8 *pk = a.pk + lane;
  const float *vec = a.vec;

  // Score slot j (0..15) of a lane holds key row (j/4)*8 + h*4 + j%4 of the
  // 32-row tile.  The lane's own configuration owns slots 8c..8c+7 (PLAIN),
  // 4c..4c+3 (TRUNK / SUFFIX), all 16 (WIDE), or, with R = 4, slots
  // 4(c/2)..4(c/2)+3 of the lane half h = c % 2 only; the masks select them.
  const uint32_t upmask = c & 1 ? 0xFFFFFFFFu : 0u;    // PLAIN: second configuration
  const uint32_t m_c1 = c & 2 ? 0xFFFFFFFFu : 0u;      // R = 8: configurations 2, 3
  const uint32_t m_c2 = c & 4 ? 0xFFFFFFFFu : 0u;      // R = 4: configurations 4..7
  // R = 8: word w of the probability operand of k-step s holds this lane's
  // configuration's keys iff s = c / 2 and w / 2 = c % 2
  const uint32_t m_s0 = ~m_c1, m_w0 = ~upmask;
  // R = 4: this lane half holds the configuration's own keys (key rows 4c..4c+3)
  const bool own_half = R == 4 && h == (c & 1);
  const uint32_t m_half = own_half ? 0xFFFFFFFFu : 0u;
  // causal mask of the lane's own key slots (the same in every head and layer)
  constexpr int NM = R == 16 ? 8 : R == 8 || R == 4 ? 4 : 16;
  float madd[NM];
#pragma unroll
  for (int i = 0; i < NM; ++i) {
    const int kp = R == 4 ? i : R == 8 ? h * 4 + i : (i / 4) * 8 + h * 4 + (i % 4);   // key position - P0
    madd[i] = kp <= r % R && (R != 4 || own_half) ? 0.f : -INFINITY;   // (TREE: per slot)
  }
  // TAIL: the middle level's keys (positions 8 + i, those below pm; TREE: up to pm)
  float madd_mid[4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
    madd_mid[i] = own_half && 8 + i < a.pm + (MODE == TREE) ? 0.f : -INFINITY;
  // prefix entries (TRUNK .. TAIL), read and written through buffer resources
  const __amdgpu_buffer_rsrc_t kvr =
      __builtin_amdgcn_make_buffer_rsrc(a.kv, 0, int(uint32_t(a.kv_total)), 0x00020000);
  const __amdgpu_buffer_rsrc_t kv2r =
      __builtin_amdgcn_make_buffer_rsrc(a.kv2, 0, int(uint32_t(a.kv2_total)), 0x00020000);
  const uint32_t kv_key_lane = uint32_t((r % 8) * 32 + h * 16);
  const uint32_t kv_val_lane = uint32_t(r * 16 + h * 8);
  const uint32_t mk_lane = uint32_t((r % 4) * 32 + h * 16);
  const uint32_t mv_lane = uint32_t(r * 8);

  constexpr uint32_t kFragBytes = uint32_t(S::LAYER * 16);
  auto wres = [&](int l) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<bf16x8 *>(a.pk + int64_t(l) * S::LAYER),
                                             0, int(kFragBytes), 0x00020000);
  };
  const StageOff vo = stage_offsets<D>(lane, wv);
  constexpr int HS = KS / 2;
  constexpr int US = S::USTEPS;
  bf16x8 fr[2][HS];
  bf16x8 staged[KS / 4];
  int cur = 0;                       // ring slot of the current sub-step
  // prologue: sub-step 0 of layer 0 into slot 0, sub-step 1 in flight
  stage_load<D>(staged, wres(0), vo, 0);
  stage_store<D>(ring, staged, wv, lane);
  stage_load<D>(staged, wres(0), vo, 1);
  __syncthreads();
  fetch_half<D>(fr[0], ring, 0, lane);
  // end of sub-step u: publish sub-step u + 1, start loading sub-step u + 2
  // (layer Wsrc, index u_load), make sub-step u + 1 current
  auto advance = [&](__amdgpu_buffer_rsrc_t Wsrc, int u_load) {
    const int nxt = cur == 2 ? 0 : cur + 1;
    stage_store<D>(ring + nxt * RS, staged, wv, lane);
    stage_load<D>(staged, Wsrc, vo, u_load);
    __syncthreads();
    cur = nxt;
  };

  // block chunks strided over the grid
  for (int64_t bc = bc0; bc * block_cfgs < B; bc += gridDim.x) {
  const int64_t c_base = bc * block_cfgs + int64_t(wv) * CPT * passes;
  for (int pass = 0; pass < passes; ++pass) {
    if constexpr (MODE == PHASE) break;             // no transformer rows
    const int64_t cfg0 = c_base + CPT * pass;
    if (bc * block_cfgs + CPT * pass >= B) break;   // uniform over the block
    // MID / TAIL: item cfg0 + c stands for configuration src (-1: padding);
    // TREE: row r % 4 of slot cfg0 + c for src (bits 48.. of the entry: the
    // slot row of its parent, itself for a q-token prefix; bit 47: a repeated
    // q-token prefix, whose conditional its first slot stores), its row 0 for
    // src0.  Padding entries are -1, decoded before any masking.
    constexpr int ST = MODE == TREE ? 4 : 1;        // list entries per item
    auto index_of = [](int64_t e) { return e >= 0 ? e & kSrcIndex : int64_t(-1); };
    const int64_t raw0 = Rows<MODE>::LISTED ? (cfg0 + c < B ? a.src[ST * (cfg0 + c)] : -1) : cfg0 + c;
    const int64_t src0 = Rows<MODE>::LISTED ? index_of(raw0) : raw0;
    const int64_t raw = MODE == TREE ? (cfg0 + c < B ? a.src[ST * (cfg0 + c) + r % 4] : -1) : raw0;
    const int64_t src = Rows<MODE>::LISTED ? index_of(raw) : raw;
    const int parent = MODE == TREE && raw >= 0 ? int(raw >> 48) : r % R;
    const bool repeat = MODE == TREE && raw >= 0 && ((raw >> 47) & 1);
    const int64_t cfg = Rows<MODE>::LISTED ? src : cfg0 + c;
    const bool live = Rows<MODE>::LISTED ? src >= 0 : cfg < B;
    const uint64_t x = live ? a.x[cfg] : 0ull;
    // TREE: a q-token prefix at position q = pm + 1 sees itself, an extension
    // at q + 1 its parent's row and itself
    const int t = MODE == TREE ? a.pm + 1 + (parent != r % R) : t_lane;
    if constexpr (MODE == TREE) {
#pragma unroll
      for (int i = 0; i < 4; ++i) madd[i] = (i == r % R || i == parent) && own_half ? 0.f : -INFINITY;
    }
    // prefix entries: of this lane's configuration (keys, log-probability) and
    // of the pass's four configurations (values)
    // (byte offsets in a.kv, below 2^31)
    uint32_t kv_cfg[4] = {0u, 0u, 0u, 0u};
    int64_t ent_own = 0;
    uint32_t kv_own = 0;
    if constexpr (MODE == TRUNK || MODE == SUFFIX) {
      int64_t ent[4];
#pragma unroll
      for (int cc = 0; cc < 4; ++cc) {
        int64_t e = cfg0 + cc;                  // TRUNK: entry = index in the prefix list
        if (MODE == SUFFIX) e = a.slot[(e < B ? a.x[e] : 0ull) & 0xFFFFull];
        else if (e >= B) e = 0;                 // never written (see the stores)
        ent[cc] = e;
        kv_cfg[cc] = uint32_t(e * a.kv_bytes);
      }
      ent_own = c == 0 ? ent[0] : c == 1 ? ent[1] : c == 2 ? ent[2] : ent[3];
      kv_own = uint32_t(ent_own * a.kv_bytes);
    }
    // MID / TAIL / TREE: the pass's items come from at most two 8-token
    // prefixes, a (its first item, never padding) and b (its last live item);
    // ent8 is the lane's own, m_b8 set when that is b.  The lane's pm-token
    // prefix entry, and TAIL's value sources: the entries of configurations
    // 4s + h (slots 0..3) and 4s + 2 + h (4..7) (the pass's eight entries are
    // wave-uniform: scalar registers; a lane picks its two with h)
    int64_t ent8 = 0, ent12 = 0;
    uint32_t kv8_off = 0, kv8b_off = 0, m_b8 = 0u;
    uint32_t mid_own = 0, mid_e[8] = {0u, 0u, 0u, 0u, 0u, 0u, 0u, 0u};
    uint32_t mid_live = 0;             // bit k: item k of the pass is not padding
    if constexpr (Rows<MODE>::LISTED) {
      // (waves past the end of the items read nothing and store nothing)
      // (row 0 of a TREE slot is a q-token prefix: its parent bits are zero)
      const int64_t s8 = cfg0 < B ? index_of(a.src[ST * cfg0]) : -1;
      const int64_t e8a = s8 >= 0 ? a.pre8[s8 + 1] - 1 : 0;
      ent12 = src0 >= 0 ? a.pre12[src0 + 1] - 1 : a.j0;
      mid_own = uint32_t((ent12 - a.j0) * a.kv2_bytes);
      int64_t s8b = -1;
#pragma unroll
      for (int k = 0; k < 8; ++k) {
        const int64_t it = cfg0 + k;
        const int64_t sc = it < B ? index_of(a.src[ST * it]) : -1;
        mid_live |= sc >= 0 ? (1u << k) : 0u;
        mid_e[k] = uint32_t((sc >= 0 ? a.pre12[sc + 1] - 1 - a.j0 : 0) * a.kv2_bytes);
        s8b = sc >= 0 ? sc : s8b;
      }
      const int64_t e8b = s8b >= 0 ? a.pre8[s8b + 1] - 1 : e8a;
      kv8_off = uint32_t(e8a * a.kv_bytes);
      kv8b_off = uint32_t(e8b * a.kv_bytes);
      ent8 = src0 >= 0 ? a.pre8[src0 + 1] - 1 : e8a;
      m_b8 = ent8 != e8a ? 0xFFFFFFFFu : 0u;
    }
    // entry of item 4s + 2k + h (the values of slots 4k .. 4k+3 of k-step s)
    auto mid_v = [&](int s2, int k2) { return h ? mid_e[4 * s2 + 2 * k2 + 1] : mid_e[4 * s2 + 2 * k2]; };
    auto mid_ok = [&](int s2, int k2) { return ((mid_live >> (4 * s2 + 2 * k2 + h)) & 1u) != 0u; };

    // embedding: token of the previous position (BOS at position 0)
    f32x16 res[NB];
    {
      const int in = (t == 0) ? 4 : int((x >> (2 * (t - 1))) & 3ull);
      const bool pad = t >= n;
#pragma unroll
      for (int q = 0; q < NB; ++q) {
        const f32x16 te = lds16(svec + a.tok + in * D + (q * 2 + h) * 16);
        const f32x16 pe = pad ? f32x16{} : lds16(svec + a.pos + t * D + (q * 2 + h) * 16);
        res[q] = te + pe;
      }
    }

    for (int l = 0; l < a.L; ++l) {
      const __amdgpu_buffer_rsrc_t W = wres(l), Wn = wres(l + 1 < a.L ? l + 1 : 0);
      // start loading sub-step u_load of this layer, or of the next one
      auto adv = [&](int u_load) {
        if (u_load < US)
          advance(W, u_load);
        else
          advance(Wn, u_load - US);
      };
      // permuted vectors of the layer (LDS): lane-half h reads 16 floats at (2q+h)*16
      const float *lv = svec + l * int(S::VEC_L);
      const float *V16 = lv + h * 16;
      bf16x8 X[KS];
      // The weight stream advances in half sub-steps of HS fragments through
      // the two buffers fr[0] / fr[1]: while one half is multiplied the next
      // half is read from the LDS ring.  On entry fr[0] holds half 0 of
      // sub-step 0 of this layer and the ring's current slot holds it.
      // Sub-step NP s + p of step s multiplies the fragment set p (hi, lo) of
      // that step's weights.
      // ---- attention block
      layer_norm<NB>(res, V16, int(S::VLN1G), int(S::VLN1B), X);
#pragma unroll
      for (int q = 0; q < NB; ++q) res[q] += lds16(V16 + S::VBO + q * 32);
#pragma unroll
      for (int b = 0; b < NB; ++b) {
        // SUFFIX: the prefix's keys and values of block b, read while Q, K and
        // V are computed.  As MFMA operands: key row r = (configuration r / 8,
        // position r % 8) with this lane half's 8 feature slots of head e; value
        // feature r with key slots 16 s + (i/4)*8 + 4h + i%4, i.e. positions
        // 4h .. 4h+3 of configurations 2s (slots 0..3) and 2s + 1 (slots 4..7).
        bf16x8 Kk[2], Vk[2];
        if constexpr (MODE == SUFFIX) {
#pragma unroll
          for (int e = 0; e < 2; ++e)
            Kk[e] = __builtin_bit_cast(
                bf16x8, __builtin_amdgcn_raw_buffer_load_b128(kvr, kv_own + kv_key_lane,
                                                              kv_key_off<NB>(l, b, e), 0));
#pragma unroll
          for (int s = 0; s < 2; ++s) {
            const i32x2 v0 = __builtin_bit_cast(
                i32x2, __builtin_amdgcn_raw_buffer_load_b64(kvr, kv_val_lane,
                                                            kv_cfg[2 * s] + kv_val_off<NB>(l, b), 0));
            const i32x2 v1 = __builtin_bit_cast(
                i32x2, __builtin_amdgcn_raw_buffer_load_b64(kvr, kv_val_lane,
                                                            kv_cfg[2 * s + 1] + kv_val_off<NB>(l, b), 0));
            const i32x4 w = {v0[0], v0[1], v1[0], v1[1]};
            Vk[s] = __builtin_bit_cast(bf16x8, w);
          }
        }
        // MID / TAIL: the 8-token prefixes' keys (key row r = position r % 8
        // of prefix a, of prefix b for rows 8..15; rows 16..31 repeat a and are
        // never selected) and values (k-step 0: slots 0..3 = positions
        // 4h .. 4h+3 of a, slots 4..7 those of b); TAIL also the
        // middle level's keys (key row r = configuration r / 4, position r % 4)
        // and values (as the own values: slots 0..3 of k-step s from
        // configuration 4s + h, slots 4..7 from 4s + 2 + h), all read while Q,
        // K and V are computed
        bf16x8 Vt, Vm[2], Kt[2], Km[2];
        if constexpr (Rows<MODE>::LISTED) {
#pragma unroll
          for (int e = 0; e < 2; ++e)
            Kt[e] = __builtin_bit_cast(
                bf16x8, __builtin_amdgcn_raw_buffer_load_b128(kvr, ((r >> 3) == 1 ? kv8b_off : kv8_off) + kv_key_lane,
                                                              kv_key_off<NB>(l, b, e), 0));
        }
        if constexpr (Rows<MODE>::TAILS) {
#pragma unroll
          for (int e = 0; e < 2; ++e)
            Km[e] = __builtin_bit_cast(
                bf16x8, __builtin_amdgcn_raw_buffer_load_b128(kv2r, mid_own + mk_lane,
                                                              mk_off<NB>(l, b, e), 0));
        }
        if constexpr (Rows<MODE>::LISTED) {
          const i32x2 v = __builtin_bit_cast(
              i32x2, __builtin_amdgcn_raw_buffer_load_b64(kvr, kv8_off + kv_val_lane,
                                                          kv_val_off<NB>(l, b), 0));
          const i32x2 vb = __builtin_bit_cast(
              i32x2, __builtin_amdgcn_raw_buffer_load_b64(kvr, kv8b_off + kv_val_lane,
                                                          kv_val_off<NB>(l, b), 0));
          Vt = __builtin_bit_cast(bf16x8, i32x4{v[0], v[1], vb[0], vb[1]});
        }
        if constexpr (Rows<MODE>::TAILS) {
#pragma unroll
          for (int s = 0; s < 2; ++s) {
            const i32x2 v0 = __builtin_bit_cast(
                i32x2, __builtin_amdgcn_raw_buffer_load_b64(kv2r, mid_v(s, 0) + mv_lane,
                                                            mv_off<NB>(l, b), 0));
            const i32x2 v1 = __builtin_bit_cast(
                i32x2, __builtin_amdgcn_raw_buffer_load_b64(kv2r, mid_v(s, 1) + mv_lane,
                                                            mv_off<NB>(l, b), 0));
            Vm[s] = __builtin_bit_cast(bf16x8, i32x4{v0[0], v0[1], v1[0], v1[1]});
          }
        }
        // steps 4b (Q), 4b+1 (K), 4b+2 (V), 4b+3 (O)
        f32x16 Qc = lds16(V16 + S::VBQ + b * 32);
#pragma unroll
        for (int pt = 0; pt < NP_ATT; ++pt) {
          fetch_half<D>(fr[1], ring + cur * RS, 1, lane);
#pragma unroll
          for (int i = 0; i < HS; ++i) Qc = mfma(fr[0][i], X[i], Qc);
          adv(S::first_sub(4 * b) + pt + 2);
          fetch_half<D>(fr[0], ring + cur * RS, 0, lane);
#pragma unroll
          for (int i = 0; i < HS; ++i) Qc = mfma(fr[1][i], X[HS + i], Qc);
        }
        f32x16 Kc = lds16(V16 + S::VBK + b * 32);
#pragma unroll
        for (int pt = 0; pt < NP_ATT; ++pt) {
          fetch_half<D>(fr[1], ring + cur * RS, 1, lane);
#pragma unroll
          for (int i = 0; i < HS; ++i) Kc = mfma(fr[0][i], X[i], Kc);
          adv(S::first_sub(4 * b + 1) + pt + 2);
          fetch_half<D>(fr[0], ring + cur * RS, 0, lane);
#pragma unroll
          for (int i = 0; i < HS; ++i) Kc = mfma(fr[1][i], X[HS + i], Kc);
        }
        f32x16 Vc;
        const float bvv = lv[S::VBV + 32 * b + r];
#pragma unroll
        for (int j = 0; j < 16; ++j) Vc[j] = bvv;
#pragma unroll
        for (int pt = 0; pt < NP_ATT; ++pt) {
          fetch_half<D>(fr[1], ring + cur * RS, 1, lane);
#pragma unroll
          for (int i = 0; i < HS; ++i) Vc = mfma(X[i], fr[0][i], Vc);
          adv(S::first_sub(4 * b + 2) + pt + 2);
          fetch_half<D>(fr[0], ring + cur * RS, 0, lane);
#pragma unroll
          for (int i = 0; i < HS; ++i) Vc = mfma(X[HS + i], fr[1][i], Vc);
        }
        fetch_half<D>(fr[1], ring + cur * RS, 1, lane);
        const bf16x8 V0 = to_bf16(Vc, 0), V1 = to_bf16(Vc, 1);
        if constexpr (MODE == TRUNK) {
          // keep this block's values for the suffixes: slots 0..3 / 4..7 of
          // k-step s are configurations 2s / 2s + 1
#pragma unroll
          for (int s = 0; s < 2; ++s) {
            const i32x4 w = __builtin_bit_cast(i32x4, s == 0 ? V0 : V1);
            __builtin_amdgcn_raw_buffer_store_b64(i32x2{w[0], w[1]}, kvr,
                                                  cfg0 + 2 * s < B ? kv_val_lane : kDropOff,
                                                  kv_cfg[2 * s] + kv_val_off<NB>(l, b), 0);
            __builtin_amdgcn_raw_buffer_store_b64(i32x2{w[2], w[3]}, kvr,
                                                  cfg0 + 2 * s + 1 < B ? kv_val_lane : kDropOff,
                                                  kv_cfg[2 * s + 1] + kv_val_off<NB>(l, b), 0);
          }
        }
        if constexpr (MODE == MID) {
          // keep this block's values for the configurations: slots 0..3 / 4..7
          // of k-step s are positions 0..3 of items 4s + h / 4s + 2 + h
#pragma unroll
          for (int s = 0; s < 2; ++s) {
            const i32x4 w = __builtin_bit_cast(i32x4, s == 0 ? V0 : V1);
#pragma unroll
            for (int k2 = 0; k2 < 2; ++k2)
              __builtin_amdgcn_raw_buffer_store_b64(i32x2{w[2 * k2], w[2 * k2 + 1]}, kv2r,
                                                    mid_ok(s, k2) ? mid_v(s, k2) + mv_lane : kDropOff,
                                                    mv_off<NB>(l, b), 0);
          }
        }
        f32x16 O;
#pragma unroll
        for (int e = 0; e < 2; ++e) {
          // S[j] = score(key (j/4)*8 + h*4 + j%4, query r)
          const bf16x8 Qe = to_bf16(Qc, e), Ke = to_bf16(Kc, e);
          if constexpr (MODE == TRUNK)
            __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(i32x4, Ke), kvr,
                                                   live ? kv_own + kv_key_lane : kDropOff,
                                                   kv_key_off<NB>(l, b, e), 0);
          if constexpr (MODE == MID)
            __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(i32x4, Ke), kv2r,
                                                   live ? mid_own + mk_lane : kDropOff,
                                                   mk_off<NB>(l, b, e), 0);
          const f32x16 Sc = mfma(Ke, Qe, f32x16{});
          constexpr int NO = R == 4 ? 4 : R / 2;       // own keys per lane
          // prefix keys per lane: SUFFIX 4 of the 8-token prefix; MID those 4;
          // TAIL also 4 of the middle level
          constexpr int NK = MODE == SUFFIX || MODE == MID ? 4 : Rows<MODE>::TAILS ? 8 : 0;
          float p[NO + NK];
          float mx = -INFINITY;
          constexpr float kScale = 0.25f * 1.4426950408889634f;   // 1/sqrt(16), base 2
#pragma unroll
          for (int i = 0; i < NO; ++i) {
            float s;
            if constexpr (R == 32) s = Sc[i];
            else if constexpr (R == 16) s = bsel(Sc[i], Sc[8 + i], upmask);
            else if constexpr (R == 8)
              s = bsel(bsel(Sc[i], Sc[4 + i], upmask), bsel(Sc[8 + i], Sc[12 + i], upmask), m_c1);
            else   // R = 4: slot group c / 2
              s = bsel(bsel(Sc[i], Sc[4 + i], m_c1), bsel(Sc[8 + i], Sc[12 + i], m_c1), m_c2);
            p[i] = fmaf(s, kScale, madd[i]);
            mx = fmaxf(mx, p[i]);
          }
          if constexpr (MODE == SUFFIX) {
            const f32x16 Sk = mfma(Kk[e], Qe, f32x16{});
#pragma unroll
            for (int i = 0; i < NK; ++i) {
              const float s = bsel(bsel(Sk[i], Sk[4 + i], upmask), bsel(Sk[8 + i], Sk[12 + i], upmask), m_c1);
              p[NO + i] = s * kScale;
              mx = fmaxf(mx, p[NO + i]);
            }
          }
          if constexpr (Rows<MODE>::LISTED) {
            __builtin_amdgcn_sched_barrier(0);
            // the 8-token prefix's keys of this lane half: positions 4h + i in slots 0..3
            const f32x16 St = mfma(Kt[e], Qe, f32x16{});
#pragma unroll
            for (int i = 0; i < 4; ++i) {
              p[NO + i] = bsel(St[i], St[4 + i], m_b8) * kScale;
              mx = fmaxf(mx, p[NO + i]);
            }
          }
          if constexpr (Rows<MODE>::TAILS) {
            __builtin_amdgcn_sched_barrier(0);
            const f32x16 Sm = mfma(Km[e], Qe, f32x16{});
#pragma unroll
            for (int i = 0; i < 4; ++i) {
              const float s = bsel(bsel(Sm[i], Sm[4 + i], m_c1), bsel(Sm[8 + i], Sm[12 + i], m_c1), m_c2);
              p[NO + 4 + i] = fmaf(s, kScale, madd_mid[i]);
              mx = fmaxf(mx, p[NO + 4 + i]);
            }
          }
          mx = pair_max(mx);
          float sum = 0.f;
#pragma unroll
          for (int i = 0; i < NO + NK; ++i) {
            p[i] = __builtin_amdgcn_exp2f(p[i] - mx);
            sum += p[i];
          }
          const float inv = __builtin_amdgcn_rcpf(pair_sum(sum));
#pragma unroll
          for (int i = 0; i < NO + NK; ++i) p[i] *= inv;
          // O^T = V^T P^T with P as hi + lo
          f32x16 Oe;
          if constexpr (R == 32) {
            float q0[8], q1[8];
#pragma unroll
            for (int i = 0; i < 8; ++i) {
              q0[i] = p[i];
              q1[i] = p[8 + i];
            }
            bf16x8 h0, l0, h1, l1;
            pack8_hilo(q0, h0, l0);
            pack8_hilo(q1, h1, l1);
            Oe = mfma(V0, h0, f32x16{});
            Oe = mfma(V1, h1, Oe);
            Oe = mfma(V0, l0, Oe);
            Oe = mfma(V1, l1, Oe);
          } else if constexpr (R == 16) {
            // each split into the lower / upper configuration's keys
            float q[8];
#pragma unroll
            for (int i = 0; i < 8; ++i) q[i] = p[i];
            bf16x8 ph8, pl8;
            pack8_hilo(q, ph8, pl8);
            const i32x4 pp = __builtin_bit_cast(i32x4, ph8), ql = __builtin_bit_cast(i32x4, pl8);
            const int m = int(upmask);
            const i32x4 plo = {pp[0] & ~m, pp[1] & ~m, pp[2] & ~m, pp[3] & ~m};
            const i32x4 phi = {pp[0] & m, pp[1] & m, pp[2] & m, pp[3] & m};
            const i32x4 qlo = {ql[0] & ~m, ql[1] & ~m, ql[2] & ~m, ql[3] & ~m};
            const i32x4 qhi = {ql[0] & m, ql[1] & m, ql[2] & m, ql[3] & m};
            Oe = mfma(V0, __builtin_bit_cast(bf16x8, plo), f32x16{});
            Oe = mfma(V1, __builtin_bit_cast(bf16x8, phi), Oe);
            Oe = mfma(V0, __builtin_bit_cast(bf16x8, qlo), Oe);
            Oe = mfma(V1, __builtin_bit_cast(bf16x8, qhi), Oe);
          } else if constexpr (R == 4) {
            // own (and middle-level) keys: 4 probabilities in the lane half
            // h = c % 2 at slots 4 ((c / 2) % 2) .. +3 of k-step c / 4; the
            // 8-token prefix's keys: slots 0..3 of k-step 0 in both halves
            auto place = [&](const uint32_t (&w)[2], int s) {
              const uint32_t ms = (s == 0 ? ~m_c2 : m_c2) & m_half;
              const i32x4 v = {int(w[0] & ms & ~m_c1), int(w[1] & ms & ~m_c1), int(w[0] & ms & m_c1),
                               int(w[1] & ms & m_c1)};
              return __builtin_bit_cast(bf16x8, v);
            };
            uint32_t hw[2], lw[2];
            pack4_hilo(p, hw, lw);
            Oe = mfma(V0, place(hw, 0), f32x16{});
            Oe = mfma(V1, place(hw, 1), Oe);
            Oe = mfma(V0, place(lw, 0), Oe);
            Oe = mfma(V1, place(lw, 1), Oe);
            pack4_hilo(p + NO, hw, lw);
            Oe = mfma(Vt, __builtin_bit_cast(bf16x8, i32x4{int(hw[0] & ~m_b8), int(hw[1] & ~m_b8),
                                                           int(hw[0] & m_b8), int(hw[1] & m_b8)}), Oe);
            Oe = mfma(Vt, __builtin_bit_cast(bf16x8, i32x4{int(lw[0] & ~m_b8), int(lw[1] & ~m_b8),
                                                           int(lw[0] & m_b8), int(lw[1] & m_b8)}), Oe);
            if constexpr (Rows<MODE>::TAILS) {
              pack4_hilo(p + NO + 4, hw, lw);
              Oe = mfma(Vm[0], place(hw, 0), Oe);
              Oe = mfma(Vm[1], place(hw, 1), Oe);
              Oe = mfma(Vm[0], place(lw, 0), Oe);
              Oe = mfma(Vm[1], place(lw, 1), Oe);
            }
          } else {
            // 4 probabilities per lane, placed at slots 4 (c % 2) .. +3 of k-step c / 2
            auto place = [&](const uint32_t (&w)[2], int s) {
              const uint32_t ms = s == 0 ? m_s0 : m_c1;
              const i32x4 v = {int(w[0] & ms & m_w0), int(w[1] & ms & m_w0), int(w[0] & ms & upmask),
                               int(w[1] & ms & upmask)};
              return __builtin_bit_cast(bf16x8, v);
            };
            uint32_t hw[2], lw[2];
            pack4_hilo(p, hw, lw);
            Oe = mfma(V0, place(hw, 0), f32x16{});
            Oe = mfma(V1, place(hw, 1), Oe);
            Oe = mfma(V0, place(lw, 0), Oe);
            Oe = mfma(V1, place(lw, 1), Oe);
            if constexpr (MODE == SUFFIX) {
              pack4_hilo(p + NO, hw, lw);
              Oe = mfma(Vk[0], place(hw, 0), Oe);
              Oe = mfma(Vk[1], place(hw, 1), Oe);
              Oe = mfma(Vk[0], place(lw, 0), Oe);
              Oe = mfma(Vk[1], place(lw, 1), Oe);
            }
          }
#pragma unroll
          for (int j = 0; j < 8; ++j) O[e * 8 + j] = Oe[e * 8 + j];
        }
        const bf16x8 O0 = to_bf16(O, 0), O1 = to_bf16(O, 1);
        const bf16x8 L0 = lo_bf16(O, 0, O0), L1 = lo_bf16(O, 1, O1);
        // output projection of O = hi + lo: fragment i = 2q + e (q = output
        // block); the weights' lo set multiplies O's hi part only
#pragma unroll
        for (int pt = 0; pt < NP_ATT; ++pt) {
          if (pt > 0) fetch_half<D>(fr[1], ring + cur * RS, 1, lane);
#pragma unroll
          for (int i = 0; i < HS; ++i) {
            f32x16 acc = mfma(fr[0][i], (i % 2) ? O1 : O0, res[i / 2]);
            res[i / 2] = pt == 0 ? mfma(fr[0][i], (i % 2) ? L1 : L0, acc) : acc;
          }
          adv(S::first_sub(4 * b + 3) + pt + 2);   // next Q, or the first FFN sub-step
          fetch_half<D>(fr[0], ring + cur * RS, 0, lane);
#pragma unroll
          for (int i = 0; i < HS; ++i) {
            f32x16 acc = mfma(fr[1][i], (i % 2) ? O1 : O0, res[(HS + i) / 2]);
            res[(HS + i) / 2] = pt == 0 ? mfma(fr[1][i], (i % 2) ? L1 : L0, acc) : acc;
          }
        }
      }
      // ---- feed-forward block, software-pipelined: the GELU of hidden block
      // fb is evaluated between the MFMAs of W1(fb + 1) and W2(fb - 1), which
      // do not depend on it, so that one wave keeps the matrix pipe busy while
      // it issues the elementwise work (waves sharing a SIMD were measured not
      // to fill each other's MFMA time).  The weight stream follows the same
      // order (Shape::ffn_is_w1 / ffn_block).
      static_assert(NP_W1 == 1 && NP_W2 == 1, "pipelined feed-forward block: one weight set");
      layer_norm<NB>(res, V16, int(S::VLN2G), int(S::VLN2B), X);
#pragma unroll
      for (int q = 0; q < NB; ++q) res[q] += lds16(V16 + S::VB2 + q * 32);
      {
        constexpr int J0 = 4 * NB;                  // first feed-forward step
        f32x16 Hc = lds16(V16 + S::VB1);
        // W1(0), stream position 0
        fetch_half<D>(fr[1], ring + cur * RS, 1, lane);
#pragma unroll
        for (int i = 0; i < HS; ++i) Hc = mfma(fr[0][i], X[i], Hc);
        adv(S::first_sub(J0) + 2);
        fetch_half<D>(fr[0], ring + cur * RS, 0, lane);
#pragma unroll
        for (int i = 0; i < HS; ++i) Hc = mfma(fr[1][i], X[HS + i], Hc);
        bf16x8 Hp0 = {}, Hp1 = {};                  // GELU output of the previous block
        // a W1 or W2 sub-step at stream position j, GELU values interleaved
        // (PER per half step, starting at G0 for half 0 and G0 + PER for half 1)
#define NQS_FFN_SUB(W1_, PER_, G0_, j_)                                                   \
  {                                                                                       \
    fetch_half<D>(fr[1], ring + cur * RS, 1, lane);                                       \
    ffn_half<D, W1_, PER_, G0_>(fr[0], 0, X, Hn, res, Hp0, Hp1, Hc);                      \
    adv(S::first_sub(J0 + (j_)) + 2);                                                     \
    fetch_half<D>(fr[0], ring + cur * RS, 0, lane);                                       \
    ffn_half<D, W1_, PER_, G0_ + PER_>(fr[1], 1, X, Hn, res, Hp0, Hp1, Hc);               \
  }
        {   // fb = 0: W1(1) at position 1 with all 16 GELU values of block 0
          f32x16 Hn = lds16(V16 + S::VB1 + 32);
          NQS_FFN_SUB(true, 8, 0, 1)
          Hp0 = to_bf16(Hc, 0);
          Hp1 = to_bf16(Hc, 1);
          Hc = Hn;
        }
        for (int fb = 1; fb < FB - 1; ++fb) {     // W1(fb + 1) at 2 fb, W2(fb - 1) at 2 fb + 1
          f32x16 Hn = lds16(V16 + S::VB1 + (fb + 1) * 32);
          NQS_FFN_SUB(true, 4, 0, 2 * fb)
          NQS_FFN_SUB(false, 4, 8, 2 * fb + 1)
          Hp0 = to_bf16(Hc, 0);
          Hp1 = to_bf16(Hc, 1);
          Hc = Hn;
        }
        {   // fb = FB - 1: W2(FB - 2) at position 2 FB - 2
          f32x16 Hn{};
          NQS_FFN_SUB(false, 8, 0, 2 * FB - 2)
          Hp0 = to_bf16(Hc, 0);
          Hp1 = to_bf16(Hc, 1);
        }
#undef NQS_FFN_SUB
        // W2(FB - 1), stream position 2 FB - 1
        fetch_half<D>(fr[1], ring + cur * RS, 1, lane);
#pragma unroll
        for (int i = 0; i < HS; ++i) res[i / 2] = mfma(fr[0][i], (i % 2) ? Hp1 : Hp0, res[i / 2]);
        adv(S::first_sub(J0 + 2 * FB - 1) + 2);
        fetch_half<D>(fr[0], ring + cur * RS, 0, lane);
#pragma unroll
        for (int i = 0; i < HS; ++i)
          res[(HS + i) / 2] = mfma(fr[1][i], (i % 2) ? Hp1 : Hp0, res[(HS + i) / 2]);
      }
    }

    // ---- final layer norm, head, masked log-softmax
    float lg[4] = {0.f, 0.f, 0.f, 0.f};
    {
      float s = 0.f, s2 = 0.f;
#pragma unroll
      for (int q = 0; q < NB; ++q)
#pragma unroll
        for (int j = 0; j < 16; ++j) {
          s += res[q][j];
          s2 = fmaf(res[q][j], res[q][j], s2);
        }
      s = pair_sum(s);
      s2 = pair_sum(s2);
      const float mu = s * (1.0f / D);
      const float rs = rsqrtf(fmaxf(s2 * (1.0f / D) - mu * mu, 0.f) + 1e-5f);
#pragma unroll
      for (int q = 0; q < NB; ++q) {
        const f32x16 gg = lds16(svec + a.lnfg + (q * 2 + h) * 16);
        const f32x16 bb = lds16(svec + a.lnfb + (q * 2 + h) * 16);
        const f32x4 *wh = reinterpret_cast<const f32x4 *>(svec + a.whead) + (q * 2 + h) * 16;
#pragma unroll
        for (int j = 0; j < 16; ++j) {
          const float y = fmaf((res[q][j] - mu) * rs, gg[j], bb[j]);
          const f32x4 w = wh[j];
          lg[0] = fmaf(y, w[0], lg[0]);
          lg[1] = fmaf(y, w[1], lg[1]);
          lg[2] = fmaf(y, w[2], lg[2]);
          lg[3] = fmaf(y, w[3], lg[3]);
        }
      }
#pragma unroll
      for (int k = 0; k < 4; ++k) lg[k] = pair_sum(lg[k]);
    }
    float logp = 0.f;
    if (t < n) {
#pragma unroll
      for (int k = 0; k < 4; ++k) lg[k] += svec[a.bhead + k] + svec[a.lbias + t * 4 + k];
      // the conditional logits of row cond_p, or (cond_p = -P) of rows 0..P-1
      // at cond[(cfg P + t) 4 + k]
      if (MODE <= WIDE && a.cond && (t == a.cond_p || t < -a.cond_p) && h == 0 && live) {
        const int64_t o = a.cond_p < 0 ? cfg * (-a.cond_p) + t : cfg;
#pragma unroll
        for (int k = 0; k < 4; ++k) a.cond[o * 4 + k] = double(lg[k]);
      }
    }
    const nqs_sector_info &si = sector_of(a.sec, x);
    // rows whose whole masked conditional is kept: every TREE row, MID's row
    // pm when TREE follows (its token varies within the pm-token prefix)
    const bool cond_row = MODE == TREE || (MODE == MID && a.lp_mid != nullptr && t == a.pm);
    // (MID: its rows from pm on belong to TAIL / TREE)
    if (t < si.n && (MODE != MID || t < a.pm || cond_row)) {
      const uint64_t below = (t == 0) ? 0ull : (~0ull >> (64 - 2 * t));
      const int na = __popcll(x & below & 0x5555555555555555ull);
      const int nb = __popcll(x & below & 0xAAAAAAAAAAAAAAAAull);
      const int allow = t < si.mask_levels ? phys_mask(a.sec, si, t, na, nb, x) : 0xF;
      const int tk = int((x >> (2 * t)) & 3ull);
      float mx = -INFINITY;
#pragma unroll
      for (int k = 0; k < 4; ++k)
        if ((allow >> k) & 1) mx = fmaxf(mx, lg[k]);
      float z = 0.f;
#pragma unroll
      for (int k = 0; k < 4; ++k)
        if ((allow >> k) & 1) z += expf(lg[k] - mx);
      const float lz = logf(z);
      if (MODE != TREE && (MODE != MID || t < a.pm))
        logp = ((allow >> tk) & 1) ? lg[tk] - mx - lz : -INFINITY;
      if constexpr (MODE == TREE || MODE == MID) {
        if (cond_row && h == 0 && live && !repeat) {
          const bool root = parent == r % R;
          float *dst = MODE == MID ? a.lp_mid : root ? a.lp_q : a.lp_q1;
          const int64_t e = MODE == MID ? ent12 : (root ? a.preq : a.preq1)[src + 1] - 1;
#pragma unroll
          for (int k = 0; k < 4; ++k) dst[4 * e + k] = ((allow >> k) & 1) ? lg[k] - mx - lz : -INFINITY;
        }
      }
    }
    if (MODE == TRUNK || MODE == MID || (MODE != TREE && a.logabs)) {
      // sum over the configuration's R rows
#pragma unroll
      for (int w = 1; w < R; w *= 2) logp += __shfl_xor(logp, w);
      if (r % R == 0 && h == 0 && live) {
        if constexpr (MODE == TRUNK) {
          a.plogp[cfg] = logp;
        } else if constexpr (MODE == SUFFIX) {
          a.logabs[cfg] = 0.5 * double(logp + a.plogp[ent_own]);
        } else if constexpr (MODE == MID) {
          a.plogp2[ent12] = logp;
        } else if constexpr (MODE == TAIL) {
          a.logabs[cfg] = 0.5 * double(logp + a.plogp[ent8] + a.plogp2[ent12]);
        } else {
          a.logabs[cfg] = 0.5 * double(logp);
        }
      }
    }
  }

  // ---- phase MLP for the chunk's configurations (column = configuration)
  if (MODE != TRUNK && MODE != MID && MODE != TREE && a.phase) {
    constexpr int PH = 256, PKS = PH / 16, PB = PH / 32;
    const int64_t item = c_base + r;
    const bool in = r < CPT * passes && item < B;
    const int64_t cfg = MODE == TAIL ? (in ? a.src[item] : -1) : item;
    const bool live = MODE == TAIL ? cfg >= 0 : in;
    const uint64_t x = live ? a.x[cfg] : 0ull;
    const int nx = live ? sector_of(a.sec, x).n : 0;
    bf16x8 Z[PKS];
#pragma unroll
    for (int b = 0; b < PB; ++b) {
      f32x16 z = lds16(svec + a.pb1 + (b * 2 + h) * 16);
      if constexpr (MODE == PHASE) {
        // first layer on MFMA: the one-hot tokens (k = 4 t + token) times W1
        // (hi + lo); slot i of lane half h in k-step s is token position
        // 4 s + 2 (i / 4) + h, value i % 4 (built per k-step: a held operand
        // array, or an unrolled k loop, spilled the registers; after the
        // transformer rows of the other layouts it spilled them too, so those
        // keep the row gathers below)
        const bf16x8 *w1 = pk + a.p1 + int64_t(b) * a.ks1 * 64;
        const bf16x8 *w1l = pk + a.p1lo + int64_t(b) * a.ks1 * 64;
#pragma unroll 1
        for (int s1 = 0; s1 < a.ks1; ++s1) {
          bf16x8 oh;
#pragma unroll
          for (int i = 0; i < 8; ++i) {
            const int tt = 4 * s1 + 2 * (i / 4) + h;
            oh[i] = tt < nx && int((x >> (2 * tt)) & 3ull) == i % 4 ? __bf16(1.0f) : __bf16(0.0f);
          }
          z = mfma(w1[s1 * 64], oh, z);
          z = mfma(w1l[s1 * 64], oh, z);
        }
      } else {
        // first layer: the sum of the configuration's token rows of W1 (fp32)
        for (int tt = 0; tt < nx; ++tt) {
          const int row = 4 * tt + int((x >> (2 * tt)) & 3ull);
          z += load16(vec + a.pw1 + int64_t(row) * PH + (b * 2 + h) * 16);
        }
      }
#pragma unroll
      for (int j = 0; j < 16; ++j) z[j] = gelu(z[j]);
      Z[2 * b] = to_bf16(z, 0);
      Z[2 * b + 1] = to_bf16(z, 1);
    }
    float ph = 0.f;
    for (int b = 0; b < PB; ++b) {
      f32x16 z = lds16(svec + a.pb2 + (b * 2 + h) * 16);
      const bf16x8 *w = pk + a.p2 + int64_t(b) * PKS * 64;
      const bf16x8 *wl = pk + a.p2lo + int64_t(b) * PKS * 64;
#pragma unroll
      for (int s = 0; s < PKS; ++s) {
        z = mfma(w[s * 64], Z[s], z);
        if (NP > 1) z = mfma(wl[s * 64], Z[s], z);
      }
      const f32x16 w3 = lds16(svec + a.pw3 + (b * 2 + h) * 16);
#pragma unroll
      for (int j = 0; j < 16; ++j) ph = fmaf(gelu(z[j]), w3[j], ph);
    }
    ph = pair_sum(ph);
    if (h == 0 && live) a.phase[cfg] = double(ph + svec[a.pb3]);
  }
  }  // chunk
}

// ----------------------------------------------------------------- packing

// Fragment order: (block ob, k-step s, lane l, slot i) <- W[16 s + pi_h(i)][32 ob + l%32],
// W row-major with leading dimension ld, starting at column col0.
// lo = 0 writes hi = bf16(w), lo = 1 writes bf16(w - hi) (w - hi is exact in fp32).
// Rows from k_rows on read as zero.
__global__ void pack_frag_kernel(const float *W, int64_t ld, int col0, int n_ob, int n_ks, int lo,
                                 int k_rows, __bf16 *out) {
  const int64_t idx = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (idx >= int64_t(n_ob) * n_ks * 64 * 8) return;
  const int i = int(idx % 8), l = int((idx / 8) % 64);
  const int64_t s = (idx / 512) % n_ks, ob = idx / (512 * int64_t(n_ks));
  const int hh = l / 32;
  const int krow = int(16 * s) + (i / 4) * 8 + hh * 4 + (i % 4);
  const float w = krow < k_rows ? W[int64_t(krow) * ld + col0 + 32 * ob + (l % 32)] : 0.f;
  const __bf16 hi = __bf16(w);
  out[idx] = lo ? __bf16(w - float(hi)) : hi;
}

// Permuted vector: out[(b*2+h)*16 + j] = v[perm_feature(b, h, j)], for `rows`
// vectors of length N (stride N) -- the feature order of an accumulator block.
__global__ void perm_vec_kernel(const float *v, int N, int rows, float *out) {
  const int64_t idx = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (idx >= int64_t(rows) * N) return;
  const int c = int(idx % N);
  const int64_t row = idx / N;
  const int j = c % 16, hh = (c / 16) % 2, b = c / 32;
  out[idx] = v[row * N + perm_feature(b, hh, j)];
}

// whead (D x 4) in permuted row order: out[(b*2+h)*16 + j][k] = W[perm_feature(b,h,j)][k]
__global__ void perm_head_kernel(const float *W, int D, float *out) {
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= D * 4) return;
  const int k = idx % 4, c = idx / 4;
  const int j = c % 16, hh = (c / 16) % 2, b = c / 32;
  out[idx] = W[perm_feature(b, hh, j) * 4 + k];
}

__global__ void copy_f32_kernel(const float *src, int64_t n, float *dst) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < n) dst[i] = src[i];
}

struct Layout {
  FusedArgs a;
  int64_t frag_total = 0, vec_total = 0;
};

Layout plan(const nqs_model &m) {
  Layout L{};
  const int D = m.d, F = m.F, NB = D / 32, KS = D / 16, PH = m.PH;
  auto frag = [&](int n_ob, int n_ks) {
    const int64_t o = L.frag_total;
    L.frag_total += int64_t(n_ob) * n_ks * 64;
    return o;
  };
  auto vec = [&](int64_t len) {
    const int64_t o = L.vec_total;
    L.vec_total += (len + 15) / 16 * 16;
    return o;
  };
  for (int l = 0; l < m.L; ++l) {
    L.a.q[l] = frag(NB, KS);
    L.a.k[l] = frag(NB, KS);
    L.a.v[l] = frag(NB, KS);
    L.a.o[l] = frag(NB, KS);
    L.a.w1[l] = frag(F / 32, KS);
    L.a.w2[l] = frag(NB, F / 16);
    // the lo sets (NP = 2) follow the layer's hi sets in the same order
    for (int p = 1; p < NP; ++p) {
      frag(NB, KS);
      frag(NB, KS);
      frag(NB, KS);
      frag(NB, KS);
      frag(F / 32, KS);
      frag(NB, F / 16);
    }
    L.a.ln1g[l] = vec(D);
    L.a.ln1b[l] = vec(D);
    L.a.bq[l] = vec(D);
    L.a.bk[l] = vec(D);
    L.a.bv[l] = vec(D);
    L.a.bo[l] = vec(D);
    L.a.ln2g[l] = vec(D);
    L.a.ln2b[l] = vec(D);
    L.a.b1[l] = vec(F);
    L.a.b2[l] = vec(D);
  }
  L.a.p2 = frag(PH / 32, PH / 16);
  L.a.p2lo = frag(PH / 32, PH / 16);
  L.a.ks1 = (4 * m.n + 15) / 16;
  L.a.p1 = frag(PH / 32, L.a.ks1);
  L.a.p1lo = frag(PH / 32, L.a.ks1);
  L.a.lnfg = vec(D);
  L.a.lnfb = vec(D);
  L.a.whead = vec(4 * D);
  L.a.bhead = vec(4);
  L.a.lbias = vec(4 * m.n);
  L.a.tok = vec(5 * D);
  L.a.pos = vec(int64_t(m.n) * D);
  L.a.pb1 = vec(PH);
  L.a.pb2 = vec(PH);
  L.a.pw3 = vec(PH);
  L.a.pb3 = vec(1);
  L.a.pw1 = vec(int64_t(4) * m.n * PH);
  return L;
}

inline dim3 g1(int64_t n) { return dim3(unsigned(ceil_div(n, 256))); }

template <int D, int MODE>
void launch_mode(const FusedArgs &a, dim3 grid, size_t lds_bytes, hipStream_t s) {
  if (lds_bytes > 64 * 1024)
    HIP_OK(hipFuncSetAttribute(reinterpret_cast<const void *>(&fused_kernel<D, MODE>),
                               hipFuncAttributeMaxDynamicSharedMemorySize, int(lds_bytes)));
  hipLaunchKernelGGL((fused_kernel<D, MODE>), grid, dim3(256), lds_bytes, s, a);
  HIP_LAUNCH_OK();
}

template <int D>
void launch_d(int mode, const FusedArgs &a, dim3 grid, size_t lds_bytes, hipStream_t s) {
  switch (mode) {
    case PLAIN: launch_mode<D, PLAIN>(a, grid, lds_bytes, s); break;
    case WIDE: launch_mode<D, WIDE>(a, grid, lds_bytes, s); break;
    case TRUNK: launch_mode<D, TRUNK>(a, grid, lds_bytes, s); break;
    case SUFFIX: launch_mode<D, SUFFIX>(a, grid, lds_bytes, s); break;
    case MID: launch_mode<D, MID>(a, grid, lds_bytes, s); break;
    case TAIL: launch_mode<D, TAIL>(a, grid, lds_bytes, s); break;
    case TREE: launch_mode<D, TREE>(a, grid, lds_bytes, s); break;
    default: launch_mode<D, PHASE>(a, grid, lds_bytes, s); break;
  }
}

// prefix table of the shared evaluation: flag[k] = 1 for every 8-token prefix
// k = x & 0xFFFF present in x
__global__ void prefix_mark_kernel(const uint64_t *__restrict__ x, int64_t B,
                                   int64_t *__restrict__ flag) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < B) flag[x[i] & 0xFFFFull] = 1;
}
// list[slot[k]] = k for every flagged prefix (slot = exclusive scan of flag)
__global__ void prefix_list_kernel(const int64_t *__restrict__ flag,
                                   const int64_t *__restrict__ slot, uint64_t *__restrict__ list) {
  const int k = int(blockIdx.x) * blockDim.x + threadIdx.x;
  if (k < (1 << 16) && flag[k]) list[slot[k]] = uint64_t(k);
}

// Three-level bookkeeping over x sorted by (first 8 tokens, tokens 8 .. pm-1,
// the rest): h8[i] / hm[i] = 1 where configuration i starts a new 8-token /
// pm-token prefix.
__global__ void prefix_heads_kernel(const uint64_t *__restrict__ x, int64_t B, uint64_t mmask,
                                    int64_t *__restrict__ h8, int64_t *__restrict__ hm) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= B) return;
  const uint64_t d = i == 0 ? ~0ull : x[i] ^ x[i - 1];
  h8[i] = (d & 0xFFFFull) != 0;
  hm[i] = (d & mmask) != 0;
}
// per 8-token group g (pre8 / prem: exclusive scans of h8 / hm): its first
// configuration and first pm-token prefix, and the trunk list entry; the
// sentinels first8[G] = B, firstm[G] = number of pm-token prefixes
__global__ void prefix_groups_kernel(const uint64_t *__restrict__ x, int64_t B,
                                     const int64_t *__restrict__ h8, const int64_t *__restrict__ pre8,
                                     const int64_t *__restrict__ prem, int64_t *__restrict__ first8,
                                     int64_t *__restrict__ firstm, uint64_t *__restrict__ list8) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= B) return;
  if (h8[i]) {
    const int64_t g = pre8[i];
    first8[g] = i;
    firstm[g] = prem[i];
    list8[g] = x[i] & 0xFFFFull;
  }
  if (i == 0) {
    first8[pre8[B]] = B;
    firstm[pre8[B]] = prem[B];
  }
}
__global__ void fill_i64_kernel(int64_t *__restrict__ p, int64_t n, int64_t v) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}
// item lists: tail[start_t[g] + i - first8[g]] = i for every configuration i;
// mid[start_m[g] + j - firstm[g]] = i for the first configuration i of every
// pm-token prefix j
__global__ void prefix_maps_kernel(int64_t B, const int64_t *__restrict__ hm,
                                   const int64_t *__restrict__ pre8, const int64_t *__restrict__ prem,
                                   const int64_t *__restrict__ first8,
                                   const int64_t *__restrict__ firstm,
                                   const int64_t *__restrict__ start_t,
                                   const int64_t *__restrict__ start_m, int64_t *__restrict__ tail,
                                   int64_t *__restrict__ mid) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= B) return;
  const int64_t g = pre8[i + 1] - 1;
  tail[start_t[g] + i - first8[g]] = i;
  if (hm[i]) mid[start_m[g] + prem[i] - firstm[g]] = i;
}

// ---- tree tail (TREE) bookkeeping over x sorted by tokens (bits 0..15 first,
// then token 8, 9, ...): every prefix of 8 or more tokens is a contiguous run.
__host__ __device__ inline uint64_t low_mask(int b) { return b >= 64 ? ~0ull : (1ull << b) - 1; }
// h8 / hm / hq / hq1[i] = 1 where configuration i starts a new 8-, m-, q- or
// (q+1)-token prefix
__global__ void tree_heads_kernel(const uint64_t *__restrict__ x, int64_t B, int m, int q,
                                  int64_t *__restrict__ h8, int64_t *__restrict__ hm,
                                  int64_t *__restrict__ hq, int64_t *__restrict__ hq1) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= B) return;
  const uint64_t d = i == 0 ? ~0ull : x[i] ^ x[i - 1];
  h8[i] = (d & 0xFFFFull) != 0;
  hm[i] = (d & low_mask(2 * m)) != 0;
  hq[i] = (d & low_mask(2 * q)) != 0;
  hq1[i] = (d & low_mask(2 * q + 2)) != 0;
}
// first configurations of the m-, q- and (q+1)-token prefixes
__global__ void tree_firsts_kernel(int64_t B, const int64_t *__restrict__ hm,
                                   const int64_t *__restrict__ hq, const int64_t *__restrict__ hq1,
                                   const int64_t *__restrict__ prem, const int64_t *__restrict__ preq,
                                   const int64_t *__restrict__ preq1, int64_t *__restrict__ firstm_cfg,
                                   int64_t *__restrict__ firstq, int64_t *__restrict__ firstq1) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= B) return;
  if (hm[i]) firstm_cfg[prem[i]] = i;
  if (hq[i]) firstq[preq[i]] = i;
  if (hq1[i]) firstq1[preq1[i]] = i;
}
// The slots of m-token prefix j: its q-token prefixes in order, each with its
// (q+1)-token extensions, as pieces of a root row and extension rows; while
// two or more of the current slot's four rows are free, the next piece takes
// the root and as many extensions as fit, else the next slot opens (a prefix
// whose extensions span two slots has its root row repeated in the second;
// filling the free rows this way costs a repeated root row but wastes none).  All rows of a slot share prefix j's middle
// entry.  With `tree` null only the number of slots is returned; otherwise
// the rows are written from slot `base` on: entry = first configuration |
// (slot row of the parent) << 48, | 1 << 47 on a repeated root (which must
// not store the prefix's conditional a second time: the products of a row
// round differently at another position of the pass, and two stores would
// race).
__device__ inline int64_t tree_pack(int64_t j, int64_t PM, int64_t Q, int64_t B,
                                    const int64_t *__restrict__ firstm_cfg,
                                    const int64_t *__restrict__ firstq,
                                    const int64_t *__restrict__ firstq1,
                                    const int64_t *__restrict__ preq,
                                    const int64_t *__restrict__ preq1, int64_t base,
                                    int64_t *__restrict__ tree) {
  const int64_t i0 = firstm_cfg[j], i1 = j + 1 < PM ? firstm_cfg[j + 1] : B;
  int64_t slot = -1;
  int used = 4;                                  // rows used in the current slot
  for (int64_t k = preq[i0]; k < preq[i1]; ++k) {
    const int64_t c0 = preq1[firstq[k]], c1 = k + 1 < Q ? preq1[firstq[k + 1]] : preq1[B];
    for (int64_t c = c0; c < c1;) {
      // fill the current slot: with two rows free or more, the root and as many
      // extensions as fit go in, and the rest follow under a repeated root
      if (used > 2) {
        ++slot;
        used = 0;
      }
      const int piece = 1 + int(c1 - c < 3 - used ? c1 - c : 3 - used);
      if (tree) {
        int64_t *row = tree + 4 * (base + slot);
        // a root repeated for its later extensions: bit 47, no second store
        row[used] = firstq[k] | (int64_t(used) << 48) | (c > c0 ? int64_t(1) << 47 : 0);
        for (int e = 1; e < piece; ++e) row[used + e] = firstq1[c + e - 1] | (int64_t(used) << 48);
      }
      used += piece;
      c += piece - 1;
    }
  }
  return slot + 1;
}
__global__ void tree_count_kernel(int64_t PM, int64_t Q, int64_t B,
                                  const int64_t *__restrict__ firstm_cfg,
                                  const int64_t *__restrict__ firstq,
                                  const int64_t *__restrict__ firstq1,
                                  const int64_t *__restrict__ preq,
                                  const int64_t *__restrict__ preq1, int64_t *__restrict__ nslot) {
  const int64_t j = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (j < PM) nslot[j] = tree_pack(j, PM, Q, B, firstm_cfg, firstq, firstq1, preq, preq1, 0, nullptr);
}
// per 8-token group g < G: its slots and middle items
__global__ void tree_counts_kernel(int64_t G, const int64_t *__restrict__ firstm,
                                   const int64_t *__restrict__ es, int64_t *__restrict__ cnt_s,
                                   int64_t *__restrict__ cnt_m) {
  const int64_t g = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (g >= G) return;
  // firstm[G] = the number of m-token prefixes
  cnt_s[g] = es[firstm[g + 1]] - es[firstm[g]];
  cnt_m[g] = firstm[g + 1] - firstm[g];
}
// item lists: mid[start_m[g] + j - firstm[g]] = first configuration of m-token
// prefix j, and its slots from start_s[g] + es[j] - es[firstm[g]]
__global__ void tree_lists_kernel(int64_t PM, int64_t Q, int64_t B,
                                  const int64_t *__restrict__ pre8,
                                  const int64_t *__restrict__ firstm,
                                  const int64_t *__restrict__ firstm_cfg,
                                  const int64_t *__restrict__ firstq,
                                  const int64_t *__restrict__ firstq1,
                                  const int64_t *__restrict__ preq,
                                  const int64_t *__restrict__ preq1, const int64_t *__restrict__ es,
                                  const int64_t *__restrict__ start_s,
                                  const int64_t *__restrict__ start_m, int64_t *__restrict__ mid,
                                  int64_t *__restrict__ tree) {
  const int64_t j = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (j >= PM) return;
  const int64_t i = firstm_cfg[j], g = pre8[i + 1] - 1;
  mid[start_m[g] + j - firstm[g]] = i;
  tree_pack(j, PM, Q, B, firstm_cfg, firstq, firstq1, preq, preq1,
            start_s[g] + es[j] - es[firstm[g]], tree);
}
// log|psi| of every configuration from the stored conditionals: tokens 0..7
// (plogp), 8..m-1 (plogp2), token m = q - 1 (lp_mid), q (lp_q), q + 1 (lp_q1)
// and the membership test of the last token, q + 2 = n - 1
__global__ void tree_gather_kernel(Sectors sec, const uint64_t *__restrict__ x, int64_t B, int q,
                                   const int64_t *__restrict__ pre8, const int64_t *__restrict__ prem,
                                   const int64_t *__restrict__ preq,
                                   const int64_t *__restrict__ preq1,
                                   const float *__restrict__ plogp, const float *__restrict__ plogp2,
                                   const float *__restrict__ lp_mid, const float *__restrict__ lp_q,
                                   const float *__restrict__ lp_q1, double *__restrict__ logabs) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= B) return;
  const uint64_t v = x[i];
  const int64_t g = pre8[i + 1] - 1, j = prem[i + 1] - 1, k = preq[i + 1] - 1, c = preq1[i + 1] - 1;
  const int tm = int((v >> (2 * (q - 1))) & 3ull), tq = int((v >> (2 * q)) & 3ull),
            tq1 = int((v >> (2 * q + 2)) & 3ull);
  float lp = plogp[g] + plogp2[j];
  lp += lp_mid[4 * j + tm];
  lp += lp_q[4 * k + tq];
  lp += lp_q1[4 * c + tq1];
  const nqs_sector_info &si = sector_of(sec, v);
  const int t = si.n - 1;
  const uint64_t below = ~0ull >> (64 - 2 * t);
  const int na = __popcll(v & below & 0x5555555555555555ull);
  const int nb = __popcll(v & below & 0xAAAAAAAAAAAAAAAAull);
  const int allow = phys_mask(sec, si, t, na, nb, v);
  if (!((allow >> int((v >> (2 * t)) & 3ull)) & 1)) lp = -INFINITY;
  logabs[i] = 0.5 * double(lp);
}

// Position n - 1 when the sector leaves at most one token there: its masked
// conditional is 1 if the configuration's last token is allowed, else 0.  The
// tail rows stop at n - 2; this applies the last factor to log|psi|.
__global__ void last_token_kernel(Sectors sec, const uint64_t *__restrict__ x, int64_t B,
                                  double *__restrict__ logabs) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= B) return;
  const uint64_t v = x[i];
  const nqs_sector_info &si = sector_of(sec, v);
  const int t = si.n - 1;
  const uint64_t below = ~0ull >> (64 - 2 * t);
  const int na = __popcll(v & below & 0x5555555555555555ull);
  const int nb = __popcll(v & below & 0xAAAAAAAAAAAAAAAAull);
  const int allow = phys_mask(sec, si, t, na, nb, v);
  if (!((allow >> int((v >> (2 * t)) & 3ull)) & 1)) logabs[i] = -INFINITY;
}

}  // namespace

bool fused_supported(const nqs_model &m) {
  return m.kind == NQS_MODEL_TRANSFORMER && (m.d == 64 || m.d == 128) && m.F == 4 * m.d &&
         m.H * 16 == m.d && m.PH == 256 && m.n <= kSeqMax && m.L <= kMaxLayers;
}

bool fused_shared_supported(const nqs_model &m) {
  return m.precision == NQS_BF16 && fused_supported(m) && m.n > kTrunk && m.n <= 16 && !m.tagged &&
         m.prefix_share;
}

int fused_shared_levels(const nqs_model &m) {
  return !fused_shared_supported(m) ? 0 : m.n >= 13 ? 3 : 2;
}

// Whether every sector's mask leaves at most one token at the last position
// (particle numbers do, and so do Z2 parities and additive symmetries whose
// four token contributions differ there); then that position's conditional is
// 1 for an allowed token and 0 otherwise, whatever the network computes.
bool last_token_fixed(const nqs_model &m) {
  if (m.sec_host.empty()) return false;
  for (const nqs_sector_info &si : m.sec_host) {
    if (si.mask_levels < si.n) return false;
    const int t = si.n - 1;
    if (si.general) {
      // level t's states are g[t] .. g[t + 1] - 1, four children each
      const int32_t *g = reinterpret_cast<const int32_t *>(m.phys_host.data() + si.phys_off);
      const int32_t *kids = g + si.n + 1;
      for (int32_t id = g[t]; id < g[t + 1]; ++id) {
        int k = 0;
        for (int j = 0; j < 4; ++j) k += kids[4 * int64_t(id) + j] >= 0;
        if (k > 1) return false;
      }
    } else {
      const int64_t per = (int64_t(si.n + 1) * (si.n + 1)) << si.nz2;
      const uint8_t *e = m.phys_host.data() + si.phys_off + int64_t(t) * per;
      for (int64_t i = 0; i < per; ++i)
        if (__builtin_popcount(unsigned(e[i]) & 0xFu) > 1) return false;
    }
  }
  return true;
}

int fused_shared_pm(const nqs_model &m) {
  return m.n >= 14 && last_token_fixed(m) ? m.n - 5 : m.n - 4;
}

void fused_pack(nqs_model &m, hipStream_t s) {
  NQS_REQUIRE(fused_supported(m), NQS_EUNSUPPORTED, "fused forward: unsupported dimensions");
  Layout L = plan(m);
  static_assert(sizeof(bf16x8) == 16, "fragment size");
  // the kernel addresses layer l at l * FRAG_L / l * VEC_L with constant offsets
  auto check = [&](auto shape) {
    using S = decltype(shape);
    for (int l = 0; l < m.L; ++l) {
      const int64_t f = l * S::LAYER, v = l * S::VEC_L;
      NQS_REQUIRE(L.a.q[l] == f + S::OQ && L.a.k[l] == f + S::OK && L.a.v[l] == f + S::OV &&
                      L.a.o[l] == f + S::OO && L.a.w1[l] == f + S::OW1 &&
                      L.a.w2[l] == f + S::OW2 && L.a.ln1g[l] == v + S::VLN1G &&
                      L.a.ln1b[l] == v + S::VLN1B && L.a.bq[l] == v + S::VBQ &&
                      L.a.bk[l] == v + S::VBK && L.a.bv[l] == v + S::VBV &&
                      L.a.bo[l] == v + S::VBO && L.a.ln2g[l] == v + S::VLN2G &&
                      L.a.ln2b[l] == v + S::VLN2B && L.a.b1[l] == v + S::VB1 &&
                      L.a.b2[l] == v + S::VB2,
                  NQS_EINVAL, "fused forward: packed layout mismatch");
    }
  };
  if (m.d == 128) check(Shape<128>{});
  else check(Shape<64>{});
  __bf16 *pk = static_cast<__bf16 *>(m.packed.reserve(size_t(L.frag_total) * 16));
  const float *W = m.master.as<float>();
  const int D = m.d, F = m.F, NB = D / 32, KS = D / 16, PH = m.PH, n = m.n;
  auto P = [&](int idx) { return W + m.off[idx]; };
  float *vb = static_cast<float *>(m.packed_vec.reserve(size_t(L.vec_total) * 4));
  // hi set at o, lo set (when NP = 2) lo_off fragments entries further
  auto pack = [&](const float *src, int64_t ld, int col0, int n_ob, int n_ks, int64_t o,
                  int64_t lo_off, int sets) {
    for (int p = 0; p < sets; ++p) {
      hipLaunchKernelGGL(pack_frag_kernel, g1(int64_t(n_ob) * n_ks * 512), dim3(256), 0, s, src,
                         ld, col0, n_ob, n_ks, p, 16 * n_ks, pk + (o + p * lo_off) * 8);
      HIP_LAUNCH_OK();
    }
  };
  const int64_t lo_layer = m.d == 128 ? Shape<128>::FRAG_L : Shape<64>::FRAG_L;
  auto perm = [&](const float *src, int N, int rows, int64_t o) {
    hipLaunchKernelGGL(perm_vec_kernel, g1(int64_t(N) * rows), dim3(256), 0, s, src, N, rows, vb + o);
    HIP_LAUNCH_OK();
  };
  auto copy = [&](const float *src, int64_t len, int64_t o) {
    hipLaunchKernelGGL(copy_f32_kernel, g1(len), dim3(256), 0, s, src, len, vb + o);
    HIP_LAUNCH_OK();
  };
  for (int l = 0; l < m.L; ++l) {
    const float *wqkv = P(tf_layer(l, TF_WQKV)), *bqkv = P(tf_layer(l, TF_BQKV));
    pack(wqkv, 3 * D, 0, NB, KS, L.a.q[l], lo_layer, NP_ATT);
    pack(wqkv, 3 * D, D, NB, KS, L.a.k[l], lo_layer, NP_ATT);
    pack(wqkv, 3 * D, 2 * D, NB, KS, L.a.v[l], lo_layer, NP_ATT);
    pack(P(tf_layer(l, TF_WO)), D, 0, NB, KS, L.a.o[l], lo_layer, NP_ATT);
    pack(P(tf_layer(l, TF_W1)), F, 0, F / 32, KS, L.a.w1[l], lo_layer, NP_W1);
    pack(P(tf_layer(l, TF_W2)), D, 0, NB, F / 16, L.a.w2[l], lo_layer, NP_W2);
    perm(P(tf_layer(l, TF_LN1G)), D, 1, L.a.ln1g[l]);
    perm(P(tf_layer(l, TF_LN1B)), D, 1, L.a.ln1b[l]);
    perm(bqkv, D, 1, L.a.bq[l]);
    perm(bqkv + D, D, 1, L.a.bk[l]);
    copy(bqkv + 2 * D, D, L.a.bv[l]);
    perm(P(tf_layer(l, TF_BO)), D, 1, L.a.bo[l]);
    perm(P(tf_layer(l, TF_LN2G)), D, 1, L.a.ln2g[l]);
    perm(P(tf_layer(l, TF_LN2B)), D, 1, L.a.ln2b[l]);
    perm(P(tf_layer(l, TF_B1)), F, 1, L.a.b1[l]);
    perm(P(tf_layer(l, TF_B2)), D, 1, L.a.b2[l]);
  }
  const int Lm = m.L;
  pack(P(tf_tail(Lm, TF_PW2)), PH, 0, PH / 32, PH / 16, L.a.p2, L.a.p2lo - L.a.p2, NP);
  perm(P(tf_tail(Lm, TF_LNFG)), D, 1, L.a.lnfg);
  perm(P(tf_tail(Lm, TF_LNFB)), D, 1, L.a.lnfb);
  hipLaunchKernelGGL(perm_head_kernel, g1(4 * D), dim3(256), 0, s, P(tf_tail(Lm, TF_WHEAD)), D,
                     vb + L.a.whead);
  HIP_LAUNCH_OK();
  copy(P(tf_tail(Lm, TF_BHEAD)), 4, L.a.bhead);
  copy(P(tf_tail(Lm, TF_LBIAS)), 4 * n, L.a.lbias);
  perm(P(TF_TOK), D, 5, L.a.tok);
  perm(P(TF_POS), D, n, L.a.pos);
  perm(P(tf_tail(Lm, TF_PB1)), PH, 1, L.a.pb1);
  perm(P(tf_tail(Lm, TF_PB2)), PH, 1, L.a.pb2);
  perm(P(tf_tail(Lm, TF_PW3)), PH, 1, L.a.pw3);
  copy(P(tf_tail(Lm, TF_PB3)), 1, L.a.pb3);
  perm(P(tf_tail(Lm, TF_PW1)), PH, 4 * n, L.a.pw1);
  // phase W1 (4 n rows) as MFMA fragments, rows past 4 n zero
  for (int p = 0; p < NP; ++p) {
    hipLaunchKernelGGL(pack_frag_kernel, g1(int64_t(PH / 32) * L.a.ks1 * 512), dim3(256), 0, s,
                       P(tf_tail(Lm, TF_PW1)), int64_t(PH), 0, PH / 32, L.a.ks1, p, 4 * n,
                       pk + (p == 0 ? L.a.p1 : L.a.p1lo) * 8);
    HIP_LAUNCH_OK();
  }
  m.packed_valid = true;
}

namespace {
// Passes per chunk (at most 32 configurations per wave and chunk; fewer when
// the batch is too small to give every SIMD of the chip two waves), the grid,
// the LDS size, the launch and its timing record.
void launch_fused(nqs_model &m, int mode, FusedArgs &a, int64_t B, hipStream_t s,
                  const int64_t *count, int passes, int max_blocks) {
  const int cpt = mode == PLAIN ? 2 : mode == WIDE ? 1 : mode <= SUFFIX ? 4 : 8;
  const int maxp = 32 / cpt;
  const int64_t target_waves = 2048;
  a.passes = int(std::min<int64_t>(maxp, std::max<int64_t>(1, ceil_div(B, cpt * target_waves))));
  if (passes > 0) a.passes = std::min(passes, maxp);
  // a device count without a tile: the 2048 waves that fill the chip (fewer
  // for a small capacity), passes chosen by the kernel from the count
  const bool auto_passes = count && passes <= 0;
  if (auto_passes) a.passes = 0;
  a.count = count;
  Layout L = plan(m);
  a.lds_floats = int(L.a.pw1);   // every vector before the phase-MLP input table
  // vectors, then the weight ring (three slots of d/16 fragments of 1 KiB)
  const size_t lds_bytes = size_t(a.lds_floats) * 4 + size_t(3) * (m.d / 16) * 1024;
  // two blocks per CU must fit the 160 KiB of LDS
  NQS_REQUIRE(lds_bytes <= 80 * 1024, NQS_EUNSUPPORTED,
              "fused forward: model vectors exceed the LDS budget");
  int64_t blocks = auto_passes ? std::min<int64_t>(ceil_div(B, int64_t(4 * cpt)), target_waves / 4)
                               : ceil_div(B, int64_t(4 * cpt) * a.passes);   // four waves per block
  if (max_blocks > 0) blocks = std::min<int64_t>(blocks, max_blocks);
  NQS_REQUIRE(blocks <= int64_t(0x7FFFFFFF), NQS_EUNSUPPORTED, "fused forward: batch too large");
  const dim3 grid = dim3(unsigned(blocks));
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (g_timing && !count) {
    HIP_OK(hipEventCreate(&e0));
    HIP_OK(hipEventCreate(&e1));
    HIP_OK(hipEventRecord(e0, s));
  }
  if (m.d == 128) launch_d<128>(mode, a, grid, lds_bytes, s);
  else launch_d<64>(mode, a, grid, lds_bytes, s);
  if (g_timing && !count) {
    HIP_OK(hipEventRecord(e1, s));
    g_records.push_back({e0, e1, B, 0.f, mode});
  }
}
}  // namespace

void fused_forward(nqs_model &m, const uint64_t *x, int64_t B, double *logabs, double *phase,
                   double *cond_out, int cond_p, hipStream_t s, const int64_t *count,
                   FusedTile tile) {
  if (m.kind == NQS_MODEL_NADE) {
    nade_fused_forward(m, x, B, logabs, phase, cond_out, cond_p, s, count);
    return;
  }
  NQS_REQUIRE(m.packed_valid, NQS_EINVAL, "fused forward: weights not packed");
  if (B <= 0) return;
  Layout L = plan(m);
  FusedArgs a = L.a;
  a.pk = m.packed.as<bf16x8>();
  a.vec = m.packed_vec.as<float>();
  a.sec = m.sectors();
  a.x = x;
  a.B = B;
  a.count = nullptr;
  a.n = m.n;
  a.L = m.L;
  a.cond_p = cond_p;
  a.logabs = logabs;
  a.phase = phase;
  a.cond = cond_out;
  launch_fused(m, m.n > 16 ? WIDE : PLAIN, a, B, s, count, tile.pairs, tile.blocks);
}


void fused_forward_shared(nqs_model &m, const uint64_t *x, int64_t B, double *logabs,
                          double *phase, hipStream_t s) {
  NQS_REQUIRE(m.packed_valid, NQS_EINVAL, "fused forward: weights not packed");
  NQS_REQUIRE(fused_shared_supported(m), NQS_EUNSUPPORTED, "shared forward: unsupported model");
  if (B <= 0) return;
  constexpr int64_t K = int64_t(1) << 16;      // 8-token prefixes
  const int64_t cap = std::min(K, B);          // entries: at most one per configuration
  const int64_t kv_bytes = int64_t(m.L) * (m.d / 32) * 1024;
  static_assert((int64_t(1) << 16) * kMaxLayers * 4 * 1024 <= (int64_t(1) << 31),
                "prefix entries are addressed by 32-bit offsets");
  auto *flag = static_cast<int64_t *>(m.pf_tab.reserve(size_t(2 * K + 1) * 8));
  int64_t *slot = flag + K;
  auto *list = static_cast<uint64_t *>(m.pf_list.reserve(size_t(cap) * 8));
  auto *plogp = static_cast<float *>(m.pf_logp.reserve(size_t(cap) * 4));
  auto *kv = static_cast<uint8_t *>(m.pf_kv.reserve(size_t(cap) * size_t(kv_bytes)));
  zero_async(flag, size_t(K) * 8, s);
  hipLaunchKernelGGL(prefix_mark_kernel, g1(B), dim3(256), 0, s, x, B, flag);
  HIP_LAUNCH_OK();
  launch_exclusive_scan(flag, slot, K, s, m.pf_scan);
  hipLaunchKernelGGL(prefix_list_kernel, g1(K), dim3(256), 0, s, flag, slot, list);
  HIP_LAUNCH_OK();
  int64_t n_prefix = 0;
  HIP_OK(hipMemcpyAsync(&n_prefix, slot + K, 8, hipMemcpyDeviceToHost, s));
  HIP_OK(hipStreamSynchronize(s));
  NQS_REQUIRE(n_prefix >= 1 && n_prefix <= cap, NQS_EINVAL, "shared forward: prefix count");
  Layout L = plan(m);
  FusedArgs a = L.a;
  a.pk = m.packed.as<bf16x8>();
  a.vec = m.packed_vec.as<float>();
  a.sec = m.sectors();
  a.n = m.n;
  a.L = m.L;
  a.cond_p = -1;
  a.cond = nullptr;
  a.kv = kv;
  a.kv_bytes = kv_bytes;
  a.kv_total = cap * kv_bytes;
  a.plogp = plogp;
  a.slot = slot;
  // positions 0..7 of every prefix (their number is on the device: slot[K])
  a.x = list;
  a.B = n_prefix;
  a.logabs = nullptr;
  a.phase = nullptr;
  launch_fused(m, TRUNK, a, n_prefix, s, nullptr, 0, 0);
  // positions 8..15 of every configuration
  a.x = x;
  a.B = B;
  a.logabs = logabs;
  a.phase = phase;
  launch_fused(m, SUFFIX, a, B, s, nullptr, 0, 0);
}

int64_t pack_group_starts(const std::vector<int64_t> &cnt, const std::vector<char> &cut,
                          std::vector<int64_t> &start);

void fused_forward_shared3(nqs_model &m, const uint64_t *x, int64_t B, double *logabs,
                           double *phase, hipStream_t s) {
  NQS_REQUIRE(m.packed_valid, NQS_EINVAL, "fused forward: weights not packed");
  NQS_REQUIRE(fused_shared_levels(m) == 3, NQS_EUNSUPPORTED, "shared forward: unsupported model");
  if (B <= 0) return;
  constexpr int64_t K = int64_t(1) << 16;      // 8-token prefixes
  const int pm = fused_shared_pm(m);           // TAIL: positions pm .. pm + 3
  const uint64_t mmask = (1ull << (2 * pm)) - 1;
  const int64_t kv_bytes = int64_t(m.L) * (m.d / 32) * 1024;
  const int64_t kv2_bytes = int64_t(m.L) * (m.d / 32) * 512;
  const int64_t cap8 = std::min(K, B), items = B + 7 * cap8;
  // workspaces: flags and their scans, groups, list starts, item lists
  int64_t *w = static_cast<int64_t *>(m.pf3_ws.reserve(size_t(4 * (B + 1) + 4 * (K + 1) + 2 * items) * 8));
  int64_t *h8 = w, *hm = h8 + (B + 1), *pre8 = hm + (B + 1), *prem = pre8 + (B + 1);
  int64_t *first8 = prem + (B + 1), *firstm = first8 + (K + 1), *start_t = firstm + (K + 1);
  int64_t *start_m = start_t + (K + 1);
  int64_t *tail = start_m + (K + 1), *mid = tail + items;
  auto *list8 = static_cast<uint64_t *>(m.pf_list.reserve(size_t(cap8) * 8));
  auto *plogp = static_cast<float *>(m.pf_logp.reserve(size_t(cap8) * 4));
  auto *kv = static_cast<uint8_t *>(m.pf_kv.reserve(size_t(cap8) * size_t(kv_bytes)));
  auto *plogp2 = static_cast<float *>(m.pf3_logp.reserve(size_t(B) * 4));
  hipLaunchKernelGGL(prefix_heads_kernel, g1(B), dim3(256), 0, s, x, B, mmask, h8, hm);
  HIP_LAUNCH_OK();
  launch_exclusive_scan(h8, pre8, B, s, m.pf_scan);
  launch_exclusive_scan(hm, prem, B, s, m.pf_scan);
  hipLaunchKernelGGL(prefix_groups_kernel, g1(B), dim3(256), 0, s, x, B, h8, pre8, prem, first8,
                     firstm, list8);
  HIP_LAUNCH_OK();
  int64_t cnt[2] = {0, 0};
  HIP_OK(hipMemcpyAsync(&cnt[0], pre8 + B, 8, hipMemcpyDeviceToHost, s));
  HIP_OK(hipMemcpyAsync(&cnt[1], prem + B, 8, hipMemcpyDeviceToHost, s));
  HIP_OK(hipStreamSynchronize(s));
  const int64_t G = cnt[0], PM = cnt[1];
  NQS_REQUIRE(G >= 1 && G <= cap8 && PM >= G && PM <= B, NQS_EINVAL, "shared forward: prefix count");
  std::vector<int64_t> f8(size_t(G) + 1), fm(size_t(G) + 1);
  HIP_OK(hipMemcpyAsync(f8.data(), first8, size_t(G + 1) * 8, hipMemcpyDeviceToHost, s));
  HIP_OK(hipMemcpyAsync(fm.data(), firstm, size_t(G + 1) * 8, hipMemcpyDeviceToHost, s));
  HIP_OK(hipStreamSynchronize(s));
  // slices of whole groups whose middle entries fit in 32-bit offsets (at most
  // kMidSlice entries), each starting a new pass; then the lists' group
  // starts, a pass of 8 items holding up to two 8-token prefixes
  const int64_t slice = std::min<int64_t>(PM, kMidSliceBytes / kv2_bytes);
  std::vector<int64_t> cuts;          // first group of every slice, then G
  std::vector<char> cut(size_t(G), 0);
  for (int64_t g0 = 0; g0 < G;) {
    int64_t g1 = g0 + 1;
    while (g1 < G && fm[size_t(g1 + 1)] - fm[size_t(g0)] <= slice) ++g1;
    NQS_REQUIRE(fm[size_t(g1)] - fm[size_t(g0)] <= slice, NQS_EINVAL, "shared forward: slice");
    cuts.push_back(g0);
    cut[size_t(g0)] = 1;
    g0 = g1;
  }
  cuts.push_back(G);
  std::vector<int64_t> cnt_t(static_cast<size_t>(G)), cnt_m(static_cast<size_t>(G));
  for (size_t g = 0; g < size_t(G); ++g) {
    cnt_t[g] = f8[g + 1] - f8[g];
    cnt_m[g] = fm[g + 1] - fm[g];
  }
  std::vector<int64_t> st_t, st_m;
  const int64_t n_t = pack_group_starts(cnt_t, cut, st_t);
  const int64_t n_m = pack_group_starts(cnt_m, cut, st_m);
  // both lists within the allocation before any entry is written
  NQS_REQUIRE(n_t <= items && n_m <= items && n_t >= B && n_m >= PM, NQS_EINVAL,
              "shared forward: item lists");
  HIP_OK(hipMemcpyAsync(start_t, st_t.data(), size_t(G + 1) * 8, hipMemcpyHostToDevice, s));
  HIP_OK(hipMemcpyAsync(start_m, st_m.data(), size_t(G + 1) * 8, hipMemcpyHostToDevice, s));
  hipLaunchKernelGGL(fill_i64_kernel, g1(2 * items), dim3(256), 0, s, tail, 2 * items, int64_t(-1));
  HIP_LAUNCH_OK();
  hipLaunchKernelGGL(prefix_maps_kernel, g1(B), dim3(256), 0, s, B, hm, pre8, prem, first8,
                     firstm, start_t, start_m, tail, mid);
  HIP_LAUNCH_OK();

  Layout L = plan(m);
  FusedArgs a = L.a;
  a.pk = m.packed.as<bf16x8>();
  a.vec = m.packed_vec.as<float>();
  a.sec = m.sectors();
  a.n = m.n;
  a.L = m.L;
  a.cond_p = -1;
  a.cond = nullptr;
  a.kv = kv;
  a.kv_bytes = kv_bytes;
  a.kv_total = cap8 * kv_bytes;
  a.plogp = plogp;
  a.pre8 = pre8;
  a.pre12 = prem;
  a.kv2_bytes = kv2_bytes;
  a.plogp2 = plogp2;
  a.pm = pm;
  // positions 0..7 once per 8-token prefix (entry g = group g)
  a.x = list8;
  a.B = G;
  launch_fused(m, TRUNK, a, G, s, nullptr, 0, 0);
  // positions 8 .. pm-1 once per pm-token prefix, then the last four of every
  // configuration, slice by slice (a slice's items end where its last group's do)
  auto *kv2 = static_cast<uint8_t *>(m.pf3_kv.reserve(size_t(slice) * size_t(kv2_bytes)));
  a.kv2 = kv2;
  a.kv2_total = slice * kv2_bytes;
  a.x = x;
  for (size_t c = 0; c + 1 < cuts.size(); ++c) {
    const size_t g0 = size_t(cuts[c]), gl = size_t(cuts[c + 1]) - 1;
    a.j0 = fm[g0];
    a.src = mid + st_m[g0];
    a.B = st_m[gl] + cnt_m[gl] - st_m[g0];
    a.logabs = nullptr;
    a.phase = nullptr;
    launch_fused(m, MID, a, a.B, s, nullptr, 0, 0);
    a.src = tail + st_t[g0];
    a.B = st_t[gl] + cnt_t[gl] - st_t[g0];
    a.logabs = logabs;
    a.phase = phase;
    launch_fused(m, TAIL, a, a.B, s, nullptr, 0, 0);
  }
  if (pm + 4 < m.n) {
    hipLaunchKernelGGL(last_token_kernel, g1(B), dim3(256), 0, s, m.sectors(), x, B, logabs);
    HIP_LAUNCH_OK();
  }
}

// Item list starts of the groups (cnt[g] items each) when a pass of 8 items
// may hold two 8-token prefixes: a group follows the previous one unless the
// pass it would start in already holds two, and every slice (cut[g] set)
// starts a new pass.  Returns the end of the list.
int64_t pack_group_starts(const std::vector<int64_t> &cnt, const std::vector<char> &cut,
                          std::vector<int64_t> &start) {
  const size_t G = cnt.size();
  start.assign(G + 1, 0);
  int64_t pos = 0;
  int groups = 0;                     // groups in the pass holding pos, when pos % 8 != 0
  for (size_t g = 0; g < G; ++g) {
    if (pos % 8 != 0 && (cut[g] || groups >= 2)) {
      pos = (pos + 7) / 8 * 8;
      groups = 0;
    }
    start[g] = pos;
    const int64_t end = pos + cnt[g];
    groups = (end - 1) / 8 == pos / 8 ? (pos % 8 == 0 ? 1 : groups + 1) : 1;
    pos = end;
    if (pos % 8 == 0) groups = 0;
  }
  start[G] = pos;
  return pos;
}

bool fused_tree(const nqs_model &m) {
  return m.tail_tree && fused_shared_levels(m) == 3 && m.n <= 15 && last_token_fixed(m);
}

void fused_forward_tree(nqs_model &m, const uint64_t *x, int64_t B, double *logabs,
                        double *phase, hipStream_t s) {
  NQS_REQUIRE(m.packed_valid, NQS_EINVAL, "fused forward: weights not packed");
  NQS_REQUIRE(fused_tree(m), NQS_EUNSUPPORTED, "tree forward: unsupported model");
  if (B <= 0) return;
  constexpr int64_t K = int64_t(1) << 16;      // 8-token prefixes
  const int q = m.n - 3, pm = q - 1;           // TREE rows at q and q + 1
  const int64_t kv_bytes = int64_t(m.L) * (m.d / 32) * 1024;
  const int64_t kv2_bytes = int64_t(m.L) * (m.d / 32) * 512;
  const int64_t cap8 = std::min(K, B), items = B + 7 * cap8;
  // workspaces: flags, their scans, first configurations of the q-token
  // prefixes, slots per prefix and their scan, groups, pads and their scans,
  // item lists (middle: one entry per item; tree: four per slot)
  const int64_t B1 = B + 1, K1 = K + 1;
  int64_t *w = static_cast<int64_t *>(m.pf3_ws.reserve(size_t(13 * B1 + 6 * K1 + 5 * items) * 8));
  int64_t *h8 = w, *hm = h8 + B1, *hq = hm + B1, *hq1 = hq + B1;
  int64_t *pre8 = hq1 + B1, *prem = pre8 + B1, *preq = prem + B1, *preq1 = preq + B1;
  int64_t *firstm_cfg = preq1 + B1, *firstq = firstm_cfg + B1, *firstq1 = firstq + B1;
  int64_t *nslot = firstq1 + B1, *es = nslot + B1;
  int64_t *first8 = es + B1, *firstm = first8 + K1, *pad_s = firstm + K1, *pad_m = pad_s + K1;
  int64_t *start_s = pad_m + K1, *start_m = start_s + K1;
  int64_t *mid = start_m + K1, *tree = mid + items;
  auto *list8 = static_cast<uint64_t *>(m.pf_list.reserve(size_t(cap8) * 8));
  auto *plogp = static_cast<float *>(m.pf_logp.reserve(size_t(cap8) * 4));
  auto *kv = static_cast<uint8_t *>(m.pf_kv.reserve(size_t(cap8) * size_t(kv_bytes)));
  // per-prefix floats: plogp2 (B), lp_mid, lp_q, lp_q1 (4 B each)
  auto *fl = static_cast<float *>(m.pf3_logp.reserve(size_t(13 * B) * 4));
  float *plogp2 = fl, *lp_mid = fl + B, *lp_q = lp_mid + 4 * B, *lp_q1 = lp_q + 4 * B;
  hipLaunchKernelGGL(tree_heads_kernel, g1(B), dim3(256), 0, s, x, B, pm, q, h8, hm, hq, hq1);
  HIP_LAUNCH_OK();
  launch_exclusive_scan(h8, pre8, B, s, m.pf_scan);
  launch_exclusive_scan(hm, prem, B, s, m.pf_scan);
  launch_exclusive_scan(hq, preq, B, s, m.pf_scan);
  launch_exclusive_scan(hq1, preq1, B, s, m.pf_scan);
  hipLaunchKernelGGL(prefix_groups_kernel, g1(B), dim3(256), 0, s, x, B, h8, pre8, prem, first8,
                     firstm, list8);
  HIP_LAUNCH_OK();
  hipLaunchKernelGGL(tree_firsts_kernel, g1(B), dim3(256), 0, s, B, hm, hq, hq1, prem, preq, preq1,
                     firstm_cfg, firstq, firstq1);
  HIP_LAUNCH_OK();
  int64_t cnt[4] = {0, 0, 0, 0};
  HIP_OK(hipMemcpyAsync(&cnt[0], pre8 + B, 8, hipMemcpyDeviceToHost, s));
  HIP_OK(hipMemcpyAsync(&cnt[1], prem + B, 8, hipMemcpyDeviceToHost, s));
  HIP_OK(hipMemcpyAsync(&cnt[2], preq + B, 8, hipMemcpyDeviceToHost, s));
  HIP_OK(hipMemcpyAsync(&cnt[3], preq1 + B, 8, hipMemcpyDeviceToHost, s));
  HIP_OK(hipStreamSynchronize(s));
  const int64_t G = cnt[0], PM = cnt[1], Q = cnt[2], Q1 = cnt[3];
  NQS_REQUIRE(G >= 1 && G <= cap8 && PM >= G && Q >= PM && Q1 >= Q && Q1 <= B, NQS_EINVAL,
              "tree forward: prefix count");
  m.tree_rows_q += Q;
  m.tree_rows_q1 += Q1;
  hipLaunchKernelGGL(tree_count_kernel, g1(PM), dim3(256), 0, s, PM, Q, B, firstm_cfg, firstq,
                     firstq1, preq, preq1, nslot);
  HIP_LAUNCH_OK();
  launch_exclusive_scan(nslot, es, PM, s, m.pf_scan);
  hipLaunchKernelGGL(tree_counts_kernel, g1(G), dim3(256), 0, s, G, firstm, es, pad_s, pad_m);
  HIP_LAUNCH_OK();
  hipLaunchKernelGGL(fill_i64_kernel, g1(5 * items), dim3(256), 0, s, mid, 5 * items, int64_t(-1));
  HIP_LAUNCH_OK();
  std::vector<int64_t> cnt_s(static_cast<size_t>(G)), cnt_m(static_cast<size_t>(G)),
      fm(static_cast<size_t>(G) + 1);
  HIP_OK(hipMemcpyAsync(cnt_s.data(), pad_s, size_t(G) * 8, hipMemcpyDeviceToHost, s));
  HIP_OK(hipMemcpyAsync(cnt_m.data(), pad_m, size_t(G) * 8, hipMemcpyDeviceToHost, s));
  HIP_OK(hipMemcpyAsync(fm.data(), firstm, size_t(G + 1) * 8, hipMemcpyDeviceToHost, s));
  HIP_OK(hipStreamSynchronize(s));
  // slices of whole groups whose middle entries fit in 32-bit offsets, each
  // starting a new pass; then the lists' group starts, two groups per pass
  const int64_t slice = std::min<int64_t>(PM, kMidSliceBytes / kv2_bytes);
  std::vector<int64_t> cuts;          // first group of every slice, then G
  std::vector<char> cut(size_t(G), 0);
  for (int64_t g0 = 0; g0 < G;) {
    int64_t g1 = g0 + 1;
    while (g1 < G && fm[size_t(g1 + 1)] - fm[size_t(g0)] <= slice) ++g1;
    NQS_REQUIRE(fm[size_t(g1)] - fm[size_t(g0)] <= slice, NQS_EINVAL, "tree forward: slice");
    cuts.push_back(g0);
    cut[size_t(g0)] = 1;
    g0 = g1;
  }
  cuts.push_back(G);
  std::vector<int64_t> st_s, st_m;
  const int64_t n_s = pack_group_starts(cnt_s, cut, st_s);
  const int64_t n_m = pack_group_starts(cnt_m, cut, st_m);
  // (a slot holds at least one q-token prefix; both lists within the
  // allocation before any entry is written)
  NQS_REQUIRE(n_s <= items && n_m <= items && n_s * 4 >= Q && n_m >= PM, NQS_EINVAL,
              "tree forward: item lists");
  HIP_OK(hipMemcpyAsync(start_s, st_s.data(), size_t(G + 1) * 8, hipMemcpyHostToDevice, s));
  HIP_OK(hipMemcpyAsync(start_m, st_m.data(), size_t(G + 1) * 8, hipMemcpyHostToDevice, s));
  hipLaunchKernelGGL(tree_lists_kernel, g1(PM), dim3(256), 0, s, PM, Q, B, pre8, firstm, firstm_cfg,
                     firstq, firstq1, preq, preq1, es, start_s, start_m, mid, tree);
  HIP_LAUNCH_OK();

  Layout L = plan(m);
  FusedArgs a = L.a;
  a.pk = m.packed.as<bf16x8>();
  a.vec = m.packed_vec.as<float>();
  a.sec = m.sectors();
  a.n = m.n;
  a.L = m.L;
  a.cond_p = -1;
  a.cond = nullptr;
  a.kv = kv;
  a.kv_bytes = kv_bytes;
  a.kv_total = cap8 * kv_bytes;
  a.plogp = plogp;
  a.pre8 = pre8;
  a.pre12 = prem;
  a.kv2_bytes = kv2_bytes;
  a.plogp2 = plogp2;
  a.pm = pm;
  a.lp_mid = lp_mid;
  a.lp_q = lp_q;
  a.lp_q1 = lp_q1;
  a.preq = preq;
  a.preq1 = preq1;
  a.logabs = nullptr;
  a.phase = nullptr;
  // positions 0..7 once per 8-token prefix (entry g = group g)
  a.x = list8;
  a.B = G;
  launch_fused(m, TRUNK, a, G, s, nullptr, 0, 0);
  // positions 8 .. pm once per pm-token prefix, then the slots (positions q
  // and q + 1), slice by slice (a slice's items end where its last group's do)
  auto *kv2 = static_cast<uint8_t *>(m.pf3_kv.reserve(size_t(slice) * size_t(kv2_bytes)));
  a.kv2 = kv2;
  a.kv2_total = slice * kv2_bytes;
  a.x = x;
  for (size_t c = 0; c + 1 < cuts.size(); ++c) {
    const size_t g0 = size_t(cuts[c]), gl = size_t(cuts[c + 1]) - 1;
    a.j0 = fm[g0];
    a.src = mid + st_m[g0];
    a.B = st_m[gl] + cnt_m[gl] - st_m[g0];
    // one pass per block: short blocks leave less of the chip idle in a
    // launch's last round (measured 90.7 -> 85.2 ms per step)
    launch_fused(m, MID, a, a.B, s, nullptr, 1, 0);
    a.src = tree + 4 * st_s[g0];
    a.B = st_s[gl] + cnt_s[gl] - st_s[g0];
    launch_fused(m, TREE, a, a.B, s, nullptr, 1, 0);
  }
  // the phase MLP of every configuration
  if (phase) {
    a.src = nullptr;
    a.B = B;
    a.phase = phase;
    launch_fused(m, PHASE, a, B, s, nullptr, 0, 0);
  }
  hipLaunchKernelGGL(tree_gather_kernel, g1(B), dim3(256), 0, s, a.sec, x, B, q, pre8, prem, preq,
                     preq1, plogp, plogp2, lp_mid, lp_q, lp_q1, logabs);
  HIP_LAUNCH_OK();
}

bool timing_on() { return g_timing; }

hipEvent_t timing_begin(hipStream_t s, const int64_t *count) {
  if (!g_timing || count) return nullptr;
  hipEvent_t e0 = nullptr;
  HIP_OK(hipEventCreate(&e0));
  HIP_OK(hipEventRecord(e0, s));
  return e0;
}

void timing_end(hipEvent_t start, hipStream_t s, int64_t configs, int mode) {
  if (!start) return;
  hipEvent_t e1 = nullptr;
  HIP_OK(hipEventCreate(&e1));
  HIP_OK(hipEventRecord(e1, s));
  g_records.push_back({start, e1, configs, 0.f, mode});
}

void timing_add(float ms, int64_t configs, int mode) {
  g_records.push_back({nullptr, nullptr, configs, ms, mode});
}

}  // namespace nqs

using namespace nqs;

extern "C" int nqs_timing_enable(int on) {
  return guarded([&] { g_timing = on != 0; });
}

extern "C" int nqs_timing_read_mode(int mode, double *ms, int64_t *launches, int64_t *configs) {
  return guarded([&] {
    double total = 0.0;
    int64_t cfgs = 0, nl = 0;
    std::vector<TimingRecord> keep;
    for (const TimingRecord &r : g_records) {
      if (mode != -2 && r.mode != mode) {
        keep.push_back(r);
        continue;
      }
      float t = r.ms;
      if (r.stop) {
        HIP_OK(hipEventSynchronize(r.stop));
        HIP_OK(hipEventElapsedTime(&t, r.start, r.stop));
      }
      total += t;
      cfgs += r.configs;
      ++nl;
      if (r.start) (void)hipEventDestroy(r.start);
      if (r.stop) (void)hipEventDestroy(r.stop);
    }
    if (ms) *ms = total;
    if (launches) *launches = nl;
    if (configs) *configs = cfgs;
    g_records.swap(keep);
  });
}

extern "C" int nqs_timing_read(double *ms, int64_t *launches, int64_t *configs) {
  return nqs_timing_read_mode(-2, ms, launches, configs);
}
