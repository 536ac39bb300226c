/*
 * nqs.h - C ABI of the MI355X (gfx950) hot path of symmetry-constrained
 * autoregressive neural-quantum-state VMC for molecular Hamiltonians
 * (A. Malyshev, J. M. Arrazola, A. I. Lvovsky, arXiv 2310.04166).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * - Return value: NQS_OK (0) or a negative status.  No C++ exception or abort
 *   crosses this boundary.  nqs_last_error() gives a message for the calling
 *   thread's most recent failure.
 * - Configurations are uint64 bit strings: bit j is the occupation of
 *   spin-orbital j = 2p + s (p spatial orbital, s = 0 alpha, s = 1 beta), so
 *   N = 2 n_spatial <= 64 qubits.  Token p of a configuration is
 *   bit(2p) + 2 bit(2p+1) in {0 empty, 1 alpha, 2 beta, 3 both}.
 * - "dev" pointers are device memory of the current HIP device, "host"
 *   pointers host memory.  The caller owns every array it passes; the library
 *   owns its handles (create / destroy) and its internal workspaces.
 * - Work is ordered on the given stream (NULL = default stream).  Calls that
 *   return a size on the host (sample_unique, local_energy, connected_pairs)
 *   synchronise that stream before returning.
 * - A handle may be used from one host thread at a time.
 */
#ifndef NQS_H
#define NQS_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define NQS_OK            0
#define NQS_EINVAL       -1   /* bad argument (null pointer, size, mismatch)      */
#define NQS_ECAPACITY    -2   /* output buffer too small; required size reported */
#define NQS_EUNSUPPORTED -3   /* N > 64, sequence > 32 tokens, unknown kind, ...  */
#define NQS_EHIP         -4   /* HIP runtime error or no usable gfx950 device     */
#define NQS_ENOMEM       -5   /* device or host allocation failed                 */

typedef struct nqs_ham nqs_ham;
typedef struct nqs_model nqs_model;
typedef struct nqs_batch nqs_batch;
typedef void *nqs_stream;     /* a hipStream_t */

/* Message of the calling thread's last failure ("" if none). */
const char *nqs_last_error(void);

/* ------------------------------------------------------------------------ */
/* Hamiltonian compiler                                                      */
/* ------------------------------------------------------------------------ */

/*
 * ham_compile - second-quantised molecular Hamiltonian to Jordan-Wigner
 * Pauli strings grouped by X/Y flip mask (paper: "System description",
 * equation for H_SQ and the Jordan-Wigner encoding of the HF state).
 *
 *   H = sum_{pq,s} h1[p,q] a+_ps a_qs
 *     + 1/2 sum_{pqrs,s,t} eri[p,q,r,s] a+_ps a+_rt a_st a_qs + e_core
 *
 * h1 (host, n_spatial^2 doubles, row-major, symmetric) and eri (host,
 * n_spatial^4 doubles, chemists' (pq|rs), 8-fold symmetric) are read only.
 * Each term is mapped with a_j = (prod_{k<j} Z_k)(X_j + iY_j)/2; Pauli
 * strings with the same X/Y support f are one "flip group".  A string acts as
 * P|x> = c (-1)^popcount(x & z) |x ^ f>, with the i-factors of its Y's folded
 * into the real coefficient c, so that
 *     <x ^ f| H |x> = sum_{t in group f} coef[t] (-1)^popcount(x & zmask[t]).
 * Strings whose coefficients cancel (odd number of Y's, which vanish for a
 * real symmetric H) are dropped; a magnitude above 1e-12 relative to the
 * largest coefficient there means asymmetric integrals (NQS_EINVAL).
 * Groups are sorted by flip ascending (the diagonal group, f = 0, first).
 * Host work only; the tables go to the device on first use.
 * (n_alpha, n_beta) is the target sector, that of the HF determinant.
 * Errors: NQS_EINVAL (null, n_spatial < 1, electrons out of range,
 * asymmetric integrals), NQS_EUNSUPPORTED (n_spatial > 32).
 */
int ham_compile(const double *h1, const double *eri, int n_spatial, double e_core,
                int n_alpha, int n_beta, nqs_ham **out);

/* Number of flip groups G and Pauli terms T of a compiled Hamiltonian. */
int ham_info(const nqs_ham *ham, int64_t *n_groups, int64_t *n_terms);

/* Host copies of the tables: flip[G] (ascending), off[G+1] (CSR offsets into
 * the term arrays), zmask[T], coef[T].  Any pointer may be NULL. */
int ham_tables(const nqs_ham *ham, uint64_t *flip, int64_t *off, uint64_t *zmask, double *coef);

/*
 * ham_z2_symmetries - Z2 symmetries of the Hamiltonian (paper: "Molecular
 * symmetries"): qubit masks m such that Z on the qubits of m commutes with H,
 * i.e. m shares an even number of qubits with every flip mask (the null space
 * over GF(2) of the flip masks).  Returned: a basis of that space modulo the
 * parities of the alpha and beta electron numbers (which the electron counts
 * fix); for integrals with point-group selection rules, one mask per
 * generator of the abelian point group.  masks (host, max_gen entries)
 * receives min(count, max_gen) masks, n_gen (host) the count.
 * Errors: NQS_EINVAL (null), NQS_ECAPACITY (count > max_gen; n_gen set).
 */
int ham_z2_symmetries(const nqs_ham *ham, int max_gen, uint64_t *masks, int *n_gen);

void ham_destroy(nqs_ham *ham);

/* ------------------------------------------------------------------------ */
/* Amplitude model                                                           */
/* ------------------------------------------------------------------------ */

#define NQS_MODEL_MLP         1   /* per-token NADE-like MLPs (Appendix B)      */
#define NQS_MODEL_TRANSFORMER 2   /* decoder-only transformer + phase MLP       */
#define NQS_MODEL_NADE        3   /* the paper's per-qubit complex-weight MLPs  */
#define NQS_MODEL_TABLE       4   /* psi given explicitly on a basis (no network) */

#define NQS_FP64 1   /* every operation in double                            */
#define NQS_FP32 2   /* every operation in float                             */
#define NQS_BF16 3   /* forward GEMMs bf16 x bf16 -> fp32 on MFMA (the attention
                        probabilities and output, and the per-qubit ansatz's
                        hidden activations, as bf16 hi + lo pairs); LN,
                        softmax, residual, log-softmax in fp32; backward in
                        fp32                                                  */

#define NQS_MU  0    /* Mask-Unphysical on every level ("Pruning strategies") */
#define NQS_DU  1    /* Discard-Unphysical on every level                     */
#define NQS_MUD 2    /* MU on levels p < n - d, DU on the last d levels       */

/*
 * amp_model_create - an autoregressive amplitude psi(x) = prod_p psi_p(x_p|x_<p)
 * (paper: ANQS product rule) over the n = dims[0] orbital tokens, with the
 * conditionals masked by the (n_alpha, n_beta) sector according to
 * strategy / d (paper: "Pruning strategies"; Algorithm 1 gives the mask).
 *
 * dims (host):
 *   MLP:         {n, n_alpha, n_beta, hidden}
 *   TRANSFORMER: {n, n_alpha, n_beta, d_model, n_layers, n_heads, ffn, phase_hidden}
 *   NADE:        {n, n_alpha, n_beta, hidden}
 *   TABLE:       {n, n_alpha, n_beta, lo_0, hi_0, ..., lo_{M-1}, hi_{M-1}}: the
 *                M basis configurations as (low, high) 32-bit halves, in
 *                strictly ascending uint64 order (n_dims = 3 + 2 M)
 * params (host, n_params doubles) is the canonical parameter vector: the
 * concatenation of the tensors below, each row-major, matrices (in, out) so
 * that a layer computes y = x W + b.
 *   MLP, for p = 0..n-1:  w1 (4p, hidden), b1 (hidden), w2 (hidden, hidden),
 *                         b2 (hidden), w3 (hidden, 8), b3 (8)
 *      outputs 0..3 are the logits of tokens 0..3, outputs 4..7 their phases;
 *      layer 1 tanh, layer 2 leaky ReLU (slope 0.01).
 *   TRANSFORMER: tok_emb (5, d) [row 4 = BOS], pos_emb (n, d), then per layer
 *      ln1_g (d), ln1_b (d), wqkv (d, 3d) [q | k | v], bqkv (3d), wo (d, d),
 *      bo (d), ln2_g (d), ln2_b (d), w1 (d, ffn), b1 (ffn), w2 (ffn, d),
 *      b2 (d); then lnf_g (d), lnf_b (d), whead (d, 4), bhead (4),
 *      logit_bias (n, 4), ph_w1 (4n, ph), ph_b1 (ph), ph_w2 (ph, ph),
 *      ph_b2 (ph), ph_w3 (ph, 1), ph_b3 (1).
 *      Pre-LN blocks (eps 1e-5), causal attention with scale 1/sqrt(d/heads),
 *      tanh-form GELU, input [BOS, x_0 .. x_{n-2}], output p = logits of
 *      token p; phase = MLP(one-hot of all n tokens) with GELU.
 *   NADE (paper: Appendix "ANQS architecture"), for qubit i = 0..2n-1: w1_re,
 *      w1_im (i, hidden), b1_re, b1_im (hidden), w2_re, w2_im (hidden,
 *      hidden), b2_re, b2_im (hidden), w3_re, w3_im (hidden, 2), b3_re,
 *      b3_im (2): complex weights W = W_re + i W_im; on the previous bits x,
 *      h1 = tanh(x W1 + b1) (complex tanh), h2 = LeReLU(Re(h1 W2 + b2)) +
 *      i LeReLU(Im(h1 W2 + b2)), z = h2 W3 + b3, log psi_i(v | x_<i) = z_v -
 *      1/2 log(e^{2 Re z_0} + e^{2 Re z_1}).  Mask-Unphysical per qubit: with
 *      one physical value v, psi_i(v) = 1 and psi_i(1 - v) = 0.  FP64, FP32,
 *      and BF16 with hidden = 64: amp_forward and local_energy then run one
 *      fused kernel per batch (all three layers on MFMA, bf16 operands, fp32
 *      accumulation, complex tanh / leaky ReLU / normaliser in fp32, log|psi|
 *      and phase summed in double); the sampler and amp_backward use the
 *      fp32 master parameters layer by layer.
 *   TABLE (local-energy equation; with psi the exact ground vector E_loc = E_0
 *      everywhere): params = log|psi| of the M basis configurations, then
 *      their phases (2 M doubles); psi = 0 outside the basis.  FP64 only.
 *      amp_forward looks x up by binary search; the sampler's conditional of
 *      token p is the Born mass of the basis configurations continuing the
 *      prefix with that token over the prefix's mass; amp_backward adds each
 *      sample's upstream weights to its basis entry.  No sectors of several
 *      molecules, no Z2 restriction (the basis is the support).
 * log|psi(x)| = 1/2 sum_p log softmax over allowed tokens; phase separate.
 * Errors: NQS_EINVAL (sizes, n_params mismatch), NQS_EUNSUPPORTED (n > 32,
 * d_model not a multiple of n_heads, unknown kind / precision / strategy,
 * BF16 with an MLP, a transformer outside the fused kernel's shapes or a
 * per-qubit ansatz with hidden != 64), NQS_EHIP / NQS_ENOMEM (device).
 */
int amp_model_create(int kind, const int32_t *dims, int n_dims, const double *params,
                     int64_t n_params, int precision, int strategy, int d,
                     nqs_model **out);

/* Number of parameters and the element size (8 or 4 bytes) of the model's
 * device master parameter vector. */
int amp_model_info(const nqs_model *m, int64_t *n_params, int32_t *param_bytes);

/* Device pointer of the master parameter vector (canonical layout, double in
 * FP64 mode, float otherwise).  After writing it, call amp_model_sync. */
int amp_model_params(nqs_model *m, void **dev_params);

/* Rebuild the model's derived device buffers (packed / bf16 weights) from the
 * master parameters, on the stream. */
int amp_model_sync(nqs_model *m, nqs_stream stream);

/* Copy the master parameters to / from host doubles (n_params of them),
 * converting to the master type; set also rebuilds the derived buffers.
 * Both synchronise the device. */
int amp_model_get_params(const nqs_model *m, double *host_out);
int amp_model_set_params(nqs_model *m, const double *host_in);

void amp_model_destroy(nqs_model *m);

/*
 * amp_model_set_sectors - let one transformer serve n_mol (1..64) molecules
 * of different sizes (the batching form of the path; the paper's masks per
 * molecule, Algorithm 1 per sector).  Molecule i has n[i] <= dims[0] orbital
 * tokens and (n_alpha[i], n_beta[i]) electrons (host arrays).  Afterwards every
 * configuration word given to the model carries its molecule index in bits
 * 58..63 (occupation bits below; so dims[0] <= 29): the molecule reads rows
 * 0..n[i]-1 of pos_emb and logit_bias, its phase-MLP input is its one-hot code
 * followed by zeros, and its conditionals are masked by its own sector.
 * n_mol = 0 returns the model to its own single sector (untagged words).
 * Errors: NQS_EINVAL (counts out of range), NQS_EUNSUPPORTED (MLP model,
 * dims[0] > 29, Z2 symmetries set).
 */
int amp_model_set_sectors(nqs_model *m, int n_mol, const int32_t *n, const int32_t *n_alpha,
                          const int32_t *n_beta);

/*
 * amp_model_set_symmetries - define the model's sector by general quantum
 * numbers (paper: "Physicality evaluation algorithm", Algorithm 1 for any
 * number of symmetries; Appendix A): n_add (0..8) additive symmetries, where
 * qubit q holding bit b contributes eig[s * 4n + 2 q + b] (host int32) to
 * symmetry s and a configuration's eigenvalue is the sum over its 2n qubits
 * (particle number: eig = b; 2 S_z: (-1)^q b; any integer combination is
 * another instance), with target sums targets[s] (host); and n_z2 (0..4) Z2
 * symmetries z2_masks (host; Z on those qubits, eigenvalues composed by
 * multiplication) with target parities z2_targets (host, 0/1 meaning +1/-1;
 * NULL = all 0).  The masked conditionals, the sampler and amp_forward then
 * keep exactly the configurations with those sums and parities (the table of
 * physical prefix states is built on the host by Algorithm 1; the kernels walk
 * a configuration's tokens through it).  The Hamiltonian's connected x' of a
 * sample are those of its own (N_alpha, N_beta) block, so local_energy applies
 * to any such sector of a number-conserving Hamiltonian.  n_add = n_z2 = 0
 * returns the model to its (n_alpha, n_beta) sector.
 * Errors: NQS_EINVAL (counts, empty sector, masks beyond the qubits),
 * NQS_EUNSUPPORTED (the model serves several molecules, more than 2^22 prefix
 * states in a level).
 */
int amp_model_set_symmetries(nqs_model *m, int n_add, const int32_t *eig, const int32_t *targets,
                             int n_z2, const uint64_t *z2_masks, const int32_t *z2_targets);

/*
 * amp_model_set_z2 - restrict the model's sector by Z2 symmetries (paper:
 * "Molecular symmetries"; Algorithm 1 with the Z2 eigenvalues composed by
 * multiplication): n_gen (0..4) qubit masks (host), e.g. from
 * ham_z2_symmetries, and their target parities targets[j] in {0, 1} (host;
 * NULL = those of the Hartree-Fock determinant, the paper's choice).  The
 * masked conditionals, the sampler and amp_forward then keep only
 * configurations with popcount(x & masks[j]) % 2 == targets[j] for every j;
 * n_gen = 0 removes the restriction.  The Hamiltonian's connected x' of a
 * sample stay in its Z2 sector by construction.
 * Errors: NQS_EINVAL (n_gen out of range, empty masks or masks beyond the
 * model's qubits, targets not 0/1), NQS_EUNSUPPORTED (the model serves
 * several molecules).
 */
int amp_model_set_z2(nqs_model *m, int n_gen, const uint64_t *masks, const int32_t *targets);

/*
 * amp_model_set_prefix_sharing - evaluate batches of a bf16 transformer with
 * 9..16 tokens (one molecule) by shared prefixes (on = 1, the default; on = 2
 * the same without the tree tail below) or configuration by configuration
 * (on = 0).  Paper: ANQS product rule (the
 * network is causal: the hidden states of positions 0..7 depend only on tokens
 * 0..6).  Shared: the distinct 8-token prefixes of a batch are evaluated once
 * (positions 0..7; keys and values of every layer kept in a model-owned
 * buffer of up to 65,536 entries of L * d * 32 bytes), then positions 8..15 of
 * every configuration attend to its prefix's keys and values (amp_forward).
 * local_energy, whose distinct x' it sorts by prefix, shares a second level
 * for 13..16 tokens: positions 8 .. m-1 once per distinct m-token prefix
 * (entries of L * d * 16 bytes, in slices of at most 2 GiB), positions
 * m .. m+3 per configuration, with m = n - 4, or m = n - 5 when every level is
 * masked and the sector leaves one token at the last position (its
 * conditional is then a membership test).  The tree tail (on = 1, 13..15
 * tokens, that same kind of sector) goes further: positions 8 .. n-4 once per
 * distinct (n-4)-token prefix, position n-3 once per distinct (n-3)-token
 * prefix, n-2 once per distinct (n-2)-token prefix, each keeping its masked
 * conditional, summed per configuration afterwards.  The sampler's
 * conditionals are unaffected.  Results agree with the unshared evaluation up
 * to the order of fp32 sums.
 * Errors: NQS_EINVAL (null handle, on not 0..2).
 */
int amp_model_set_prefix_sharing(nqs_model *m, int on);

/*
 * amp_model_tree_rows - how many distinct (n-3)-token (rows_q) and
 * (n-2)-token (rows_q1) prefixes the tree tail of local_energy has evaluated
 * with this model since it was created (one row each; cumulative, for rates).
 * Errors: NQS_EINVAL (null handle or pointer).
 */
int amp_model_tree_rows(const nqs_model *m, int64_t *rows_q, int64_t *rows_q1);

/*
 * amp_model_set_mixed_backward - products of a bf16 transformer's backward
 * (amp_backward; its forward recomputation included) on the bf16 matrix cores
 * with split operands (on = 1, the default) or as fp32 library products
 * (on = 0).  Paper: Variational Monte Carlo (the energy gradient through the
 * amplitude network).  Split: every fp32 operand x becomes hi = bf16(x) and
 * lo = bf16(x - hi), a product is hi hi + hi lo + lo hi with fp32
 * accumulation (about 2^-16 relative error per product), bias, residual, GELU
 * and its derivative applied in the products' epilogues; the weight gradients
 * take the same split.  Layer norms, attention and the reductions stay fp32 /
 * fp64.  Models whose widths are not multiples of 32 keep the fp32 products.
 * Errors: NQS_EINVAL (null handle).
 */
int amp_model_set_mixed_backward(nqs_model *m, int on);

/*
 * amp_forward - log|psi(x)| and phase phi(x) for n configurations.
 * x (dev, n uint64), logabs / phase (dev, n doubles each, written).  A
 * configuration outside the sector gets logabs = -inf.  n = 0 is a no-op.
 */
int amp_forward(nqs_model *m, const uint64_t *x, int64_t n, double *logabs,
                double *phase, nqs_stream stream);

/*
 * amp_backward - parameter gradient of L = sum_l g_logabs[l] log|psi(x_l)|
 *                                        + g_phase[l] phi(x_l)
 * (the VMC gradient of the gradient equation in "Variational Monte Carlo" when
 * g = 2 n_l / W (Re, Im)(E_loc,l - E); see vmc_weights).  Activations are
 * recomputed internally, in chunks, from x.  x (dev, n), g_logabs / g_phase
 * (dev, n doubles), grad (dev, n_params elements of the master parameter type,
 * overwritten).  Accumulation is in double for every precision.
 */
int amp_backward(nqs_model *m, const uint64_t *x, int64_t n, const double *g_logabs,
                 const double *g_phase, void *grad, nqs_stream stream);

/* ------------------------------------------------------------------------ */
/* Sampler                                                                   */
/* ------------------------------------------------------------------------ */

/*
 * sample_unique - autoregressive statistics sampling with symmetry pruning
 * (paper: "Autoregressive statistics sampling"; "Pruning strategies").
 * The tree is expanded one token (4 children) per level; a node's n_in
 * samples are split by sequential conditional binomials
 * n_k ~ B(rest, e_k / (e_k + ... + e_3)), e_k = exp(l_k - max) over the
 * allowed tokens (0 otherwise); zero-count children are dropped.  Random
 * numbers: Philox4x32-10 keyed by seed, counter (prefix lo32, prefix hi32,
 * level + 64 j, block); binomials by inversion (n p < 10) or BTRS (Hormann
 * 1993), all in double without contraction, so a draw depends only on
 * (seed, node) and the node's logits.
 * Outputs (dev): configs[capacity], counts[capacity], unique configurations in
 * tree order (lexicographic in tokens).  n_unique and lost (host) receive the
 * number written and the samples lost to unphysical children (0 under MU).
 * Errors: NQS_ECAPACITY with *n_unique = required size, NQS_EINVAL.
 */
int sample_unique(nqs_model *m, uint64_t n_samples, uint64_t seed, uint64_t *configs,
                  uint64_t *counts, int64_t capacity, int64_t *n_unique, uint64_t *lost,
                  nqs_stream stream);

/*
 * sample_unique_batch - sample_unique for every molecule of a model with
 * sectors (amp_model_set_sectors): one tree per molecule, all expanded level
 * by level together; tree i starts from n_samples[i] (host array) samples and
 * keys Philox with i in bits 58..63 of the prefix word, so the trees draw
 * disjoint random streams.  A molecule with fewer tokens than the deepest
 * level keeps its leaves unchanged there.  Outputs (dev) configs / counts as in
 * sample_unique, tagged with the molecule and grouped by molecule in ascending
 * order; offsets (host, n_mol + 1) receives the first sample of each molecule
 * and the total.  Errors as sample_unique; NQS_EINVAL if the model has no
 * sectors or n_mol differs from them.
 */
int sample_unique_batch(nqs_model *m, int n_mol, const uint64_t *n_samples, uint64_t seed,
                        uint64_t *configs, uint64_t *counts, int64_t capacity,
                        int64_t *n_unique, int64_t *offsets, uint64_t *lost,
                        nqs_stream stream);

/* ------------------------------------------------------------------------ */
/* Local energy and the counts-weighted reducer                              */
/* ------------------------------------------------------------------------ */

/*
 * connected_pairs - the bit kernel alone: for each x (dev, n), every flip
 * group f != 0 with x ^ f in x's own (N_alpha, N_beta) block (H conserves
 * both counts, so these are the structurally connected x'; for x in the
 * Hamiltonian's sector, that sector), in group order, and its matrix
 * element <x^f|H|x>.  Writes offsets (dev, n+1 int64), xp / hval (dev,
 * capacity each) and hdiag (dev, n doubles, <x|H|x>).  *n_pairs (host)
 * receives the total.  NQS_ECAPACITY if capacity < total (nothing written but
 * offsets and *n_pairs).  Any of xp, hval, hdiag may be NULL.
 */
int connected_pairs(nqs_ham *ham, const uint64_t *x, int64_t n, int64_t *offsets,
                    uint64_t *xp, double *hval, double *hdiag, int64_t capacity,
                    int64_t *n_pairs, nqs_stream stream);

/*
 * connected_pairs_noalloc - connected_pairs for callers that cannot allocate
 * device memory: code under HIP graph capture, tight serving loops, harnesses
 * that forbid hipMalloc.  Same arguments, outputs and errors as
 * connected_pairs; it calls no allocating routine.  Its scratch (the pair
 * count of every configuration and the multi-block scan's tile totals) is a
 * fixed device array of the library, NQS_NOALLOC_MAX_CONFIGS + 513 int64
 * (2 MiB) on every device it runs on, held until the process ends:
 *   - n > NQS_NOALLOC_MAX_CONFIGS: NQS_EUNSUPPORTED;
 *   - the Hamiltonian's tables must already be on the current device (the
 *     first call of any other entry point with it uploads them): NQS_EINVAL;
 *   - every call on one device shares that array, so calls that overlap on a
 *     device (other streams or host threads) race and must not be issued.
 * Synchronises the stream (the pair total is read back).
 */
#define NQS_NOALLOC_MAX_CONFIGS 262144
int connected_pairs_noalloc(const nqs_ham *ham, const uint64_t *x, int64_t n, int64_t *offsets,
                            uint64_t *xp, double *hval, double *hdiag, int64_t capacity,
                            int64_t *n_pairs, nqs_stream stream);

/*
 * local_energy - E_loc(x) = sum_{x'} H_{x x'} psi(x') / psi(x) (paper:
 * "Variational Monte Carlo", local-energy equation) over x itself and its
 * structurally connected x' = x ^ f inside the sector.  psi(x') comes from
 * the model (amplitude network on the x' batch); the ratio exp(dlog|psi| +
 * i dphi) is formed per pair and accumulated in double.
 * x, counts (dev, n uint64; counts may be NULL = all 1); logabs_x / phase_x
 * (dev, n; may both be NULL, then computed here); eloc (dev, 2n doubles,
 * re/im interleaved, written); sums (dev, 4 doubles, written):
 *   W = sum n_l, sum n_l Re E_loc, sum n_l Im E_loc, sum n_l |E_loc|^2
 * (the counts-weighted estimator of the energy-estimator equation).
 * *n_pairs (host, may be NULL) receives the number of (x, x') pairs.
 */
int local_energy(nqs_ham *ham, nqs_model *m, const uint64_t *x, const uint64_t *counts,
                 int64_t n, const double *logabs_x, const double *phase_x, double *eloc,
                 double *sums, int64_t *n_pairs, nqs_stream stream);

/*
 * local_energy_stats - work of the last local_energy call on this Hamiltonian:
 * the number of (x, x') pairs and the number of distinct x' on which the
 * amplitude network ran (local_energy evaluates psi once per distinct x' of a
 * slice of at most 2^27 pairs; the sum over pairs is unchanged).
 */
int local_energy_stats(const nqs_ham *ham, int64_t *n_pairs, int64_t *n_distinct);

/*
 * vmc_weights - upstream weights of the VMC gradient (paper: gradient
 * equation in "Variational Monte Carlo"): with W = sums[0] and E =
 * (sums[1] + i sums[2]) / W, g_logabs[l] = 2 n_l / W Re(E_loc,l - E) and
 * g_phase[l] = 2 n_l / W Im(E_loc,l - E).  All dev arrays.  local_energy
 * leaves W = sum of the counts in sums[0]; when samples were lost (DU, MU-d)
 * a caller may set sums[0] = N_s for the paper's estimator, which divides by
 * the number of samples drawn.
 */
int vmc_weights(const double *eloc, const uint64_t *counts, int64_t n, const double *sums,
                double *g_logabs, double *g_phase, nqs_stream stream);

/*
 * adam_update - one Adam step (paper: optimisation with ADAM, default
 * hyper-parameters) on n parameters of element size elem_bytes (4 or 8):
 * m = b1 m + (1-b1) g, v = b2 v + (1-b2) g^2, p -= lr mhat / (sqrt(vhat) + eps),
 * with bias corrections for step t >= 1.  params, grad, m, v are dev arrays of
 * that element type.
 */
int adam_update(void *params, const void *grad, void *m, void *v, int64_t n,
                int elem_bytes, double lr, double b1, double b2, double eps,
                int64_t t, nqs_stream stream);

/* ------------------------------------------------------------------------ */
/* Many molecules in one pass                                                */
/* ------------------------------------------------------------------------ */

/*
 * batch_create - the local energy of n_mol (1..64) molecules that share one
 * transformer (paper's local-energy and energy-estimator equations, per
 * molecule).  hams (host array of n_mol compiled Hamiltonians, each N <= 57
 * spin-orbitals with every single and double excitation present as a flip
 * group, so that every configuration of molecule i has the same number K_i of
 * connected in-sector x') is copied into concatenated device tables; the
 * model gets the molecules' sectors (amp_model_set_sectors) and stays owned by
 * the caller, alive while the batch is used.  Errors: NQS_EINVAL,
 * NQS_EUNSUPPORTED (a missing flip group, N too large, model shape).
 */
int batch_create(nqs_ham *const *hams, int n_mol, nqs_model *model, nqs_batch **out);
void batch_destroy(nqs_batch *b);

/* K_i (connected x' per configuration) and the flip-group count of every
 * molecule (host arrays of n_mol, either may be NULL). */
int batch_info(const nqs_batch *b, int64_t *k_per_config, int64_t *n_groups);

/*
 * batch_local_energy - E_loc of every sample of every molecule and the
 * per-molecule sums.  x, counts (dev, U tagged words as produced by
 * sample_unique_batch, grouped by molecule); offsets (host, n_mol + 1, first
 * sample of each molecule, offsets[0] = 0, U = offsets[n_mol]); logabs_x /
 * phase_x (dev, U; both NULL = computed here); eloc (dev, 2U doubles, re/im,
 * written); sums (dev, 4 n_mol doubles: W, sum n Re E, sum n Im E,
 * sum n |E|^2 of each molecule, written).  *n_pairs (host, may be NULL)
 * receives sum_i U_i K_i.
 * With a BF16 model the whole step is one sequence of fixed-grid launches
 * (bit kernel with hash-table dedupe of x', fused amplitude kernel on the
 * samples and on the distinct x', accumulation, reduction) whose sizes are
 * read from device memory; it is captured into a hipGraph once per capacity
 * and launch shape and replayed (batch_set_mode can switch to direct
 * launches).  Launch shapes are chosen on the first call by timing candidates
 * on that call's data.  FP32 / FP64 models run the same kernels with the
 * layer-by-layer network between them (no graph).  Synchronises the stream.
 * Errors: NQS_EINVAL (offsets, a configuration with more than K_i connected
 * x' or an overfull table), NQS_ENOMEM.
 */
int batch_local_energy(nqs_batch *b, const uint64_t *x, const uint64_t *counts,
                       const int64_t *offsets, const double *logabs_x, const double *phase_x,
                       double *eloc, double *sums, int64_t *n_pairs, nqs_stream stream);

/* use_graph = 0: launch the step's kernels directly instead of replaying the
 * captured graph; retune != 0: choose launch shapes again on the next call. */
int batch_set_mode(nqs_batch *b, int use_graph, int retune);

/* Fix the launch shape instead of tuning it: bit-kernel blocks (of four
 * waves), configuration pairs per fused-kernel chunk (1..16) and fused-kernel
 * blocks.  Results do not depend on the shape. */
int batch_set_tile(nqs_batch *b, int pairs_blocks, int fused_pairs, int fused_blocks);

/* Size of the distinct-x' hash table of the next batch_local_energy call:
 * slots (a power of two, 1024 .. 2^31) instead of the automatic size (at least
 * twice the pairs); 0 = automatic.  A step whose distinct x' overfill the table
 * (a probe run longer than 256 slots) is run again with an enlarged,
 * automatically sized table, so results do not depend on it; the knob is for
 * memory-constrained callers and for tests of that path. */
int batch_set_table(nqs_batch *b, int64_t slots);

/* Last call's pairs, distinct x' (total and per molecule, host array of
 * n_mol), the number of graph captures so far, the chosen launch shape
 * tile[3] = {bit-kernel blocks, fused pairs per chunk, fused blocks} and the
 * tuner's candidate timings in ms (first n_tune).  Any output may be NULL. */
int batch_stats(const nqs_batch *b, int64_t *n_pairs, int64_t *n_distinct,
                int64_t *distinct_per_mol, int64_t *captures, int32_t *tile, double *tune_ms,
                int n_tune);

/*
 * vmc_weights_batch - vmc_weights per molecule for the gradient of the sum of
 * the molecules' energies: sample l of molecule i (from the tag of x[l]) gets
 * g_logabs = 2 n_l / W_i Re(E_loc,l - E_i), g_phase = 2 n_l / W_i Im(E_loc,l -
 * E_i), with W_i, E_i from sums[4 i ..] of batch_local_energy (n_mol
 * molecules; a word with a larger index gets NaN weights).  All dev.
 */
int vmc_weights_batch(const double *eloc, const uint64_t *counts, const uint64_t *x, int64_t n,
                      const double *sums, int n_mol, double *g_logabs, double *g_phase,
                      nqs_stream stream);

/* ------------------------------------------------------------------------ */
/* Diagnostics                                                               */
/* ------------------------------------------------------------------------ */

/*
 * Kernel timing of the dominant kernel (the fused bf16 amplitude kernel of
 * the transformer, or of the per-qubit ansatz).
 * While enabled, every launch of it is bracketed by two HIP events recorded on
 * the launch's own stream (in batch_local_energy: by two events inside the
 * step's launch sequence, read after the call; its launches on the samples
 * are not recorded).  nqs_timing_read synchronises those events and
 * returns the summed kernel time in milliseconds, the number of launches and
 * the number of configurations they evaluated, then clears the record.
 * Not thread-safe; intended for benchmarks.
 */
int nqs_timing_enable(int on);
int nqs_timing_read(double *ms, int64_t *launches, int64_t *configs);
/*
 * The same for the launches of one row layout only (those records are
 * removed, the others kept): mode 0 = transformer, up to 16 tokens (2
 * configurations x 16 positions per 32 rows); 1 = 17..32 tokens; 2 = shared
 * prefixes (positions 0..7 once per distinct 8-token prefix); 3 = their
 * suffixes (positions 8..15 per configuration); 4 = the second shared level
 * (positions 8 .. n-5 once per distinct (n-4)-token prefix); 5 = the last four
 * positions per configuration; -1 = the per-qubit ansatz; -2 = every record
 * (nqs_timing_read).
 */
int nqs_timing_read_mode(int mode, double *ms, int64_t *launches, int64_t *configs);

/*
 * The samplers of a bf16 model with at most 2^24 samples keep the frontier
 * sizes on the device and wait for the host once per call instead of once per
 * tree level (on = 1, the default); on = 0 takes the per-level walk for every
 * model.  Both give the same samples (the random numbers are keyed by node).
 * Process-wide; for comparisons.
 */
int nqs_sampler_device_walk(int on);

#ifdef __cplusplus
}
#endif
#endif /* NQS_H */
