"""Autoregressive statistics sampling with symmetry pruning (paper:
"Autoregressive statistics sampling"; "Pruning strategies").

The tree is walked level by level.  A node is a token prefix x_<p with the
number n_in of samples that reached it.  Its n_in samples are split over the
four children by one multinomial draw, done as sequential conditional binomials
(the paper's binary rule n_L ~ B(n_in, p), n_R = n_in - n_L, generalised to
four children).  Children that receive no samples are dropped, so the network
is only evaluated on unique prefixes.

Strategies:

* ``MU``  (Mask-Unphysical): the split uses the masked conditional, so every
  sample goes to a physical child and sum(counts) = N_s.
* ``DU``  (Discard-Unphysical): the split uses the unmasked conditional and
  samples sent to unphysical children are lost.
* ``MUd`` (MU-d): MU on levels p < n - d, DU on the last d levels.

Random numbers: Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11) keyed by
the 64-bit seed, counter (prefix low 32 bits, prefix high 32 bits,
p + 64 j, block) where j is which of the three conditional binomials of the
node is drawn and block counts Philox calls.  Each call yields two uniforms.
Results therefore depend only on (seed, node), not on processing order.
When several trees are drawn with one seed (one per molecule of a batch),
tree number ``stream`` puts ``stream << 58`` into the prefix field of the
counter, so the trees use disjoint counters.

Binomial draws (all float64, no fused multiply-add):

* n p < 10 (p <= 1/2 after symmetry): inversion by sequential search with
  the pmf recurrence f(k) = f(k-1) ((n+1) s / k - s), s = p / q.
* otherwise BTRS, the transformed-rejection-with-squeeze method of
  W. Hormann, "The generation of binomial random variates", J. Statist.
  Comput. Simul. 46 (1993), with log k! from a table for k < 10 and the
  Stirling series with three correction terms above.
"""
import math

import numpy as np
import torch

MASK32 = 0xFFFFFFFF
PHILOX_M0, PHILOX_M1 = 0xD2511F53, 0xCD9E8D57
PHILOX_W0, PHILOX_W1 = 0x9E3779B9, 0xBB67AE85


def philox4x32_10(ctr, key):
    c0, c1, c2, c3 = ctr
    k0, k1 = key
    for r in range(10):
        if r:
            k0 = (k0 + PHILOX_W0) & MASK32
            k1 = (k1 + PHILOX_W1) & MASK32
        p0 = PHILOX_M0 * c0
        p1 = PHILOX_M1 * c2
        c0, c1, c2, c3 = ((p1 >> 32) ^ c1 ^ k0, p1 & MASK32,
                          (p0 >> 32) ^ c3 ^ k1, p0 & MASK32)
    return c0, c1, c2, c3


def to_unit(w_hi, w_lo):
    """Two 32-bit words to a double strictly inside (0, 1): the top 26 bits of
    each word form k < 2^52 and u = (k + 0.5) / 2^52, exact in float64."""
    return ((w_hi >> 6) * 67108864.0 + (w_lo >> 6) + 0.5) * (1.0 / 4503599627370496.0)


class UniformStream:
    def __init__(self, seed, prefix, level, j):
        self.key = (seed & MASK32, (seed >> 32) & MASK32)
        self.ctr = [prefix & MASK32, (prefix >> 32) & MASK32, level + 64 * j, 0]
        self.buf = []

    def __call__(self):
        if not self.buf:
            w = philox4x32_10(tuple(self.ctr), self.key)
            self.ctr[3] += 1
            self.buf = [to_unit(w[2], w[3]), to_unit(w[0], w[1])]
        return self.buf.pop()


_LOGFACT_SMALL = [math.log(float(math.factorial(k))) for k in range(10)]
_HALF_LOG_2PI = 0.5 * math.log(2.0 * math.pi)


def log_factorial(k):
    if k < 10:
        return _LOGFACT_SMALL[k]
    k1 = k + 1.0
    r = 1.0 / (k1 * k1)
    return ((k + 0.5) * math.log(k1) - k1 + _HALF_LOG_2PI
            + (1.0 / 12.0 - (1.0 / 360.0 - (1.0 / 1260.0) * r) * r) / k1)


def _binomial_inversion(n, p, uni):
    q = 1.0 - p
    s = p / q
    a = (n + 1) * s
    r0 = math.pow(q, n)
    while True:
        r = r0
        u = uni()
        k = 0
        while u >= r:
            u -= r
            k += 1
            if k > n:
                break
            r *= a / k - s
        if k <= n:
            return k


def _binomial_btrs(n, p, uni):
    q = 1.0 - p
    spq = math.sqrt(n * p * q)
    b = 1.15 + 2.53 * spq
    a = -0.0873 + 0.0248 * b + 0.01 * p
    c = n * p + 0.5
    vr = 0.92 - 4.2 / b
    alpha = (2.83 + 5.1 / b) * spq
    lpq = math.log(p / q)
    m = math.floor((n + 1) * p)
    h = log_factorial(m) + log_factorial(n - m)
    while True:
        u = uni() - 0.5
        v = uni()
        us = 0.5 - abs(u)
        k = math.floor((2.0 * a / us + b) * u + c)
        if k < 0 or k > n:
            continue
        if us >= 0.07 and v <= vr:
            return k
        v = math.log(v * alpha / (a / (us * us) + b))
        if v <= h - log_factorial(k) - log_factorial(n - k) + (k - m) * lpq:
            return k


def binomial(n, p, uni):
    """One draw of B(n, p) from the uniform stream ``uni``."""
    if n == 0 or p <= 0.0:
        return 0
    if p >= 1.0:
        return n
    flip = p > 0.5
    pp = 1.0 - p if flip else p
    k = _binomial_inversion(n, pp, uni) if n * pp < 10.0 else _binomial_btrs(n, pp, uni)
    return n - k if flip else k


def split_counts(n_in, weights, seed, prefix, level):
    """Multinomial split of n_in over four children with unnormalised weights
    e_k (e_k = 0 exactly for excluded children) as sequential binomials:
    child k takes B(rest, e_k / (e_k + ... + e_3))."""
    out = [0, 0, 0, 0]
    rest = n_in
    for k in range(3):
        if rest == 0:
            break
        tail = weights[k]
        for j in range(k + 1, 4):
            tail = tail + weights[j]
        if weights[k] == tail:
            out[k] = rest
        else:
            out[k] = binomial(rest, weights[k] / tail, UniformStream(seed, prefix, level, k))
        rest -= out[k]
    out[3] += rest
    return out


def child_weights(logits, allowed):
    """exp(l_k - max) over the allowed tokens, 0 elsewhere (float64)."""
    m = max(logits[k] for k in range(4) if allowed[k])
    return [math.exp(logits[k] - m) if allowed[k] else 0.0 for k in range(4)]


def sample_tree(model, n_samples, seed, strategy="MU", d=0, stream=0):
    """Returns ``(configs, counts, lost)``: unique configurations (ints) in tree
    order (lexicographic in the token sequence), their counts, and the number
    of samples lost to unphysical children (0 under MU)."""
    tag = stream << 58
    n, sec = model.n, model.sector
    mask_levels = {"MU": n, "DU": 0, "MUd": n - d}[strategy]
    frontier = [(0, n_samples, 0, 0)]     # (prefix bits, count, alpha, beta)
    lost = 0
    for p in range(n):
        with torch.no_grad():
            if hasattr(model, "token_logits"):      # per-qubit ansatz: token log-probabilities
                lg = model.token_logits([f[0] for f in frontier], p).numpy()
            else:
                toks = torch.zeros((len(frontier), n), dtype=torch.long)
                for i, (x, _, _, _) in enumerate(frontier):
                    for q in range(p):
                        toks[i, q] = ((x >> (2 * q)) & 1) + 2 * ((x >> (2 * q + 1)) & 1)
                lg = model.logits(toks)[:, p, :].numpy()
        nxt = []
        for i, (x, cnt, a, b) in enumerate(frontier):
            if getattr(sec, "general", False):         # any additive symmetries
                phys = sec.child_mask_state(p, sec.prefix_state(x, p))
            else:
                phys = sec.child_mask(p, a, b, sec.prefix_z2(x, p))
            allowed = phys if p < mask_levels else [True] * 4
            w = child_weights([float(v) for v in lg[i]], allowed)
            split = split_counts(cnt, w, seed, tag | x, p)
            for k in range(4):
                if split[k] == 0:
                    continue
                if not phys[k]:
                    lost += split[k]
                    continue
                nxt.append((x | ((k & 1) << (2 * p)) | ((k >> 1) << (2 * p + 1)),
                            split[k], a + (k & 1), b + (k >> 1)))
        frontier = nxt
    return [f[0] for f in frontier], [f[1] for f in frontier], lost
