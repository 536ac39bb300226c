"""Matrix elements of the molecular Hamiltonian (paper: "System description", H_SQ).

Conventions (readings of the paper):

* Spin-orbital j = 2p + s, p the spatial orbital, s = 0 for alpha (spin up,
  the odd orbitals of Appendix A when counted from 1) and s = 1 for beta.
  Bit j of a Python int is the occupation x_j.
* H = sum_{pq,s} h_pq a+_ps a_qs
      + 1/2 sum_{pqrs,st} (pq|rs) a+_ps a+_rt a_st a_qs + e_core,
  with (pq|rs) the chemists'-notation two-electron integral.  This fixes the
  normalisation and index order that the H_SQ equation leaves open.
* |x> = prod over j ascending (leftmost first) of (a+_j)^{x_j} |vac>, so
  a_j |x> = (-1)^{popcount(x & ((1<<j)-1))} |x - e_j>, which is what the
  Jordan-Wigner map (occupation-number interpretation kept) gives.

Two independent routes:

* ``literal_row``   applies every creation/annihilation term to |x> (tiny N).
* ``slater_condon_row`` uses the Slater-Condon rules for the diagonal, single
  and double excitations, with the phase of each excitation found by applying
  its operator string to |x>.
"""
import numpy as np


def apply_ops(ops, x):
    """Apply an operator product to |x>.

    ``ops`` lists ``(is_creation, j)`` left to right as written; the rightmost
    acts first.  Returns ``(sign, x')`` or ``None`` if the result vanishes.
    """
    sign = 1
    for is_cre, j in reversed(ops):
        occ = (x >> j) & 1
        if is_cre == bool(occ):
            return None
        if bin(x & ((1 << j) - 1)).count("1") & 1:
            sign = -sign
        x ^= (1 << j)
    return sign, x


def literal_row(h, eri, x, e_core=0.0):
    """<x'|H|x> for all x' by applying each term of H to |x>.  Returns a dict."""
    n = h.shape[0]
    row = {}

    def add(key, val):
        row[key] = row.get(key, 0.0) + val

    add(x, e_core)
    for s in (0, 1):
        for p in range(n):
            for q in range(n):
                r = apply_ops([(True, 2 * p + s), (False, 2 * q + s)], x)
                if r is not None:
                    add(r[1], r[0] * h[p, q])
    for s in (0, 1):
        for t in (0, 1):
            for p in range(n):
                for q in range(n):
                    if not (x >> (2 * q + s)) & 1:
                        continue
                    for r_ in range(n):
                        for s_ in range(n):
                            res = apply_ops([(True, 2 * p + s), (True, 2 * r_ + t),
                                             (False, 2 * s_ + t), (False, 2 * q + s)], x)
                            if res is not None:
                                add(res[1], 0.5 * res[0] * eri[p, q, r_, s_])
    return row


def _g(eri, P, Q, R, S):
    """Spin-orbital <PQ|RS> = (pr|qs) delta(s_P, s_R) delta(s_Q, s_S)."""
    if (P & 1) != (R & 1) or (Q & 1) != (S & 1):
        return 0.0
    return eri[P >> 1, R >> 1, Q >> 1, S >> 1]


def _h1(h, P, Q):
    return h[P >> 1, Q >> 1] if (P & 1) == (Q & 1) else 0.0


def slater_condon_row(h, eri, x, e_core=0.0):
    """<x'|H|x> for x itself and every spin-conserving single and double.

    Returns ``(xs, vals)``: x' values (ints) and matrix elements, x itself first.
    Every excitation that keeps the alpha and beta electron counts is listed,
    whatever its value (the connected set is structural).
    """
    N = 2 * h.shape[0]
    occ = [j for j in range(N) if (x >> j) & 1]
    vir = [j for j in range(N) if not (x >> j) & 1]
    diag = e_core
    for i in occ:
        diag += _h1(h, i, i)
    for i in occ:
        for j in occ:
            diag += 0.5 * (_g(eri, i, j, i, j) - _g(eri, i, j, j, i))
    xs, vals = [x], [diag]
    for i in occ:
        for a in vir:
            if (i & 1) != (a & 1):
                continue
            v = _h1(h, a, i)
            for j in occ:
                v += _g(eri, a, j, i, j) - _g(eri, a, j, j, i)
            sgn, xp = apply_ops([(True, a), (False, i)], x)
            xs.append(xp)
            vals.append(sgn * v)
    for ii, i in enumerate(occ):
        for j in occ[ii + 1:]:
            for aa, a in enumerate(vir):
                for b in vir[aa + 1:]:
                    if sorted([i & 1, j & 1]) != sorted([a & 1, b & 1]):
                        continue
                    v = _g(eri, a, b, i, j) - _g(eri, a, b, j, i)
                    sgn, xp = apply_ops([(True, a), (True, b), (False, j), (False, i)], x)
                    xs.append(xp)
                    vals.append(sgn * v)
    return xs, vals


def sector_matrix(h, eri, basis, route="slater_condon", e_core=0.0):
    """Dense H restricted to ``basis`` (a sorted list of ints)."""
    index = {b: k for k, b in enumerate(basis)}
    H = np.zeros((len(basis), len(basis)))
    for c, x in enumerate(basis):
        if route == "literal":
            items = literal_row(h, eri, x, e_core).items()
        else:
            items = zip(*slater_condon_row(h, eri, x, e_core))
        for xp, v in items:
            if xp in index:
                H[index[xp], c] += v
            elif v != 0.0:
                raise AssertionError("H leaves the sector")
    return H


def hf_energy(h, eri, n_alpha, n_beta):
    """Textbook closed-shell-or-not HF determinant energy:
    sum_occ h + 1/2 sum_occ,occ [J - delta_spin K] with spatial integrals."""
    occ = [(p, 0) for p in range(n_alpha)] + [(p, 1) for p in range(n_beta)]
    e = sum(h[p, p] for p, _ in occ)
    for p, s in occ:
        for q, t in occ:
            e += 0.5 * eri[p, p, q, q]
            if s == t:
                e -= 0.5 * eri[p, q, q, p]
    return e


# ------------------------------------------------------------------ Z2 symmetries
# (paper: "Molecular symmetries").  A Z2 symmetry is a tensor product of
# identities and Pauli Z on a set m of qubits that commutes with H.  Under the
# Jordan-Wigner map a term a+_P a+_R a_S a_Q (or a+_P a_Q) carries X / Y on the
# qubits where its operators do not cancel, f = e_P ^ e_R ^ e_S ^ e_Q, and Z
# (or identity) elsewhere; Z^m commutes with it iff m and f share an even
# number of qubits.  The symmetries of H are therefore the m orthogonal over
# GF(2) to the flip masks f of every term with a nonzero coefficient.

def term_flip_masks(h, eri):
    """The set of flip masks f of the terms of H with nonzero coefficients."""
    n = h.shape[0]
    masks = set()
    for p in range(n):
        for q in range(n):
            if h[p, q] != 0.0:
                for s in (0, 1):
                    masks.add((1 << (2 * p + s)) ^ (1 << (2 * q + s)))
    for p in range(n):
        for q in range(n):
            for r in range(n):
                for t in range(n):
                    if eri[p, q, r, t] == 0.0:
                        continue
                    for s in (0, 1):
                        for u in (0, 1):
                            # a+_{p s} a+_{r u} a_{t u} a_{q s}
                            masks.add((1 << (2 * p + s)) ^ (1 << (2 * r + u)) ^
                                      (1 << (2 * t + u)) ^ (1 << (2 * q + s)))
    masks.discard(0)
    return masks


def gf2_null_space(rows, nbits):
    """Basis of {m : popcount(m & f) even for every f in rows} over GF(2):
    reduced row echelon form of the rows, one basis vector per free column."""
    pivots = {}                                  # pivot column -> reduced row
    for f in rows:
        for c, r in pivots.items():
            if (f >> c) & 1:
                f ^= r
        if f == 0:
            continue
        c = f.bit_length() - 1                   # highest set bit as the pivot
        for c2 in list(pivots):                  # keep the other rows reduced
            if (pivots[c2] >> c) & 1:
                pivots[c2] ^= f
        pivots[c] = f
    basis = []
    for free in range(nbits):
        if free in pivots:
            continue
        m = 1 << free
        for c, r in pivots.items():              # solve each pivot bit from the free one
            if (r >> free) & 1:
                m |= 1 << c
        basis.append(m)
    return basis


def z2_symmetries(h, eri):
    """A basis (qubit masks) of the Z2 symmetries of H: the null space of the
    flip masks of its terms.  It includes the parities of the alpha and beta
    electron numbers (all even / all odd qubits)."""
    return gf2_null_space(term_flip_masks(h, eri), 2 * h.shape[0])


def gf2_span_key(vectors):
    """A canonical description of the span of ``vectors`` (its reduced row
    echelon basis, sorted), to compare two bases of the same space."""
    pivots = {}
    for f in vectors:
        for c, r in pivots.items():
            if (f >> c) & 1:
                f ^= r
        if f == 0:
            continue
        c = f.bit_length() - 1
        for c2 in list(pivots):
            if (pivots[c2] >> c) & 1:
                pivots[c2] ^= f
        pivots[c] = f
    return tuple(sorted(pivots.values()))
