"""Seeded one- and two-electron integrals with the structure of a small molecule.

Recipe (spatial orbitals p, q, r, s are 0-indexed, n of them):

* ``h[p, p] = -2 + 0.1 p`` (no noise); for p < q, drawn row-major over the
  upper triangle, ``h[p, q] = N(0, 0.1) * exp(-|p - q| / 3)`` and mirrored.
* ``rank`` symmetric factors ``L^k`` (k = 0 .. rank-1, drawn in that order
  after h); for p <= q, row-major, ``L^k[p, q] = N(0, 0.3) * exp(-|p - q| / 2)``
  and mirrored.
* ``eri[p, q, r, s] = sum_k L^k[p, q] L^k[r, s]`` (chemists' notation (pq|rs)),
  accumulated in the fixed order k = 0, 1, ... so that all eight symmetric
  copies of every element are bitwise identical.

``N(0, s)`` is a normal draw with standard deviation ``s`` from
``numpy.random.default_rng(seed)`` (PCG64).  The factorised form makes the
two-electron tensor positive semidefinite as a (pq) x (rs) matrix, as real
electron-repulsion integrals are.

Point-group structure (optional): ``irreps[p]`` labels spatial orbital p with
an element of an abelian group Z2^K written as a K-bit integer (the irreps of
a molecule's largest abelian point subgroup, e.g. C2v or D2h).  The draws are
made as above and then ``h[p, q]`` is zeroed unless ``irreps[p] == irreps[q]``,
and ``L^k[p, q]`` unless ``irreps[p] ^ irreps[q] == k % 2^K``, so that
``(pq|rs)`` vanishes unless ``irreps[p] ^ irreps[q] ^ irreps[r] ^ irreps[s]``
is 0: the selection rules of a molecule with that point group.
"""
import numpy as np


def make_integrals(n, rank, seed, irreps=None):
    """Return ``(h, eri)`` as float64 arrays of shapes (n, n) and (n, n, n, n)."""
    rng = np.random.default_rng(seed)
    h = np.zeros((n, n))
    for p in range(n):
        h[p, p] = -2.0 + 0.1 * p
    for p in range(n):
        for q in range(p + 1, n):
            v = rng.normal(0.0, 0.1) * np.exp(-abs(p - q) / 3.0)
            h[p, q] = v
            h[q, p] = v
    factors = np.zeros((rank, n, n))
    for k in range(rank):
        for p in range(n):
            for q in range(p, n):
                v = rng.normal(0.0, 0.3) * np.exp(-abs(p - q) / 2.0)
                factors[k, p, q] = v
                factors[k, q, p] = v
    if irreps is not None:
        g = np.asarray(irreps, dtype=np.int64)
        assert g.shape == (n,) and g.min() >= 0
        order = 1
        while order <= g.max():
            order *= 2
        h = np.where(g[:, None] == g[None, :], h, 0.0)
        for k in range(rank):
            factors[k] = np.where((g[:, None] ^ g[None, :]) == k % order, factors[k], 0.0)
    flat = factors.reshape(rank, n * n)
    v = np.zeros((n * n, n * n))
    for k in range(rank):
        v += np.multiply.outer(flat[k], flat[k])
    return h, v.reshape(n, n, n, n)
