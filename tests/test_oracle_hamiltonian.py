"""Pins of the oracle's Hamiltonian matrix elements."""
from math import comb

import numpy as np
import pytest

from oracle.hamiltonian import (hf_energy, literal_row, sector_matrix,
                                slater_condon_row)
from oracle.sector import Sector, hf_config
from synth import make_integrals


def k_closed_form(n, na, nb):
    """Spin-conserving singles + doubles of any determinant of the sector."""
    return (na * (n - na) + nb * (n - nb) + comb(na, 2) * comb(n - na, 2)
            + comb(nb, 2) * comb(n - nb, 2) + na * (n - na) * nb * (n - nb))


@pytest.fixture(scope="module")
def tiny():
    h, eri = make_integrals(6, 12, 1)
    sec = Sector(6, 2, 2)
    return h, eri, sec, sec.enumerate()


def test_integrals_symmetry_bitwise():
    h, eri = make_integrals(6, 12, 1)
    assert np.array_equal(h, h.T)
    for perm in [(1, 0, 2, 3), (0, 1, 3, 2), (2, 3, 0, 1), (3, 2, 1, 0)]:
        assert np.array_equal(eri, eri.transpose(perm))
    assert np.all(np.diag(h) == -2.0 + 0.1 * np.arange(6))
    # factorised two-electron tensor is positive semidefinite as a (pq),(rs) matrix
    assert np.linalg.eigvalsh(eri.reshape(36, 36)).min() > -1e-12


def test_literal_equals_slater_condon(tiny):
    h, eri, sec, basis = tiny
    Hl = sector_matrix(h, eri, basis, route="literal")
    Hs = sector_matrix(h, eri, basis, route="slater_condon")
    assert np.max(np.abs(Hl - Hs)) < 1e-13
    assert np.max(np.abs(Hs - Hs.T)) < 1e-14


def test_literal_row_stays_in_sector(tiny):
    h, eri, sec, basis = tiny
    for x in basis[::17]:
        for xp, v in literal_row(h, eri, x).items():
            assert sec.contains(xp) or abs(v) < 1e-15


def test_hf_diagonal_is_textbook_hf_energy():
    for n, na, nb, rank, seed in [(6, 2, 2, 12, 1), (10, 5, 5, 20, 2), (15, 7, 7, 30, 3), (6, 3, 1, 6, 9)]:
        h, eri = make_integrals(n, rank, seed)
        xs, vals = slater_condon_row(h, eri, hf_config(n, na, nb))
        assert abs(vals[0] - hf_energy(h, eri, na, nb)) < 1e-12


@pytest.mark.parametrize("n,na,nb,expect", [(6, 2, 2, 92), (10, 5, 5, 875), (15, 7, 7, 4424)])
def test_connected_count(n, na, nb, expect):
    h, eri = make_integrals(n, 2 * n, n)
    sec = Sector(n, na, nb)
    assert k_closed_form(n, na, nb) == expect
    rng = np.random.default_rng(0)
    basis_sample = [hf_config(n, na, nb)]
    if n <= 10:
        basis = sec.enumerate()
        basis_sample += [basis[i] for i in rng.integers(0, len(basis), 3)]
    for x in basis_sample:
        xs, _ = slater_condon_row(h, eri, x)
        assert len(xs) == expect + 1 and len(set(xs)) == expect + 1
        assert all(sec.contains(xp) for xp in xs)


def test_one_electron_sector_is_h():
    """One alpha electron: H restricted to the sector is the matrix h itself."""
    h, eri = make_integrals(5, 10, 4)
    basis = Sector(5, 1, 0).enumerate()          # x = 1 << 2p, ascending in p
    H = sector_matrix(h, eri, basis)
    assert np.max(np.abs(H - h)) < 1e-14


def test_noninteracting_fermions():
    """eri = 0: ground energy is the sum of the lowest orbital energies per spin
    (pins the fermionic signs of one-body hopping)."""
    h, _ = make_integrals(6, 12, 1)
    h = h + np.diag(np.linspace(0.0, 0.3, 6))
    lam = np.linalg.eigvalsh(h)
    basis = Sector(6, 2, 3).enumerate()
    H = sector_matrix(h, np.zeros((6,) * 4), basis)
    w = np.linalg.eigvalsh(H)
    assert abs(w[0] - (lam[:2].sum() + lam[:3].sum())) < 1e-12
    # whole spectrum: all sums of 2 distinct + 3 distinct orbital energies
    from itertools import combinations
    spec = sorted(sum(lam[list(a)]) + sum(lam[list(b)])
                  for a in combinations(range(6), 2) for b in combinations(range(6), 3))
    assert np.max(np.abs(np.sort(w) - np.array(spec))) < 1e-11


def test_two_electron_opposite_spin():
    """1 alpha + 1 beta: spectrum equals that of h(x)1 + 1(x)h + V with
    V[(p'q'),(pq)] = (p'p|q'q) on the product space (pins the two-body index order)."""
    n = 4
    h, eri = make_integrals(n, 8, 7)
    H = sector_matrix(h, eri, Sector(n, 1, 1).enumerate())
    I = np.eye(n)
    V = np.einsum("abcd->acbd", eri).reshape(n * n, n * n)    # [(p'q'), (p q)] = (p'p|q'q)
    M = np.kron(h, I) + np.kron(I, h) + V
    assert np.max(np.abs(np.linalg.eigvalsh(H) - np.linalg.eigvalsh(M))) < 1e-12


def test_two_electron_same_spin():
    """2 alpha electrons: spectrum equals h(x)1 + 1(x)h + V on the antisymmetric
    subspace (pins the exchange sign)."""
    n = 5
    h, eri = make_integrals(n, 10, 8)
    H = sector_matrix(h, eri, Sector(n, 2, 0).enumerate())
    I = np.eye(n)
    V = np.einsum("abcd->acbd", eri).reshape(n * n, n * n)
    M = np.kron(h, I) + np.kron(I, h) + V
    S = np.zeros((n * n, n * n))
    for p in range(n):
        for q in range(n):
            S[q * n + p, p * n + q] = 1.0
    A = (np.eye(n * n) - S) / 2
    w, U = np.linalg.eigh(A)
    Q = U[:, w > 0.5]
    assert np.max(np.abs(np.linalg.eigvalsh(H) - np.linalg.eigvalsh(Q.T @ M @ Q))) < 1e-12
