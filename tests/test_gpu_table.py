"""The network-free amplitude (NQS_MODEL_TABLE) through the C ABI: local energy
against the literal full matrix and the zero-variance property at the exact
ground vector (local-energy equation), the sampler against exact Born
probabilities, lookups outside the basis, and the backward's scatter."""
import numpy as np
import pytest
import torch
from scipy.stats import chi2

from oracle.ed import ground_state
from oracle.hamiltonian import sector_matrix
from oracle.sector import Sector
from synth import make_integrals

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def nqs():
    from paper_2310_04166_amd import nqs as mod
    mod.lib()
    return mod


@pytest.fixture(scope="module")
def tiny():
    h, eri = make_integrals(6, 12, 1)
    sec = Sector(6, 2, 2)
    basis = sec.enumerate()
    H = sector_matrix(h, eri, basis, route="literal")
    return h, eri, sec, basis, H


def dev(a):
    return torch.as_tensor(np.asarray(a, dtype=np.uint64).view(np.int64)).cuda()


def test_table_zero_variance_at_ground_vector(nqs, tiny):
    """psi = the exact ground vector of the 225-determinant sector (12
    spin-orbitals, 2+2 electrons): E_loc(x) = E_0 within 1e-10 on every
    configuration where |psi| > 1e-6; the estimator's variance vanishes."""
    h, eri, sec, basis, H = tiny
    e0, v0 = ground_state(H)
    keep = np.abs(v0) > 1e-6
    la = np.where(keep, np.log(np.abs(v0) + 1e-300), -np.inf)
    ph = np.where(v0 < 0, np.pi, 0.0)
    m = nqs.table_model(6, 2, 2, basis, la, ph)
    ham = nqs.ham_compile(h, eri, 2, 2)
    xs = [x for x, k in zip(basis, keep) if k]
    eloc, sums, _ = nqs.local_energy(ham, m, dev(xs))
    e = eloc.cpu().numpy()
    s = sums.cpu().numpy()
    print(f"E_0 {e0:.12f}: max |E_loc - E_0| {np.max(np.abs(e - e0)):.1e} over {len(xs)}")
    assert np.max(np.abs(e - e0)) < 1e-10
    W, E = s[0], s[1] / s[0]
    assert abs(E - e0) < 1e-10 and s[3] / W - E * E < 1e-8


def test_table_eloc_equals_h_psi_over_psi(nqs, tiny):
    """A random complex psi on the sector: E_loc(x) = (H psi)(x) / psi(x), H
    the literal operator-application matrix (rel 1e-10)."""
    h, eri, sec, basis, H = tiny
    rng = np.random.default_rng(3)
    la = rng.normal(0.0, 0.7, len(basis))
    ph = rng.uniform(-np.pi, np.pi, len(basis))
    psi = np.exp(la + 1j * ph)
    m = nqs.table_model(6, 2, 2, basis, la, ph)
    ham = nqs.ham_compile(h, eri, 2, 2)
    eloc, _, npairs = nqs.local_energy(ham, m, dev(basis))
    want = (H.T @ psi) / psi
    got = eloc.cpu().numpy()
    assert npairs == 225 * 92
    assert np.max(np.abs(got - want) / np.abs(want)) < 1e-10


def test_table_forward_outside_basis_and_backward(nqs, tiny):
    """A table on every second sector configuration: lookups return the entry,
    -inf for a configuration outside the basis (in the sector or not); the
    backward adds each sample's upstream weights to its entry."""
    h, eri, sec, basis, H = tiny
    sub = basis[::2]
    rng = np.random.default_rng(4)
    la, ph = rng.normal(size=len(sub)), rng.normal(size=len(sub))
    m = nqs.table_model(6, 2, 2, sub, la, ph)
    probe = [basis[0], basis[1], basis[224], 0b111111]
    out_l, out_p = (v.cpu().numpy() for v in nqs.amp_forward(m, dev(probe)))
    assert out_l[0] == la[0] and out_p[0] == ph[0]
    assert out_l[2] == la[112] and out_p[2] == ph[112]
    assert np.isneginf(out_l[1]) and np.isneginf(out_l[3])
    pick = [3, 50, 112]
    g = np.array([0.5, -1.25, 2.0])
    f = np.array([0.125, 0.0, -3.0])
    grad = nqs.amp_backward(m, dev([sub[i] for i in pick]), torch.tensor(g).cuda(),
                            torch.tensor(f).cuda()).cpu().numpy()
    want = np.zeros(2 * len(sub))
    want[pick] = g
    want[[len(sub) + i for i in pick]] = f
    assert np.array_equal(grad, want)


@pytest.mark.parametrize("strategy", ["MU", "DU"])
def test_table_sampler_follows_born_probabilities(nqs, tiny, strategy):
    """1e6 samples of the ground vector: every sample in the basis, counts sum
    to 1e6, chi-square against |psi|^2 / sum |psi|^2 (the conditionals are the
    table's marginals, so the mask changes nothing)."""
    h, eri, sec, basis, H = tiny
    e0, v0 = ground_state(H)
    keep = np.abs(v0) > 1e-6
    la = np.where(keep, np.log(np.abs(v0) + 1e-300), -np.inf)
    m = nqs.table_model(6, 2, 2, basis, la, np.zeros(len(basis)), strategy)
    x, c, lost = nqs.sample_unique(m, 1_000_000, 5)
    got = dict(zip(x.cpu().numpy().view(np.uint64).tolist(), c.cpu().tolist()))
    assert lost == 0 and sum(got.values()) == 1_000_000
    allowed = {int(b) for b, k in zip(basis, keep) if k}
    assert set(got) <= allowed
    p = np.where(keep, v0 ** 2, 0.0)
    expect = p / p.sum() * 1e6
    obs = np.array([got.get(int(b), 0) for b in basis], float)
    sel = expect > 5
    stat = np.sum((obs[sel] - expect[sel]) ** 2 / expect[sel])
    pval = chi2.sf(stat, sel.sum() - 1)
    print(f"table sampler {strategy}: chi2 {stat:.1f} on {sel.sum() - 1} dof, p = {pval:.3f}")
    assert pval > 1e-3
