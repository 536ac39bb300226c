"""Pins of the oracle's per-qubit complex-weight ansatz (paper: Appendix "ANQS
architecture"; Mask-Unphysical per qubit, "Pruning strategies")."""
import itertools

import numpy as np
import pytest
import scipy.stats as st
import torch

from oracle.nade import NADEModel
from oracle.sampler import sample_tree
from oracle.sector import Sector
from synth import make_nade_params, nade_param_spec, make_integrals

N_ORB, H = 4, 16


def model(sector, seed=1, mask_levels=None, std=0.3, **kw):
    return NADEModel(make_nade_params(N_ORB, H, seed=seed, std=std, bias_std=0.2, **kw), sector,
                     mask_levels=mask_levels)


def test_masked_model_is_normalised_on_the_sector():
    for na, nb in ((2, 1), (2, 2), (1, 3)):
        sec = Sector(N_ORB, na, nb)
        la, _ = model(sec).amplitudes(sec.enumerate())
        assert abs(torch.exp(2 * la).sum().item() - 1.0) < 1e-12


def test_unmasked_model_is_normalised_on_all_bit_strings():
    """DU everywhere: the product of normalised binary conditionals is a
    distribution over all 2^N strings."""
    m = model(Sector(N_ORB, 2, 2), mask_levels=0)
    la, _ = m.amplitudes(range(1 << (2 * N_ORB)))
    assert abs(torch.exp(2 * la).sum().item() - 1.0) < 1e-12


def test_constant_outputs_give_independent_bernoulli_qubits():
    """With W3 = 0 and real b3 = (c0, c1) each qubit is an independent
    Bernoulli with P(1) = e^{2 c1} / (e^{2 c0} + e^{2 c1}) and the phase is 0
    (the normaliser, product and gather against the closed form)."""
    p = make_nade_params(N_ORB, H, seed=3, std=0.3)
    rng = np.random.default_rng(0)
    q = []
    for i in range(2 * N_ORB):
        p[f"nade{i}.w3_re"][:] = 0.0
        p[f"nade{i}.w3_im"][:] = 0.0
        p[f"nade{i}.b3_im"][:] = 0.0
        c = rng.normal(size=2)
        p[f"nade{i}.b3_re"][:] = c
        q.append(np.exp(2 * c[1]) / (np.exp(2 * c[0]) + np.exp(2 * c[1])))
    m = NADEModel(p, Sector(N_ORB, 2, 2), mask_levels=0)
    xs = list(range(1 << (2 * N_ORB)))
    la, ph = m.amplitudes(xs)
    want = [sum(np.log(q[i] if (x >> i) & 1 else 1 - q[i]) for i in range(2 * N_ORB)) / 2 for x in xs]
    assert np.max(np.abs(la.detach().numpy() - np.array(want))) < 1e-12
    assert np.max(np.abs(ph.detach().numpy())) == 0.0


def test_last_conditional_is_always_masked():
    """Mask-Unphysical side effect ("Pruning strategies"): the value of the last
    qubit is fixed by the counts, so its conditional is 1 on every sector state."""
    sec = Sector(N_ORB, 2, 1)
    m = model(sec)
    xs = sec.enumerate()
    bits = m.bits_of(xs, m.N)
    lc = m.log_cond(bits, xs)
    last = lc[torch.arange(len(xs)), m.N - 1, bits[:, m.N - 1]]
    assert torch.all(last.real == 0.0) and torch.all(last.imag == 0.0)


def test_token_view_matches_the_qubit_product():
    """log|psi(x)| = 1/2 sum_p token_logits(x, p)[x_p], and the token
    log-probabilities of every physical prefix sum to one."""
    sec = Sector(N_ORB, 2, 2)
    m = model(sec)
    xs = sec.enumerate()
    la, _ = m.amplitudes(xs)
    tot = torch.zeros(len(xs), dtype=torch.float64)
    for p in range(N_ORB):
        tl = m.token_logits(xs, p)
        tok = torch.tensor([((x >> (2 * p)) & 1) + 2 * ((x >> (2 * p + 1)) & 1) for x in xs])
        tot += tl[torch.arange(len(xs)), tok]
        assert torch.max(torch.abs(torch.logsumexp(tl, 1))).item() < 1e-12
    assert torch.max(torch.abs(la - 0.5 * tot)).item() < 1e-12


def test_sampler_distribution_chi_square():
    sec = Sector(N_ORB, 2, 2)
    m = model(sec, seed=5, std=0.4)
    xs = sec.enumerate()
    probs = torch.exp(2 * m.amplitudes(xs)[0]).detach().numpy()
    cfg, cnt, lost = sample_tree(m, 200_000, 11)
    assert lost == 0 and sum(cnt) == 200_000 and all(sec.contains(x) for x in cfg)
    obs = np.zeros(len(xs))
    idx = {x: i for i, x in enumerate(xs)}
    for x, c in zip(cfg, cnt):
        obs[idx[x]] = c
    exp = probs * 200_000
    keep = exp > 5
    chi2 = np.sum((obs[keep] - exp[keep]) ** 2 / exp[keep])
    assert st.chi2.sf(chi2, keep.sum() - 1) > 1e-3


def test_gradient_matches_finite_differences():
    sec = Sector(N_ORB, 2, 2)
    params = make_nade_params(N_ORB, H, seed=7, std=0.3, bias_std=0.2)
    spec = nade_param_spec(N_ORB, H)
    xs = sec.enumerate()[:12]
    g = np.random.default_rng(1).normal(size=(2, len(xs)))

    def surrogate(p, grad=False):
        m = NADEModel(p, sec, requires_grad=grad)
        la, ph = m.amplitudes(xs)
        L = torch.sum(torch.tensor(g[0]) * la) + torch.sum(torch.tensor(g[1]) * ph)
        if grad:
            L.backward()
            return m.flat_grad(spec)
        return L.item()
    ga = surrogate(params, True)
    rng = np.random.default_rng(2)
    flat_names = [(k, j) for k, shp in spec for j in range(int(np.prod(shp)))]
    for t in rng.choice(len(flat_names), 25, replace=False):
        k, j = flat_names[t]
        h = 1e-6
        pp = {a: b.copy() for a, b in params.items()}
        pm = {a: b.copy() for a, b in params.items()}
        pp[k].reshape(-1)[j] += h
        pm[k].reshape(-1)[j] -= h
        fd = (surrogate(pp) - surrogate(pm)) / (2 * h)
        assert abs(fd - ga[t]) < 1e-6 * max(1.0, abs(ga[t]))
