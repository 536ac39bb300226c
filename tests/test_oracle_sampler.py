"""Pins of the oracle's random numbers, binomial draws and tree sampler."""
import numpy as np
import pytest
import scipy.stats as st

from oracle.model import MLPModel, TransformerModel
from oracle.sampler import (UniformStream, binomial, philox4x32_10,
                            sample_tree, split_counts, to_unit)
from oracle.sector import Sector
from oracle.vmc import exact_probabilities
from synth import make_mlp_params, make_transformer_params


def test_philox_known_answers():
    """Known-answer vectors of Philox4x32-10 (Random123 distribution, kat_vectors)."""
    assert philox4x32_10((0, 0, 0, 0), (0, 0)) == (0x6627e8d5, 0xe169c58d, 0xbc57ac4c, 0x9b00dbd8)
    f = 0xFFFFFFFF
    assert philox4x32_10((f, f, f, f), (f, f)) == (0x408f276d, 0x41c83b0e, 0xa20bc7c6, 0x6d5451fd)
    assert philox4x32_10((0x243f6a88, 0x85a308d3, 0x13198a2e, 0x03707344),
                         (0xa4093822, 0x299f31d0)) == (0xd16cfe09, 0x94fdcceb, 0x5001e420, 0x24126ea1)


def test_unit_interval_open():
    assert 0.0 < to_unit(0, 0) < 1e-15
    assert 1.0 - 1e-15 < to_unit(0xFFFFFFFF, 0xFFFFFFFF) < 1.0
    u = [UniformStream(7, 0, 0, 0)() for _ in range(1)]
    s = UniformStream(12345, 99, 3, 1)
    vals = np.array([s() for _ in range(20000)])
    assert st.kstest(vals, "uniform").pvalue > 1e-3


@pytest.mark.parametrize("n,p", [(7, 0.3), (40, 0.1), (1000, 0.004), (60, 0.5), (500, 0.3),
                                 (10_000, 0.77), (1_000_000, 0.45), (25, 0.97)])
def test_binomial_distribution(n, p):
    """Chi-square of 4000 draws against the exact binomial pmf."""
    draws = np.array([binomial(n, p, UniformStream(2024, i, 1, 2)) for i in range(4000)])
    assert draws.min() >= 0 and draws.max() <= n
    lo, hi = st.binom.ppf(1e-4, n, p), st.binom.ppf(1 - 1e-4, n, p)
    edges = np.unique(np.round(np.linspace(lo, hi + 1, 25)))
    obs = np.histogram(draws, bins=np.concatenate([[-0.5], edges[1:-1] - 0.5, [n + 0.5]]))[0]
    cdf = st.binom.cdf(np.concatenate([edges[1:-1] - 1, [n]]), n, p)
    exp = np.diff(np.concatenate([[0.0], cdf])) * len(draws)
    keep = exp > 5
    chi = ((obs[keep] - exp[keep]) ** 2 / exp[keep]).sum()
    assert st.chi2.sf(chi, keep.sum() - 1) > 1e-4
    assert abs(draws.mean() - n * p) < 5 * np.sqrt(n * p * (1 - p) / len(draws)) + 1e-9


def test_binomial_edge_cases():
    s = UniformStream(1, 2, 3, 0)
    assert binomial(0, 0.3, s) == 0
    assert binomial(17, 0.0, s) == 0
    assert binomial(17, 1.0, s) == 17


def test_split_counts_exact_cases():
    assert split_counts(100, [0.0, 1.0, 0.0, 0.0], 1, 0, 0) == [0, 100, 0, 0]
    assert split_counts(100, [0.0, 0.0, 0.0, 2.5], 1, 0, 0) == [0, 0, 0, 100]
    for seed in range(20):
        c = split_counts(1000, [0.3, 0.0, 1.0, 0.2], seed, 5, 2)
        assert sum(c) == 1000 and c[1] == 0


def _chi2_pvalue(configs, counts, basis, probs, n_s):
    idx = {x: i for i, x in enumerate(basis)}
    obs = np.zeros(len(basis))
    for x, c in zip(configs, counts):
        obs[idx[x]] += c
    exp = probs * n_s
    order = np.argsort(exp)
    # pool the smallest bins until every bin expects >= 5
    bins_o, bins_e, acc_o, acc_e = [], [], 0.0, 0.0
    for i in order:
        acc_o += obs[i]
        acc_e += exp[i]
        if acc_e >= 5:
            bins_o.append(acc_o); bins_e.append(acc_e); acc_o = acc_e = 0.0
    if acc_e > 0:
        bins_o[-1] += acc_o; bins_e[-1] += acc_e
    bins_o, bins_e = np.array(bins_o), np.array(bins_e)
    chi = ((bins_o - bins_e) ** 2 / bins_e).sum()
    return st.chi2.sf(chi, len(bins_o) - 1)


def test_tree_sampler_mu_distribution():
    sec = Sector(6, 2, 2)
    m = MLPModel(make_mlp_params(6, 64, seed=11, std=0.5), sec)
    basis = sec.enumerate()
    probs = exact_probabilities(m, basis)
    pvals = []
    for seed in range(12):
        cfg, cnt, lost = sample_tree(m, 10_000, seed)
        assert lost == 0 and sum(cnt) == 10_000 and min(cnt) > 0
        assert len(set(cfg)) == len(cfg)
        assert all(sec.contains(x) for x in cfg)
        pvals.append(_chi2_pvalue(cfg, cnt, basis, probs, 10_000))
    assert min(pvals) > 1e-4
    assert st.kstest(pvals, "uniform").pvalue > 1e-3


def test_tree_sampler_deterministic_and_tree_order():
    sec = Sector(6, 3, 2)
    m = TransformerModel(make_transformer_params(6, 3, 2, 16, 1, phase_hidden=16, seed=2, std=0.3),
                         sec, 2)
    a = sample_tree(m, 5000, 99)
    b = sample_tree(m, 5000, 99)
    assert a == b
    toks = [[((x >> (2 * p)) & 1) + 2 * ((x >> (2 * p + 1)) & 1) for p in range(6)] for x in a[0]]
    assert toks == sorted(toks)


def test_tree_sampler_du_loses_samples():
    """Discard-Unphysical: lost + kept = N_s; the kept fraction estimates the
    sector's share of the unmasked distribution."""
    sec = Sector(6, 2, 2)
    m = MLPModel(make_mlp_params(6, 64, seed=12, std=0.5), sec, mask_levels=0)
    share = exact_probabilities(m, sec.enumerate()).sum()
    cfg, cnt, lost = sample_tree(m, 20_000, 3, strategy="DU")
    assert lost + sum(cnt) == 20_000 and lost > 0
    assert all(sec.contains(x) for x in cfg)
    kept = sum(cnt) / 20_000
    assert abs(kept - share) < 5 * np.sqrt(share * (1 - share) / 20_000)


def test_tree_sampler_mud_distribution():
    """MU-d: the sampled distribution is that of the model masked on the first
    n - d levels only, conditioned on the samples that survive."""
    sec = Sector(6, 2, 2)
    m = MLPModel(make_mlp_params(6, 64, seed=13, std=0.5), sec, mask_levels=4)
    basis = sec.enumerate()
    probs = exact_probabilities(m, basis)
    cfg, cnt, lost = sample_tree(m, 20_000, 5, strategy="MUd", d=2)
    assert lost + sum(cnt) == 20_000
    pv = _chi2_pvalue(cfg, cnt, basis, probs / probs.sum(), sum(cnt))
    assert pv > 1e-4


def test_tree_sampler_streams():
    """Stream 0 is the single-tree sampler; another stream draws a different,
    equally valid sample (every config in the sector, counts summing to N_s)."""
    from oracle.model import TransformerModel
    from oracle.sector import Sector
    from synth import make_transformer_params
    sec = Sector(6, 3, 2)
    params = make_transformer_params(14, 0, 0, 16, 2, phase_hidden=32, seed=2, std=0.3)
    m = TransformerModel(params, sec, 4)
    a = sample_tree(m, 5000, 17)
    b = sample_tree(m, 5000, 17, stream=0)
    c = sample_tree(m, 5000, 17, stream=3)
    assert a == b
    assert a[0] != c[0] or a[1] != c[1]
    assert sum(c[1]) == 5000 and c[2] == 0
    assert all(sec.contains(x) for x in c[0])
