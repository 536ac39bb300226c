"""Pins of the oracle's amplitude networks and Mask-Unphysical conditionals."""
import math

import numpy as np
import pytest
import torch

from oracle.model import (MLPModel, TransformerModel, build_model,
                          tokens_from_ints)
from oracle.sector import Sector
from oracle.vmc import exact_probabilities
from synth import make_mlp_params, make_transformer_params, workload


def tf_model(n, na, nb, d=16, L=2, H=4, std=0.3, seed=0, hf_bias=0.0, mask_levels=None):
    p = make_transformer_params(n, na, nb, d, L, phase_hidden=32, seed=seed, std=std,
                                hf_bias=hf_bias)
    return TransformerModel(p, Sector(n, na, nb), H, mask_levels=mask_levels)


def mlp_model(n, na, nb, std=0.5, seed=0, mask_levels=None):
    return MLPModel(make_mlp_params(n, 64, seed=seed, std=std), Sector(n, na, nb),
                    mask_levels=mask_levels)


@pytest.mark.parametrize("kind", ["mlp", "tf"])
def test_normalised_over_sector(kind):
    m = mlp_model(6, 2, 2) if kind == "mlp" else tf_model(6, 2, 2)
    p = exact_probabilities(m, m.sector.enumerate())
    assert abs(p.sum() - 1.0) < 1e-12
    assert p.min() > 0


def test_normalised_fp32_workload_sector():
    cfg, h, eri, params = workload("fp32")
    params = dict(params)
    m = build_model(cfg, params)
    basis = m.sector.enumerate()
    p = np.concatenate([exact_probabilities(m, basis[i:i + 8192]) for i in range(0, len(basis), 8192)])
    assert len(basis) == 63504
    assert abs(p.sum() - 1.0) < 1e-11


def test_masked_conditionals_sum_to_one():
    m = tf_model(6, 3, 1)
    rng = np.random.default_rng(1)
    toks = torch.from_numpy(rng.integers(0, 4, size=(200, 6)))
    lp = m.log_cond(toks)
    mask = m.masks(toks)
    probs = torch.exp(lp)
    # rows whose prefix is physical sum to 1; masked tokens have probability exactly 0
    phys_prefix = torch.ones(200, 6, dtype=torch.bool)
    for i in range(200):
        a = b = 0
        for p in range(6):
            phys_prefix[i, p] = m.sector.token_phys(p, a, b)
            a += int(toks[i, p]) & 1
            b += int(toks[i, p]) >> 1
    s = probs.sum(-1)[phys_prefix]
    assert torch.max(torch.abs(s - 1)) < 1e-14
    sel = (~mask) & phys_prefix.unsqueeze(-1)
    assert torch.all(probs[sel] == 0)


def test_zero_weight_model_closed_form():
    """All-zero parameters: each conditional is uniform over the physical
    tokens, so p(x) = prod_p 1 / #physical(p)."""
    sec = Sector(5, 2, 3)
    params = {k: np.zeros_like(v) for k, v in make_transformer_params(5, 2, 3, 8, 1, phase_hidden=8).items()}
    m = TransformerModel(params, sec, 2)
    basis = sec.enumerate()
    p = exact_probabilities(m, basis)
    for x, px in zip(basis, p):
        expect, a, b = 1.0, 0, 0
        for q in range(5):
            expect /= sum(sec.child_mask(q, a, b))
            t = ((x >> (2 * q)) & 1) + 2 * ((x >> (2 * q + 1)) & 1)
            a, b = a + (t & 1), b + (t >> 1)
        assert abs(px - expect) < 1e-15


@pytest.mark.parametrize("kind", ["mlp", "tf"])
def test_autoregressive_causality(kind):
    """Logits at position p depend on tokens < p only."""
    m = mlp_model(6, 2, 2) if kind == "mlp" else tf_model(6, 2, 2)
    rng = np.random.default_rng(2)
    toks = torch.from_numpy(rng.integers(0, 4, size=(32, 6)))
    base = m.logits(toks)
    for p in range(6):
        t2 = toks.clone()
        t2[:, p:] = torch.from_numpy(rng.integers(0, 4, size=(32, 6 - p)))
        assert torch.max(torch.abs(m.logits(t2)[:, :p + 1] - base[:, :p + 1])) < 1e-14
        if p < 5:
            assert torch.max(torch.abs(m.logits(t2)[:, p + 1:] - base[:, p + 1:])) > 1e-6


def test_transformer_against_scalar_loops():
    """The batched transformer against a scalar loop over positions and heads."""
    n, d, H = 4, 8, 2
    m = tf_model(n, 2, 1, d=d, L=1, H=H, std=0.4, seed=3)
    t = {k: v.detach().numpy() for k, v in m.t.items()}
    toks = [1, 3, 0, 2]
    inp = [4] + toks[:-1]

    def ln(v, g, b):
        mu = sum(v) / len(v)
        var = sum((e - mu) ** 2 for e in v) / len(v)
        return [(e - mu) / math.sqrt(var + 1e-5) * gg + bb for e, gg, bb in zip(v, g, b)]

    def lin(v, W, b):
        return [sum(v[i] * W[i][j] for i in range(len(v))) + b[j] for j in range(len(b))]

    def gelu(z):
        return 0.5 * z * (1 + math.tanh(math.sqrt(2 / math.pi) * (z + 0.044715 * z ** 3)))

    hs = [[t["tok_emb"][inp[p]][j] + t["pos_emb"][p][j] for j in range(d)] for p in range(n)]
    a = [ln(v, t["l0.ln1_g"], t["l0.ln1_b"]) for v in hs]
    qkv = [lin(v, t["l0.wqkv"], t["l0.bqkv"]) for v in a]
    dh = d // H
    outs = []
    for p in range(n):
        o = []
        for hh in range(H):
            q = qkv[p][hh * dh:(hh + 1) * dh]
            sc = [sum(q[i] * qkv[s][d + hh * dh + i] for i in range(dh)) / math.sqrt(dh) for s in range(p + 1)]
            mx = max(sc)
            w = [math.exp(v - mx) for v in sc]
            z = sum(w)
            o += [sum(w[s] / z * qkv[s][2 * d + hh * dh + i] for s in range(p + 1)) for i in range(dh)]
        outs.append(o)
    hs = [[hs[p][j] + v for j, v in enumerate(lin(outs[p], t["l0.wo"], t["l0.bo"]))] for p in range(n)]
    a = [ln(v, t["l0.ln2_g"], t["l0.ln2_b"]) for v in hs]
    f = [lin([gelu(z) for z in lin(v, t["l0.w1"], t["l0.b1"])], t["l0.w2"], t["l0.b2"]) for v in a]
    hs = [[hs[p][j] + f[p][j] for j in range(d)] for p in range(n)]
    lg = [[a + b for a, b in zip(lin(ln(v, t["lnf_g"], t["lnf_b"]), t["whead"], t["bhead"]), t["logit_bias"][p])]
          for p, v in enumerate(hs)]
    got = m.logits(torch.tensor([toks]))[0].detach().numpy()
    assert np.max(np.abs(got - np.array(lg))) < 1e-12


def test_hf_bias_peaks_distribution():
    m = tf_model(6, 2, 2, std=0.02, hf_bias=4.0)
    basis = m.sector.enumerate()
    p = exact_probabilities(m, basis)
    assert basis[int(np.argmax(p))] == m.sector.x_hf


def test_du_levels_unmasked():
    """With no masked levels the conditionals are the plain softmax, and the
    sector carries less than all of the probability."""
    m = mlp_model(6, 2, 2, mask_levels=0)
    p = exact_probabilities(m, m.sector.enumerate())
    assert 0 < p.sum() < 1
    full = 0.0
    toks = tokens_from_ints(list(range(1 << 12)), 6)
    with torch.no_grad():
        full = torch.exp(2 * m.log_abs(toks)).sum().item()
    assert abs(full - 1.0) < 1e-12


# ------------------------------------------------ model shared by molecules

def shared_params(n_max=14, d=16, L=2, occ_bias=0.0, seed=3):
    return make_transformer_params(n_max, 0, 0, d, L, phase_hidden=32, seed=seed, std=0.3,
                                   occ_bias=occ_bias, bias_std=0.1)


@pytest.mark.parametrize("n,na,nb", [(6, 3, 4), (10, 4, 5), (14, 7, 7)])
def test_shared_model_equals_truncated_tables(n, na, nb):
    """A molecule of n tokens on a model with 14 positions equals a model whose
    position tables are cut to n rows (the absent positions contribute nothing)."""
    full = shared_params()
    cut = dict(full)
    cut["pos_emb"] = full["pos_emb"][:n]
    cut["logit_bias"] = full["logit_bias"][:n]
    cut["ph_w1"] = full["ph_w1"][:4 * n]
    sec = Sector(n, na, nb)
    rng = np.random.default_rng(n)
    xs = [sec.enumerate()[i] for i in rng.choice(len(sec.enumerate()), 50)] if n < 14 else \
        [sec.x_hf]
    a = TransformerModel(full, sec, 4).amplitudes(xs)
    b = TransformerModel(cut, sec, 4).amplitudes(xs)
    for u, v in zip(a, b):
        assert torch.max(torch.abs(u - v)).item() < 1e-13


def test_shared_model_normalised():
    m = TransformerModel(shared_params(), Sector(6, 3, 4), 4)
    p = exact_probabilities(m, m.sector.enumerate())
    assert abs(p.sum() - 1.0) < 1e-12


@pytest.mark.parametrize("n,na,nb", [(6, 2, 3), (6, 3, 3), (8, 4, 3), (8, 5, 5)])
def test_occupation_bias_peaks_hf_of_any_sector(n, na, nb):
    """Under the symmetry mask a per-electron logit bias favours the
    Hartree-Fock state of whatever sector the molecule has."""
    p = make_transformer_params(14, 0, 0, 16, 2, phase_hidden=32, seed=5, std=0.02,
                                occ_bias=4.0)
    m = TransformerModel(p, Sector(n, na, nb), 4)
    basis = m.sector.enumerate()
    assert basis[int(np.argmax(exact_probabilities(m, basis)))] == m.sector.x_hf
