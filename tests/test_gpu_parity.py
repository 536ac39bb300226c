"""GPU parity of the HIP path (through the C ABI) against the FP64 CPU oracle."""
import math

import numpy as np
import pytest
import torch

from oracle.hamiltonian import slater_condon_row
from oracle.model import MLPModel, TransformerModel, build_model, tokens_from_ints
from oracle.sampler import sample_tree
from oracle.sector import Sector, hf_config
from oracle.vmc import (energy_stats, exact_probabilities, gradient, local_energies,
                        surrogate_weights)
from synth import (flatten_params, make_integrals, make_mlp_params, make_transformer_params,
                   mlp_param_spec, transformer_param_spec, workload)

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def nqs():
    from paper_2310_04166_amd import nqs as mod
    mod.lib()
    assert torch.cuda.is_available()
    return mod


def dev(a):
    return torch.as_tensor(np.asarray(a, dtype=np.uint64).view(np.int64)).cuda()


def log(msg):
    print(msg, flush=True)


def sector_sample(n, na, nb, count, seed):
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(count):
        a = rng.choice(n, na, replace=False)
        b = rng.choice(n, nb, replace=False)
        out.append(int(sum(1 << (2 * int(p)) for p in a) | sum(1 << (2 * int(p) + 1) for p in b)))
    return out


# ------------------------------------------------------------------ bit work

@pytest.mark.parametrize("n,na,nb,count", [(6, 2, 2, 225), (10, 5, 5, 37), (15, 7, 7, 5), (8, 3, 4, 61),
                                           (32, 2, 2, 4)])
def test_connected_pairs_bit_exact(nqs, n, na, nb, count):
    """Connected sets, order and matrix elements against the oracle's
    Slater-Condon rows; n = 32 fills the 64-bit word (the last case occupies
    spin-orbitals 62 and 63)."""
    log(f"connected_pairs n={n} ({na},{nb}) count={count}")
    h, eri = make_integrals(n, 2 * n, 100 + n)
    H = nqs.ham_compile(h, eri, na, nb)
    sec = Sector(n, na, nb)
    xs = sec.enumerate() if count == 225 else [hf_config(n, na, nb)] + sector_sample(n, na, nb, count - 1, n)
    if n == 32:
        xs.append((1 << 0) | (1 << 62) | (1 << 11) | (1 << 63))
    off, xp, hv, hd = nqs.connected_pairs(H, dev(xs))
    off, xp, hv, hd = (t.cpu().numpy() for t in (off, xp, hv, hd))
    xp = xp.view(np.uint64)
    for i, x in enumerate(xs):
        ref_x, ref_v = slater_condon_row(h, eri, x)
        got_x = [int(v) for v in xp[off[i]:off[i + 1]]]
        assert sorted(got_x) == sorted(ref_x[1:]), i              # bit-exact connected set
        assert got_x == sorted(got_x, key=lambda v: v ^ x)          # flip-group order
        ref = dict(zip(ref_x, ref_v))
        got_v = hv[off[i]:off[i + 1]]
        scale = max(abs(v) for v in ref_v)
        for gx, gv in zip(got_x, got_v):
            assert abs(gv - ref[gx]) <= 1e-12 * scale
            if abs(ref[gx]) > 1e-12 * scale:
                assert np.sign(gv) == np.sign(ref[gx])
        assert abs(hd[i] - ref_v[0]) <= 1e-12 * abs(ref_v[0])


def test_connected_pairs_offsets_of_many_samples(nqs):
    """10,001 samples (the offsets' scan runs in tiles of 1024 plus a scan of the
    tile totals): offsets equal the cumulative connected counts, the per-sample
    count (92 at 12 spin-orbitals, 2+2) being exact combinatorics."""
    n, na, nb = 6, 2, 2
    h, eri = make_integrals(n, 2 * n, 106)
    H = nqs.ham_compile(h, eri, na, nb)
    xs = (Sector(n, na, nb).enumerate() * 45)[:10001]
    off, xp, _, _ = nqs.connected_pairs(H, dev(xs))
    off = off.cpu().numpy()
    assert np.array_equal(off, 92 * np.arange(len(xs) + 1))
    xp = xp.cpu().numpy().view(np.uint64)
    for i in (0, 1023, 1024, 5000, 10000):          # tiles' edges and the tail
        ref_x, _ = slater_condon_row(h, eri, xs[i])
        assert sorted(int(v) for v in xp[off[i]:off[i + 1]]) == sorted(ref_x[1:])


def test_connected_pairs_edge_cases(nqs):
    h, eri = make_integrals(6, 12, 1)
    H = nqs.ham_compile(h, eri, 2, 2)
    off, xp, hv, hd = nqs.connected_pairs(H, torch.zeros(0, dtype=torch.int64, device="cuda"))
    assert off.cpu().tolist() == [0] and xp.numel() == 0
    # capacity too small
    with pytest.raises(nqs.NQSError) as e:
        nqs.connected_pairs(H, dev([0b1111]), capacity=10)
    assert e.value.status == -2
    # empty and full shells: no connected configurations at all
    H0 = nqs.ham_compile(h, eri, 0, 6)
    off, xp, _, hd = nqs.connected_pairs(H0, dev([0xAAA]))
    assert xp.numel() == 0
    ref = slater_condon_row(h, eri, 0xAAA)
    assert len(ref[0]) == 1 and abs(hd.item() - ref[1][0]) < 1e-12


# --------------------------------------------------------------- amplitudes

def gpu_model(nqs, kind, dims, params, spec, precision, strategy="MU", d=0):
    return nqs.Model(kind, dims, flatten_params(params, spec), precision, strategy, d)


@pytest.mark.parametrize("precision,tol", [("fp64", 1e-12), ("fp32", 2e-5)])
def test_mlp_forward(nqs, precision, tol):
    log(f"mlp forward {precision}")
    sec = Sector(6, 2, 2)
    params = make_mlp_params(6, 64, seed=21, std=0.5)
    ref = MLPModel(params, sec)
    m = gpu_model(nqs, nqs.MODEL_MLP, [6, 2, 2, 64], params, mlp_param_spec(6, 64), precision)
    xs = sec.enumerate()
    la, ph = nqs.amp_forward(m, dev(xs))
    rla, rph = ref.amplitudes(xs)
    assert np.max(np.abs(la.cpu().numpy() - rla.detach().numpy())) < tol * 10
    assert np.max(np.abs(ph.cpu().numpy() - rph.detach().numpy())) < tol * 10


@pytest.mark.parametrize("precision,tol", [("fp64", 1e-11), ("fp32", 5e-5)])
def test_transformer_forward(nqs, precision, tol):
    log(f"transformer forward {precision}")
    n, na, nb, d, L, H = 7, 3, 2, 32, 2, 4
    sec = Sector(n, na, nb)
    params = make_transformer_params(n, na, nb, d, L, phase_hidden=48, seed=22, std=0.3)
    spec = transformer_param_spec(n, d, L, 4 * d, 48)
    ref = TransformerModel(params, sec, H)
    m = gpu_model(nqs, nqs.MODEL_TRANSFORMER, [n, na, nb, d, L, H, 4 * d, 48], params, spec, precision)
    xs = sec.enumerate()                       # 735 configurations: many tiles and a ragged tail
    la, ph = nqs.amp_forward(m, dev(xs))
    rla, rph = ref.amplitudes(xs)
    assert np.max(np.abs(la.cpu().numpy() - rla.detach().numpy())) < tol
    assert np.max(np.abs(ph.cpu().numpy() - rph.detach().numpy())) < tol
    # outside the sector: -inf
    la_out, _ = nqs.amp_forward(m, dev([0, (1 << (2 * n)) - 1]))
    assert torch.all(torch.isinf(la_out)) and torch.all(la_out < 0)


def test_fp32_workload_forward(nqs):
    cfg, h, eri, params = workload("fp32")
    sec = Sector(cfg["n"], cfg["n_alpha"], cfg["n_beta"])
    ref = build_model(cfg, params, sec)
    m = gpu_model(nqs, nqs.MODEL_TRANSFORMER, nqs.model_dims(cfg), params,
                  transformer_param_spec(10, 64, 2, 256, 256), "fp32")
    xs = sector_sample(10, 5, 5, 3001, 3)
    la, ph = nqs.amp_forward(m, dev(xs))
    rla, rph = ref.amplitudes(xs)
    assert np.max(np.abs(la.cpu().numpy() - rla.detach().numpy())) < 5e-5
    assert np.max(np.abs(ph.cpu().numpy() - rph.detach().numpy())) < 5e-5


# ------------------------------------------------------------- local energy

def test_local_energy_fp64_tiny(nqs):
    """E_loc of every sector configuration, FP64 mode: 1e-10 relative."""
    log("local_energy fp64 tiny")
    cfg, h, eri, _ = workload("tiny")
    sec = Sector(6, 2, 2)
    params = make_mlp_params(6, 64, seed=31, std=0.5)
    ref = MLPModel(params, sec)
    m = gpu_model(nqs, nqs.MODEL_MLP, [6, 2, 2, 64], params, mlp_param_spec(6, 64), "fp64")
    H = nqs.ham_compile(h, eri, 2, 2)
    xs = sec.enumerate()
    counts = np.arange(1, len(xs) + 1, dtype=np.int64)
    eloc, sums, npairs = nqs.local_energy(H, m, dev(xs), torch.as_tensor(counts).cuda())
    assert npairs == 225 * 92
    want = local_energies(ref, h, eri, xs)
    got = eloc.cpu().numpy()
    assert np.max(np.abs(got - want) / np.abs(want)) < 1e-10
    W, E, var = energy_stats(want, counts)
    s = sums.cpu().numpy()
    assert s[0] == W
    assert abs(s[1] / W - E.real) < 1e-10 * abs(E) and abs(s[2] / W - E.imag) < 1e-10 * abs(E)


def test_local_energy_distinct_count(nqs):
    """The amplitude network runs on exactly the distinct connected x'."""
    cfg, h, eri, params = workload("fp32")
    m = gpu_model(nqs, nqs.MODEL_TRANSFORMER, nqs.model_dims(cfg), params,
                  transformer_param_spec(10, 64, 2, 256, 256), "fp32")
    H = nqs.ham_compile(h, eri, 5, 5)
    x, c, _ = nqs.sample_unique(m, 100_000, 4)
    eloc, sums, npairs = nqs.local_energy(H, m, x, c)
    pairs, distinct = nqs.local_energy_stats(H)
    xs = [int(v) for v in x.cpu().numpy().view(np.uint64)]
    ref = set()
    for xx in xs:
        ref.update(slater_condon_row(h, eri, xx)[0][1:])
    assert pairs == npairs == len(xs) * 875
    assert distinct == len(ref)


def test_local_energy_fp32_workload(nqs):
    """fp32 transformer at 20 spin-orbitals on sampled configurations."""
    log("local_energy fp32 workload")
    cfg, h, eri, params = workload("fp32")
    sec = Sector(10, 5, 5)
    ref = build_model(cfg, params, sec)
    m = gpu_model(nqs, nqs.MODEL_TRANSFORMER, nqs.model_dims(cfg), params,
                  transformer_param_spec(10, 64, 2, 256, 256), "fp32")
    H = nqs.ham_compile(h, eri, 5, 5)
    xs = [hf_config(10, 5, 5)] + sector_sample(10, 5, 5, 40, 9)
    eloc, sums, npairs = nqs.local_energy(H, m, dev(xs))
    assert npairs == len(xs) * 875
    want = local_energies(ref, h, eri, xs)
    got = eloc.cpu().numpy()
    assert np.max(np.abs(got - want)) < 1e-4 * max(1.0, np.max(np.abs(want)))


# ------------------------------------------------------------------ sampler

def test_sampler_replay_fp64_bit_exact(nqs):
    """FP64 conditionals + the same Philox keys: counts identical to the oracle."""
    log("sampler replay fp64")
    sec = Sector(6, 2, 2)
    params = make_mlp_params(6, 64, seed=41, std=0.5)
    ref = MLPModel(params, sec)
    m = gpu_model(nqs, nqs.MODEL_MLP, [6, 2, 2, 64], params, mlp_param_spec(6, 64), "fp64")
    for seed in (0, 1, 12345678901234):
        cfg_o, cnt_o, lost_o = sample_tree(ref, 10_000, seed)
        c, k, lost = nqs.sample_unique(m, 10_000, seed)
        assert lost == 0 == lost_o
        assert [int(v) for v in c.cpu().numpy().view(np.uint64)] == cfg_o
        assert k.cpu().tolist() == cnt_o


def test_sampler_replay_transformer_fp64(nqs):
    n, na, nb, d = 8, 3, 4, 32
    sec = Sector(n, na, nb)
    params = make_transformer_params(n, na, nb, d, 2, phase_hidden=32, seed=42, std=0.3, hf_bias=1.0)
    ref = TransformerModel(params, sec, 4)
    m = gpu_model(nqs, nqs.MODEL_TRANSFORMER, [n, na, nb, d, 2, 4, 4 * d, 32], params,
                  transformer_param_spec(n, d, 2, 4 * d, 32), "fp64")
    cfg_o, cnt_o, _ = sample_tree(ref, 200_000, 77)
    c, k, _ = nqs.sample_unique(m, 200_000, 77)
    assert [int(v) for v in c.cpu().numpy().view(np.uint64)] == cfg_o
    assert k.cpu().tolist() == cnt_o


@pytest.mark.parametrize("strategy,d", [("DU", 0), ("MUd", 2)])
def test_sampler_replay_du_mud(nqs, strategy, d):
    sec = Sector(6, 2, 2)
    params = make_mlp_params(6, 64, seed=43, std=0.5)
    ml = {"DU": 0, "MUd": 6 - d}[strategy]
    ref = MLPModel(params, sec, mask_levels=ml)
    m = gpu_model(nqs, nqs.MODEL_MLP, [6, 2, 2, 64], params, mlp_param_spec(6, 64), "fp64",
                  strategy, d)
    cfg_o, cnt_o, lost_o = sample_tree(ref, 50_000, 5, strategy=strategy, d=d)
    c, k, lost = nqs.sample_unique(m, 50_000, 5)
    assert lost == lost_o > 0
    assert [int(v) for v in c.cpu().numpy().view(np.uint64)] == cfg_o
    assert k.cpu().tolist() == cnt_o
    # the model's log|psi| is the unmasked one on the DU levels
    la, _ = nqs.amp_forward(m, dev(cfg_o))
    assert np.max(np.abs(la.cpu().numpy() - ref.amplitudes(cfg_o)[0].detach().numpy())) < 1e-12


def test_sampler_fp32_chi_square(nqs):
    """fp32 conditionals: distribution against the exact (oracle) sector probabilities."""
    import scipy.stats as st
    cfg, h, eri, params = workload("fp32")
    sec = Sector(10, 5, 5)
    ref = build_model(cfg, params, sec)
    basis = sec.enumerate()
    probs = np.concatenate([exact_probabilities(ref, basis[i:i + 8192]) for i in range(0, len(basis), 8192)])
    m = gpu_model(nqs, nqs.MODEL_TRANSFORMER, nqs.model_dims(cfg), params,
                  transformer_param_spec(10, 64, 2, 256, 256), "fp32")
    pvals = []
    index = {x: i for i, x in enumerate(basis)}
    for seed in range(5):
        c, k, lost = nqs.sample_unique(m, 100_000, seed)
        c = c.cpu().numpy().view(np.uint64)
        k = k.cpu().numpy()
        assert lost == 0 and k.sum() == 100_000 and k.min() > 0
        assert len(set(c.tolist())) == len(c)
        obs = np.zeros(len(basis))
        for x, cnt in zip(c, k):
            obs[index[int(x)]] = cnt                          # also checks: every sample in sector
        exp = probs * 100_000
        order = np.argsort(exp)
        bo, be, ao, ae = [], [], 0.0, 0.0
        for i in order:
            ao += obs[i]; ae += exp[i]
            if ae >= 5:
                bo.append(ao); be.append(ae); ao = ae = 0.0
        bo[-1] += ao; be[-1] += ae
        bo, be = np.array(bo), np.array(be)
        pvals.append(st.chi2.sf(((bo - be) ** 2 / be).sum(), len(bo) - 1))
    assert min(pvals) > 1e-4, pvals


def test_sampler_edge_cases(nqs):
    sec = Sector(6, 2, 2)
    params = make_mlp_params(6, 64, seed=44, std=0.5)
    m = gpu_model(nqs, nqs.MODEL_MLP, [6, 2, 2, 64], params, mlp_param_spec(6, 64), "fp64")
    c, k, lost = nqs.sample_unique(m, 0, 1)
    assert c.numel() == 0 and lost == 0
    c, k, lost = nqs.sample_unique(m, 1, 1)
    assert c.numel() == 1 and k.item() == 1
    with pytest.raises(nqs.NQSError) as e:
        nqs.sample_unique(m, 10_000, 1, capacity=3)
    assert e.value.status == -2


# ----------------------------------------------------------------- gradient

def test_backward_mlp_fp64(nqs):
    log("backward mlp fp64")
    cfg, h, eri, _ = workload("tiny")
    sec = Sector(6, 2, 2)
    params = make_mlp_params(6, 64, seed=51, std=0.5, bias_std=0.1)
    spec = mlp_param_spec(6, 64)
    xs = sec.enumerate()
    counts = np.random.default_rng(0).integers(1, 50, len(xs))
    ref = MLPModel(params, sec)
    eloc = local_energies(ref, h, eri, xs)
    g_ref = gradient(MLPModel(params, sec, requires_grad=True), xs, counts, eloc, spec)
    gl, gp = surrogate_weights(counts, eloc)
    m = gpu_model(nqs, nqs.MODEL_MLP, [6, 2, 2, 64], params, spec, "fp64")
    g = nqs.amp_backward(m, dev(xs), torch.as_tensor(gl).cuda(), torch.as_tensor(gp).cuda())
    g = g.cpu().numpy()
    assert np.max(np.abs(g - g_ref)) < 1e-10 * np.max(np.abs(g_ref))


@pytest.mark.parametrize("precision,tol", [("fp64", 1e-10), ("fp32", 2e-4)])
def test_backward_transformer(nqs, precision, tol):
    log(f"backward transformer {precision}")
    n, na, nb, d, L, H, PH = 7, 3, 2, 32, 2, 4, 48
    h, eri = make_integrals(n, 2 * n, 61)
    sec = Sector(n, na, nb)
    params = make_transformer_params(n, na, nb, d, L, phase_hidden=PH, seed=62, std=0.3, bias_std=0.1)
    spec = transformer_param_spec(n, d, L, 4 * d, PH)
    xs = sec.enumerate()
    counts = np.random.default_rng(1).integers(1, 50, len(xs))
    ref = TransformerModel(params, sec, H)
    eloc = local_energies(ref, h, eri, xs)
    g_ref = gradient(TransformerModel(params, sec, H, requires_grad=True), xs, counts, eloc, spec)
    gl, gp = surrogate_weights(counts, eloc)
    m = gpu_model(nqs, nqs.MODEL_TRANSFORMER, [n, na, nb, d, L, H, 4 * d, PH], params, spec, precision)
    g = nqs.amp_backward(m, dev(xs), torch.as_tensor(gl).cuda(), torch.as_tensor(gp).cuda())
    g = g.double().cpu().numpy()
    assert np.max(np.abs(g - g_ref)) < tol * np.max(np.abs(g_ref))


def test_transformer_32_tokens_fp64(nqs):
    """32 tokens (64 spin-orbitals, the whole configuration word) on the FP64
    layer path, whose attention then takes its general kernel: the sampler's
    unique configurations and counts replayed bit-exactly, amplitudes and the
    VMC gradient (synthetic complex local energies) against the oracle.  A
    negative occupation bias pushes the electrons towards the last orbitals, so
    most samples use bits 60..63."""
    n, na, nb, d, L, H, PH = 32, 2, 2, 32, 1, 4, 32
    sec = Sector(n, na, nb)
    params = make_transformer_params(n, na, nb, d, L, phase_hidden=PH, seed=48, std=0.3,
                                     occ_bias=-4.0)
    spec = transformer_param_spec(n, d, L, 4 * d, PH)
    ref = TransformerModel(params, sec, H)
    m = gpu_model(nqs, nqs.MODEL_TRANSFORMER, [n, na, nb, d, L, H, 4 * d, PH], params, spec, "fp64")
    cfg_o, cnt_o, lost_o = sample_tree(ref, 20_000, 9)
    c, k, lost = nqs.sample_unique(m, 20_000, 9)
    got = [int(v) for v in c.cpu().numpy().view(np.uint64)]
    assert lost == 0 == lost_o
    assert got == cfg_o and k.cpu().tolist() == cnt_o
    assert sum(1 for v in got if v >> 60) > len(got) // 2
    la, ph = nqs.amp_forward(m, c)
    rla, rph = (v.detach().numpy() for v in ref.amplitudes(cfg_o))
    assert np.max(np.abs(la.cpu().numpy() - rla)) < 1e-10
    assert np.max(np.abs(ph.cpu().numpy() - rph)) < 1e-10
    rng = np.random.default_rng(2)
    eloc = rng.normal(size=len(got)) + 1j * rng.normal(size=len(got))
    counts = np.asarray(cnt_o)
    g_ref = gradient(TransformerModel(params, sec, H, requires_grad=True), cfg_o, counts, eloc, spec)
    gl, gp = surrogate_weights(counts, eloc)
    g = nqs.amp_backward(m, c, torch.as_tensor(gl).cuda(), torch.as_tensor(gp).cuda())
    g = g.double().cpu().numpy()
    err = np.max(np.abs(g - g_ref))
    log(f"32 tokens: {len(got)} unique, gradient err {err:.2e} of {np.max(np.abs(g_ref)):.2e}")
    assert err < 1e-10 * np.max(np.abs(g_ref))


def test_vmc_weights_and_adam(nqs):
    rng = np.random.default_rng(3)
    eloc = rng.normal(size=50) + 1j * rng.normal(size=50)
    counts = rng.integers(1, 9, 50)
    W, E, _ = energy_stats(eloc, counts)
    sums = torch.tensor([W, np.sum(counts * eloc.real), np.sum(counts * eloc.imag), 0.0]).cuda()
    gl, gp = nqs.vmc_weights(torch.as_tensor(eloc).cuda(), torch.as_tensor(counts).cuda(), sums)
    rl, rp = surrogate_weights(counts, eloc)
    assert np.max(np.abs(gl.cpu().numpy() - rl)) < 1e-14
    assert np.max(np.abs(gp.cpu().numpy() - rp)) < 1e-14
    p = torch.tensor(rng.normal(size=100)).cuda()
    g = torch.tensor(rng.normal(size=100)).cuda()
    mo, ve = torch.zeros(100, dtype=torch.float64).cuda(), torch.zeros(100, dtype=torch.float64).cuda()
    ref_p = p.clone()
    opt = torch.optim.Adam([ref_p.requires_grad_()], lr=1e-2)
    ref_p.grad = g.clone()
    opt.step()
    nqs.adam_update(p.data_ptr(), g, mo, ve, lr=1e-2, t=1)
    assert torch.max(torch.abs(p - ref_p.detach())).item() < 1e-12


@pytest.mark.parametrize("dtype,tol", [(torch.float64, 1e-12), (torch.float32, 2e-6)])
def test_adam_several_steps(nqs, dtype, tol):
    """Five steps with changing gradients (the bias corrections of step t) against
    torch.optim.Adam in its default configuration."""
    rng = np.random.default_rng(4)
    p = torch.tensor(rng.normal(size=1000), dtype=dtype).cuda()
    ref_p = p.clone().requires_grad_()
    opt = torch.optim.Adam([ref_p], lr=1e-3)
    mo, ve = torch.zeros_like(p), torch.zeros_like(p)
    for t in range(1, 6):
        g = torch.tensor(rng.normal(size=1000) * 10 ** rng.uniform(-3, 1), dtype=dtype).cuda()
        ref_p.grad = g.clone()
        opt.step()
        nqs.adam_update(p.data_ptr(), g, mo, ve, lr=1e-3, t=t)
        assert torch.max(torch.abs(p - ref_p.detach())).item() < tol, t
