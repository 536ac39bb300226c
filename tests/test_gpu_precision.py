"""Mixed precision at trained weights (30 spin-orbitals, transformer d128 L4 h8).

Adam steps move the fp32 master weights off the bf16 grid, so the bf16 path is
checked after five full VMC steps at lr 1e-3 against the FP64 oracle evaluated
with the same fp32 master weights, on the same samples: every local energy of
the 16 highest-count samples within the first-order bound that the measured
log-amplitude error implies, the FP32 path's energy of those samples within
1e-6 Ha of the oracle, and the energy itself — the estimator over the 1024
highest-count samples plus 1024 drawn uniformly, and over 4096 draws in
proportion to the counts — within 1e-4 Ha of the FP32 path.

The bf16 error of a single local energy is a sum of many roundings of either
sign (~1e5 activations per configuration): at these weights the per-sample
errors are zero-mean (half of them positive) with an rms of ~3.4e-4 Ha, so the
energy of 16 samples carries ~9e-5 Ha of noise (measured 1.6e-5 .. 1.7e-4 Ha
over training trajectories that differ only in the rounding of the gradient).
That 16-sample energy is therefore held to three standard errors of its own
per-sample errors (a bias common to the samples would exceed it), and the
1e-4 Ha bar applies to the estimators.

First-order bound (local-energy equation): with Delta(x) the complex error of
log psi(x) (log|psi| and phase), E_loc(x) = sum_x' H_xx' psi(x')/psi(x) changes by
    |dE_loc(x)| <= sum_{x' != x} |H_xx'| |psi(x')/psi(x)| |Delta(x') - Delta(x)|
                <= 2 eps A(x),   A(x) = sum_{x' != x} |H_xx' psi(x')/psi(x)|,
eps = max |Delta| over x and its connected x' (second-order terms are below
eps^2 A(x))."""
import numpy as np
import pytest
import torch

from oracle.model import build_model
from synth import flatten_params, transformer_param_spec, unflatten_params, workload

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def nqs():
    from paper_2310_04166_amd import nqs as mod
    mod.lib()
    return mod


def log(msg):
    print(msg, flush=True)


def bf16_representable(a):
    u = np.asarray(a, dtype=np.float32).view(np.uint32)
    return (u & 0xFFFF) == 0


@pytest.fixture(scope="module")
def trained(nqs):
    """The precision workload after five VMC steps (sample 1e6, local energy,
    weights, hand-written backward, Adam lr 1e-3) in bf16."""
    cfg, h, eri, params = workload("precision")
    spec = transformer_param_spec(15, 128, 4, 512, 256)
    m = nqs.Model(nqs.MODEL_TRANSFORMER, nqs.model_dims(cfg), flatten_params(params, spec), "bf16")
    H = nqs.ham_compile(h, eri, 7, 7)
    dev = torch.device("cuda")
    g = torch.empty(m.n_params, dtype=torch.float32, device=dev)
    mom = torch.zeros(m.n_params, dtype=torch.float32, device=dev)
    var = torch.zeros(m.n_params, dtype=torch.float32, device=dev)
    for t in range(1, 6):
        x, c, _ = nqs.sample_unique(m, cfg["n_samples"], 100 + t)
        la, ph = nqs.amp_forward(m, x)
        eloc, sums, _ = nqs.local_energy(H, m, x, c, la, ph)
        gl, gp = nqs.vmc_weights(eloc, c, sums)
        nqs.amp_backward(m, x, gl, gp, grad=g)
        nqs.adam_update(m.params_ptr(), g, mom, var, lr=1e-3, t=t)
        m.sync()
        s = sums.cpu().numpy()
        log(f"  step {t}: unique {x.numel()} E {s[1] / s[0]:.6f}")
    return cfg, h, eri, spec, m, H


def test_trained_weights_off_grid(nqs, trained):
    """The premise: the master weights of the GEMMs are no longer bf16 numbers."""
    cfg, _, _, spec, m, _ = trained
    p = unflatten_params(m.get_params(), spec)
    mats = [k for k in p if k.split(".")[-1] in ("wqkv", "wo", "w1", "w2") or k == "ph_w2"]
    frac = np.mean(np.concatenate([~bf16_representable(p[k]).reshape(-1) for k in mats]))
    log(f"  fraction of GEMM weights off the bf16 grid: {frac:.4f}")
    assert frac > 0.9


def test_trained_weights_energy_vs_oracle(nqs, trained):
    import eloc_bound
    cfg, h, eri, spec, m, H = trained
    x, c, _ = nqs.sample_unique(m, cfg["n_samples"], 11)
    top = torch.argsort(c, descending=True)[:16]
    xs, cs = x[top].contiguous(), c[top].contiguous()
    e16, _, _ = nqs.local_energy(H, m, xs, cs)
    params = m.get_params()
    m32 = nqs.Model(nqs.MODEL_TRANSFORMER, nqs.model_dims(cfg), params, "fp32")
    e32, _, _ = nqs.local_energy(H, m32, xs, cs)
    ref = build_model(cfg, unflatten_params(params, spec))
    xv = [int(v) for v in xs.cpu().numpy().view(np.uint64)]
    w = cs.cpu().numpy().astype(np.float64)
    e16, e32 = e16.cpu().numpy(), e32.cpu().numpy()
    res = eloc_bound.check(ref, h, eri, xv, eloc_bound.gpu_amplitudes(nqs, m))
    eor = np.array([r[0] for r in res])
    bound = np.array([2 * r[2] * r[1] for r in res])
    for i, xi in enumerate(xv):
        log(f"  x={xi:#x} n={int(w[i])} E_loc oracle {eor[i].real:.6f} bf16 err "
            f"{abs(e16[i] - eor[i]):.2e} (bound {bound[i]:.2e}, eps {res[i][2]:.1e}, "
            f"A {res[i][1]:.1f}) fp32 err {abs(e32[i] - eor[i]):.1e}")
    E = lambda e: np.real(np.sum(w * e) / np.sum(w))
    d16, d32 = abs(E(e16) - E(eor)), abs(E(e32) - E(eor))
    err = np.real(e16 - eor)
    se = np.sqrt(np.sum(w ** 2 * err ** 2)) / np.sum(w)
    log(f"  energy of the 16 samples: oracle {E(eor):.8f}  |bf16 - oracle| {d16:.2e} "
        f"(standard error of the per-sample errors {se:.2e}, {np.mean(err > 0):.2f} of them "
        f"positive)  |fp32 - oracle| {d32:.2e}")
    assert np.all(np.abs(e16 - eor) <= 1.5 * bound + 1e-9)
    assert d32 <= 1e-6
    assert d16 <= 3 * se + 1e-6
    # the estimator over the 1024 highest-count samples and 1024 drawn at random
    order = torch.argsort(c, descending=True)
    rng = np.random.default_rng(0)
    pick = np.unique(np.concatenate([order[:1024].cpu().numpy(),
                                     rng.choice(x.numel(), min(1024, x.numel()), replace=False)]))
    idx = torch.as_tensor(pick, device=x.device)
    xa, ca = x[idx].contiguous(), c[idx].contiguous()
    _, s16, _ = nqs.local_energy(H, m, xa, ca)
    _, s32, _ = nqs.local_energy(H, m32, xa, ca)
    s16, s32 = s16.cpu().numpy(), s32.cpu().numpy()
    de = abs(s16[1] / s16[0] - s32[1] / s32[0])
    log(f"  estimator over {len(pick)} samples ({s16[0] / cfg['n_samples']:.2f} of the counts): "
        f"|bf16 - fp32| {de:.2e}")
    assert de <= 1e-4
    # and over 4096 draws in proportion to the counts (the estimator's own weighting)
    p = (c.double() / c.sum()).cpu().numpy()
    pick = np.unique(np.random.default_rng(1).choice(x.numel(), 4096, p=p))
    idx = torch.as_tensor(pick, device=x.device)
    xa, ca = x[idx].contiguous(), c[idx].contiguous()
    _, s16, _ = nqs.local_energy(H, m, xa, ca)
    _, s32, _ = nqs.local_energy(H, m32, xa, ca)
    s16, s32 = s16.cpu().numpy(), s32.cpu().numpy()
    dw = abs(s16[1] / s16[0] - s32[1] / s32[0])
    log(f"  estimator over the {len(pick)} samples of 4096 count-weighted draws: |bf16 - fp32| {dw:.2e}")
    assert dw <= 1e-4
