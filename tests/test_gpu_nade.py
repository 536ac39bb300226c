"""GPU parity of the paper's per-qubit complex-weight ansatz (NQS_MODEL_NADE;
paper: Appendix "ANQS architecture", qubit-level Mask-Unphysical) against the
oracle (oracle/nade.py)."""
import numpy as np
import pytest
import torch

from oracle.nade import NADEModel
from oracle.sampler import sample_tree
from oracle.sector import Sector
from oracle.vmc import local_energies
from synth import flatten_params, make_integrals, make_nade_params, nade_param_spec

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


def pair(nqs, n, na, nb, hidden, seed, precision="fp64", strategy="MU", d=0, std=0.3):
    params = make_nade_params(n, hidden, seed=seed, std=std, bias_std=0.2)
    sec = Sector(n, na, nb)
    ml = {"MU": n, "DU": 0, "MUd": n - d}[strategy]
    ref = NADEModel(params, sec, mask_levels=ml)
    m = nqs.Model(nqs.MODEL_NADE, [n, na, nb, hidden],
                  flatten_params(params, nade_param_spec(n, hidden)), precision, strategy, d)
    return params, sec, ref, m


@pytest.mark.parametrize("n,na,nb,hidden,precision,std,tol", [
    (4, 2, 1, 16, "fp64", 0.3, 1e-12), (6, 2, 2, 64, "fp64", 0.3, 1e-12),
    (6, 2, 2, 64, "fp32", 0.1, 1e-4)])
def test_forward(nqs, n, na, nb, hidden, precision, std, tol):
    """FP32 tolerance: the complex tanh has poles at i pi / 2, near which float32
    rounding of its argument is amplified; smaller weights keep away from them."""
    _, sec, ref, m = pair(nqs, n, na, nb, hidden, 3, precision, std=std)
    xs = sec.enumerate()
    la, ph = nqs.amp_forward(m, dev(xs))
    rla, rph = ref.amplitudes(xs)
    e_la = np.max(np.abs(la.cpu().numpy() - rla.detach().numpy()))
    e_ph = np.max(np.abs(ph.cpu().numpy() - rph.detach().numpy()))
    log(f"nade forward n={n} H={hidden} {precision}: |dla| {e_la:.2e} |dph| {e_ph:.2e}")
    assert e_la < tol and e_ph < tol
    assert abs(np.exp(2 * la.cpu().numpy()).sum() - 1.0) < max(tol, 1e-10)


def test_forward_discard_unphysical(nqs):
    """DU: no masks, the amplitude of every bit string is the network's."""
    _, sec, ref, m = pair(nqs, 4, 2, 1, 16, 4, strategy="DU")
    xs = list(range(256))
    la, ph = nqs.amp_forward(m, dev(xs))
    rla, rph = ref.amplitudes(xs)
    rla = rla.detach().numpy()
    # unmasked strings far outside the sector have |log psi| of several tens and
    # drive the complex tanh near its poles, whose condition number amplifies the
    # different FP64 summation orders of the two GEMMs: bound relative to the value
    scale = np.maximum(np.abs(rla), 1.0)
    e_la = np.max(np.abs(la.cpu().numpy() - rla) / scale)
    rph = rph.detach().numpy()
    e_ph = np.max(np.abs(ph.cpu().numpy() - rph) / np.maximum(np.abs(rph), 1.0))
    log(f"nade forward DU on all strings: max |log psi| {np.max(np.abs(rla)):.1f}, "
        f"rel err {e_la:.2e} / {e_ph:.2e}")
    assert e_la < 1e-10 and e_ph < 1e-10
    assert abs(np.exp(2 * la.cpu().numpy()).sum() - 1.0) < 1e-10


@pytest.mark.parametrize("strategy,d", [("MU", 0), ("DU", 0), ("MUd", 1)])
def test_sampler_replay_fp64(nqs, strategy, d):
    _, sec, ref, m = pair(nqs, 5, 2, 2, 32, 6, strategy=strategy, d=d, std=0.2)
    cfg_o, cnt_o, lost_o = sample_tree(ref, 40_000, 9, strategy=strategy, d=d)
    c, k, lost = nqs.sample_unique(m, 40_000, 9)
    log(f"nade sampler {strategy}: {len(cfg_o)} unique, lost {lost_o}")
    assert lost == lost_o
    assert [int(v) for v in c.cpu().numpy().view(np.uint64)] == cfg_o
    assert k.cpu().tolist() == cnt_o


@pytest.mark.parametrize("precision,tol", [("fp64", 1e-10), ("fp32", 2e-4)])
def test_backward(nqs, precision, tol):
    params, sec, _, m = pair(nqs, 4, 2, 2, 16, 8, precision)
    spec = nade_param_spec(4, 16)
    xs = sec.enumerate()
    rng = np.random.default_rng(2)
    g = rng.normal(size=(2, len(xs)))
    grad = nqs.amp_backward(m, dev(xs), torch.tensor(g[0]).cuda(), torch.tensor(g[1]).cuda())
    ref = NADEModel(params, sec, requires_grad=True)
    la, ph = ref.amplitudes(xs)
    (torch.sum(torch.tensor(g[0]) * la) + torch.sum(torch.tensor(g[1]) * ph)).backward()
    want = ref.flat_grad(spec)
    err = np.max(np.abs(grad.double().cpu().numpy() - want)) / np.max(np.abs(want))
    log(f"nade backward {precision}: max rel err {err:.2e}")
    assert err < tol


def test_local_energy_fp64(nqs):
    h, eri = make_integrals(5, 10, 3)
    _, sec, ref, m = pair(nqs, 5, 2, 2, 32, 11)
    ham = nqs.ham_compile(h, eri, 2, 2)
    xs = sec.enumerate()[::3]
    eloc, _, _ = nqs.local_energy(ham, m, dev(xs), torch.ones(len(xs), dtype=torch.int64).cuda())
    want = local_energies(ref, h, eri, xs)
    assert np.max(np.abs(eloc.cpu().numpy() - want) / np.maximum(np.abs(want), 1.0)) < 1e-10
