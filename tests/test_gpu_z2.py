"""GPU parity of the Z2-restricted sector (paper: "Molecular symmetries",
Algorithm 1 with Z2 eigenvalues) against the oracle.

Integrals with orbital irreps give the Hamiltonian point-group Z2 symmetries;
the library finds them (ham_z2_symmetries), the model is restricted to the
Hartree-Fock determinant's eigenvalues (amp_model_set_z2), and sampler,
forward and local energy are compared with the oracle restricted the same way.
"""
import numpy as np
import pytest
import torch

from oracle.ed import ground_state
from oracle.hamiltonian import sector_matrix, z2_symmetries
from oracle.model import MLPModel, TransformerModel
from oracle.sampler import sample_tree
from oracle.sector import Sector
from oracle.vmc import local_energies
from synth import (flatten_params, make_integrals, make_mlp_params, make_transformer_params,
                   mlp_param_spec, transformer_param_spec)

pytestmark = pytest.mark.gpu

TINY_IRREPS = [0, 0, 1, 2, 1, 3]                 # Z2 x Z2: two spatial symmetries
MID_IRREPS = [0, 1, 2, 4, 0, 3, 5, 6, 7, 1]      # Z2^3: three spatial symmetries


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


def tiny(nqs):
    h, eri = make_integrals(6, 12, 1, irreps=TINY_IRREPS)
    ham = nqs.ham_compile(h, eri, 2, 2)
    masks = ham.z2_symmetries()
    sec = Sector(6, 2, 2, z2_symmetries(h, eri))
    return h, eri, ham, masks, sec


def test_sampler_replay_and_forward_fp64(nqs):
    h, eri, ham, masks, sec = tiny(nqs)
    assert len(masks) == 2
    params = make_mlp_params(6, 64, seed=43, std=0.5)
    ref = MLPModel(params, sec)
    m = nqs.Model(nqs.MODEL_MLP, [6, 2, 2, 64], flatten_params(params, mlp_param_spec(6, 64)),
                  "fp64")
    m.set_z2(masks)
    cfg_o, cnt_o, lost_o = sample_tree(ref, 50_000, 5)
    c, k, lost = nqs.sample_unique(m, 50_000, 5)
    log(f"Z2 tiny: {len(cfg_o)} unique of a {len(sec.enumerate())}-determinant sector")
    assert lost == lost_o == 0
    assert [int(v) for v in c.cpu().numpy().view(np.uint64)] == cfg_o
    assert k.cpu().tolist() == cnt_o
    assert all(sec.contains(x) for x in cfg_o)
    # forward on the whole Z2 sector and on (2, 2) determinants outside it
    xs = sec.enumerate()
    la, ph = nqs.amp_forward(m, dev(xs))
    rla, rph = ref.amplitudes(xs)
    assert np.max(np.abs(la.cpu().numpy() - rla.detach().numpy())) < 1e-12
    assert np.max(np.abs(ph.cpu().numpy() - rph.detach().numpy())) < 1e-12
    assert abs(np.exp(2 * la.cpu().numpy()).sum() - 1.0) < 1e-12
    outside = [x for x in Sector(6, 2, 2).enumerate() if not sec.contains(x)]
    la_out, _ = nqs.amp_forward(m, dev(outside))
    assert torch.all(torch.isneginf(la_out))
    # removing the restriction gives back the plain (2, 2) model
    m.set_z2([])
    la_plain, _ = nqs.amp_forward(m, dev(outside))
    assert torch.all(torch.isfinite(la_plain))


def test_local_energy_fp64(nqs):
    h, eri, ham, masks, sec = tiny(nqs)
    params = make_mlp_params(6, 64, seed=44, std=0.5)
    ref = MLPModel(params, sec)
    m = nqs.Model(nqs.MODEL_MLP, [6, 2, 2, 64], flatten_params(params, mlp_param_spec(6, 64)),
                  "fp64")
    m.set_z2(masks)
    xs = sec.enumerate()
    eloc, sums, _ = nqs.local_energy(ham, m, dev(xs), torch.ones(len(xs), dtype=torch.int64).cuda())
    got = eloc.cpu().numpy()
    got = got[..., 0] + 1j * got[..., 1] if got.ndim == 2 else got
    expect = local_energies(ref, h, eri, xs)
    assert np.max(np.abs(got - expect) / np.maximum(np.abs(expect), 1.0)) < 1e-10


def test_bf16_fused_forward_and_sampler_with_three_symmetries(nqs):
    """20 spin-orbitals, 5+5 electrons, Z2^3 point group: the fused bf16 kernel's
    masks keep exactly the Z2 sector and the sampler stays in it."""
    n = 10
    h, eri = make_integrals(n, 20, 2, irreps=MID_IRREPS)
    ham = nqs.ham_compile(h, eri, 5, 5)
    masks = ham.z2_symmetries()
    assert len(masks) == 3
    sec = Sector(n, 5, 5, z2_symmetries(h, eri))
    params = make_transformer_params(n, 5, 5, 64, 2, seed=7, hf_bias=1.0, round_to="bf16")
    spec = transformer_param_spec(n, 64, 2, 256, 256)
    ref = TransformerModel(params, sec, 4)
    m = nqs.Model(nqs.MODEL_TRANSFORMER, [n, 5, 5, 64, 2, 4, 256, 256],
                  flatten_params(params, spec), "bf16")
    m.set_z2(masks)
    xs = sec.enumerate()
    log(f"Z2^3 sector: {len(xs)} of {len(Sector(n, 5, 5).enumerate())} determinants")
    la, ph = nqs.amp_forward(m, dev(xs))
    la = la.cpu().numpy()
    with torch.no_grad():
        rla = np.concatenate([ref.amplitudes(xs[i:i + 4096])[0].numpy()
                              for i in range(0, len(xs), 4096)])
    assert np.all(np.isfinite(la))
    assert np.max(np.abs(la - rla)) < 3e-2
    assert abs(np.exp(2 * la).sum() - 1.0) < 1e-3
    outside = [x for x in Sector(n, 5, 5).enumerate() if not sec.contains(x)][:2000]
    la_out, _ = nqs.amp_forward(m, dev(outside))
    assert torch.all(torch.isneginf(la_out))
    c, k, lost = nqs.sample_unique(m, 200_000, 3)
    assert lost == 0 and int(k.sum()) == 200_000
    members = set(xs)
    assert all(int(v) in members for v in c.cpu().numpy().view(np.uint64))


def test_vmc_reaches_the_z2_block_ground_state(nqs):
    """The optimisation of the chemical-accuracy test, restricted to the HF
    determinant's Z2 sector, reaches the lowest energy of that block."""
    h, eri, ham, masks, sec = tiny(nqs)
    basis = sec.enumerate()
    e_block = ground_state(sector_matrix(h, eri, basis, route="literal"))[0]
    params = make_mlp_params(6, 64, seed=1)
    model = nqs.Model(nqs.MODEL_MLP, [6, 2, 2, 64],
                      flatten_params(params, mlp_param_spec(6, 64)), "fp64")
    model.set_z2(masks)
    grad = torch.zeros(model.n_params, dtype=torch.float64, device="cuda")
    mo, ve = torch.zeros_like(grad), torch.zeros_like(grad)
    for t in range(1, 4001):
        ns = 10 ** 5 if t <= 100 else 10 ** 6 if t <= 200 else 10 ** 7 if t <= 1000 else 10 ** 8
        x, c, lost = nqs.sample_unique(model, ns, t)
        la, ph = nqs.amp_forward(model, x)
        eloc, sums, _ = nqs.local_energy(ham, model, x, c, la, ph)
        gl, gp = nqs.vmc_weights(eloc, c, sums)
        grad = nqs.amp_backward(model, x, gl, gp, grad=grad)
        nqs.adam_update(model.params_ptr(), grad, mo, ve, lr=1e-3, t=t)
        model.sync()
    la, ph = nqs.amp_forward(model, dev(basis))
    psi = np.exp(la.cpu().numpy() + 1j * ph.cpu().numpy())
    H = sector_matrix(h, eri, basis, route="literal")
    e_var = float(np.real(np.vdot(psi, H @ psi) / np.vdot(psi, psi)))
    log(f"Z2 block of {len(basis)} determinants: E_block {e_block:.8f}, optimised {e_var:.8f}, "
        f"error {e_var - e_block:.3e} Ha")
    assert e_block - 1e-9 <= e_var < e_block + 1.6e-3
