"""Sectors defined by general quantum numbers on the GPU (amp_model_set_symmetries;
paper: "Physicality evaluation algorithm", Algorithm 1 for any number of
symmetries; Appendix A) against the oracle's GeneralSector: sampler replay bit
for bit, FP64 amplitudes and local energies, the bf16 fused kernel's masks, Z2
parities composed with an additive symmetry, and the empty-sector error."""
import numpy as np
import pytest
import torch

from oracle.hamiltonian import slater_condon_row, z2_symmetries
from oracle.model import MLPModel, TransformerModel
from oracle.sampler import sample_tree
from oracle.sector import GeneralSector, Sector, particle_number_eigs
from oracle.vmc import local_energies
from synth import (flatten_params, make_integrals, make_mlp_params, make_transformer_params,
                   mlp_param_spec, transformer_param_spec)

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def nqs():
    from paper_2310_04166_amd import nqs as mod
    mod.lib()
    return mod


def dev(a):
    return torch.as_tensor(np.asarray(a, dtype=np.uint64).view(np.int64)).cuda()


def weighted_n(n):
    """N_alpha + 2 N_beta: alpha qubits count 1, beta qubits 2."""
    return [b * (1 if q % 2 == 0 else 2) for q in range(2 * n) for b in (0, 1)]


@pytest.mark.parametrize("name,eig,targets", [
    ("total N = 4", lambda n: [particle_number_eigs(n)], [4]),
    ("N_alpha + 2 N_beta = 6", lambda n: [weighted_n(n)], [6]),
])
def test_mlp_fp64_replay_amplitudes_local_energy(nqs, name, eig, targets):
    n = 6
    sec = GeneralSector(n, eig(n), targets)
    members = sec.enumerate()
    params = make_mlp_params(n, 64, seed=21, std=0.5)
    ref = MLPModel(params, sec)
    m = nqs.Model(nqs.MODEL_MLP, [n, 2, 2, 64], flatten_params(params, mlp_param_spec(n, 64)),
                  "fp64")
    m.set_symmetries(eig(n), targets)
    # sampler: the same Philox keys and FP64 conditionals give the same tree
    ox, oc, olost = sample_tree(ref, 40_000, 9)
    x, c, lost = nqs.sample_unique(m, 40_000, 9)
    xv = [int(v) for v in x.cpu().numpy().view(np.uint64)]
    print(f"{name}: {len(members)} members, {len(xv)} unique samples, "
          f"(N_alpha, N_beta) blocks {sorted({(bin(v & 0x555).count('1'), bin(v & 0xAAA).count('1')) for v in xv})}")
    assert lost == olost == 0 and xv == ox and c.cpu().tolist() == oc
    # amplitudes on the whole sector and outside it
    la, ph = nqs.amp_forward(m, dev(members))
    rla, rph = (v.detach().numpy() for v in ref.amplitudes(members))
    assert np.max(np.abs(la.cpu().numpy() - rla)) < 1e-12
    assert np.max(np.abs(ph.cpu().numpy() - rph)) < 1e-12
    assert abs(np.exp(2 * la.cpu().numpy()).sum() - 1.0) < 1e-12
    inside = set(members)
    outside = [v for v in range(1 << 12) if v not in inside][::37]
    la_out, _ = nqs.amp_forward(m, dev(outside))
    assert torch.all(torch.isneginf(la_out))
    # local energies of samples from several (N_alpha, N_beta) blocks: each
    # sample's own block of connected x'
    h, eri = make_integrals(n, 12, 5)
    ham = nqs.ham_compile(h, eri, 2, 2)
    eloc, _, npairs = nqs.local_energy(ham, m, x, c)
    want = local_energies(ref, h, eri, ox)
    assert npairs == sum(len(slater_condon_row(h, eri, v)[0]) - 1 for v in ox)
    assert np.max(np.abs(eloc.cpu().numpy() - want) / np.abs(want)) < 1e-10


def test_additive_symmetry_with_z2_parities(nqs):
    """Total particle number 4 composed with the four Z2 symmetries of the
    12-spin-orbital system with point-group labels (the oracle's null space of
    the flip masks: two point-group generators and the alpha / beta parities,
    which the total particle number alone does not fix), targets those of the
    HF determinant."""
    n = 6
    irreps = [0, 0, 1, 2, 1, 3]
    h, eri = make_integrals(n, 12, 1, irreps=irreps)
    z2 = z2_symmetries(h, eri)
    assert len(z2) == 4
    hf = 0b1111
    zt = [bin(hf & mk).count("1") & 1 for mk in z2]
    sec = GeneralSector(n, [particle_number_eigs(n)], [4], z2, zt)
    params = make_mlp_params(n, 64, seed=22, std=0.5)
    ref = MLPModel(params, sec)
    m = nqs.Model(nqs.MODEL_MLP, [n, 2, 2, 64], flatten_params(params, mlp_param_spec(n, 64)),
                  "fp64")
    m.set_symmetries([particle_number_eigs(n)], [4], z2, zt)
    ox, oc, _ = sample_tree(ref, 20_000, 4)
    x, c, lost = nqs.sample_unique(m, 20_000, 4)
    assert [int(v) for v in x.cpu().numpy().view(np.uint64)] == ox and c.cpu().tolist() == oc
    assert all(sec.contains(v) for v in ox)
    la, _ = nqs.amp_forward(m, dev(sec.enumerate()))
    assert abs(np.exp(2 * la.cpu().numpy()).sum() - 1.0) < 1e-12
    # back to the plain (2, 2) sector
    m.set_symmetries()
    la2, _ = nqs.amp_forward(m, dev(Sector(n, 2, 2).enumerate()))
    assert abs(np.exp(2 * la2.cpu().numpy()).sum() - 1.0) < 1e-12


def test_bf16_fused_masks_on_general_sector(nqs):
    """The fused bf16 transformer on the N_alpha + 2 N_beta = 10 sector of 16
    spin-orbitals: -inf exactly outside it, normalised on it, amplitudes within
    the bf16 tolerance of the FP64 oracle, samples inside it."""
    n = 8
    eig, targets = [weighted_n(n)], [10]
    sec = GeneralSector(n, eig, targets)
    members = sec.enumerate()
    params = make_transformer_params(n, 4, 3, 64, 2, seed=5, std=0.05, round_to="bf16")
    ref = TransformerModel(params, sec, 4)
    m = nqs.Model(nqs.MODEL_TRANSFORMER, [n, 4, 3, 64, 2, 4, 256, 256],
                  flatten_params(params, transformer_param_spec(n, 64, 2, 256, 256)), "bf16")
    m.set_symmetries(eig, targets)
    la, _ = nqs.amp_forward(m, dev(members))
    with torch.no_grad():
        rla = np.concatenate([ref.amplitudes(members[i:i + 2048])[0].numpy()
                              for i in range(0, len(members), 2048)])
    la = la.cpu().numpy()
    print(f"bf16 general sector: {len(members)} members, max |dlog psi| {np.max(np.abs(la - rla)):.1e}")
    assert np.max(np.abs(la - rla)) < 2e-2
    assert abs(np.exp(2 * la).sum() - 1.0) < 1e-3
    inside = set(members)
    outside = [v for v in range(0, 1 << 16, 7) if v not in inside]
    la_out, _ = nqs.amp_forward(m, dev(outside))
    assert torch.all(torch.isneginf(la_out))
    x, c, lost = nqs.sample_unique(m, 200_000, 2)
    assert lost == 0 and int(c.sum()) == 200_000
    assert all(int(v) in inside for v in x.cpu().numpy().view(np.uint64))


def test_empty_general_sector_is_an_error(nqs):
    n = 4
    params = make_mlp_params(n, 16, seed=1)
    m = nqs.Model(nqs.MODEL_MLP, [n, 2, 2, 16], flatten_params(params, mlp_param_spec(n, 16)),
                  "fp64")
    with pytest.raises(nqs.NQSError) as e:
        m.set_symmetries([particle_number_eigs(n)], [9])      # 9 electrons on 8 qubits
    assert e.value.status == -1
