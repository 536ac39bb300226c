"""Pins of the oracle's Z2 symmetries (paper: "Molecular symmetries") and of
Algorithm 1 with Z2 eigenvalues composed by multiplication.

The synthetic integrals carry orbital irreps of Z2 x Z2 (a C2v-like point
group), so the Hamiltonian has two spatial Z2 symmetries besides the parities
of the alpha and beta electron numbers: four in all, as Table 1 lists for LiH.
"""
import itertools

import numpy as np
import pytest
import torch

from oracle.ed import ground_state
from oracle.hamiltonian import gf2_span_key, literal_row, sector_matrix, z2_symmetries
from oracle.model import MLPModel
from oracle.sampler import sample_tree
from oracle.sector import Sector, eigs, tokens_of
from oracle.vmc import exact_probabilities
from synth import make_integrals, make_mlp_params

N_ORB, RANK, SEED = 6, 12, 1
IRREPS = [0, 0, 1, 2, 1, 3]
ALPHA = sum(1 << (2 * p) for p in range(N_ORB))
BETA = ALPHA << 1


def irrep_mask(bit):
    return sum(3 << (2 * p) for p in range(N_ORB) if (IRREPS[p] >> bit) & 1)


@pytest.fixture(scope="module")
def sym():
    h, eri = make_integrals(N_ORB, RANK, SEED, irreps=IRREPS)
    return h, eri, z2_symmetries(h, eri)


def parity(x, m):
    return bin(x & m).count("1") & 1


def test_generic_integrals_have_only_the_electron_parities():
    h, eri = make_integrals(N_ORB, RANK, SEED)
    assert gf2_span_key(z2_symmetries(h, eri)) == gf2_span_key([ALPHA, BETA])


def test_irreps_give_four_symmetries(sym):
    _, _, gens = sym
    assert len(gens) == 4
    assert gf2_span_key(gens) == gf2_span_key([ALPHA, BETA, irrep_mask(0), irrep_mask(1)])


def test_symmetries_commute_with_the_literal_hamiltonian(sym):
    """Every nonzero matrix element (operator application, all 4-electron
    determinants) connects determinants of equal parity for each generator;
    a single-qubit Z is broken by some element."""
    h, eri, gens = sym
    dets = [sum(1 << j for j in c) for c in itertools.combinations(range(2 * N_ORB), 4)]
    broken = {1 << j: False for j in range(2 * N_ORB)}
    for x in dets:
        for xp, v in literal_row(h, eri, x).items():
            if abs(v) < 1e-14 or xp == x:
                continue
            for m in gens:
                assert parity(x, m) == parity(xp, m)
            for m in broken:
                broken[m] |= parity(x, m) != parity(xp, m)
    assert all(broken.values())


def test_sector_size_and_tree_count(sym):
    """With Z2: the sector is the (2, 2) determinants with the HF eigenvalues
    (brute force); the tree walk of the physical-children masks reaches
    exactly them."""
    _, _, gens = sym
    full = Sector(N_ORB, 2, 2)
    sec = Sector(N_ORB, 2, 2, gens)
    brute = [x for x in full.enumerate()
             if all(parity(x, m) == parity(sec.x_hf, m) for m in gens)]
    assert sec.enumerate() == brute
    assert len(full.enumerate()) == 225 and 0 < len(brute) < 225

    def walk(p, x, a, b):
        if p == N_ORB:
            return [x]
        out = []
        for k, ok in enumerate(sec.child_mask(p, a, b, sec.prefix_z2(x, p))):
            if ok:
                out += walk(p + 1, x | ((k & 1) << (2 * p)) | ((k >> 1) << (2 * p + 1)),
                            a + (k & 1), b + (k >> 1))
        return out
    assert sorted(walk(0, 0, 0, 0)) == brute


def test_isphys_with_z2_matches_brute_force(sym):
    """Algorithm 1 on every token prefix equals: some completion is in the sector."""
    _, _, gens = sym
    sec = Sector(N_ORB, 2, 2, gens)
    members = set(sec.enumerate())
    for p in range(N_ORB + 1):
        for prefix in itertools.product(range(4), repeat=p):
            x = sum(((t & 1) << (2 * q)) | ((t >> 1) << (2 * q + 1)) for q, t in enumerate(prefix))
            a = sum(t & 1 for t in prefix)
            b = sum(t >> 1 for t in prefix)
            expect = any((x | (y << (2 * p))) in members for y in range(1 << (2 * (N_ORB - p))))
            assert sec.token_phys(p, a, b, sec.prefix_z2(x, p)) == expect


def test_ground_state_lies_in_one_z2_block(sym):
    """H is block diagonal in the Z2 eigenvalues: the ground vector of the full
    (2, 2) sector is supported on determinants of a single set of eigenvalues,
    and the HF block's lowest energy is variational."""
    h, eri, gens = sym
    full = Sector(N_ORB, 2, 2)
    basis = full.enumerate()
    H = sector_matrix(h, eri, basis, route="literal")
    e0, v0 = ground_state(H)
    support = {tuple(parity(x, m) for m in gens) for x, v in zip(basis, v0) if abs(v) > 1e-9}
    assert len(support) == 1
    sec = Sector(N_ORB, 2, 2, gens)
    Hs = sector_matrix(h, eri, sec.enumerate(), route="literal")
    assert ground_state(Hs)[0] >= e0 - 1e-10


def test_masked_model_is_normalised_on_the_z2_sector(sym):
    _, _, gens = sym
    sec = Sector(N_ORB, 2, 2, gens)
    m = MLPModel(make_mlp_params(N_ORB, 64, seed=3, std=0.5), sec)
    probs = exact_probabilities(m, sec.enumerate())
    assert abs(probs.sum() - 1.0) < 1e-12
    # a (2, 2) determinant outside the Z2 sector has amplitude zero
    outside = [x for x in Sector(N_ORB, 2, 2).enumerate() if not sec.contains(x)]
    la, _ = m.amplitudes(outside[:20])
    assert torch.all(torch.isinf(la.detach()))


def test_sampler_stays_in_the_z2_sector(sym):
    _, _, gens = sym
    sec = Sector(N_ORB, 2, 2, gens)
    m = MLPModel(make_mlp_params(N_ORB, 64, seed=3, std=0.5), sec)
    cfg, cnt, lost = sample_tree(m, 20_000, 9)
    assert lost == 0 and sum(cnt) == 20_000
    assert all(sec.contains(x) for x in cfg)
    assert all(eigs(x, sec.N, gens)[2:] == sec.s_ref[2:] for x in cfg)
