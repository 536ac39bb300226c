"""Pins of the oracle's general sector (Algorithm 1 with any additive quantum
numbers and Z2 parities; paper: "Physicality evaluation algorithm", Appendix A)."""
import itertools
from math import comb

import numpy as np
import pytest
import torch

from oracle.model import MLPModel
from oracle.sector import GeneralSector, Sector, particle_number_eigs, two_sz_eigs
from oracle.vmc import exact_probabilities
from synth import make_mlp_params


def brute_force(n, eig, targets, z2=(), z2_targets=()):
    out = []
    for x in range(1 << (2 * n)):
        sums = tuple(sum(e[2 * i + ((x >> i) & 1)] for i in range(2 * n)) for e in eig)
        par = tuple(bin(x & m).count("1") & 1 for m in z2)
        if sums == tuple(targets) and par == tuple(z2_targets or (0,) * len(z2)):
            out.append(x)
    return out


def test_reduces_to_the_particle_number_and_spin_sector():
    """Particle number and 2 S_z as general additive symmetries give the same
    configurations and the same child masks as the (N_alpha, N_beta) sector."""
    n = 5
    for na, nb in ((2, 2), (3, 1), (0, 4), (5, 5)):
        g = GeneralSector(n, [particle_number_eigs(n), two_sz_eigs(n)], [na + nb, na - nb])
        s = Sector(n, na, nb)
        assert g.enumerate() == s.enumerate()
        for x in s.enumerate()[:40]:
            for p in range(n):
                a = bin(x & 0x5555555555 & ((1 << (2 * p)) - 1)).count("1")
                b = bin(x & 0xAAAAAAAAAA & ((1 << (2 * p)) - 1)).count("1")
                assert g.child_mask_state(p, g.prefix_state(x, p)) == s.child_mask(p, a, b)


@pytest.mark.parametrize("eig_fn,targets,size", [
    (lambda n: [particle_number_eigs(n)], [4], comb(12, 4)),         # total N only: 495
    (lambda n: [two_sz_eigs(n)], [0], sum(comb(6, k) ** 2 for k in range(7))),  # S_z = 0: 924
    # N_alpha + 2 N_beta = 6: (6,0), (4,1), (2,2), (0,3)
    (lambda n: [[b * (1 if i % 2 == 0 else 2) for i in range(2 * n) for b in (0, 1)]], [6],
     comb(6, 6) + comb(6, 4) * 6 + comb(6, 2) ** 2 + comb(6, 3)),
])
def test_sector_equals_brute_force_and_closed_form(eig_fn, targets, size):
    n = 6
    eig = eig_fn(n)
    g = GeneralSector(n, eig, targets)
    got = g.enumerate()
    assert got == brute_force(n, eig, targets)
    assert len(got) == size


def test_with_z2_parities_and_token_prefixes():
    """Total particle number 4 on 8 qubits with two Z2 masks: the sector equals
    brute force, and every token prefix is physical exactly when some member of
    the sector starts with it."""
    n = 4
    eig, z2, zt = [particle_number_eigs(n)], (0b00110011, 0b01011010), (1, 0)
    g = GeneralSector(n, eig, [4], z2, zt)
    members = g.enumerate()
    assert members == brute_force(n, eig, [4], z2, zt)
    for p in range(n + 1):
        for toks in itertools.product(range(4), repeat=p):
            x = sum(t << (2 * q) for q, t in enumerate(toks))
            below = (1 << (2 * p)) - 1
            reachable = any((y & below) == x for y in members)
            assert g.isphys(2 * p, g.prefix_state(x, p)) == reachable


def test_masked_model_normalised_on_general_sector():
    """The MLP with Mask-Unphysical over the total-particle-number sector:
    Born probabilities sum to 1 over the 495 members and vanish outside."""
    n = 6
    g = GeneralSector(n, [particle_number_eigs(n)], [4])
    m = MLPModel(make_mlp_params(n, 16, seed=3, std=0.5), g)
    p = exact_probabilities(m, g.enumerate())
    assert abs(p.sum() - 1.0) < 1e-12 and p.min() > 0
    outside = [x for x in Sector(n, 2, 2).enumerate()[:5]] + [0b111111]
    inside = set(g.enumerate())
    q = exact_probabilities(m, [x for x in outside if x not in inside])
    assert np.all(q == 0)
