"""Pins of the oracle's sector enumeration and of Algorithm 1 (IsPhys)."""
import json
import os
from itertools import product
from math import comb

import pytest

from oracle.sector import Sector, eigs, hf_config, tokens_of, config_of

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "table1_sector_sizes.json")


def physical_leaf_count(sec):
    """Number of physical leaves, walking only through nodes Algorithm 1 keeps."""
    n = sec.n
    layer = {(0, 0): 1}
    for p in range(n):
        nxt = {}
        for (a, b), w in layer.items():
            for k in range(4):
                a2, b2 = a + (k & 1), b + (k >> 1)
                if sec.token_phys(p + 1, a2, b2):
                    nxt[(a2, b2)] = nxt.get((a2, b2), 0) + w
        layer = nxt
    return sum(layer.values())


@pytest.mark.parametrize("row", json.load(open(GOLDEN))["rows"], ids=lambda r: r["molecule"])
def test_table1_without_z2(row):
    n, ne = row["N"] // 2, row["n_e"]
    sec = Sector(n, ne // 2, ne // 2)
    assert physical_leaf_count(sec) == row["without_z2"]
    assert comb(n, ne // 2) ** 2 == row["without_z2"]
    if row["without_z2"] <= 50_000:
        basis = sec.enumerate()
        assert len(basis) == row["without_z2"]
        assert all(sec.contains(x) for x in basis[:: max(1, len(basis) // 500)])


@pytest.mark.parametrize("n,na,nb", [(4, 1, 2), (5, 2, 2), (6, 2, 2), (6, 3, 1), (6, 0, 3)])
def test_isphys_closed_form_and_brute_force(n, na, nb):
    sec = Sector(n, na, nb)
    for p in range(n + 1):
        for a in range(n + 1):
            for b in range(n + 1):
                closed = (a <= na <= a + n - p) and (b <= nb <= b + n - p)
                assert sec.token_phys(p, a, b) == closed
    # brute force: a prefix is physical iff some continuation lands in the sector
    for p in range(n + 1):
        for prefix in product(range(4), repeat=p):
            conts = product(range(4), repeat=n - p)
            brute = any(sec.contains(config_of(list(prefix) + list(c))) for c in conts)
            a = sum(t & 1 for t in prefix)
            b = sum(t >> 1 for t in prefix)
            assert sec.token_phys(p, a, b) == brute


def test_isphys_qubit_level_brute_force():
    """Algorithm 1 on the binary tree at odd qubit depths (mid-token)."""
    sec = Sector(4, 2, 1)
    N = sec.N
    for i in range(1, N + 2):
        for bits in product((0, 1), repeat=i - 1):
            x = sum(bit << j for j, bit in enumerate(bits))
            s = eigs(x, i - 1)
            brute = any(sec.contains(x | (c << (i - 1))) for c in range(1 << (N - i + 1)))
            assert sec.isphys(i, s) == brute


def test_ad_hoc_particle_number_rule():
    """A prefix holding more than n_e electrons is never physical."""
    sec = Sector(6, 2, 2)
    for p in range(7):
        for a in range(7):
            for b in range(7):
                if a + b > 4:
                    assert not sec.token_phys(p, a, b)


def test_last_token_always_masked():
    """With particle number fixed, the last token of a physical prefix is forced."""
    for n, na, nb in [(6, 2, 2), (10, 5, 5), (15, 7, 7)]:
        sec = Sector(n, na, nb)
        for a in range(n + 1):
            for b in range(n + 1):
                if sec.token_phys(n - 1, a, b):
                    assert sum(sec.child_mask(n - 1, a, b)) == 1


def test_hf_and_sz_eigenvalues():
    sec = Sector(6, 2, 2)
    x = hf_config(6, 2, 2)
    assert x == 0b1111
    assert eigs(x, 12) == (4, 0)
    assert eigs(hf_config(6, 3, 1), 12) == (4, 2)
    assert tokens_of(x, 6) == [3, 3, 0, 0, 0, 0]
    assert config_of(tokens_of(0b100110, 3)) == 0b100110
