"""connected_pairs_noalloc (the entry point that allocates nothing, its scratch
in a fixed device array) against connected_pairs on the same inputs: two calls
in a row, the second with fewer configurations, bit-identical offsets, x',
matrix elements and diagonals; its size limit and preconditions."""
import numpy as np
import pytest
import torch

from oracle.sector import Sector
from synth import make_integrals

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def nqs():
    from paper_2310_04166_amd import nqs as mod
    mod.lib()
    return mod


def dev(a):
    return torch.as_tensor(np.asarray(a, dtype=np.uint64).view(np.int64)).cuda()


def compare(nqs, H, x):
    off, xp, hv, hd = nqs.connected_pairs(H, x)
    n, total = x.numel(), xp.numel()
    o2 = torch.full((n + 1,), -1, dtype=torch.int64, device="cuda")
    xp2 = torch.full((total + 7,), -1, dtype=torch.int64, device="cuda")
    hv2 = torch.full((total + 7,), np.nan, dtype=torch.float64, device="cuda")
    hd2 = torch.full((max(n, 1),), np.nan, dtype=torch.float64, device="cuda")
    got = nqs.connected_pairs_noalloc(H, x, o2, xp2, hv2, hd2)
    assert got == total
    assert torch.equal(o2, off)
    assert torch.equal(xp2[:total], xp) and torch.equal(hv2[:total], hv)
    assert torch.equal(hd2[:n], hd)
    assert bool(torch.all(xp2[total:] == -1))          # nothing beyond the pairs
    return total


def test_noalloc_matches_connected_pairs_two_calls(nqs):
    """20 spin-orbitals, 5+5: first 20,001 configurations (a 20-tile scan over
    the fixed workspace), then 3,001 (the one-block scan), then 9,217 (10
    tiles) -- the array keeps the previous call's contents in between."""
    h, eri = make_integrals(10, 20, 7)
    H = nqs.ham_compile(h, eri, 5, 5)
    basis = Sector(10, 5, 5).enumerate()
    rng = np.random.default_rng(3)
    for n in (20_001, 3_001, 9_217):
        xs = [basis[i] for i in rng.choice(len(basis), n, replace=False)]
        total = compare(nqs, H, dev(xs))
        print(f"n = {n}: {total} pairs", flush=True)
        assert total == 875 * n


def test_noalloc_limits(nqs):
    h, eri = make_integrals(6, 12, 1)
    H = nqs.ham_compile(h, eri, 2, 2)
    xs = dev(Sector(6, 2, 2).enumerate())
    o = torch.empty(226, dtype=torch.int64, device="cuda")
    hd = torch.empty(225, dtype=torch.float64, device="cuda")
    small = torch.empty(10, dtype=torch.int64, device="cuda")
    smallh = torch.empty(10, dtype=torch.float64, device="cuda")
    # the tables are not on the device before any other call with the Hamiltonian
    with pytest.raises(nqs.NQSError) as e:
        nqs.connected_pairs_noalloc(H, xs, o, small, smallh, hd)
    assert e.value.status == -1
    nqs.connected_pairs(H, xs[:1])                      # uploads the tables
    with pytest.raises(nqs.NQSError) as e:
        nqs.connected_pairs_noalloc(H, xs, o, small, smallh, hd)
    assert e.value.status == -2                         # capacity
    big = torch.zeros(nqs.NOALLOC_MAX_CONFIGS + 1, dtype=torch.int64, device="cuda")
    ob = torch.empty(big.numel() + 1, dtype=torch.int64, device="cuda")
    with pytest.raises(nqs.NQSError) as e:
        nqs.connected_pairs_noalloc(H, big, ob, small, smallh, hd)
    assert e.value.status == -3
    # empty input
    assert nqs.connected_pairs_noalloc(H, xs[:0], o[:1], small, smallh, hd) == 0
    assert int(o[0]) == 0
