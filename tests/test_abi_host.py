"""Host-side tests of the C-ABI library: it loads, exports every declared
symbol, and its Hamiltonian compiler (host C++) reproduces the oracle's
matrix elements.  No GPU work is launched here."""
import os
import re

import numpy as np
import pytest

from oracle.hamiltonian import sector_matrix, slater_condon_row
from oracle.sector import Sector
from synth import make_integrals

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def nqs():
    from paper_2310_04166_amd import nqs as mod
    if not os.path.exists(mod.LIB_PATH):
        from paper_2310_04166_amd.build import build
        build()
    mod.lib()
    return mod


def declared_functions():
    text = open(os.path.join(ROOT, "include", "nqs.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:int|void|const char \*)\s*\*?\s*(\w+)\s*\(", text, flags=re.M)))


def test_exports_every_declared_symbol(nqs):
    names = declared_functions()
    assert len(names) >= 15
    L = nqs.lib()
    for name in names:
        assert hasattr(L, name), name
    assert set(names) == set(nqs.EXPORTS)


def table_matrix(tables, basis):
    flip, off, z, c = tables
    index = {int(b): i for i, b in enumerate(basis)}
    H = np.zeros((len(basis), len(basis)))
    for col, x in enumerate(basis):
        for g in range(len(flip)):
            xp = x ^ int(flip[g])
            if xp not in index:
                continue
            v = 0.0
            for t in range(off[g], off[g + 1]):
                v += -c[t] if bin(x & int(z[t])).count("1") & 1 else c[t]
            H[index[xp], col] += v
    return H


def test_compiled_tables_reproduce_oracle_matrix(nqs):
    h, eri = make_integrals(6, 12, 1)
    H = nqs.ham_compile(h, eri, 2, 2)
    basis = Sector(6, 2, 2).enumerate()
    M = table_matrix(H.tables(), basis)
    ref = sector_matrix(h, eri, basis, route="literal")
    assert np.max(np.abs(M - ref)) < 1e-13


def test_compiled_tables_other_sector_and_core(nqs):
    h, eri = make_integrals(5, 7, 11)
    H = nqs.ham_compile(h, eri, 3, 1, e_core=0.75)
    basis = Sector(5, 3, 1).enumerate()
    M = table_matrix(H.tables(), basis)
    ref = sector_matrix(h, eri, basis, e_core=0.75)
    assert np.max(np.abs(M - ref)) < 1e-13


@pytest.mark.parametrize("n,na,nb,G", [(6, 2, 2, 286), (10, 5, 5, 2536), (15, 7, 7, 13966)])
def test_group_counts_and_connected_rows(nqs, n, na, nb, G):
    """Flip groups: diagonal + same-spin pairs + same-spin quadruples + alpha-beta
    pair products; and one row per size against the oracle's Slater-Condon row."""
    from math import comb
    h, eri = make_integrals(n, 2 * n, n)
    H = nqs.ham_compile(h, eri, na, nb)
    assert H.info()[0] == G == 1 + 2 * comb(n, 2) + 2 * comb(n, 4) + comb(n, 2) ** 2
    flip, off, z, c = H.tables()
    assert flip[0] == 0 and np.all(np.diff(flip.astype(np.float64)) > 0)
    from oracle.sector import hf_config
    x = hf_config(n, na, nb)
    xs, vals = slater_condon_row(h, eri, x)
    ref = dict(zip(xs, vals))
    got = {}
    for g in range(len(flip)):
        xp = x ^ int(flip[g])
        if bin(xp & 0x5555555555555555).count("1") != na or bin(xp & 0xAAAAAAAAAAAAAAAA).count("1") != nb:
            continue
        s = 0.0
        for t in range(off[g], off[g + 1]):
            s += -c[t] if bin(x & int(z[t])).count("1") & 1 else c[t]
        got[xp] = s
    assert set(got) == set(ref)
    assert max(abs(got[k] - ref[k]) for k in ref) < 1e-12


def test_identity_coefficient_is_normalised_trace(nqs):
    """The coefficient of the identity string is Tr H / 2^N over the Fock space."""
    n = 4
    h, eri = make_integrals(n, 6, 12)
    H = nqs.ham_compile(h, eri, 2, 2, e_core=0.3)
    flip, off, z, c = H.tables()
    ident = [c[t] for t in range(off[0], off[1]) if z[t] == 0]
    trace = sum(slater_condon_row(h, eri, x, 0.3)[1][0] for x in range(1 << (2 * n)))
    assert abs(ident[0] - trace / (1 << (2 * n))) < 1e-13


def test_error_codes(nqs):
    h, eri = make_integrals(4, 4, 1)
    with pytest.raises(nqs.NQSError) as e:
        nqs.ham_compile(np.zeros((33, 33)), np.zeros((33,) * 4), 1, 1)
    assert e.value.status == -3
    bad = h.copy()
    bad[0, 1] += 1e-3
    with pytest.raises(nqs.NQSError) as e:
        nqs.ham_compile(bad, eri, 1, 1)
    assert e.value.status == -1
    with pytest.raises(nqs.NQSError) as e:
        nqs.ham_compile(h, eri, 5, 1)
    assert e.value.status == -1
    asym = eri.copy()
    asym[0, 1, 2, 3] += 1e-3
    with pytest.raises(nqs.NQSError) as e:
        nqs.ham_compile(h, asym, 2, 2)
    assert e.value.status == -1
    with pytest.raises(nqs.NQSError) as e:
        nqs.Model(nqs.MODEL_MLP, [6, 2, 2, 64], np.zeros(10), "fp64")
    assert e.value.status == -1 and "32304" in str(e.value)
    with pytest.raises(nqs.NQSError) as e:
        nqs.Model(nqs.MODEL_MLP, [6, 2, 2, 64], np.zeros(32304), "bf16")
    assert e.value.status == -3
    with pytest.raises(nqs.NQSError) as e:
        nqs.Model(nqs.MODEL_TRANSFORMER, [6, 2, 2, 30, 1, 4, 120, 8], np.zeros(10), "fp32")
    assert e.value.status == -3
    with pytest.raises(nqs.NQSError) as e:
        nqs.Model(nqs.MODEL_MLP, [40, 2, 2, 64], np.zeros(10), "fp64")
    assert e.value.status == -3


@pytest.mark.parametrize("n,irreps,count", [
    (6, None, 0),                                   # generic integrals: no point group
    (6, [0, 0, 1, 2, 1, 3], 2),                     # Z2 x Z2 (C2v-like)
    (8, [0, 1, 2, 4, 3, 5, 6, 7], 3),               # Z2^3 (D2h-like)
])
def test_z2_symmetries_span_the_oracle_null_space(nqs, n, irreps, count):
    """ham_z2_symmetries (host C++, from the compiled flip groups) together with
    the alpha / beta parity masks spans the oracle's null space of the terms'
    flip masks (built from the integrals)."""
    from oracle.hamiltonian import gf2_span_key, z2_symmetries
    h, eri = make_integrals(n, 2 * n, 7, irreps=irreps)
    H = nqs.ham_compile(h, eri, n // 2, n // 2)
    got = H.z2_symmetries()
    alpha = sum(1 << (2 * p) for p in range(n))
    assert len(got) == count
    assert gf2_span_key(got + [alpha, alpha << 1]) == gf2_span_key(z2_symmetries(h, eri))
