"""Pins of the oracle's local energy, energy estimator and gradient."""
import numpy as np
import pytest
import torch

from oracle.ed import ground_state
from oracle.hamiltonian import sector_matrix
from oracle.model import MLPModel, TableModel, TransformerModel
from oracle.sector import Sector
from oracle.vmc import (energy_stats, exact_energy, exact_probabilities,
                        gradient, local_energies)
from synth import (make_integrals, make_mlp_params, make_transformer_params,
                   mlp_param_spec, transformer_param_spec)


@pytest.fixture(scope="module")
def tiny():
    h, eri = make_integrals(6, 12, 1)
    sec = Sector(6, 2, 2)
    basis = sec.enumerate()
    H = sector_matrix(h, eri, basis, route="literal")
    return h, eri, sec, basis, H


def test_eloc_identity_full_matrix(tiny):
    """E_loc(x) = (H psi)(x) / psi(x), H from literal operator application."""
    h, eri, sec, basis, H = tiny
    m = MLPModel(make_mlp_params(6, 64, seed=4, std=0.5), sec)
    with torch.no_grad():
        la, ph = m.amplitudes(basis)
    psi = np.exp(la.numpy() + 1j * ph.numpy())
    expect = (H.T @ psi) / psi
    got = local_energies(m, h, eri, basis)
    assert np.max(np.abs(got - expect) / np.abs(expect)) < 1e-12


def test_zero_variance_at_ground_state(tiny):
    """A table ansatz equal to the exact ground vector has E_loc = E_0 everywhere."""
    h, eri, sec, basis, H = tiny
    e0, v0 = ground_state(H)
    # E_loc is defined where psi(x) != 0; the ground vector has symmetry zeros
    keep = [x for x, v in zip(basis, v0) if abs(v) > 1e-6]
    assert len(keep) > 100
    got = local_energies(TableModel(basis, v0), h, eri, keep)
    assert np.max(np.abs(got - e0)) < 1e-10


def test_variational_bound_and_estimator(tiny):
    h, eri, sec, basis, H = tiny
    e0, _ = ground_state(H)
    m = MLPModel(make_mlp_params(6, 64, seed=5, std=0.5), sec)
    p = exact_probabilities(m, basis)
    eloc = local_energies(m, h, eri, basis)
    W, E, var = energy_stats(eloc, p)
    assert abs(W - 1.0) < 1e-12
    assert abs(E - exact_energy(m, H, basis)) < 1e-12
    assert E.real >= e0 - 1e-12 and var > 0
    # integer counts: the estimator is the counts-weighted mean
    counts = np.arange(1, len(basis) + 1)
    W, E2, _ = energy_stats(eloc, counts)
    assert W == counts.sum()
    ref = np.dot(counts, eloc) / counts.sum()
    assert abs(E2 - ref) < 1e-12 * abs(ref)


def _fd_check(model_factory, spec, h, eri, basis, H, idx, eps=1e-6):
    """Gradient formula with exact weights vs central finite differences of the
    exact energy E(theta) = <psi|H|psi> over the enumerated sector."""
    m = model_factory(None)
    p = exact_probabilities(m, basis)
    eloc = local_energies(m, h, eri, basis)
    m = model_factory(True)
    g = gradient(m, basis, p, eloc, spec)
    flat0 = np.concatenate([m.t[k].detach().numpy().reshape(-1) for k, _ in spec])
    for i in idx:
        vals = []
        for sgn in (1, -1):
            f = flat0.copy()
            f[i] += sgn * eps
            mm = model_factory(None, f)
            vals.append(exact_energy(mm, H, basis).real)
        fd = (vals[0] - vals[1]) / (2 * eps)
        assert abs(fd - g[i]) <= 1e-6 * max(1e-3, abs(fd)) + 1e-9, (i, fd, g[i])


def test_gradient_matches_finite_differences_mlp(tiny):
    h, eri, sec, basis, H = tiny
    spec = mlp_param_spec(6, 64)
    base = make_mlp_params(6, 64, seed=6, std=0.5, bias_std=0.1)

    def factory(rg, flat=None):
        params = base
        if flat is not None:
            from synth import unflatten_params
            params = unflatten_params(flat, spec)
        return MLPModel(params, sec, requires_grad=bool(rg))

    rng = np.random.default_rng(0)
    P = sum(int(np.prod(s)) for _, s in spec)
    # first subnetwork (bias-only input) plus random parameters elsewhere
    idx = np.concatenate([[0, 1, 64, 4200], rng.choice(P, 12, replace=False)])
    _fd_check(factory, spec, h, eri, basis, H, idx)


def test_gradient_matches_finite_differences_transformer(tiny):
    h, eri, sec, basis, H = tiny
    spec = transformer_param_spec(6, 16, 1, 64, 32)
    base = make_transformer_params(6, 2, 2, 16, 1, phase_hidden=32, seed=7, std=0.3, bias_std=0.1)

    def factory(rg, flat=None):
        params = base
        if flat is not None:
            from synth import unflatten_params
            params = unflatten_params(flat, spec)
        return TransformerModel(params, sec, 2, requires_grad=bool(rg))

    rng = np.random.default_rng(1)
    P = sum(int(np.prod(s)) for _, s in spec)
    _fd_check(factory, spec, h, eri, basis, H, rng.choice(P, 12, replace=False))
