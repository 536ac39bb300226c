"""Local energy, energy estimator and VMC gradient (paper: "Variational Monte
Carlo": the local-energy, energy-estimator and gradient equations).

* E_loc(x) = sum_{x'} H_{x x'} psi(x') / psi(x), summed over x itself and
  every spin-conserving single and double of x (the structural connected set;
  no value threshold).  H is real symmetric, so H_{x x'} = <x'|H|x>.
* E = sum_l n_l E_loc(x_l) / W with W = sum_l n_l (W = N_s under
  Mask-Unphysical; dividing by W is the reading used when samples are lost).
* grad E = 2 Re{ E[E_loc grad ln psi*] - E[E_loc] E[grad ln psi*] }.  With
  ln psi* = log|psi| - i phi this is
  (2/W) sum_l n_l [Re(E_loc,l - E) grad log|psi_l| + Im(E_loc,l - E) grad phi_l],
  with E_loc and E held constant.  Gradients come from float64 autograd.
"""
import numpy as np
import torch

from .hamiltonian import slater_condon_row


def local_energy(model, h, eri, x, e_core=0.0):
    """E_loc(x) as a Python complex, plus the (x', H_x'x) list it summed."""
    xs, vals = slater_condon_row(h, eri, int(x), e_core)
    with torch.no_grad():
        la, ph = model.amplitudes(xs)
    la, ph = la.numpy(), ph.numpy()
    ratio = np.exp((la - la[0]) + 1j * (ph - ph[0]))
    return complex(np.sum(np.asarray(vals) * ratio)), xs, vals


def local_energies(model, h, eri, xs, e_core=0.0):
    return np.array([local_energy(model, h, eri, x, e_core)[0] for x in xs])


def energy_stats(eloc, counts):
    """(W, E, variance) with E complex and variance = sum n |E_loc - E|^2 / W."""
    n = np.asarray(counts, dtype=np.float64)
    W = n.sum()
    E = np.sum(n * eloc) / W
    var = np.sum(n * np.abs(eloc - E) ** 2) / W
    return W, E, var


def gradient(model, xs, counts, eloc, spec):
    """VMC gradient in the canonical flat parameter order ``spec``."""
    n = np.asarray(counts, dtype=np.float64)
    W, E, _ = energy_stats(eloc, n)
    cr = torch.tensor(2.0 * n / W * np.real(eloc - E))
    ci = torch.tensor(2.0 * n / W * np.imag(eloc - E))
    for v in model.t.values():
        v.grad = None
    la, ph = model.amplitudes(xs)
    (torch.sum(cr * la) + torch.sum(ci * ph)).backward()
    return model.flat_grad(spec)


def surrogate_weights(counts, eloc):
    """Upstream weights (d L/d log|psi_l|, d L/d phi_l) of the gradient."""
    n = np.asarray(counts, dtype=np.float64)
    W, E, _ = energy_stats(eloc, n)
    return 2.0 * n / W * np.real(eloc - E), 2.0 * n / W * np.imag(eloc - E)


def exact_probabilities(model, basis):
    """|psi(x)|^2 over an enumerated basis (the masked model's Born weights)."""
    with torch.no_grad():
        la, _ = model.amplitudes(basis)
    return np.exp(2.0 * la.numpy())


def exact_energy(model, H, basis):
    """<psi|H|psi> / <psi|psi> over the enumerated sector, psi from the model."""
    with torch.no_grad():
        la, ph = model.amplitudes(basis)
    psi = np.exp(la.numpy() + 1j * ph.numpy())
    return np.vdot(psi, H @ psi) / np.vdot(psi, psi)
