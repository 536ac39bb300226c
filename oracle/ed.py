"""Exact diagonalisation inside the symmetry sector (the FCI reference energy)."""
import numpy as np
import scipy.sparse.linalg as sla


def ground_state(H):
    """Lowest eigenpair of a dense symmetric sector matrix."""
    w, v = np.linalg.eigh(H)
    return w[0], v[:, 0]


def ground_energy_sparse(H):
    return sla.eigsh(H, k=1, which="SA")[0][0]
