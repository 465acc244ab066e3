"""Oracle gamma matrices (test infrastructure only).

Chiral (Weyl) basis of Euclidean Hermitian gamma matrices:
gamma_k = [[0, -i sigma_k], [i sigma_k, 0]] for k = x, y, z and
gamma_t = [[0, 1], [1, 0]]; gamma_5 = gamma_x gamma_y gamma_z gamma_t, which
is diag(1, 1, -1, -1) in this basis.  The paper fixes no basis; the spectrum of
the operator does not depend on it.
"""
from __future__ import annotations

import numpy as np

SIGMA = np.array(
    [[[0, 1], [1, 0]], [[0, -1j], [1j, 0]], [[1, 0], [0, -1]]], dtype=np.complex128
)


def gammas() -> np.ndarray:
    """gamma_mu for mu = x, y, z, t, shape (4, 4, 4)."""
    g = np.zeros((4, 4, 4), dtype=np.complex128)
    z2 = np.zeros((2, 2))
    for k in range(3):
        g[k] = np.block([[z2, -1j * SIGMA[k]], [1j * SIGMA[k], z2]])
    g[3] = np.block([[z2, np.eye(2)], [np.eye(2), z2]])
    return g


def gamma5() -> np.ndarray:
    g = gammas()
    return g[0] @ g[1] @ g[2] @ g[3]


def chiral_projectors():
    """P_plus = (1 + gamma_5)/2 and P_minus = (1 - gamma_5)/2."""
    g5 = gamma5()
    one = np.eye(4)
    return 0.5 * (one + g5), 0.5 * (one - g5)
