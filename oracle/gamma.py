"""Euclidean Dirac matrices in the chiral basis (oracle; test infrastructure only).

The paper does not fix a gamma basis.  This one is Hermitian, satisfies
{gamma_mu, gamma_nu} = 2 delta_{mu nu}, and has gamma_5 = gamma_1 gamma_2
gamma_3 gamma_4 = diag(1, 1, -1, -1):

    gamma_k = [[0, -i sigma_k], [i sigma_k, 0]]   (k = 1, 2, 3)
    gamma_4 = [[0, 1], [1, 0]]

Index 0..3 below is the paper's mu = 1..4.
"""
from __future__ import annotations

import numpy as np

_SIGMA = (
    np.array([[0, 1], [1, 0]], dtype=complex),
    np.array([[0, -1j], [1j, 0]], dtype=complex),
    np.array([[1, 0], [0, -1]], dtype=complex),
)
_Z2 = np.zeros((2, 2), dtype=complex)
_I2 = np.eye(2, dtype=complex)

GAMMA = np.stack(
    [np.block([[_Z2, -1j * s], [1j * s, _Z2]]) for s in _SIGMA] + [np.block([[_Z2, _I2], [_I2, _Z2]])]
)
GAMMA5 = GAMMA[0] @ GAMMA[1] @ GAMMA[2] @ GAMMA[3]
IDENTITY = np.eye(4, dtype=complex)


def spin_mul(g: np.ndarray, psi: np.ndarray) -> np.ndarray:
    """Apply a 4x4 spin matrix to the spin axis of a [..site..][4][Nc][Nv] field."""
    return np.einsum("st,...tcv->...scv", g, psi)
