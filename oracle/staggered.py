"""Staggered operator D_S (oracle; test infrastructure only).

Sec. 3, the D_S equation:

    D_S(x,y) = sum_mu eta_mu(x) (1/2) [ V_mu(x) delta_{x+mu,y}
                                       - V_mu(x-mu)^dag delta_{x-mu,y} ]

plus a mass term m delta_{x,y} (the paper's operator has none; m = 0
reproduces it).  Fields: V [Nt][Nz][Ny][Nx][4][Nc][Nc], psi
[Nt][Nz][Ny][Nx][Nc][Nv], all complex128.
"""
from __future__ import annotations

import numpy as np

from .lattice import dims_of, eta, shift


def _transport(u: np.ndarray, psi: np.ndarray) -> np.ndarray:
    """(u psi)(x) = u(x) psi(x) on the colour index; u [...][Nc][Nc], psi [...][Nc][Nv]."""
    return u @ psi


def hopping(V: np.ndarray, psi: np.ndarray) -> np.ndarray:
    """The sum over mu of the D_S equation applied to psi (no mass term)."""
    et = eta(dims_of(psi))
    out = np.zeros_like(psi)
    for mu in range(4):
        forward = _transport(V[..., mu, :, :], shift(psi, mu, +1))
        v_back = shift(V[..., mu, :, :], mu, -1)                       # V_mu(x - mu)
        backward = _transport(np.conj(np.swapaxes(v_back, -1, -2)), shift(psi, mu, -1))
        out += 0.5 * et[mu][..., None, None] * (forward - backward)
    return out


def apply(V: np.ndarray, psi: np.ndarray, mass: float = 0.0, adjoint: bool = False) -> np.ndarray:
    """(D_S psi)(x), or (D_S^dag psi)(x) if ``adjoint``.

    The hopping part is anti-Hermitian, so the adjoint negates it and keeps the
    (real) mass term.
    """
    hop = hopping(V, psi)
    return mass * psi + (-hop if adjoint else hop)
