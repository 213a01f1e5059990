"""Gauge compression of the links V (oracle; test infrastructure only).

Sec. 4 names reducing the stored colour columns of V (N_c -> N_c - 1) as a
next tuning step, and Sec. 5 notes that it cannot be used for 36 of the 40
Brillouin links W, which are not special unitary.  For an SU(3) matrix u the
third row is fixed by the first two: unitarity makes it orthogonal to both,
and det u = 1 fixes its phase, so

    u_2j = conj(u_0k u_1l - u_0l u_1k),   (j, k, l) a cyclic permutation of (0, 1, 2).

Reading taken here (the paper gives no layout): the stored part of each link
is its first two rows, ``[..site..][4][2][3]`` (12 reals instead of 18), and
the operators on compressed links are the operators on the reconstructed
links.  For a unitary u with det u = e^{i a} the reconstruction returns the
third row times e^{-i a}; for non-unitary matrices it is not u.
"""
from __future__ import annotations

import numpy as np

from . import staggered, wilson


def compress(V: np.ndarray) -> np.ndarray:
    """First two rows of every link: [..][3][3] -> [..][2][3]."""
    return np.ascontiguousarray(V[..., :2, :])


def reconstruct(Vc: np.ndarray) -> np.ndarray:
    """Full links from their first two rows (the SU(3) completion)."""
    a, b = Vc[..., 0, :], Vc[..., 1, :]
    third = np.empty_like(a)
    for j in range(3):
        k, l = (j + 1) % 3, (j + 2) % 3
        third[..., j] = np.conj(a[..., k] * b[..., l] - a[..., l] * b[..., k])
    return np.concatenate([Vc, third[..., None, :]], axis=-2)


def apply(op: str, Vc: np.ndarray, psi: np.ndarray, mass: float = 0.0, adjoint: bool = False) -> np.ndarray:
    """D_S or D_W on compressed links."""
    V = reconstruct(Vc)
    if op == "staggered":
        return staggered.apply(V, psi, mass, adjoint)
    if op == "wilson":
        return wilson.apply(V, psi, mass, adjoint)
    raise ValueError(f"gauge compression is defined for staggered and wilson links, not {op!r}")
