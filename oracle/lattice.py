"""Lattice geometry (oracle; test infrastructure only).

Coordinates are 0-based, ``x_mu in [0, N_mu)``; direction ``mu = 0..3`` is the
paper's mu = 1..4, i.e. (x, y, z, t).  Fields are numpy arrays whose four
leading axes are ``[Nt][Nz][Ny][Nx]``, the C-order image of the paper's
Fortran ``(..., Nx, Ny, Nz, Nt)`` with the space-time index slowest (Sec. 2).
Boundaries are periodic in all four directions.
"""
from __future__ import annotations

import numpy as np

# direction mu -> numpy axis of a [Nt][Nz][Ny][Nx] field
MU_AXIS = (3, 2, 1, 0)


def dims_of(field: np.ndarray) -> tuple:
    """(Nx, Ny, Nz, Nt) of a field with leading axes [Nt][Nz][Ny][Nx]."""
    nt, nz, ny, nx = field.shape[:4]
    return (nx, ny, nz, nt)


def shift(field: np.ndarray, mu: int, step: int) -> np.ndarray:
    """Return g with g(x) = field(x + step * mu_hat), periodic."""
    return np.roll(field, -step, axis=MU_AXIS[mu])


def shift_by(field: np.ndarray, d) -> np.ndarray:
    """Return g with g(x) = field(x + d) for an integer displacement d."""
    out = field
    for mu, s in enumerate(d):
        if s:
            out = np.roll(out, -int(s), axis=MU_AXIS[mu])
    return out


def coordinates(dims) -> np.ndarray:
    """Array c of shape (4, Nt, Nz, Ny, Nx) with c[mu] = x_mu."""
    nx, ny, nz, nt = dims
    t, z, y, x = np.meshgrid(np.arange(nt), np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    return np.stack([x, y, z, t])


def eta(dims) -> np.ndarray:
    """Staggered phases of Sec. 3: eta_1 = 1, eta_2 = (-1)^{x_1},
    eta_3 = (-1)^{x_1+x_2}, eta_4 = (-1)^{x_1+x_2+x_3}, with 0-based x.

    Returns shape (4, Nt, Nz, Ny, Nx), entries +-1.
    """
    c = coordinates(dims)
    out = np.empty(c.shape, dtype=np.float64)
    for mu in range(4):
        s = c[:mu].sum(axis=0) if mu else np.zeros(c.shape[1:], dtype=np.int64)
        out[mu] = np.where(s % 2 == 0, 1.0, -1.0)
    return out


def site_index(coord, dims) -> int:
    """Lexicographic site index s = x + Nx (y + Ny (z + Nz t))."""
    nx, ny, nz, _ = dims
    x, y, z, t = coord
    return int(x + nx * (y + ny * (z + nz * t)))


def site_coord(s: int, dims) -> tuple:
    nx, ny, nz, _ = dims
    x = s % nx
    s //= nx
    y = s % ny
    s //= ny
    z = s % nz
    return (x, y, z, s // nz)
