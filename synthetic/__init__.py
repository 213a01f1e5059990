"""Seeded synthetic inputs: gauge links and right-hand-side blocks.

This module is the only code shared by the FP64 CPU oracle and the GPU path.
It draws random numbers and nothing else: it holds no part of any Dirac
operator, link product or solver.

Distributions (all from ``numpy.random.Generator(PCG64(seed))``):

* ``haar_su3``: Haar-random SU(3).  A 3x3 matrix of iid CN(0,1) entries is
  QR-factorised, the columns of Q are re-phased by ``R_ii/|R_ii|`` (which makes
  Q Haar-distributed on U(3)), and Q is divided by the principal cube root of
  its determinant, giving det = 1.
* ``smooth_su3``: ``exp(i * eps * H)`` with ``H = sum_a h_a lambda_a / 2``,
  ``h_a ~ N(0,1)`` iid and ``lambda_a`` the eight Gell-Mann matrices;
  exponentiated through the eigendecomposition of the Hermitian ``H``.
  ``eps = 0.3`` gives a smooth, smeared-looking field.
* ``gaussian``: iid complex Gaussian CN(0,1), i.e. real and imaginary parts
  iid N(0, 1/2).

Field layouts (C order, site index slowest, ``dims = (Nx, Ny, Nz, Nt)``):

* links ``[Nt][Nz][Ny][Nx][4][Nc][Nc]``
* Wilson-type spinor block ``[Nt][Nz][Ny][Nx][4][Nc][Nv]``
* staggered spinor block ``[Nt][Nz][Ny][Nx][Nc][Nv]``
"""
from __future__ import annotations

import numpy as np

__all__ = [
    "rng", "haar_su3", "smooth_su3", "gaussian", "gauge_links",
    "wilson_spinor", "staggered_spinor", "lattice_shape", "round_to",
]


def rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def lattice_shape(dims) -> tuple:
    nx, ny, nz, nt = (int(d) for d in dims)
    return (nt, nz, ny, nx)


def gaussian(shape, seed: int) -> np.ndarray:
    g = rng(seed)
    re = g.standard_normal(shape)
    im = g.standard_normal(shape)
    return (re + 1j * im) * np.sqrt(0.5)


def haar_su3(count: int, seed: int, nc: int = 3) -> np.ndarray:
    g = rng(seed)
    z = (g.standard_normal((count, nc, nc)) + 1j * g.standard_normal((count, nc, nc))) * np.sqrt(0.5)
    q, r = np.linalg.qr(z)
    d = np.diagonal(r, axis1=-2, axis2=-1)
    q = q * (d / np.abs(d))[:, None, :]
    det = np.linalg.det(q)
    q = q / (det ** (1.0 / nc))[:, None, None]
    return q


def _gell_mann() -> np.ndarray:
    lam = np.zeros((8, 3, 3), dtype=complex)
    lam[0][0, 1] = lam[0][1, 0] = 1
    lam[1][0, 1], lam[1][1, 0] = -1j, 1j
    lam[2][0, 0], lam[2][1, 1] = 1, -1
    lam[3][0, 2] = lam[3][2, 0] = 1
    lam[4][0, 2], lam[4][2, 0] = -1j, 1j
    lam[5][1, 2] = lam[5][2, 1] = 1
    lam[6][1, 2], lam[6][2, 1] = -1j, 1j
    lam[7][0, 0] = lam[7][1, 1] = 1 / np.sqrt(3)
    lam[7][2, 2] = -2 / np.sqrt(3)
    return lam


def smooth_su3(count: int, seed: int, eps: float = 0.3) -> np.ndarray:
    g = rng(seed)
    h = g.standard_normal((count, 8))
    herm = np.einsum("na,aij->nij", h, _gell_mann() / 2)
    w, v = np.linalg.eigh(herm)
    return np.einsum("nij,nj,nkj->nik", v, np.exp(1j * eps * w), v.conj())


def gauge_links(dims, kind: str, seed: int, nc: int = 3) -> np.ndarray:
    """Links ``[Nt][Nz][Ny][Nx][4][Nc][Nc]`` complex128.

    kind: "haar", "smooth" (eps=0.3), "unit" (all identity).
    """
    shape = lattice_shape(dims) + (4,)
    n = int(np.prod(shape))
    if kind == "haar":
        u = haar_su3(n, seed, nc)
    elif kind == "smooth":
        if nc != 3:
            raise ValueError("smooth links are defined for Nc=3 only")
        u = smooth_su3(n, seed)
    elif kind == "unit":
        u = np.broadcast_to(np.eye(nc, dtype=complex), (n, nc, nc)).copy()
    else:
        raise ValueError(f"unknown link kind {kind!r}")
    return u.reshape(shape + (nc, nc))


def wilson_spinor(dims, nv: int, seed: int, nc: int = 3) -> np.ndarray:
    return gaussian(lattice_shape(dims) + (4, nc, nv), seed)


def staggered_spinor(dims, nv: int, seed: int, nc: int = 3) -> np.ndarray:
    return gaussian(lattice_shape(dims) + (nc, nv), seed)


def round_to(a: np.ndarray, precision: str) -> np.ndarray:
    """Round a complex128 array to the storage precision and back to complex128.

    ``"c64"`` rounds each real component to IEEE binary32 (round to nearest
    even), ``"c128"`` leaves it unchanged.  The result is what a device buffer
    of that precision holds, promoted exactly.
    """
    if precision == "c64":
        return a.astype(np.complex64).astype(np.complex128)
    if precision == "c128":
        return np.asarray(a, dtype=np.complex128)
    raise ValueError(f"unknown precision {precision!r}")
