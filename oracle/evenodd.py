"""Even-odd (Schur complement) form of D_W (oracle; test infrastructure only).

The paper lists eo-decomposition among the next tuning steps for D_W (Sec. 4,
end of the Wilson performance discussion) without spelling it out; this is the
standard construction, written out from its definition.

* parity(x) = (x_1 + x_2 + x_3 + x_4) mod 2 (0-based coordinates); with all
  extents even the periodic lattice splits into two checkerboards and every
  hop of D_W connects opposite parities.
* D_W = A + H with A = (4 + m0) (c_SW = 0: a multiple of the identity) and H
  the hopping part  -1/2 sum_mu [(1 - gamma_mu) V_mu(x) psi(x+mu)
  + (1 + gamma_mu) V_mu(x-mu)^dag psi(x-mu)].  On (even, odd) blocks
  D_W = [[A, H_eo], [H_oe, A]].
* Schur complement on the even sites:  M = A - H_eo A^-1 H_oe, and
  D_W x = b  <=>  M x_e = b_e - H_eo A^-1 b_o,  x_o = A^-1 (b_o - H_oe x_e).
  M^dag = A - (H^dag)_eo A^-1 (H^dag)_oe with H^dag = gamma_5 H gamma_5.

Packed (checkerboard) layout of one parity p: [Nt][Nz][Ny][Nx/2][...]; in
row (y, z, t) packed index i holds x = 2 i + ((p + y + z + t) mod 2).
"""
from __future__ import annotations

import numpy as np

from . import solver, wilson
from .lattice import coordinates


def parity(dims) -> np.ndarray:
    """(x + y + z + t) mod 2 with shape (Nt, Nz, Ny, Nx)."""
    return coordinates(dims).sum(axis=0) % 2


def _check(dims):
    if any(n % 2 for n in dims):
        raise ValueError(f"even-odd splitting needs even extents, got {dims}")


def pack(field: np.ndarray, p: int) -> np.ndarray:
    """Sites of parity p of a [Nt][Nz][Ny][Nx][...] field, packed along x."""
    nt, nz, ny, nx = field.shape[:4]
    _check((nx, ny, nz, nt))
    out = np.empty((nt, nz, ny, nx // 2) + field.shape[4:], dtype=field.dtype)
    for t in range(nt):
        for z in range(nz):
            for y in range(ny):
                r = (p + y + z + t) % 2
                out[t, z, y] = field[t, z, y, r::2]
    return out


def unpack(even: np.ndarray, odd: np.ndarray) -> np.ndarray:
    nt, nz, ny, nh = even.shape[:4]
    out = np.empty((nt, nz, ny, 2 * nh) + even.shape[4:], dtype=np.result_type(even, odd))
    for t in range(nt):
        for z in range(nz):
            for y in range(ny):
                r = (y + z + t) % 2
                out[t, z, y, r::2] = even[t, z, y]
                out[t, z, y, (1 - r)::2] = odd[t, z, y]
    return out


def hop(V: np.ndarray, psi: np.ndarray, adjoint: bool = False) -> np.ndarray:
    """H psi = D_W psi - (4 + m0) psi: the hop form of D_W with 4 + m0 = 0."""
    return wilson.apply_hop(V, psi, -4.0, adjoint)


def hop_eo(V: np.ndarray, psi_in: np.ndarray, p_out: int, adjoint: bool = False) -> np.ndarray:
    """H restricted to output parity p_out, input parity 1 - p_out (packed fields)."""
    zero = np.zeros_like(psi_in)
    full = unpack(psi_in, zero) if p_out == 1 else unpack(zero, psi_in)
    return pack(hop(V, full, adjoint), p_out)


def schur(V: np.ndarray, xe: np.ndarray, m0: float, adjoint: bool = False) -> np.ndarray:
    """M x_e = A x_e - H_eo (H_oe x_e) / A on packed even fields (M^dag if adjoint)."""
    a = 4.0 + m0
    return a * xe - hop_eo(V, hop_eo(V, xe, 1, adjoint), 0, adjoint) / a


def solve(V: np.ndarray, b: np.ndarray, m0: float, tol: float = 1e-12, maxiter: int = 10000):
    """x = D_W^-1 b through CGNR on the Schur complement; returns (x, iterations)."""
    a = 4.0 + m0
    be, bo = pack(b, 0), pack(b, 1)
    rhs = be - hop_eo(V, bo, 0) / a
    xe, iters, _ = solver.cgnr(lambda v: schur(V, v, m0), lambda v: schur(V, v, m0, True), rhs, tol, maxiter)
    xo = (bo - hop_eo(V, xe, 1)) / a
    return unpack(xe, xo), iters
