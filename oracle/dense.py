"""Brute-force dense Dirac matrices (oracle; test infrastructure only).

Each matrix is filled entry block by entry block from the delta-function form
of its definition, looping over sites x and computing neighbour coordinates
with explicit modular arithmetic.  Nothing here uses the shift-based code of
the other oracle modules, so agreement between the two is a check on both.

Row/column index: Wilson-type (site * 4 + spin) * Nc + colour; staggered
site * Nc + colour; site = x + Nx (y + Ny (z + Nz t)).  With that order
``D @ psi.reshape(-1, Nv)`` is the operator applied to a [site][4][Nc][Nv]
(or [site][Nc][Nv]) block.
"""
from __future__ import annotations

import itertools
import math

import numpy as np

from .gamma import GAMMA

_RHO = (None, 64 / 432, 16 / 432, 4 / 432, 1 / 432)
_LAMBDA = (-240 / 64, 8 / 64, 4 / 64, 2 / 64, 1 / 64)


def _sites(dims):
    nx, ny, nz, nt = dims
    for t in range(nt):
        for z in range(nz):
            for y in range(ny):
                for x in range(nx):
                    yield (x, y, z, t)


def _index(c, dims) -> int:
    nx, ny, nz, _ = dims
    return c[0] + nx * (c[1] + ny * (c[2] + nz * c[3]))


def _move(c, d, dims):
    return tuple((c[i] + d[i]) % dims[i] for i in range(4))


def _unit(mu, s=1):
    e = [0, 0, 0, 0]
    e[mu] = s
    return tuple(e)


def _link(V, c, mu):
    """V_mu at coordinate c from a [Nt][Nz][Ny][Nx][4][Nc][Nc] array."""
    return V[c[3], c[2], c[1], c[0], mu]


def staggered(V: np.ndarray, mass: float = 0.0) -> np.ndarray:
    nt, nz, ny, nx = V.shape[:4]
    dims = (nx, ny, nz, nt)
    nc = V.shape[-1]
    n = nx * ny * nz * nt * nc
    D = np.zeros((n, n), dtype=np.complex128)
    for c in _sites(dims):
        i = _index(c, dims) * nc
        D[i:i + nc, i:i + nc] += mass * np.eye(nc)
        for mu in range(4):
            eta = (-1) ** sum(c[:mu])
            fwd = _move(c, _unit(mu), dims)
            bwd = _move(c, _unit(mu, -1), dims)
            j = _index(fwd, dims) * nc
            D[i:i + nc, j:j + nc] += 0.5 * eta * _link(V, c, mu)
            j = _index(bwd, dims) * nc
            D[i:i + nc, j:j + nc] -= 0.5 * eta * _link(V, bwd, mu).conj().T
    return D


def _spin_colour_block(D, i, j, spin, colour):
    m = np.kron(spin, colour)
    D[i:i + m.shape[0], j:j + m.shape[1]] += m


def wilson(V: np.ndarray, m0: float = 0.0) -> np.ndarray:
    """D_W(x,y) = sum_mu gamma_mu nabla_mu(x,y) - Laplace(x,y)/2 + m0 delta_{x,y}."""
    nt, nz, ny, nx = V.shape[:4]
    dims = (nx, ny, nz, nt)
    nc = V.shape[-1]
    bs = 4 * nc
    n = nx * ny * nz * nt * bs
    D = np.zeros((n, n), dtype=np.complex128)
    one = np.eye(4)
    for c in _sites(dims):
        i = _index(c, dims) * bs
        # m0 delta - (1/2)(-8 delta)
        _spin_colour_block(D, i, i, (m0 + 4.0) * one, np.eye(nc))
        for mu in range(4):
            fwd = _move(c, _unit(mu), dims)
            bwd = _move(c, _unit(mu, -1), dims)
            u_f = _link(V, c, mu)
            u_b = _link(V, bwd, mu).conj().T
            # gamma_mu nabla_mu: +1/2 V_mu(x) at x+mu, -1/2 V_{-mu}(x) at x-mu
            _spin_colour_block(D, i, _index(fwd, dims) * bs, 0.5 * GAMMA[mu], u_f)
            _spin_colour_block(D, i, _index(bwd, dims) * bs, -0.5 * GAMMA[mu], u_b)
            # -(1/2) Laplace: coefficient 1 for each of the 8 neighbours
            _spin_colour_block(D, i, _index(fwd, dims) * bs, -0.5 * one, u_f)
            _spin_colour_block(D, i, _index(bwd, dims) * bs, -0.5 * one, u_b)
    return D


def _path_average(V, c, d, dims):
    """W_d at coordinate c: mean over all orderings of the hops of d of the
    ordered link product, V_{-mu}(y) = V_mu(y - mu)^dag."""
    steps = [(mu, s) for mu, s in enumerate(d) if s]
    nc = V.shape[-1]
    acc = np.zeros((nc, nc), dtype=np.complex128)
    for order in itertools.permutations(steps):
        prod = np.eye(nc, dtype=np.complex128)
        pos = c
        for mu, s in order:
            if s > 0:
                link = _link(V, pos, mu)
            else:
                link = _link(V, _move(pos, _unit(mu, -1), dims), mu).conj().T
            prod = prod @ link
            pos = _move(pos, _unit(mu, s), dims)
        acc += prod
    return acc / math.factorial(len(steps))


def brillouin(V: np.ndarray, m0: float = 0.0) -> np.ndarray:
    """D_B(x, x+d) = sum_mu gamma_mu rho_k d_mu W_d(x) - (1/2) lambda_k W_d(x),
    D_B(x, x) = m0 - lambda_0/2, with W_d built from V path by path at every site."""
    nt, nz, ny, nx = V.shape[:4]
    dims = (nx, ny, nz, nt)
    nc = V.shape[-1]
    bs = 4 * nc
    n = nx * ny * nz * nt * bs
    D = np.zeros((n, n), dtype=np.complex128)
    for c in _sites(dims):
        i = _index(c, dims) * bs
        _spin_colour_block(D, i, i, (m0 - 0.5 * _LAMBDA[0]) * np.eye(4), np.eye(nc))
        for d in itertools.product((-1, 0, 1), repeat=4):
            k = sum(1 for s in d if s)
            if k == 0:
                continue
            w = _path_average(V, c, d, dims)
            spin = -0.5 * _LAMBDA[k] * np.eye(4)
            for mu in range(4):
                if d[mu]:
                    spin = spin + _RHO[k] * d[mu] * GAMMA[mu]
            _spin_colour_block(D, i, _index(_move(c, d, dims), dims) * bs, spin, w)
    return D
