"""Krylov solvers in FP64 (oracle; test infrastructure only).

The paper has no solver.  These are the textbook algorithms the GPU solver is
checked against:

* ``cg``: conjugate gradients (Hestenes-Stiefel) for a Hermitian positive
  definite operator, one independent iteration per right-hand side (the last
  axis of every field), stopping each column when ||r||/||b|| <= tol;
* ``cgnr``: CG on the normal equations D^dag D x = D^dag b;
* ``relative_residual``: ||b - D x||_2 / ||b||_2 per right-hand side, the
  certificate every solve is checked by (several x meet a tolerance, so
  residuals, not solutions, are compared);
* ``wilson_residual_slab``: the squared norms that certificate needs for D_W
  (Sec. 4, eq. def_wils), restricted to the time slices t0 <= t < t1, so a
  lattice whose FP64 oracle application does not fit at once can be
  certified slab by slab (the stencil reaches one slice in t).
"""
from __future__ import annotations

import numpy as np

from . import wilson


def _dot(a: np.ndarray, b: np.ndarray) -> np.ndarray:
    """Per right-hand-side inner product <a, b> over all axes but the last."""
    nv = a.shape[-1]
    return np.einsum("iv,iv->v", np.conj(a.reshape(-1, nv)), b.reshape(-1, nv))


def norm2(a: np.ndarray) -> np.ndarray:
    return np.real(_dot(a, a))


def relative_residual(apply_d, b: np.ndarray, x: np.ndarray) -> np.ndarray:
    r = b - apply_d(x)
    return np.sqrt(norm2(r) / norm2(b))


def cg(apply_a, b: np.ndarray, tol: float = 1e-12, maxiter: int = 10000, x0=None):
    """Returns (x, iterations per column, final ||r||/||b|| per column)."""
    x = np.zeros_like(b) if x0 is None else x0.copy()
    r = b - apply_a(x)
    p = r.copy()
    rr = norm2(r)
    bb = norm2(b)
    active = np.sqrt(rr / bb) > tol
    iters = np.zeros(b.shape[-1], dtype=int)
    for _ in range(maxiter):
        if not active.any():
            break
        q = apply_a(p)
        pq = np.real(_dot(p, q))
        alpha = np.where(active, rr / np.where(pq != 0, pq, 1), 0.0)
        x = x + alpha * p
        r = r - alpha * q
        rr_new = norm2(r)
        beta = np.where(active, rr_new / np.where(rr != 0, rr, 1), 0.0)
        p = np.where(active, r + beta * p, p)
        rr = np.where(active, rr_new, rr)
        iters += active
        active = active & (np.sqrt(rr / bb) > tol)
    return x, iters, np.sqrt(rr / bb)


def cgnr(apply_d, apply_ddag, b: np.ndarray, tol: float = 1e-12, maxiter: int = 10000, x0=None):
    """CG on D^dag D x = D^dag b; tol applies to the normal-equation residual."""
    return cg(lambda v: apply_ddag(apply_d(v)), apply_ddag(b), tol, maxiter, x0)


def wilson_residual_slab(V: np.ndarray, b: np.ndarray, x: np.ndarray, m0: float, t0: int, t1: int):
    """(||r_v||^2, ||b_v||^2) per right-hand side v over the sites with
    t0 <= t < t1, r = b - D_W x.

    D_W x on those slices needs x and V on the slices t0 - 1 .. t1 only (one hop
    in t; the backward link V_t(x - t) sits on slice t - 1).  The oracle's D_W
    is applied to that periodic window of t1 - t0 + 2 slices and its two outer
    slices, the only ones the window's own wrap reaches, are dropped.  Fields
    are [Nt][Nz][Ny][Nx][...] arrays (memory maps work: only the window is
    read).
    """
    nt = V.shape[0]
    if not 0 <= t0 < t1 <= nt:
        raise ValueError(f"need 0 <= t0 < t1 <= Nt, got {t0}, {t1}, {nt}")
    rows = [(t0 - 1 + k) % nt for k in range(t1 - t0 + 2)]
    dx = wilson.apply_hop(np.asarray(V[rows], dtype=np.complex128), np.asarray(x[rows], dtype=np.complex128),
                          m0)[1:-1]
    bs = np.asarray(b[t0:t1], dtype=np.complex128)
    return norm2(bs - dx), norm2(bs)
