"""Operators evaluated at a sample of sites (oracle; test infrastructure only).

The operators are local: out(x) needs the links at x (and at the backward
neighbours) and psi on the 3^4 hypercube around x.  These functions compute
out(x) for a list of coordinates only, by explicit neighbour gathers, so a
lattice whose full FP64 application would not fit the host (e.g. D_B on 32^4
at N_v = 12) can still be checked at sampled sites.  They use the hop forms:

* D_S: m psi(x) + sum_mu eta_mu(x)/2 [V_mu(x) psi(x+mu) - V_mu(x-mu)^dag psi(x-mu)]
  (Sec. 3);
* D_W: (4 + m0) psi(x) - 1/2 sum_mu [(1 - gamma_mu) V_mu(x) psi(x+mu)
  + (1 + gamma_mu) V_mu(x-mu)^dag psi(x-mu)] (eq. def_wils, c_SW = 0);
* D_B: (m0 - lambda_0/2) psi(x) + sum_{d != 0} [-lambda_k/2 + rho_k d.gamma]
  W_d(x) psi(x+d) (eqs. def_bril, def_der, def_lap) with every W_d(x) built
  from V by the path average of Tab. 1 at the sampled site itself.

``coords`` is an integer array of shape (n, 4) holding (x, y, z, t).
"""
from __future__ import annotations

import itertools
import math

import numpy as np

from .gamma import GAMMA, IDENTITY

_RHO = (None, 64 / 432, 16 / 432, 4 / 432, 1 / 432)
_LAMBDA = (-240 / 64, 8 / 64, 4 / 64, 2 / 64, 1 / 64)


def sample_sites(dims, count: int, seed: int) -> np.ndarray:
    """``count`` distinct random coordinates plus the 16 corners of the lattice
    (which exercise every periodic wrap)."""
    g = np.random.Generator(np.random.PCG64(seed))
    total = int(np.prod(dims))
    idx = g.choice(total, size=min(count, total), replace=False)
    nx, ny, nz, _ = dims
    c = np.stack([idx % nx, (idx // nx) % ny, (idx // (nx * ny)) % nz, idx // (nx * ny * nz)], axis=1)
    corners = np.array([[a * (dims[0] - 1), b * (dims[1] - 1), cc * (dims[2] - 1), d * (dims[3] - 1)]
                        for a, b, cc, d in itertools.product((0, 1), repeat=4)])
    return np.unique(np.concatenate([c, corners]), axis=0)


def _dims(field) -> tuple:
    nt, nz, ny, nx = field.shape[:4]
    return (nx, ny, nz, nt)


def _at(field: np.ndarray, coords: np.ndarray, d=(0, 0, 0, 0)) -> np.ndarray:
    """field(x + d) for every x in coords."""
    dims = _dims(field)
    c = (coords + np.asarray(d)[None, :]) % np.asarray(dims)[None, :]
    return field[c[:, 3], c[:, 2], c[:, 1], c[:, 0]]


def _unit(mu: int, s: int = 1):
    e = [0, 0, 0, 0]
    e[mu] = s
    return e


def _dag(u):
    return np.conj(np.swapaxes(u, -1, -2))


def staggered_at(V, psi, mass, coords, adjoint=False):
    out = mass * _at(psi, coords)
    sgn = -1.0 if adjoint else 1.0
    for mu in range(4):
        eta = np.where(coords[:, :mu].sum(axis=1) % 2 == 0, 1.0, -1.0)[:, None, None]
        fwd = _at(V, coords)[:, mu] @ _at(psi, coords, _unit(mu))
        bwd = _dag(_at(V, coords, _unit(mu, -1))[:, mu]) @ _at(psi, coords, _unit(mu, -1))
        out = out + sgn * 0.5 * eta * (fwd - bwd)
    return out


def _spin(g, f):
    return np.einsum("st,ntcv->nscv", g, f)


def wilson_at(V, psi, m0, coords, adjoint=False):
    sgn = -1.0 if adjoint else 1.0
    out = (4.0 + m0) * _at(psi, coords)
    for mu in range(4):
        fwd = _at(V, coords)[:, mu][:, None] @ _at(psi, coords, _unit(mu))
        bwd = _dag(_at(V, coords, _unit(mu, -1))[:, mu])[:, None] @ _at(psi, coords, _unit(mu, -1))
        out = out - 0.5 * _spin(IDENTITY - sgn * GAMMA[mu], fwd) - 0.5 * _spin(IDENTITY + sgn * GAMMA[mu], bwd)
    return out


def path_link_at(V, coords, d) -> np.ndarray:
    """W_d(x) for x in coords: mean over the k! hop orderings of the path
    product, V_{-mu}(y) = V_mu(y - mu)^dag (Tab. 1)."""
    steps = [(mu, s) for mu, s in enumerate(d) if s]
    nc = V.shape[-1]
    acc = np.zeros((len(coords), nc, nc), dtype=np.complex128)
    for order in itertools.permutations(steps):
        prod = None
        pos = np.zeros(4, dtype=int)
        for mu, s in order:
            if s > 0:
                link = _at(V, coords, pos)[:, mu]
            else:
                link = _dag(_at(V, coords, pos + np.array(_unit(mu, -1)))[:, mu])
            prod = link if prod is None else prod @ link
            pos = pos + np.array(_unit(mu, s))
        acc += prod
    return acc / math.factorial(len(steps))


def brillouin_at(V, psi, m0, coords, adjoint=False):
    sgn = -1.0 if adjoint else 1.0
    out = (m0 - 0.5 * _LAMBDA[0]) * _at(psi, coords)
    for d in itertools.product((-1, 0, 1), repeat=4):
        k = sum(1 for s in d if s)
        if k == 0:
            continue
        spin = -0.5 * _LAMBDA[k] * IDENTITY + sgn * _RHO[k] * sum(d[mu] * GAMMA[mu] for mu in range(4))
        w = path_link_at(V, coords, d)
        out = out + _spin(spin, w[:, None] @ _at(psi, coords, d))
    return out


def link_grad_at(op: str, chi, psi, coords, mu: int) -> np.ndarray:
    """G_mu(x) for x in coords (see ``oracle.grad`` for the formula)."""
    e = _unit(mu)
    if op == "staggered":
        eta_x = np.where(coords[:, :mu].sum(axis=1) % 2 == 0, 1.0, -1.0)[:, None, None]
        cf = (coords + np.array(e)) % np.asarray(_dims(psi))
        eta_f = np.where(cf[:, :mu].sum(axis=1) % 2 == 0, 1.0, -1.0)[:, None, None]
        t1 = 0.5 * eta_x * (_at(chi, coords) @ _dag(_at(psi, coords, e)))
        t2 = -0.5 * eta_f * (_at(psi, coords) @ _dag(_at(chi, coords, e)))
        return t1 + t2
    if op == "wilson":
        phi_f = _spin(-0.5 * (IDENTITY - GAMMA[mu]), _at(psi, coords, e))
        phi_b = _spin(-0.5 * (IDENTITY + GAMMA[mu]), _at(psi, coords))
        t1 = np.einsum("nsav,nsbv->nab", _at(chi, coords), np.conj(phi_f))
        t2 = np.einsum("nsav,nsbv->nab", phi_b, np.conj(_at(chi, coords, e)))
        return t1 + t2
    raise ValueError(op)


def _stored_directions():
    """The 40 stored displacements in slot order (Tab. 1 caption: slot
    n(d) - 41, n(d) = sum_mu (d_mu + 1) 3^mu, for the d with n(d) > 40)."""
    out = []
    for n in range(41, 81):
        out.append((n % 3 - 1, (n // 3) % 3 - 1, (n // 9) % 3 - 1, n // 27 - 1))
    return out


def _bri_spin(d):
    k = sum(1 for s in d if s)
    return -0.5 * _LAMBDA[k] * IDENTITY + _RHO[k] * sum(d[mu] * GAMMA[mu] for mu in range(4))


def brillouin_w_grad_at(chi, psi, coords) -> np.ndarray:
    """G_{W_d}(x) for x in coords and the 40 stored d, shape (n, 40, Nc, Nc):
    the gradient of Re<chi, D_B psi> with respect to the stored W (see
    ``oracle.grad.link_grad_brillouin_W``).  W_d(x) enters out(x) through the
    hop S_d W_d(x) psi(x + d), S_d = -lambda_k/2 + rho_k d.gamma, and out(x + d)
    through the hop along -d, S_{-d} W_d(x)^dag psi(x); only chi and psi at x
    and x + d take part."""
    nc = psi.shape[-2]
    G = np.zeros((len(coords), 40, nc, nc), dtype=np.complex128)
    for j, d in enumerate(_stored_directions()):
        md = tuple(-c for c in d)
        a_f = _spin(_dag(_bri_spin(d)), _at(chi, coords))
        a_b = _spin(_dag(_bri_spin(md)), _at(chi, coords, d))
        t1 = np.einsum("nsav,nsbv->nab", a_f, np.conj(_at(psi, coords, d)))
        t2 = np.einsum("nsav,nsbv->nab", _at(psi, coords), np.conj(a_b))
        G[:, j] = t1 + t2
    return G


def _hop_link_at(V, coords, pos, mu, s):
    """The link of the hop s mu that starts at x + pos, for x in coords:
    V_mu(x + pos), or V_mu(x + pos - mu)^dag against the link."""
    if s > 0:
        return _at(V, coords, pos)[:, mu]
    return _dag(_at(V, coords, pos + np.array(_unit(mu, -1)))[:, mu])


def brillouin_links_backward_at(V, G_W, coords, mu: int) -> np.ndarray:
    """G_V(y, mu) for y in coords: the gradient with respect to V_mu(y) of
    Re sum conj(G_W) W[V] (see ``oracle.grad.brillouin_links_backward``).
    A path uses the link in its hop along mu.  For every stored d with
    d_mu != 0, every ordering of its hops and the position i of the mu hop,
    the path starts at y less the displacement of the hops before i (a hop
    along the link), or at y + mu less it (a hop against the link, from
    y + mu to y).  That hop receives P^dag G_{W_d}(start) Q^dag / k!, P and Q
    the products of the hops before and after it, or the adjoint of that
    against the link."""
    nc = V.shape[-1]
    eye = np.broadcast_to(np.eye(nc, dtype=np.complex128), (len(coords), nc, nc))
    out = np.zeros((len(coords), nc, nc), dtype=np.complex128)
    for j, d in enumerate(_stored_directions()):
        s = d[mu]
        if s == 0:
            continue
        steps = [(m, c) for m, c in enumerate(d) if c]
        orders = list(itertools.permutations(steps))
        for order in orders:
            i = order.index((mu, s))
            start = np.zeros(4, dtype=int) if s > 0 else np.array(_unit(mu))
            for m, c in order[:i]:
                start = start - np.array(_unit(m, c))
            pos = start.copy()
            P = eye
            for m, c in order[:i]:
                P = P @ _hop_link_at(V, coords, pos, m, c)
                pos = pos + np.array(_unit(m, c))
            pos = pos + np.array(_unit(mu, s))
            Q = eye
            for m, c in order[i + 1:]:
                Q = Q @ _hop_link_at(V, coords, pos, m, c)
                pos = pos + np.array(_unit(m, c))
            X = _dag(P) @ _at(G_W, coords, start)[:, j] @ _dag(Q) / len(orders)
            out += X if s > 0 else _dag(X)
    return out


def loss_at(op: str, V, chi, psi, mass, coords) -> float:
    """Re sum over the listed sites of conj(chi(x)) * (D psi)(x)."""
    if op == "staggered":
        out = staggered_at(V, psi, mass, coords)
    elif op == "wilson":
        out = wilson_at(V, psi, mass, coords)
    else:
        raise ValueError(op)
    c = coords
    return float(np.real(np.vdot(chi[c[:, 3], c[:, 2], c[:, 1], c[:, 0]], out)))


def fd_link_grad_local(op: str, V, chi, psi, mass, link, h: float = 1.0) -> complex:
    """Central difference of L = Re sum_x conj(chi) (D psi) in the real and
    imaginary part of one link entry ``link = (t, z, y, x, mu, a, b)``.

    Only out(x) and out(x + mu) depend on V_mu(x), so the difference of L
    equals that of the loss restricted to those two sites; L is affine in the
    entry, so the difference is exact.  ``V`` is perturbed in place and
    restored.
    """
    t, z, y, x, mu, _, _ = link
    dims = _dims(V)
    here = np.array([x, y, z, t])
    there = here.copy()
    there[mu] = (there[mu] + 1) % dims[mu]
    sites = np.stack([here, there])
    if there[mu] == here[mu]:
        sites = sites[:1]
    saved = V[link]
    parts = []
    try:
        for step in (1.0, 1j):
            V[link] = saved + h * step
            lp = loss_at(op, V, chi, psi, mass, sites)
            V[link] = saved - h * step
            lm = loss_at(op, V, chi, psi, mass, sites)
            parts.append((lp - lm) / (2 * h))
    finally:
        V[link] = saved
    return parts[0] + 1j * parts[1]
