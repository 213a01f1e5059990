"""Link gradient of L = Re sum_x chi(x)^dag (D psi)(x) (oracle; test
infrastructure only).

The paper has no gradients.  The loss is the real part of the sum over all
sites, right-hand sides, spins and colours of conj(chi) * (D psi).  Links are
treated as free complex matrices, and the gradient follows the PyTorch
convention for a real function of a complex variable:
G = dL/d(Re V) + i dL/d(Im V).

Derivation, used as written below.  A link V_mu(x) enters D twice: the forward
hop into out(x), with spin-colour factor P_+ (x) V acting on psi(x+mu), and the
backward hop into out(x+mu), with P_- (x) V^dag acting on psi(x).  For
L = Re sum conj(chi_a) V_ab phi_b the gradient is G_ab = chi_a conj(phi_b); for
L = Re sum conj(chi_a) conj(V_ba) phi_b it is G_ba = phi_b conj(chi_a).  Hence

    G_mu(x) = sum_v sum_s [ chi(x)_s (x) conj((P_+ psi(x+mu))_s)
                          + (P_- psi(x))_s (x) conj(chi(x+mu)_s) ]

with (x) the outer product over colour.  Staggered: P_+ = eta_mu(x)/2,
P_- = -eta_mu(x+mu)/2 (Sec. 3).  Wilson: P_+ = -(1 - gamma_mu)/2,
P_- = -(1 + gamma_mu)/2 (the hop form of eq. def_wils).  The mass term does not
depend on the links.

L is affine in the real and imaginary part of every single link, so a central
difference in one link component is exact for any step (``fd_link_grad``).

Brillouin.  With the stored W taken as free matrices, W_d(x) (d stored) enters
the hop term of d into out(x), factor S_d = -lambda_k/2 + rho_k d.gamma (the
hop form of eqs. def_bril, def_der, def_lap), and, as W_{-d}(x + d) =
W_d(x)^dag, the hop term of -d into out(x + d), factor S_{-d}:

    G_{W_d}(x) = sum_v sum_s [ (S_d^dag chi(x))_s (x) conj(psi(x+d)_s)
                             + psi(x)_s (x) conj((S_{-d}^dag chi(x+d))_s) ].

Through the construction of W from V (Tab. 1) the chain rule runs over every
path product M = A_1 ... A_k of every stored d: with P and Q the products
before and after hop i, delta L = Re tr(G_M^dag P delta A_i Q) gives the
gradient P^dag G_M Q^dag / k! for A_i, and its adjoint for the link V_mu(y)
when the hop runs against it (A_i = V_mu(y)^dag).  L is then a polynomial of
degree at most 4 along any line V + t Delta, so a five-point central
difference is exact.
"""
from __future__ import annotations

import numpy as np

import itertools

from . import brillouin, staggered, wilson
from .gamma import GAMMA, IDENTITY, spin_mul
from .lattice import dims_of, eta, shift, shift_by


def loss(op: str, U: np.ndarray, chi: np.ndarray, psi: np.ndarray, mass: float = 0.0) -> float:
    """L = Re sum conj(chi) * (D psi)."""
    if op == "staggered":
        out = staggered.apply(U, psi, mass)
    elif op == "wilson":
        out = wilson.apply(U, psi, mass)
    elif op == "brillouin":
        out = brillouin.apply(U, psi, mass)
    else:
        raise ValueError(op)
    return float(np.real(np.vdot(chi, out)))


def link_grad_staggered(chi: np.ndarray, psi: np.ndarray) -> np.ndarray:
    """G [Nt][Nz][Ny][Nx][4][Nc][Nc] for D_S; chi, psi [...][Nc][Nv]."""
    et = eta(dims_of(psi))
    nc = psi.shape[-2]
    G = np.zeros(psi.shape[:4] + (4, nc, nc), dtype=np.complex128)
    for mu in range(4):
        e_x = et[mu][..., None, None]
        e_xp = shift(et[mu], mu, +1)[..., None, None]
        t1 = (0.5 * e_x) * (chi @ np.conj(np.swapaxes(shift(psi, mu, +1), -1, -2)))
        t2 = (-0.5 * e_xp) * (psi @ np.conj(np.swapaxes(shift(chi, mu, +1), -1, -2)))
        G[..., mu, :, :] = t1 + t2
    return G


def link_grad_wilson(chi: np.ndarray, psi: np.ndarray) -> np.ndarray:
    """G [Nt][Nz][Ny][Nx][4][Nc][Nc] for D_W (c_SW = 0); chi, psi [...][4][Nc][Nv]."""
    nc = psi.shape[-2]
    G = np.zeros(psi.shape[:4] + (4, nc, nc), dtype=np.complex128)
    for mu in range(4):
        phi_f = spin_mul(-0.5 * (IDENTITY - GAMMA[mu]), shift(psi, mu, +1))
        phi_b = spin_mul(-0.5 * (IDENTITY + GAMMA[mu]), psi)
        chi_f = shift(chi, mu, +1)
        t1 = np.einsum("...sav,...sbv->...ab", chi, np.conj(phi_f))
        t2 = np.einsum("...sav,...sbv->...ab", phi_b, np.conj(chi_f))
        G[..., mu, :, :] = t1 + t2
    return G


def _dag(u: np.ndarray) -> np.ndarray:
    return np.conj(np.swapaxes(u, -1, -2))


def _spin_factor(d) -> np.ndarray:
    k = brillouin.hops(d)
    return -0.5 * brillouin.LAMBDA[k] * IDENTITY + brillouin.RHO[k] * sum(c * GAMMA[mu] for mu, c in enumerate(d))


def link_grad_brillouin_W(chi: np.ndarray, psi: np.ndarray) -> np.ndarray:
    """G [..][40][Nc][Nc] with respect to the stored W (free matrices); chi, psi [..][4][Nc][Nv]."""
    nc = psi.shape[-2]
    G = np.zeros(psi.shape[:4] + (40, nc, nc), dtype=np.complex128)
    for j, d in enumerate(brillouin.STORED):
        md = tuple(-c for c in d)
        a_f = spin_mul(_dag(_spin_factor(d)), chi)
        a_b = spin_mul(_dag(_spin_factor(md)), shift_by(chi, d))
        t1 = np.einsum("...sav,...sbv->...ab", a_f, np.conj(shift_by(psi, d)))
        t2 = np.einsum("...sav,...sbv->...ab", psi, np.conj(a_b))
        G[..., j, :, :] = t1 + t2
    return G


def brillouin_links_backward(V: np.ndarray, G_W: np.ndarray) -> np.ndarray:
    """Gradient with respect to V of Re sum conj(G_W) W[V] (the adjoint of the W construction)."""
    nc = V.shape[-1]
    G_V = np.zeros(V.shape, dtype=np.complex128)
    eye = np.broadcast_to(np.eye(nc, dtype=np.complex128), V.shape[:4] + (nc, nc))
    for j, d in enumerate(brillouin.STORED):
        G = G_W[..., j, :, :]
        steps = [(mu, c) for mu, c in enumerate(d) if c]
        orders = list(itertools.permutations(steps))
        for order in orders:
            hops, offs = [], []
            off = [0, 0, 0, 0]
            for mu, sgn in order:
                hops.append(shift_by(brillouin._hop_link(V, mu, sgn), off))
                offs.append(tuple(off))
                off[mu] += sgn
            for i, (mu, sgn) in enumerate(order):
                P, Q = eye, eye
                for h in hops[:i]:
                    P = P @ h
                for h in hops[i + 1:]:
                    Q = Q @ h
                X = _dag(P) @ G @ _dag(Q) / len(orders)
                if sgn > 0:
                    # A_i(x) = V_mu(x + off_i): the gradient lands at y = x + off_i
                    G_V[..., mu, :, :] += shift_by(X, tuple(-o for o in offs[i]))
                else:
                    # A_i(x) = V_mu(x + off_i - mu)^dag
                    back = list(-o for o in offs[i])
                    back[mu] += 1
                    G_V[..., mu, :, :] += _dag(shift_by(X, tuple(back)))
    return G_V


def link_grad_brillouin(V: np.ndarray, chi: np.ndarray, psi: np.ndarray) -> np.ndarray:
    """G [..][4][Nc][Nc] of L = Re<chi, D_B[W(V)] psi> with respect to the one-hop links V."""
    return brillouin_links_backward(V, link_grad_brillouin_W(chi, psi))


def link_grad(op: str, chi: np.ndarray, psi: np.ndarray) -> np.ndarray:
    if op == "staggered":
        return link_grad_staggered(chi, psi)
    if op == "wilson":
        return link_grad_wilson(chi, psi)
    raise ValueError(op)


def fd_link_grad(op: str, U: np.ndarray, chi: np.ndarray, psi: np.ndarray, links, mass: float = 0.0,
                 h: float = 1.0) -> np.ndarray:
    """Central differences of L in Re and Im of single link entries.

    ``links`` is a list of (t, z, y, x, mu, a, b); returns the complex
    dL/dRe + i dL/dIm for each.  Exact for any h because L is affine in each
    entry.
    """
    out = np.zeros(len(links), dtype=np.complex128)
    for n, idx in enumerate(links):
        parts = []
        for step in (1.0, 1j):
            Up = U.copy()
            Um = U.copy()
            Up[idx] += h * step
            Um[idx] -= h * step
            parts.append((loss(op, Up, chi, psi, mass) - loss(op, Um, chi, psi, mass)) / (2 * h))
        out[n] = parts[0] + 1j * parts[1]
    return out
