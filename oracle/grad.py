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
"""
from __future__ import annotations

import numpy as np

from . import staggered, wilson
from .gamma import GAMMA, IDENTITY, spin_mul
from .lattice import dims_of, eta, shift


def loss(op: str, U: np.ndarray, chi: np.ndarray, psi: np.ndarray, mass: float = 0.0) -> float:
    """L = Re sum conj(chi) * (D psi)."""
    if op == "staggered":
        out = staggered.apply(U, psi, mass)
    elif op == "wilson":
        out = wilson.apply(U, psi, mass)
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
