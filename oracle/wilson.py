"""Wilson operator D_W at c_SW = 0 (oracle; test infrastructure only).

Sec. 4, eq. def_wils with c_SW = 0 (all of the paper's Wilson benchmarks):

    D_W = sum_mu gamma_mu nabla_mu^std - (1/2) Laplace^std + m0

    nabla_mu^std psi(x) = (1/2) [ V_mu(x) psi(x+mu) - V_{-mu}(x) psi(x-mu) ]
    Laplace^std psi(x)  = -8 psi(x) + sum over the 4 positive and 4 negative
                          directions of V_{+-mu}(x) psi(x+-mu)

with V_{-mu}(x) = V_mu(x-mu)^dag, the one-hop case of the relation
W_{-dir}(x) = W_dir(x-dir)^dag stated with Tab. 1 (lattice spacing a = 1).

``apply`` is the literal form above.  ``apply_hop`` is its algebraic
rearrangement (4 + m0) psi - (1/2) sum_mu [(1 - gamma_mu) V_mu(x) psi(x+mu)
+ (1 + gamma_mu) V_mu(x-mu)^dag psi(x-mu)]; the tests assert the two agree.

Fields: V [Nt][Nz][Ny][Nx][4][Nc][Nc], psi [Nt][Nz][Ny][Nx][4][Nc][Nv].
"""
from __future__ import annotations

import numpy as np

from .gamma import GAMMA, GAMMA5, IDENTITY, spin_mul
from .lattice import shift


def _transport(u: np.ndarray, psi: np.ndarray) -> np.ndarray:
    """u(x) acting on the colour index of a [...][4][Nc][Nv] field."""
    return u[..., None, :, :] @ psi


def _dagger(u: np.ndarray) -> np.ndarray:
    return np.conj(np.swapaxes(u, -1, -2))


def link_forward(V: np.ndarray, psi: np.ndarray, mu: int) -> np.ndarray:
    """V_mu(x) psi(x + mu)."""
    return _transport(V[..., mu, :, :], shift(psi, mu, +1))


def link_backward(V: np.ndarray, psi: np.ndarray, mu: int) -> np.ndarray:
    """V_{-mu}(x) psi(x - mu) = V_mu(x - mu)^dag psi(x - mu)."""
    return _transport(_dagger(shift(V[..., mu, :, :], mu, -1)), shift(psi, mu, -1))


def nabla_std(V: np.ndarray, psi: np.ndarray, mu: int) -> np.ndarray:
    return 0.5 * (link_forward(V, psi, mu) - link_backward(V, psi, mu))


def laplace_std(V: np.ndarray, psi: np.ndarray) -> np.ndarray:
    out = -8.0 * psi
    for mu in range(4):
        out = out + link_forward(V, psi, mu) + link_backward(V, psi, mu)
    return out


def apply(V: np.ndarray, psi: np.ndarray, m0: float = 0.0, adjoint: bool = False) -> np.ndarray:
    """(D_W psi)(x) from eq. def_wils; D_W^dag = gamma_5 D_W gamma_5 if ``adjoint``.

    The adjoint identity follows from the definition: nabla^std is
    anti-Hermitian, Laplace^std Hermitian and gamma_5 anticommutes with every
    gamma_mu; the tests check it against <chi, D psi> = <D^dag chi, psi>.
    """
    if adjoint:
        return spin_mul(GAMMA5, apply(V, spin_mul(GAMMA5, psi), m0))
    out = m0 * psi - 0.5 * laplace_std(V, psi)
    for mu in range(4):
        out = out + spin_mul(GAMMA[mu], nabla_std(V, psi, mu))
    return out


def apply_hop(V: np.ndarray, psi: np.ndarray, m0: float = 0.0, adjoint: bool = False) -> np.ndarray:
    """Hop form of the same operator; ``adjoint`` flips the sign of every gamma_mu."""
    sgn = -1.0 if adjoint else 1.0
    out = (4.0 + m0) * psi
    for mu in range(4):
        out = out - 0.5 * spin_mul(IDENTITY - sgn * GAMMA[mu], link_forward(V, psi, mu))
        out = out - 0.5 * spin_mul(IDENTITY + sgn * GAMMA[mu], link_backward(V, psi, mu))
    return out
