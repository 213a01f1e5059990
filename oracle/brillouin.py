"""Brillouin operator D_B at c_SW = 0 and its off-axis links W (oracle; test
infrastructure only).

Sec. 5, eq. def_bril with c_SW = 0:

    D_B = sum_mu gamma_mu nabla_mu^iso - (1/2) Laplace^bri + m0

eq. def_der (54-point isotropic derivative) and eq. def_lap (81-point
Laplacian), with (rho_1..rho_4) = (64, 16, 4, 1)/432 and
(lambda_0..lambda_4) = (-240, 8, 4, 2, 1)/64.

Readings of the paper taken here (listed with the rest in the design notes):

* The sums over "mutually unequal" indices run over unordered sets of distinct
  axes with both signs, so every geometric displacement d in {-1,0,1}^4 \\ {0}
  appears once.  nabla_mu^iso then has 2 + 12 + 24 + 16 = 54 points and
  Laplace^bri 1 + 8 + 24 + 32 + 16 = 81, the counts the paper states, and
  rho_1 + 6 rho_2 + 12 rho_3 + 8 rho_4 = 1/2, lambda_0 + 8 lambda_1 +
  24 lambda_2 + 32 lambda_3 + 16 lambda_4 = 0.
* The 4-hop term of def_der carries W_{mu+nu+rho+sigma} (the printed index
  list omits sigma); the 4-hop row of Tab. 1 continues the path at
  x+mu+nu+rho (the printed site repeats sigma).
* "perm(s)" in Tab. 1 means all k! orderings of the k hops, each weighted
  1/k!, with V_{-mu}(y) = V_mu(y-mu)^dag.

Storage (Tab. 1 caption): of the 80 non-trivial directions only 40 are kept,
the rest follow from W_{-d}(x) = W_d(x-d)^dag.  Direction d is kept iff its
highest-index non-zero component is +1, equivalently
n(d) = sum_mu (d_mu + 1) 3^mu > 40; it sits in slot n(d) - 41.
Stored W: [Nt][Nz][Ny][Nx][40][Nc][Nc].
"""
from __future__ import annotations

import itertools
import math

import numpy as np

from .gamma import GAMMA, GAMMA5, spin_mul
from .lattice import shift, shift_by

RHO = {1: 64 / 432, 2: 16 / 432, 3: 4 / 432, 4: 1 / 432}
LAMBDA = {0: -240 / 64, 1: 8 / 64, 2: 4 / 64, 3: 2 / 64, 4: 1 / 64}

DIRECTIONS = [d for d in itertools.product((-1, 0, 1), repeat=4) if any(d)]
# itertools.product varies the last entry fastest; reverse so entry mu is d_mu
DIRECTIONS = [tuple(reversed(d)) for d in DIRECTIONS]


def hops(d) -> int:
    """k(d): number of non-zero components (the hop count)."""
    return sum(1 for c in d if c)


def code(d) -> int:
    """n(d) = sum_mu (d_mu + 1) 3^mu in [0, 80]; n(0) = 40 and n(-d) = 80 - n(d)."""
    return sum((c + 1) * 3 ** mu for mu, c in enumerate(d))


def slot(d):
    """Storage slot of d in the 40-entry W array, or None if d is not stored."""
    n = code(d)
    return n - 41 if n > 40 else None


STORED = sorted((d for d in DIRECTIONS if slot(d) is not None), key=slot)


def _dagger(u: np.ndarray) -> np.ndarray:
    return np.conj(np.swapaxes(u, -1, -2))


def _hop_link(V: np.ndarray, mu: int, sign: int) -> np.ndarray:
    """The field y -> V_{sign mu}(y): V_mu(y) for sign +1, V_mu(y - mu)^dag for -1."""
    if sign > 0:
        return V[..., mu, :, :]
    return _dagger(shift(V[..., mu, :, :], mu, -1))


def path_link(V: np.ndarray, d) -> np.ndarray:
    """W_d(x) of Tab. 1: average over all k! hop orderings of the path product."""
    steps = [(mu, c) for mu, c in enumerate(d) if c]
    nc = V.shape[-1]
    total = np.zeros(V.shape[:4] + (nc, nc), dtype=np.complex128)
    orders = list(itertools.permutations(steps))
    for order in orders:
        prod = None
        offset = [0, 0, 0, 0]
        for mu, sgn in order:
            link = shift_by(_hop_link(V, mu, sgn), offset)
            prod = link if prod is None else prod @ link
            offset[mu] += sgn
        total += prod
    assert len(orders) == math.factorial(len(steps))
    return total / len(orders)


def build_all(V: np.ndarray) -> dict:
    """All 80 W_d fields, each built from its own paths (no symmetry used)."""
    return {d: path_link(V, d) for d in DIRECTIONS}


def pack(w_all: dict) -> np.ndarray:
    """Stored 40-direction array [..][40][Nc][Nc] from the full set."""
    return np.stack([w_all[d] for d in STORED], axis=4)


def build(V: np.ndarray) -> np.ndarray:
    """Stored W [Nt][Nz][Ny][Nx][40][Nc][Nc] built from V (Tab. 1)."""
    return np.stack([path_link(V, d) for d in STORED], axis=4)


def link(W: np.ndarray, d) -> np.ndarray:
    """W_d(x) for any d != 0 from the stored array, using
    W_d(x) = W_{-d}(x + d)^dag for the directions that are not stored."""
    s = slot(d)
    if s is not None:
        return W[..., s, :, :]
    neg = tuple(-c for c in d)
    return _dagger(shift_by(W[..., slot(neg), :, :], d))


def _transport(u: np.ndarray, psi: np.ndarray) -> np.ndarray:
    return u[..., None, :, :] @ psi


def term(W: np.ndarray, psi: np.ndarray, d) -> np.ndarray:
    """W_d(x) psi(x + d)."""
    return _transport(link(W, d), shift_by(psi, d))


def nabla_iso(W: np.ndarray, psi: np.ndarray, mu: int) -> np.ndarray:
    """eq. def_der: sum over the 27 displacements o orthogonal to mu (|o| = 0..3
    non-zero entries) of rho_{1+|o|} [W_{mu+o} psi(x+mu+o) - W_{-mu+o} psi(x-mu+o)]."""
    out = np.zeros_like(psi)
    others = [nu for nu in range(4) if nu != mu]
    for o_vals in itertools.product((-1, 0, 1), repeat=3):
        o = [0, 0, 0, 0]
        for nu, c in zip(others, o_vals):
            o[nu] = c
        k = 1 + hops(o)
        plus = list(o)
        plus[mu] = +1
        minus = list(o)
        minus[mu] = -1
        out = out + RHO[k] * (term(W, psi, tuple(plus)) - term(W, psi, tuple(minus)))
    return out


def laplace_bri(W: np.ndarray, psi: np.ndarray) -> np.ndarray:
    """eq. def_lap: lambda_0 psi(x) + sum_{d != 0} lambda_{k(d)} W_d(x) psi(x+d)."""
    out = LAMBDA[0] * psi
    for d in DIRECTIONS:
        out = out + LAMBDA[hops(d)] * term(W, psi, d)
    return out


def apply(W: np.ndarray, psi: np.ndarray, m0: float = 0.0, adjoint: bool = False) -> np.ndarray:
    """(D_B psi)(x) from eq. def_bril; D_B^dag = gamma_5 D_B gamma_5 if ``adjoint``
    (nabla^iso is anti-Hermitian and Laplace^bri Hermitian, given the W relation)."""
    if adjoint:
        return spin_mul(GAMMA5, apply(W, spin_mul(GAMMA5, psi), m0))
    out = m0 * psi - 0.5 * laplace_bri(W, psi)
    for mu in range(4):
        out = out + spin_mul(GAMMA[mu], nabla_iso(W, psi, mu))
    return out


def apply_hop(W: np.ndarray, psi: np.ndarray, m0: float = 0.0, adjoint: bool = False) -> np.ndarray:
    """Rearranged form: (m0 - lambda_0/2) psi + sum_d [-lambda_k/2 + rho_k d.gamma] W_d psi(x+d);
    ``adjoint`` flips the sign of d.gamma."""
    sgn = -1.0 if adjoint else 1.0
    out = (m0 - 0.5 * LAMBDA[0]) * psi
    for d in DIRECTIONS:
        k = hops(d)
        spin = -0.5 * LAMBDA[k] * np.eye(4) + sgn * RHO[k] * sum(c * GAMMA[mu] for mu, c in enumerate(d))
        out = out + spin_mul(spin, term(W, psi, d))
    return out
