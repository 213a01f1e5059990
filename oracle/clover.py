"""Clover (Sheikholeslami-Wohlert) term of D_W and D_B (oracle; test infrastructure only).

Eqs. def_wils and def_bril (Secs. 4 and 5) both end in the site-local term
-(c_SW/2) sum_{mu<nu} sigma_{mu nu} F_{mu nu}(x) delta_{x,y}; all of the paper's
benchmarks take c_SW = 0 and it defines neither sigma nor F.  Reading taken
here (the standard clover-leaf construction):

* sigma_{mu nu} = (i/2) [gamma_mu, gamma_nu], Hermitian, with the gamma
  matrices of gamma.py;
* Q_{mu nu}(x) = sum of the four plaquettes of the (mu, nu) plane that start
  and end at x, each run in the sense x -> x+a -> x+a+b -> x+b -> x for
  (a, b) = (mu, nu), (nu, -mu), (-mu, -nu), (-nu, mu), with V_{-mu}(x) =
  V_mu(x-mu)^dag;
* F_{mu nu}(x) = (Q_{mu nu}(x) - Q_{mu nu}(x)^dag) / (8 i): Hermitian, no
  trace subtraction.

The term is then Hermitian (so (D + C)^dag = D^dag + C) and commutes with
gamma_5; in the chiral basis it is block diagonal with one 6x6 block for
spins (0, 1) and one for spins (2, 3), row index 3 s' + c within a block.

Packed storage of the term (the library's interface format), per site two
blocks b = 0, 1 of 18 complex words each: words 0..2 hold the real diagonal
as (H_00, H_11), (H_22, H_33), (H_44, H_55) in (re, im); words 3..17 hold the
upper triangle H_ij, i < j, row by row.
"""
from __future__ import annotations

import numpy as np

from . import brillouin, wilson
from .gamma import GAMMA
from .lattice import shift

PAIRS = [(mu, nu) for mu in range(4) for nu in range(mu + 1, 4)]
UPPER = [(i, j) for i in range(6) for j in range(i + 1, 6)]


def sigma(mu: int, nu: int) -> np.ndarray:
    g = GAMMA
    return 0.5j * (g[mu] @ g[nu] - g[nu] @ g[mu])


def _dagger(u: np.ndarray) -> np.ndarray:
    return np.conj(np.swapaxes(u, -1, -2))


def _hop(V: np.ndarray, a) -> np.ndarray:
    """Field of the link from x to x + a for a signed direction a = (mu, +-1)."""
    mu, s = a
    return V[..., mu, :, :] if s > 0 else _dagger(shift(V[..., mu, :, :], mu, -1))


def _step(field: np.ndarray, a) -> np.ndarray:
    """g(x) = field(x + a)."""
    mu, s = a
    return shift(field, mu, s)


def plaquette(V: np.ndarray, a, b) -> np.ndarray:
    """Product of the links along x -> x+a -> x+a+b -> x+b -> x, at every x."""
    neg = lambda d: (d[0], -d[1])  # noqa: E731
    l1 = _hop(V, a)
    l2 = _step(_hop(V, b), a)
    l3 = _step(_step(_hop(V, neg(a)), a), b)
    l4 = _step(_hop(V, neg(b)), b)
    return l1 @ l2 @ l3 @ l4


def leaves(V: np.ndarray, mu: int, nu: int) -> np.ndarray:
    """Q_{mu nu}(x): the four plaquettes of the clover leaf at x."""
    m, n = (mu, 1), (nu, 1)
    mm, nn = (mu, -1), (nu, -1)
    return plaquette(V, m, n) + plaquette(V, n, mm) + plaquette(V, mm, nn) + plaquette(V, nn, m)


def field_strength(V: np.ndarray, mu: int, nu: int) -> np.ndarray:
    q = leaves(V, mu, nu)
    return (q - _dagger(q)) / 8j


def term(V: np.ndarray, c_sw: float) -> np.ndarray:
    """-(c_SW/2) sum_{mu<nu} sigma_{mu nu} (x) F_{mu nu}(x) as [..site..][12][12],
    index 3 s + c (spin s, colour c)."""
    lat = V.shape[:4]
    out = np.zeros(lat + (12, 12), dtype=complex)
    for mu, nu in PAIRS:
        f = field_strength(V, mu, nu)
        out += np.einsum("st,...ab->...satb", sigma(mu, nu), f).reshape(lat + (12, 12))
    return -0.5 * c_sw * out


def apply_term(T: np.ndarray, psi: np.ndarray) -> np.ndarray:
    """T(x) psi(x) for a [..site..][4][3][Nv] field."""
    lat, nv = psi.shape[:4], psi.shape[-1]
    return (T @ psi.reshape(lat + (12, nv))).reshape(psi.shape)


def wilson_apply(V: np.ndarray, psi: np.ndarray, m0: float, c_sw: float, adjoint: bool = False) -> np.ndarray:
    """Eq. def_wils with its clover term; the term is Hermitian, so the adjoint
    adds it unchanged."""
    return wilson.apply(V, psi, m0, adjoint) + apply_term(term(V, c_sw), psi)


def brillouin_apply(V: np.ndarray, W: np.ndarray, psi: np.ndarray, m0: float, c_sw: float,
                    adjoint: bool = False) -> np.ndarray:
    """Eq. def_bril with its clover term (F from the one-hop links V)."""
    return brillouin.apply(W, psi, m0, adjoint) + apply_term(term(V, c_sw), psi)


def pack(T: np.ndarray) -> np.ndarray:
    """[..site..][12][12] block-diagonal Hermitian term -> [..site..][2][18] packed words."""
    lat = T.shape[:-2]
    out = np.zeros(lat + (2, 18), dtype=complex)
    for b in range(2):
        h = T[..., 6 * b:6 * b + 6, 6 * b:6 * b + 6]
        for k in range(3):
            out[..., b, k] = h[..., 2 * k, 2 * k].real + 1j * h[..., 2 * k + 1, 2 * k + 1].real
        for w, (i, j) in enumerate(UPPER):
            out[..., b, 3 + w] = h[..., i, j]
    return out


def unpack(P: np.ndarray) -> np.ndarray:
    """Inverse of ``pack``: [..site..][2][18] -> [..site..][12][12]."""
    lat = P.shape[:-2]
    out = np.zeros(lat + (12, 12), dtype=complex)
    for b in range(2):
        o = 6 * b
        for k in range(3):
            out[..., o + 2 * k, o + 2 * k] = P[..., b, k].real
            out[..., o + 2 * k + 1, o + 2 * k + 1] = P[..., b, k].imag
        for w, (i, j) in enumerate(UPPER):
            out[..., o + i, o + j] = P[..., b, 3 + w]
            out[..., o + j, o + i] = np.conj(P[..., b, 3 + w])
    return out
