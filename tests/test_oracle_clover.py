"""Pins for the oracle's clover term (eqs. def_wils / def_bril, c_SW != 0).

The expected values of the abelian and two-link cases below are worked out by
hand from the definitions (plaquette phases, the chiral-basis sigma_{mu nu}),
not by re-running the oracle's formulas.
"""
import numpy as np
import pytest

import synthetic
from oracle import brillouin, clover, lattice, wilson
from oracle.gamma import GAMMA5, spin_mul
from tests.helpers import coords, dag, random_gauge

DIMS = (4, 4, 2, 4)
C_SW = 1.7


def _unit(dims):
    return synthetic.gauge_links(dims, "unit", 0)


def _spin_diag(T):
    """Diagonal spin factor d_s of a term T = diag(d) (x) 1_colour, checked to have that form."""
    lat = T.shape[:-2]
    d = np.stack([T[..., 3 * s, 3 * s] for s in range(4)], -1)
    expect = np.zeros(lat + (12, 12), dtype=complex)
    for s in range(4):
        for c in range(3):
            expect[..., 3 * s + c, 3 * s + c] = d[..., s]
    assert np.abs(T - expect).max() < 1e-13
    return d


def test_sigma_hermitian_and_chiral():
    for mu, nu in clover.PAIRS:
        s = clover.sigma(mu, nu)
        assert np.abs(s - dag(s)).max() < 1e-15
        assert np.abs(s @ GAMMA5 - GAMMA5 @ s).max() < 1e-15
    # sigma_12 = -diag(sigma_3, sigma_3) and sigma_34 = diag(sigma_3, -sigma_3) in the chiral basis
    assert np.allclose(clover.sigma(0, 1), np.diag([-1, 1, -1, 1]))
    assert np.allclose(clover.sigma(2, 3), np.diag([1, -1, -1, 1]))


def test_free_field_has_no_clover_term():
    assert np.abs(clover.term(_unit(DIMS), C_SW)).max() < 1e-15


@pytest.mark.parametrize("plane", [(0, 1), (2, 3), (1, 3)])
def test_abelian_field_strength(plane):
    # V_nu(x) = exp(i phi(x_mu)) with every other link 1: the plaquette of the
    # (mu, nu) plane with lower corner x has angle a(x_mu) = phi(x_mu + 1) - phi(x_mu),
    # and the four leaves at x carry a(x_mu) twice and a(x_mu - 1) twice, so
    # F_{mu nu}(x) = [sin a(x_mu) + sin a(x_mu - 1)] / 2 and every other F vanishes.
    mu, nu = plane
    n = DIMS[mu]
    phi = np.random.default_rng(11).uniform(-np.pi, np.pi, n)
    x = coords(DIMS)[mu]
    V = _unit(DIMS).copy()
    V[..., nu, :, :] = np.exp(1j * phi[x])[..., None, None] * np.eye(3)
    a = np.roll(phi, -1) - phi
    f = 0.5 * (np.sin(a) + np.sin(np.roll(a, 1)))[x]
    F = clover.field_strength(V, mu, nu)
    assert np.abs(F - f[..., None, None] * np.eye(3)).max() < 1e-14
    for p in clover.PAIRS:
        if p != plane:
            assert np.abs(clover.field_strength(V, *p)).max() < 1e-14
    # term = -(c/2) f sigma_{mu nu}: sigma_12 = -diag(1,-1,1,-1), sigma_34 = diag(1,-1,-1,1),
    # sigma_24 = diag(sigma_2, -sigma_2) (not diagonal; checked through the block structure)
    T = clover.term(V, C_SW)
    if plane == (0, 1):
        d = _spin_diag(T)
        assert np.abs(d - 0.5 * C_SW * f[..., None] * np.array([1, -1, 1, -1])).max() < 1e-14
    elif plane == (2, 3):
        d = _spin_diag(T)
        assert np.abs(d - (-0.5) * C_SW * f[..., None] * np.array([1, -1, -1, 1])).max() < 1e-14
    else:
        s2 = np.array([[0, -1j], [1j, 0]])
        spin = np.zeros((4, 4), dtype=complex)
        spin[:2, :2], spin[2:, 2:] = s2, -s2
        expect = -0.5 * C_SW * f[..., None, None, None, None] * np.einsum("st,ab->satb", spin, np.eye(3))
        assert np.abs(T - expect.reshape(T.shape)).max() < 1e-14


def test_two_link_leaf_order():
    # V_x(x0) = A and V_y(x0 + x) = B, all other links 1.  At x0 the (x, y)
    # leaves are A B (first leaf), A^dag (fourth leaf: it ends with the step
    # from x0 + x back to x0) and 1, 1, so F_xy(x0) = (A B + A^dag - h.c.) / (8 i).
    A = synthetic.haar_su3(1, 21)[0]
    B = synthetic.haar_su3(1, 22)[0]
    V = _unit(DIMS).copy()
    V[0, 0, 0, 0, 0] = A
    V[0, 0, 0, 1, 1] = B
    q = A @ B + dag(A) + 2 * np.eye(3)
    F = clover.field_strength(V, 0, 1)
    assert np.abs(F[0, 0, 0, 0] - (q - dag(q)) / 8j).max() < 1e-14
    # at x0 + x + y the third leaf runs x0+x+y -> x0+y -> x0 -> x0+x -> x0+x+y,
    # i.e. 1 . 1 . A . B, and the fourth starts with the step down to x0 + x: B^dag
    q2 = A @ B + dag(B) + 2 * np.eye(3)
    assert np.abs(F[0, 0, 1, 1] - (q2 - dag(q2)) / 8j).max() < 1e-14


def test_term_hermitian_block_diagonal():
    V = synthetic.gauge_links(DIMS, "haar", 12)
    T = clover.term(V, C_SW)
    assert np.abs(T - dag(T)).max() < 1e-14
    assert np.abs(T[..., :6, 6:]).max() < 1e-15
    assert np.abs(T[..., 6:, :6]).max() < 1e-15
    assert np.abs(T).max() > 0.1
    # spin trace of sigma vanishes: the colour trace over each spin pair cancels
    tr = np.einsum("...ii->...", T)
    assert np.abs(tr).max() < 1e-13


def test_gauge_covariance():
    V = synthetic.gauge_links(DIMS, "haar", 13)
    g = random_gauge(DIMS, 14)
    vg = np.empty_like(V)
    for mu in range(4):
        vg[..., mu, :, :] = g @ V[..., mu, :, :] @ dag(lattice.shift(g, mu, 1))
    G = np.zeros(DIMS[::-1] + (12, 12), dtype=complex)
    for s in range(4):
        G[..., 3 * s:3 * s + 3, 3 * s:3 * s + 3] = g
    lhs = clover.term(vg, C_SW)
    rhs = G @ clover.term(V, C_SW) @ dag(G)
    assert np.abs(lhs - rhs).max() < 1e-13


def test_pack_unpack():
    V = synthetic.gauge_links(DIMS, "haar", 15)
    T = clover.term(V, C_SW)
    P = clover.pack(T)
    assert P.shape == DIMS[::-1] + (2, 18)
    assert np.abs(clover.unpack(P) - T).max() < 1e-15
    # layout: words 0..2 hold the diagonal pairwise, word 3 is H_01 of the block, word 17 is H_45
    assert np.allclose(P[..., 1, 1], T[..., 8, 8].real + 1j * T[..., 9, 9].real)
    assert np.allclose(P[..., 0, 3], T[..., 0, 1])
    assert np.allclose(P[..., 1, 17], T[..., 10, 11])
    assert np.allclose(P[..., 0, 8], T[..., 1, 2])


def test_wilson_with_clover_adjoint_and_gamma5():
    V = synthetic.gauge_links(DIMS, "smooth", 16)
    psi = synthetic.wilson_spinor(DIMS, 2, 17)
    chi = synthetic.wilson_spinor(DIMS, 2, 18)
    lhs = np.vdot(chi, clover.wilson_apply(V, psi, 0.1, C_SW))
    rhs = np.vdot(clover.wilson_apply(V, chi, 0.1, C_SW, adjoint=True), psi)
    assert abs(lhs - rhs) < 1e-12 * abs(lhs)
    g5 = spin_mul(GAMMA5, clover.wilson_apply(V, spin_mul(GAMMA5, psi), 0.1, C_SW))
    assert np.abs(g5 - clover.wilson_apply(V, psi, 0.1, C_SW, adjoint=True)).max() < 1e-13
    # c_SW = 0 is the operator without the term
    assert np.abs(clover.wilson_apply(V, psi, 0.1, 0.0) - wilson.apply(V, psi, 0.1)).max() < 1e-15


def test_brillouin_with_clover_adjoint():
    dims = (4, 2, 2, 4)
    V = synthetic.gauge_links(dims, "haar", 19)
    W = brillouin.build(V)
    psi = synthetic.wilson_spinor(dims, 1, 20)
    chi = synthetic.wilson_spinor(dims, 1, 23)
    lhs = np.vdot(chi, clover.brillouin_apply(V, W, psi, 0.1, C_SW))
    rhs = np.vdot(clover.brillouin_apply(V, W, chi, 0.1, C_SW, adjoint=True), psi)
    assert abs(lhs - rhs) < 1e-12 * abs(lhs)
