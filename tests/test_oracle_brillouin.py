"""Pins for the oracle's W (Tab. 1) and D_B (Sec. 5, eqs. def_bril/def_der/def_lap)."""
import itertools
import math
from fractions import Fraction

import numpy as np
import pytest

import synthetic
from oracle import brillouin as B
from oracle import dense, lattice
from oracle.gamma import GAMMA, GAMMA5, spin_mul
from tests.helpers import dag, plane_wave, random_gauge, read_golden

DIMS = (3, 4, 3, 5)


def _golden():
    rows = read_golden("table1_offaxis.txt")
    table = {int(r[0]): (int(r[1]), int(r[2])) for r in rows if r[0].isdigit()}
    named = {r[0]: int(r[1]) for r in rows if not r[0].isdigit()}
    return table, named


def test_direction_counts_match_table1():
    table, named = _golden()
    assert len(B.DIRECTIONS) + 1 == named["directions_total"]
    assert len(B.DIRECTIONS) == named["directions_nontrivial"]
    assert len(B.STORED) == named["directions_stored"]
    for k, (terms, paths) in table.items():
        assert sum(1 for d in B.DIRECTIONS if B.hops(d) == k) == terms
        assert math.factorial(k) == paths
    assert sorted(B.slot(d) for d in B.STORED) == list(range(40))
    for d in B.DIRECTIONS:
        neg = tuple(-c for c in d)
        assert B.code(d) + B.code(neg) == 80
        assert (B.slot(d) is None) != (B.slot(neg) is None)


def test_stencil_point_counts():
    _, named = _golden()
    for mu in range(4):
        pts = {d for d in B.DIRECTIONS if d[mu] != 0}
        assert len(pts) == named["nabla_points"]
    assert len(B.DIRECTIONS) + 1 == named["laplace_points"]


def test_coefficients_and_sum_rules():
    rows = {r[0]: r[1:] for r in read_golden("coefficients.txt")}
    rho = [Fraction(int(v), int(rows["rho"][-1])) for v in rows["rho"][:-1]]
    lam = [Fraction(int(v), int(rows["lambda"][-1])) for v in rows["lambda"][:-1]]
    for k in range(1, 5):
        assert abs(B.RHO[k] - float(rho[k - 1])) < 1e-16
    for k in range(5):
        assert abs(B.LAMBDA[k] - float(lam[k])) < 1e-16
    # derivative normalised (nabla(p) -> i p), Laplacian annihilates constants
    assert rho[0] + 6 * rho[1] + 12 * rho[2] + 8 * rho[3] == Fraction(1, 2)
    assert lam[0] + 8 * lam[1] + 24 * lam[2] + 32 * lam[3] + 16 * lam[4] == 0


def test_w_unit_links():
    u = synthetic.gauge_links(DIMS, "unit", 0)
    w = B.build(u)
    assert np.abs(w - np.eye(3)).max() < 1e-15


def test_w_constant_u1_links():
    theta = np.array([0.3, -0.8, 1.2, 0.45])
    u = synthetic.gauge_links(DIMS, "unit", 0) * np.exp(1j * theta)[None, None, None, None, :, None, None]
    w = B.build(u)
    for d in B.STORED:
        phase = np.exp(1j * np.dot(theta, d))
        assert np.abs(w[..., B.slot(d), :, :] - phase * np.eye(3)).max() < 1e-14


def test_w_special_unitary_only_on_axis():
    _, named = _golden()
    u = synthetic.gauge_links(DIMS, "haar", 1)
    w = B.build(u)
    not_su3 = 0
    for d in B.STORED:
        ws = w[..., B.slot(d), :, :]
        unit_err = np.abs(ws @ dag(ws) - np.eye(3)).max()
        if B.hops(d) == 1:
            assert unit_err < 1e-13
            assert np.abs(np.linalg.det(ws) - 1).max() < 1e-13
        else:
            assert unit_err > 1e-2
            not_su3 += 1
    assert not_su3 == named["stored_not_special_unitary"]


def test_w_reverse_relation():
    # W_{-d}(x) = W_d(x - d)^dag, each side built from its own paths
    u = synthetic.gauge_links(DIMS, "haar", 2)
    w_all = B.build_all(u)
    for d in B.DIRECTIONS:
        neg = tuple(-c for c in d)
        rhs = dag(lattice.shift_by(w_all[d], neg))
        assert np.abs(w_all[neg] - rhs).max() < 1e-13
    w40 = B.pack(w_all)
    for d in B.DIRECTIONS:
        assert np.abs(B.link(w40, d) - w_all[d]).max() < 1e-13


def test_w_gauge_covariance():
    u = synthetic.gauge_links(DIMS, "haar", 3)
    g = random_gauge(DIMS, 4)
    ug = np.empty_like(u)
    for mu in range(4):
        ug[..., mu, :, :] = g @ u[..., mu, :, :] @ dag(lattice.shift(g, mu, 1))
    w = B.build(u)
    wg = B.build(ug)
    for d in B.STORED:
        s = B.slot(d)
        expect = g @ w[..., s, :, :] @ dag(lattice.shift_by(g, d))
        assert np.abs(wg[..., s, :, :] - expect).max() < 1e-13


def test_w_two_hop_by_hand():
    # Tab. 1 row 2 written out for d = +x - t at one site
    u = synthetic.gauge_links(DIMS, "haar", 5)
    w = B.build(u)
    nx, ny, nz, nt = DIMS
    x, y, z, t = 2, 1, 0, 0
    V = lambda c, mu: u[c[3] % nt, c[2] % nz, c[1] % ny, c[0] % nx, mu]
    p1 = V((x, y, z, t), 0) @ dag(V((x + 1, y, z, t - 1), 3))
    p2 = dag(V((x, y, z, t - 1), 3)) @ V((x, y, z, t - 1), 0)
    d = (1, 0, 0, -1)
    s = B.slot(tuple(-c for c in d))
    # d is not stored (highest non-zero entry is -1): use the relation
    got = B.link(w, d)[t, z, y, x]
    assert s is not None
    assert np.abs(got - 0.5 * (p1 + p2)).max() < 1e-14


def _nabla_symbol(p, mu):
    return 1j * np.sin(p[mu]) * np.prod([(2 + np.cos(p[nu])) / 3 for nu in range(4) if nu != mu])


def _lap_symbol(p):
    return 4 * (np.prod(np.cos(p / 2) ** 2) - 1)


@pytest.mark.parametrize("n", [(0, 0, 0, 0), (1, 2, 1, 3), (2, 1, 0, 4), (1, 3, 2, 1)])
def test_free_field_closed_form(n):
    wave, p = plane_wave(DIMS, n)
    u = synthetic.gauge_links(DIMS, "unit", 0)
    w = B.build(u)
    col = np.array([1.0, 0.5j, -0.25])
    s = np.array([0.7, -1j, 0.1, 1.0])
    psi = wave[..., None, None, None] * np.einsum("s,c->sc", s, col)[..., None]
    # derivative and Laplacian separately
    for mu in range(4):
        got = B.nabla_iso(w, psi, mu)
        assert np.abs(got - _nabla_symbol(p, mu) * psi).max() < 1e-14
    assert np.abs(B.laplace_bri(w, psi) - _lap_symbol(p) * psi).max() < 1e-14
    m0 = 0.1
    symbol = (m0 - 0.5 * _lap_symbol(p)) * np.eye(4) + sum(GAMMA[mu] * _nabla_symbol(p, mu) for mu in range(4))
    expect = wave[..., None, None, None] * np.einsum("s,c->sc", symbol @ s, col)[..., None]
    assert np.abs(B.apply(w, psi, m0) - expect).max() < 1e-13


def test_doublers_heavy():
    # at any corner p in {0, pi}^4 other than 0 the free operator is m0 + 2 (no doublers)
    for corner in itertools.product((0, np.pi), repeat=4):
        p = np.array(corner)
        if not p.any():
            continue
        assert abs(_lap_symbol(p) + 4) < 1e-15
        for mu in range(4):
            assert abs(_nabla_symbol(p, mu)) < 1e-15


def test_literal_matches_hop_form():
    u = synthetic.gauge_links(DIMS, "haar", 6)
    w = B.build(u)
    psi = synthetic.wilson_spinor(DIMS, 2, 7)
    for adj in (False, True):
        a = B.apply(w, psi, 0.1, adjoint=adj)
        b = B.apply_hop(w, psi, 0.1, adjoint=adj)
        assert np.abs(a - b).max() < 1e-13


def test_gamma5_hermiticity():
    u = synthetic.gauge_links(DIMS, "haar", 8)
    w = B.build(u)
    chi = synthetic.wilson_spinor(DIMS, 2, 9)
    psi = synthetic.wilson_spinor(DIMS, 2, 10)
    lhs = np.vdot(chi, B.apply(w, psi, 0.1))
    rhs = np.vdot(spin_mul(GAMMA5, B.apply(w, spin_mul(GAMMA5, chi), 0.1)), psi)
    assert abs(lhs - rhs) < 1e-12 * abs(lhs)
    rhs2 = np.vdot(B.apply(w, chi, 0.1, adjoint=True), psi)
    assert abs(lhs - rhs2) < 1e-12 * abs(lhs)


def test_gauge_covariance():
    u = synthetic.gauge_links(DIMS, "haar", 11)
    g = random_gauge(DIMS, 12)
    ug = np.empty_like(u)
    for mu in range(4):
        ug[..., mu, :, :] = g @ u[..., mu, :, :] @ dag(lattice.shift(g, mu, 1))
    psi = synthetic.wilson_spinor(DIMS, 2, 13)
    lhs = B.apply(B.build(ug), g[..., None, :, :] @ psi, 0.1)
    rhs = g[..., None, :, :] @ B.apply(B.build(u), psi, 0.1)
    assert np.abs(lhs - rhs).max() < 1e-13


def test_dense_matches_apply():
    dims = (3, 2, 3, 2)
    u = synthetic.gauge_links(dims, "haar", 14)
    psi = synthetic.wilson_spinor(dims, 2, 15)
    D = dense.brillouin(u, 0.1)
    ref = (D @ psi.reshape(-1, 2)).reshape(psi.shape)
    assert np.abs(B.apply(B.build(u), psi, 0.1) - ref).max() < 1e-13
