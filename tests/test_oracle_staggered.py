"""Pins for the oracle's D_S (Sec. 3): closed forms, invariants, brute force."""
import numpy as np
import pytest

import synthetic
from oracle import dense, lattice, staggered
from tests.helpers import coords, dag, plane_wave, random_gauge

DIMS = (4, 6, 2, 8)   # anisotropic and even, so axis mix-ups show


def _unit_links(dims):
    return synthetic.gauge_links(dims, "unit", 0)


@pytest.mark.parametrize("n", [(0, 0, 0, 0), (1, 2, 1, 3), (3, 5, 1, 7), (2, 3, 0, 1)])
def test_free_field_plane_wave(n):
    # U = 1: D_S (e^{ipx} c) = (m + i sum_mu eta_mu(x) sin p_mu) e^{ipx} c, pointwise
    wave, p = plane_wave(DIMS, n)
    col = np.array([0.3 - 0.2j, 1.1, -0.7j])
    psi = wave[..., None, None] * col[:, None]
    m = 0.37
    out = staggered.apply(_unit_links(DIMS), psi, m)
    et = lattice.eta(DIMS)
    factor = m + 1j * sum(et[mu] * np.sin(p[mu]) for mu in range(4))
    assert np.abs(out - factor[..., None, None] * psi).max() < 1e-13


def test_free_field_square():
    # massless, U = 1: D_S^2 e^{ipx} = -sum sin^2 p e^{ipx}
    wave, p = plane_wave(DIMS, (1, 1, 1, 3))
    psi = wave[..., None, None] * np.ones((3, 2))
    u = _unit_links(DIMS)
    out = staggered.apply(u, staggered.apply(u, psi))
    assert np.abs(out + np.sum(np.sin(p) ** 2) * psi).max() < 1e-13


def test_constant_u1_links_shift_momentum():
    theta = np.array([0.3, -0.7, 1.1, 0.2])
    u = _unit_links(DIMS) * np.exp(1j * theta)[None, None, None, None, :, None, None]
    wave, p = plane_wave(DIMS, (1, 2, 1, 1))
    psi = wave[..., None, None] * np.array([1.0, 2.0, -1j])[:, None]
    out = staggered.apply(u, psi)
    et = lattice.eta(DIMS)
    factor = 1j * sum(et[mu] * np.sin(p[mu] + theta[mu]) for mu in range(4))
    assert np.abs(out - factor[..., None, None] * psi).max() < 1e-13


def test_anti_hermitian_massless():
    u = synthetic.gauge_links(DIMS, "haar", 1)
    chi = synthetic.staggered_spinor(DIMS, 3, 2)
    psi = synthetic.staggered_spinor(DIMS, 3, 3)
    a = np.vdot(chi, staggered.apply(u, psi))
    b = np.vdot(staggered.apply(u, chi), psi)
    assert abs(a + b) < 1e-12 * abs(a)


def test_adjoint_with_mass():
    u = synthetic.gauge_links(DIMS, "haar", 1)
    chi = synthetic.staggered_spinor(DIMS, 2, 2)
    psi = synthetic.staggered_spinor(DIMS, 2, 3)
    a = np.vdot(chi, staggered.apply(u, psi, 0.4))
    b = np.vdot(staggered.apply(u, chi, 0.4, adjoint=True), psi)
    assert abs(a - b) < 1e-12 * abs(a)


def test_epsilon_anticommutes():
    u = synthetic.gauge_links(DIMS, "haar", 4)
    psi = synthetic.staggered_spinor(DIMS, 2, 5)
    c = coords(DIMS)
    eps = ((-1.0) ** c.sum(axis=0))[..., None, None]
    lhs = eps * staggered.apply(u, eps * psi)
    assert np.abs(lhs + staggered.apply(u, psi)).max() < 1e-13


def test_gauge_covariance():
    u = synthetic.gauge_links(DIMS, "haar", 6)
    g = random_gauge(DIMS, 7)
    psi = synthetic.staggered_spinor(DIMS, 2, 8)
    ug = np.empty_like(u)
    for mu in range(4):
        ug[..., mu, :, :] = g @ u[..., mu, :, :] @ dag(lattice.shift(g, mu, 1))
    lhs = staggered.apply(ug, g @ psi, 0.2)
    rhs = g @ staggered.apply(u, psi, 0.2)
    assert np.abs(lhs - rhs).max() < 1e-13


def test_dense_matches_apply():
    dims = (4, 2, 4, 2)
    u = synthetic.gauge_links(dims, "haar", 9)
    psi = synthetic.staggered_spinor(dims, 3, 10)
    D = dense.staggered(u, 0.15)
    ref = (D @ psi.reshape(-1, 3)).reshape(psi.shape)
    assert np.abs(staggered.apply(u, psi, 0.15) - ref).max() < 1e-13


def test_dense_free_spectrum():
    dims = (4, 2, 4, 2)
    D = dense.staggered(_unit_links(dims), 0.0)
    ev = np.linalg.eigvals(D)
    assert np.abs(ev.real).max() < 1e-12
    ps = [2 * np.pi * np.arange(n) / n for n in dims]
    grid = np.meshgrid(*ps, indexing="ij")
    s = sum(np.sin(q) ** 2 for q in grid).ravel()
    expect = np.sort(np.repeat(s, 3))
    assert np.allclose(np.sort(np.abs(ev) ** 2), expect, atol=1e-12)
    # +- symmetric spectrum
    assert np.allclose(np.sort(ev.imag), np.sort(-ev.imag), atol=1e-12)
