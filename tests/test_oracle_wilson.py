"""Pins for the oracle's D_W (Sec. 4, eq. def_wils at c_SW = 0)."""
import numpy as np
import pytest

import synthetic
from oracle import dense, lattice, wilson
from oracle.gamma import GAMMA, GAMMA5, spin_mul
from tests.helpers import dag, plane_wave, random_gauge

DIMS = (4, 3, 2, 5)


def _unit(dims):
    return synthetic.gauge_links(dims, "unit", 0)


def _free_symbol(p, m0):
    return (m0 + np.sum(1 - np.cos(p))) * np.eye(4) + 1j * sum(GAMMA[mu] * np.sin(p[mu]) for mu in range(4))


@pytest.mark.parametrize("n", [(0, 0, 0, 0), (1, 1, 1, 1), (3, 2, 1, 4), (2, 0, 1, 2)])
def test_free_field_plane_wave(n):
    wave, p = plane_wave(DIMS, n)
    s = np.array([1.0, -0.5j, 0.2, 0.9 + 0.1j])
    c = np.array([0.4, 1j, -1.0])
    psi = wave[..., None, None, None] * np.einsum("s,c->sc", s, c)[..., None]
    m0 = 0.1
    out = wilson.apply(_unit(DIMS), psi, m0)
    expect = wave[..., None, None, None] * np.einsum("s,c->sc", _free_symbol(p, m0) @ s, c)[..., None]
    assert np.abs(out - expect).max() < 1e-13


def test_constant_u1_links():
    theta = np.array([0.5, -0.25, 0.8, 1.3])
    u = _unit(DIMS) * np.exp(1j * theta)[None, None, None, None, :, None, None]
    wave, p = plane_wave(DIMS, (1, 2, 1, 2))
    s = np.array([0.3, 1.0, -1j, 0.5])
    psi = wave[..., None, None, None] * np.einsum("s,c->sc", s, np.ones(3))[..., None]
    out = wilson.apply(u, psi, 0.0)
    expect = wave[..., None, None, None] * np.einsum("s,c->sc", _free_symbol(p + theta, 0.0) @ s, np.ones(3))[..., None]
    assert np.abs(out - expect).max() < 1e-13


def test_literal_matches_hop_form():
    u = synthetic.gauge_links(DIMS, "haar", 1)
    psi = synthetic.wilson_spinor(DIMS, 3, 2)
    for adj in (False, True):
        a = wilson.apply(u, psi, 0.3, adjoint=adj)
        b = wilson.apply_hop(u, psi, 0.3, adjoint=adj)
        assert np.abs(a - b).max() < 1e-13


def test_gamma5_hermiticity_general_links():
    # holds for arbitrary complex links, not only unitary ones
    shape = synthetic.lattice_shape(DIMS) + (4, 3, 3)
    u = synthetic.gaussian(shape, 3)
    chi = synthetic.wilson_spinor(DIMS, 2, 4)
    psi = synthetic.wilson_spinor(DIMS, 2, 5)
    lhs = np.vdot(chi, wilson.apply(u, psi, 0.1))
    rhs = np.vdot(spin_mul(GAMMA5, wilson.apply(u, spin_mul(GAMMA5, chi), 0.1)), psi)
    assert abs(lhs - rhs) < 1e-12 * abs(lhs)
    rhs2 = np.vdot(wilson.apply(u, chi, 0.1, adjoint=True), psi)
    assert abs(lhs - rhs2) < 1e-12 * abs(lhs)


def test_gauge_covariance():
    u = synthetic.gauge_links(DIMS, "smooth", 6)
    g = random_gauge(DIMS, 7)
    psi = synthetic.wilson_spinor(DIMS, 2, 8)
    ug = np.empty_like(u)
    for mu in range(4):
        ug[..., mu, :, :] = g @ u[..., mu, :, :] @ dag(lattice.shift(g, mu, 1))
    lhs = wilson.apply(ug, g[..., None, :, :] @ psi, 0.1)
    rhs = g[..., None, :, :] @ wilson.apply(u, psi, 0.1)
    assert np.abs(lhs - rhs).max() < 1e-13


def test_dense_matches_apply():
    dims = (4, 2, 2, 3)
    u = synthetic.gauge_links(dims, "haar", 9)
    psi = synthetic.wilson_spinor(dims, 2, 10)
    D = dense.wilson(u, 0.1)
    ref = (D @ psi.reshape(-1, 2)).reshape(psi.shape)
    assert np.abs(wilson.apply(u, psi, 0.1) - ref).max() < 1e-13


def test_dense_free_spectrum():
    dims = (4, 2, 2, 3)
    m0 = 0.1
    ev = np.linalg.eigvals(dense.wilson(_unit(dims), m0))
    ps = [2 * np.pi * np.arange(n) / n for n in dims]
    expect = []
    for p in np.stack(np.meshgrid(*ps, indexing="ij"), -1).reshape(-1, 4):
        re = m0 + np.sum(1 - np.cos(p))
        im = np.sqrt(np.sum(np.sin(p) ** 2))
        expect += [re + 1j * im] * 6 + [re - 1j * im] * 6   # multiplicity 2 N_c each
    key = lambda z: (np.round(z.real, 9), np.round(z.imag, 9))
    assert np.allclose(sorted(ev, key=key), sorted(expect, key=key), atol=1e-10)
