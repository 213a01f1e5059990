"""Pins for the oracle's gamma basis, geometry and the seeded generators."""
import numpy as np
import pytest

import synthetic
from oracle import gamma, lattice
from tests.helpers import coords


def test_clifford_algebra():
    g = gamma.GAMMA
    for mu in range(4):
        assert np.allclose(g[mu], g[mu].conj().T)
        for nu in range(4):
            anti = g[mu] @ g[nu] + g[nu] @ g[mu]
            assert np.allclose(anti, 2.0 * (mu == nu) * np.eye(4), atol=1e-15)


def test_gamma5_chiral():
    g5 = gamma.GAMMA5
    assert np.allclose(g5, np.diag([1, 1, -1, -1]))
    for mu in range(4):
        assert np.allclose(g5 @ gamma.GAMMA[mu], -gamma.GAMMA[mu] @ g5)


def test_projectors_rank_two():
    for mu in range(4):
        for s in (+1, -1):
            p = np.eye(4) + s * gamma.GAMMA[mu]
            assert np.linalg.matrix_rank(p) == 2
            assert np.allclose(p @ p, 2 * p)


def test_eta_phases():
    dims = (4, 6, 2, 8)
    et = lattice.eta(dims)
    c = coords(dims)
    # eta_1 = 1, eta_2 = (-1)^x, eta_3 = (-1)^(x+y), eta_4 = (-1)^(x+y+z) at 0-based x
    assert np.all(et[0] == 1)
    assert np.all(et[1] == (-1.0) ** c[0])
    assert np.all(et[2] == (-1.0) ** (c[0] + c[1]))
    assert np.all(et[3] == (-1.0) ** (c[0] + c[1] + c[2]))
    # eta_mu does not depend on x_mu (needed for the backward hop)
    for mu in range(4):
        assert np.array_equal(et[mu], lattice.shift(et[mu], mu, 1))


def test_shift_direction_and_axes():
    dims = (3, 4, 5, 6)
    c = coords(dims)
    for mu in range(4):
        s = lattice.shift(c[mu], mu, +1)
        assert np.array_equal(s, (c[mu] + 1) % dims[mu])
        for nu in range(4):
            if nu != mu:
                assert np.array_equal(lattice.shift(c[nu], mu, 1), c[nu])


def test_site_index_roundtrip():
    dims = (3, 4, 5, 2)
    for s in range(np.prod(dims)):
        assert lattice.site_index(lattice.site_coord(s, dims), dims) == s


@pytest.mark.parametrize("kind", ["haar", "smooth"])
def test_links_special_unitary(kind):
    u = synthetic.gauge_links((4, 2, 2, 6), kind, 7)
    eye = np.einsum("...ab,...cb->...ac", u, u.conj())
    assert np.abs(eye - np.eye(3)).max() < 1e-13
    assert np.abs(np.linalg.det(u) - 1).max() < 1e-13


def test_haar_moments():
    # For Haar SU(3): E[tr U] = 0 and E[|tr U|^2] = 1
    u = synthetic.haar_su3(200000, 3)
    tr = np.trace(u, axis1=1, axis2=2)
    assert abs(tr.mean()) < 0.01
    assert abs(np.mean(np.abs(tr) ** 2) - 1.0) < 0.02


def test_smooth_links_near_identity():
    u = synthetic.gauge_links((4, 4, 4, 4), "smooth", 1)
    dist = np.abs(np.trace(u, axis1=-2, axis2=-1).real / 3 - 1).mean()
    assert 0.0 < dist < 0.1


def test_gaussian_moments():
    z = synthetic.gaussian((400000,), 5)
    assert abs(np.mean(np.abs(z) ** 2) - 1) < 0.01
    assert abs(np.mean(z.real ** 2) - 0.5) < 0.01
    assert abs(z.mean()) < 0.01


def test_generators_deterministic():
    a = synthetic.wilson_spinor((2, 2, 2, 2), 3, 11)
    b = synthetic.wilson_spinor((2, 2, 2, 2), 3, 11)
    assert np.array_equal(a, b)
    assert a.shape == (2, 2, 2, 2, 4, 3, 3)
