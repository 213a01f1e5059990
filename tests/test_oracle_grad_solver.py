"""Pins for the oracle's link gradient, solvers and site-sampled evaluation."""
import numpy as np
import pytest

import synthetic
from oracle import brillouin, dense, grad, local, solver, staggered, wilson
from tests.helpers import rel_l2

DIMS = (4, 2, 2, 4)


def _fields(op, seed):
    u = synthetic.gauge_links(DIMS, "haar", seed)
    if op == "staggered":
        return u, synthetic.staggered_spinor(DIMS, 2, seed + 1), synthetic.staggered_spinor(DIMS, 2, seed + 2)
    return u, synthetic.wilson_spinor(DIMS, 2, seed + 1), synthetic.wilson_spinor(DIMS, 2, seed + 2)


@pytest.mark.parametrize("op", ["staggered", "wilson"])
def test_link_grad_exact_central_difference(op):
    u, chi, psi = _fields(op, 20)
    G = grad.link_grad(op, chi, psi)
    g = np.random.Generator(np.random.PCG64(3))
    links = [(int(g.integers(DIMS[3])), int(g.integers(DIMS[2])), int(g.integers(DIMS[1])),
              int(g.integers(DIMS[0])), int(g.integers(4)), int(g.integers(3)), int(g.integers(3)))
             for _ in range(12)]
    for h in (1.0, 0.25):
        fd = grad.fd_link_grad(op, u, chi, psi, links, mass=0.3, h=h)
        an = np.array([G[l] for l in links])
        assert np.abs(fd - an).max() < 1e-12 * np.abs(an).max()


@pytest.mark.parametrize("op", ["staggered", "wilson"])
def test_link_grad_directional(op):
    # L(V + D) - L(V - D) = 2 Re <G, D> for any direction D (L affine per link)
    u, chi, psi = _fields(op, 30)
    G = grad.link_grad(op, chi, psi)
    delta = synthetic.gaussian(u.shape, 31) * 0.1
    lhs = grad.loss(op, u + delta, chi, psi) - grad.loss(op, u - delta, chi, psi)
    # L is linear in the links (each hop is linear in one link), so the
    # difference over a global perturbation is exact as well
    rhs = 2 * np.real(np.vdot(G, delta))
    assert abs(lhs - rhs) < 1e-11 * abs(rhs)


def test_cg_matches_dense_solve():
    g = np.random.Generator(np.random.PCG64(1))
    n = 40
    a = g.standard_normal((n, n)) + 1j * g.standard_normal((n, n))
    A = a.conj().T @ a + 0.5 * np.eye(n)
    b = g.standard_normal((n, 3)) + 1j * g.standard_normal((n, 3))
    x, it, rr = solver.cg(lambda v: A @ v, b, tol=1e-13, maxiter=500)
    assert np.all(rr <= 1e-13)
    assert rel_l2(x, np.linalg.solve(A, b)) < 1e-10


def test_cgnr_wilson_matches_dense():
    dims = (2, 4, 2, 4)
    u = synthetic.gauge_links(dims, "smooth", 2)
    b = synthetic.wilson_spinor(dims, 2, 3)
    m0 = 0.05
    x, it, _ = solver.cgnr(lambda v: wilson.apply(u, v, m0), lambda v: wilson.apply(u, v, m0, True),
                           b, tol=1e-13, maxiter=5000)
    D = dense.wilson(u, m0)
    ref = np.linalg.solve(D, b.reshape(-1, 2)).reshape(b.shape)
    assert rel_l2(x, ref) < 1e-9
    res = solver.relative_residual(lambda v: wilson.apply(u, v, m0), b, x)
    assert np.all(res < 1e-10)


@pytest.mark.parametrize("adj", [False, True])
def test_local_matches_full(adj):
    dims = (4, 3, 3, 4)
    sites = local.sample_sites(dims, 30, 9)
    idx = (sites[:, 3], sites[:, 2], sites[:, 1], sites[:, 0])
    u = synthetic.gauge_links(dims, "haar", 1)
    ps = synthetic.staggered_spinor(dims, 2, 2)
    assert np.abs(local.staggered_at(u, ps, 0.2, sites, adj) - staggered.apply(u, ps, 0.2, adj)[idx]).max() < 1e-13
    pw = synthetic.wilson_spinor(dims, 2, 3)
    assert np.abs(local.wilson_at(u, pw, 0.1, sites, adj) - wilson.apply(u, pw, 0.1, adj)[idx]).max() < 1e-13
    full = brillouin.apply(brillouin.build(u), pw, 0.1, adj)[idx]
    assert np.abs(local.brillouin_at(u, pw, 0.1, sites, adj) - full).max() < 1e-13


@pytest.mark.parametrize("op", ["staggered", "wilson"])
def test_local_link_grad(op):
    dims = (4, 3, 2, 4)
    sites = local.sample_sites(dims, 10, 4)
    idx = (sites[:, 3], sites[:, 2], sites[:, 1], sites[:, 0])
    if op == "staggered":
        chi, psi = synthetic.staggered_spinor(dims, 2, 1), synthetic.staggered_spinor(dims, 2, 2)
    else:
        chi, psi = synthetic.wilson_spinor(dims, 2, 1), synthetic.wilson_spinor(dims, 2, 2)
    G = grad.link_grad(op, chi, psi)
    for mu in range(4):
        assert np.abs(local.link_grad_at(op, chi, psi, sites, mu) - G[idx][:, mu]).max() < 1e-13


def test_local_brillouin_gradients():
    # the sampled-site forms of the gradient with respect to W and of the
    # adjoint of the W construction equal the whole-lattice oracle there
    dims = (4, 3, 3, 4)
    sites = local.sample_sites(dims, 12, 6)
    idx = (sites[:, 3], sites[:, 2], sites[:, 1], sites[:, 0])
    chi, psi = synthetic.wilson_spinor(dims, 2, 7), synthetic.wilson_spinor(dims, 2, 8)
    gw = grad.link_grad_brillouin_W(chi, psi)
    assert np.abs(local.brillouin_w_grad_at(chi, psi, sites) - gw[idx]).max() < 1e-13
    v = synthetic.gauge_links(dims, "haar", 9)
    gv = grad.brillouin_links_backward(v, gw)
    for mu in range(4):
        assert np.abs(local.brillouin_links_backward_at(v, gw, sites, mu) - gv[idx][:, mu]).max() < 1e-12


@pytest.mark.parametrize("op", ["staggered", "wilson"])
def test_local_fd_matches_full_fd(op):
    u, chi, psi = _fields(op, 40)
    links = [(1, 0, 1, 3, 0, 2, 1), (3, 1, 0, 0, 3, 0, 0), (0, 1, 1, 2, 1, 1, 2), (2, 0, 0, 1, 2, 2, 2)]
    full = grad.fd_link_grad(op, u, chi, psi, links, mass=0.2)
    for n, l in enumerate(links):
        assert abs(local.fd_link_grad_local(op, u, chi, psi, 0.2, l) - full[n]) < 1e-12 * abs(full[n]) + 1e-14
