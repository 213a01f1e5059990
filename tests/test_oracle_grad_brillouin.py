"""Pins for the oracle's Brillouin link gradients: with respect to the stored W
(L is linear in W, so a central difference is exact) and, through the
construction of W (Tab. 1), with respect to V (L is a polynomial of degree at
most 4 along any line V + t Delta, so a five-point central difference is
exact).  The losses are evaluated with the literal operator (eq. def_bril)
and the path products of Tab. 1, not with the hop form the gradients use."""
import numpy as np

import synthetic
from oracle import brillouin, grad

DIMS = (3, 3, 2, 3)
M0 = 0.1


def _setup(seed):
    v = synthetic.gauge_links(DIMS, "haar", seed)
    chi = synthetic.wilson_spinor(DIMS, 2, seed + 1)
    psi = synthetic.wilson_spinor(DIMS, 2, seed + 2)
    return v, chi, psi


def _loss_v(v, chi, psi):
    return grad.loss("brillouin", brillouin.build(v), chi, psi, M0)


def _five_point(f, h):
    return (f(-2 * h) - 8 * f(-h) + 8 * f(h) - f(2 * h)) / (12 * h)


def test_gradient_wrt_W_directional():
    v, chi, psi = _setup(30)
    W = brillouin.build(v)
    G = grad.link_grad_brillouin_W(chi, psi)
    delta = synthetic.gaussian(W.shape, 33)
    h = 0.5
    fd = (grad.loss("brillouin", W + h * delta, chi, psi, M0) - grad.loss("brillouin", W - h * delta, chi, psi, M0)) / (2 * h)
    exact = float(np.real(np.vdot(G, delta)))
    assert abs(fd - exact) < 1e-11 * (abs(exact) + 1)


def test_gradient_wrt_V_directional():
    v, chi, psi = _setup(40)
    G = grad.link_grad_brillouin(v, chi, psi)
    delta = synthetic.gaussian(v.shape, 43)
    fd = _five_point(lambda t: _loss_v(v + t * delta, chi, psi), 0.25)
    exact = float(np.real(np.vdot(G, delta)))
    assert abs(fd - exact) < 1e-9 * (abs(exact) + 1)


def test_gradient_wrt_V_single_entries():
    v, chi, psi = _setup(50)
    G = grad.link_grad_brillouin(v, chi, psi)
    for idx in [(0, 0, 0, 0, 0, 0, 1), (2, 1, 2, 1, 3, 2, 2), (1, 0, 1, 2, 1, 1, 0)]:
        parts = []
        for step in (1.0, 1j):
            def f(t, step=step):
                w = v.copy()
                w[idx] += t * step
                return _loss_v(w, chi, psi)
            parts.append(_five_point(f, 0.5))
        assert abs(parts[0] + 1j * parts[1] - G[idx]) < 1e-9 * (abs(G[idx]) + 1)


def test_links_backward_is_adjoint_of_the_construction():
    # d/dt Re<G_W, W[V + t Delta]> at t = 0 equals Re<links_backward(V, G_W), Delta>
    v, _, _ = _setup(60)
    gw = synthetic.gaussian(v.shape[:4] + (40, 3, 3), 61)
    delta = synthetic.gaussian(v.shape, 62)
    gv = grad.brillouin_links_backward(v, gw)
    fd = _five_point(lambda t: float(np.real(np.vdot(gw, brillouin.build(v + t * delta)))), 0.3)
    exact = float(np.real(np.vdot(gv, delta)))
    assert abs(fd - exact) < 1e-9 * (abs(exact) + 1)
