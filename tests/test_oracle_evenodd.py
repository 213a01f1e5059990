"""Pins of the even-odd (Schur complement) oracle against the brute-force
dense Wilson matrix and the full-lattice operator."""
import numpy as np
import pytest

import synthetic
from oracle import dense, evenodd, solver, wilson
from oracle.lattice import site_index


DIMS = (4, 2, 2, 4)


def _fields(nv, seed):
    u = synthetic.gauge_links(DIMS, "haar", seed)
    p = synthetic.wilson_spinor(DIMS, nv, seed + 1)
    return u, p


def test_pack_unpack_roundtrip_and_parity():
    f = synthetic.wilson_spinor(DIMS, 3, 5)
    assert np.array_equal(evenodd.unpack(evenodd.pack(f, 0), evenodd.pack(f, 1)), f)
    par = evenodd.parity(DIMS)
    for p in (0, 1):
        assert np.all(evenodd.pack(par, p) == p)


def test_odd_extent_rejected():
    f = synthetic.wilson_spinor((3, 2, 2, 2), 1, 5)
    with pytest.raises(ValueError):
        evenodd.pack(f, 0)


def _parity_indices(nc=3):
    # dense row index (site * 4 + spin) * Nc + colour, split by site parity
    nx, ny, nz, nt = DIMS
    ev, od = [], []
    for t in range(nt):
        for z in range(nz):
            for y in range(ny):
                for x in range(nx):
                    s = site_index((x, y, z, t), DIMS)
                    rows = [(s * 4 + sp) * nc + c for sp in range(4) for c in range(nc)]
                    (ev if (x + y + z + t) % 2 == 0 else od).extend(rows)
    return np.array(ev), np.array(od)


def test_dense_diagonal_blocks_are_multiples_of_identity():
    # every hop connects opposite parities: D_ee = D_oo = (4 + m0) 1
    u, _ = _fields(1, 11)
    m0 = 0.3
    D = dense.wilson(u, m0)
    ev, od = _parity_indices()
    assert np.allclose(D[np.ix_(ev, ev)], (4 + m0) * np.eye(len(ev)), atol=1e-13)
    assert np.allclose(D[np.ix_(od, od)], (4 + m0) * np.eye(len(od)), atol=1e-13)


def test_schur_matches_dense_schur_complement():
    nv, m0 = 2, 0.1
    u, p = _fields(nv, 21)
    D = dense.wilson(u, m0)
    ev, od = _parity_indices()
    S = D[np.ix_(ev, ev)] - D[np.ix_(ev, od)] @ np.linalg.solve(D[np.ix_(od, od)], D[np.ix_(od, ev)])
    xe = evenodd.pack(p, 0)
    full = evenodd.unpack(xe, np.zeros_like(xe)).reshape(-1, nv)
    ref_full = np.zeros_like(full)
    ref_full[ev] = S @ full[ev]
    ref = evenodd.pack(ref_full.reshape(p.shape), 0)
    got = evenodd.schur(u, xe, m0)
    assert np.linalg.norm(got - ref) / np.linalg.norm(ref) < 1e-13


def test_schur_adjoint_identity():
    nv, m0 = 2, 0.2
    u, p = _fields(nv, 31)
    chi = evenodd.pack(synthetic.wilson_spinor(DIMS, nv, 33), 0)
    psi = evenodd.pack(p, 0)
    lhs = solver._dot(chi, evenodd.schur(u, psi, m0))
    rhs = solver._dot(evenodd.schur(u, chi, m0, True), psi)
    assert np.allclose(lhs, rhs, rtol=1e-12, atol=1e-12)


def test_hop_split_reproduces_operator():
    # D psi = A psi + (H_eo psi_o, H_oe psi_e)
    nv, m0 = 2, -0.3
    u, p = _fields(nv, 41)
    pe, po = evenodd.pack(p, 0), evenodd.pack(p, 1)
    got = (4 + m0) * p + evenodd.unpack(evenodd.hop_eo(u, po, 0), evenodd.hop_eo(u, pe, 1))
    ref = wilson.apply(u, p, m0)
    assert np.linalg.norm(got - ref) / np.linalg.norm(ref) < 1e-13


def test_even_odd_solve_matches_dense_solve():
    nv, m0 = 2, 0.05
    u = synthetic.gauge_links(DIMS, "smooth", 51)
    b = synthetic.wilson_spinor(DIMS, nv, 52)
    x, iters = evenodd.solve(u, b, m0, tol=1e-12)
    res = solver.relative_residual(lambda v: wilson.apply(u, v, m0), b, x)
    assert np.all(res < 1e-10)
    ref = np.linalg.solve(dense.wilson(u, m0), b.reshape(-1, nv)).reshape(b.shape)
    assert np.linalg.norm(x - ref) / np.linalg.norm(ref) < 1e-9
