"""Pins for the oracle's gauge compression (two stored rows per SU(3) link)."""
import numpy as np

import synthetic
from oracle import compress, staggered, wilson

DIMS = (4, 3, 2, 4)


def test_hand_examples():
    # a cyclic permutation matrix (det +1) and a diagonal SU(3) element, completed by hand
    p = np.array([[0, 1, 0], [0, 0, 1], [1, 0, 0]], dtype=complex)
    assert np.array_equal(compress.reconstruct(p[:2]), p)
    al, be = 0.7, -1.9
    d = np.diag([np.exp(1j * al), np.exp(1j * be), np.exp(-1j * (al + be))])
    assert np.abs(compress.reconstruct(d[:2]) - d).max() < 1e-15
    assert np.array_equal(compress.reconstruct(np.eye(3, dtype=complex)[:2]), np.eye(3))


def test_su3_links_round_trip():
    for kind, seed in (("haar", 1), ("smooth", 2)):
        V = synthetic.gauge_links(DIMS, kind, seed)
        Vc = compress.compress(V)
        assert Vc.shape == V.shape[:-2] + (2, 3)
        assert np.abs(compress.reconstruct(Vc) - V).max() < 1e-14


def test_unitary_with_phase_and_non_unitary():
    u = synthetic.haar_su3(20, 3)
    a = np.random.default_rng(4).uniform(-np.pi, np.pi, 20)
    w = u * np.exp(1j * a / 3)[:, None, None]          # det w = e^{i a}
    r = compress.reconstruct(w[:, :2])
    assert np.abs(r[:, :2] - w[:, :2]).max() == 0
    assert np.abs(r[:, 2] - w[:, 2] * np.exp(-1j * a)[:, None]).max() < 1e-14
    # for any two rows the completed third row is orthogonal to both
    m = synthetic.gaussian((20, 2, 3), 5)
    c = compress.reconstruct(m)[:, 2]
    assert np.abs(np.einsum("nj,nj->n", np.conj(m[:, 0]), c)).max() < 1e-13
    assert np.abs(np.einsum("nj,nj->n", np.conj(m[:, 1]), c)).max() < 1e-13


def test_operators_on_compressed_links():
    V = synthetic.gauge_links(DIMS, "haar", 6)
    Vc = compress.compress(V)
    psi = synthetic.wilson_spinor(DIMS, 2, 7)
    chi = synthetic.staggered_spinor(DIMS, 2, 8)
    for adj in (False, True):
        assert np.abs(compress.apply("wilson", Vc, psi, 0.1, adj) - wilson.apply(V, psi, 0.1, adj)).max() < 1e-13
        assert np.abs(compress.apply("staggered", Vc, chi, 0.2, adj)
                      - staggered.apply(V, chi, 0.2, adj)).max() < 1e-13
