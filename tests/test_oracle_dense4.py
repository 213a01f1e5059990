"""Brute-force dense matrices on a 4^4 lattice (dimension 768 for D_S, 3072
for D_W and D_B).  With every extent 4 the +mu and -mu hops of a site, and the
80 Brillouin displacements, land on distinct sites, so each term of the
definitions has its own matrix block.  The matrices are filled entry block by
entry block from the delta-function forms (``oracle.dense``, explicit
coordinate loops) and checked against

* the shift-based operators of the oracle (Sec. 3 D_S equation; Sec. 4 eq.
  def_wils; Sec. 5 eqs. def_bril, def_der, def_lap with the W of Tab. 1) on
  Haar-random links;
* the closed-form free-field (U = 1) spectra:
    D_S (m = 0):  +- i sqrt(sum_mu sin^2 p_mu)
    D_W:          m0 + sum_mu (1 - cos p_mu) +- i sqrt(sum_mu sin^2 p_mu)
    D_B:          m0 + 2 [1 - prod_mu cos^2(p_mu / 2)]
                  +- i sqrt(sum_mu [sin p_mu prod_{nu != mu} (2 + cos p_nu) / 3]^2)
  over the momenta p_mu = 2 pi n_mu / 4, each Wilson-type eigenvalue with
  multiplicity 2 N_c;
* anti-Hermiticity of the massless D_S and gamma_5-hermiticity of D_W and D_B
  as matrix identities."""
import numpy as np
import pytest

import synthetic
from oracle import brillouin as B
from oracle import dense, staggered, wilson
from oracle.gamma import GAMMA5

DIMS = (4, 4, 4, 4)
NC = 3


def _unit_links(dims):
    nx, ny, nz, nt = dims
    return np.broadcast_to(np.eye(NC, dtype=np.complex128), (nt, nz, ny, nx, 4, NC, NC)).copy()


def _momenta(dims):
    ps = [2 * np.pi * np.arange(n) / n for n in dims]
    return np.stack(np.meshgrid(*ps, indexing="ij"), -1).reshape(-1, 4)


def _sorted(z):
    return sorted(z, key=lambda w: (np.round(w.real, 8), np.round(w.imag, 8)))


def _gamma5_full(n_sites):
    return np.kron(np.eye(n_sites), np.kron(GAMMA5, np.eye(NC)))


@pytest.fixture(scope="module")
def haar():
    return synthetic.gauge_links(DIMS, "haar", 41)


def test_staggered_dense_4to4(haar):
    D = dense.staggered(haar, 0.2)
    psi = synthetic.staggered_spinor(DIMS, 3, 42)
    ref = (D @ psi.reshape(-1, 3)).reshape(psi.shape)
    assert np.abs(staggered.apply(haar, psi, 0.2) - ref).max() < 1e-13
    D0 = dense.staggered(haar, 0.0)
    assert np.abs(D0 + D0.conj().T).max() < 1e-14            # anti-Hermitian at m = 0
    ev = np.linalg.eigvals(dense.staggered(_unit_links(DIMS), 0.0))
    s = np.array([np.sum(np.sin(p) ** 2) for p in _momenta(DIMS)])
    assert np.abs(ev.real).max() < 1e-12
    assert np.allclose(np.sort(np.abs(ev) ** 2), np.sort(np.repeat(s, NC)), atol=1e-12)
    assert np.allclose(np.sort(ev.imag), np.sort(-ev.imag), atol=1e-12)


def test_wilson_dense_4to4(haar):
    m0 = 0.1
    D = dense.wilson(haar, m0)
    psi = synthetic.wilson_spinor(DIMS, 3, 43)
    ref = (D @ psi.reshape(-1, 3)).reshape(psi.shape)
    assert np.abs(wilson.apply(haar, psi, m0) - ref).max() < 1e-13
    g5 = _gamma5_full(int(np.prod(DIMS)))
    assert np.abs(g5 @ D @ g5 - D.conj().T).max() < 1e-14      # gamma_5-hermiticity
    ev = np.linalg.eigvals(dense.wilson(_unit_links(DIMS), m0))
    expect = []
    for p in _momenta(DIMS):
        re = m0 + np.sum(1 - np.cos(p))
        im = np.sqrt(np.sum(np.sin(p) ** 2))
        expect += [re + 1j * im] * (2 * NC) + [re - 1j * im] * (2 * NC)
    assert np.allclose(_sorted(ev), _sorted(expect), atol=1e-10)


def test_brillouin_dense_4to4(haar):
    m0 = 0.1
    D = dense.brillouin(haar, m0)
    psi = synthetic.wilson_spinor(DIMS, 2, 44)
    ref = (D @ psi.reshape(-1, 2)).reshape(psi.shape)
    assert np.abs(B.apply(B.build(haar), psi, m0) - ref).max() < 1e-13
    g5 = _gamma5_full(int(np.prod(DIMS)))
    assert np.abs(g5 @ D @ g5 - D.conj().T).max() < 1e-14
    ev = np.linalg.eigvals(dense.brillouin(_unit_links(DIMS), m0))
    expect = []
    for p in _momenta(DIMS):
        re = m0 + 2 * (1 - np.prod(np.cos(p / 2) ** 2))
        der = [np.sin(p[mu]) * np.prod([(2 + np.cos(p[nu])) / 3 for nu in range(4) if nu != mu])
               for mu in range(4)]
        im = np.sqrt(np.sum(np.square(der)))
        expect += [re + 1j * im] * (2 * NC) + [re - 1j * im] * (2 * NC)
    assert np.allclose(_sorted(ev), _sorted(expect), atol=1e-10)
    # the 81-point stencil: every block row has 81 non-zero 12 x 12 blocks
    blocks = np.abs(D[:4 * NC].reshape(4 * NC, -1, 4 * NC)).sum(axis=(0, 2))
    assert np.count_nonzero(blocks > 1e-14) == 81
