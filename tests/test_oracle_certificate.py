"""The slab-wise residual certificate of the solver tests, against the
whole-lattice oracle: the per-slab squared norms must add up to the residual
of the literal D_W (eq. def_wils) over the full lattice, every slice must be
covered (a perturbation of x on any one slice shows up), and the exact
solution from the dense matrix must certify to rounding level."""
import numpy as np
import pytest

import synthetic
from oracle import dense, solver, wilson
from tests import residual_certificate as rc


def _fields(dims, nv, seed):
    u = synthetic.gauge_links(dims, "smooth", seed)
    b = synthetic.wilson_spinor(dims, nv, seed + 1)
    x = synthetic.wilson_spinor(dims, nv, seed + 2)
    return u, b, x


@pytest.mark.parametrize("dims,cuts", [((4, 3, 2, 7), (0, 2, 3, 7)), ((3, 2, 2, 2), (0, 1, 2)),
                                       ((2, 3, 2, 5), (0, 5))])
def test_slabs_add_up_to_the_full_residual(dims, cuts):
    nv, m0 = 3, 0.05
    u, b, x = _fields(dims, nv, 1)
    full = solver.relative_residual(lambda v: wilson.apply(u, v, m0), b, x)
    rr = bb = 0.0
    for t0, t1 in zip(cuts[:-1], cuts[1:]):
        a, c = solver.wilson_residual_slab(u, b, x, m0, t0, t1)
        rr, bb = rr + a, bb + c
    assert np.allclose(np.sqrt(rr / bb), full, rtol=1e-13)


def test_slab_bounds_are_checked():
    u, b, x = _fields((2, 2, 2, 4), 1, 2)
    with pytest.raises(ValueError):
        solver.wilson_residual_slab(u, b, x, 0.1, 2, 2)
    with pytest.raises(ValueError):
        solver.wilson_residual_slab(u, b, x, 0.1, 0, 5)


def test_slab_partition_covers_every_slice():
    for nt, parts in ((64, 16), (7, 3), (5, 16), (1, 4)):
        s = rc.slabs(nt, parts)
        assert s[0][0] == 0 and s[-1][1] == nt
        assert all(a < b for a, b in s)
        assert all(s[k][1] == s[k + 1][0] for k in range(len(s) - 1))


def test_worker_processes_certify_the_dense_solution(tmp_path):
    # exact solution of D_W x = b from the dense matrix: residual at rounding
    # level; a change of x at one site of the last slice is seen
    dims, nv, m0 = (2, 2, 2, 5), 2, 0.05
    u, b, _ = _fields(dims, nv, 3)
    x = np.linalg.solve(dense.wilson(u, m0), b.reshape(-1, nv)).reshape(b.shape)
    paths = {}
    for name, arr in (("u", u), ("b", b), ("x", x)):
        paths[name] = str(tmp_path / f"{name}.npy")
        np.save(paths[name], arr)
    res = rc.certify(paths["u"], paths["b"], paths["x"], m0, workers=3)
    assert np.all(res < 1e-13)
    x[-1, 1, 0, 1, 2, 1, 1] += 1e-6
    np.save(paths["x"], x)
    res = rc.certify(paths["u"], paths["b"], paths["x"], m0, workers=3)
    ref = solver.relative_residual(lambda v: wilson.apply(u, v, m0), b, x)
    assert res[1] > 1e-8 and res[0] < 1e-13
    assert np.allclose(res, ref, rtol=1e-6)
