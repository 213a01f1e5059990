"""Mixed-precision solver: the residual of the returned x is recomputed by the
oracle (several x meet a tolerance, so residuals, not solutions, are compared;
on a lattice small enough for a dense solve the solution is also checked)."""
import numpy as np
import pytest

import synthetic
from oracle import dense, local, solver, staggered, wilson
from tests.gpu_util import down, say, up

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_1808_05506_amd import dslash as D  # noqa: E402


@pytest.mark.parametrize("inner,itol", [("c64", 1e-5), ("bf16", 0.05), ("f16", 1e-2)])
def test_wilson_solve_small(inner, itol):
    dims, nv, m0 = (4, 4, 4, 4), 3, 0.05
    say(f"case solve wilson {dims} nv={nv} inner={inner}")
    u = synthetic.gauge_links(dims, "smooth", 3)
    b = synthetic.wilson_spinor(dims, nv, 103)
    x, info = D.solve("wilson", up(u, "c128"), up(b, "c128"), m0, inner=inner, tol=1e-10, inner_tol=itol)
    say(f"info {info}")
    assert info["status"] == 0
    xs = down(x)
    res = solver.relative_residual(lambda v: wilson.apply(u, v, m0), b, xs)
    say(f"oracle residuals {res}")
    assert np.all(res <= 1e-10)
    assert np.allclose(info["relres"], res, rtol=1e-3, atol=1e-13)
    ref = np.linalg.solve(dense.wilson(u, m0), b.reshape(-1, nv)).reshape(b.shape)
    assert np.linalg.norm(xs - ref) / np.linalg.norm(ref) < 1e-7


@pytest.mark.parametrize("inner", ["c64", "bf16"])
def test_staggered_solve(inner):
    dims, nv, m = (6, 4, 4, 8), 4, 0.05
    say(f"case solve staggered {dims} nv={nv} inner={inner}")
    u = synthetic.gauge_links(dims, "haar", 6)
    b = synthetic.staggered_spinor(dims, nv, 106)
    x, info = D.solve("staggered", up(u, "c128"), up(b, "c128"), m, inner=inner, tol=1e-10,
                      inner_tol=1e-4 if inner == "c64" else 0.05)
    say(f"info {info}")
    res = solver.relative_residual(lambda v: staggered.apply(u, v, m), b, down(x))
    say(f"oracle residuals {res}")
    assert info["status"] == 0 and np.all(res <= 1e-10)


def test_solve_zero_rhs_column_and_warm_start():
    dims, nv, m0 = (4, 4, 2, 4), 2, 0.1
    u = synthetic.gauge_links(dims, "smooth", 7)
    b = synthetic.wilson_spinor(dims, nv, 107)
    b[..., 1] = 0.0
    say("case solve zero column")
    x, info = D.solve("wilson", up(u, "c128"), up(b, "c128"), m0, inner="c64", tol=1e-10, inner_tol=1e-5)
    xs = down(x)
    assert info["status"] == 0
    assert np.all(xs[..., 1] == 0)
    res = solver.relative_residual(lambda v: wilson.apply(u, v, m0), b[..., :1], xs[..., :1])
    assert res[0] <= 1e-10
    # warm start from the solution: no inner iterations needed
    x2, info2 = D.solve("wilson", up(u, "c128"), up(b, "c128"), m0, inner="c64", tol=1e-10, inner_tol=1e-5, x0=x)
    assert info2["outer_iters"] == 0 and info2["inner_iters"] == 0


def test_solve_iteration_limit_reports_noconv():
    dims, nv, m0 = (4, 4, 4, 4), 1, 0.05
    u = synthetic.gauge_links(dims, "smooth", 8)
    b = synthetic.wilson_spinor(dims, nv, 108)
    say("case solve noconv")
    x, info = D.solve("wilson", up(u, "c128"), up(b, "c128"), m0, inner="bf16", tol=1e-10, inner_tol=0.5,
                      max_outer=1, max_inner=3)
    assert info["status"] == 5
    assert info["relres"][0] > 1e-10


@pytest.mark.parametrize("inner,itol", [("c64", 1e-5), ("bf16", 0.05), ("f16", 5e-3)])
def test_wilson_solve_nv12_row_kernels(inner, itol):
    # N_v = 12 on rows of 12 sites: the inner applies run the row-staged
    # t-marching D_W kernel and the vector updates take their 16-byte forms
    dims, nv, m0 = (12, 4, 2, 4), 12, 0.05
    say(f"case solve wilson {dims} nv={nv} inner={inner}")
    u = synthetic.gauge_links(dims, "smooth", 9)
    b = synthetic.wilson_spinor(dims, nv, 109)
    x, info = D.solve("wilson", up(u, "c128"), up(b, "c128"), m0, inner=inner, tol=1e-10, inner_tol=itol)
    say(f"info {info}")
    assert info["status"] == 0
    res = solver.relative_residual(lambda v: wilson.apply(u, v, m0), b, down(x))
    say(f"oracle residuals {res}")
    assert np.all(res <= 1e-10)
    assert np.allclose(info["relres"], res, rtol=1e-3, atol=1e-13)


def test_solve_rejects_bad_initial_guess():
    # x0 is checked before anything reaches the library: a host tensor, the
    # wrong precision or the wrong shape raise ValueError
    dims, nv, m0 = (4, 4, 4, 4), 2, 0.05
    u = synthetic.gauge_links(dims, "smooth", 3)
    b = synthetic.wilson_spinor(dims, nv, 103)
    U, B = up(u, "c128"), up(b, "c128")
    say("case solve bad x0")
    bad = [torch.zeros(B.shape, dtype=torch.complex128),                  # on the host
           torch.zeros_like(B).to(torch.complex64),                       # FP32
           torch.zeros(B.shape[:-1] + (nv + 1,), dtype=torch.complex128, device=B.device),   # shape
           torch.zeros_like(B).transpose(0, 1)]                           # not contiguous
    for x0 in bad:
        with pytest.raises(ValueError):
            D.solve("wilson", U, B, m0, inner="c64", x0=x0)
    with pytest.raises(ValueError):
        D.solve("brillouin", U, B, m0)
    with pytest.raises(ValueError):
        D.solve("wilson", U, B, m0, inner="c128")


@pytest.mark.parametrize("inner", ["c64", "bf16"])
def test_solve_with_caller_links(inner):
    # dslash_solve with the caller's low-precision links: the same iterations
    # and solution as the call that converts them itself, and per-column counts
    dims, nv, m0 = (12, 4, 2, 4), 12, 0.05
    say(f"case solve caller links inner={inner}")
    u = synthetic.gauge_links(dims, "smooth", 9)
    b = synthetic.wilson_spinor(dims, nv, 109)
    U, B = up(u, "c128"), up(b, "c128")
    x1, i1 = D.solve("wilson", U, B, m0, inner=inner, inner_tol=1e-5 if inner == "c64" else 0.05)
    x2, i2 = D.solve("wilson", U, B, m0, inner=inner, inner_tol=1e-5 if inner == "c64" else 0.05,
                     U_lo=D.convert(U, inner))
    assert i1 == i2
    assert torch.equal(x1, x2)
    assert len(i1["inner_iters_per_column"]) == nv and min(i1["inner_iters_per_column"]) > 0
    res = solver.relative_residual(lambda v: wilson.apply(u, v, m0), b, down(x2))
    assert np.all(res <= 1e-10)
