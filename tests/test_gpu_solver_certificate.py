"""Residual certificate of the solver workload over every site: D_W x = b on
32^3 x 64, N_v = 12, m0 = 0.05, smooth links (seed 3), right-hand sides seed
103, solved to ||b - D x|| / ||b|| <= 1e-10 on the full lattice and on the
even-odd Schur complement with FP32, BF16 and FP16 inner storage at the inner
tolerances the benchmark times.  The FP64 oracle recomputes the residual of
the returned x per column over the whole lattice (in t-slabs, in parallel
host processes); several x meet the tolerance, so residuals, not solutions,
are compared."""
import os

import numpy as np
import pytest

import bench
import synthetic
from tests import residual_certificate as rc
from tests.gpu_util import say, up

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_1808_05506_amd import dslash as D  # noqa: E402

CASES = [(form, inner, itol) for form in ("full", "eo") for inner, itol in bench.SOLVE_SETTINGS[form]]


@pytest.fixture(scope="module")
def system(tmp_path_factory):
    dims, nv = bench.SOLVE_DIMS, bench.SOLVE_NV
    say(f"solver certificate: generating {dims} N_v={nv} (links seed 3, rhs seed 103)")
    d = tmp_path_factory.mktemp("certificate")
    paths = {k: str(d / f"{k}.npy") for k in ("u", "b", "x")}
    u = synthetic.gauge_links(dims, "smooth", 3)
    np.save(paths["u"], u)
    U = up(u, "c128")
    del u
    b = synthetic.wilson_spinor(dims, nv, 103)
    np.save(paths["b"], b)
    B = up(b, "c128")
    del b
    yield U, B, paths
    del U, B
    torch.cuda.empty_cache()
    for p in paths.values():
        if os.path.exists(p):
            os.remove(p)


@pytest.mark.parametrize("form,inner,itol", CASES)
def test_wilson_solve_32cube64_nv12_certified(system, form, inner, itol):
    U, B, paths = system
    say(f"case solve wilson {bench.SOLVE_DIMS} nv={bench.SOLVE_NV} {form} inner={inner} inner_tol={itol}")
    x, info = D.solve("wilson", U, B, bench.SOLVE_M0, inner=inner, tol=bench.SOLVE_TOL, inner_tol=itol,
                      eo=form == "eo")
    say(f"{info['inner_iters']} inner / {info['outer_iters']} outer, status {info['status']}, "
        f"GPU max relres {max(info['relres']):.3e}")
    assert info["status"] == 0
    np.save(paths["x"], x.cpu().numpy())
    del x
    torch.cuda.empty_cache()
    res = rc.certify(paths["u"], paths["b"], paths["x"], bench.SOLVE_M0)
    os.remove(paths["x"])
    say(f"oracle ||b - D x|| / ||b|| per column: max {res.max():.3e} "
        f"(" + " ".join(f"{r:.2e}" for r in res) + ")")
    assert np.all(res <= bench.SOLVE_TOL)
    assert np.allclose(info["relres"], res, rtol=1e-3, atol=1e-13)
