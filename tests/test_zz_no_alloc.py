"""dslash_solve_noalloc (workspace in the library's static device array)
against dslash_solve with a caller workspace, through the C ABI: two calls in
a row, the second on a smaller problem, each giving the same solution bit for
bit, the same residuals and iteration counts, and a residual the oracle
certifies; a problem beyond the static array is refused before any launch."""
import ctypes

import numpy as np
import pytest

import synthetic
from oracle import solver, wilson
from tests.gpu_util import down, say, up

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_1808_05506_amd import dslash as D  # noqa: E402

LIB = D._lib
vp, ip, i, d, sz = ctypes.c_void_p, ctypes.POINTER(ctypes.c_int), ctypes.c_int, ctypes.c_double, ctypes.c_size_t
LIB.dslash_solve_noalloc.argtypes = [vp, vp, vp, vp, ip, i, i, d, i, d, d, i, i, ctypes.POINTER(ctypes.c_double), ip,
                                     vp]
LIB.dslash_solve_noalloc.restype = ctypes.c_int
MAX_BYTES = 128 << 20


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr())


def _run(dims, nv, inner, itol, seed, noalloc):
    m0 = 0.05
    u = synthetic.gauge_links(dims, "smooth", seed)
    b = synthetic.wilson_spinor(dims, nv, seed + 100)
    U, B = up(u, "c128"), up(b, "c128")
    code = {"c64": 0, "bf16": 2, "f16": 3}[inner]
    U_lo = D.convert(U, inner)
    x = torch.zeros_like(B)
    dims_c = (ctypes.c_int * 4)(*dims)
    rel = (ctypes.c_double * nv)()
    it = (ctypes.c_int * (2 * nv))()
    stream = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    if noalloc:
        rc = LIB.dslash_solve_noalloc(_ptr(U), _ptr(U_lo), _ptr(B), _ptr(x), dims_c, 3, nv, m0, code, 1e-10, itol, 50,
                                      20000, rel, it, stream)
    else:
        nbytes = LIB.dslash_solve_workspace_bytes(dims_c, 3, nv, code)
        assert 0 < nbytes <= MAX_BYTES
        ws = torch.empty(nbytes, dtype=torch.uint8, device=B.device)
        rc = LIB.dslash_solve(_ptr(U), _ptr(U_lo), _ptr(B), _ptr(x), dims_c, 3, nv, m0, code, 1e-10, itol, 50, 20000,
                              _ptr(ws), nbytes, rel, it, stream)
    assert rc == 0, LIB.dslash_last_error()
    torch.cuda.synchronize()
    return u, b, m0, x, list(rel), list(it)


@pytest.mark.parametrize("inner,itol", [("c64", 1e-5), ("bf16", 0.05)])
def test_noalloc_solve_matches_workspace_solve(inner, itol):
    # a larger problem first, then a smaller one on the same static array
    for dims, nv, seed in (((12, 4, 4, 8), 12, 5), ((4, 4, 2, 4), 3, 6)):
        say(f"case solve no-alloc {dims} nv={nv} inner={inner}")
        u, b, m0, x_ws, rel_ws, it_ws = _run(dims, nv, inner, itol, seed, noalloc=False)
        _, _, _, x_na, rel_na, it_na = _run(dims, nv, inner, itol, seed, noalloc=True)
        assert torch.equal(x_na, x_ws)
        assert rel_na == rel_ws and it_na == it_ws
        res = solver.relative_residual(lambda v: wilson.apply(u, v, m0), b, down(x_na))
        say(f"oracle residuals max {res.max():.2e}")
        assert np.all(res <= 1e-10)


def test_noalloc_refuses_problems_beyond_the_array():
    dims, nv = (16, 16, 16, 16), 12
    dims_c = (ctypes.c_int * 4)(*dims)
    assert LIB.dslash_solve_workspace_bytes(dims_c, 3, nv, 0) > MAX_BYTES
    rel = (ctypes.c_double * nv)()
    it = (ctypes.c_int * (2 * nv))()
    A, B, C, L = 1 << 40, 2 << 40, 3 << 40, 4 << 40   # never dereferenced: refused before any launch
    rc = LIB.dslash_solve_noalloc(A, L, B, C, dims_c, 3, nv, 0.05, 0, 1e-10, 1e-5, 10, 100, rel, it, None)
    assert rc == 6
    assert b"static scratch" in LIB.dslash_last_error()
