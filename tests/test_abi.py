"""C ABI: exported symbols and synchronous argument validation (no GPU needed:
every call here fails validation before any HIP call)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "dslash.h")
LIB = os.path.join(ROOT, "paper_1808_05506_amd", "libdslash.so")

pytestmark = pytest.mark.skipif(not os.path.exists(LIB), reason="libdslash.so not built")


@pytest.fixture(scope="module")
def lib():
    l = ctypes.CDLL(LIB)
    l.dslash_last_error.restype = ctypes.c_char_p
    l.dslash_status_string.restype = ctypes.c_char_p
    vp, ip, i, d, sz = ctypes.c_void_p, ctypes.POINTER(ctypes.c_int), ctypes.c_int, ctypes.c_double, ctypes.c_size_t
    l.dslash_apply.argtypes = [i, vp, vp, vp, ip, i, i, d, i, vp]
    l.dslash_apply_adjoint.argtypes = [i, vp, vp, vp, ip, i, i, d, i, vp]
    l.dslash_backward.argtypes = [i, vp, vp, vp, vp, vp, ip, i, i, d, i, vp]
    l.dslash_brillouin_links.argtypes = [vp, vp, ip, i, i, vp]
    l.dslash_convert.argtypes = [vp, i, vp, i, sz, vp]
    l.dslash_solve_workspace_bytes.argtypes = [ip, i, i, i]
    l.dslash_solve_workspace_bytes.restype = sz
    l.dslash_solve.argtypes = [vp, vp, vp, vp, ip, i, i, d, i, d, d, i, i, vp, sz,
                               ctypes.POINTER(ctypes.c_double), ip, vp]
    l.dslash_solve_op_workspace_bytes.argtypes = [i, ip, i, i, i]
    l.dslash_solve_op_workspace_bytes.restype = sz
    l.dslash_solve_op.argtypes = [i, vp, vp, vp, ip, i, i, d, i, d, d, i, i, vp, sz,
                                  ctypes.POINTER(ctypes.c_double), ip, vp]
    l.dslash_eo_pack.argtypes = [vp, vp, vp, ip, sz, vp]
    l.dslash_eo_unpack.argtypes = [vp, vp, vp, ip, sz, vp]
    l.dslash_eo_hop.argtypes = [vp, vp, vp, vp, ip, i, i, i, i, i, vp]
    l.dslash_solve_eo_workspace_bytes.argtypes = [ip, i, i, i]
    l.dslash_solve_eo_workspace_bytes.restype = sz
    l.dslash_solve_eo.argtypes = [vp, vp, vp, ip, i, i, d, i, d, d, i, i, vp, sz,
                                  ctypes.POINTER(ctypes.c_double), ip, vp]
    l.dslash_clover_field.argtypes = [vp, vp, ip, i, d, i, vp]
    l.dslash_apply_clover.argtypes = [i, vp, vp, vp, vp, ip, i, i, d, i, i, vp]
    l.dslash_compress_links.argtypes = [vp, vp, ip, i, i, vp]
    l.dslash_apply_compressed.argtypes = [i, vp, vp, vp, ip, i, i, d, i, i, vp]
    l.dslash_brillouin_links_backward.argtypes = [vp, vp, vp, vp, ip, i, i, vp]
    l.dslash_brillouin_links_backward_workspace_bytes.argtypes = [ip, i, i]
    l.dslash_brillouin_links_backward_workspace_bytes.restype = sz
    l.dslash_brillouin_links_backward_ws.argtypes = [vp, vp, vp, vp, vp, sz, ip, i, i, vp]
    l.dslash_apply_brillouin_fly.argtypes = [vp, vp, vp, ip, i, i, d, i, i, vp]
    return l


def _dims(*d):
    return (ctypes.c_int * 4)(*d)


def test_exports_every_declared_symbol(lib):
    text = open(HEADER).read()
    declared = set(re.findall(r"^\s*(?:int|size_t|const char\*)\s+(dslash_\w+)\s*\(", text, re.M))
    assert len(declared) == 27
    for name in declared:
        assert hasattr(lib, name), name
    assert lib.dslash_version() == 201


def test_reload_tuning_reads_the_environment_again(lib, monkeypatch):
    # host only: re-reading the knobs touches no device
    monkeypatch.setenv("DSLASH_TSTEPS", "4")
    assert lib.dslash_reload_tuning() == 0
    monkeypatch.delenv("DSLASH_TSTEPS")
    assert lib.dslash_reload_tuning() == 0


def test_solve_signatures_follow_the_header():
    # the full-lattice Wilson solve takes the FP64 links, the caller's
    # low-precision links and per-column iteration counts; the op-taking
    # variant converts the links itself
    text = " ".join(open(HEADER).read().split())
    assert ("size_t dslash_solve_workspace_bytes(const int dims[4], int Nc, int Nv, int inner_dtype);" in text)
    assert ("int dslash_solve(const void* U64, const void* U_lo, const void* b64, void* x64, const int dims[4], "
            "int Nc, int Nv, double mass, int inner_dtype, double tol, double inner_tol, int max_outer, "
            "int max_inner, void* workspace, size_t ws_bytes, double* final_relres, int* iters, void* stream);"
            in text)
    assert "iters (host, 2 * Nv ints, nullable)" in text
    assert "int dslash_solve_op(int op, const void* U64, const void* b64, void* x64," in text


def test_status_strings(lib):
    for code in range(7):
        assert lib.dslash_status_string(code)
    assert lib.dslash_status_string(99) == b"unknown status"


A, B, C = 0x10000, 0x4000000, 0x8000000   # fake device addresses, never dereferenced


@pytest.mark.parametrize("fn", ["dslash_apply", "dslash_apply_adjoint"])
def test_apply_validation(lib, fn):
    f = getattr(lib, fn)
    d = _dims(4, 4, 4, 4)
    assert f(1, None, B, C, d, 3, 12, 0.1, 0, None) == 1            # NULL U
    assert f(1, A, B, C, None, 3, 12, 0.1, 0, None) == 1            # NULL dims
    assert f(7, A, B, C, d, 3, 12, 0.1, 0, None) == 1               # bad op
    assert f(1, A, B, C, d, 3, 12, 0.1, 9, None) == 1               # bad dtype
    assert f(1, A, B, C, d, 3, 0, 0.1, 0, None) == 1                # Nv < 1
    assert f(1, A, B, C, _dims(4, 1, 4, 4), 3, 2, 0.1, 0, None) == 1  # extent < 2
    assert f(1, A, B, C, d, 2, 12, 0.1, 0, None) == 2               # Nc != 3
    assert f(0, A, B, C, _dims(4, 3, 4, 4), 3, 2, 0.0, 0, None) == 1  # odd extent, staggered
    assert b"even" in lib.dslash_last_error()
    assert f(1, A, B, B, d, 3, 12, 0.1, 0, None) == 3               # in == out
    assert f(1, A, B, B + 64, d, 3, 12, 0.1, 0, None) == 3          # overlapping out
    assert f(1, B + 8, A, B, d, 3, 12, 0.1, 0, None) == 3           # out overlaps U
    assert f(1, A, B, C, _dims(2048, 2048, 1024, 2), 3, 1, 0.1, 0, None) == 1  # volume >= 2^31


def test_backward_validation(lib):
    d = _dims(4, 4, 4, 4)
    assert lib.dslash_backward(1, A, None, B, C, 0, d, 3, 2, 0.1, 0, None) == 1       # NULL grad_out
    assert lib.dslash_backward(1, A, B, C, 0x9000000, 0, d, 3, 2, 0.1, 2, None) == 2  # bf16 backward
    assert lib.dslash_backward(2, A, B, C, C + 0x100, 0, d, 3, 2, 0.1, 0, None) == 3  # Brillouin grad_U overlaps in
    assert lib.dslash_backward(1, A, B, C, None, B, d, 3, 2, 0.1, 0, None) == 3       # grad_in == grad_out
    assert lib.dslash_backward(1, A, B, C, C, None, d, 3, 2, 0.1, 0, None) == 3       # grad_U == in


def test_links_convert_validation(lib):
    d = _dims(4, 4, 4, 4)
    assert lib.dslash_brillouin_links(None, B, d, 3, 0, None) == 1
    assert lib.dslash_brillouin_links(A, B, d, 3, 2, None) == 2
    assert lib.dslash_brillouin_links(A, A, d, 3, 0, None) == 3
    assert lib.dslash_convert(A, 0, B, 7, 10, None) == 1
    assert lib.dslash_convert(A, 0, A, 1, 10, None) == 3
    assert lib.dslash_convert(None, 0, None, 1, 0, None) == 0    # n == 0 is a no-op


def test_solve_validation(lib):
    d = _dims(4, 4, 4, 4)
    L = 0x30000000                                                  # fake low-precision links
    assert lib.dslash_solve_workspace_bytes(d, 3, 2, 2) > 0
    assert lib.dslash_solve_workspace_bytes(d, 3, 2, 1) == 0        # C128 inner not allowed
    assert lib.dslash_solve_workspace_bytes(d, 4, 2, 2) == 0
    # the caller's links take no workspace
    assert lib.dslash_solve_workspace_bytes(d, 3, 2, 2) < lib.dslash_solve_op_workspace_bytes(1, d, 3, 2, 2)
    rel = (ctypes.c_double * 2)()
    it = (ctypes.c_int * 4)()
    ws = 0x20000000
    need = lib.dslash_solve_workspace_bytes(d, 3, 2, 2)
    assert lib.dslash_solve(A, L, B, C, d, 3, 2, 0.05, 2, 1e-10, 0.1, 10, 100, None, 0, rel, it, None) == 6
    assert lib.dslash_solve(A, L, B, C, d, 3, 2, 0.05, 2, 1e-10, 0.1, 10, 100, ws, need - 1, rel, it, None) == 6
    assert lib.dslash_solve(A, None, B, C, d, 3, 2, 0.05, 2, 1e-10, 0.1, 10, 100, ws, need, rel, it, None) == 1
    assert lib.dslash_solve(A, L, B, C, d, 3, 2, 0.05, 2, -1.0, 0.1, 10, 100, ws, need, rel, it, None) == 1
    assert lib.dslash_solve(A, L, B, C, d, 3, 2, 0.05, 2, 1e-10, 1.5, 10, 100, ws, need, rel, it, None) == 1
    assert lib.dslash_solve(A, L, B, C, d, 3, 2, 0.05, 0, 1e-10, 0.1, 0, 100, ws, need, rel, it, None) == 1
    assert lib.dslash_solve(A, L, B, B, d, 3, 2, 0.05, 2, 1e-10, 0.1, 10, 100, ws, need, rel, it, None) == 3
    assert lib.dslash_solve(A, ws, B, C, d, 3, 2, 0.05, 2, 1e-10, 0.1, 10, 100, ws, need, rel, it, None) == 3
    assert lib.dslash_solve(A, L, B, C, d, 3, 2, 0.05, 1, 1e-10, 0.1, 10, 100, ws, need, rel, it, None) == 1
    # the op-taking variant: STAGGERED and WILSON only
    need_op = lib.dslash_solve_op_workspace_bytes(1, d, 3, 2, 2)
    assert lib.dslash_solve_op_workspace_bytes(2, d, 3, 2, 2) == 0
    assert lib.dslash_solve_op(2, A, B, C, d, 3, 2, 0.05, 2, 1e-10, 0.1, 10, 100, ws, 1 << 30, rel, it, None) == 1
    assert b"BRILLOUIN" in lib.dslash_last_error()
    assert lib.dslash_solve_op(1, A, B, C, d, 3, 2, 0.05, 2, 1e-10, 0.1, 10, 100, ws, need_op - 1, rel, it,
                               None) == 6
    assert lib.dslash_solve_op(0, A, B, C, _dims(4, 3, 4, 4), 3, 2, 0.05, 2, 1e-10, 0.1, 10, 100, ws, 1 << 30, rel,
                               it, None) == 1


def test_binding_rejects_cpu_tensors():
    torch = pytest.importorskip("torch")
    from paper_1808_05506_amd import dslash as D
    u = torch.zeros(2, 2, 2, 2, 4, 3, 3, dtype=torch.complex64)
    p = torch.zeros(2, 2, 2, 2, 4, 3, 1, dtype=torch.complex64)
    with pytest.raises(ValueError):
        D.apply("wilson", u, p, 0.1)
    with pytest.raises(ValueError):
        D.op_code("clover")
    # the adjoint of the W construction: an unknown method, W with the walk
    # through V, and the W-based methods without W are refused before any call
    v = torch.zeros(2, 2, 2, 2, 4, 3, 3, dtype=torch.complex64)
    gw = torch.zeros(2, 2, 2, 2, 40, 3, 3, dtype=torch.complex64)
    with pytest.raises(ValueError):
        D.brillouin_links_backward(v, gw, gw, method="tree")
    with pytest.raises(ValueError):
        D.brillouin_links_backward(v, gw, gw, method="walk")
    for method in ("subsets", "levels"):
        with pytest.raises(ValueError):
            D.brillouin_links_backward(v, gw, None, method=method)
    with pytest.raises(ValueError):
        D.brillouin_links_backward(v, gw)  # CPU tensors


def test_even_odd_validation(lib):
    even, odd = _dims(4, 4, 4, 4), _dims(4, 3, 4, 4)
    D = 0x20000000
    assert lib.dslash_eo_pack(A, B, C, odd, 96, None) == 1                   # odd extent
    assert lib.dslash_eo_pack(A, B, C, even, 0, None) == 1                   # no bytes
    assert lib.dslash_eo_pack(A, A, C, even, 96, None) == 3                  # full overlaps even
    assert lib.dslash_eo_unpack(None, B, C, even, 96, None) == 1             # NULL
    assert lib.dslash_eo_hop(A, B, C, D, even, 3, 2, 2, 0, 0, None) == 1     # parity 2
    assert lib.dslash_eo_hop(A, B, C, C, even, 3, 2, 0, 0, 0, None) == 3     # in == out
    assert lib.dslash_eo_hop(A, B, C, D, odd, 3, 2, 0, 0, 0, None) == 1      # odd extent
    assert lib.dslash_eo_hop(A, B, C, D, even, 2, 2, 0, 0, 0, None) == 2     # Nc != 3
    assert lib.dslash_solve_eo_workspace_bytes(odd, 3, 2, 2) == 0
    assert lib.dslash_solve_eo_workspace_bytes(even, 3, 2, 1) == 0          # FP64 inner
    assert lib.dslash_solve_eo_workspace_bytes(even, 3, 2, 2) > 0
    rel = (ctypes.c_double * 2)()
    it = (ctypes.c_int * 4)()
    assert lib.dslash_solve_eo(A, B, C, odd, 3, 2, 0.1, 2, 1e-10, 0.1, 10, 10, D, 1 << 30, rel, it, None) == 1
    assert lib.dslash_solve_eo(A, B, C, even, 3, 2, 0.1, 2, 1e-10, 0.1, 10, 10, D, 16, rel, it, None) == 6
    assert lib.dslash_solve_eo(A, B, C, even, 3, 2, -4.0, 2, 1e-10, 0.1, 10, 10, D, 1 << 30, rel, it, None) == 1


def test_clover_validation(lib):
    dims = _dims(4, 4, 4, 4)
    D = 0x20000000
    assert lib.dslash_clover_field(None, B, dims, 3, 1.0, 0, None) == 1           # NULL V
    assert lib.dslash_clover_field(A, A, dims, 3, 1.0, 0, None) == 3              # V == C
    assert lib.dslash_clover_field(A, B, _dims(4, 1, 4, 4), 3, 1.0, 0, None) == 1  # extent 1
    assert lib.dslash_clover_field(A, B, dims, 2, 1.0, 0, None) == 2              # Nc != 3
    assert lib.dslash_clover_field(A, B, dims, 3, 1.0, 7, None) == 1              # dtype
    assert lib.dslash_apply_clover(0, A, B, C, D, dims, 3, 2, 0.1, 0, 0, None) == 1  # staggered
    assert lib.dslash_apply_clover(1, A, None, C, D, dims, 3, 2, 0.1, 0, 0, None) == 1  # no C
    assert lib.dslash_apply_clover(1, A, B, C, C, dims, 3, 2, 0.1, 0, 0, None) == 3  # in == out
    assert lib.dslash_apply_clover(1, A, B, C, B, dims, 3, 2, 0.1, 0, 0, None) == 3  # out == C


def test_compressed_validation(lib):
    dims = _dims(4, 4, 4, 4)
    D = 0x20000000
    assert lib.dslash_compress_links(None, B, dims, 3, 0, None) == 1            # NULL V
    assert lib.dslash_compress_links(A, A, dims, 3, 0, None) == 3               # V == Vc
    assert lib.dslash_compress_links(A, B, dims, 2, 0, None) == 2               # Nc != 3
    assert lib.dslash_apply_compressed(2, A, C, D, dims, 3, 2, 0.1, 0, 0, None) == 1  # brillouin
    assert lib.dslash_apply_compressed(1, A, C, C, dims, 3, 2, 0.1, 0, 0, None) == 3  # in == out
    assert lib.dslash_apply_compressed(1, None, C, D, dims, 3, 2, 0.1, 0, 0, None) == 1  # NULL Vc
    assert lib.dslash_apply_compressed(0, A, C, D, _dims(4, 3, 4, 4), 3, 2, 0.0, 0, 0, None) == 1  # odd, staggered


def test_brillouin_links_backward_validation(lib):
    dims = _dims(4, 4, 4, 4)
    D = 0x20000000
    assert lib.dslash_brillouin_links_backward(None, None, B, C, dims, 3, 0, None) == 1   # NULL V
    assert lib.dslash_brillouin_links_backward(A, None, B, A, dims, 3, 0, None) == 3      # grad_V == V
    assert lib.dslash_brillouin_links_backward(A, None, B, B, dims, 3, 0, None) == 3      # grad_V == grad_W
    assert lib.dslash_brillouin_links_backward(A, D, B, D, dims, 3, 0, None) == 3         # grad_V == W
    assert lib.dslash_brillouin_links_backward(A, None, B, C, dims, 3, 2, None) == 2      # BF16
    assert lib.dslash_brillouin_links_backward(A, None, B, C, dims, 2, 0, None) == 2      # Nc != 3


def test_brillouin_links_backward_ws_validation(lib):
    dims = _dims(4, 4, 4, 4)
    D, E = 0x20000000, 0x30000000
    nw = lib.dslash_brillouin_links_backward_workspace_bytes(dims, 3, 0)
    assert nw == 256 * 756 * 8                    # grad_W, W (360 words a site each) and V (36), C64
    assert lib.dslash_brillouin_links_backward_workspace_bytes(dims, 3, 1) == 2 * nw   # C128
    assert lib.dslash_brillouin_links_backward_workspace_bytes(dims, 3, 2) == 0        # BF16
    assert lib.dslash_brillouin_links_backward_workspace_bytes(dims, 2, 0) == 0        # Nc != 3
    assert lib.dslash_brillouin_links_backward_workspace_bytes(_dims(4, 4, 0, 4), 3, 0) == 0
    ws = lib.dslash_brillouin_links_backward_ws
    assert ws(A, None, B, C, E, nw, dims, 3, 0, None) == 1          # W is required
    assert ws(A, D, B, C, None, nw, dims, 3, 0, None) == 1          # NULL workspace
    assert ws(A, D, B, C, E, nw - 1, dims, 3, 0, None) == 1         # workspace too small
    assert ws(A, D, B, C, E + 8, nw, dims, 3, 0, None) == 1         # workspace 8 bytes off 16
    assert ws(A, D, B, A, E, nw, dims, 3, 0, None) == 3             # grad_V == V
    assert ws(A, D, B, D, E, nw, dims, 3, 0, None) == 3             # grad_V == W
    assert ws(A, D, B, C, B, nw, dims, 3, 0, None) == 3             # workspace == grad_W
    assert ws(A, D, B, C, D + 16, nw, dims, 3, 0, None) == 3        # workspace overlaps W
    assert ws(A, D, B, C, C - 16, nw, dims, 3, 0, None) == 3        # workspace runs into grad_V
    assert ws(A, D, B, C, E, nw, dims, 3, 2, None) == 2             # BF16
    assert ws(A, D, B, C, E, nw, dims, 2, 0, None) == 2             # Nc != 3


def test_brillouin_fly_validation(lib):
    dims = _dims(16, 4, 4, 4)
    D = 0x20000000
    assert lib.dslash_apply_brillouin_fly(None, C, D, dims, 3, 12, 0.1, 0, 0, None) == 1   # NULL V
    assert lib.dslash_apply_brillouin_fly(A, C, C, dims, 3, 12, 0.1, 0, 0, None) == 3      # in == out
    assert lib.dslash_apply_brillouin_fly(A, C, D, dims, 3, 5, 0.1, 0, 0, None) == 2       # N_v = 5
    assert lib.dslash_apply_brillouin_fly(A, C, D, dims, 3, 12, 0.1, 0, 1, None) == 2      # C128
    assert lib.dslash_apply_brillouin_fly(A, C, D, _dims(8, 4, 4, 4), 3, 12, 0.1, 0, 0, None) == 2  # rows of 8
