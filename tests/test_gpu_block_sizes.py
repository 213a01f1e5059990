"""D_W, D_S and D_B at other block sizes N_v (the number of right-hand sides is
the method's free parameter, Sec. 2): the row-staged kernels at N_v = 4, 8, 16
and 24 against the FP64 oracle through the C ABI.

Where the library's launch rule covers a shape, the test runs it with
DSLASH_ROWS=2 (the row-staged kernel or an error), so that a fall back to the
direct kernel cannot pass; where it does not, that setting must fail and the
default must still give the oracle's result through the direct kernel."""
import pytest

import synthetic
from oracle import brillouin, staggered, wilson
from tests.gpu_util import compare, down, rounded, say, set_knob, up

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_1808_05506_amd import dslash as D  # noqa: E402

from tests.helpers import brillouin_rows_cover, staggered_rows_cover, wilson_rows_cover  # noqa: E402


def _fields(dims, nv, dt, seed):
    u = rounded(synthetic.gauge_links(dims, "haar", seed), dt)
    p = rounded(synthetic.wilson_spinor(dims, nv, seed + 1), dt)
    return u, p


# one chunk (16), chunks of 12 or 8 (24), 32 in one to four chunks, 40 with a
# partial chunk (14 + 14 + 12 at N_v = 8 and 16), two t segments (N_t = 11 at
# 8 steps), and 20 sites, which 8-byte storage at N_v = 8 and 16 does not cover
SHAPES = [(16, 4, 2, 6), (24, 3, 2, 5), (32, 2, 3, 3), (40, 2, 2, 3), (16, 2, 2, 11), (20, 3, 2, 5)]


@pytest.mark.parametrize("dt", ["c64", "bf16", "f16"])
@pytest.mark.parametrize("adj", [False, True])
@pytest.mark.parametrize("nv", [4, 8, 16, 24])
@pytest.mark.parametrize("dims", SHAPES)
def test_wilson_rows_other_block_sizes(dims, nv, adj, dt, monkeypatch):
    covered = wilson_rows_cover(dims[0], nv, dt)
    say(f"case wilson block size {dims} nv={nv} {dt} adj={adj} rows={covered}")
    u, p = _fields(dims, nv, dt, 500 + nv)
    U, P = up(u, dt), up(p, dt)
    ref = wilson.apply(u, p, 0.1, adj)
    if covered:
        set_knob(monkeypatch, "DSLASH_ROWS", "2")
        out = D.apply("wilson", U, P, 0.1, adjoint=adj)
    else:
        set_knob(monkeypatch, "DSLASH_ROWS", "2")
        with pytest.raises(D.DslashError):
            D.apply("wilson", U, P, 0.1, adjoint=adj)
        set_knob(monkeypatch, "DSLASH_ROWS", None)
        out = D.apply("wilson", U, P, 0.1, adjoint=adj)
    compare(down(out), ref, dt, f"D_W nv={nv}")


def test_the_row_rule_covers_the_benchmark_block_sizes():
    # 16^3 x 32 (D_W) and 32^4 (D_S): every block size of the benchmark rows
    # takes the row-staged kernel in each storage
    for nv in (4, 8, 12, 16, 24):
        for dt in ("c64", "bf16", "f16"):
            assert wilson_rows_cover(16, nv, dt), (nv, dt)
        assert staggered_rows_cover(32, nv, "c64"), nv


@pytest.mark.parametrize("nv", [4, 24])
def test_wilson_16cube32_other_block_sizes(nv, monkeypatch):
    # the benchmark's D_W lattice, 16^3 x 32, m0 = 0.1, exp(0.3 i H) links
    # (seed 1), FP32, at N_v = 4 and 24 through the row-staged kernel
    dims, dt = (16, 16, 16, 32), "c64"
    say(f"case wilson 16^3x32 nv={nv}")
    u = rounded(synthetic.gauge_links(dims, "smooth", 1), dt)
    p = rounded(synthetic.wilson_spinor(dims, nv, 101), dt)
    set_knob(monkeypatch, "DSLASH_ROWS", "2")
    out = D.apply("wilson", up(u, dt), up(p, dt), 0.1)
    compare(down(out), wilson.apply_hop(u, p, 0.1), dt, f"D_W 16^3x32 nv={nv}")


@pytest.mark.parametrize("dt", ["c64", "bf16"])
@pytest.mark.parametrize("adj", [False, True])
def test_columns_do_not_depend_on_the_block_size(dt, adj, monkeypatch):
    # every column is computed with the same arithmetic in the same order
    # whatever the block holds, so D applied to a block of 24 columns equals,
    # bit for bit, D applied to each of its blocks of 4, 8 and 12 columns, at
    # a fixed t-segment length (the -t hop of a segment's first step is added
    # in another order than the carried one) and in the buffer scheme that the
    # other block sizes take (half-spinor rows for FP32, the own-row buffer for
    # BF16; N_v = 12 takes it from DSLASH_MARCH_PP once DSLASH_TSTEPS is set)
    dims = (16, 4, 4, 16)
    say(f"case block-size invariance {dt} adj={adj}")
    u, p = _fields(dims, 24, dt, 520)
    U = up(u, dt)
    set_knob(monkeypatch, "DSLASH_ROWS", "2")
    set_knob(monkeypatch, "DSLASH_TSTEPS", "8")
    set_knob(monkeypatch, "DSLASH_MARCH_PP", "3" if dt == "c64" else "2")
    P = up(p, dt)
    full = D.apply("wilson", U, P, 0.1, adjoint=adj)
    axis = -1 if dt == "c64" else -2
    for k in (4, 8, 12):
        for c0 in range(0, 24, k):
            sl = [slice(None)] * full.dim()
            sl[axis] = slice(c0, c0 + k)
            part = D.apply("wilson", U, P[tuple(sl)].contiguous(), 0.1, adjoint=adj)
            torch.cuda.synchronize()
            assert torch.equal(part, full[tuple(sl)]), (k, c0)


# (D_S takes even extents) one chunk (16), 8 sites (a single chunk at
# N_v >= 8 only), chunks of 12 or 8 (24), 40 with a partial chunk, two t
# segments (N_t = 12 at 8 steps)
STAG_SHAPES = [(16, 4, 2, 6), (8, 4, 2, 4), (24, 4, 2, 6), (40, 2, 2, 4), (16, 2, 2, 12)]


@pytest.mark.parametrize("dt", ["c64", "c128"])
@pytest.mark.parametrize("adj", [False, True])
@pytest.mark.parametrize("nv", [4, 8, 16, 24])
@pytest.mark.parametrize("dims", STAG_SHAPES)
def test_staggered_rows_other_block_sizes(dims, nv, adj, dt, monkeypatch):
    covered = staggered_rows_cover(dims[0], nv, dt)
    say(f"case staggered block size {dims} nv={nv} {dt} adj={adj} rows={covered}")
    u = rounded(synthetic.gauge_links(dims, "haar", 600 + nv), dt)
    p = rounded(synthetic.staggered_spinor(dims, nv, 601 + nv), dt)
    U, P = up(u, dt), up(p, dt)
    ref = staggered.apply(u, p, 0.15, adj)
    set_knob(monkeypatch, "DSLASH_ROWS", "2")
    if covered:
        out = D.apply("staggered", U, P, 0.15, adjoint=adj)
    else:
        with pytest.raises(D.DslashError):
            D.apply("staggered", U, P, 0.15, adjoint=adj)
        set_knob(monkeypatch, "DSLASH_ROWS", None)
        out = D.apply("staggered", U, P, 0.15, adjoint=adj)
    compare(down(out), ref, dt, f"D_S nv={nv}")


@pytest.mark.parametrize("adj", [False, True])
def test_staggered_columns_do_not_depend_on_the_block_size(adj, monkeypatch):
    # as for D_W: a block of 24 columns equals its blocks of 4, 8 and 12
    # columns bit for bit at a fixed t-segment length and prefetch depth
    dims, dt = (16, 4, 4, 16), "c64"
    say(f"case D_S block-size invariance adj={adj}")
    u = rounded(synthetic.gauge_links(dims, "haar", 620), dt)
    p = rounded(synthetic.staggered_spinor(dims, 24, 621), dt)
    U, P = up(u, dt), up(p, dt)
    set_knob(monkeypatch, "DSLASH_ROWS", "2")
    set_knob(monkeypatch, "DSLASH_TSTEPS", "8")
    set_knob(monkeypatch, "DSLASH_ROW_DEPTH", "3")
    full = D.apply("staggered", U, P, 0.15, adjoint=adj)
    for k in (4, 8, 12):
        for c0 in range(0, 24, k):
            part = D.apply("staggered", U, P[..., c0:c0 + k].contiguous(), 0.15, adjoint=adj)
            torch.cuda.synchronize()
            assert torch.equal(part, full[..., c0:c0 + k]), (k, c0)


# one chunk (16), 20 sites (one chunk at N_v = 4, 10 + 10 below the 12-site
# minimum at N_v = 8 and 16, two chunks of 10 with two halo pieces a thread at
# N_v = 24), 24 sites (12 + 12 or three chunks of 8)
BRI_SHAPES = [(16, 3, 3, 3), (20, 3, 2, 3), (24, 2, 3, 3)]


@pytest.mark.parametrize("adj", [False, True])
@pytest.mark.parametrize("nv", [4, 8, 16, 24])
@pytest.mark.parametrize("dims", BRI_SHAPES)
def test_brillouin_rows_other_block_sizes(dims, nv, adj, monkeypatch):
    dt = "c64"
    covered = brillouin_rows_cover(dims[0], nv, dt)
    say(f"case brillouin block size {dims} nv={nv} adj={adj} rows={covered}")
    w = rounded(brillouin.build(synthetic.gauge_links(dims, "haar", 640 + nv)), dt)
    p = rounded(synthetic.wilson_spinor(dims, nv, 641 + nv), dt)
    W, P = up(w, dt), up(p, dt)
    ref = brillouin.apply(w, p, 0.1, adj)
    set_knob(monkeypatch, "DSLASH_ROWS", "2")
    if covered:
        out = D.apply("brillouin", W, P, 0.1, adjoint=adj)
    else:
        with pytest.raises(D.DslashError):
            D.apply("brillouin", W, P, 0.1, adjoint=adj)
        set_knob(monkeypatch, "DSLASH_ROWS", None)
        out = D.apply("brillouin", W, P, 0.1, adjoint=adj)
    compare(down(out), ref, dt, f"D_B nv={nv}")
