"""GPU parity of D_S, D_W, D_B (and adjoints), the W construction and the
precision conversions against the FP64 oracle, through the C ABI."""

import numpy as np
import pytest

import synthetic
from oracle import brillouin, local, staggered, wilson
from tests.gpu_util import compare, down, rounded, say, up, set_knob
from tests.helpers import wilson_rows_cover

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_1808_05506_amd import dslash as D  # noqa: E402


def _stag_fields(dims, nv, lseed, pseed, dt):
    u = rounded(synthetic.gauge_links(dims, "haar", lseed), dt)
    p = rounded(synthetic.staggered_spinor(dims, nv, pseed), dt)
    return u, p


def _wil_fields(dims, nv, lseed, pseed, dt, kind="smooth"):
    u = rounded(synthetic.gauge_links(dims, kind, lseed), dt)
    p = rounded(synthetic.wilson_spinor(dims, nv, pseed), dt)
    return u, p


@pytest.mark.parametrize("dt", ["c64", "c128"])
@pytest.mark.parametrize("adj", [False, True])
def test_staggered_8to4_nv4(dt, adj):
    # D_S on an 8^4 periodic lattice, N_v = 4, Haar links (seed 0), Gaussian rhs (seed 100), m = 0
    dims, nv = (8, 8, 8, 8), 4
    say(f"case staggered {dims} nv={nv} {dt} adj={adj}")
    u, p = _stag_fields(dims, nv, 0, 100, dt)
    out = D.apply("staggered", up(u, dt), up(p, dt), 0.0, adjoint=adj)
    compare(down(out), staggered.apply(u, p, 0.0, adj), dt, "D_S 8^4")


@pytest.mark.parametrize("dt", ["c64", "c128"])
@pytest.mark.parametrize("adj", [False, True])
@pytest.mark.parametrize("dims,nv,mass", [((4, 6, 2, 4), 3, 0.3), ((6, 2, 4, 10), 7, -0.2), ((2, 2, 2, 2), 1, 0.5)])
def test_staggered_shapes(dt, adj, dims, nv, mass):
    say(f"case staggered {dims} nv={nv} {dt} adj={adj}")
    u, p = _stag_fields(dims, nv, 11, 12, dt)
    out = D.apply("staggered", up(u, dt), up(p, dt), mass, adjoint=adj)
    compare(down(out), staggered.apply(u, p, mass, adj), dt, "D_S")


@pytest.mark.parametrize("dt", ["c64", "c128"])
@pytest.mark.parametrize("adj", [False, True])
@pytest.mark.parametrize("dims,nv", [((4, 6, 2, 4), 3), ((5, 3, 4, 7), 5), ((2, 2, 2, 2), 1), ((4, 4, 2, 6), 13),
                                     ((3, 2, 2, 3), 70)])
def test_wilson_shapes(dt, adj, dims, nv):
    # ragged volumes (not a multiple of the sites per block), odd extents,
    # extent 2 (forward and backward neighbour coincide), N_v above 64 lanes
    say(f"case wilson {dims} nv={nv} {dt} adj={adj}")
    u, p = _wil_fields(dims, nv, 21, 22, dt, "haar")
    out = D.apply("wilson", up(u, dt), up(p, dt), 0.1, adjoint=adj)
    compare(down(out), wilson.apply(u, p, 0.1, adj), dt, "D_W")


@pytest.mark.parametrize("dt", ["c64", "c128"])
def test_wilson_16cube32_nv12(dt):
    # the benchmark workload: 16^3 x 32, N_v = 12, m0 = 0.1, exp(0.3 i H) links (seed 1), rhs seed 101
    dims, nv = (16, 16, 16, 32), 12
    say(f"case wilson {dims} nv={nv} {dt} (bench workload)")
    u, p = _wil_fields(dims, nv, 1, 101, dt)
    out = D.apply("wilson", up(u, dt), up(p, dt), 0.1)
    res = down(out)
    ref = wilson.apply_hop(u, p, 0.1)
    compare(res, ref, dt, "D_W 16^3x32")


@pytest.mark.parametrize("dt", ["c64", "c128"])
@pytest.mark.parametrize("adj", [False, True])
@pytest.mark.parametrize("dims,nv", [((4, 4, 4, 4), 3), ((3, 4, 5, 3), 2), ((2, 4, 2, 3), 5)])
def test_brillouin_shapes(dt, adj, dims, nv):
    say(f"case brillouin {dims} nv={nv} {dt} adj={adj}")
    v = synthetic.gauge_links(dims, "haar", 31)
    w = rounded(brillouin.build(v), dt)
    p = rounded(synthetic.wilson_spinor(dims, nv, 32), dt)
    out = D.apply("brillouin", up(w, dt), up(p, dt), 0.1, adjoint=adj)
    compare(down(out), brillouin.apply(w, p, 0.1, adj), dt, "D_B")


@pytest.mark.parametrize("dt", ["c64", "c128"])
@pytest.mark.parametrize("dims", [(4, 3, 4, 5), (3, 3, 3, 3), (2, 3, 2, 4)])
def test_brillouin_links(dt, dims):
    say(f"case W build {dims} {dt}")
    v = rounded(synthetic.gauge_links(dims, "haar", 41), dt)
    w = D.brillouin_links(up(v, dt))
    compare(down(w), brillouin.build(v), dt, "W")


@pytest.mark.parametrize("dt", ["c64", "c128"])
def test_brillouin_32to4_nv12_sampled(dt):
    # 32^4, N_v = 12, Haar links (seed 2), rhs seed 102: W built on the GPU,
    # then D_B; the oracle evaluates out(x) from V and psi at sampled sites
    # (W rebuilt from V by its own path products at each site)
    dims, nv = (32, 32, 32, 32), 12
    say(f"case brillouin {dims} nv={nv} {dt} sampled")
    v = rounded(synthetic.gauge_links(dims, "haar", 2), dt)
    p = rounded(synthetic.wilson_spinor(dims, nv, 102), dt)
    V = up(v, dt)
    W = D.brillouin_links(V)
    P = up(p, dt)
    del V
    out = D.apply("brillouin", W, P, 0.1)
    sites = local.sample_sites(dims, 48, 7)
    idx = (sites[:, 3], sites[:, 2], sites[:, 1], sites[:, 0])
    it = torch.as_tensor(np.stack(idx), device=out.device)
    got = out[it[0], it[1], it[2], it[3]].cpu().numpy().astype(np.complex128)
    del W, P, out
    torch.cuda.empty_cache()
    ref = local.brillouin_at(v, p, 0.1, sites)
    compare(got, ref, dt, "D_B 32^4 sampled")


@pytest.mark.parametrize("dt", ["bf16", "f16"])
@pytest.mark.parametrize("op", ["staggered", "wilson", "brillouin"])
@pytest.mark.parametrize("adj", [False, True])
def test_low_precision_storage(dt, op, adj):
    dims, nv = (4, 6, 4, 4), 6
    say(f"case {op} {dims} nv={nv} {dt} adj={adj}")
    if op == "staggered":
        u, p = _stag_fields(dims, nv, 51, 52, dt)
        ref = staggered.apply(u, p, 0.2, adj)
    elif op == "wilson":
        u, p = _wil_fields(dims, nv, 51, 52, dt)
        ref = wilson.apply(u, p, 0.2, adj)
    else:
        u = rounded(brillouin.build(synthetic.gauge_links(dims, "haar", 51)), dt)
        p = rounded(synthetic.wilson_spinor(dims, nv, 52), dt)
        ref = brillouin.apply(u, p, 0.2, adj)
    out = D.apply(op, up(u, dt), up(p, dt), 0.2, adjoint=adj)
    compare(down(out), ref, dt, f"{op} {dt}")


def test_bitwise_determinism_across_launch_shapes(monkeypatch):
    # every output element has one writer summing in a fixed order, so the
    # result must not depend on the number of sites per workgroup
    dims, nv = (8, 6, 8, 8), 12
    u, p = _wil_fields(dims, nv, 61, 62, "c64")
    U, P = up(u, "c64"), up(p, "c64")
    outs = {}
    for sb in (None, "1", "5", "16", "21"):
        set_knob(monkeypatch, "DSLASH_SITES_PER_BLOCK", sb)
        say(f"case determinism sites_per_block={sb}")
        for op, uu in (("wilson", U),):
            outs[(op, sb, 0)] = D.apply(op, uu, P, 0.1).cpu()
            outs[(op, sb, 1)] = D.apply(op, uu, P, 0.1).cpu()
    ref = outs[("wilson", None, 0)]
    for k, v in outs.items():
        assert torch.equal(v, ref), k


def test_convert_matches_host_rounding():
    a = synthetic.gaussian((1000, 7), 71) * 3.0
    say("case convert")
    x64 = up(a, "c128")
    for dt in ("c64", "bf16", "f16"):
        got = down(D.convert(x64, dt))
        exp = rounded(rounded(a, "c64"), dt) if dt != "c64" else rounded(a, "c64")
        assert np.array_equal(got, exp), dt
    # widening is exact
    b16 = up(a, "bf16")
    assert np.array_equal(down(D.convert(b16, "c64")), rounded(a, "bf16"))


def test_errors_raise():
    dims = (4, 4, 4, 4)
    u, p = _wil_fields(dims, 2, 1, 2, "c64")
    U, P = up(u, "c64"), up(p, "c64")
    with pytest.raises(D.DslashError):
        D.apply("wilson", U, P, 0.1, out=P)       # in == out
    with pytest.raises(ValueError):
        D.apply("staggered", U, P, 0.1)           # wrong spinor shape for the op


@pytest.mark.parametrize("kernel", ["march", "rows"])
@pytest.mark.parametrize("dt", ["c64", "bf16", "f16"])
@pytest.mark.parametrize("adj", [False, True])
@pytest.mark.parametrize("dims", [(16, 4, 2, 6), (20, 3, 4, 5), (11, 2, 2, 3), (12, 2, 2, 3), (32, 2, 3, 2)])
def test_wilson_row_staged_path(kernel, dt, adj, dims, monkeypatch):
    # N_v = 12 runs an LDS row-staged kernel where the launch rule covers the
    # row (by default the t-marching one; DSLASH_TSTEPS=0 selects one output
    # row per workgroup; DSLASH_ROWS=2 then requires it), the direct kernel
    # elsewhere (11 and 20 sites in FP32 storage); 20 and 32 sites split into
    # chunks (a partial one for 20)
    nv = 12
    set_knob(monkeypatch, "DSLASH_TSTEPS", "8" if kernel == "march" else "0")
    if wilson_rows_cover(dims[0], nv, dt):
        set_knob(monkeypatch, "DSLASH_ROWS", "2")
    say(f"case wilson {kernel} {dims} nv={nv} {dt} adj={adj}")
    u, p = _wil_fields(dims, nv, 81, 82, dt, "haar")
    out = D.apply("wilson", up(u, dt), up(p, dt), 0.1, adjoint=adj)
    compare(down(out), wilson.apply(u, p, 0.1, adj), dt, f"D_W {kernel}")


@pytest.mark.parametrize("dims,tsteps", [((16, 2, 2, 11), "8"), ((12, 3, 2, 17), "8"), ((16, 2, 3, 7), "3"),
                                         ((16, 2, 2, 5), "1"), ((16, 2, 2, 4), "64"), ((13, 2, 2, 35), "16")])
@pytest.mark.parametrize("adj", [False, True])
@pytest.mark.parametrize("pp", ["0", "1", "2", "3"])
def test_wilson_march_segments(dims, tsteps, adj, pp, monkeypatch):
    # t-marching workgroups over several t segments, a partial last one, one
    # step per workgroup (no carried -t hop) and a segment longer than N_t,
    # with one row buffer, two used in turn, an own-row buffer plus two, and
    # the same with half-spinor neighbour rows
    nv, dt = 12, "c64"
    set_knob(monkeypatch, "DSLASH_TSTEPS", tsteps)
    set_knob(monkeypatch, "DSLASH_MARCH_PP", pp)
    say(f"case wilson march segments {dims} T={tsteps} pp={pp} adj={adj}")
    u, p = _wil_fields(dims, nv, 83, 84, dt, "haar")
    out = D.apply("wilson", up(u, dt), up(p, dt), 0.1, adjoint=adj)
    compare(down(out), wilson.apply(u, p, 0.1, adj), dt, "D_W march segments")


def test_march_buffer_modes_on_the_headline_lattice(monkeypatch):
    # 16^3 x 32, N_v = 12, FP32: the default launch marches 16 steps with the
    # own-row buffer.  Two buffers in turn do the one-buffer kernel's arithmetic
    # (bitwise equal at the same segment length); the own-row buffer folds the
    # diagonal term into the accumulator (equal to rounding); staging the
    # neighbour rows as half spinors does the same arithmetic as staging them
    # whole (bitwise equal).  All match the oracle.
    dims, nv, dt = (16, 16, 16, 32), 12, "c64"
    say("case wilson march buffer modes")
    u, p = _wil_fields(dims, nv, 85, 86, dt, "smooth")
    U, P = up(u, dt), up(p, dt)
    ref = wilson.apply(u, p, 0.1)
    default = D.apply("wilson", U, P, 0.1)
    compare(down(default), ref, dt, "D_W 16^3x32 default launch")
    set_knob(monkeypatch, "DSLASH_TSTEPS", "16")
    outs = {}
    for mode in ("0", "1", "2", "3"):
        set_knob(monkeypatch, "DSLASH_MARCH_PP", mode)
        outs[mode] = D.apply("wilson", U, P, 0.1)
        compare(down(outs[mode]), ref, dt, f"D_W 16^3x32 buffers mode {mode}")
    torch.cuda.synchronize()
    assert torch.equal(outs["0"], outs["1"])
    assert torch.equal(outs["2"], default)
    assert torch.equal(outs["3"], outs["2"])


@pytest.mark.parametrize("kernel", ["march", "rows"])
def test_row_staged_determinism_across_chunk_sizes(kernel, monkeypatch):
    dims, nv = (22, 4, 4, 4), 12
    set_knob(monkeypatch, "DSLASH_TSTEPS", "8" if kernel == "march" else "0")
    u, p = _wil_fields(dims, nv, 91, 92, "c64")
    U, P = up(u, "c64"), up(p, "c64")
    outs = []
    for r in ("12", "16", "21"):
        set_knob(monkeypatch, "DSLASH_ROW_SITES", r)
        say(f"case {kernel} determinism R={r}")
        outs.append(D.apply("wilson", U, P, 0.1).cpu())
    for o in outs[1:]:
        assert torch.equal(o, outs[0])
    compare(outs[0].numpy().astype(np.complex128), wilson.apply(u, p, 0.1), "c64", "D_W rows R sweep")


_SROW_DIMS = [(16, 4, 2, 6), (20, 2, 4, 6), (12, 2, 2, 4), (14, 2, 2, 2), (32, 2, 2, 2), (24, 4, 2, 2)]


@pytest.mark.parametrize("kernel", ["march", "rows", "direct"])
@pytest.mark.parametrize("dt", ["c64", "c128"])
@pytest.mark.parametrize("adj", [False, True])
@pytest.mark.parametrize("dims", _SROW_DIMS)
def test_staggered_row_staged_path(kernel, dt, adj, dims, monkeypatch):
    # N_v = 12 with rows of >= 6 sites runs the LDS row-staged D_S kernels:
    # t-marching by default, one output row per workgroup with DSLASH_TSTEPS=0
    # (DSLASH_ROWS=0 forces the direct kernel, 2 the row-staged one or an
    # error); 20 sites split into 11 + 9, 24 into 12 + 12, 32 into 16 + 16, 12
    # to 16 fill one chunk
    nv = 12
    set_knob(monkeypatch, "DSLASH_ROWS", "0" if kernel == "direct" else "2")
    if kernel == "rows":
        set_knob(monkeypatch, "DSLASH_TSTEPS", "0")
    say(f"case staggered {kernel} {dims} nv={nv} {dt} adj={adj}")
    u, p = _stag_fields(dims, nv, 71, 72, dt)
    out = D.apply("staggered", up(u, dt), up(p, dt), 0.15, adjoint=adj)
    compare(down(out), staggered.apply(u, p, 0.15, adj), dt, f"D_S {kernel}")


@pytest.mark.parametrize("kernel,depth", [("rows", "3"), ("rows", "7"), ("march", "2"), ("march", "3"), ("march", "4")])
def test_staggered_rows_determinism_across_chunk_sizes(kernel, depth, monkeypatch):
    dims, nv = (22, 4, 2, 4), 12
    set_knob(monkeypatch, "DSLASH_ROW_DEPTH", depth)
    set_knob(monkeypatch, "DSLASH_TSTEPS", "0" if kernel == "rows" else "3")
    u, p = _stag_fields(dims, nv, 73, 74, "c64")
    U, P = up(u, "c64"), up(p, "c64")
    outs = []
    for r in ("12", "16", "21"):
        set_knob(monkeypatch, "DSLASH_ROW_SITES", r)
        say(f"case staggered {kernel} determinism R={r} depth={depth}")
        outs.append(D.apply("staggered", U, P, 0.0).cpu())
    for o in outs[1:]:
        assert torch.equal(o, outs[0])
    compare(outs[0].numpy().astype(np.complex128), staggered.apply(u, p, 0.0), "c64", "D_S rows R sweep")


@pytest.mark.parametrize("dims,tsteps", [((16, 2, 2, 12), "8"), ((12, 4, 2, 18), "8"), ((16, 2, 4, 6), "4"),
                                         ((16, 2, 2, 6), "1"), ((16, 2, 2, 4), "64"), ((20, 2, 2, 34), "16")])
@pytest.mark.parametrize("adj", [False, True])
@pytest.mark.parametrize("dt", ["c64", "c128"])
def test_staggered_march_segments(dims, tsteps, adj, dt, monkeypatch):
    # t-marching D_S (even extents, as the operator requires) over several t
    # segments, a partial last one, one step per workgroup (no carried -t hop),
    # a segment longer than N_t, and chunks of 11 + 9 sites
    nv = 12
    set_knob(monkeypatch, "DSLASH_TSTEPS", tsteps)
    say(f"case staggered march segments {dims} T={tsteps} {dt} adj={adj}")
    u, p = _stag_fields(dims, nv, 75, 76, dt)
    out = D.apply("staggered", up(u, dt), up(p, dt), 0.1, adjoint=adj)
    compare(down(out), staggered.apply(u, p, 0.1, adj), dt, "D_S march segments")


@pytest.mark.parametrize("dt", ["c64", "c128"])
def test_staggered_32to4_nv12_sampled(dt):
    # 32^4, N_v = 12, Haar links (seed 2), rhs seed 102, m = 0: the
    # row-staged kernel at full size against the oracle at sampled sites
    dims, nv = (32, 32, 32, 32), 12
    say(f"case staggered {dims} nv={nv} {dt} sampled")
    u = rounded(synthetic.gauge_links(dims, "haar", 2), dt)
    p = rounded(synthetic.staggered_spinor(dims, nv, 102), dt)
    out = D.apply("staggered", up(u, dt), up(p, dt), 0.0)
    sites = local.sample_sites(dims, 64, 8)
    idx = (sites[:, 3], sites[:, 2], sites[:, 1], sites[:, 0])
    it = torch.as_tensor(np.stack(idx), device=out.device)
    got = out[it[0], it[1], it[2], it[3]].cpu().numpy().astype(np.complex128)
    del out
    torch.cuda.empty_cache()
    compare(got, local.staggered_at(u, p, 0.0, sites), dt, "D_S 32^4 sampled")


@pytest.mark.parametrize("kernel", ["rows", "direct"])
@pytest.mark.parametrize("adj", [False, True])
@pytest.mark.parametrize("dims", [(16, 3, 2, 4), (12, 2, 3, 3), (24, 3, 2, 2), (20, 2, 2, 3)])
def test_brillouin_row_staged_path(kernel, adj, dims, monkeypatch):
    # N_v = 12 in FP32 with rows of >= 12 sites runs the row-staged D_B kernel
    # (27 staged rows per output row, own-site and neighbour-site links);
    # 24 sites split into 12 + 12, 20 sites fall back to the direct kernel
    # (the even split 10 + 10 is below 12 sites); DSLASH_ROWS=0 forces the direct one
    nv, dt = 12, "c64"
    set_knob(monkeypatch, "DSLASH_ROWS", "1" if kernel == "rows" else "0")
    say(f"case brillouin {kernel} {dims} nv={nv} {dt} adj={adj}")
    v = synthetic.gauge_links(dims, "haar", 33)
    w = rounded(brillouin.build(v), dt)
    p = rounded(synthetic.wilson_spinor(dims, nv, 34), dt)
    out = D.apply("brillouin", up(w, dt), up(p, dt), 0.1, adjoint=adj)
    compare(down(out), brillouin.apply(w, p, 0.1, adj), dt, f"D_B {kernel}")


# FP64, N_v = 12, the direct-to-LDS row-staged kernel: one chunk of 16,
# N_y = 2 (the -y and +y rows coincide), chunks of 16 + 4, a chunk of 12, odd
# N_y
@pytest.mark.parametrize("adj", [False, True])
@pytest.mark.parametrize("dims", [(16, 4, 2, 3), (20, 2, 3, 3), (12, 6, 2, 2), (16, 3, 2, 3)])
def test_brillouin_fp64_row_staged(dims, adj):
    nv, dt = 12, "c128"
    say(f"case brillouin fp64 rows {dims} adj={adj}")
    v = synthetic.gauge_links(dims, "haar", 35)
    w = brillouin.build(v)
    p = synthetic.wilson_spinor(dims, nv, 36)
    out = D.apply("brillouin", up(w, dt), up(p, dt), 0.1, adjoint=adj)
    compare(down(out), brillouin.apply(w, p, 0.1, adj), dt, "D_B fp64 rows")


@pytest.mark.parametrize("dt", ["c64", "c128", "bf16", "f16"])
@pytest.mark.parametrize("op", ["wilson", "staggered"])
@pytest.mark.parametrize("compressed", [False, True])
@pytest.mark.parametrize("adj", [False, True])
def test_single_rhs_contiguous_loads(dt, op, compressed, adj):
    # N_v = 1: a site's spinor and links are contiguous runs, which the
    # N_v = 1 form of the direct kernels loads as 16-byte pieces (fields
    # 16-byte aligned, as every torch allocation is)
    if compressed and dt in ("bf16", "f16"):
        pytest.skip("compressed links are stored in C64 and C128")
    dims = (8, 6, 4, 6)
    say(f"case single rhs {op} {dt} compressed={compressed} adj={adj}")
    if op == "wilson":
        u, p = _wil_fields(dims, 1, 93, 94, dt, "haar")
    else:
        u, p = _stag_fields(dims, 1, 93, 94, dt)
    U, P = up(u, dt), up(p, dt)
    mass = 0.1 if op == "wilson" else 0.2
    if compressed:
        ref = (wilson if op == "wilson" else staggered).apply(u, p, mass, adj)
        out = D.apply_compressed(op, D.compress_links(U), P, mass, adjoint=adj)
    else:
        ref = (wilson if op == "wilson" else staggered).apply(u, p, mass, adj)
        out = D.apply(op, U, P, mass, adjoint=adj)
    compare(down(out), ref, dt, f"{op} N_v=1")


@pytest.mark.parametrize("op", ["wilson", "staggered"])
def test_fields_off_16_byte_alignment(op):
    # a field that starts 8 bytes into an allocation takes the per-word
    # kernels (the 16-byte forms require aligned fields) and gives the same
    # result as the aligned field
    dims, dt = (16, 4, 2, 4), "c64"
    say(f"case misaligned fields {op}")
    for nv in (1, 12):
        if op == "wilson":
            u, p = _wil_fields(dims, nv, 95, 96, dt, "haar")
        else:
            u, p = _stag_fields(dims, nv, 95, 96, dt)
        U, P = up(u, dt), up(p, dt)
        flatP = torch.empty(P.numel() + 1, dtype=P.dtype, device=P.device)
        Pm = flatP[1:].view(P.shape)
        Pm.copy_(P)
        flatO = torch.empty_like(flatP)
        Om = flatO[1:].view(P.shape)
        assert Pm.data_ptr() % 16 == 8 and Om.data_ptr() % 16 == 8
        aligned = D.apply(op, U, P, 0.1)
        D.apply(op, U, Pm, 0.1, out=Om)
        ref = (wilson if op == "wilson" else staggered).apply(u, p, 0.1)
        compare(down(Om), ref, dt, f"{op} misaligned nv={nv}")
        compare(down(aligned), ref, dt, f"{op} aligned nv={nv}")


@pytest.mark.parametrize("dt", ["c64", "c128"])
def test_staggered_march_tile_orders(dt, monkeypatch):
    # the D_S march's workgroups in (y, z) tiles (default: eight tiles, here
    # 1 x 3), other tiles and the plain order ("0"): the same arithmetic per
    # workgroup, so the same bits; 20-site rows in two chunks, t segments of 4
    # with a short last one
    dims, nv = (20, 4, 6, 10), 12
    u, p = _stag_fields(dims, nv, 95, 96, dt)
    U, P = up(u, dt), up(p, dt)
    set_knob(monkeypatch, "DSLASH_ROWS", "2")
    set_knob(monkeypatch, "DSLASH_TSTEPS", "4")
    outs = []
    for by, bz in ((None, None), ("1", "1"), ("4", "2"), ("2", "6"), ("0", "0")):
        set_knob(monkeypatch, "DSLASH_MARCH_TILE_Y", by)
        set_knob(monkeypatch, "DSLASH_MARCH_TILE_Z", bz)
        say(f"case staggered march tile {by} x {bz} {dt}")
        outs.append(D.apply("staggered", U, P, 0.05).cpu())
    for o in outs[1:]:
        assert torch.equal(o, outs[0])
    compare(outs[0].numpy().astype(np.complex128), staggered.apply(u, p, 0.05), dt, "D_S march tile orders")


@pytest.mark.parametrize("dt", ["c64", "c128"])
def test_brillouin_tile_orders(dt, monkeypatch):
    # the D_B row kernels' chunks in (y, z) tiles (default here: the whole
    # 6 x 4 plane in FP32, 3 x 4 in FP64), other tiles and the t-band order
    # ("0"): the
    # same arithmetic per chunk, so the same bits; FP32 in chunks of 12 + 12,
    # FP64 (direct-to-LDS kernel) in 16 + 8
    dims, nv = (24, 6, 4, 3), 12
    v = synthetic.gauge_links(dims, "haar", 37)
    w = rounded(brillouin.build(v), dt)
    p = rounded(synthetic.wilson_spinor(dims, nv, 38), dt)
    W, P = up(w, dt), up(p, dt)
    set_knob(monkeypatch, "DSLASH_ROWS", "2")
    outs = []
    for by, bz in ((None, None), ("2", "2"), ("3", "1"), ("1", "4"), ("0", "0")):
        set_knob(monkeypatch, "DSLASH_BRI_TILE_Y", by)
        set_knob(monkeypatch, "DSLASH_BRI_TILE_Z", bz)
        say(f"case brillouin tile {by} x {bz} {dt}")
        outs.append(D.apply("brillouin", W, P, 0.1).cpu())
    for o in outs[1:]:
        assert torch.equal(o, outs[0])
    compare(outs[0].numpy().astype(np.complex128), brillouin.apply(w, p, 0.1), dt, "D_B tile orders")


@pytest.mark.parametrize("dt", ["c64", "bf16"])
def test_wilson_march_tile_orders(dt, monkeypatch):
    # the D_W march's workgroups in (y, z) tiles (the default when the grid
    # runs in several rounds; forced here), other tiles and the plane order:
    # the same arithmetic per workgroup, so the same bits; 4-step segments
    # with a short last one
    dims, nv = (16, 4, 6, 10), 12
    u, p = _wil_fields(dims, nv, 97, 98, dt)
    U, P = up(u, dt), up(p, dt)
    set_knob(monkeypatch, "DSLASH_ROWS", "2")
    set_knob(monkeypatch, "DSLASH_TSTEPS", "4")
    outs = []
    for by, bz in (("0", "0"), ("2", "3"), ("4", "2"), ("1", "1"), ("1", "3")):
        set_knob(monkeypatch, "DSLASH_WMARCH_TILE_Y", by)
        set_knob(monkeypatch, "DSLASH_WMARCH_TILE_Z", bz)
        say(f"case wilson march tile {by} x {bz} {dt}")
        outs.append(D.apply("wilson", U, P, 0.1).cpu())
    for o in outs[1:]:
        assert torch.equal(o, outs[0])
    compare(down(outs[0]), wilson.apply(u, p, 0.1), dt, "D_W march tile orders")
