"""GPU parity of the clover term (build from the links, and D_W / D_B with the
term added) against the oracle, through the C ABI."""
import numpy as np
import pytest

import synthetic
from oracle import brillouin, clover, wilson
from tests.gpu_util import compare, down, rounded, say, up, set_knob

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_1808_05506_amd import dslash as D  # noqa: E402

C_SW = 1.3


@pytest.mark.parametrize("dt", ["c64", "c128", "bf16", "f16"])
@pytest.mark.parametrize("dims,kind", [((4, 4, 2, 4), "haar"), ((6, 2, 3, 5), "haar"), ((16, 4, 2, 4), "smooth")])
def test_clover_field_matches_oracle(dt, dims, kind):
    say(f"case clover field {dims} {kind} {dt}")
    v = rounded(synthetic.gauge_links(dims, kind, 81), dt)
    C = D.clover_field(up(v, dt), C_SW)
    compare(down(C), clover.pack(clover.term(v, C_SW)), dt, "clover field")


def test_clover_field_zero_csw_and_unit_links():
    dims = (4, 2, 2, 4)
    v = synthetic.gauge_links(dims, "haar", 82)
    assert torch.count_nonzero(D.clover_field(up(v, "c64"), 0.0)) == 0
    u = synthetic.gauge_links(dims, "unit", 0)
    assert torch.count_nonzero(D.clover_field(up(u, "c128"), C_SW)) == 0


# Wilson: N_v = 3 and FP64 take the direct kernel; N_v = 12 with FP32
# arithmetic the row-staged one (rows of 16 sites; two chunks of 13).
@pytest.mark.parametrize("dt", ["c64", "c128", "bf16", "f16"])
@pytest.mark.parametrize("adj", [False, True])
@pytest.mark.parametrize("dims,nv", [((4, 4, 2, 4), 3), ((16, 4, 2, 4), 12), ((26, 2, 2, 2), 12)])
def test_wilson_clover_matches_oracle(dt, adj, dims, nv):
    say(f"case wilson clover {dims} nv={nv} {dt} adj={adj}")
    v = rounded(synthetic.gauge_links(dims, "smooth", 83), dt)
    p = rounded(synthetic.wilson_spinor(dims, nv, 84), dt)
    c = rounded(clover.pack(clover.term(v, C_SW)), dt)
    out = D.apply("wilson", up(v, dt), up(p, dt), 0.1, adjoint=adj, clover=up(c, dt))
    ref = wilson.apply(v, p, 0.1, adj) + clover.apply_term(clover.unpack(c), p)
    compare(down(out), ref, dt, "D_W + C")


# Brillouin: row-staged for N_v = 12 C64 with rows of at least 12 sites
# (one chunk of 13; two chunks of 12), the direct kernel otherwise.
@pytest.mark.parametrize("dt", ["c64", "c128", "bf16"])
@pytest.mark.parametrize("adj", [False, True])
@pytest.mark.parametrize("dims,nv", [((4, 3, 2, 3), 2), ((13, 3, 2, 3), 12), ((24, 2, 3, 2), 12)])
def test_brillouin_clover_matches_oracle(dt, adj, dims, nv):
    say(f"case brillouin clover {dims} nv={nv} {dt} adj={adj}")
    v = synthetic.gauge_links(dims, "haar", 85)
    w = rounded(brillouin.build(v), dt)
    p = rounded(synthetic.wilson_spinor(dims, nv, 86), dt)
    c = rounded(clover.pack(clover.term(v, C_SW)), dt)
    out = D.apply("brillouin", up(w, dt), up(p, dt), 0.1, adjoint=adj, clover=up(c, dt))
    ref = brillouin.apply(w, p, 0.1, adj) + clover.apply_term(clover.unpack(c), p)
    compare(down(out), ref, dt, "D_B + C")


@pytest.mark.parametrize("op", ["wilson", "brillouin"])
def test_clover_end_to_end_c128(op):
    # links -> clover field on the GPU -> (D + C) psi, against the oracle's operator
    dims, nv = (4, 4, 2, 4), 2
    say(f"case clover end to end {op}")
    v = synthetic.gauge_links(dims, "haar", 87)
    p = synthetic.wilson_spinor(dims, nv, 88)
    V = up(v, "c128")
    C = D.clover_field(V, C_SW)
    if op == "wilson":
        out = D.apply(op, V, up(p, "c128"), 0.05, clover=C)
        ref = clover.wilson_apply(v, p, 0.05, C_SW)
    else:
        out = D.apply(op, D.brillouin_links(V), up(p, "c128"), 0.05, clover=C)
        ref = clover.brillouin_apply(v, brillouin.build(v), p, 0.05, C_SW)
    compare(down(out), ref, "c128", f"{op} + clover end to end")


def test_row_staged_clover_equals_direct(monkeypatch):
    dims, nv, dt = (16, 4, 2, 4), 12, "c64"
    say("case wilson clover rows vs direct")
    V = up(synthetic.gauge_links(dims, "smooth", 89), dt)
    P = up(synthetic.wilson_spinor(dims, nv, 90), dt)
    C = D.clover_field(V, C_SW)
    rows = D.apply("wilson", V, P, 0.1, clover=C)
    set_knob(monkeypatch, "DSLASH_ROWS", "0")
    direct = D.apply("wilson", V, P, 0.1, clover=C)
    torch.cuda.synchronize()
    compare(down(rows), down(direct), dt, "rows vs direct")


def test_clover_rejects_staggered_and_bad_shape():
    dims = (4, 2, 2, 4)
    V = up(synthetic.gauge_links(dims, "haar", 91), "c64")
    P = up(synthetic.staggered_spinor(dims, 2, 92), "c64")
    C = D.clover_field(V, C_SW)
    with pytest.raises(D.DslashError):
        D.apply("staggered", V, P, 0.0, clover=C)
    W = up(synthetic.wilson_spinor(dims, 2, 93), "c64")
    with pytest.raises(ValueError):
        D.apply("wilson", V, W, 0.1, clover=C[..., :1, :])
