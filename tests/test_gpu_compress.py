"""GPU parity of gauge compression (two stored rows per link, the third
completed in the kernels) against the oracle, through the C ABI."""
import numpy as np
import pytest

import synthetic
from oracle import compress
from tests.gpu_util import compare, down, rounded, say, up, set_knob

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_1808_05506_amd import dslash as D  # noqa: E402


@pytest.mark.parametrize("dt", ["c64", "c128", "bf16", "f16"])
def test_compress_links_bit_exact(dt):
    dims = (4, 2, 3, 4)
    v = rounded(synthetic.gauge_links(dims, "haar", 71), dt)
    Vc = D.compress_links(up(v, dt))
    assert np.array_equal(down(Vc), compress.compress(v))


# N_v = 12 at rows of 16 sites (and two chunks of 13) runs the row-staged
# kernels (D_W: t-marching, FP32 arithmetic, half-spinor rows for FP32
# storage; D_S: C64, C128); the rest the direct kernels.
@pytest.mark.parametrize("dt", ["c64", "c128", "bf16", "f16"])
@pytest.mark.parametrize("adj", [False, True])
@pytest.mark.parametrize("dims,nv", [((4, 3, 2, 5), 1), ((6, 4, 2, 4), 3), ((16, 4, 2, 8), 12), ((26, 2, 2, 4), 12)])
def test_wilson_compressed_matches_oracle(dt, adj, dims, nv):
    say(f"case wilson compressed {dims} nv={nv} {dt} adj={adj}")
    vc = rounded(compress.compress(synthetic.gauge_links(dims, "smooth", 72)), dt)
    p = rounded(synthetic.wilson_spinor(dims, nv, 73), dt)
    out = D.apply_compressed("wilson", up(vc, dt), up(p, dt), 0.1, adjoint=adj)
    compare(down(out), compress.apply("wilson", vc, p, 0.1, adj), dt, "D_W compressed")


@pytest.mark.parametrize("pp", ["0", "3"])
@pytest.mark.parametrize("adj", [False, True])
def test_wilson_compressed_march_modes(pp, adj, monkeypatch):
    # FP32 D_W on compressed links through the t-marching kernel over three
    # t segments (8 + 8 + 4) with one row buffer and with half-spinor rows
    dims, nv, dt = (16, 2, 4, 20), 12, "c64"
    set_knob(monkeypatch, "DSLASH_TSTEPS", "8")
    set_knob(monkeypatch, "DSLASH_MARCH_PP", pp)
    say(f"case wilson compressed march pp={pp} adj={adj}")
    vc = rounded(compress.compress(synthetic.gauge_links(dims, "haar", 80)), dt)
    p = rounded(synthetic.wilson_spinor(dims, nv, 81), dt)
    out = D.apply_compressed("wilson", up(vc, dt), up(p, dt), 0.1, adjoint=adj)
    compare(down(out), compress.apply("wilson", vc, p, 0.1, adj), dt, "D_W compressed march")


@pytest.mark.parametrize("dt", ["c64", "c128", "bf16"])
@pytest.mark.parametrize("adj", [False, True])
@pytest.mark.parametrize("dims,nv", [((4, 2, 2, 4), 2), ((16, 4, 2, 4), 12), ((26, 2, 4, 2), 12)])
def test_staggered_compressed_matches_oracle(dt, adj, dims, nv):
    say(f"case staggered compressed {dims} nv={nv} {dt} adj={adj}")
    vc = rounded(compress.compress(synthetic.gauge_links(dims, "haar", 74)), dt)
    p = rounded(synthetic.staggered_spinor(dims, nv, 75), dt)
    out = D.apply_compressed("staggered", up(vc, dt), up(p, dt), 0.05, adjoint=adj)
    compare(down(out), compress.apply("staggered", vc, p, 0.05, adj), dt, "D_S compressed")


@pytest.mark.parametrize("op", ["wilson", "staggered"])
def test_compressed_equals_full_for_su3_links(op):
    # FP64 storage: the completed third row equals the stored one to rounding
    dims, nv = (16, 4, 2, 4), 12
    say(f"case compressed vs full {op}")
    V = up(synthetic.gauge_links(dims, "haar", 76), "c128")
    gen = synthetic.wilson_spinor if op == "wilson" else synthetic.staggered_spinor
    P = up(gen(dims, nv, 77), "c128")
    full = D.apply(op, V, P, 0.1)
    comp = D.apply_compressed(op, D.compress_links(V), P, 0.1)
    compare(down(comp), down(full), "c128", f"{op} compressed vs full")


def test_compressed_rejects_brillouin():
    dims = (4, 2, 2, 4)
    V = up(synthetic.gauge_links(dims, "haar", 78), "c64")
    P = up(synthetic.wilson_spinor(dims, 2, 79), "c64")
    with pytest.raises(ValueError):
        D.apply_compressed("brillouin", D.compress_links(V), P, 0.1)
