"""GPU backward pass: link gradient and grad_in against the oracle, autograd
gradcheck, and exact finite differences at the full 24^3 x 48 workload."""
import numpy as np
import pytest

import synthetic
from oracle import grad, local, staggered, wilson
from tests.gpu_util import compare, down, rounded, say, set_knob, up
from tests.helpers import grad_rows_cover

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_1808_05506_amd import dslash as D  # noqa: E402


def _fields(op, dims, nv, seed, dt, kind="haar"):
    u = rounded(synthetic.gauge_links(dims, kind, seed), dt)
    gen = synthetic.staggered_spinor if op == "staggered" else synthetic.wilson_spinor
    chi = rounded(gen(dims, nv, seed + 1), dt)
    psi = rounded(gen(dims, nv, seed + 2), dt)
    return u, chi, psi


@pytest.mark.parametrize("dt", ["c64", "c128"])
@pytest.mark.parametrize("op", ["staggered", "wilson"])
@pytest.mark.parametrize("dims,nv", [((4, 6, 2, 4), 3), ((6, 2, 4, 2), 13), ((2, 4, 2, 2), 70)])
def test_backward_matches_oracle(dt, op, dims, nv):
    say(f"case backward {op} {dims} nv={nv} {dt}")
    u, chi, psi = _fields(op, dims, nv, 100, dt)
    gU, gin = D.backward(op, up(u, dt), up(chi, dt), up(psi, dt), 0.3)
    compare(down(gU), grad.link_grad(op, chi, psi), dt, f"grad_U {op}")
    adj = staggered.apply(u, chi, 0.3, True) if op == "staggered" else wilson.apply(u, chi, 0.3, True)
    compare(down(gin), adj, dt, f"grad_in {op}")


@pytest.mark.parametrize("op", ["staggered", "wilson"])
@pytest.mark.parametrize("adjoint", [False, True])
def test_autograd_gradcheck(op, adjoint):
    say(f"case gradcheck {op} adjoint={adjoint}")
    dims, nv = (4, 2, 2, 2), 2
    u, chi, psi = _fields(op, dims, nv, 200, "c128")
    U = up(u, "c128").requires_grad_(True)
    P = up(psi, "c128").requires_grad_(True)
    fn = lambda a, b: D.dslash(op, a, b, 0.2, adjoint)
    assert torch.autograd.gradcheck(fn, (U, P), eps=1e-6, atol=1e-7, rtol=1e-6, fast_mode=True)


@pytest.mark.parametrize("entry", ["dslash", "apply"])
@pytest.mark.parametrize("op", ["staggered", "wilson"])
def test_autograd_loss_gradient(op, entry):
    # L = Re sum conj(chi) (D psi): torch's gradient equals the oracle's link
    # gradient, through dslash and through apply on inputs that require grad
    say(f"case autograd loss {op} via {entry}")
    dims, nv = (4, 4, 2, 2), 3
    u, chi, psi = _fields(op, dims, nv, 300, "c128")
    U = up(u, "c128").requires_grad_(True)
    P = up(psi, "c128").requires_grad_(True)
    C = up(chi, "c128")
    L = (C.conj() * getattr(D, entry)(op, U, P, 0.1)).real.sum()
    L.backward()
    compare(down(U.grad), grad.link_grad(op, chi, psi), "c128", f"autograd grad_U {op}")
    adj = staggered.apply(u, chi, 0.1, True) if op == "staggered" else wilson.apply(u, chi, 0.1, True)
    compare(down(P.grad), adj, "c128", f"autograd grad_psi {op}")


@pytest.mark.parametrize("op,kind,seed", [("staggered", "haar", 4), ("wilson", "smooth", 5)])
def test_link_grad_24cube48_nv12(op, kind, seed):
    # full workload: 24^3 x 48, N_v = 12, FP32; chi, psi Gaussian (seeds 104/105)
    dims, nv, dt = (24, 24, 24, 48), 12, "c64"
    say(f"case link grad {op} {dims} nv={nv} {dt}")
    u = rounded(synthetic.gauge_links(dims, kind, seed), dt)
    gen = synthetic.staggered_spinor if op == "staggered" else synthetic.wilson_spinor
    chi = rounded(gen(dims, nv, 104), dt)
    psi = rounded(gen(dims, nv, 105), dt)
    gU, _ = D.backward(op, up(u, dt), up(chi, dt), up(psi, dt), 0.0, need_grad_in=False)
    G = down(gU)
    del gU
    # oracle gradient at sampled links
    sites = local.sample_sites(dims, 64, 9)
    idx = (sites[:, 3], sites[:, 2], sites[:, 1], sites[:, 0])
    ref = np.stack([local.link_grad_at(op, chi, psi, sites, mu) for mu in range(4)], axis=1)
    compare(G[idx], ref, dt, f"grad_U {op} 24^3x48 sampled")
    # exact central differences on 16 random link entries (seed 200)
    g = np.random.Generator(np.random.PCG64(200))
    links = [(int(g.integers(dims[3])), int(g.integers(dims[2])), int(g.integers(dims[1])),
              int(g.integers(dims[0])), int(g.integers(4)), int(g.integers(3)), int(g.integers(3)))
             for _ in range(16)]
    fd = np.array([local.fd_link_grad_local(op, u, chi, psi, 0.0, l) for l in links])
    got = np.array([G[l] for l in links])
    scale = np.sqrt(np.mean(np.abs(ref) ** 2))
    err = np.abs(got - fd)
    say(f"FD 16 links: max |GPU - FD| = {err.max():.3e} (rms grad {scale:.3e})")
    assert np.all(err <= 1e-5 * (np.abs(fd) + scale))


_ROW_DIMS_W = [(16, 4, 2, 6), (20, 3, 4, 5), (11, 2, 2, 3), (12, 2, 2, 3), (32, 2, 3, 2)]
_ROW_DIMS_S = [(16, 4, 2, 6), (20, 2, 4, 6), (12, 2, 2, 4), (14, 2, 2, 2), (32, 2, 2, 2)]  # D_S: even extents


@pytest.mark.parametrize("nv", [4, 8, 12, 16, 24])
@pytest.mark.parametrize("op,dt,dims", [("wilson", "c64", d) for d in _ROW_DIMS_W]
                         + [("staggered", dt, d) for dt in ("c64", "c128") for d in _ROW_DIMS_S])
def test_link_grad_row_staged_path(op, dt, dims, nv, monkeypatch):
    # the LDS row-staged gradient kernel (D_W in C64, D_S in C64 and C128) at
    # every block size it is built for, required (DSLASH_ROWS=2) where the
    # launch rule covers the row: 20 sites split into 11 + 9 (N_v = 12) or
    # 10 + 10, 32 into 16 + 16 or 32 at N_v = 4, 11 to 16 fill one chunk with
    # the wrap-around halo; rows the rule leaves out take the direct kernel
    covered = grad_rows_cover(dims[0], nv, op, dt)
    say(f"case link grad rows {op} {dims} nv={nv} {dt} rows={covered}")
    u, chi, psi = _fields(op, dims, nv, 400, dt)
    if covered:
        set_knob(monkeypatch, "DSLASH_ROWS", "2")
    gU, _ = D.backward(op, up(u, dt), up(chi, dt), up(psi, dt), 0.2, need_grad_in=False)
    compare(down(gU), grad.link_grad(op, chi, psi), dt, f"grad_U rows {op}")


@pytest.mark.parametrize("op", ["wilson", "staggered"])
def test_link_grad_rows_determinism_across_chunk_sizes(op, monkeypatch):
    dims, nv, dt = (22, 4, 2, 4), 12, "c64"
    u, chi, psi = _fields(op, dims, nv, 410, dt)
    U, C, P = up(u, dt), up(chi, dt), up(psi, dt)
    outs = []
    for r in ("12", "16", "21"):
        set_knob(monkeypatch, "DSLASH_ROW_SITES", r)
        say(f"case link grad rows determinism {op} R={r}")
        outs.append(D.backward(op, U, C, P, 0.0, need_grad_in=False)[0].cpu())
    for o in outs[1:]:
        assert torch.equal(o, outs[0])
    compare(outs[0].numpy().astype(np.complex128), grad.link_grad(op, chi, psi), dt, f"grad_U rows R sweep {op}")


def test_link_grad_wilson_tile_orders(monkeypatch):
    # the D_W gradient's chunk order in (y, z) tiles (the default: 6 x 2 here)
    # against other tiles and the t-band order ("0"): the same arithmetic per
    # chunk, so the same bits, over several tiles and 10 + 10 site chunks
    dims, nv, dt = (20, 6, 4, 5), 12, "c64"
    u, chi, psi = _fields("wilson", dims, nv, 420, dt)
    U, C, P = up(u, dt), up(chi, dt), up(psi, dt)
    set_knob(monkeypatch, "DSLASH_ROWS", "2")
    outs = []
    for by, bz in ((None, None), ("3", "2"), ("2", "4"), ("6", "1"), ("1", "1"), ("0", "0")):
        set_knob(monkeypatch, "DSLASH_GRAD_TILE_Y", by)
        set_knob(monkeypatch, "DSLASH_GRAD_TILE_Z", bz)
        say(f"case link grad wilson tile {by} x {bz}")
        outs.append(D.backward("wilson", U, C, P, 0.0, need_grad_in=False)[0].cpu())
    for o in outs[1:]:
        assert torch.equal(o, outs[0])
    compare(outs[0].numpy().astype(np.complex128), grad.link_grad("wilson", chi, psi), dt, "grad_U tile orders")
