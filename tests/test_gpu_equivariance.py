"""Right-hand-side permutation equivariance: the N_v columns of a block are
independent vectors (the paper's N_v right-hand sides, Sec. 2), so applying
an operator to the columns in another order must give the same columns in
that order.  Every kernel computes each column with the same arithmetic in
the same order, so the forward operators are checked bitwise; the link
gradient sums over the columns, so a joint permutation of chi and psi may
change only its rounding."""
import numpy as np
import pytest

import synthetic
from tests.gpu_util import up, say

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_1808_05506_amd import dslash as D  # noqa: E402

# (op, dims, N_v, link kind): the N_v = 12 cases take the row-staged kernels
CASES = [
    ("staggered", (16, 4, 4, 8), 12, "haar"),
    ("staggered", (6, 4, 2, 4), 5, "haar"),
    ("wilson", (16, 4, 4, 8), 12, "smooth"),
    ("wilson", (5, 3, 4, 3), 7, "haar"),
    ("brillouin", (12, 4, 4, 4), 12, "haar"),
    ("brillouin", (4, 3, 3, 3), 3, "haar"),
]


def _fields(op, dims, nv, kind, seed):
    u = synthetic.gauge_links(dims, kind, seed)
    gen = synthetic.staggered_spinor if op == "staggered" else synthetic.wilson_spinor
    return u, gen(dims, nv, seed + 1)


@pytest.mark.parametrize("dt", ["c64", "c128"])
@pytest.mark.parametrize("adj", [False, True])
@pytest.mark.parametrize("op,dims,nv,kind", CASES)
def test_rhs_permutation_bitwise(op, dims, nv, kind, dt, adj):
    say(f"case equivariance {op} {dims} nv={nv} {dt} adj={adj}")
    u, p = _fields(op, dims, nv, kind, 300)
    U = up(u, dt)
    if op == "brillouin":
        U = D.brillouin_links(U)
    P = up(p, dt)
    perm = torch.from_numpy(np.random.Generator(np.random.PCG64(nv)).permutation(nv)).to(P.device)
    out = D.apply(op, U, P, 0.1 if op != "staggered" else 0.0, adjoint=adj)
    out_p = D.apply(op, U, P[..., perm].contiguous(), 0.1 if op != "staggered" else 0.0, adjoint=adj)
    assert torch.equal(out_p, out[..., perm])


@pytest.mark.parametrize("op", ["staggered", "wilson"])
def test_link_gradient_invariant_under_joint_permutation(op):
    dims, nv = (16, 4, 4, 8), 12
    say(f"case gradient permutation {op}")
    u, c = _fields(op, dims, nv, "haar", 310)
    _, p = _fields(op, dims, nv, "haar", 320)
    U, C, P = up(u, "c64"), up(c, "c64"), up(p, "c64")
    perm = torch.arange(nv - 1, -1, -1, device=P.device)
    g, _ = D.backward(op, U, C, P, 0.0, need_grad_in=False)
    gp, _ = D.backward(op, U, C[..., perm].contiguous(), P[..., perm].contiguous(), 0.0, need_grad_in=False)
    rel = float(torch.linalg.vector_norm(gp - g) / torch.linalg.vector_norm(g))
    say(f"relative change {rel:.2e}")
    assert rel <= 1e-6
