"""GPU parity of D_B with the off-axis links built on the fly from V (no W
array) against the oracle, through the C ABI."""
import numpy as np
import pytest

import synthetic
from oracle import brillouin, local
from tests.gpu_util import compare, down, rounded, say, up

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_1808_05506_amd import dslash as D  # noqa: E402


# rows of 12 sites (one chunk), 13 (one chunk) and two chunks of 13
@pytest.mark.parametrize("adj", [False, True])
@pytest.mark.parametrize("dims", [(12, 3, 2, 3), (13, 2, 3, 3), (26, 3, 2, 2)])
def test_fly_matches_oracle(adj, dims):
    say(f"case brillouin fly {dims} adj={adj}")
    v = rounded(synthetic.gauge_links(dims, "haar", 160), "c64")
    p = rounded(synthetic.wilson_spinor(dims, 12, 161), "c64")
    out = D.apply_brillouin_fly(up(v, "c64"), up(p, "c64"), 0.1, adjoint=adj)
    compare(down(out), brillouin.apply(brillouin.build(v), p, 0.1, adj), "c64", "D_B fly")


# (N_v, rows): one chunk of 16 at N_v = 4, 8, 16; chunks of 8 at N_v = 24;
# 24-site rows in chunks of 12 or 8; one chunk of 20 at N_v = 4 (80 threads,
# the second wave partly filled)
@pytest.mark.parametrize("adj", [False, True])
@pytest.mark.parametrize("nv,dims", [(4, (16, 3, 2, 3)), (8, (16, 2, 3, 3)), (16, (16, 3, 2, 2)),
                                     (24, (16, 2, 2, 3)), (8, (24, 2, 2, 3)), (24, (24, 2, 3, 2)),
                                     (4, (20, 2, 2, 3))])
def test_fly_other_block_sizes(nv, dims, adj):
    say(f"case brillouin fly {dims} nv={nv} adj={adj}")
    v = rounded(synthetic.gauge_links(dims, "haar", 170 + nv), "c64")
    p = rounded(synthetic.wilson_spinor(dims, nv, 171 + nv), "c64")
    out = D.apply_brillouin_fly(up(v, "c64"), up(p, "c64"), 0.1, adjoint=adj)
    compare(down(out), brillouin.apply(brillouin.build(v), p, 0.1, adj), "c64", f"D_B fly nv={nv}")


def test_fly_equals_stored_w():
    dims = (16, 4, 4, 4)
    say("case brillouin fly vs stored W")
    V = up(synthetic.gauge_links(dims, "haar", 162), "c64")
    P = up(synthetic.wilson_spinor(dims, 12, 163), "c64")
    fly = D.apply_brillouin_fly(V, P, 0.1)
    stored = D.apply("brillouin", D.brillouin_links(V), P, 0.1)
    compare(down(fly), down(stored), "c64", "fly vs stored")


def test_fly_32to4_sampled():
    # the D_B benchmark workload: 32^4, N_v = 12, Haar links (seed 2), rhs seed 102
    dims, nv = (32, 32, 32, 32), 12
    say("case brillouin fly 32^4 sampled")
    v = rounded(synthetic.gauge_links(dims, "haar", 2), "c64")
    p = rounded(synthetic.wilson_spinor(dims, nv, 102), "c64")
    out = D.apply_brillouin_fly(up(v, "c64"), up(p, "c64"), 0.1)
    sites = local.sample_sites(dims, 32, 9)
    it = torch.as_tensor(np.stack((sites[:, 3], sites[:, 2], sites[:, 1], sites[:, 0])), device=out.device)
    got = out[it[0], it[1], it[2], it[3]].cpu().numpy().astype(np.complex128)
    del out
    torch.cuda.empty_cache()
    compare(got, local.brillouin_at(v, p, 0.1, sites), "c64", "D_B fly 32^4 sampled")


def test_fly_unsupported_configuration():
    dims = (8, 4, 4, 4)
    V = up(synthetic.gauge_links(dims, "haar", 164), "c64")
    P = up(synthetic.wilson_spinor(dims, 12, 165), "c64")
    with pytest.raises(D.DslashError):
        D.apply_brillouin_fly(V, P, 0.1)
