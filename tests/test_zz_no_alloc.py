"""The allocation-free constraints entry point (chemora_constraints_noalloc,
partial sums in a static device buffer) against chemora_constraints with a
caller workspace, through the C ABI: two calls in a row on one GPU, the
second on a smaller grid (the buffer keeps the first call's partials), each
bitwise equal in the norms and the H, M^i fields."""
import numpy as np
import pytest
import torch

from paper_1410_1764_amd import chemora as C
from tests.test_oracle_bssn import _smooth_random

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("order", [4, 6])
def test_constraints_noalloc_matches_workspace_version(order):
    for n, seed in (((70, 40, 17), 3), ((22, 18, 11), 4)):
        g = order // 2 + 1
        gr = C.Grid(n, g, tuple(1.0 / v for v in n), system=C.BSSN, fd_order=order)
        st = gr.upload(_smooth_random(n, seed))
        gr.fill_ghosts(st)
        hm_a = gr.new_state()[: 4 * gr.strides[3]].clone()
        hm_b = hm_a.clone()
        na = gr.constraints(st, hm=hm_a)
        nb = torch.full((4,), np.nan, dtype=torch.float64, device="cuda")
        gr.constraints_noalloc(st, nb, hm=hm_b)
        torch.cuda.synchronize()
        print("noalloc", n, order, na.cpu().numpy(), nb.cpu().numpy(), flush=True)
        assert torch.equal(na, nb)
        assert torch.equal(hm_a, hm_b)
        assert bool(torch.all(nb > 0))
