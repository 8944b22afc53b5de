"""The Python example of the README runs as written: one ray through a solid
50^3 block of a 128^3 grid gives exactly the lattice points inside the block
(worked out in binary32 from the block's dyadic planes), the composite
differentiates, and a refresh with the same occupancy (given directly, or as a
density cache) changes nothing."""
import numpy as np
import pytest
import torch

from paper_2404_10272_amd import api

pytestmark = pytest.mark.gpu


def test_readme_example():
    occ = torch.zeros((1, 128, 128, 128), dtype=torch.uint8, device="cuda")
    occ[0, 40:90, 40:90, 40:90] = 1
    boxes = [[-1.5, -1.5, -1.5, 1.5, 1.5, 1.5]]
    grid = api.build_vdb(occ, boxes, internal_log2=4)
    o = torch.tensor([[0.0, 0.0, -4.0]], device="cuda")
    d = torch.tensor([[0.0, 0.0, 1.0]], device="cuda")
    out = api.sample_rays(grid, o, d, near=2.0, far=6.0, step=api.make_step("const", dt=5e-3))
    t0 = out["t0"].cpu().numpy()
    S = int(out["offsets"][-1].item())
    # The block's planes z = -1.5 + m*3/128 (m = 40, 90) are dyadic, so the ray
    # (o_z = -4, d_z = 1) crosses them exactly at t = 3.4375 and 4.609375, and
    # the samples are the lattice points t_n = fl(2 + fl(n * 5e-3)) in that
    # interval (upper end included), in binary32.
    dt = np.float32(5e-3)
    n = np.arange(1000, dtype=np.float32)
    lat = np.float32(2.0) + n * dt
    sel = n[(lat > np.float32(3.4375)) & (lat <= np.float32(4.609375))]
    assert S == sel.size == 234
    np.testing.assert_array_equal(t0, np.float32(2.0) + sel * dt)
    np.testing.assert_array_equal(out["t1"].cpu().numpy(), np.float32(2.0) + (sel + np.float32(1.0)) * dt)
    assert np.all(out["ray_ids"].cpu().numpy() == 0)
    sigma = torch.rand(S, device="cuda", requires_grad=True)
    rgb = torch.rand(S, 3, device="cuda", requires_grad=True)
    C, A = api.composite(sigma, rgb, out["offsets"], out["t0"], out["t1"])
    C.sum().backward()
    assert torch.isfinite(sigma.grad).all() and 0 < A.item() <= 1
    grid.refresh(occ)
    out2 = api.sample_rays(grid, o, d, near=2.0, far=6.0, step=api.make_step("const", dt=5e-3))
    assert torch.equal(out2["t0"], out["t0"])
    # the density-cache refresh with the occupancy as density leaves the same grid
    cache = torch.zeros(occ.shape, device="cuda")
    grid.refresh_density(cache, density=occ.float(), decay=0.95, threshold=0.01)
    assert torch.equal(cache, occ.float())
    out3 = api.sample_rays(grid, o, d, near=2.0, far=6.0, step=api.make_step("const", dt=5e-3))
    assert torch.equal(out3["t0"], out["t0"])
