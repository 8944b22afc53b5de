"""ogv_sample_rays_noalloc (the entry point for callers that cannot allocate:
its workspace is the library's static per-device scratch array) against
ogv_sample_rays with a caller-allocated workspace, through the C-ABI.

Three calls in a row on the same device scratch, each smaller than the one
before or on another lattice: 300,000 object-scene rays (VDB, image lanes),
99,840 four-cascade rays (growing step, whose table lives in the scratch),
then the 4,096-ray small workload; the output must equal the existing entry
point's bit for bit each time, and the small one the oracle's too.  Also: an
exact and a too-small capacity, and a call too large for the scratch
rejected before any work."""
import numpy as np
import pytest
import torch

import oracle
from paper_2404_10272_amd import api, scenes

pytestmark = pytest.mark.gpu


def _noalloc(g, o, d, w, variant, width, cap):
    n = o.shape[0]
    offsets = torch.full((n + 1,), -3, dtype=torch.int64, device="cuda")
    ids = torch.full((cap + 8,), -7, dtype=torch.int32, device="cuda")
    t0 = torch.full((cap + 8,), -1.0, device="cuda")
    t1 = torch.full((cap + 8,), -1.0, device="cuda")
    overflow = torch.full((1,), 9, dtype=torch.int32, device="cuda")
    api.sample_rays_noalloc(g, o, d, w.near, w.far, w.step, offsets, ids[:cap], t0[:cap], t1[:cap], overflow,
                            variant, image_width=width)
    torch.cuda.synchronize()
    return offsets, ids, t0, t1, overflow


def _with_workspace(g, o, d, w, variant, width, cap):
    sp = api.Sampler(g, o.shape[0], w.near, w.far, w.step, variant, image_width=width)
    ids = torch.full((cap,), -7, dtype=torch.int32, device="cuda")
    t0 = torch.full((cap,), -1.0, device="cuda")
    t1 = torch.full((cap,), -1.0, device="cuda")
    offsets, overflow = sp.rays(o, d, ids, t0, t1)
    torch.cuda.synchronize()
    return offsets.clone(), ids, t0, t1, overflow.clone()


def _case(name, rows):
    w = scenes.workload(name)
    n = rows * w.image[0]
    o = torch.from_numpy(np.ascontiguousarray(w.origins[:n])).cuda()
    d = torch.from_numpy(np.ascontiguousarray(w.dirs[:n])).cuda()
    occ = torch.from_numpy(w.occ).cuda()
    return w, o, d, api.build_vdb(occ, w.boxes, w.ilog2)


def _check(w, o, d, g, variant, width):
    ref = _with_workspace(g, o, d, w, variant, width, 1)        # sizes the output
    S = int(ref[0][-1].item())
    ref = _with_workspace(g, o, d, w, variant, width, S)
    got = _noalloc(g, o, d, w, variant, width, S)
    for k, (a, b) in enumerate(zip(got[:4], ref[:4])):
        a = a[:b.numel()] if k > 0 else a
        assert torch.equal(a, b), f"{w.name} output {k} differs from ogv_sample_rays"
    assert int(got[4].item()) == 0 and int(ref[4].item()) == 0
    assert bool((got[1][S:] == -7).all()), "wrote past the capacity"
    # a too-small capacity: flagged, offsets complete, nothing past it written
    cap = S // 3
    small = _noalloc(g, o, d, w, variant, width, cap)
    assert int(small[4].item()) == 1
    assert torch.equal(small[0], ref[0])
    assert torch.equal(small[2][:cap], ref[2][:cap])
    assert bool((small[1][cap:] == -7).all())
    return S, got


def test_noalloc_matches_sample_rays_over_calls_of_shrinking_size():
    n = []
    w, o, d, g = _case("object", 375)          # 300,000 rays
    S1, _ = _check(w, o, d, g, "branch", w.image[0])
    n.append(o.shape[0])
    print("object", o.shape[0], S1, flush=True)
    w, o, d, g = _case("unbounded", 78)        # 99,840 rays, growing step
    S2, _ = _check(w, o, d, g, "skip", w.image[0])
    n.append(o.shape[0])
    print("unbounded", o.shape[0], S2, flush=True)
    w, o, d, g = _case("small", 64)            # 4,096 rays
    S3, got = _check(w, o, d, g, "branch", 0)
    n.append(o.shape[0])
    print("small", o.shape[0], S3, flush=True)
    assert n[0] > n[1] > n[2] and min(S1, S2, S3) > 0
    ref = oracle.sample_rays(oracle.Scene(w.occ, w.boxes), w.origins, w.dirs, w.near, w.far, w.step,
                             "dense_branch")
    np.testing.assert_array_equal(got[0].cpu().numpy(), ref["offsets"])
    np.testing.assert_array_equal(got[1][:S3].cpu().numpy(), ref["ray_ids"])
    np.testing.assert_array_equal(got[2][:S3].cpu().numpy(), ref["t0"])
    np.testing.assert_array_equal(got[3][:S3].cpu().numpy(), ref["t1"])


def test_noalloc_rejects_a_call_larger_than_its_scratch():
    w, _, _, g = _case("small", 1)
    n = 2_000_000                               # about 300 MB of workspace
    o = torch.zeros((n, 3), device="cuda")
    d = torch.ones((n, 3), device="cuda")
    need = api.workspace_bytes(n, w.near, w.far, api.make_step(w.step))
    assert need > api.NOALLOC_SCRATCH_BYTES
    offsets = torch.full((n + 1,), -3, dtype=torch.int64, device="cuda")
    buf = torch.zeros(16, device="cuda")
    ids = torch.zeros(16, dtype=torch.int32, device="cuda")
    overflow = torch.zeros(1, dtype=torch.int32, device="cuda")
    with pytest.raises(api.OgvError, match="static scratch"):
        api.sample_rays_noalloc(g, o, d, w.near, w.far, w.step, offsets, ids, buf, buf, overflow)
    torch.cuda.synchronize()
    assert bool((offsets == -3).all()), "a rejected call must do nothing"
