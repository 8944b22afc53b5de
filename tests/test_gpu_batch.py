"""Batched multi-scene sampling: one graph-captured pass over 16 uneven scenes.

Parity: the batch's CSR equals, scene by scene, the CPU oracle's (reduced ray
images, every full-size ray, and a seeded subset of the full-size rays
against a second oracle method), bit for bit; at full size the CSR also
equals the single-scene path's, a consistency property.  Graph
replays are checked against an eager pass after each replay, with other work
on the stream in between.
"""
import numpy as np
import pytest
import torch

import oracle
from paper_2404_10272_amd import api, scenes

pytestmark = pytest.mark.gpu


def _gpu_scenes(ws, kind="vdb", tiled=True):
    out = []
    for w in ws:
        occ = torch.from_numpy(w.occ).cuda()
        g = api.build_vdb(occ, w.boxes, w.ilog2) if kind == "vdb" else api.build_dense(occ, w.boxes)
        out.append((g, torch.from_numpy(w.origins).cuda(), torch.from_numpy(w.dirs).cuda(), w.near, w.far, w.step,
                    w.image[0] if tiled else 0))
    return out


def _run(batch, graph=True):
    off = batch.offsets
    # count once to size outputs (a first eager pass with capacity 0)
    z = torch.zeros(1, dtype=torch.int32, device="cuda")
    zf = torch.zeros(1, dtype=torch.float32, device="cuda")
    batch.launch(z[:0], zf[:0], zf[:0], graph=False)
    torch.cuda.synchronize()
    S = int(off[-1].item())
    ids = torch.empty(S, dtype=torch.int32, device="cuda")
    t0 = torch.empty(S, dtype=torch.float32, device="cuda")
    t1 = torch.empty(S, dtype=torch.float32, device="cuda")
    offsets, overflow = batch.launch(ids, t0, t1, graph=graph)
    torch.cuda.synchronize()
    assert int(overflow.item()) == 0
    return {"offsets": offsets.cpu().numpy().copy(), "ray_ids": ids.cpu().numpy(), "t0": t0.cpu().numpy(),
            "t1": t1.cpu().numpy()}, (ids, t0, t1)


def _split(res, base, n, s):
    a, b = base[s], base[s] + n
    off = res["offsets"][a:b + 1]
    lo, hi = off[0], off[-1]
    return {"offsets": off - lo, "ray_ids": res["ray_ids"][lo:hi] - a, "t0": res["t0"][lo:hi], "t1": res["t1"][lo:hi]}


def _same(got, ref, what):
    for k in ("offsets", "ray_ids", "t0", "t1"):
        np.testing.assert_array_equal(got[k], ref[k], err_msg=f"{what} {k}")


@pytest.mark.parametrize("kind", ["vdb", "dense"])
def test_batch_matches_oracle_reduced(kind):
    ws = scenes.batched(ray_sides=[s // 8 for s in scenes.BATCH_SIDES])
    ws[3].step = {"kind": "cone", "dt": 0.0, "cone": 1 / 64, "dt_min": 4e-3}   # one growing-step scene
    batch = api.Batch(_gpu_scenes(ws, kind), "skip", tune=(256, 2))
    res, _ = _run(batch)
    base = batch.info()["ray_base"]
    for s, w in enumerate(ws):
        ref = oracle.sample_rays(oracle.Scene(w.occ, w.boxes), w.origins, w.dirs, w.near, w.far, w.step,
                                 "dense_branch")
        ref.pop("voxel_ids")
        print("scene", s, w.R, w.n_rays, flush=True)
        _same(_split(res, base, w.n_rays, s), ref, f"scene {s}")


def test_batch_rejects_voxel_steps():
    # a batch walks each VDB hierarchically; OGV_VOXEL is a single-scene option
    ws = scenes.batched(n_scenes=2, ray_sides=[64, 64])
    for v in ("voxel_branch", "voxel_skip", "subleaf_branch", "subleaf_skip"):
        with pytest.raises(api.OgvError):
            api.Batch(_gpu_scenes(ws), v, tune=(256, 2))


def test_graph_replays_match_eager_and_tunes_agree():
    ws = scenes.batched(ray_sides=[s // 4 for s in scenes.BATCH_SIDES])
    gs = _gpu_scenes(ws)
    tuned = api.Batch(gs, "skip")
    info = tuned.info()
    assert info["tuned"] and info["chunk"] % 256 == 0 and info["blocks_per_cu"] >= 1
    eager, _ = _run(tuned, graph=False)
    S = eager["t0"].size
    ids = torch.empty(S, dtype=torch.int32, device="cuda")
    t0 = torch.empty(S, dtype=torch.float32, device="cuda")
    t1 = torch.empty(S, dtype=torch.float32, device="cuda")
    for rep in range(3):
        for t in (ids, t0, t1):
            t.zero_()
        junk = torch.randn(1 << 20, device="cuda").sum()   # unrelated work between replays
        tuned.launch(ids, t0, t1, graph=True)
        torch.cuda.synchronize()
        got = {"offsets": tuned.offsets.cpu().numpy(), "ray_ids": ids.cpu().numpy(), "t0": t0.cpu().numpy(),
               "t1": t1.cpu().numpy()}
        _same(got, eager, f"replay {rep}")
        del junk
    fixed = api.Batch(gs, "branch", tune=(4096, 8))
    other, _ = _run(fixed)
    _same(other, eager, "fixed tune, branch variant")
    untiled = api.Batch(_gpu_scenes(ws, tiled=False), "skip", tune=(512, 2))
    other, _ = _run(untiled)
    _same(other, eager, "no image tiling")


def test_full_batch_matches_single_scene_calls():
    ws = scenes.batched()
    gs = _gpu_scenes(ws)
    batch = api.Batch(gs, "skip")
    assert batch.n_rays == 5955584
    res, _ = _run(batch)
    base = batch.info()["ray_base"]
    rng = np.random.default_rng(5)
    for s, (w, (g, o, d, near, far, step, width)) in enumerate(zip(ws, gs)):
        bat = _split(res, base, w.n_rays, s)
        # every ray's samples against the oracle (its dense voxel walk, the fastest of its methods)
        full = oracle.sample_rays(oracle.Scene(w.occ, w.boxes), w.origins, w.dirs, w.near, w.far, w.step,
                                  "dense_branch")
        _same(bat, full, f"scene {s}, all rays")
        del full
        # the batch's samples of a seeded subset of rays against the oracle
        pick = np.sort(rng.choice(w.n_rays, size=min(w.n_rays, 1500), replace=False))
        ref = oracle.sample_rays(oracle.Scene(w.occ, w.boxes), w.origins[pick], w.dirs[pick], w.near, w.far, w.step,
                                 "hdda_skip", ilog2=w.ilog2)
        cnt = np.diff(bat["offsets"])[pick]
        np.testing.assert_array_equal(cnt, np.diff(ref["offsets"]), err_msg=f"scene {s} counts")
        for key in ("t0", "t1"):
            got = np.concatenate([bat[key][bat["offsets"][i]:bat["offsets"][i + 1]] for i in pick])
            np.testing.assert_array_equal(got, ref[key], err_msg=f"scene {s} {key}")
        # and, as a consistency property at full size, the same CSR as a single-scene call
        one = api.sample_rays(g, o, d, near, far, api.make_step(step), "skip")
        _same(bat, {k: v.cpu().numpy() for k, v in one.items()}, f"scene {s}")
