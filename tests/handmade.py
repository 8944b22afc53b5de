"""Loads the hand-made grids of tests/golden/handmade_cases.json into arrays."""
import json
import os

import numpy as np

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "handmade_cases.json")


def load():
    with open(GOLDEN) as f:
        return json.load(f)


def grid_of(case):
    R = case["R"]
    boxes = np.asarray(case.get("boxes", [[0, 0, 0, R, R, R]]), np.float32)
    L = boxes.shape[0]
    occ = np.zeros((L, R, R, R), np.uint8)
    spec = case["occupied"]
    if spec == "all":
        occ[:] = 1
    elif spec == "level1":
        occ[1] = 1
    elif spec == "block000_plus_voxel_9_0_0":
        occ[0, :8, :8, :8] = 1
        occ[0, 9, 0, 0] = 1
    else:
        for lev, i, j, k in spec:
            occ[lev, i, j, k] = 1
    return occ, boxes


def step_of(case):
    s = case["step"]
    return {"kind": s["kind"], "dt": float(s.get("dt", 0.0)), "cone": float(s.get("cone", 0.0)),
            "dt_min": float(s.get("dt_min", 0.0))}
