"""CPU oracle for the occupancy-grid ray sampler and the volume-rendering composite.

TEST INFRASTRUCTURE ONLY: the tests, the smoke check and the CPU-baseline leg of
the benchmark may import this package; the product path (the HIP library and
its Python binding) never does, and this package never imports the product.

* ``og_oracle.c`` (loaded here through ctypes) enumerates the fixed-step
  samples of every ray in independent ways: brute force over the lattice, a
  dense voxel DDA, and a VDB tree with hierarchical DDA (whose leaf voxels
  may also merge into uniform 4^3 sub-blocks), each DDA driven as in
  Alg. 1 ("DDA branch") or Alg. 2 ("DDA skip") of the paper's supplementary
  material, and counts the cells each walk visits.  Its header states the
  binary32 definition.
* ``composite.py`` is the FP64 volume-rendering composite and its gradient.
"""
import ctypes
import os

import numpy as np

from .composite import (composite_forward, composite_backward, composite_loss_grad,  # noqa: F401
                        composite_forward_all, composite_backward_all)
from .render import blob_field, render_blobs, render_blobs_all  # noqa: F401
from .distance import chessboard_distance, chessboard_distance_brute  # noqa: F401

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libogoracle.so")

BRUTE, DENSE_BRANCH, DENSE_SKIP, HDDA_BRANCH, HDDA_SKIP, SUBLEAF_BRANCH, SUBLEAF_SKIP = 0, 1, 2, 3, 4, 5, 6
METHODS = {"brute": BRUTE, "dense_branch": DENSE_BRANCH, "dense_skip": DENSE_SKIP,
           "hdda_branch": HDDA_BRANCH, "hdda_skip": HDDA_SKIP,
           "subleaf_branch": SUBLEAF_BRANCH, "subleaf_skip": SUBLEAF_SKIP}


class _Grid(ctypes.Structure):
    _fields_ = [("L", ctypes.c_int32), ("R", ctypes.c_int32),
                ("box", ctypes.POINTER(ctypes.c_float)), ("occ", ctypes.POINTER(ctypes.c_uint8))]


class _Step(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("dt", ctypes.c_float),
                ("cone", ctypes.c_float), ("dt_min", ctypes.c_float)]


_lib = None


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH) or os.path.getmtime(LIB_PATH) < os.path.getmtime(os.path.join(HERE, "og_oracle.c")):
        from .build import build
        build()
    lib = ctypes.CDLL(LIB_PATH)
    P = ctypes.POINTER
    f32p, i32p, i64p = P(ctypes.c_float), P(ctypes.c_int32), P(ctypes.c_int64)
    lib.orc_ray.argtypes = [P(_Grid), ctypes.c_void_p, P(_Step), f32p, f32p, ctypes.c_float, ctypes.c_float,
                            ctypes.c_int32, f32p, f32p, i32p, ctypes.c_int64]
    lib.orc_ray.restype = ctypes.c_int64
    lib.orc_count.argtypes = [P(_Grid), ctypes.c_void_p, P(_Step), f32p, f32p, ctypes.c_int64, ctypes.c_float,
                              ctypes.c_float, ctypes.c_int32, i64p, ctypes.c_int32]
    lib.orc_count.restype = ctypes.c_int32
    lib.orc_cells.argtypes = lib.orc_count.argtypes
    lib.orc_cells.restype = ctypes.c_int32
    lib.orc_fill.argtypes = [P(_Grid), ctypes.c_void_p, P(_Step), f32p, f32p, ctypes.c_int64, ctypes.c_float,
                             ctypes.c_float, ctypes.c_int32, i64p, i32p, f32p, f32p, i32p, ctypes.c_int32]
    lib.orc_fill.restype = ctypes.c_int64
    lib.orc_vdb_build.argtypes = [P(_Grid), ctypes.c_int32]
    lib.orc_vdb_build.restype = ctypes.c_void_p
    lib.orc_vdb_stats.argtypes = [ctypes.c_void_p, i64p]
    lib.orc_vdb_free.argtypes = [ctypes.c_void_p]
    lib.orc_planes.argtypes = [f32p, ctypes.c_int32, ctypes.c_int32, ctypes.c_float, ctypes.c_float, f32p]
    lib.orc_lattice.argtypes = [P(_Step), ctypes.c_float, ctypes.c_int64, f32p]
    _lib = lib
    return lib


def _fptr(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_float)) if a is not None else None


def _iptr(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)) if a is not None else None


def _lptr(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)) if a is not None else None


def make_step(kind="const", dt=0.0, cone=0.0, dt_min=0.0):
    """kind 'const': t_n = t_min + n*dt; kind 'cone': t_{n+1} = t_n + max(t_n*cone, dt_min)."""
    return {"kind": kind, "dt": float(dt), "cone": float(cone), "dt_min": float(dt_min)}


class Scene:
    """A cascade of L binary occupancy grids of R^3 voxels (finest first)."""

    def __init__(self, occ, boxes):
        occ = np.ascontiguousarray(occ, dtype=np.uint8)
        if occ.ndim == 3:
            occ = occ[None]
        boxes = np.ascontiguousarray(np.asarray(boxes, dtype=np.float32).reshape(-1, 6))
        assert occ.shape[0] == boxes.shape[0] and occ.shape[1] == occ.shape[2] == occ.shape[3]
        self.occ, self.boxes = occ, boxes
        self.L, self.R = occ.shape[0], occ.shape[1]
        self._g = _Grid(self.L, self.R, _fptr(self.boxes), self.occ.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8)))
        self._vdb = {}

    def vdb(self, ilog2):
        """The oracle's own VDB tree with internal nodes of 2^ilog2 leaves per axis."""
        if ilog2 not in self._vdb:
            h = _load().orc_vdb_build(ctypes.byref(self._g), int(ilog2))
            if not h:
                raise ValueError("oracle VDB build rejected the grid")
            self._vdb[ilog2] = h
        return self._vdb[ilog2]

    def vdb_stats(self, ilog2):
        out = np.zeros(6, np.int64)
        _load().orc_vdb_stats(self.vdb(ilog2), _lptr(out))
        keys = ["nodes", "leaves", "slot_full", "slot_empty", "root_full", "root_empty"]
        return dict(zip(keys, (int(v) for v in out)))

    def __del__(self):
        lib = _lib
        if lib is not None:
            for h in getattr(self, "_vdb", {}).values():
                lib.orc_vdb_free(h)


def _step_struct(step):
    kind = {"const": 0, "cone": 1}[step["kind"]]
    return _Step(kind, step["dt"], step["cone"], step["dt_min"])


def _method_args(scene, method, ilog2):
    m = METHODS[method] if isinstance(method, str) else int(method)
    vdb = scene.vdb(ilog2) if m in (HDDA_BRANCH, HDDA_SKIP, SUBLEAF_BRANCH, SUBLEAF_SKIP) else None
    return m, vdb


def ray_samples(scene, o, d, tmin, tmax, step, method="brute", ilog2=3):
    """Samples of one ray: (t0[S], t1[S], voxel_id[S])."""
    lib = _load()
    m, vdb = _method_args(scene, method, ilog2)
    o = np.ascontiguousarray(o, np.float32).reshape(3)
    d = np.ascontiguousarray(d, np.float32).reshape(3)
    st = _step_struct(step)
    n = lib.orc_ray(ctypes.byref(scene._g), vdb, ctypes.byref(st), _fptr(o), _fptr(d), tmin, tmax, m,
                    None, None, None, 0)
    t0 = np.zeros(n, np.float32)
    t1 = np.zeros(n, np.float32)
    vox = np.zeros(n, np.int32)
    lib.orc_ray(ctypes.byref(scene._g), vdb, ctypes.byref(st), _fptr(o), _fptr(d), tmin, tmax, m,
                _fptr(t0), _fptr(t1), _iptr(vox), n)
    return t0, t1, vox


def sample_counts(scene, origins, dirs, tmin, tmax, step, method="hdda_skip", ilog2=3, threads=0):
    """Per-ray sample counts (int64[N])."""
    lib = _load()
    m, vdb = _method_args(scene, method, ilog2)
    o = np.ascontiguousarray(origins, np.float32).reshape(-1, 3)
    d = np.ascontiguousarray(dirs, np.float32).reshape(-1, 3)
    counts = np.zeros(o.shape[0], np.int64)
    st = _step_struct(step)
    rc = lib.orc_count(ctypes.byref(scene._g), vdb, ctypes.byref(st), _fptr(o), _fptr(d), o.shape[0],
                       tmin, tmax, m, _lptr(counts), int(threads))
    if rc != 0:
        raise ValueError("oracle rejected the method")
    return counts


def cell_counts(scene, origins, dirs, tmin, tmax, step, method="hdda_branch", ilog2=3, threads=0):
    """Cells each ray's walk visits (int64[N]) for a DDA method (not brute force)."""
    lib = _load()
    m, vdb = _method_args(scene, method, ilog2)
    o = np.ascontiguousarray(origins, np.float32).reshape(-1, 3)
    d = np.ascontiguousarray(dirs, np.float32).reshape(-1, 3)
    cells = np.zeros(o.shape[0], np.int64)
    st = _step_struct(step)
    rc = lib.orc_cells(ctypes.byref(scene._g), vdb, ctypes.byref(st), _fptr(o), _fptr(d), o.shape[0],
                       tmin, tmax, m, _lptr(cells), int(threads))
    if rc != 0:
        raise ValueError("oracle rejected the method")
    return cells


def sample_rays(scene, origins, dirs, tmin, tmax, step, method="hdda_skip", ilog2=3, threads=0):
    """Packed samples of all rays: dict(offsets[N+1], ray_ids[S], t0[S], t1[S], voxel_ids[S])."""
    lib = _load()
    m, vdb = _method_args(scene, method, ilog2)
    o = np.ascontiguousarray(origins, np.float32).reshape(-1, 3)
    d = np.ascontiguousarray(dirs, np.float32).reshape(-1, 3)
    counts = sample_counts(scene, o, d, tmin, tmax, step, method, ilog2, threads)
    offsets = np.zeros(o.shape[0] + 1, np.int64)
    np.cumsum(counts, out=offsets[1:])
    S = int(offsets[-1])
    out = {"offsets": offsets, "ray_ids": np.zeros(S, np.int32), "t0": np.zeros(S, np.float32),
           "t1": np.zeros(S, np.float32), "voxel_ids": np.zeros(S, np.int32)}
    st = _step_struct(step)
    bad = lib.orc_fill(ctypes.byref(scene._g), vdb, ctypes.byref(st), _fptr(o), _fptr(d), o.shape[0], tmin, tmax,
                       m, _lptr(offsets), _iptr(out["ray_ids"]), _fptr(out["t0"]), _fptr(out["t1"]),
                       _iptr(out["voxel_ids"]), int(threads))
    if bad:
        raise RuntimeError(f"oracle fill disagreed with its own counts on {bad} rays")
    return out


def planes(box, R, axis, o, d):
    """(P[R+1], T[R+1]) of one axis as the oracle computes them."""
    lib = _load()
    box = np.ascontiguousarray(box, np.float32).reshape(6)
    out = np.zeros(2 * (R + 1), np.float32)
    lib.orc_planes(_fptr(box), R, axis, o, d, _fptr(out))
    return out[:R + 1], out[R + 1:]


def lattice(step, tmin, n):
    lib = _load()
    out = np.zeros(n, np.float32)
    st = _step_struct(step)
    lib.orc_lattice(ctypes.byref(st), tmin, n, _fptr(out))
    return out
