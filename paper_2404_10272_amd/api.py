"""Python binding of the ogvdb C-ABI (include/ogvdb.h).

Argument marshalling only: every step of sampling and compositing runs in
the HIP kernels of libogvdb.so.  PyTorch provides device memory and the
current stream.  If the library is not built, every call raises: there is no
fallback path.
"""
import ctypes
import os

import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libogvdb.so")

BRANCH, SKIP, VOXEL, SUBLEAF = 0, 1, 2, 4
STEP_CONST, STEP_CONE = 0, 1


class OgvError(RuntimeError):
    pass


class _Step(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("dt", ctypes.c_float), ("cone", ctypes.c_float),
                ("dt_min", ctypes.c_float)]


class _Info(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("n_levels", ctypes.c_int32), ("res", ctypes.c_int32),
                ("internal_log2", ctypes.c_int32), ("bytes", ctypes.c_int64), ("n_nodes", ctypes.c_int64),
                ("n_leaves", ctypes.c_int64), ("n_tiles_full", ctypes.c_int64), ("n_tiles_empty", ctypes.c_int64),
                ("n_root_tiles_full", ctypes.c_int64), ("n_root_tiles_empty", ctypes.c_int64)]


class _Opts(ctypes.Structure):
    _fields_ = [("variant", ctypes.c_int32), ("image_width", ctypes.c_int32)]


class _Scene(ctypes.Structure):
    _fields_ = [("grid", ctypes.c_void_p), ("origins", ctypes.c_void_p), ("dirs", ctypes.c_void_p),
                ("n_rays", ctypes.c_int64), ("near_t", ctypes.c_float), ("far_t", ctypes.c_float), ("step", _Step),
                ("image_width", ctypes.c_int32)]


class _Tune(ctypes.Structure):
    _fields_ = [("chunk", ctypes.c_int32), ("blocks_per_cu", ctypes.c_int32)]


class _BatchInfo(ctypes.Structure):
    _fields_ = [("n_rays", ctypes.c_int64), ("n_scenes", ctypes.c_int32), ("tune", _Tune), ("tuned", ctypes.c_int32),
                ("tune_ms", ctypes.c_float)]


MAX_BLOBS = 16


class _BlobField(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32), ("centre", (ctypes.c_float * 3) * MAX_BLOBS),
                ("radius", ctypes.c_float * MAX_BLOBS), ("density", ctypes.c_float * MAX_BLOBS),
                ("colour", (ctypes.c_float * 3) * MAX_BLOBS)]


_lib = None
VP, I32, I64, F32, SZ = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_float, ctypes.c_size_t

# name -> (restype, argtypes); the exported C-ABI
SIGNATURES = {
    "ogv_dense_build": (I32, [I32, I32, VP, VP, ctypes.POINTER(VP), VP]),
    "ogv_vdb_build": (I32, [I32, I32, VP, VP, I32, ctypes.POINTER(VP), VP]),
    "ogv_dist_build": (I32, [I32, I32, VP, VP, ctypes.POINTER(VP), VP]),
    "ogv_grid_distances": (I32, [VP, VP, VP]),
    "ogv_grid_info_get": (I32, [VP, ctypes.POINTER(_Info)]),
    "ogv_grid_to_dense": (I32, [VP, VP, VP]),
    "ogv_grid_destroy": (None, [VP]),
    "ogv_grid_refresh": (I32, [VP, VP, VP]),
    "ogv_grid_refresh_density": (I32, [VP, VP, VP, F32, F32, VP, VP]),
    "ogv_sample_workspace_size": (I32, [I64, F32, F32, ctypes.POINTER(_Step), ctypes.POINTER(SZ)]),
    "ogv_sample_count": (I32, [VP, ctypes.POINTER(_Opts), VP, VP, I64, F32, F32, ctypes.POINTER(_Step), VP, VP, SZ,
                               VP]),
    "ogv_sample_count_raw": (I32, [VP, ctypes.POINTER(_Opts), VP, VP, I64, F32, F32, ctypes.POINTER(_Step), VP, SZ,
                                   VP]),
    "ogv_sample_scan": (I32, [I64, VP, VP, SZ, VP]),
    "ogv_sample_fill": (I32, [VP, ctypes.POINTER(_Opts), VP, VP, I64, F32, F32, ctypes.POINTER(_Step), VP, I64, VP, VP,
                              VP, VP, VP, SZ, VP]),
    "ogv_sample_rays": (I32, [VP, ctypes.POINTER(_Opts), VP, VP, I64, F32, F32, ctypes.POINTER(_Step), VP, I64, VP, VP,
                              VP, VP, VP, VP, SZ, VP]),
    "ogv_sample_rays_noalloc": (I32, [VP, ctypes.POINTER(_Opts), VP, VP, I64, F32, F32, ctypes.POINTER(_Step), VP,
                                      I64, VP, VP, VP, VP, VP, VP]),
    "ogv_composite_fwd": (I32, [VP, I64, VP, VP, VP, VP, VP, VP, VP]),
    "ogv_composite_bwd": (I32, [VP, I64, I64, VP, VP, VP, VP, VP, VP, VP, VP, VP]),
    "ogv_render_blobs": (I32, [VP, I64, VP, VP, VP, VP, ctypes.POINTER(_BlobField), VP, VP, VP]),
    "ogv_batch_create": (I32, [ctypes.POINTER(_Scene), I32, I32, ctypes.POINTER(_Tune), ctypes.POINTER(VP), VP]),
    "ogv_batch_info_get": (I32, [VP, ctypes.POINTER(_BatchInfo), VP]),
    "ogv_batch_launch": (I32, [VP, VP, I64, VP, VP, VP, VP, VP]),
    "ogv_batch_launch_eager": (I32, [VP, VP, I64, VP, VP, VP, VP, VP]),
    "ogv_batch_destroy": (None, [VP]),
    "ogv_last_error": (ctypes.c_char_p, []),
    "ogv_version": (ctypes.c_char_p, []),
}


def lib():
    """The loaded libogvdb.so; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise OgvError(f"{LIB_PATH} is not built (run __graft_entry__.build()); no fallback exists")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def _check(status):
    if status != 0:
        msg = lib().ogv_last_error().decode(errors="replace")
        raise OgvError(f"ogvdb status {status}: {msg}")


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


def _stream(stream=None):
    s = torch.cuda.current_stream() if stream is None else stream
    return ctypes.c_void_p(s.cuda_stream)


def make_step(kind="const", dt=0.0, cone=0.0, dt_min=0.0):
    if isinstance(kind, dict):
        kind, dt, cone, dt_min = kind["kind"], kind.get("dt", 0.0), kind.get("cone", 0.0), kind.get("dt_min", 0.0)
    k = {"const": STEP_CONST, "cone": STEP_CONE}[kind]
    return _Step(k, float(dt), float(cone), float(dt_min))


def _variant(v):
    """Loop variant: "branch", "skip", "voxel_branch", "voxel_skip" (VDB grids
    walked one voxel per step), "subleaf_branch", "subleaf_skip" (VDB grids
    walked with steps over uniform sub-blocks of leaves too) or the ogvdb.h
    value."""
    names = {"branch": BRANCH, "skip": SKIP, "voxel_branch": BRANCH | VOXEL, "voxel_skip": SKIP | VOXEL,
             "subleaf_branch": BRANCH | SUBLEAF, "subleaf_skip": SKIP | SUBLEAF}
    if isinstance(v, str):
        return names[v]
    if v not in names.values():
        raise ValueError(f"unknown variant {v!r}")
    return int(v)


class Grid:
    """A built grid on the current device: dense bitfield (plain method) or VDB tree."""

    def __init__(self, handle, kind, boxes, shape=None):
        self._h = handle
        self.kind = kind
        self.boxes = boxes
        self.shape = shape          # (L, R, R, R) of the occupancy it was built from
        self._occ_in_use = None     # occupancy a refresh may still be reading

    @property
    def handle(self):
        return self._h

    def info(self):
        inf = _Info()
        _check(lib().ogv_grid_info_get(self._h, ctypes.byref(inf)))
        return {k: getattr(inf, k) for k, _ in _Info._fields_}

    def to_dense(self):
        i = self.info()
        out = torch.empty((i["n_levels"],) + (i["res"],) * 3, dtype=torch.uint8, device="cuda")
        _check(lib().ogv_grid_to_dense(self._h, _ptr(out), _stream()))
        return out

    def refresh(self, occ, stream=None):
        """Re-derives this grid from a new occupancy of the same shape, in
        place and asynchronously (no allocation, no host synchronization)."""
        if occ.dim() == 3:
            occ = occ.unsqueeze(0)
        if not occ.is_cuda:
            raise OgvError("occupancy must be a device tensor")
        occ = occ.to(torch.uint8).contiguous()
        if self.shape is not None and tuple(occ.shape) != tuple(self.shape):
            raise OgvError(f"occupancy shape {tuple(occ.shape)} differs from the grid's {tuple(self.shape)}")
        _check(lib().ogv_grid_refresh(self._h, _ptr(occ), _stream(stream)))
        self._occ_in_use = occ

    def refresh_density(self, cache, density=None, decay=0.95, threshold=0.01, changed=None, stream=None):
        """Re-derives this grid from a float32 density cache of its shape, in
        place and asynchronously: with `density`, the cache is first updated
        to max(decay*cache, density); a voxel is occupied when its cache
        value exceeds `threshold`.  `changed` (int32 [2], optional) receives
        the number of voxels that changed and whether the tree's structure
        did."""
        for t in (cache, density):
            if t is None:
                continue
            if not t.is_cuda or t.dtype != torch.float32 or not t.is_contiguous():
                raise OgvError("density tensors must be contiguous float32 device tensors")
            if self.shape is not None and tuple(t.shape) != tuple(self.shape):
                raise OgvError(f"density shape {tuple(t.shape)} differs from the grid's {tuple(self.shape)}")
        if changed is not None and (changed.dtype != torch.int32 or changed.numel() < 2 or not changed.is_cuda):
            raise OgvError("changed must be an int32 device tensor of 2 entries")
        _check(lib().ogv_grid_refresh_density(self._h, _ptr(cache), _ptr(density), float(decay), float(threshold),
                                              _ptr(changed), _stream(stream)))
        self._occ_in_use = (cache, density)

    def distances(self):
        """A distance grid's capped chessboard distances, uint8 [L][R][R][R]."""
        out = torch.empty(tuple(self.shape), dtype=torch.uint8, device="cuda")
        _check(lib().ogv_grid_distances(self._h, _ptr(out), _stream()))
        return out

    def close(self):
        if self._h:
            lib().ogv_grid_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _grid_args(occ, boxes):
    if occ.dim() == 3:
        occ = occ.unsqueeze(0)
    if not occ.is_cuda:
        raise OgvError("occupancy must be a device tensor")
    occ = occ.to(torch.uint8).contiguous()
    L, R = occ.shape[0], occ.shape[1]
    if occ.shape[1:] != (R, R, R):
        raise OgvError("occupancy must be [L][R][R][R]")
    b = (ctypes.c_float * (6 * L))(*[float(x) for x in torch.as_tensor(boxes, dtype=torch.float32).reshape(-1)])
    return occ, L, R, b


def build_dense(occ, boxes, stream=None):
    occ, L, R, b = _grid_args(occ, boxes)
    h = ctypes.c_void_p()
    _check(lib().ogv_dense_build(L, R, b, _ptr(occ), ctypes.byref(h), _stream(stream)))
    return Grid(h, "dense", boxes, tuple(occ.shape))


def build_dist(occ, boxes, stream=None):
    """Dense bitfield plus capped chessboard distances (a third traversal)."""
    occ, L, R, b = _grid_args(occ, boxes)
    h = ctypes.c_void_p()
    _check(lib().ogv_dist_build(L, R, b, _ptr(occ), ctypes.byref(h), _stream(stream)))
    return Grid(h, "dist", boxes, tuple(occ.shape))


def build_vdb(occ, boxes, internal_log2=4, stream=None):
    occ, L, R, b = _grid_args(occ, boxes)
    h = ctypes.c_void_p()
    _check(lib().ogv_vdb_build(L, R, b, _ptr(occ), int(internal_log2), ctypes.byref(h), _stream(stream)))
    return Grid(h, "vdb", boxes, tuple(occ.shape))


def workspace_bytes(n_rays, near, far, step):
    n = ctypes.c_size_t()
    _check(lib().ogv_sample_workspace_size(int(n_rays), float(near), float(far), ctypes.byref(step),
                                           ctypes.byref(n)))
    return n.value


def _rays(origins, dirs):
    o = origins.contiguous()
    d = dirs.contiguous()
    if o.dtype != torch.float32 or d.dtype != torch.float32 or o.shape != d.shape or o.shape[-1] != 3:
        raise OgvError("origins/dirs must be float32 [N][3] of equal shape")
    if not (o.is_cuda and d.is_cuda):
        raise OgvError("rays must be device tensors")
    return o, d, o.shape[0]


class Sampler:
    """Reusable sampling call on one grid with fixed ray count and lattice;
    holds the workspace so repeated calls allocate nothing but outputs."""

    def __init__(self, grid, n_rays, near, far, step, variant="branch", device="cuda", image_width=0):
        self.grid = grid
        self.n = int(n_rays)
        self.near, self.far = float(near), float(far)
        self.step = step if isinstance(step, _Step) else make_step(step)
        self.variant = _variant(variant)
        self.opts = _Opts(self.variant, int(image_width))
        self.ws_bytes = workspace_bytes(self.n, self.near, self.far, self.step)
        self.ws = torch.empty(max(self.ws_bytes, 1), dtype=torch.uint8, device=device)
        self.offsets = torch.empty(self.n + 1, dtype=torch.int64, device=device)
        self.overflow = torch.zeros(1, dtype=torch.int32, device=device)

    def count(self, o, d, stream=None):
        _check(lib().ogv_sample_count(self.grid.handle, ctypes.byref(self.opts), _ptr(o), _ptr(d), self.n, self.near, self.far,
                                      ctypes.byref(self.step), _ptr(self.offsets), _ptr(self.ws), self.ws_bytes,
                                      _stream(stream)))
        return self.offsets

    def count_raw(self, o, d, stream=None):
        """The walk half of count(): counts and runs stay in the workspace."""
        _check(lib().ogv_sample_count_raw(self.grid.handle, ctypes.byref(self.opts), _ptr(o), _ptr(d), self.n,
                                          self.near, self.far, ctypes.byref(self.step), _ptr(self.ws), self.ws_bytes,
                                          _stream(stream)))

    def scan(self, stream=None):
        """The scan half of count(): offsets from the counts count_raw() left."""
        _check(lib().ogv_sample_scan(self.n, _ptr(self.offsets), _ptr(self.ws), self.ws_bytes, _stream(stream)))
        return self.offsets

    def fill(self, o, d, ray_ids, t0, t1, voxel_ids=None, stream=None):
        _check(lib().ogv_sample_fill(self.grid.handle, ctypes.byref(self.opts), _ptr(o), _ptr(d), self.n, self.near, self.far,
                                     ctypes.byref(self.step), _ptr(self.offsets), int(t0.numel()), _ptr(ray_ids),
                                     _ptr(t0), _ptr(t1), _ptr(voxel_ids), _ptr(self.ws), self.ws_bytes,
                                     _stream(stream)))

    def rays(self, o, d, ray_ids, t0, t1, voxel_ids=None, stream=None):
        """Count + scan + fill with no host round trip (capacity = len(t0))."""
        _check(lib().ogv_sample_rays(self.grid.handle, ctypes.byref(self.opts), _ptr(o), _ptr(d), self.n, self.near, self.far,
                                     ctypes.byref(self.step), _ptr(self.offsets), int(t0.numel()), _ptr(ray_ids),
                                     _ptr(t0), _ptr(t1), _ptr(voxel_ids), _ptr(self.overflow), _ptr(self.ws),
                                     self.ws_bytes, _stream(stream)))
        return self.offsets, self.overflow


def sample_rays(grid, origins, dirs, near, far, step, variant="branch", voxel_ids=False, image_width=0):
    """Packed samples of every ray: dict(offsets[N+1], ray_ids[S], t0[S], t1[S], voxel_ids[S]?).

    Counts first, reads the total (one device->host sync), allocates the
    exact outputs, then fills.
    """
    o, d, n = _rays(origins, dirs)
    sp = Sampler(grid, n, near, far, step, variant, device=o.device, image_width=image_width)
    offsets = sp.count(o, d)
    total = int(offsets[n].item())
    dev = o.device
    out = {"offsets": offsets,
           "ray_ids": torch.empty(total, dtype=torch.int32, device=dev),
           "t0": torch.empty(total, dtype=torch.float32, device=dev),
           "t1": torch.empty(total, dtype=torch.float32, device=dev)}
    vox = torch.empty(total, dtype=torch.int32, device=dev) if voxel_ids else None
    sp.fill(o, d, out["ray_ids"], out["t0"], out["t1"], vox)
    if voxel_ids:
        out["voxel_ids"] = vox
    return out


NOALLOC_SCRATCH_BYTES = 64 << 20


def sample_rays_noalloc(grid, origins, dirs, near, far, step, offsets, ray_ids, t0, t1, overflow,
                        variant="branch", voxel_ids=None, image_width=0, stream=None):
    """ogv_sample_rays_noalloc: count + scan + fill into caller-allocated
    outputs (offsets int64 [N+1], ray_ids/t0/t1 of capacity len(t0),
    overflow int32 [1]) with the library's static per-device workspace; the
    call allocates nothing.  Returns (offsets, overflow)."""
    o, d, n = _rays(origins, dirs)
    st = step if isinstance(step, _Step) else make_step(step)
    opts = _Opts(_variant(variant), int(image_width))
    _check(lib().ogv_sample_rays_noalloc(grid.handle, ctypes.byref(opts), _ptr(o), _ptr(d), n, float(near),
                                         float(far), ctypes.byref(st), _ptr(offsets), int(t0.numel()),
                                         _ptr(ray_ids), _ptr(t0), _ptr(t1), _ptr(voxel_ids), _ptr(overflow),
                                         _stream(stream)))
    return offsets, overflow


# ---------------------------------------------------------------- batches

class Batch:
    """Many scenes sampled in one graph-captured pass (see ogv_batch_create).

    scenes: list of (grid, origins, dirs, near, far, step[, image_width]).
    tune: None to autotune, or (chunk, blocks_per_cu).  The grids and ray
    tensors are kept alive by this object.
    """

    def __init__(self, scenes, variant="branch", tune=None, stream=None):
        self._keep = []
        arr = (_Scene * len(scenes))()
        for i, sc in enumerate(scenes):
            grid, o, d, near, far, step = sc[:6]
            width = int(sc[6]) if len(sc) > 6 else 0
            o, d, n = _rays(o, d)
            self._keep += [grid, o, d]
            st = step if isinstance(step, _Step) else make_step(step)
            arr[i] = _Scene(grid.handle, o.data_ptr(), d.data_ptr(), n, float(near), float(far), st, width)
        t = None if tune is None else ctypes.byref(_Tune(int(tune[0]), int(tune[1])))
        h = ctypes.c_void_p()
        _check(lib().ogv_batch_create(arr, len(scenes), _variant(variant), t, ctypes.byref(h), _stream(stream)))
        self._h = h
        self.n_scenes = len(scenes)
        info = self.info()
        self.n_rays = info["n_rays"]
        self.offsets = torch.empty(self.n_rays + 1, dtype=torch.int64, device="cuda")
        self.overflow = torch.zeros(1, dtype=torch.int32, device="cuda")

    def info(self):
        inf = _BatchInfo()
        base = (ctypes.c_int64 * self.n_scenes)()
        _check(lib().ogv_batch_info_get(self._h, ctypes.byref(inf), base))
        return {"n_rays": inf.n_rays, "n_scenes": inf.n_scenes, "chunk": inf.tune.chunk,
                "blocks_per_cu": inf.tune.blocks_per_cu, "tuned": bool(inf.tuned), "tune_ms": inf.tune_ms,
                "ray_base": list(base)}

    def launch(self, ray_ids, t0, t1, graph=True, stream=None):
        fn = lib().ogv_batch_launch if graph else lib().ogv_batch_launch_eager
        _check(fn(self._h, _ptr(self.offsets), int(t0.numel()), _ptr(ray_ids), _ptr(t0), _ptr(t1),
                  _ptr(self.overflow), _stream(stream)))
        return self.offsets, self.overflow

    def close(self):
        if getattr(self, "_h", None):
            lib().ogv_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ---------------------------------------------------------------- composite

def composite_forward(offsets, t0, t1, sigma, rgb):
    n = offsets.numel() - 1
    out_rgb = torch.empty((n, 3), dtype=torch.float32, device=sigma.device)
    out_a = torch.empty(n, dtype=torch.float32, device=sigma.device)
    _check(lib().ogv_composite_fwd(_ptr(offsets), n, _ptr(t0), _ptr(t1), _ptr(sigma), _ptr(rgb), _ptr(out_rgb),
                                   _ptr(out_a), _stream()))
    return out_rgb, out_a


def composite_backward(offsets, t0, t1, sigma, rgb, g_rgb, g_opacity):
    d_sigma = torch.empty_like(sigma)   # every entry is written (zero where no ray owns it)
    d_rgb = torch.empty_like(rgb)
    n = offsets.numel() - 1
    _check(lib().ogv_composite_bwd(_ptr(offsets), n, sigma.numel(), _ptr(t0), _ptr(t1), _ptr(sigma), _ptr(rgb), _ptr(g_rgb),
                                   _ptr(g_opacity), _ptr(d_sigma), _ptr(d_rgb), _stream()))
    return d_sigma, d_rgb


def blob_field(centres, radii, densities, colours):
    """The C struct of a Gaussian-blob field from K centres [K,3], radii [K],
    densities [K] and colours [K,3] (1 <= K <= 16)."""
    import numpy as np
    c = np.asarray(centres, np.float32).reshape(-1, 3)
    k = c.shape[0]
    f = _BlobField()
    f.n = k
    for i in range(min(k, MAX_BLOBS)):
        for q in range(3):
            f.centre[i][q] = float(c[i, q])
            f.colour[i][q] = float(np.asarray(colours, np.float32).reshape(-1, 3)[i, q])
        f.radius[i] = float(np.asarray(radii, np.float32)[i])
        f.density[i] = float(np.asarray(densities, np.float32)[i])
    return f


def render_blobs(offsets, origins, dirs, t0, t1, field):
    """Pixel (rgb[N,3], opacity[N]) of packed samples rendered through a blob
    field (each sample at its interval midpoint), one fused pass."""
    o, d, n = _rays(origins, dirs)
    out_rgb = torch.empty((n, 3), dtype=torch.float32, device=o.device)
    out_a = torch.empty(n, dtype=torch.float32, device=o.device)
    _check(lib().ogv_render_blobs(_ptr(offsets), n, _ptr(o), _ptr(d), _ptr(t0), _ptr(t1), ctypes.byref(field),
                                  _ptr(out_rgb), _ptr(out_a), _stream()))
    return out_rgb, out_a


class Composite(torch.autograd.Function):
    """(sigma[S], rgb[S,3]) -> (pixel rgb[N,3], opacity[N]) over packed samples;
    the sampler's outputs (offsets, t0, t1) are constants."""

    @staticmethod
    def forward(ctx, sigma, rgb, offsets, t0, t1):
        sigma = sigma.contiguous().float()
        rgb = rgb.contiguous().float()
        out_rgb, out_a = composite_forward(offsets, t0, t1, sigma, rgb)
        ctx.save_for_backward(sigma, rgb, offsets, t0, t1)
        return out_rgb, out_a

    @staticmethod
    def backward(ctx, g_rgb, g_a):
        sigma, rgb, offsets, t0, t1 = ctx.saved_tensors
        if g_rgb is None:
            g_rgb = torch.zeros((offsets.numel() - 1, 3), dtype=torch.float32, device=sigma.device)
        g_rgb = g_rgb.contiguous().float()
        g_a = g_a.contiguous().float() if g_a is not None else None
        d_sigma, d_rgb = composite_backward(offsets, t0, t1, sigma, rgb, g_rgb, g_a)
        return d_sigma, d_rgb, None, None, None


def composite(sigma, rgb, offsets, t0, t1):
    return Composite.apply(sigma, rgb, offsets, t0, t1)
