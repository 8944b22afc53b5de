"""Seeded synthetic occupancy grids and pinhole cameras.

These stand in for the trained occupancy grids and the test cameras of the
paper's NeRF-Synthetic (one 128^3 grid, 800x800 images) and Mip-NeRF 360
(four nested 128^3 cascades, unbounded scenes) experiments (Sec. 4.1); the
datasets and trained weights themselves are not used.  This module only draws
inputs: it holds none of the sampler's arithmetic, and both the HIP path and
the CPU oracle take their inputs from it.

Every generator is a pure function of its seed (numpy default_rng).
Occupancy targets are hit exactly by thresholding a field at its quantile.

Workloads (``workload(name)``):
  small      64^3 grid over [-1.5,1.5]^3, union of 6 random spheres (voxel
             centre inside), 64x64 rays from radius 4, 40 deg FOV,
             near 2, far 6, step fl32(3*sqrt(3)/1024); internal nodes 8^3.
  object     128^3 over [-1.5,1.5]^3, 3-octave value noise on a union of 12
             random ellipsoid shells, 6.0 % occupied; 800x800 rays from a
             random direction at radius 4, 40 deg FOV, near 2, far 6,
             step 5e-3; internal nodes 16^3.
  unbounded  4 nested 128^3 cascades over [-2^k,2^k]^3, k=0..3, 4-octave
             value noise thresholded at 15/10/6/3 %; 1280x832 rays from a
             camera in [-0.5,0.5]^3 with a random orientation, 60 deg
             horizontal FOV; near 0.05, far 1e3, growing step
             max(t/256, 1e-3); internal nodes 16^3.
  batched    16 scenes, sides from {64,128,256}, occupancy U(2 %, 20 %),
             ray images 1024^2 x4, 768^2, 512^2 x3, 384^2, 256^2 x3,
             128^2 x2, 64^2 x2 (5,955,584 rays), object-style cameras.
"""
from dataclasses import dataclass, field
import math

import numpy as np

SEED_BASE = {"small": 1000, "object": 2000, "unbounded": 3000, "composite": 4000, "batched": 5000, "render": 6000}


@dataclass
class Workload:
    name: str
    occ: np.ndarray          # uint8 [L][R][R][R], finest level first
    boxes: np.ndarray        # float32 [L][6]: min xyz, max xyz
    origins: np.ndarray      # float32 [N][3]
    dirs: np.ndarray         # float32 [N][3], unit length
    near: float
    far: float
    step: dict               # {"kind": "const"|"cone", "dt", "cone", "dt_min"}
    ilog2: int               # internal node = 2^ilog2 leaf blocks per axis
    image: tuple = (0, 0)    # (width, height) of the ray image
    meta: dict = field(default_factory=dict)

    @property
    def n_rays(self):
        return int(self.origins.shape[0])

    @property
    def R(self):
        return int(self.occ.shape[1])

    @property
    def L(self):
        return int(self.occ.shape[0])


# --------------------------------------------------------------------------
# fields

def voxel_centres(R, lo, hi):
    """Centres of R voxels along one axis of [lo, hi], float64."""
    return lo + (np.arange(R) + 0.5) * ((hi - lo) / R)


def _lattice_weights(x, lo, hi, cells):
    """Smoothstep interpolation matrix (len(x), cells+1) of a value-noise lattice."""
    u = (np.asarray(x, np.float64) - lo) / (hi - lo) * cells
    u = np.clip(u, 0.0, cells - 1e-9)
    i = np.floor(u).astype(np.int64)
    f = u - i
    s = f * f * (3.0 - 2.0 * f)
    W = np.zeros((u.shape[0], cells + 1))
    rows = np.arange(u.shape[0])
    W[rows, i] = 1.0 - s
    W[rows, i + 1] = s
    return W


def value_noise(xs, ys, zs, lo, hi, base_cells, octaves, rng):
    """Multi-octave value noise sampled on the tensor grid xs x ys x zs.

    Each octave is a random lattice of values in [0,1) over [lo,hi]^3 with
    base_cells * 2^o cells per axis, interpolated with smoothstep weights
    (separably) and weighted 0.5^o.
    """
    out = np.zeros((len(xs), len(ys), len(zs)))
    amp = 1.0
    for o in range(octaves):
        cells = base_cells * (2 ** o)
        V = rng.random((cells + 1,) * 3)
        Wx = _lattice_weights(xs, lo, hi, cells)
        Wy = _lattice_weights(ys, lo, hi, cells)
        Wz = _lattice_weights(zs, lo, hi, cells)
        f = np.tensordot(Wx, V, axes=(1, 0))                        # x, j, k
        f = np.tensordot(f, Wy, axes=(1, 1))                        # x, k, y
        f = np.tensordot(f, Wz, axes=(1, 1))                        # x, y, z
        out += amp * f
        amp *= 0.5
    return out


def threshold_top(field_values, frac, allowed=None):
    """uint8 mask of exactly round(frac * size) voxels with the largest field
    values (only among `allowed` voxels when given)."""
    flat = field_values.reshape(-1).astype(np.float64)
    k = int(round(frac * flat.size))
    if allowed is not None:
        flat = np.where(allowed.reshape(-1), flat, -np.inf)
        k = min(k, int(np.count_nonzero(allowed)))
    mask = np.zeros(flat.size, np.uint8)
    if k > 0:
        idx = np.argpartition(-flat, k - 1)[:k]
        mask[idx] = 1
    return mask.reshape(field_values.shape)


def random_rotation(rng):
    q, r = np.linalg.qr(rng.normal(size=(3, 3)))
    q = q * np.sign(np.diag(r))
    if np.linalg.det(q) < 0:
        q[:, 0] = -q[:, 0]
    return q


def spheres_grid(R, box_lo, box_hi, n_spheres, rng):
    """Voxel centre inside a union of spheres, r ~ U(0.2,0.5), c ~ U(-0.8,0.8)^3."""
    centres = rng.uniform(-0.8, 0.8, size=(n_spheres, 3))
    radii = rng.uniform(0.2, 0.5, size=n_spheres)
    c = voxel_centres(R, box_lo, box_hi)
    X, Y, Z = np.meshgrid(c, c, c, indexing="ij")
    occ = np.zeros((R, R, R), bool)
    for ctr, rad in zip(centres, radii):
        occ |= (X - ctr[0]) ** 2 + (Y - ctr[1]) ** 2 + (Z - ctr[2]) ** 2 < rad * rad
    return occ.astype(np.uint8)


def shells_mask(R, box_lo, box_hi, n_shells, rng):
    """Union of random ellipsoid shells |q - 1| < 0.1, q the ellipsoidal radius."""
    c = voxel_centres(R, box_lo, box_hi)
    X, Y, Z = np.meshgrid(c, c, c, indexing="ij")
    P = np.stack([X, Y, Z], -1).reshape(-1, 3)
    mask = np.zeros(P.shape[0], bool)
    for _ in range(n_shells):
        ctr = rng.uniform(-0.7, 0.7, size=3)
        semi = rng.uniform(0.25, 0.7, size=3)
        Q = random_rotation(rng)
        local = (P - ctr) @ Q / semi
        q = np.sqrt(np.einsum("ij,ij->i", local, local))
        mask |= np.abs(q - 1.0) < 0.1
    return mask.reshape(R, R, R)


# --------------------------------------------------------------------------
# cameras

def look_at_camera(position, target=(0.0, 0.0, 0.0), up=(0.0, 0.0, 1.0)):
    """Columns: right, up, backward (the camera looks along -backward)."""
    pos = np.asarray(position, np.float64)
    fwd = np.asarray(target, np.float64) - pos
    fwd /= np.linalg.norm(fwd)
    right = np.cross(fwd, np.asarray(up, np.float64))
    right /= np.linalg.norm(right)
    true_up = np.cross(right, fwd)
    return np.stack([right, true_up, -fwd], 1)


def pinhole_rays(width, height, fov_x_deg, cam_to_world, position):
    """Unit ray directions through pixel centres (+0.5), float32; origins = position."""
    focal = 0.5 * width / math.tan(math.radians(fov_x_deg) / 2.0)
    px = (np.arange(width) + 0.5 - 0.5 * width) / focal
    py = (0.5 * height - (np.arange(height) + 0.5)) / focal
    X, Y = np.meshgrid(px, py, indexing="xy")          # row-major: y slow, x fast
    dirs_cam = np.stack([X, Y, -np.ones_like(X)], -1).reshape(-1, 3)
    dirs = dirs_cam @ np.asarray(cam_to_world, np.float64).T
    dirs /= np.linalg.norm(dirs, axis=1, keepdims=True)
    origins = np.broadcast_to(np.asarray(position, np.float64), dirs.shape)
    return np.ascontiguousarray(origins, np.float32), np.ascontiguousarray(dirs, np.float32)


def orbit_position(radius, azimuth, elevation):
    return radius * np.array([math.cos(elevation) * math.cos(azimuth),
                              math.cos(elevation) * math.sin(azimuth),
                              math.sin(elevation)])


def object_camera_rays(width, height, rng, radius=4.0, fov=40.0):
    az = rng.uniform(0.0, 2.0 * math.pi)
    el = math.radians(rng.uniform(-85.0, 85.0))
    pos = orbit_position(radius, az, el)
    return pinhole_rays(width, height, fov, look_at_camera(pos), pos)


# --------------------------------------------------------------------------
# workloads

def _box(lo, hi):
    return np.asarray([[lo, lo, lo, hi, hi, hi]], np.float32)


def small(seed=SEED_BASE["small"]):
    rng = np.random.default_rng(seed)
    occ = spheres_grid(64, -1.5, 1.5, 6, rng)[None]
    pos = orbit_position(4.0, 0.5, 0.3)
    o, d = pinhole_rays(64, 64, 40.0, look_at_camera(pos), pos)
    dt = float(np.float32(3.0 * math.sqrt(3.0) / 1024.0))
    return Workload("small", occ, _box(-1.5, 1.5), o, d, 2.0, 6.0,
                    {"kind": "const", "dt": dt, "cone": 0.0, "dt_min": 0.0}, 3, (64, 64))


def object_grid(seed=SEED_BASE["object"], R=128, frac=0.06):
    rng = np.random.default_rng(seed)
    shells = shells_mask(R, -1.5, 1.5, 12, rng)
    c = voxel_centres(R, -1.5, 1.5)
    noise = value_noise(c, c, c, -1.5, 1.5, 4, 3, rng)
    return threshold_top(noise, frac, allowed=shells)[None], rng


def object_scene(seed=SEED_BASE["object"], width=800, height=800):
    occ, rng = object_grid(seed)
    o, d = object_camera_rays(width, height, rng)
    return Workload("object", occ, _box(-1.5, 1.5), o, d, 2.0, 6.0,
                    {"kind": "const", "dt": 5e-3, "cone": 0.0, "dt_min": 0.0}, 4, (width, height))


def object_extra_cameras(k=4, width=800, height=800):
    """k more views of the object scene's grid, camera j drawn like the
    primary one from its own generator (seed SEED_BASE["object"] + j, j = 1..k):
    a list of (seed, origins, dirs)."""
    out = []
    for j in range(1, k + 1):
        seed = SEED_BASE["object"] + j
        o, d = object_camera_rays(width, height, np.random.default_rng(seed))
        out.append((seed, o, d))
    return out


def unbounded(seed=SEED_BASE["unbounded"], width=1280, height=832, R=128):
    rng = np.random.default_rng(seed)
    fracs = [0.15, 0.10, 0.06, 0.03]
    occ = np.zeros((4, R, R, R), np.uint8)
    boxes = np.zeros((4, 6), np.float32)
    # one world-space noise field over [-8,8]^3 sampled by every cascade
    lattices = []
    for o in range(4):
        cells = 8 * 2 ** o
        lattices.append((cells, rng.random((cells + 1,) * 3)))
    for k in range(4):
        half = 2.0 ** k
        boxes[k] = [-half, -half, -half, half, half, half]
        c = voxel_centres(R, -half, half)
        f = np.zeros((R, R, R))
        amp = 1.0
        for cells, V in lattices:
            Wx = _lattice_weights(c, -8.0, 8.0, cells)
            g = np.tensordot(Wx, V, axes=(1, 0))
            g = np.tensordot(g, Wx, axes=(1, 1))
            g = np.tensordot(g, Wx, axes=(1, 1))
            f += amp * g
            amp *= 0.5
        occ[k] = threshold_top(f, fracs[k])
    pos = rng.uniform(-0.5, 0.5, size=3)
    o, d = pinhole_rays(width, height, 60.0, random_rotation(rng), pos)
    return Workload("unbounded", occ, boxes, o, d, 0.05, 1e3,
                    {"kind": "cone", "dt": 0.0, "cone": 1.0 / 256.0, "dt_min": 1e-3}, 4, (width, height))


BATCH_SIDES = [1024] * 4 + [768] + [512] * 3 + [384] + [256] * 3 + [128] * 2 + [64] * 2


def batched(seed=SEED_BASE["batched"], n_scenes=16, ray_sides=None):
    """16 scenes of uneven grid size, occupancy and ray count."""
    rng = np.random.default_rng(seed)
    sides = list(BATCH_SIDES if ray_sides is None else ray_sides)[:n_scenes]
    out = []
    for s in range(n_scenes):
        R = int(rng.choice([64, 128, 256]))
        frac = float(rng.uniform(0.02, 0.20))
        c = voxel_centres(R, -1.5, 1.5)
        noise = value_noise(c, c, c, -1.5, 1.5, 4, 3, rng)
        occ = threshold_top(noise, frac)[None]
        o, d = object_camera_rays(sides[s], sides[s], rng)
        out.append(Workload(f"batched{s}", occ, _box(-1.5, 1.5), o, d, 2.0, 6.0,
                            {"kind": "const", "dt": 5e-3, "cone": 0.0, "dt_min": 0.0}, 4, (sides[s], sides[s]),
                            {"occupancy": frac}))
    return out


def composite_inputs(n_samples, n_rays, seed=SEED_BASE["composite"]):
    """sigma ~ exp(N(0,1)), rgb ~ U[0,1]^3 per sample; target pixel ~ U[0,1]^3."""
    rng = np.random.default_rng(seed)
    sigma = np.exp(rng.normal(size=n_samples)).astype(np.float32)
    rgb = rng.random((n_samples, 3)).astype(np.float32)
    target = rng.random((n_rays, 3)).astype(np.float32)
    return sigma, rgb, target


def blob_field(n_blobs=12, seed=SEED_BASE["render"]):
    """A synthetic radiance field standing in for a trained one: Gaussian blobs
    with centres ~ U(-0.7, 0.7)^3 (where the object scene's shells sit), radii
    ~ U(0.2, 0.5), densities ~ U(5, 40) and colours ~ U[0,1]^3.  Returns
    float32 arrays (centres [K,3], radii [K], densities [K], colours [K,3])."""
    rng = np.random.default_rng(seed)
    centres = rng.uniform(-0.7, 0.7, size=(n_blobs, 3)).astype(np.float32)
    radii = rng.uniform(0.2, 0.5, size=n_blobs).astype(np.float32)
    dens = rng.uniform(5.0, 40.0, size=n_blobs).astype(np.float32)
    cols = rng.random((n_blobs, 3)).astype(np.float32)
    return centres, radii, dens, cols


def workload(name, **kw):
    return {"small": small, "object": object_scene, "unbounded": unbounded}[name](**kw)


def random_rays(n, rng, lo=-2.0, hi=2.0):
    """Rays with origins in [lo,hi]^3 and random unit directions (tests)."""
    o = rng.uniform(lo, hi, size=(n, 3))
    d = rng.normal(size=(n, 3))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    return o.astype(np.float32), d.astype(np.float32)
