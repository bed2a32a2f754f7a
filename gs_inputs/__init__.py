"""Seeded synthetic inputs for the Gaussian-parameter path.

This module only *draws inputs*: Gaussian parameters, training cameras and
synthetic gradients.  It holds none of the method's arithmetic (no culling,
no optimizer math).  Both the CPU oracle and the HIP path consume what it
produces; neither imports the other.

Workload shapes follow the paper's setting: 59 FP32 parameters per Gaussian
(Sec. 2.3: mean 3, scale 3, quaternion 4, opacity 1, SH degree 3 = 48), large
aerial scenes rendered at 1152x864 (Table 2, Mill-19), 4M-40M Gaussians
(Sec. 5.6).  The paper's datasets are not available; these generators stand in
for them.

Column layout of one Gaussian (G = geometric group, A = appearance group):
  G[0:3] mean (x, y, z)         G[3:6] log-scale       G[6:10] quaternion (w, x, y, z)
  A[0]   opacity logit          A[1:49] SH coefficients, 16 x RGB
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

GEO_DIM = 10
APP_DIM = 49
TOTAL_DIM = GEO_DIM + APP_DIM

# ---------------------------------------------------------------------------
# Counter-based generator: SplitMix64 (Steele, Lea & Flood, "Fast splittable
# pseudorandom number generators", OOPSLA 2014).  The i-th output of a
# SplitMix64 stream seeded with s is mix(s + (i+1)*GAMMA).  The HIP harness
# kernel implements the same published definition independently.
# ---------------------------------------------------------------------------
GAMMA = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)


def _mix64(z: np.ndarray) -> np.ndarray:
    z = np.asarray(z, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = (z ^ (z >> np.uint64(30))) * _M1
        z = (z ^ (z >> np.uint64(27))) * _M2
    return z ^ (z >> np.uint64(31))


def splitmix_at(seed, index) -> np.ndarray:
    """Output number `index` (0-based) of the SplitMix64 stream seeded with `seed`."""
    s = np.asarray(seed, dtype=np.uint64)
    i = np.asarray(index, dtype=np.uint64)
    with np.errstate(over="ignore"):
        return _mix64(s + (i + np.uint64(1)) * GAMMA)


# Gradient value from one 64-bit hash: the four 16-bit fields are summed
# exactly (Irwin-Hall of order 4), centred, and scaled to standard deviation
# `sigma` with one FP64 multiply and one round-to-nearest cast to FP32.
_IH_MEAN2 = 4 * 65535            # twice the mean of the sum of four 16-bit fields
_IH_VAR = 4.0 * (65536.0 * 65536.0 - 1.0) / 12.0


def grad_scale(sigma: float) -> float:
    """FP64 factor that maps (2*S - 4*65535) to a value of std `sigma`."""
    return sigma / math.sqrt(_IH_VAR) / 2.0


def hash_grads(seed: int, step: int, keys: np.ndarray, cols: np.ndarray,
               sigma: float = 1e-3) -> np.ndarray:
    """Synthetic gradients g[i][j] for Gaussian key keys[i] and global column cols[j].

    key derivation: s1 = at(seed, step); s2 = at(s1, key); h = at(s2, col).
    Global columns are 0..9 for G and 10..58 for A.
    """
    keys = np.asarray(keys, dtype=np.uint64).reshape(-1, 1)
    cols = np.asarray(cols, dtype=np.uint64).reshape(1, -1)
    s1 = splitmix_at(np.uint64(seed), np.uint64(step))
    s2 = splitmix_at(s1, keys)
    h = splitmix_at(s2, cols)
    mask = np.uint64(0xFFFF)
    s = (h & mask) + ((h >> np.uint64(16)) & mask) + ((h >> np.uint64(32)) & mask) + (h >> np.uint64(48))
    centred = (s.astype(np.int64) * 2 - _IH_MEAN2).astype(np.float64)
    return (centred * grad_scale(sigma)).astype(np.float32)


def step_grads(seed: int, step: int, ids: np.ndarray, sigma: float = 1e-3):
    """Compact gradients for the visible ids of one step: (g_geo [M,10], g_app [M,49])."""
    g = hash_grads(seed, step, ids, np.arange(TOTAL_DIM), sigma)
    return np.ascontiguousarray(g[:, :GEO_DIM]), np.ascontiguousarray(g[:, GEO_DIM:])


# ---------------------------------------------------------------------------
# Scenes
# ---------------------------------------------------------------------------
@dataclass
class Scene:
    geo: np.ndarray          # [N,10] float32
    app: np.ndarray          # [N,49] float32

    @property
    def n(self) -> int:
        return self.geo.shape[0]


def make_scene(n: int, seed: int = 0, box=((-50, 50), (-50, 50), (-50, 50)),
               chunk: int = 1 << 22) -> Scene:
    """Gaussians drawn in the fixed order pos, log-scale, quat, opacity, SH.

    pos ~ U(box), log-scale ~ N(-3, 0.5), quat = normalised 4-D standard normal
    (uniform on S^3, stored w,x,y,z), opacity logit ~ N(0, 1), SH ~ N(0, 0.1).
    Generated in chunks so large N never materialises FP64 copies of everything.
    """
    rng = np.random.default_rng(seed)
    geo = np.empty((n, GEO_DIM), np.float32)
    app = np.empty((n, APP_DIM), np.float32)
    lo = np.array([b[0] for b in box], np.float64)
    hi = np.array([b[1] for b in box], np.float64)
    for s in range(0, n, chunk):
        e = min(n, s + chunk)
        k = e - s
        geo[s:e, 0:3] = rng.uniform(lo, hi, size=(k, 3))
        geo[s:e, 3:6] = rng.normal(-3.0, 0.5, size=(k, 3))
        q = rng.normal(size=(k, 4))
        q /= np.linalg.norm(q, axis=1, keepdims=True)
        geo[s:e, 6:10] = q
        app[s:e, 0] = rng.normal(0.0, 1.0, size=k)
        app[s:e, 1:] = rng.normal(0.0, 0.1, size=(k, APP_DIM - 1))
    return Scene(geo, app)


# ---------------------------------------------------------------------------
# Cameras (OpenCV axes: x right, y down, z forward; world up = +z)
# ---------------------------------------------------------------------------
@dataclass
class Camera:
    R: np.ndarray            # [3,3] float32, world -> camera
    t: np.ndarray            # [3] float32
    fx: float
    fy: float
    cx: float
    cy: float
    width: int
    height: int
    near: float = 0.01
    far: float = 1000.0

    def as_floats(self) -> np.ndarray:
        """Flat float32 vector: R(9), t(3), fx, fy, cx, cy, W, H, near, far."""
        return np.concatenate([
            self.R.astype(np.float32).ravel(), self.t.astype(np.float32),
            np.array([self.fx, self.fy, self.cx, self.cy, self.width, self.height,
                      self.near, self.far], np.float32)])


def look_at(center, forward, width, height, fx, fy, near=0.01, far=1000.0) -> Camera:
    f = np.asarray(forward, np.float64)
    f = f / np.linalg.norm(f)
    up = np.array([0.0, 0.0, 1.0])
    right = np.cross(f, up)
    if np.linalg.norm(right) < 1e-6:
        right = np.cross(f, np.array([0.0, 1.0, 0.0]))
    right /= np.linalg.norm(right)
    down = np.cross(f, right)
    R = np.stack([right, down, f]).astype(np.float64)
    t = -R @ np.asarray(center, np.float64)
    return Camera(R.astype(np.float32), t.astype(np.float32), float(fx), float(fy),
                  width / 2.0, height / 2.0, int(width), int(height), near, far)


def orbit_cameras(k: int, seed: int = 0, radius: float = 80.0, target_box: float = 20.0,
                  width: int = 1280, height: int = 720, focal: float = 1000.0) -> list[Camera]:
    """Cameras on a sphere of the given radius looking at U[-b,b]^3 targets."""
    rng = np.random.default_rng(seed + 1_000_003)
    cams = []
    for _ in range(k):
        d = rng.normal(size=3)
        c = radius * d / np.linalg.norm(d)
        tgt = rng.uniform(-target_box, target_box, size=3)
        cams.append(look_at(c, tgt - c, width, height, focal, focal))
    return cams


def aerial_cameras(k: int, half_x: float, half_y: float, seed: int = 0,
                   height_range=(150.0, 250.0), tilt_deg=(20.0, 45.0),
                   width: int = 1152, height: int = 864, focal: float = 1100.0, far: float = 1000.0) -> list[Camera]:
    """Half nadir, half oblique cameras over an aerial box (tilt from nadir in degrees)."""
    rng = np.random.default_rng(seed + 2_000_003)
    cams = []
    for i in range(k):
        c = np.array([rng.uniform(-half_x, half_x), rng.uniform(-half_y, half_y),
                      rng.uniform(*height_range)])
        if i % 2 == 0:
            f = np.array([0.0, 0.0, -1.0])
        else:
            tilt = math.radians(rng.uniform(*tilt_deg))
            az = rng.uniform(0.0, 2 * math.pi)
            f = np.array([math.sin(tilt) * math.cos(az), math.sin(tilt) * math.sin(az), -math.cos(tilt)])
        cams.append(look_at(c, f, width, height, focal, focal, far=far))
    return cams


# ---------------------------------------------------------------------------
# Workload recipes (sizes of the paper-shaped configurations)
# ---------------------------------------------------------------------------
LR_POS = 1.6e-4
LR_OTHER = 5e-3


def lr_columns() -> tuple[np.ndarray, np.ndarray]:
    """Per-column learning rates: positions 1.6e-4, everything else 5e-3."""
    lg = np.full(GEO_DIM, LR_OTHER, np.float32)
    lg[0:3] = LR_POS
    la = np.full(APP_DIM, LR_OTHER, np.float32)
    return lg, la


@dataclass
class Workload:
    name: str
    n: int
    steps: int
    scene_box: tuple
    cameras: list = field(default_factory=list)
    camera_order: np.ndarray | None = None
    seed: int = 0

    def camera_for_step(self, t: int) -> Camera:
        k = len(self.cameras)
        idx = (t - 1) % k
        if self.camera_order is not None:
            idx = int(self.camera_order[idx])
        return self.cameras[idx]


def workload(name: str, n: int | None = None, seed: int = 0, tilt_deg=(20.0, 45.0)) -> Workload:
    """Paper-shaped synthetic workloads.

    small  : 100k Gaussians in [-50,50]^3, 10 orbit cameras 1280x720 f=1000, 20 steps
    aerial4m / aerial18m / aerial40m: aerial boxes 1000x1000x100 / 2000x2000x150 /
             3000x3000x200 with 1600 / 3000 / 4000 cameras 1152x864 f=1100 at
             150-250 m, half nadir and half oblique; 200 / 500 / 1000 steps.
    aerial40m_f8: the 40M workload with the visible fraction matched to the
             paper's average use of 8.28% of the Gaussians per iteration: cameras
             at 900-1300 m with the far plane at 3000 m (mean f about 8.4%);
             nothing else changes.
    """
    if name == "small":
        n = n or 100_000
        box = ((-50, 50), (-50, 50), (-50, 50))
        return Workload(name, n, 20, box, orbit_cameras(10, seed), None, seed)
    spec = {"aerial4m": (4_000_000, 1000.0, 100.0, 1600, 200, (150.0, 250.0), 1000.0),
            "aerial18m": (18_000_000, 2000.0, 150.0, 3000, 500, (150.0, 250.0), 1000.0),
            "aerial40m": (40_000_000, 3000.0, 200.0, 4000, 1000, (150.0, 250.0), 1000.0),
            "aerial40m_f8": (40_000_000, 3000.0, 200.0, 4000, 1000, (900.0, 1300.0), 3000.0)}[name]
    n0, side, ztop, ncam, steps, heights, far = spec
    n = n or n0
    box = ((-side / 2, side / 2), (-side / 2, side / 2), (0.0, ztop))
    cams = aerial_cameras(ncam, side / 2, side / 2, seed, height_range=heights, tilt_deg=tilt_deg, far=far)
    order = np.random.default_rng(seed + 3_000_017).permutation(ncam)
    return Workload(name, n, steps, box, cams, order, seed)


def batched_scene_sizes(n_scenes: int = 16, lo: float = 5e5, hi: float = 8e6, seed: int = 0) -> list[int]:
    """Scene sizes log-uniform in [lo, hi] (seeded)."""
    rng = np.random.default_rng(seed + 4_000_037)
    return [int(round(math.exp(rng.uniform(math.log(lo), math.log(hi))))) for _ in range(n_scenes)]


def aerial_box_for(n: int, n_ref: int = 4_000_000, side_ref: float = 1000.0, height: float = 100.0):
    """Aerial box with the 4M-Gaussian workload's density: side 1000 * sqrt(n / 4M)."""
    half = side_ref * math.sqrt(n / n_ref) / 2
    return ((-half, half), (-half, half), (0.0, height)), half


def device_scene(n, box, seed, dev):
    """Seeded synthetic scene drawn on the device (same distributions as
    make_scene, torch's generator instead of numpy's)."""
    import torch
    gen = torch.Generator(device=dev)
    gen.manual_seed(seed)
    lo = torch.tensor([b[0] for b in box], device=dev, dtype=torch.float32)
    hi = torch.tensor([b[1] for b in box], device=dev, dtype=torch.float32)
    geo = torch.empty((n, 10), device=dev, dtype=torch.float32)
    geo[:, 0:3] = torch.rand((n, 3), generator=gen, device=dev) * (hi - lo) + lo
    geo[:, 3:6] = torch.randn((n, 3), generator=gen, device=dev) * 0.5 - 3.0
    q = torch.randn((n, 4), generator=gen, device=dev)
    geo[:, 6:10] = q / q.norm(dim=1, keepdim=True)
    app = torch.randn((n, 49), generator=gen, device=dev) * 0.1
    app[:, 0] = torch.randn(n, generator=gen, device=dev)
    return geo, app
