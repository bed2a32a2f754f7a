"""Pins of the oracle's FP32 cull against geometry it does not compute itself.

The cull formula is not printed in the paper (Sec. 2.4 step 1 only says what
is culled); the oracle fixes it as the 3-sigma EWA screen box.  These tests
pin that arithmetic against:
  * exact tangent-plane extents of the 3-sigma ellipsoid (FP64 closed form,
    rotation from scipy), which the EWA linearisation must reproduce for small
    distant Gaussians -- along u, v and both diagonals, so a, b (with sign) and
    c are each checked;
  * brute-force projection of sampled ellipsoid surface points;
  * exact invariants (q vs -q, q vs 2q), near/far planes, NaN rows, behind-camera
    rows, centre-inside-image rows;
  * exp_gs against the libm exponential.
"""
import math

import numpy as np
import pytest
from scipy.spatial.transform import Rotation

import gs_inputs as gi
from oracle import oracle as orc

TAU = None


def _cam(fx=1000.0, W=1280, H=720, R=None, t=None, near=0.01, far=1000.0):
    R = np.eye(3, dtype=np.float32) if R is None else R.astype(np.float32)
    t = np.zeros(3, np.float32) if t is None else t.astype(np.float32)
    return gi.Camera(R, t, fx, fx, W / 2.0, H / 2.0, W, H, near, far)


def _small_far_gaussians(n, rng, cam):
    """Gaussians 20-80 units in front of a camera, inside 60% of the field of
    view, with 3-sigma sizes of a few pixels to tens of pixels."""
    z = rng.uniform(20, 80, n)
    u = rng.uniform(0.2, 0.8, n) * cam.width
    v = rng.uniform(0.2, 0.8, n) * cam.height
    xc = (u - cam.cx) / cam.fx * z
    yc = (v - cam.cy) / cam.fy * z
    pc = np.stack([xc, yc, z], 1)
    R = cam.R.astype(np.float64)
    world = (pc - cam.t.astype(np.float64)) @ R          # R^T (pc - t)
    geo = np.zeros((n, 10), np.float32)
    geo[:, :3] = world
    # sigma_px = sigma * f / z in [0.7, 7] px -> 3-sigma radius 2-20 px
    spx = rng.uniform(0.7, 7.0, (n, 3))
    geo[:, 3:6] = np.log(spx * z[:, None] / cam.fx)
    q = rng.normal(size=(n, 4))
    geo[:, 6:10] = q / np.linalg.norm(q, axis=1, keepdims=True)
    return geo


def _cov_cam(geo, cam):
    """FP64 camera-space centre and covariance from the definition of a 3D
    Gaussian: Sigma = Rq diag(exp(s))^2 Rq^T (rotation by scipy)."""
    g = geo.astype(np.float64)
    quat_xyzw = np.concatenate([g[:, 7:10], g[:, 6:7]], 1)
    Rq = Rotation.from_quat(quat_xyzw).as_matrix()
    S2 = np.exp(2 * g[:, 3:6])
    Sig = np.einsum("nij,nj,nkj->nik", Rq, S2, Rq)
    R = cam.R.astype(np.float64)
    mu = g[:, :3] @ R.T + cam.t.astype(np.float64)
    Sc = np.einsum("ij,njk,lk->nil", R, Sig, R)
    return mu, Sc


def _tangent_extent(mu, Sc, nvec_const, nz):
    """Range of k with plane normal n = nvec_const + k*(0,0,-1)... solved for
    the planes through the camera centre tangent to the 3-sigma ellipsoid:
        (n.mu)^2 = 9 n^T Sigma n,   n = (a0, a1, -k)."""
    a = np.asarray(nvec_const, np.float64)
    p = mu[:, 0] * a[0] + mu[:, 1] * a[1]               # a.mu_xy
    s_aa = (a[0] * a[0] * Sc[:, 0, 0] + 2 * a[0] * a[1] * Sc[:, 0, 1] + a[1] * a[1] * Sc[:, 1, 1])
    s_az = a[0] * Sc[:, 0, 2] + a[1] * Sc[:, 1, 2]
    # (p - k mu_z)^2 = 9 (s_aa - 2 k s_az + k^2 s_zz)
    A = mu[:, 2] ** 2 - 9 * Sc[:, 2, 2]
    B = -2 * (p * mu[:, 2] - 9 * s_az)
    Cc = p ** 2 - 9 * s_aa
    disc = np.sqrt(B * B - 4 * A * Cc)
    k1 = (-B - disc) / (2 * A)
    k2 = (-B + disc) / (2 * A)
    return np.minimum(k1, k2), np.maximum(k1, k2)


def test_exp_gs_matches_libm_within_two_ulp():
    x = np.linspace(-87, 88, 40001).astype(np.float32)
    e = orc.exp_gs(x).astype(np.float64)
    ref = np.exp(x.astype(np.float64))
    ulp = np.spacing(ref.astype(np.float32)).astype(np.float64)
    assert np.max(np.abs(e - ref) / ulp) <= 2.0
    assert orc.exp_gs(np.array([0.0], np.float32))[0] == 1.0
    assert np.isnan(orc.exp_gs(np.array([np.nan], np.float32))[0])


@pytest.mark.parametrize("seed", [0, 1])
def test_ewa_box_matches_tangent_planes(seed):
    rng = np.random.default_rng(seed)
    cams = [_cam(), gi.orbit_cameras(1, seed=seed)[0]]
    for cam in cams:
        geo = _small_far_gaussians(400, rng, cam)
        keep, det = orc.cull(geo, cam, detail=True)
        u, v = det[:, 3].astype(np.float64), det[:, 4].astype(np.float64)
        a = det[:, 5].astype(np.float64) - 0.3
        b = det[:, 6].astype(np.float64)
        c = det[:, 7].astype(np.float64) - 0.3
        mu, Sc = _cov_cam(geo, cam)
        f = cam.fx
        checks = [((1, 0), 1.0, u, a, cam.cx),            # x/z -> u
                  ((0, 1), 1.0, v, c, cam.cy),            # y/z -> v
                  ((1, 1), 1.0, None, a + 2 * b + c, None),
                  ((1, -1), 1.0, None, a - 2 * b + c, None)]
        for nvec, _, centre, var_px, off in checks:
            k1, k2 = _tangent_extent(mu, Sc, nvec, 1.0)
            half_exact = 0.5 * (k2 - k1) * f
            half_ewa = 3.0 * np.sqrt(var_px)
            rel = np.abs(half_exact - half_ewa) / half_ewa
            assert rel.max() < 2e-3, (nvec, rel.max())
            if centre is not None:
                mid_exact = 0.5 * (k1 + k2) * f + off
                assert np.max(np.abs(mid_exact - centre) / half_ewa) < 2e-2
        assert keep.all()


def test_sampled_ellipsoid_silhouette_matches_tangent_planes_and_radius():
    """Brute force: project 20k points of each 3-sigma ellipsoid surface.  Their
    extents lie inside the tangent-plane extents and reach them, and the EWA
    radius covers the sampled half-widths (the centre shift is second order)."""
    rng = np.random.default_rng(5)
    cam = _cam()
    geo = _small_far_gaussians(50, rng, cam)
    keep, det = orc.cull(geo, cam, detail=True)
    mu, Sc = _cov_cam(geo, cam)
    ku1, ku2 = _tangent_extent(mu, Sc, (1, 0), 1.0)
    kv1, kv2 = _tangent_extent(mu, Sc, (0, 1), 1.0)
    g = geo.astype(np.float64)
    quat_xyzw = np.concatenate([g[:, 7:10], g[:, 6:7]], 1)
    Rq = Rotation.from_quat(quat_xyzw).as_matrix()
    s = rng.normal(size=(20000, 3))
    s /= np.linalg.norm(s, axis=1, keepdims=True)
    for i in range(geo.shape[0]):
        L = Rq[i] * np.exp(g[i, 3:6])[None, :]
        pts = g[i, :3] + 3.0 * s @ L.T                  # 3-sigma ellipsoid surface
        pc = pts @ cam.R.astype(np.float64).T + cam.t
        xz, yz = pc[:, 0] / pc[:, 2], pc[:, 1] / pc[:, 2]
        for lo, hi, k1, k2 in ((xz.min(), xz.max(), ku1[i], ku2[i]), (yz.min(), yz.max(), kv1[i], kv2[i])):
            width = k2 - k1
            assert lo >= k1 - 1e-12 and hi <= k2 + 1e-12
            assert (hi - lo) >= 0.995 * width
        r = det[i, 10]
        half_u = 0.5 * (xz.max() - xz.min()) * cam.fx
        half_v = 0.5 * (yz.max() - yz.min()) * cam.fy
        assert half_u <= r and half_v <= r
        mid_u = 0.5 * (xz.max() + xz.min()) * cam.fx + cam.cx
        assert abs(mid_u - det[i, 3]) <= 0.02 * r


def test_quaternion_sign_and_scale_invariance_bitwise():
    rng = np.random.default_rng(1)
    sc = gi.make_scene(3000, seed=2)
    cam = gi.orbit_cameras(3, seed=0)[1]
    k0, d0 = orc.cull(sc.geo, cam, detail=True)
    neg = sc.geo.copy(); neg[:, 6:10] *= -1
    k1, d1 = orc.cull(neg, cam, detail=True)
    dbl = sc.geo.copy(); dbl[:, 6:10] *= 2
    k2, d2 = orc.cull(dbl, cam, detail=True)
    assert np.array_equal(k0, k1) and np.array_equal(d0.view(np.uint32), d1.view(np.uint32))
    assert np.array_equal(k0, k2) and np.array_equal(d0.view(np.uint32), d2.view(np.uint32))
    assert 0.2 < k0.mean() < 0.9


def test_isotropic_scale_mask_independent_of_rotation():
    rng = np.random.default_rng(3)
    sc = gi.make_scene(20000, seed=3)
    sc.geo[:, 4] = sc.geo[:, 3]
    sc.geo[:, 5] = sc.geo[:, 3]
    cam = gi.orbit_cameras(1, seed=4)[0]
    k0, d0 = orc.cull(sc.geo, cam, detail=True)
    other = sc.geo.copy()
    q = rng.normal(size=(other.shape[0], 4))
    other[:, 6:10] = q / np.linalg.norm(q, axis=1, keepdims=True)
    k1 = orc.cull(other, cam)
    diff = k0 != k1
    u, v, r = d0[:, 3], d0[:, 4], d0[:, 10]
    margin = np.minimum.reduce([u + r, cam.width - (u - r), v + r, cam.height - (v - r)])
    assert np.all(np.abs(margin[diff]) <= 1.5)


def test_near_far_and_degenerate_rows():
    cam = _cam(near=0.5, far=100.0)
    zs = np.array([0.5, np.nextafter(np.float32(0.5), np.float32(1)), 50.0,
                   np.nextafter(np.float32(100), np.float32(0)), 100.0, -5.0], np.float32)
    geo = np.zeros((zs.shape[0], 10), np.float32)
    geo[:, 2] = zs
    geo[:, 3:6] = -6.0
    geo[:, 6] = 1.0
    keep = orc.cull(geo, cam)
    assert keep.tolist() == [False, True, True, True, False, False]
    for col in range(10):
        g = geo[2:3].copy()
        g[0, col] = np.nan
        assert not orc.cull(g, cam)[0]


def test_centre_inside_image_implies_keep():
    rng = np.random.default_rng(8)
    cam = gi.orbit_cameras(1, seed=9)[0]
    sc = gi.make_scene(20000, seed=9)
    keep, det = orc.cull(sc.geo, cam, detail=True)
    u, v, z = det[:, 3], det[:, 4], det[:, 2]
    inside = (u >= 0) & (u < cam.width) & (v >= 0) & (v < cam.height) & (z > cam.near) & (z < cam.far)
    assert inside.sum() > 1000
    assert keep[inside].all()
    # and a centre more than the radius outside the image is culled
    r = det[:, 10]
    far_out = (u + r <= 0) | (u - r >= cam.width) | (v + r <= 0) | (v - r >= cam.height)
    assert not keep[far_out].any()


def test_compaction_brute_force():
    rng = np.random.default_rng(0)
    for n in [0, 1, 7, 1000]:
        keep = rng.random(n) < 0.3
        ids = orc.compact(keep)
        assert ids.dtype == np.uint32
        assert ids.tolist() == [i for i in range(n) if keep[i]]


def test_batched_lists_brute_force():
    """Union / per-camera lists of a batch agree with per-camera culls row by
    row, and the gradient sum adds each row's camera gradients in slot order."""
    rng = np.random.default_rng(4)
    sizes = [700, 1500, 300]
    geo = np.concatenate([gi.make_scene(n, seed=i).geo for i, n in enumerate(sizes)])
    row0 = np.concatenate([[0], np.cumsum(sizes)])
    cams = [gi.orbit_cameras(3, seed=10 + s) for s in range(3)]
    union, cam_pos, start = orc.cull_multi(geo, row0, cams)
    vis = np.zeros((geo.shape[0], 3), bool)
    for s in range(3):
        for c in range(3):
            vis[row0[s]:row0[s + 1], c] = orc.cull(geo[row0[s]:row0[s + 1]], cams[s][c])
    assert np.array_equal(union, np.nonzero(vis.any(1))[0])
    for c in range(3):
        assert np.array_equal(union[cam_pos[c]], np.nonzero(vis[:, c])[0])
        for s in range(3):
            assert start[s, 1 + c] == vis[:row0[s], c].sum()
    for s in range(3):
        assert start[s, 0] == vis[:row0[s]].any(1).sum()
    g_cam = [rng.normal(size=(cp.shape[0], 5)).astype(np.float32) for cp in cam_pos]
    out = orc.grad_sum_multi(cam_pos, g_cam, union.shape[0])
    for p in rng.choice(union.shape[0], 50, replace=False):
        acc = np.zeros(5, np.float32)
        for c in range(3):
            hit = np.nonzero(cam_pos[c] == p)[0]
            if hit.size:
                acc = acc + g_cam[c][hit[0]]
        assert np.array_equal(out[p], acc)
