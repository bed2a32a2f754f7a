"""Seeded input generators: determinism, published generator values, shapes."""
import os

import numpy as np

import gs_inputs as gi

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def test_splitmix64_published_outputs():
    vals = [int(x) for x in open(os.path.join(GOLDEN, "splitmix64_seed1234567.txt"))
            if x.strip() and not x.startswith("#")]
    got = gi.splitmix_at(np.uint64(1234567), np.arange(5, dtype=np.uint64))
    assert [int(v) for v in got] == vals


def test_grads_deterministic_and_order_independent():
    ids = np.array([5, 17, 99, 3], np.uint32)
    a = gi.hash_grads(0, 7, ids, np.arange(59))
    b = gi.hash_grads(0, 7, ids[::-1], np.arange(59))[::-1]
    assert np.array_equal(a, b)
    assert not np.array_equal(a, gi.hash_grads(0, 8, ids, np.arange(59)))
    assert not np.array_equal(a, gi.hash_grads(1, 7, ids, np.arange(59)))
    g_geo, g_app = gi.step_grads(0, 7, ids)
    assert np.array_equal(np.concatenate([g_geo, g_app], 1), a)


def test_grads_distribution():
    g = gi.hash_grads(3, 1, np.arange(20000), np.arange(59)).astype(np.float64)
    assert abs(g.mean()) < 2e-6
    assert abs(g.std() / 1e-3 - 1.0) < 5e-3
    # Irwin-Hall of order 4 is bounded by +-2*sqrt(3) standard deviations
    assert np.abs(g).max() <= 2 * np.sqrt(3) * 1e-3 * (1 + 1e-6)


def test_scene_shapes_and_seed():
    s = gi.make_scene(1000, seed=4)
    t = gi.make_scene(1000, seed=4)
    assert s.geo.shape == (1000, 10) and s.app.shape == (1000, 49)
    assert s.geo.dtype == np.float32 and s.app.dtype == np.float32
    assert np.array_equal(s.geo, t.geo) and np.array_equal(s.app, t.app)
    q = s.geo[:, 6:10].astype(np.float64)
    assert np.allclose(np.linalg.norm(q, axis=1), 1.0, atol=1e-6)
    assert np.all(np.abs(s.geo[:, :3]) <= 50)


def test_camera_lookat_orthonormal_and_forward():
    cams = gi.orbit_cameras(5, seed=1) + gi.aerial_cameras(6, 500, 500, seed=1)
    for c in cams:
        R = c.R.astype(np.float64)
        assert np.allclose(R @ R.T, np.eye(3), atol=1e-6)
        assert np.linalg.det(R) > 0.999
    nadir = gi.aerial_cameras(2, 500, 500, seed=2)[0]
    # a nadir camera looks straight down: camera z axis = world -z
    assert np.allclose(nadir.R[2], [0, 0, -1], atol=1e-6)
    # a point below the camera projects to the principal point
    centre = -nadir.R.T.astype(np.float64) @ nadir.t.astype(np.float64)
    p = nadir.R.astype(np.float64) @ (centre - [0, 0, 100]) + nadir.t
    assert abs(p[0]) < 1e-3 and abs(p[1]) < 1e-3 and abs(p[2] - 100) < 1e-3


def test_workloads():
    w = gi.workload("small")
    assert w.n == 100_000 and len(w.cameras) == 10 and w.steps == 20
    a = gi.workload("aerial4m", n=1000)
    assert len(a.cameras) == 1600 and a.steps == 200
    assert sorted(a.camera_order.tolist()) == list(range(1600))
    assert a.camera_for_step(1) is a.cameras[a.camera_order[0]]
