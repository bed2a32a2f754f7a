"""GPU parity of the batched form (many scenes x many cameras per launch),
the autotuned variants and hipGraph replay with a device step counter."""
import sys

import numpy as np
import pytest
import torch

import gs_inputs as gi
from oracle import oracle as orc

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def g():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2509_15645_amd import gsdp
    return gsdp


def bits(a):
    return np.ascontiguousarray(a, np.float32).view(np.uint32)


def _morton(pos):
    """Permutation sorting rows by the 30-bit Morton code of their position
    (10 bits per axis over the rows' bounding box)."""
    lo, hi = pos.min(0), pos.max(0)
    q = ((pos - lo) / np.maximum(hi - lo, 1e-30) * 1023).astype(np.int64).clip(0, 1023)
    code = np.zeros(pos.shape[0], np.int64)
    for b in range(10):
        for a in range(3):
            code |= ((q[:, a] >> b) & 1) << (3 * b + a)
    return np.argsort(code, kind="stable")


def _batch(sizes, cams_per_scene, n_sets, seed=0, spatial=False, aerial=False):
    """Scenes of uneven size concatenated on 1024-row boundaries (padding rows
    have NaN positions and are never visible); spatial: each scene's rows
    sorted by the Morton code of their position; aerial: the aerial box of
    the scene's size with nadir and oblique cameras above it (else a cube
    with orbiting cameras)."""
    geos, apps, row0 = [], [], [0]
    sets = [[] for _ in range(n_sets)]
    for s, n in enumerate(sizes):
        if aerial:
            box, half = gi.aerial_box_for(n)
            sc = gi.make_scene(n, seed=seed + s, box=box)
        else:
            sc = gi.make_scene(n, seed=seed + s)
        geo_s, app_s = sc.geo, sc.app
        if spatial:
            perm = _morton(geo_s[:, :3].astype(np.float64))
            geo_s, app_s = geo_s[perm], app_s[perm]
        pad = (-n) % 1024
        g = np.concatenate([geo_s, np.full((pad, 10), np.nan, np.float32)])
        g[n:, 6] = 1.0
        geos.append(g)
        apps.append(np.concatenate([app_s, np.zeros((pad, 49), np.float32)]))
        row0.append(row0[-1] + n + pad)
        if aerial:
            cams = gi.aerial_cameras(cams_per_scene * n_sets, half, half, seed=seed + 100 * s)
        else:
            cams = gi.orbit_cameras(cams_per_scene * n_sets, seed=seed + 100 * s)
        for k in range(n_sets):
            sets[k].append(cams[k * cams_per_scene:(k + 1) * cams_per_scene])
    return np.concatenate(geos), np.concatenate(apps), np.array(row0), sets


def _compare_lists(multi, ref, tag):
    u, ids, cc, cams, ss = multi.lists()
    union, cam_pos, start = ref
    assert u == union.shape[0], tag
    assert np.array_equal(ids, union.astype(np.uint32)), tag
    for c in range(len(cam_pos)):
        assert cc[c] == cam_pos[c].shape[0], (tag, c)
        assert np.array_equal(cams[c], cam_pos[c].astype(np.uint32)), (tag, c)
    assert np.array_equal(ss.astype(np.int64), start), tag
    return u, cc


@pytest.mark.parametrize("kind", ["generated", "morton", "aerial-morton"])
def test_batched_scenes_cameras_vs_oracle(g, kind):
    """With rows in spatial order most wavefronts lie outside most cameras'
    frusta, so the wavefront box test decides them; the lists, sums and
    states must not change.  The aerial case uses all 32 camera slots."""
    if kind == "aerial-morton":
        sizes, C = [40_000, 120_000, 25_000], 32
    else:
        sizes, C = [30_000, 100_000, 7_000, 60_000], 8
    n_sets, steps = 2, 3
    geo, app, row0, sets = _batch(sizes, C, n_sets, spatial=kind != "generated", aerial=kind.startswith("aerial"))
    lg, la = gi.lr_columns()
    model = g.Model(geo, app, lg, la, max_steps=16, cull_mode=1, app_state="bf16", sr_seed=5)
    o4 = orc.DeferredF32(geo, app, lg, la, app_state="bf16", sr_seed=5)
    multi = g.Multi(model, row0, sets)
    D = 59
    g_cam_dev = torch.zeros((C, multi.cap_cam, D), dtype=torch.float32, device="cuda")
    out_g = torch.zeros((multi.cap_union, 10), dtype=torch.float32, device="cuda")
    out_a = torch.zeros((multi.cap_union, 49), dtype=torch.float32, device="cuda")
    gath_g = torch.zeros((multi.cap_union, 10), dtype=torch.float32, device="cuda")
    gath_a = torch.zeros((multi.cap_union, 49), dtype=torch.float32, device="cuda")
    rng = np.random.default_rng(7)
    for t in range(1, steps + 1):
        g.gs_cull_multi(model, multi, t)
        # the union's current rows, gathered once for all cameras
        g.gs_gather(model, t, multi.union_ids, multi.union_count, gath_g, gath_a, capacity=multi.cap_union)
        torch.cuda.synchronize()
        ref = orc.cull_multi(o4.current_geo(t), row0, sets[(t - 1) % n_sets])
        u, cc = _compare_lists(multi, ref, f"step {t}")
        cg, ca = o4.current(t, ref[0])
        assert np.array_equal(bits(gath_g[:u].cpu().numpy()), bits(cg)), f"gather geo step {t}"
        assert np.array_equal(bits(gath_a[:u].cpu().numpy()), bits(ca)), f"gather app step {t}"
        g_cam = [rng.normal(0, 1e-3, (cc[c], D)).astype(np.float32) for c in range(C)]
        g_cam_dev.zero_()
        for c in range(C):
            g_cam_dev[c, :cc[c]] = torch.from_numpy(g_cam[c]).cuda()
        g.gs_grad_sum_multi(multi, 49, g_cam_dev, out_g, out_a)
        gsum = orc.grad_sum_multi(ref[1], g_cam, u)
        torch.cuda.synchronize()
        assert np.array_equal(bits(out_g[:u].cpu().numpy()), bits(gsum[:, :10])), t
        assert np.array_equal(bits(out_a[:u].cpu().numpy()), bits(gsum[:, 10:])), t
        # the recorded chunk starts: per 128 union positions and camera slot,
        # the first list entry at or after the chunk (a sorted-search of the lists)
        nch = (u + 127) // 128
        cs = multi.chunk_start[:nch].cpu().numpy().view(np.uint32)
        pos = multi.cam_pos.cpu().numpy().view(np.uint32)
        for c in range(C):
            want = np.searchsorted(pos[c, :cc[c]], 128 * np.arange(nch), side="left")
            assert np.array_equal(cs[:, c], want), (t, c)
        # and the same sum with binary searches instead of the chunk starts
        saved = multi.c.chunk_start
        multi.c.chunk_start = None
        og2, oa2 = torch.zeros_like(out_g), torch.zeros_like(out_a)
        g.gs_grad_sum_multi(multi, 49, g_cam_dev, og2, oa2)
        multi.c.chunk_start = saved
        torch.cuda.synchronize()
        assert torch.equal(og2[:u].view(torch.int32), out_g[:u].view(torch.int32)), t
        assert torch.equal(oa2[:u].view(torch.int32), out_a[:u].view(torch.int32)), t
        g.gs_adam_step_deferred(model, t, multi.union_ids, multi.union_count, out_g, out_a,
                                capacity=multi.cap_union)
        o4.step(t, ref[0], gsum[:, :10], gsum[:, 10:])
        say(f"[batched] step {t}: union {u} per-camera {cc}")
    st = model.state()
    for k, name in ((0, "geo"), (1, "app")):
        for part, refv in (("w", o4.w[k]), ("m", o4.m[k]), ("v", o4.v[k])):
            got = st[f"{name}_{part}"]
            assert np.array_equal(bits(got), bits(refv)), f"{name}_{part}"


def test_grad_sum_union_capacity_overflow(g):
    """A union capacity below the union's size, with a ragged last chunk: the
    union count is reported in full, the first cap_union ids are written, the
    camera lists (large enough) still name positions past the capacity, and
    the gradient sums of the first cap_union positions equal the oracle's,
    with the recorded chunk starts and with binary searches."""
    sizes, C = [30_000, 60_000], 8
    geo, app, row0, sets = _batch(sizes, C, 1, seed=13)
    lg, la = gi.lr_columns()
    model = g.Model(geo, app, lg, la, max_steps=8, cull_mode=1)
    ref = orc.cull_multi(geo, row0, sets[0])
    U = ref[0].shape[0]
    cap = (U // 2) // 128 * 128 + 37
    assert 128 < cap < U
    multi = g.Multi(model, row0, sets, cap_union=cap)
    g.gs_cull_multi(model, multi, 1)
    torch.cuda.synchronize()
    u, ids, cc, cams, _ = multi.lists()
    assert u == U and np.array_equal(ids, ref[0][:cap].astype(np.uint32))
    assert any(int(c.max()) >= cap for c in cams if c.size), "no list names a position past the capacity"
    for c in range(C):
        assert np.array_equal(cams[c], ref[1][c].astype(np.uint32)), c
    D = 59
    rng = np.random.default_rng(17)
    g_cam = [rng.normal(0, 1e-3, (cc[c], D)).astype(np.float32) for c in range(C)]
    g_cam_dev = torch.zeros((C, multi.cap_cam, D), dtype=torch.float32, device="cuda")
    for c in range(C):
        g_cam_dev[c, :cc[c]] = torch.from_numpy(g_cam[c]).cuda()
    gsum = orc.grad_sum_multi(ref[1], g_cam, U)
    for use_chunks in (True, False):
        saved = multi.c.chunk_start
        if not use_chunks:
            multi.c.chunk_start = None
        out_g = torch.full((cap, 10), 7.0, dtype=torch.float32, device="cuda")
        out_a = torch.full((cap, 49), 7.0, dtype=torch.float32, device="cuda")
        g.gs_grad_sum_multi(multi, 49, g_cam_dev, out_g, out_a)
        multi.c.chunk_start = saved
        torch.cuda.synchronize()
        assert np.array_equal(bits(out_g.cpu().numpy()), bits(gsum[:cap, :10])), use_chunks
        assert np.array_equal(bits(out_a.cpu().numpy()), bits(gsum[:cap, 10:])), use_chunks
    say(f"[union overflow] union {U} capacity {cap}: sums of the first {cap} positions equal the oracle's")


def test_batched_variants_agree_and_autotune(g):
    sizes, C = [50_000, 20_000, 80_000], 16
    geo, app, row0, sets = _batch(sizes, C, 1, seed=3)
    lg, la = gi.lr_columns()
    model = g.Model(geo, app, lg, la, max_steps=8, cull_mode=1)
    multi = g.Multi(model, row0, sets)
    ref = orc.cull_multi(geo, row0, sets[0])
    for v in range(15):
        multi.c.variant = v
        g.gs_cull_multi(model, multi, 1)
        torch.cuda.synchronize()
        _compare_lists(multi, ref, f"variant {v}")
    times = g.gs_cull_multi_autotune(model, multi, 1)
    say(f"[autotune] times ms {['%.3f' % x for x in times]} -> variant {multi.c.variant}")
    assert len(times) == 15 and 0 <= multi.c.variant < 15
    assert times[multi.c.variant] == min(times)
    g.gs_cull_multi(model, multi, 1)
    torch.cuda.synchronize()
    _compare_lists(multi, ref, "after autotune")
    assert model.ws_header()["error"] == 0


def _graph_step(g, model, multi, g_cam_dev, out_g, out_a, gath_g, gath_a):
    g.gs_cull_multi(model, multi, 0)
    g.gs_gather(model, 0, multi.union_ids, multi.union_count, gath_g, gath_a, capacity=multi.cap_union)
    g.gs_grad_sum_multi(multi, 49, g_cam_dev, out_g, out_a)
    g.gs_adam_step_deferred(model, 0, multi.union_ids, multi.union_count, out_g, out_a, capacity=multi.cap_union)
    g.gs_step_advance(model.step_dev)


def test_batched_step_graph_replay_matches_eager(g):
    """One batched step captured in a hipGraph with the step read from device
    memory, replayed 4 times: every replay equals the eager step."""
    sizes, C, n_sets = [20_000, 40_000], 4, 2
    geo, app, row0, sets = _batch(sizes, C, n_sets, seed=9)
    lg, la = gi.lr_columns()
    mk = lambda: g.Model(geo, app, lg, la, max_steps=16, cull_mode=1, app_state="bf16", sr_seed=2)
    eager, graphed = mk(), mk()
    me, mg = g.Multi(eager, row0, sets), g.Multi(graphed, row0, sets)
    D = 59
    bufs = {}
    for name, mu in (("e", me), ("g", mg)):
        gc = torch.from_numpy(np.random.default_rng(1).normal(0, 1e-3, (C, mu.cap_cam, D)).astype(np.float32)).cuda()
        bufs[name] = (gc, torch.zeros((mu.cap_union, 10), device="cuda"), torch.zeros((mu.cap_union, 49), device="cuda"),
                      torch.zeros((mu.cap_union, 10), device="cuda"), torch.zeros((mu.cap_union, 49), device="cuda"))
    graphed.step_dev.fill_(1)
    torch.cuda.synchronize()
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        pass
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        _graph_step(g, graphed, mg, *bufs["g"])
    torch.cuda.synchronize()
    for t in range(1, 5):
        ge, oge, oae, gge, gae = bufs["e"]
        g.gs_cull_multi(eager, me, t)
        g.gs_gather(eager, t, me.union_ids, me.union_count, gge, gae, capacity=me.cap_union)
        g.gs_grad_sum_multi(me, 49, ge, oge, oae)
        g.gs_adam_step_deferred(eager, t, me.union_ids, me.union_count, oge, oae, capacity=me.cap_union)
        graph.replay()
        torch.cuda.synchronize()
        assert int(graphed.step_dev.item()) == t + 1
        a, b = eager.state(), graphed.state()
        for key in a:
            # compare bit patterns: padding rows hold NaN geometry
            assert a[key].tobytes() == b[key].tobytes(), (t, key)
        ue, ug = me.lists(), mg.lists()
        assert ue[0] == ug[0] and np.array_equal(ue[1], ug[1])
        u = ue[0]
        for k in (3, 4):
            assert torch.equal(bufs["e"][k][:u].view(torch.int32), bufs["g"][k][:u].view(torch.int32)), (t, k)
        say(f"[graph] replay {t}: union {ue[0]} identical to eager")


def _crop(cam, x0, x1):
    return gi.Camera(cam.R, cam.t, cam.fx, cam.fy, cam.cx - x0, cam.cy, x1 - x0, cam.height, cam.near, cam.far)


def test_image_split_planner_matches_oracle_search(g):
    """Balance-aware image split (Sec. 4.4): 5-step binary search from the
    midpoint toward the less populated side, counts from both crops."""
    sc = gi.make_scene(100_000, seed=21)
    lg, la = gi.lr_columns()
    model = g.Model(sc.geo, sc.app, lg, la, max_steps=8, cull_mode=1)
    for cam in gi.orbit_cameras(3, seed=22):
        x, counts = g.gs_plan_image_split(model, cam, 1, 0.3)
        xx, ref = orc.image_split_plan(sc.geo, cam, 0.3)
        say(f"[split] full {ref[0]} -> x={x} left {counts[1]} right {counts[2]}")
        assert counts[0] == ref[0] and x == xx
        if x == 0:
            continue
        assert counts[1] == ref[1] and counts[2] == ref[2]
        assert abs(ref[1] - ref[2]) < 0.35 * (ref[1] + ref[2])
        # the split image trains as a batch of the two crops
        multi = g.Multi(model, [0, model.n], [[[_crop(cam, 0, x), _crop(cam, x, cam.width)]]])
        g.gs_cull_multi(model, multi, 1)
        torch.cuda.synchronize()
        ref_l = orc.cull_multi(sc.geo, [0, model.n], [[orc.crop_camera(cam, 0, x), orc.crop_camera(cam, x, cam.width)]])
        _compare_lists(multi, ref_l, "split batch")
    x, _ = g.gs_plan_image_split(model, gi.orbit_cameras(1, seed=22)[0], 1, 0.99)
    assert x == 0


def test_split_image_training_steps_vs_oracle(g):
    """Training with the balance-aware split (Sec. 4.4) end to end: each step
    plans the split on the current geometry, culls both crops as one batch,
    gathers the union, sums the two crops' gradients in crop order and takes
    one deferred Adam step.  Split column, lists, gathered rows, summed
    gradients and the final state against the oracle's plan, cull, restore,
    sum and FP32 deferred model, bit for bit."""
    n, steps, D = 100_000, 4, 59
    sc = gi.make_scene(n, seed=31)
    lg, la = gi.lr_columns()
    model = g.Model(sc.geo, sc.app, lg, la, max_steps=8, cull_mode=1)
    o3 = orc.DeferredF32(sc.geo, sc.app, lg, la)
    cams = gi.orbit_cameras(steps, seed=32)
    rng = np.random.default_rng(33)
    splits = 0
    for t in range(1, steps + 1):
        cam = cams[t - 1]
        x, counts = g.gs_plan_image_split(model, cam, t, 0.3)
        cur = o3.current_geo(t)
        xx, ref_counts = orc.image_split_plan(cur, cam, 0.3)
        assert x == xx and counts[0] == ref_counts[0], t
        if x:
            assert tuple(counts[1:]) == tuple(ref_counts[1:]), t
        if x:
            crops, ref_crops = [_crop(cam, 0, x), _crop(cam, x, cam.width)], \
                [orc.crop_camera(cam, 0, x), orc.crop_camera(cam, x, cam.width)]
            splits += 1
        else:
            crops, ref_crops = [cam], [cam]
        multi = g.Multi(model, [0, n], [[crops]])
        gath_g = torch.zeros((multi.cap_union, 10), device="cuda")
        gath_a = torch.zeros((multi.cap_union, 49), device="cuda")
        out_g = torch.zeros((multi.cap_union, 10), device="cuda")
        out_a = torch.zeros((multi.cap_union, 49), device="cuda")
        # the batch's camera set is (t - 1) % n_sets = 0 with one set
        g.gs_cull_multi(model, multi, t)
        g.gs_gather(model, t, multi.union_ids, multi.union_count, gath_g, gath_a, capacity=multi.cap_union)
        torch.cuda.synchronize()
        ref = orc.cull_multi(cur, [0, n], [ref_crops])
        u, cc = _compare_lists(multi, ref, f"split step {t}")
        cg, ca = o3.current(t, ref[0])
        assert np.array_equal(bits(gath_g[:u].cpu().numpy()), bits(cg)), t
        assert np.array_equal(bits(gath_a[:u].cpu().numpy()), bits(ca)), t
        g_cam = [rng.normal(0, 1e-3, (cc[c], D)).astype(np.float32) for c in range(len(crops))]
        g_cam_dev = torch.zeros((len(crops), multi.cap_cam, D), dtype=torch.float32, device="cuda")
        for c in range(len(crops)):
            g_cam_dev[c, :cc[c]] = torch.from_numpy(g_cam[c]).cuda()
        g.gs_grad_sum_multi(multi, 49, g_cam_dev, out_g, out_a)
        g.gs_adam_step_deferred(model, t, multi.union_ids, multi.union_count, out_g, out_a, capacity=multi.cap_union)
        gsum = orc.grad_sum_multi(ref[1], g_cam, u)
        torch.cuda.synchronize()
        assert np.array_equal(bits(out_g[:u].cpu().numpy()), bits(gsum[:, :10])), t
        assert np.array_equal(bits(out_a[:u].cpu().numpy()), bits(gsum[:, 10:])), t
        o3.step(t, ref[0].astype(np.uint32), gsum[:, :10], gsum[:, 10:])
        say(f"[split train] step {t}: x={x} union {u} crops {cc}")
    assert splits >= 2
    g.gs_adam_flush(model, steps)
    o3.flush(steps)
    st = model.state()
    for k, name in ((0, "geo"), (1, "app")):
        for part, refv in (("w", o3.w[k]), ("m", o3.m[k]), ("v", o3.v[k])):
            assert np.array_equal(bits(st[f"{name}_{part}"]), bits(refv)), f"{name}_{part}"
