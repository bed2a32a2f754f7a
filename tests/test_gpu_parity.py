"""GPU parity of the HIP path against the CPU oracle (run with -m gpu).

Cull + compaction: visible-id lists bit-exact against the oracle's FP32 cull
of the same FP32 current geometry (the oracle's own FP32 state model O3).
Gather / Adam / flush: bit-exact against O3, and within the FP32 tolerance of
the dense FP64 Adam definition (error per element |w - w64| / max(|w64|, tau),
tau = the group's initial scale; bound 1e-6 for the 20-step workload).
"""
import sys

import numpy as np
import pytest
import torch

import gs_inputs as gi
from oracle import oracle as orc
from precision_bound import check_bound

pytestmark = pytest.mark.gpu

TAU_GEO = np.array([1, 1, 1, .5, .5, .5, .5, .5, .5, .5])
TAU_APP = np.array([1.0] + [0.1] * 48)


def say(*a):
    print(*a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def g():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2509_15645_amd import gsdp
    return gsdp


def u32(t):
    return t.cpu().numpy().view(np.uint32)


def bits(a):
    return np.ascontiguousarray(a, np.float32).view(np.uint32)


def run_cull(g, model, cam, t, cap=None, fill=-1):
    cap = max(model.n, 1) if cap is None else cap
    ids = torch.full((max(cap, 1),), fill, dtype=torch.int32, device="cuda")
    count = torch.zeros(1, dtype=torch.int32, device="cuda")
    g.gs_cull(model, cam, t, ids, count, capacity=cap)
    torch.cuda.synchronize()
    m = int(count.item())
    return ids, count, m


def model_for(g, geo, app=None, **kw):
    n = geo.shape[0]
    if app is None:
        app = np.zeros((n, 49), np.float32)
    lg, la = gi.lr_columns()
    kw.setdefault("max_steps", 64)
    return g.Model(geo, app, lg, la, **kw)


# ---------------------------------------------------------------- cull
# cull_mode, cull summaries: the exact cull, the band cull from the geometry
# rows and the band cull from the summaries
CULLS = [(0, False), (1, False), (1, True)]


@pytest.mark.parametrize("mode,summ", CULLS)
@pytest.mark.parametrize("n", [0, 1, 5, 1023, 1024, 1025, 3007, 100_000])
def test_cull_step1_matches_oracle(g, n, mode, summ):
    say(f"[cull] n={n} mode={mode} summaries={summ}")
    sc = gi.make_scene(n, seed=n % 7)
    model = model_for(g, sc.geo, sc.app, cull_mode=mode, cull_summary=summ)
    for cam in gi.orbit_cameras(4, seed=n % 5):
        ids, count, m = run_cull(g, model, cam, 1)
        ref = orc.compact(orc.cull(sc.geo, cam))
        assert m == ref.shape[0]
        assert np.array_equal(u32(ids[:m]), ref)
    assert model.ws_header()["error"] == 0


def test_cull_aerial_full_scale_step1(g):
    w = gi.workload("aerial4m")
    say(f"[cull aerial] n={w.n}")
    sc = gi.make_scene(w.n, seed=0, box=w.scene_box)
    model = model_for(g, sc.geo, sc.app)
    fr = []
    for t in (1, 2, 3):
        cam = w.camera_for_step(t)
        ids, count, m = run_cull(g, model, cam, 1)
        ref = orc.compact(orc.cull(sc.geo, cam))
        assert m == ref.shape[0]
        assert np.array_equal(u32(ids[:m]), ref)
        fr.append(m / w.n)
    say(f"[cull aerial] visible fractions {fr}")


def test_cull_aerial18m_group_prefix(g):
    """18M Gaussians (the large aerial configuration): more than 16384 tiles,
    so the compaction takes the per-group sums (the smaller models sum the
    earlier tiles directly).  Ids bit-exact against the oracle's cull."""
    w = gi.workload("aerial18m")
    say(f"[cull aerial18m] n={w.n}")
    sc = gi.make_scene(w.n, seed=1, box=w.scene_box)
    model = model_for(g, sc.geo, np.zeros((w.n, 1), np.float32))
    del sc.app
    for t in (1, 2):
        cam = w.camera_for_step(t)
        ids, count, m = run_cull(g, model, cam, 1)
        ref = orc.compact(orc.cull(sc.geo, cam))
        assert m == ref.shape[0]
        assert np.array_equal(u32(ids[:m]), ref)
        say(f"[cull aerial18m] step {t}: M={m}")
    assert model.ws_header()["error"] == 0


def _boundary_scene(cam, n, rng):
    """Gaussians whose centres sit on and around the image border and the
    near/far planes, plus NaN, Inf and behind-camera rows."""
    u = rng.choice([-8.0, -3.0, -1.0, -0.5, 0.0, 0.25, 1.0, cam.width - 1.0, cam.width - 0.5, cam.width,
                    cam.width + 0.5, cam.width + 3.0], n) + rng.normal(0, 0.3, n)
    v = rng.uniform(-10, cam.height + 10, n)
    swap = rng.random(n) < 0.5
    u2 = np.where(swap, rng.uniform(-10, cam.width + 10, n), u)
    v2 = np.where(swap, rng.choice([-4.0, -1.0, 0.0, cam.height - 0.5, cam.height, cam.height + 2.0], n)
                  + rng.normal(0, 0.3, n), v)
    z = rng.choice([cam.near, cam.near * 1.0000001, 1.0, 20.0, 200.0, cam.far * 0.9999999, cam.far], n)
    z = z * np.where(rng.random(n) < 0.05, -1, 1)
    xc = (u2 - cam.cx) / cam.fx * z
    yc = (v2 - cam.cy) / cam.fy * z
    pc = np.stack([xc, yc, z], 1)
    world = (pc - cam.t.astype(np.float64)) @ cam.R.astype(np.float64)
    geo = np.zeros((n, 10), np.float32)
    geo[:, :3] = world
    geo[:, 3:6] = rng.normal(-3, 1.5, (n, 3))
    q = rng.normal(size=(n, 4))
    geo[:, 6:10] = q / np.linalg.norm(q, axis=1, keepdims=True)
    bad = rng.choice(n, n // 50, replace=False)
    geo[bad, rng.integers(0, 10, bad.shape[0])] = rng.choice([np.nan, np.inf, -np.inf], bad.shape[0])
    geo[rng.choice(n, 5, replace=False), 6:10] = 0.0        # zero quaternion
    geo[rng.choice(n, 5, replace=False), 3:6] = 200.0       # huge scale (exp clamp)
    geo[rng.choice(n, 5, replace=False), 3:6] = -200.0      # tiny scale
    return geo


@pytest.mark.parametrize("mode,summ", CULLS)
def test_cull_boundary_and_degenerate_rows(g, mode, summ):
    rng = np.random.default_rng(42)
    for seed, cam in enumerate(gi.orbit_cameras(3, seed=3)):
        geo = _boundary_scene(cam, 50_000, rng)
        model = model_for(g, geo, cull_mode=mode, cull_summary=summ)
        ids, count, m = run_cull(g, model, cam, 1)
        keep = orc.cull(geo, cam)
        ref = orc.compact(keep)
        say(f"[cull boundary] cam {seed}: M={m} ref={ref.shape[0]}")
        assert m == ref.shape[0]
        assert np.array_equal(u32(ids[:m]), ref)


def test_cull_capacity_overflow_and_determinism(g):
    sc = gi.make_scene(30_000, seed=9)
    model = model_for(g, sc.geo, sc.app)
    cam = gi.orbit_cameras(1, seed=9)[0]
    ref = orc.compact(orc.cull(sc.geo, cam))
    cap = ref.shape[0] // 2
    ids, count, m = run_cull(g, model, cam, 1, cap=cap + 100, fill=-7)
    assert m == ref.shape[0]
    ids2, _, m2 = run_cull(g, model, cam, 1, cap=cap)
    assert m2 == ref.shape[0]
    assert np.array_equal(u32(ids2), ref[:cap])
    # capacity 0 still counts
    _, _, m0 = run_cull(g, model, cam, 1, cap=0)
    assert m0 == ref.shape[0]
    a, _, _ = run_cull(g, model, cam, 1)
    b, _, _ = run_cull(g, model, cam, 1)
    assert torch.equal(a, b)


# ---------------------------------------------------------------- harness pieces
def test_synth_grad_matches_host_generator(g):
    rng = np.random.default_rng(0)
    ids = np.sort(rng.choice(1 << 22, 5000, replace=False)).astype(np.uint32)
    dids = torch.from_numpy(ids.view(np.int32)).cuda()
    count = torch.tensor([ids.shape[0]], dtype=torch.int32, device="cuda")
    for col0, dim in ((0, 10), (10, 49)):
        out = torch.zeros((ids.shape[0], dim), dtype=torch.float32, device="cuda")
        g.gs_synth_grad(7, 3, dids, count, out, col0)
        ref = gi.hash_grads(7, 3, ids, np.arange(col0, col0 + dim))
        assert np.array_equal(bits(out.cpu().numpy()), bits(ref))


def test_scatter_grad(g):
    rng = np.random.default_rng(1)
    n, m, dim = 10_000, 3_000, 49
    ids = np.sort(rng.choice(n, m, replace=False)).astype(np.int32)
    gc = rng.normal(size=(m, dim)).astype(np.float32)
    dids = torch.from_numpy(ids).cuda()
    count = torch.tensor([m], dtype=torch.int32, device="cuda")
    dense = torch.zeros((n, dim), dtype=torch.float32, device="cuda")
    dgc = torch.from_numpy(gc).cuda()
    g.gs_scatter_grad(dids, count, dgc, dense)
    ref = np.zeros((n, dim), np.float32)
    ref[ids] = gc
    assert np.array_equal(dense.cpu().numpy(), ref)
    g.gs_scatter_grad(dids, count, dgc, dense, accumulate=True)
    assert np.array_equal(dense.cpu().numpy(), ref + ref)


# ---------------------------------------------------------------- full path
def _compare_state(model, o3, tag):
    st = model.state()
    for k, name in ((0, "geo"), (1, "app")):
        for part, ref in (("w", o3.w[k]), ("m", o3.m[k]), ("v", o3.v[k])):
            got = st[f"{name}_{part}"]
            if not np.array_equal(bits(got), bits(ref)):
                bad = np.nonzero(bits(got) != bits(ref))
                raise AssertionError(f"{tag}: {name}_{part} differs at {bad[0][:5]},{bad[1][:5]}")
        for part, ref in (("ms", o3.ms[k]), ("vs", o3.vs[k])):
            if f"{name}_{part}" in st:
                assert np.array_equal(bits(st[f"{name}_{part}"]), bits(ref)), f"{tag}: {name}_{part}"


@pytest.mark.parametrize("max_defer,layout,grad_mode,cull_mode,states,geo_mode,sched", [
    (0, "separate", "compact", 0, ("f32", "f32"), 0, False),
    (15, "separate", "compact", 1, ("f32", "f32"), 0, False),
    (0, "interleaved", "dense", 1, ("f32", "f32"), 0, False),
    (15, "interleaved", "dense", 0, ("f32", "f32"), 0, False),
    (0, "interleaved", "compact", 1, ("f32", "f32"), 0, False),
    (0, "interleaved", "compact", 1, ("bf16", "bf16"), 0, False),
    (15, "separate", "dense", 1, ("f32", "bf16"), 0, False),
    (0, "separate", "compact", 0, ("bf16", "f32"), 0, False),
    (0, "interleaved", "compact", 1, ("f32", "f32"), 1, False),
    (15, "separate", "dense", 0, ("bf16", "bf16"), 1, False),
    (0, "interleaved", "compact", 1, ("fp8", "fp8"), 0, False),
    (15, "separate", "compact", 1, ("f32", "fp8"), 0, False),
    (0, "separate", "dense", 0, ("bf16", "fp8"), 0, False),
    (0, "fused", "compact", 1, ("f32", "f32"), 0, False),
    (15, "fused", "compact", 1, ("bf16", "fp8"), 0, False),
    (15, "fused", "compact", 1, ("bf16", "bf16"), 0, False),
    (0, "fused", "compact", 0, ("f32", "f32"), 0, True),
    (15, "fused", "dense", 1, ("f32", "f32"), 0, False),
    (15, "interleaved", "compact", 1, ("f32", "f32"), 0, True),
    (0, "separate", "dense", 0, ("f32", "f32"), 1, True),
    # FP8 moments with MAX = inf and compact gradients in the fused and separate layouts
    (0, "fused", "compact", 1, ("fp8", "fp8"), 0, False),
    (0, "separate", "compact", 0, ("f32", "fp8"), 0, False),
    (0, "fused", "compact", 1, ("bf16", "fp8"), 0, True),
])
def test_small_workload_path_vs_oracle(g, max_defer, layout, grad_mode, cull_mode, states, geo_mode, sched):
    """100k Gaussians, 10 orbit cameras, 20 steps: every step's visible ids and
    gathered rows bit-exact vs O3; state bit-exact after steps and after the
    flush; flushed parameters within 1e-6 of dense FP64 Adam.  `sched` runs a
    per-step learning-rate multiplier (decay with noise)."""
    w = gi.workload("small")
    sc = gi.make_scene(w.n, seed=0, box=w.scene_box)
    lg, la = gi.lr_columns()
    lr_scale = None
    if sched:
        rng = np.random.default_rng(9)
        lr_scale = 0.01 ** (np.arange(34) / 33.0) * rng.uniform(0.5, 2.0, 34)
    model = g.Model(sc.geo, sc.app, lg, la, max_steps=32, max_defer=max_defer, app_layout=layout,
                    cull_mode=cull_mode, geo_state=states[0], app_state=states[1], sr_seed=77,
                    geo_mode=geo_mode, lr_scale=lr_scale)
    quant = states != ("f32", "f32")
    o3 = orc.DeferredF32(sc.geo, sc.app, lg, la, max_defer=max_defer, state=states[0], app_state=states[1],
                         sr_seed=77, geo_dense=bool(geo_mode), sched=lr_scale, track_bound=quant)
    dense = orc.DenseAdamF64(sc.geo, sc.app, lg, la, sched=lr_scale)
    n = w.n
    out_g = torch.zeros((n, 10), dtype=torch.float32, device="cuda")
    out_a = torch.zeros((n, 49), dtype=torch.float32, device="cuda")
    gd_g = torch.zeros((n, 10), dtype=torch.float32, device="cuda")
    gd_a = torch.zeros((n, 49), dtype=torch.float32, device="cuda")
    state0 = None
    for t in range(1, w.steps + 1):
        cam = w.camera_for_step(t)
        ids, count, m = run_cull(g, model, cam, t)
        valid = o3.cull_current(t, cam)
        assert m == valid.shape[0], f"step {t}"
        assert np.array_equal(u32(ids[:m]), valid), f"step {t}"
        if t == 3:
            state0 = model.state()
        g.gs_gather(model, t, ids, count, out_g, out_a)
        torch.cuda.synchronize()
        cg, ca = o3.current(t, valid)
        assert np.array_equal(bits(out_g[:m].cpu().numpy()), bits(cg)), f"gather geo step {t}"
        assert np.array_equal(bits(out_a[:m].cpu().numpy()), bits(ca)), f"gather app step {t}"
        if t == 3:
            st = model.state()       # gather is read-only on the stored state
            for key in st:
                assert st[key].tobytes() == state0[key].tobytes(), key
        gg, ga = gi.step_grads(0, t, valid)
        dgg, dga = torch.from_numpy(gg).cuda(), torch.from_numpy(ga).cuda()
        if grad_mode == "compact":
            g.gs_adam_step_deferred(model, t, ids, count, dgg, dga)
        else:
            g.gs_scatter_grad(ids, count, dgg, gd_g)
            g.gs_scatter_grad(ids, count, dga, gd_a)
            g.gs_adam_step_deferred(model, t, ids, count, g_geo_dense=gd_g, g_app_dense=gd_a)
        o3.step(t, valid, gg, ga)
        dense.step(t, valid, gg, ga)
        if t % 5 == 0:
            _compare_state(model, o3, f"step {t}")
            assert np.array_equal(model.last_step.cpu().numpy(), o3.last_step(t))
        say(f"[path K={max_defer} {layout} {grad_mode} cull={cull_mode}] step {t}: M={m} "
            f"restored={model.ws_header()['restored_last']}")
    if grad_mode == "dense":
        assert not gd_g.any() and not gd_a.any()
    g.gs_adam_flush(model, w.steps)
    o3.flush(w.steps)
    _compare_state(model, o3, "after flush")
    assert np.all(model.last_step.cpu().numpy() == w.steps)
    st = model.state()
    e_geo = np.abs(st["geo_w"] - dense.w[0]) / np.maximum(np.abs(dense.w[0]), TAU_GEO)
    e_app = np.abs(st["app_w"] - dense.w[1]) / np.maximum(np.abs(dense.w[1]), TAU_APP)
    say(f"[path {states}] vs dense FP64: geo max {e_geo.max():.3e} mean {e_geo.mean():.3e}; "
        f"app max {e_app.max():.3e} mean {e_app.mean():.3e}")
    if not quant:
        assert e_geo.max() <= 1e-6 and e_app.max() <= 1e-6
    else:
        # quantised moments: every element within the a-posteriori bound the
        # oracle carried along its (bit-identical) trajectory
        res = check_bound((st["geo_w"], st["app_w"]), o3, dense, w.steps, (lg, la), f"path {states}")
        for k, (e, b) in enumerate(res):
            say(f"[path {states}] group {k}: |w - w64| / (lr T) max {e:.3e}, bound max {b:.3e}")
    assert model.ws_header()["error"] == 0


@pytest.mark.parametrize("opt,max_defer,layout,states,sched", [
    ("sgd_momentum", 0, "interleaved", ("f32", "f32"), False),
    ("sgd_momentum", 15, "separate", ("f32", "f32"), True),
    ("sgd_momentum", 0, "fused", ("bf16", "bf16"), True),
    ("adamw", 0, "interleaved", ("f32", "f32"), True),
    ("adamw", 15, "separate", ("bf16", "f32"), False),
])
def test_small_workload_optimizer_variants_vs_oracle(g, opt, max_defer, layout, states, sched):
    """Deferred SGD with momentum and deferred AdamW (the optimizer extensions
    of Sec. 4.3): ids, gathered rows and stored state bit-exact vs the FP32
    oracle model every step and after the flush; FP32 state within 1e-6 of the
    dense FP64 definition."""
    w = gi.workload("small")
    sc = gi.make_scene(w.n, seed=0, box=w.scene_box)
    lg, la = gi.lr_columns()
    lr_scale = None
    if sched:
        rng = np.random.default_rng(4)
        lr_scale = 0.01 ** (np.arange(34) / 33.0) * rng.uniform(0.5, 2.0, 34)
    mu, lam = 0.9, 0.05
    model = g.Model(sc.geo, sc.app, lg, la, beta1=mu, max_steps=32, max_defer=max_defer, app_layout=layout,
                    cull_mode=1, geo_state=states[0], app_state=states[1], sr_seed=5, lr_scale=lr_scale,
                    optimizer=opt, weight_decay=lam)
    if opt == "sgd_momentum":
        o3 = orc.DeferredSGDMF32(sc.geo, sc.app, lg, la, mu=mu, max_defer=max_defer, state=states[0],
                                 app_state=states[1], sr_seed=5, sched=lr_scale)
        dense = orc.DenseSGDMF64(sc.geo, sc.app, lg, la, mu=mu, sched=lr_scale)
    else:
        o3 = orc.DeferredAdamWF32(sc.geo, sc.app, lg, la, weight_decay=lam, max_defer=max_defer, state=states[0],
                                  app_state=states[1], sr_seed=5, sched=lr_scale)
        dense = orc.DenseAdamWF64(sc.geo, sc.app, lg, la, weight_decay=lam, sched=lr_scale)
    n = w.n
    out_g = torch.zeros((n, 10), dtype=torch.float32, device="cuda")
    out_a = torch.zeros((n, 49), dtype=torch.float32, device="cuda")

    def compare(tag):
        st = model.state()
        for k, name in ((0, "geo"), (1, "app")):
            parts = [("w", o3.w[k]), ("m", o3.m[k])] + ([("v", o3.v[k])] if opt == "adamw" else [])
            for part, ref in parts:
                assert np.array_equal(bits(st[f"{name}_{part}"]), bits(ref)), f"{tag}: {name}_{part}"

    for t in range(1, w.steps + 1):
        cam = w.camera_for_step(t)
        ids, count, m = run_cull(g, model, cam, t)
        valid = o3.cull_current(t, cam)
        assert m == valid.shape[0] and np.array_equal(u32(ids[:m]), valid), f"step {t}"
        g.gs_gather(model, t, ids, count, out_g, out_a)
        torch.cuda.synchronize()
        cg, ca = o3.current(t, valid)
        assert np.array_equal(bits(out_g[:m].cpu().numpy()), bits(cg)), f"gather geo step {t}"
        assert np.array_equal(bits(out_a[:m].cpu().numpy()), bits(ca)), f"gather app step {t}"
        gg, ga = gi.step_grads(0, t, valid)
        g.gs_adam_step_deferred(model, t, ids, count, torch.from_numpy(gg).cuda(), torch.from_numpy(ga).cuda())
        o3.step(t, valid, gg, ga)
        dense.step(t, valid, gg, ga)
        if t % 5 == 0:
            compare(f"step {t}")
            assert np.array_equal(model.last_step.cpu().numpy(), o3.last_step(t))
        say(f"[{opt} K={max_defer} {layout} {states}] step {t}: M={m}")
    g.gs_adam_flush(model, w.steps)
    o3.flush(w.steps)
    compare("after flush")
    if states == ("f32", "f32"):
        st = model.state()
        e_geo = np.abs(st["geo_w"] - dense.w[0]) / np.maximum(np.abs(dense.w[0]), TAU_GEO)
        e_app = np.abs(st["app_w"] - dense.w[1]) / np.maximum(np.abs(dense.w[1]), TAU_APP)
        say(f"[{opt}] vs dense FP64: geo max {e_geo.max():.3e}; app max {e_app.max():.3e}")
        assert e_geo.max() <= 1e-6 and e_app.max() <= 1e-6


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_band_cull_adversarial_deferred_rows(g, seed):
    """Stale geometry near the image border and the near plane, deferred up
    to t-1 steps, with moments at the Adam ratio bound |m|/sqrt(v) ~ 7.27 and
    large learning rates so the restore moves rows across the border: the band
    cull must give exactly the exact cull of the restored geometry."""
    rng = np.random.default_rng(100 + seed)
    cam = gi.orbit_cameras(1, seed=seed)[0]
    n, t = 200_000, 50
    geo = _boundary_scene(cam, n, rng)
    geo[:, 3:6] = rng.normal(-3, 1.0, (n, 3))
    good = rng.random(n) < 0.97                       # keep a few NaN/Inf rows
    bad_rows = ~np.all(np.isfinite(geo), axis=1)
    geo[bad_rows & good] = np.nan_to_num(geo[bad_rows & good], nan=1.0, posinf=5.0, neginf=-5.0)
    # quaternions of squared norm just below and above 1/4 (the summary's limit)
    qs = rng.choice(n, n // 100, replace=False)
    geo[qs, 6:10] *= rng.choice([0.3, 0.4999, 0.5, 0.5001, 0.7], qs.shape[0])[:, None].astype(np.float32)
    v = (10.0 ** rng.uniform(-12, -4, (n, 10))).astype(np.float32)
    ratio = rng.choice([7.26, 7.0, 3.0, 0.5], (n, 10)) * rng.choice([-1.0, 1.0], (n, 10))
    m = (ratio * np.sqrt(v.astype(np.float64))).astype(np.float32)
    m[rng.random((n, 10)) < 0.01] = 0.0
    d = rng.integers(0, t, n)
    lr_geo = np.array([0.02, 0.02, 0.02, 0.05, 0.05, 0.05, 0.05, 0.05, 0.05, 0.05], np.float32)
    la = np.full(49, 5e-3, np.float32)
    o3 = orc.DeferredF32(geo, np.zeros((n, 49), np.float32), lr_geo, la)
    o3.m[0][:] = m
    o3.v[0][:] = v
    o3.counter[:] = d
    valid = o3.cull_current(t, cam)
    got = {}
    # exact cull, band cull from the geometry rows, band cull from the summaries
    for mode, summ in ((0, False), (1, False), (1, True)):
        model = g.Model(geo, np.zeros((n, 49), np.float32), lr_geo, la, max_steps=64, cull_mode=mode,
                        cull_summary=summ)
        model.geo_m.copy_(torch.from_numpy(m))
        model.geo_v.copy_(torch.from_numpy(v))
        model.last_step.copy_(torch.from_numpy((t - 1 - d).astype(np.int32)))
        model.lut_seek(t)
        ids, count, mm = run_cull(g, model, cam, t)
        key = (mode, summ)
        got[key] = (u32(ids[:mm]), model.ws_header()["restored_last"])
        assert mm == valid.shape[0], (key, mm, valid.shape[0])
        assert np.array_equal(got[key][0], valid), key
        assert model.ws_header()["error"] == 0
    say(f"[band adversarial {seed}] M={valid.shape[0]} restored exact={got[(0, False)][1]} "
        f"band={got[(1, False)][1]} band from summaries={got[(1, True)][1]}")
    assert got[(1, False)][1] < got[(0, False)][1] and got[(1, True)][1] < got[(0, False)][1]


def test_row_probe_leaves_rows_unchanged(g):
    """The row probe loads (and stores back) listed rows without changing a
    byte; ids past the row count are skipped."""
    rows = torch.randint(0, 255, (5000, 704), dtype=torch.uint8, device="cuda")
    before = rows.clone()
    ids = torch.tensor(sorted(set(np.random.default_rng(1).integers(0, 6000, 900).tolist())), dtype=torch.int32,
                       device="cuda")
    sink = torch.full((1,), 7.0, dtype=torch.float32, device="cuda")
    for wr in (False, True):
        g.gs_row_probe(ids, ids.numel(), rows, wr, sink)
    torch.cuda.synchronize()
    assert torch.equal(rows, before) and float(sink.item()) == 7.0


def test_stream_read_probe(g):
    """The measurement helper reads and stores nothing; misaligned or ragged
    sizes are rejected."""
    buf = torch.ones(1 << 20, dtype=torch.float32, device="cuda")
    sink = torch.full((1,), 7.0, dtype=torch.float32, device="cuda")
    g.gs_stream_read_probe(buf, sink)
    g.gs_stream_read_probe(buf[: 4 * 1001], sink)
    torch.cuda.synchronize()
    assert float(sink.item()) == 7.0
    with pytest.raises(RuntimeError):
        g.gs_stream_read_probe(buf[:6], sink)
    with pytest.raises(RuntimeError):
        g.gs_stream_read_probe(buf[1:5], sink)
