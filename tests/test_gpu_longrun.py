"""Long-run and full-size parity of the HIP path (run with -m gpu).

Paper Sec. 5.5 claims training identical to plain Adam up to the eps
factor-out; these tests check it over the long runs of the aerial workloads:
  * 4M Gaussians (the 4M aerial configuration), 200 steps with MAX = inf and
    100 steps with MAX = 15: every step's visible ids and, every 50 steps and
    after the flush, the FULL state bit-exact against the oracle's FP32 model
    (O3); on a seeded row sample, the flushed parameters against dense FP64
    Adam within max(1e-6, 3 x the error of a plain dense FP32 Adam) per element
    (relative to max(|w64|, tau)).
  * 18M and 40M Gaussians (and the 40M workload with the visible fraction
    matched to the paper's 8.28%) on a seeded sample of whole 128-row blocks (exact:
    Adam is per row given the visible sets, and an FP8 block scale depends on
    its block's rows only): every step the sample's visible ids and gathered
    rows bit-exact against the oracle's own cull and restore of the sample,
    the sample's state bit-exact after the flush (moments, FP8 block scales,
    last steps), and against dense FP64 Adam: FP32 state by the same
    max(1e-6, 3 x dense FP32) rule, BF16 / FP8 state within the a-posteriori
    bound the oracle carries per element.
  * The batched form at full size (16 scenes, 0.5M-8M Gaussians each, 32
    cameras per scene): one step's union and per-camera lists against the
    oracle's cull of every (scene, camera) pair.
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


def bits(a):
    a = np.ascontiguousarray(a)
    return a.view(np.uint32) if a.dtype == np.float32 else a


def rel(w, ref, tau):
    return np.abs(np.asarray(w, np.float64) - ref) / np.maximum(np.abs(ref), tau)


def fp32_gate(w_got, dense, d32, tag):
    """Gate of a long FP32 run: per element max(1e-6, 3 x dense FP32's worst
    error) against dense FP64 (the error unit is relative to max(|w64|, tau))."""
    for k, tau in ((0, TAU_GEO), (1, TAU_APP)):
        e = rel(w_got[k], dense.w[k], tau)
        e32 = rel(d32.w[k], dense.w[k], tau)
        lim = max(1e-6, 3.0 * float(e32.max()))
        say(f"[{tag}] group {k}: max {e.max():.3e} mean {e.mean():.3e}; dense FP32 max {e32.max():.3e}; "
            f"limit {lim:.3e}")
        assert e.max() <= lim, (tag, k, float(e.max()), lim)


def _sample_hits(sample, vis):
    """Positions in `sample` (ascending) of the visible ids found in it, and
    the positions in `vis` of those ids."""
    pos = np.searchsorted(sample, vis)
    hit = (pos < sample.shape[0]) & (sample[np.minimum(pos, sample.shape[0] - 1)] == vis)
    return pos[hit].astype(np.uint32), np.nonzero(hit)[0]


def _compare_full(model, o3, tag):
    st = model.state()
    for k, name in ((0, "geo"), (1, "app")):
        for part, ref in (("w", o3.w[k]), ("m", o3.m[k]), ("v", o3.v[k])):
            got = st[f"{name}_{part}"]
            if not np.array_equal(bits(got), bits(ref)):
                bad = np.nonzero(bits(got) != bits(ref))
                raise AssertionError(f"{tag}: {name}_{part} differs at rows {bad[0][:5]} cols {bad[1][:5]}")


@pytest.mark.parametrize("max_defer,steps", [(0, 200), (15, 100)])
def test_aerial4m_long_run_vs_oracle(g, max_defer, steps):
    w = gi.workload("aerial4m")
    n = w.n
    say(f"[4m long] K={max_defer} steps={steps}")
    sc = gi.make_scene(n, seed=0, box=w.scene_box)
    lg, la = gi.lr_columns()
    model = g.Model(sc.geo, sc.app, lg, la, max_steps=steps + 4, max_defer=max_defer, cull_mode=1,
                    app_layout="fused")
    o3 = orc.DeferredF32(sc.geo, sc.app, lg, la, max_defer=max_defer)
    rng = np.random.default_rng(3)
    sample = np.sort(rng.choice(n, 1 << 16, replace=False)).astype(np.int64)
    dense = orc.DenseAdamF64(sc.geo[sample], sc.app[sample], lg, la)
    d32 = orc.DenseAdamF32(sc.geo[sample], sc.app[sample], lg, la)
    del sc
    cap = n // 4
    ids = torch.zeros(cap, dtype=torch.int32, device="cuda")
    count = torch.zeros(1, dtype=torch.int32, device="cuda")
    gbuf_g = torch.zeros((cap, 10), dtype=torch.float32, device="cuda")
    gbuf_a = torch.zeros((cap, 49), dtype=torch.float32, device="cuda")
    for t in range(1, steps + 1):
        cam = w.camera_for_step(t)
        g.gs_cull(model, cam, t, ids, count)
        g.gs_synth_grad(0, t, ids, count, gbuf_g, 0)
        g.gs_synth_grad(0, t, ids, count, gbuf_a, 10)
        g.gs_adam_step_deferred(model, t, ids, count, gbuf_g, gbuf_a)
        torch.cuda.synchronize()
        m = int(count.item())
        valid = o3.cull_current(t, cam)
        assert m == valid.shape[0] and np.array_equal(ids[:m].cpu().numpy().view(np.uint32), valid), f"step {t}"
        gg, ga = gi.step_grads(0, t, valid)
        o3.step(t, valid, gg, ga)
        local, rows = _sample_hits(sample, valid.astype(np.int64))
        dense.step(t, local, gg[rows], ga[rows])
        d32.step(t, local, gg[rows], ga[rows])
        if t % 50 == 0:
            _compare_full(model, o3, f"step {t}")
            assert np.array_equal(model.last_step.cpu().numpy(), o3.last_step(t)), f"last step {t}"
            say(f"[4m long] K={max_defer} step {t}: M={m} state bit-exact")
    g.gs_adam_flush(model, steps)
    o3.flush(steps)
    dense_state = (model.geo_w[torch.from_numpy(sample).cuda()].cpu().numpy(),
                   model.app_w[torch.from_numpy(sample).cuda()].cpu().numpy())
    _compare_full(model, o3, "after flush")
    assert np.all(model.last_step.cpu().numpy() == steps)
    fp32_gate(dense_state, dense, d32, f"4m K={max_defer} T={steps}")
    assert model.ws_header()["error"] == 0


@pytest.mark.parametrize("workload,state,steps", [("aerial18m", "f32", 200), ("aerial40m", "f32", 300),
                                                  ("aerial40m", "bf16", 300), ("aerial40m", "fp8", 300),
                                                  ("aerial40m_f8", "f32", 60), ("aerial40m_f8", "bf16", 60)])
def test_aerial_sampled_long_run(g, workload, state, steps):
    w = gi.workload(workload)
    n, dev = w.n, torch.device("cuda")
    say(f"[sampled] {workload} {state} steps={steps}")
    geo0, app0 = gi.device_scene(n, w.scene_box, 7, dev)
    lg, la = gi.lr_columns()
    model = g.Model(geo0, app0, lg, la, max_steps=steps + 4, cull_mode=1, app_layout="fused",
                    geo_state=state, app_state=state, sr_seed=11)
    rng = np.random.default_rng(5)
    blk = np.sort(rng.choice(n // 128, 512, replace=False))
    sample = (blk[:, None] * 128 + np.arange(128)).ravel().astype(np.int64)
    sidx = torch.from_numpy(sample).to(dev)
    gs_, as_ = geo0[sidx].cpu().numpy(), app0[sidx].cpu().numpy()
    del geo0, app0
    quant = state != "f32"
    o3 = orc.DeferredF32(gs_, as_, lg, la, state=state, sr_seed=11, keys=sample, track_bound=quant)
    dense = orc.DenseAdamF64(gs_, as_, lg, la)
    d32 = None if quant else orc.DenseAdamF32(gs_, as_, lg, la)
    cap = n // 2                     # a high oblique camera of the 8% workload sees up to 27%
    ids = torch.zeros(cap, dtype=torch.int32, device=dev)
    count = torch.zeros(1, dtype=torch.int32, device=dev)
    out_g = torch.zeros((cap, 10), dtype=torch.float32, device=dev)
    out_a = torch.zeros((cap, 49), dtype=torch.float32, device=dev)
    touched = np.zeros(sample.shape[0], bool)
    for t in range(1, steps + 1):
        cam = w.camera_for_step(t)
        g.gs_cull(model, cam, t, ids, count)
        g.gs_gather(model, t, ids, count, out_g, out_a)
        m = int(count.item())
        assert m <= cap
        # (a camera at the edge of the box may see nothing: keep the buffers non-empty)
        gg = torch.empty((max(m, 1), 10), dtype=torch.float32, device=dev)
        ga = torch.empty((max(m, 1), 49), dtype=torch.float32, device=dev)
        mt = torch.tensor([m], dtype=torch.int32, device=dev)
        g.gs_synth_grad(31, t, None, mt, gg, 0)
        g.gs_synth_grad(31, t, None, mt, ga, 10)
        g.gs_adam_step_deferred(model, t, ids, count, gg, ga)
        vis = ids[:m].long().cpu().numpy()
        local, rows = _sample_hits(sample, vis)
        # the oracle's own cull of the sample's current geometry
        ref = o3.cull_current(t, cam)
        assert np.array_equal(local, ref), f"step {t}: sampled visible ids differ"
        rows_t = torch.from_numpy(rows).to(dev)
        if local.size:
            cg, ca = o3.current(t, local)
            assert np.array_equal(bits(out_g[rows_t].cpu().numpy()), bits(cg)), f"gather geo step {t}"
            assert np.array_equal(bits(out_a[rows_t].cpu().numpy()), bits(ca)), f"gather app step {t}"
        sg, sa = gg[rows_t].cpu().numpy(), ga[rows_t].cpu().numpy()
        o3.step(t, local, sg, sa)
        dense.step(t, local, sg, sa)
        if d32 is not None:
            d32.step(t, local, sg, sa)
        touched[local] = True
        if t % 50 == 0:
            say(f"[sampled] {workload} {state} step {t}: M={m} ({m / n:.4%}), sample rows touched {touched.sum()}")
    g.gs_adam_flush(model, steps)
    o3.flush(steps)
    torch.cuda.synchronize()
    assert model.ws_header()["error"] == 0
    got_w = (model.geo_w[sidx].cpu().numpy(), model.app_w[sidx].cpu().numpy())
    for k, (wt, mt_, vt_) in enumerate(((model.geo_w, model.geo_m, model.geo_v),
                                        (model.app_w, model.app_m, model.app_v))):
        for part, ten, ref in (("w", wt, o3.w[k]), ("m", mt_, o3.m[k]), ("v", vt_, o3.v[k])):
            x = ten[sidx]
            x = x.view(torch.int16).cpu().numpy().view(np.uint16) if x.dtype == torch.bfloat16 else x.cpu().numpy()
            assert np.array_equal(bits(x), bits(ref)), (state, k, part)
    if state == "fp8":
        bt = torch.from_numpy(blk).to(dev)
        for k, (ms, vs) in enumerate(((model.geo_ms, model.geo_vs), (model.app_ms, model.app_vs))):
            assert np.array_equal(bits(ms[bt].cpu().numpy()), bits(o3.ms[k])), ("m scale", k)
            assert np.array_equal(bits(vs[bt].cpu().numpy()), bits(o3.vs[k])), ("v scale", k)
    assert np.all(model.last_step[sidx].cpu().numpy() == steps)
    say(f"[sampled] {workload} {state}: {touched.sum()} of {sample.shape[0]} sampled rows touched; "
        f"sample state bit-exact")
    if quant:
        res = check_bound(got_w, o3, dense, steps, (lg, la), f"{workload} {state}")
        for k, (e, b) in enumerate(res):
            say(f"[sampled] {workload} {state} group {k}: |w - w64| / (lr T) max {e:.3e}, bound max {b:.3e}")
    else:
        fp32_gate(got_w, dense, d32, f"{workload} f32 T={steps}")


def test_batched16_full_size_lists(g):
    """The batched configuration at full size: 16 scenes of log-uniform size
    (0.5M-8M, 44.8M Gaussians), 32 cameras each, rows in generation order; the
    union and all 32 per-camera lists of one step against the oracle."""
    dev = torch.device("cuda")
    sizes = gi.batched_scene_sizes(16)
    C = 32
    geos, row0, sets = [], [0], [[]]
    for s, n in enumerate(sizes):
        box, half = gi.aerial_box_for(n)
        g_, _ = gi.device_scene(n, box, 1000 + s, dev)
        pad = (-n) % g.MULTI_ALIGN
        gp = torch.full((pad, 10), float("nan"), device=dev)
        gp[:, 6] = 1.0
        geos.append(torch.cat([g_, gp]))
        row0.append(row0[-1] + n + pad)
        sets[0].append(gi.aerial_cameras(C, half, half, seed=s))
    geo = torch.cat(geos)
    del geos
    N = int(geo.shape[0])
    say(f"[batched16 full] {N} rows in {len(sizes)} scenes x {C} cameras")
    lg, la = gi.lr_columns()
    model = g.Model(geo, torch.zeros((N, 1), device=dev), lg, la[:1], max_steps=4, cull_mode=1)
    multi = g.Multi(model, row0, sets, cap_union=N, cap_cam=N // 8)
    g.gs_cull_multi(model, multi, 1)
    torch.cuda.synchronize()
    geo_h = geo.cpu().numpy()
    del geo
    union, cam_pos, start = orc.cull_multi(geo_h, row0, sets[0])
    u, ids, cc, cams, ss = multi.lists()
    assert u == union.shape[0] and np.array_equal(ids, union.astype(np.uint32))
    for c in range(C):
        assert cc[c] == cam_pos[c].shape[0] and np.array_equal(cams[c], cam_pos[c].astype(np.uint32)), c
    assert np.array_equal(ss.astype(np.int64), start)
    say(f"[batched16 full] union {u}, per-camera {min(cc)}..{max(cc)}: lists bit-exact")
