"""Chunk records of the cull summaries (run with -m gpu).

- The device build equals the records' definition (include/gsdp.h) evaluated
  on the host from the summaries, on rows with every summary case.
- With rows in a spatial order (Morton code of the position), over training
  runs whose updates move positions far enough to leave their chunk's box:
  every summary stays inside its chunk's record after each update and after
  the flush; no chunk the summary cull skips holds a row the oracle's cull
  of the current geometry keeps; the summary cull with records lists exactly
  what the cull without them lists and what the oracle lists (also with the
  camera read from a device table); and the states stay bit-identical (FP32,
  BF16 and FP8 moments, whose two-pass update widens the records too).
- At 18M rows (the compaction's group sums filled by the summary cull), around
  the 2^16-step boundary, and for empty, single-row and ragged models, the
  cull with records lists what the oracle, or the cull without records, lists.
"""
import sys

import numpy as np
import pytest
import torch

import gs_inputs as gi
from oracle import oracle as orc
from test_gpu_parity import _compare_state
from test_gpu_summary import _rows

pytestmark = pytest.mark.gpu

CH = 1024


def say(*a):
    print(*a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def g():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2509_15645_amd import gsdp
    assert gsdp.GS_CHUNK_ROWS == CH
    return gsdp


def _split(sumw):
    w = np.ascontiguousarray(sumw, np.float32).view(np.uint32).reshape(-1, 4)
    cen = w[:, :3].copy().view(np.float32)
    s = (w[:, 3] & np.uint32(0xFFFE0000)).view(np.float32)
    return cen, s


def host_chunks(sumw):
    """Records (lo x, y, z, s, hi x, y, z, 0) of the summaries, as the header
    defines them: the box of the centres of rows whose s is not a NaN, the
    largest s, a NaN s when any row's is."""
    cen, s = _split(sumw)
    n = cen.shape[0]
    rec = np.zeros(((n + CH - 1) // CH, 8), np.float32)
    for c in range(rec.shape[0]):
        cc, sc = cen[c * CH:(c + 1) * CH], s[c * CH:(c + 1) * CH]
        good = ~np.isnan(sc)
        rec[c, 0:3] = cc[good].min(0) if good.any() else np.inf
        rec[c, 4:7] = cc[good].max(0) if good.any() else -np.inf
        rec[c, 3] = sc.max() if good.all() else np.nan
    return rec


def same_records(a, b):
    a, b = np.asarray(a, np.float32), np.asarray(b, np.float32)
    return (np.array_equal(a[:, [0, 1, 2, 4, 5, 6, 7]], b[:, [0, 1, 2, 4, 5, 6, 7]]) and
            np.array_equal(np.isnan(a[:, 3]), np.isnan(b[:, 3])) and
            np.array_equal(a[~np.isnan(a[:, 3]), 3], b[~np.isnan(b[:, 3]), 3]))


def check_contained(model, what):
    """Every row's summary lies inside its chunk's record."""
    torch.cuda.synchronize()
    n = model.n
    cen, s = _split(model.cull_sum[:n].cpu().numpy())
    rec = model.cull_chunk.cpu().numpy()
    r = rec[np.arange(n) // CH]
    bad_s = np.isnan(s)
    assert np.all(np.isnan(r[bad_s, 3])), what + ": a NaN summary in a chunk without a NaN s"
    ok = ~bad_s
    assert np.all(cen[ok] >= r[ok, 0:3]) and np.all(cen[ok] <= r[ok, 4:7]), what + ": centre outside its box"
    assert np.all((s[ok] <= r[ok, 3]) | np.isnan(r[ok, 3])), what + ": s above its chunk's"


def _morton(pos):
    lo, hi = pos.min(0), pos.max(0)
    q = ((pos - lo) / np.maximum(hi - lo, 1e-30) * 1023).astype(np.int64).clip(0, 1023)
    code = np.zeros(pos.shape[0], np.int64)
    for b in range(10):
        for a in range(3):
            code |= ((q[:, a] >> b) & 1) << (3 * b + a)
    return np.argsort(code, kind="stable")


def _scene(n, seed, half=1000.0):
    """Aerial box 2 half x 2 half x 100 m, rows in Morton order."""
    box = ((-half, half), (-half, half), (0.0, 100.0))
    sc = gi.make_scene(n, seed=seed, box=box)
    perm = _morton(sc.geo[:, :3].astype(np.float64))
    return np.ascontiguousarray(sc.geo[perm]), np.ascontiguousarray(sc.app[perm]), half


def test_chunk_build_matches_definition(g):
    rng = np.random.default_rng(17)
    for n in (1, 1000, 1024, 1025, 100_003):
        geo = _rows(rng, n)
        lg, la = gi.lr_columns()
        model = g.Model(geo, np.zeros((n, 49), np.float32), lg, la, max_steps=8, cull_mode=1, cull_chunks=True)
        assert model.cull_chunk is not None and model.cull_chunk.shape == ((n + CH - 1) // CH, 8)
        torch.cuda.synchronize()
        ref = host_chunks(model.cull_sum[:n].cpu().numpy())
        got = model.cull_chunk.cpu().numpy()
        say(f"[chunk build] n={n}: {int(np.isnan(ref[:, 3]).sum())} of {ref.shape[0]} chunks with a NaN s")
        assert same_records(got, ref)


def test_chunk_records_need_summaries(g):
    n = 5000
    sc = gi.make_scene(n, seed=3)
    lg, la = gi.lr_columns()
    a = g.Model(sc.geo, sc.app, lg, la, max_steps=4, cull_mode=1, cull_summary=False, cull_chunks=True)
    assert a.cull_sum is None and a.cull_chunk is None
    b = g.Model(sc.geo, sc.app, lg, la, max_steps=4, cull_mode=1)
    assert b.cull_sum is not None and b.cull_chunk is None
    c = g.Model(sc.geo, sc.app, lg, la, max_steps=4, cull_mode=1, max_defer=15, cull_chunks=True)
    flags = torch.zeros(8, dtype=torch.uint8, device="cuda")
    with pytest.raises(g.GsError, match="UNSUPPORTED"):
        g.gs_cull_chunk_flags(c, gi.orbit_cameras(1, seed=1)[0], 1, flags)


@pytest.mark.parametrize("state,pos_lr", [("f32", 1.6e-4), ("f32", 2.0), ("bf16", 2.0), ("fp8", 2.0)])
def test_chunk_cull_lockstep_vs_oracle(g, state, pos_lr):
    n, steps = 400_000, 12
    geo, app, half = _scene(n, seed=21)
    lg, la = gi.lr_columns()
    lg = lg.copy()
    lg[0:3] = pos_lr                     # 2 m a step: rows leave their chunk's box
    kw = dict(max_steps=steps + 2, cull_mode=1, app_layout="fused", geo_state=state, app_state=state, sr_seed=5)
    a = g.Model(geo, app, lg, la, cull_chunks=True, **kw)
    b = g.Model(geo, app, lg, la, **kw)
    assert a.cull_chunk is not None and b.cull_chunk is None and b.cull_sum is not None
    o = orc.DeferredF32(geo, app, lg, la, state=state, sr_seed=5)
    cams = gi.aerial_cameras(steps, half, half, seed=8)
    table = g.camera_table(a, cams)
    ids = [torch.zeros(n, dtype=torch.int32, device="cuda") for _ in range(3)]
    cnt = [torch.zeros(1, dtype=torch.int32, device="cuda") for _ in range(3)]
    flags = torch.zeros(a.cull_chunk.shape[0], dtype=torch.uint8, device="cuda")
    out_g = torch.zeros((n, 10), dtype=torch.float32, device="cuda")
    out_a = torch.zeros((n, 49), dtype=torch.float32, device="cuda")
    check_contained(a, "built")
    skipped = []
    for t in range(1, steps + 1):
        cam = cams[t - 1]
        g.gs_cull(a, cam, t, ids[0], cnt[0])
        g.gs_cull(b, cam, t, ids[1], cnt[1])
        g.gs_cull_table(a, table, t, ids[2], cnt[2])
        g.gs_cull_chunk_flags(a, cam, t, flags)
        torch.cuda.synchronize()
        m = int(cnt[0].item())
        valid = o.cull_current(t, cam)
        assert m == valid.shape[0], f"step {t}: {m} visible, the oracle {valid.shape[0]}"
        got = ids[0][:m].cpu().numpy().view(np.uint32)
        assert np.array_equal(got, valid), f"step {t}: ids differ from the oracle's"
        for k in (1, 2):
            assert int(cnt[k].item()) == m and torch.equal(ids[k][:m], ids[0][:m]), f"step {t}: path {k}"
        f = flags.cpu().numpy().astype(bool)
        assert not f[valid // CH].any(), f"step {t}: a skipped chunk holds a visible row"
        skipped.append(f.mean())
        g.gs_gather(a, t, ids[0], cnt[0], out_g, out_a)
        gg, ga = gi.step_grads(0, t, valid)
        dg, da = torch.from_numpy(gg).cuda(), torch.from_numpy(ga).cuda()
        for model in (a, b):
            g.gs_adam_step_deferred(model, t, ids[0], cnt[0], dg, da)
        o.step(t, valid, gg, ga)
        check_contained(a, f"after update {t}")
    say(f"[chunks {state} lr {pos_lr}] skipped {np.mean(skipped):.3f} of the chunks on average "
        f"(min {np.min(skipped):.3f}), visible {m} at the last step")
    assert np.mean(skipped) > 0.5
    for model in (a, b):
        g.gs_adam_flush(model, steps)
    o.flush(steps)
    check_contained(a, "after the flush")
    sa, sb = a.state(), b.state()
    for k in sa:
        assert np.array_equal(np.asarray(sa[k]).view(np.uint8), np.asarray(sb[k]).view(np.uint8)), k
    _compare_state(a, o, "after the flush")
    # a rebuild gives tight records again, which hold every summary
    widened = a.cull_chunk.clone()
    a.cull_summary_build()
    torch.cuda.synchronize()
    tight = a.cull_chunk.cpu().numpy()
    assert same_records(tight, host_chunks(a.cull_sum[:n].cpu().numpy()))
    w = widened.cpu().numpy()
    assert np.all(w[:, 0:3] <= tight[:, 0:3]) and np.all(w[:, 4:7] >= tight[:, 4:7])


def test_chunk_records_after_densify(g):
    """Densification writes the new model's rows and rebuilds its summaries
    and chunk records, tight."""
    n, steps = 60_000, 4
    geo, app, half = _scene(n, seed=5)
    lg, la = gi.lr_columns()
    model = g.Model(geo, app, lg, la, max_steps=steps + 8, cull_mode=1, app_layout="fused", cull_chunks=True)
    cams = gi.aerial_cameras(steps, half, half, seed=3)
    ids = torch.zeros(n, dtype=torch.int32, device="cuda")
    cnt = torch.zeros(1, dtype=torch.int32, device="cuda")
    gg = torch.empty((n, 10), dtype=torch.float32, device="cuda")
    ga = torch.empty((n, 49), dtype=torch.float32, device="cuda")
    accum = torch.zeros(n, dtype=torch.float32, device="cuda")
    for t in range(1, steps + 1):
        g.gs_cull(model, cams[t - 1], t, ids, cnt)
        g.gs_synth_grad(3, t, ids, cnt, gg, 0)
        g.gs_synth_grad(3, t, ids, cnt, ga, 10)
        g.gs_adam_step_deferred(model, t, ids, cnt, gg, ga)
    g.gs_adam_flush(model, steps)
    rng = np.random.default_rng(2)
    accum.copy_(torch.from_numpy(rng.exponential(3e-4, n).astype(np.float32)))
    denom = torch.ones(n, dtype=torch.float32, device="cuda")
    new, counts = g.densify(model, steps, accum, denom, scene_extent=2 * half)
    torch.cuda.synchronize()
    say(f"[chunks densify] {n} rows -> {new.n} (originals, clones, children {counts})")
    assert new.n != n and new.cull_chunk is not None
    assert new.cull_chunk.shape[0] == (new.n + CH - 1) // CH
    assert same_records(new.cull_chunk.cpu().numpy(), host_chunks(new.cull_sum[:new.n].cpu().numpy()))
    check_contained(new, "after densify")


def test_chunk_cull_grouped_aerial18m(g):
    """18M Gaussians (more than 16384 tiles: the compaction takes the group
    sums, which the chunk scan clears and the summary cull adds to, with no
    separate reduction), rows in Morton order.  Step 1 bit-exact against the
    oracle's cull; then, over updates that move positions 2 m a step, the cull
    with chunk records equals the cull without them and the cull from a device
    camera table, and no skipped chunk holds a kept row."""
    w = gi.workload("aerial18m")
    sc = gi.make_scene(w.n, seed=1, box=w.scene_box)
    del sc.app
    perm = _morton(sc.geo[:, :3].astype(np.float64))
    geo = np.ascontiguousarray(sc.geo[perm])
    del sc, perm
    n, steps = w.n, 3
    say(f"[chunks grouped] n={n}")
    lg, la = gi.lr_columns()
    lg = lg.copy()
    lg[0:3] = 2.0
    app = np.zeros((n, 1), np.float32)
    kw = dict(max_steps=steps + 2, cull_mode=1, app_layout="fused")
    a = g.Model(geo, app, lg, la, cull_chunks=True, **kw)
    b = g.Model(geo, app, lg, la, **kw)
    cams = [w.camera_for_step(t) for t in range(1, steps + 1)]
    table = g.camera_table(a, cams)
    ids = [torch.zeros(n, dtype=torch.int32, device="cuda") for _ in range(3)]
    cnt = [torch.zeros(1, dtype=torch.int32, device="cuda") for _ in range(3)]
    flags = torch.zeros(a.cull_chunk.shape[0], dtype=torch.uint8, device="cuda")
    gg = torch.empty((n, 10), dtype=torch.float32, device="cuda")
    ga = torch.empty((n, 1), dtype=torch.float32, device="cuda")
    for t in range(1, steps + 1):
        g.gs_cull(a, cams[t - 1], t, ids[0], cnt[0])
        g.gs_cull(b, cams[t - 1], t, ids[1], cnt[1])
        g.gs_cull_table(a, table, t, ids[2], cnt[2])
        g.gs_cull_chunk_flags(a, cams[t - 1], t, flags)
        torch.cuda.synchronize()
        m = int(cnt[0].item())
        for k in (1, 2):
            assert int(cnt[k].item()) == m and torch.equal(ids[k][:m], ids[0][:m]), f"step {t}: path {k}"
        kept = ids[0][:m].cpu().numpy().view(np.uint32)
        f = flags.cpu().numpy().astype(bool)
        assert not f[kept // CH].any(), f"step {t}: a skipped chunk holds a kept row"
        if t == 1:
            ref = orc.compact(orc.cull(geo, cams[0]))
            assert m == ref.shape[0] and np.array_equal(kept, ref), "step 1: ids differ from the oracle's"
        say(f"[chunks grouped] step {t}: M={m}, {f.mean():.3f} of the chunks skipped")
        assert f.mean() > 0.5
        g.gs_synth_grad(6, t, ids[0], cnt[0], gg, 0)
        g.gs_synth_grad(6, t, ids[0], cnt[0], ga, 10)
        for model in (a, b):
            g.gs_adam_step_deferred(model, t, ids[0], cnt[0], gg, ga)
    assert a.ws_header()["error"] == 0 and b.ws_header()["error"] == 0
    check_contained(a, "after the updates")


@pytest.mark.parametrize("T,t0", [(70_000, 65_530), (65_536, 65_524)])
def test_chunk_cull_across_the_16_bit_step_boundary(g, T, t0):
    """Past 2^16 steps the summary cull also reads the last-step array, with
    chunk records too; around the boundary the cull with records lists what
    the cull from the geometry rows lists, and the states stay equal."""
    n = 60_000
    geo, app, half = _scene(n, seed=31, half=300.0)
    lg, la = gi.lr_columns()
    lg = lg.copy()
    lg[0:3] = 0.5
    cams = gi.aerial_cameras(16, half, half, seed=31)
    kw = dict(max_steps=T, cull_mode=1, app_layout="fused", sr_seed=2)
    a = g.Model(geo, app, lg, la, cull_chunks=True, **kw)
    b = g.Model(geo, app, lg, la, cull_summary=False, **kw)
    for m in (a, b):
        m.lut_seek(t0)
    ids = [torch.zeros(n, dtype=torch.int32, device="cuda") for _ in range(2)]
    cnt = [torch.zeros(1, dtype=torch.int32, device="cuda") for _ in range(2)]
    flags = torch.zeros(a.cull_chunk.shape[0], dtype=torch.uint8, device="cuda")
    gg = torch.empty((n, 10), dtype=torch.float32, device="cuda")
    ga = torch.empty((n, 49), dtype=torch.float32, device="cuda")
    skipped = 0.0
    for t in range(t0, min(T, t0 + 12) + 1):
        cam = cams[t % 16]
        for k, m in enumerate((a, b)):
            g.gs_cull(m, cam, t, ids[k], cnt[k])
        g.gs_cull_chunk_flags(a, cam, t, flags)
        torch.cuda.synchronize()
        mm = int(cnt[0].item())
        assert mm == int(cnt[1].item()) and torch.equal(ids[0][:mm], ids[1][:mm]), t
        f = flags.cpu().numpy().astype(bool)
        assert not f[ids[0][:mm].cpu().numpy() // CH].any(), t
        skipped = max(skipped, f.mean())
        g.gs_synth_grad(4, t, ids[0], cnt[0], gg, 0)
        g.gs_synth_grad(4, t, ids[0], cnt[0], ga, 10)
        for m in (a, b):
            g.gs_adam_step_deferred(m, t, ids[0], cnt[0], gg, ga)
    assert skipped > 0.3
    check_contained(a, "after the updates")
    sa, sb = a.state(), b.state()
    for key in sa:
        assert sa[key].tobytes() == sb[key].tobytes(), key
    assert a.ws_header()["error"] == 0 and b.ws_header()["error"] == 0
    say(f"[chunks 16-bit boundary] T={T}: steps {t0}..{min(T, t0 + 12)} equal, up to {skipped:.2f} skipped")


@pytest.mark.parametrize("n", [0, 1, 5, 1023, 1024, 1025, 3007])
def test_chunk_cull_small_and_ragged(g, n):
    """Empty, single-row and ragged models (a last chunk of 1..1023 rows): the
    cull with chunk records lists what the oracle's cull of the current
    geometry lists, over updates that move positions 2 m a step."""
    say(f"[chunks small] n={n}")
    geo, app, half = _scene(max(n, 1), seed=40 + n, half=100.0)
    geo, app = geo[:n], app[:n]
    lg, la = gi.lr_columns()
    lg = lg.copy()
    lg[0:3] = 2.0
    kw = dict(max_steps=6, cull_mode=1, app_layout="fused", sr_seed=3)
    a = g.Model(geo, app, lg, la, cull_chunks=True, **kw)
    # (an empty model keeps one unused record: the binding allocates nothing empty)
    assert a.cull_chunk is not None and a.cull_chunk.shape[0] == max((n + CH - 1) // CH, 1)
    o = orc.DeferredF32(geo, app, lg, la, sr_seed=3)
    # two cameras over the middle (every tiny model has visible rows), two anywhere
    near, far = gi.aerial_cameras(2, 5.0, 5.0, seed=n), gi.aerial_cameras(2, half, half, seed=n)
    cams = [near[0], far[0], near[1], far[1]]
    ids = torch.full((max(n, 1),), -1, dtype=torch.int32, device="cuda")
    cnt = torch.zeros(1, dtype=torch.int32, device="cuda")
    for t in range(1, 5):
        g.gs_cull(a, cams[t - 1], t, ids, cnt)
        torch.cuda.synchronize()
        m = int(cnt.item())
        valid = o.cull_current(t, cams[t - 1])
        assert m == valid.shape[0] and np.array_equal(ids[:m].cpu().numpy().view(np.uint32), valid), t
        gg, ga = gi.step_grads(0, t, valid)
        # compact gradients of at least one row (an empty tensor has no address)
        dg = torch.zeros((max(m, 1), 10), dtype=torch.float32, device="cuda")
        da = torch.zeros((max(m, 1), 49), dtype=torch.float32, device="cuda")
        dg[:m], da[:m] = torch.from_numpy(gg), torch.from_numpy(ga)
        g.gs_adam_step_deferred(a, t, ids, cnt, dg, da, capacity=dg.shape[0])
        o.step(t, valid, gg, ga)
        if n:
            check_contained(a, f"after update {t}")
    assert a.ws_header()["error"] == 0
