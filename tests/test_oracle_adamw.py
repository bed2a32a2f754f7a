"""Pins of the oracle's AdamW models (decoupled weight decay, the other
optimizer named in Sec. 4.3) against the mathematics they follow:

  * dense FP64 AdamW == torch.optim.AdamW (FP64) driven with the same per-step
    rates: an independent library;
  * the decayed restore tables == their direct sum / product (brute force);
  * deferred FP64 == dense FP64 with eps = 0 (exact up to rounding), at
    MAX = inf and 15, with and without a rate schedule, after the flush;
  * weight decay 0 reduces the FP32 model to the Adam FP32 model bit for bit;
  * the FP32 model stays within FP32 rounding of the dense FP64 definition.
"""
import numpy as np
import pytest
import torch

import gs_inputs as gi
from oracle import oracle as orc

B1, B2, LAM = 0.9, 0.999, 0.05
TAU_GEO = np.array([1, 1, 1, .5, .5, .5, .5, .5, .5, .5])
TAU_APP = np.array([1.0] + [0.1] * 48)


def rel_err(w, ref, tau):
    return np.abs(np.asarray(w, np.float64) - ref) / np.maximum(np.abs(ref), tau)


def _vis(n, steps, p, seed):
    rng = np.random.default_rng(seed)
    return [np.nonzero(rng.random(n) < p)[0] for _ in range(steps)]


def _grads(t, ids, seed):
    rng = np.random.default_rng(seed * 7919 + t)
    return (rng.normal(0, 1e-3, (ids.shape[0], 10)).astype(np.float32),
            rng.normal(0, 1e-3, (ids.shape[0], 49)).astype(np.float32))


def _sched(steps, seed):
    rng = np.random.default_rng(seed)
    return 0.01 ** (np.arange(steps + 2) / (steps + 1)) * rng.uniform(0.5, 2.0, steps + 2)


def test_dense_adamw_matches_torch_adamw():
    n, steps = 200, 25
    s = gi.make_scene(n, seed=1)
    lg, la = gi.lr_columns()
    lg, la = lg * 20, la * 20          # larger rates make the decay term visible
    sc = _sched(steps, 2)
    dense = orc.DenseAdamWF64(s.geo, s.app, lg, la, eps=1e-8, weight_decay=LAM, sched=sc)
    cols = [torch.tensor(s.geo[:, c], dtype=torch.float64, requires_grad=True) for c in range(10)] + \
           [torch.tensor(s.app[:, c], dtype=torch.float64, requires_grad=True) for c in range(49)]
    rates = list(lg.astype(np.float64)) + list(la.astype(np.float64))
    opt = torch.optim.AdamW([{"params": [p], "lr": float(r)} for p, r in zip(cols, rates)], betas=(B1, B2),
                            eps=1e-8, weight_decay=LAM, foreach=False)
    for t, ids in enumerate(_vis(n, steps, 0.3, 3), start=1):
        gg, ga = _grads(t, ids, 4)
        dense.step(t, ids, gg, ga)
        full = np.zeros((n, 59))
        full[ids, :10] = gg
        full[ids, 10:] = ga
        for c, p in enumerate(cols):
            p.grad = torch.tensor(full[:, c], dtype=torch.float64)
        for grp, r in zip(opt.param_groups, rates):
            grp["lr"] = float(r * sc[t])
        opt.step()
    ref = np.stack([p.detach().numpy() for p in cols], 1)
    got = np.concatenate([dense.w[0], dense.w[1]], 1)
    assert np.max(np.abs(got - ref) / np.maximum(np.abs(ref), 1e-3)) < 1e-12


@pytest.mark.parametrize("t", [2, 17, 100])
def test_decayed_tables_equal_direct_sum(t):
    sc = _sched(120, 5)
    lr = 5e-3
    W, P = orc.lut_adamw(B1, B2, LAM, lr, t, t - 1, sc)
    r = B1 / np.sqrt(B2)
    c = lambda k: B1 / (np.sqrt(B2 / (1 - B2 ** k)) * (1 - B1 ** k))
    q = lambda k: 1 - lr * sc[k] * LAM
    # the backward recurrence over the skipped steps, most recent first:
    # Wl[d] = r Wl[d-1] + P[d-1] s c(t-d),  P[d] = P[d-1] q(t-d)
    rw, rp = 0.0, 1.0
    for d in range(t):
        if d > 0:
            rw = r * rw + rp * sc[t - d] * c(t - d)
            rp = rp * q(t - d)
        assert abs(W[d] - rw) <= 1e-13 * max(1.0, abs(rw))
        assert abs(P[d] - rp) <= 1e-15
    Wf, Pf, qt = orc.lut_adamw_spec(B1, B2, LAM, np.float32(lr), t, t - 1, sc)
    assert np.all(np.abs(Wf.astype(np.float64) - W) <= 2 * np.spacing(np.abs(W).astype(np.float32)))
    assert np.all(np.abs(Pf.astype(np.float64) - P) <= 2 * np.spacing(np.abs(P).astype(np.float32)))
    assert abs(float(qt) - q(t)) <= np.spacing(np.float32(1.0))


@pytest.mark.parametrize("max_defer,sched", [(0, False), (15, False), (0, True), (15, True)])
def test_deferred_adamw_f64_equals_dense_with_eps_zero(max_defer, sched):
    n, steps = 400, 60
    s = gi.make_scene(n, seed=6)
    lg, la = gi.lr_columns()
    sc = _sched(steps, 7) if sched else None
    dense = orc.DenseAdamWF64(s.geo, s.app, lg, la, eps=0.0, weight_decay=LAM, sched=sc)
    o2 = orc.DeferredAdamWF64(s.geo, s.app, lg, la, eps=0.0, weight_decay=LAM, max_defer=max_defer, sched=sc)
    plain = orc.DenseAdamF64(s.geo, s.app, lg, la, eps=0.0, sched=sc)
    vis = _vis(n, steps, 0.05, 8)
    vis[0] = np.arange(n)              # with eps = 0 every row needs v > 0 before it steps
    for t, ids in enumerate(vis, start=1):
        g = _grads(t, ids, 9)
        dense.step(t, ids, *g)
        o2.step(t, ids, *g)
        plain.step(t, ids, *g)
    o2.flush(steps)
    for k in range(2):
        assert np.max(rel_err(o2.w[k], dense.w[k], 1e-3)) < 1e-12
    # the decay really acts (a dropped P or q would fail above)
    assert np.max(rel_err(plain.w[1], dense.w[1], 1e-3)) > 1e-6


def test_zero_decay_reduces_to_adam_bitwise():
    n, steps = 1500, 15
    s = gi.make_scene(n, seed=12)
    lg, la = gi.lr_columns()
    aw = orc.DeferredAdamWF32(s.geo, s.app, lg, la, weight_decay=0.0, max_defer=15, state="bf16", sr_seed=4)
    ad = orc.DeferredF32(s.geo, s.app, lg, la, max_defer=15, state="bf16", sr_seed=4)
    for t, ids in enumerate(_vis(n, steps, 0.3, 13), start=1):
        g = gi.step_grads(0, t, ids)
        aw.step(t, ids, *g)
        ad.step(t, ids, *g)
    aw.flush(steps)
    ad.flush(steps)
    for k in range(2):
        assert np.array_equal(aw.w[k].view(np.uint32), ad.w[k].view(np.uint32))
        assert np.array_equal(aw.m[k], ad.m[k]) and np.array_equal(aw.v[k], ad.v[k])


def test_adamw_f32_model_within_fp32_rounding_of_dense():
    n, steps = 2000, 20
    s = gi.make_scene(n, seed=10)
    lg, la = gi.lr_columns()
    sc = _sched(steps, 3)
    o3 = orc.DeferredAdamWF32(s.geo, s.app, lg, la, weight_decay=LAM, max_defer=15, sched=sc)
    dense = orc.DenseAdamWF64(s.geo, s.app, lg, la, weight_decay=LAM, sched=sc)
    for t, ids in enumerate(_vis(n, steps, 0.3, 11), start=1):
        g = gi.step_grads(0, t, ids)
        o3.step(t, ids, *g)
        dense.step(t, ids, *g)
    o3.flush(steps)
    for k, tau in ((0, TAU_GEO), (1, TAU_APP)):
        assert np.max(rel_err(o3.w[k], dense.w[k], tau)) < 1e-6
