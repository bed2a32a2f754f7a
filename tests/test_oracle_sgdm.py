"""Pins of the oracle's SGD-with-momentum models (the momentum-optimizer
extension of Sec. 4.3) against the mathematics they follow:

  * dense FP64 SGD-momentum == torch.optim.SGD (FP64, momentum, no dampening,
    no Nesterov) driven with the same per-step rates: an independent library;
  * the table recurrence == the direct sum over skipped steps (brute force);
  * deferred FP64 == dense FP64 exactly up to rounding, at MAX = inf and 15,
    with and without a rate schedule, after steps and after the flush (with
    momentum there is no eps to factor out, so deferral is exact);
  * the FP32 model stays within FP32 rounding of the dense FP64 definition;
  * BF16 buffers stay within the stated bound.
"""
import numpy as np
import pytest
import torch

import gs_inputs as gi
from oracle import oracle as orc

MU = 0.9
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


def test_dense_sgdm_matches_torch_sgd():
    n, steps = 300, 25
    s = gi.make_scene(n, seed=1)
    lg, la = gi.lr_columns()
    sc = _sched(steps, 2)
    dense = orc.DenseSGDMF64(s.geo, s.app, lg, la, mu=MU, sched=sc)
    # one torch parameter per column so every column has its own rate
    cols = [torch.tensor(s.geo[:, c], dtype=torch.float64, requires_grad=True) for c in range(10)] + \
           [torch.tensor(s.app[:, c], dtype=torch.float64, requires_grad=True) for c in range(49)]
    rates = list(lg.astype(np.float64)) + list(la.astype(np.float64))
    opt = torch.optim.SGD([{"params": [p], "lr": float(r)} for p, r in zip(cols, rates)], momentum=MU,
                          dampening=0.0, nesterov=False, foreach=False)
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
    assert np.max(np.abs(got - ref) / np.maximum(np.abs(ref), 1e-3)) < 1e-13


@pytest.mark.parametrize("t", [2, 17, 100])
def test_table_direct_sum_equals_recurrence(t):
    """The oracle's sum over the skipped steps against the backward
    recurrence Ws[d] = mu (Ws[d-1] + s_{t-d}) (zero-gradient momentum steps
    taken one at a time, most recent first)."""
    sc = _sched(120, 5)
    W, M = orc.lut_sgdm(MU, t, t - 1, sc)
    rec = 0.0
    for d in range(t):
        if d > 0:
            rec = MU * (rec + sc[t - d])
        assert abs(W[d] - rec) <= 1e-14 * max(1.0, abs(rec))
        assert abs(M[d] - MU ** (d + 1)) <= 1e-15
    Wf, Mf, ss = orc.lut_sgdm_spec(MU, t, t - 1, sc)
    assert np.all(np.abs(Wf.astype(np.float64) - W) <= np.spacing(np.abs(W).astype(np.float32)))
    assert ss == np.float32(sc[t])


@pytest.mark.parametrize("max_defer,sched", [(0, False), (15, False), (0, True), (15, True)])
def test_deferred_sgdm_f64_equals_dense(max_defer, sched):
    n, steps = 400, 60
    s = gi.make_scene(n, seed=6)
    lg, la = gi.lr_columns()
    sc = _sched(steps, 7) if sched else None
    dense = orc.DenseSGDMF64(s.geo, s.app, lg, la, mu=MU, sched=sc)
    o2 = orc.DeferredSGDMF64(s.geo, s.app, lg, la, mu=MU, max_defer=max_defer, sched=sc)
    for t, ids in enumerate(_vis(n, steps, 0.05, 8), start=1):
        g = _grads(t, ids, 9)
        dense.step(t, ids, *g)
        o2.step(t, ids, *g)
    if max_defer:
        assert o2.counter.max() <= max_defer
    o2.flush(steps)
    for k in range(2):
        assert np.max(rel_err(o2.w[k], dense.w[k], 1e-3)) < 1e-12
        assert np.max(np.abs(o2.m[k] - dense.m[k])) < 1e-12 * np.max(np.abs(dense.m[k]))


@pytest.mark.parametrize("state,bound", [("f32", 1e-6), ("bf16", None)])
def test_sgdm_f32_model_tracks_dense(state, bound):
    n, steps = 2000, 20
    s = gi.make_scene(n, seed=10)
    lg, la = gi.lr_columns()
    o3 = orc.DeferredSGDMF32(s.geo, s.app, lg, la, mu=MU, max_defer=15, state=state, sr_seed=3)
    dense = orc.DenseSGDMF64(s.geo, s.app, lg, la, mu=MU)
    for t, ids in enumerate(_vis(n, steps, 0.3, 11), start=1):
        g = gi.step_grads(0, t, ids)
        o3.step(t, ids, *g)
        dense.step(t, ids, *g)
    o3.flush(steps)
    for k, (tau, lr) in enumerate(((TAU_GEO, lg), (TAU_APP, la))):
        if bound is not None:
            assert np.max(rel_err(o3.w[k], dense.w[k], tau)) < bound
        else:
            # One BF16 rounding of the buffer errs below 2^-7 relative and
            # |buf| <= sum_j mu^j max|g| = max|g| / (1 - mu); the error then
            # decays with mu, moving w by at most lr / (1 - mu) times it.  Per
            # update w also takes one FP32 rounding (half an ulp of |w|).  So
            # |w - w64| / (lr T) <= 2^-7 max|g| / (1-mu)^2 + ulp(max|w|) / (2 lr).
            gmax = max(np.abs(gi.step_grads(0, t, np.arange(n))[k]).max() for t in range(1, steps + 1))
            wmax = np.abs(dense.w[k]).max(0)
            ulp = np.spacing(wmax.astype(np.float32)).astype(np.float64)
            lr64 = lr.astype(np.float64)
            bound_col = 2.0 ** -7 * gmax / (1 - MU) ** 2 + ulp / (2 * lr64)
            err = np.abs(o3.w[k] - dense.w[k]) / (lr64 * steps)
            assert np.all(err.max(0) <= bound_col), (err.max(0) / bound_col).max()
