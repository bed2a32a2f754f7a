"""Pins of the oracle's optimizer models against the mathematics they follow.

  * dense FP64 Adam (Eq. 1) == torch.optim.Adam in FP64 (independent library);
  * first step moves w by exactly lr*g/(|g|+eps) (closed form);
  * the LUT recurrence of the deferred-update figure == the direct sum of Eq. 3;
  * hand-stepping d zero-gradient dense steps == one restore (Eq. 2-3, eps = 0);
  * deferred FP64 (O2) == dense FP64 with eps = 0, at MAX = inf and MAX = 15,
    for the state after any step and after a flush (the method is exact up to
    rounding apart from the eps factor-out, Sec. 4.3.1 / Sec. 5.5);
  * with eps = 1e-15 the eps factor-out error stays far below FP32 resolution;
  * the FP32 model O3 stays within FP32 rounding of O2, and its FP32 LUT
    within one rounding of the paper's FP64 LUT;
  * the saturating counter never exceeds MAX and forces exactly the rows that
    reach it (Sec. 4.3.2, listing's update set).
"""
import numpy as np
import pytest
import torch

import gs_inputs as gi
from oracle import oracle as orc
from precision_bound import check_bound

B1, B2 = 0.9, 0.999
TAU_GEO = np.array([1, 1, 1, .5, .5, .5, .5, .5, .5, .5])
TAU_APP = np.array([1.0] + [0.1] * 48)


def rel_err(w, ref, tau):
    return np.abs(np.asarray(w, np.float64) - ref) / np.maximum(np.abs(ref), tau)


def _scene(n, seed):
    s = gi.make_scene(n, seed=seed)
    lg, la = gi.lr_columns()
    return s, lg, la


def _vis_sequence(n, steps, p, seed, first_all=True):
    rng = np.random.default_rng(seed)
    out = []
    for t in range(1, steps + 1):
        vis = np.ones(n, bool) if (t == 1 and first_all) else rng.random(n) < p
        out.append(np.nonzero(vis)[0])
    return out


def _gauss_grads(t, ids, seed=0):
    rng = np.random.default_rng(seed * 100003 + t)
    return (rng.normal(0, 1e-3, (ids.shape[0], 10)).astype(np.float32),
            rng.normal(0, 1e-3, (ids.shape[0], 49)).astype(np.float32))


def test_dense_adam_matches_torch_adam():
    n = 300
    s, lg, la = _scene(n, 0)
    dense = orc.DenseAdamF64(s.geo, s.app, lg, la, eps=1e-15)
    groups = [(0, slice(0, 3)), (0, slice(3, 10)), (1, slice(0, 49))]
    params = [torch.tensor(np.array([s.geo, s.app][g][:, sl], np.float64), requires_grad=True)
              for g, sl in groups]
    lrs = [float(lg[0]), float(lg[3]), float(la[0])]
    opt = torch.optim.Adam([{"params": [p], "lr": lr} for p, lr in zip(params, lrs)],
                           betas=(B1, B2), eps=1e-15, foreach=False)
    for t, ids in enumerate(_vis_sequence(n, 25, 0.3, 1), start=1):
        g_geo, g_app = _gauss_grads(t, ids)
        dense.step(t, ids, g_geo, g_app)
        full = [np.zeros((n, 10)), np.zeros((n, 49))]
        full[0][ids] = g_geo
        full[1][ids] = g_app
        for p, (g, sl) in zip(params, groups):
            p.grad = torch.tensor(full[g][:, sl])
        opt.step()
    for p, (g, sl) in zip(params, groups):
        ref = p.detach().numpy()
        assert np.max(np.abs(dense.w[g][:, sl] - ref) / np.maximum(np.abs(ref), 1e-3)) < 1e-13


def test_first_step_closed_form():
    n = 200
    s, lg, la = _scene(n, 1)
    dense = orc.DenseAdamF64(s.geo, s.app, lg, la, eps=1e-15)
    ids = np.arange(n)
    g_geo, g_app = _gauss_grads(1, ids)
    dense.step(1, ids, g_geo, g_app)
    for k, (g, lr, w0) in enumerate(((g_geo, lg, s.geo), (g_app, la, s.app))):
        g = g.astype(np.float64)
        expect = w0.astype(np.float64) - lr.astype(np.float64) * g / (np.abs(g) + 1e-15)
        assert np.max(np.abs(dense.w[k] - expect)) < 1e-15


@pytest.mark.parametrize("t", [2, 5, 17, 100, 1000])
def test_restore_coefficients_equal_the_pseudocode_recurrence(t):
    """The oracle's restore coefficients (the sum of Eq. 3 over the skipped
    steps) against the paper's way of building its lookup table for step t,
    a recurrence from the most recent skipped step backwards (Sec. 4.3.2):
    W[0] = 0, W[d] = (b1/sqrt(b2)) W[d-1] + b1/(sqrt(b2/(1-b2^(t-d))) (1-b1^(t-d)))."""
    dmax = min(t - 1, 300)
    coef, m_dec, v_dec = orc.restore_coeff(B1, B2, t, dmax)
    W = 0.0
    for d in range(dmax + 1):
        if d > 0:
            k = t - d
            W = B1 / np.sqrt(B2) * W + B1 / (np.sqrt(B2 / (1 - B2 ** k)) * (1 - B1 ** k))
        assert abs(coef[d] - W) <= 4e-15 * max(abs(W), 1e-300)
        assert m_dec[d] == pytest.approx(B1 ** (d + 1), rel=1e-15)
        assert v_dec[d] == pytest.approx(B2 ** (d + 1), rel=1e-15)


@pytest.mark.parametrize("L,d", [(1, 1), (3, 5), (10, 40), (50, 200)])
def test_restore_equals_hand_stepping_zero_grads(L, d):
    """Dense Adam with eps = 0 run L steps with gradients, then d steps with
    g = 0, equals the restore of Eq. 2-3 from the state after step L."""
    n = 64
    s, lg, la = _scene(n, 2)
    dense = orc.DenseAdamF64(s.geo, s.app, lg, la, eps=0.0)
    ids = np.arange(n)
    for t in range(1, L + 1):
        dense.step(t, ids, *_gauss_grads(t, ids))
    w_L = [x.copy() for x in dense.w]
    m_L = [x.copy() for x in dense.m]
    v_L = [x.copy() for x in dense.v]
    empty = np.zeros(0, np.int64)
    for t in range(L + 1, L + d + 1):
        dense.step(t, empty, np.zeros((0, 10), np.float32), np.zeros((0, 49), np.float32))
    t = L + d + 1
    coef, _, _ = orc.restore_coeff(B1, B2, t, d)
    for k, lr in enumerate((lg, la)):
        restored = w_L[k] - coef[d] * lr.astype(np.float64) * m_L[k] / np.sqrt(v_L[k])
        assert np.max(np.abs(restored - dense.w[k]) / np.maximum(np.abs(dense.w[k]), 1e-3)) < 1e-13
        # moments decay by b^d over the d zero steps
        assert np.allclose(dense.m[k], m_L[k] * B1 ** d, rtol=1e-13, atol=0)
        assert np.allclose(dense.v[k], v_L[k] * B2 ** d, rtol=1e-13, atol=0)


@pytest.mark.parametrize("max_defer", [0, 15])
def test_deferred_f64_equals_dense_with_eps_zero(max_defer):
    n, steps = 400, 60
    s, lg, la = _scene(n, 3)
    dense = orc.DenseAdamF64(s.geo, s.app, lg, la, eps=0.0)
    o2 = orc.DeferredF64(s.geo, s.app, lg, la, eps=0.0, max_defer=max_defer)
    for t, ids in enumerate(_vis_sequence(n, steps, 0.05, 4), start=1):
        g = _gauss_grads(t, ids, 4)
        dense.step(t, ids, *g)
        o2.step(t, ids, *g)
        if t in (7, 33):
            cg, ca = o2.current(t + 1)
            for k, cur in enumerate((cg, ca)):
                assert np.max(rel_err(cur, dense.w[k], 1e-3)) < 1e-12
    if max_defer:
        assert o2.counter.max() <= max_defer
    o2.flush(steps)
    for k in range(2):
        assert np.max(rel_err(o2.w[k], dense.w[k], 1e-3)) < 1e-12
        # moments: m can cancel (b1^(d+1) m + (1-b1) g), so compare on the group's scale
        assert np.max(np.abs(o2.m[k] - dense.m[k])) < 1e-12 * np.max(np.abs(dense.m[k]))
        assert np.max(np.abs(o2.v[k] - dense.v[k]) / np.maximum(np.abs(dense.v[k]), 1e-30)) < 1e-12


def test_eps_factor_out_error_is_tiny_at_1e_15():
    """The only approximation is factoring eps out of the restore (Sec. 4.3.1,
    Sec. 5.5).  Its error is linear in eps and, at eps = 1e-15, below FP32
    resolution of the parameters."""
    n, steps = 400, 60
    s, lg, la = _scene(n, 5)
    errs = []
    for eps in (1e-15, 1e-12):
        dense = orc.DenseAdamF64(s.geo, s.app, lg, la, eps=eps)
        o2 = orc.DeferredF64(s.geo, s.app, lg, la, eps=eps)
        for t, ids in enumerate(_vis_sequence(n, steps, 0.1, 6, first_all=False), start=1):
            g = gi.step_grads(0, t, ids)
            dense.step(t, ids, *g)
            o2.step(t, ids, *g)
        o2.flush(steps)
        errs.append(max(np.max(rel_err(o2.w[0], dense.w[0], TAU_GEO)),
                        np.max(rel_err(o2.w[1], dense.w[1], TAU_APP))))
    assert errs[0] < 6e-8
    assert 500 < errs[1] / errs[0] < 2000


@pytest.mark.parametrize("t", [2, 17, 100, 1000])
def test_spec_lut_within_one_rounding_of_paper_lut(t):
    dmax = t - 1
    lut, mom, var = orc.restore_coeff(B1, B2, t, dmax)
    Wf, Mf, Vf, ss, bc = orc.lut_spec(B1, B2, t, dmax)
    for a, b in ((Wf, lut), (Mf, mom), (Vf, var)):
        ulp = np.spacing(np.abs(b).astype(np.float32)).astype(np.float64)
        assert np.all(np.abs(a.astype(np.float64) - b) <= ulp)
    assert abs(float(ss) - 1 / (1 - B1 ** t)) <= np.spacing(np.float32(ss))
    assert abs(float(bc) - np.sqrt(1 - B2 ** t)) <= np.spacing(np.float32(bc))


@pytest.mark.parametrize("max_defer", [0, 15])
def test_f32_model_within_fp32_rounding_of_f64(max_defer):
    n, steps = 2000, 20
    s, lg, la = _scene(n, 7)
    o2 = orc.DeferredF64(s.geo, s.app, lg, la, max_defer=max_defer)
    o3 = orc.DeferredF32(s.geo, s.app, lg, la, max_defer=max_defer)
    dense = orc.DenseAdamF64(s.geo, s.app, lg, la)
    for t, ids in enumerate(_vis_sequence(n, steps, 0.3, 8, first_all=False), start=1):
        g = gi.step_grads(0, t, ids)
        o2.step(t, ids, *g)
        o3.step(t, ids, *g)
        dense.step(t, ids, *g)
        cg3, _ = o3.current(t + 1)
        cg2, _ = o2.current(t + 1)
        assert np.max(rel_err(cg3, cg2, TAU_GEO)) < 1e-6
    assert np.array_equal(o2.counter, o3.counter)
    o2.flush(steps)
    o3.flush(steps)
    for k, tau in ((0, TAU_GEO), (1, TAU_APP)):
        assert np.max(rel_err(o3.w[k], o2.w[k], tau)) < 1e-6
        assert np.max(rel_err(o3.w[k], dense.w[k], tau)) < 1e-6


def test_saturation_forces_exactly_the_rows_at_max():
    n, steps, MAX = 300, 50, 15
    s, lg, la = _scene(n, 9)
    o2 = orc.DeferredF64(s.geo, s.app, lg, la, max_defer=MAX)
    forced_total = 0
    for t, ids in enumerate(_vis_sequence(n, steps, 0.02, 10, first_all=False), start=1):
        before = o2.counter.copy()
        valid, sat = o2.step(t, ids, *_gauss_grads(t, ids))
        expect = np.setdiff1d(np.nonzero(before == MAX)[0], ids)
        assert np.array_equal(np.sort(sat), expect)
        assert o2.counter.max() <= MAX
        forced_total += sat.shape[0]
    # at a 2% visible rate nearly every row is forced once every 16 steps
    assert forced_total > 0.8 * n * (steps - MAX) / (MAX + 1)


def test_bf16_stochastic_rounding_is_unbiased_and_brackets():
    """Averaged over all 2^16 random inputs, BF16 stochastic rounding returns
    the FP32 value exactly; every result is one of the two BF16 neighbours."""
    rng = np.random.default_rng(11)
    f = orc.lib().orc_bf16_sr
    xs = np.concatenate([rng.normal(0, 1e-3, 20), rng.normal(0, 1e3, 5), [1.0, -2.5, 3e-39, 6.1e-5]])
    for x in xs.astype(np.float32):
        outs = np.array([f(float(x), r) for r in range(0, 65536, 1)], np.uint16)
        vals = (outs.astype(np.uint32) << 16).view(np.float32).astype(np.float64)
        lo = (np.array([x], np.float32).view(np.uint32) & np.uint32(0xffff0000)).view(np.float32)[0]
        assert set(np.unique(outs)).issubset({int(np.array([lo]).view(np.uint32)[0] >> 16),
                                              int(np.array([lo]).view(np.uint32)[0] >> 16) + 1})
        assert vals.mean() == pytest.approx(float(x), rel=1e-12, abs=1e-45)
    inf = f(float("inf"), 12345)
    assert inf == 0x7f80
    assert f(float("nan"), 0) & 0x7f80 == 0x7f80


def test_bf16_state_tracks_fp32_state():
    """O4 (BF16 moments, stochastic rounding) stays within its a-posteriori
    bound of dense FP64 Adam over 30 steps, and within BF16-level error of O3
    (FP32 moments); O3 with the dense-geometry split matches dense FP64 Adam to
    FP32 rounding."""
    n, steps = 2000, 30
    s, lg, la = _scene(n, 12)
    o3 = orc.DeferredF32(s.geo, s.app, lg, la)
    o4 = orc.DeferredF32(s.geo, s.app, lg, la, state="bf16", sr_seed=3, track_bound=True)
    od = orc.DeferredF32(s.geo, s.app, lg, la, geo_dense=True)
    dense = orc.DenseAdamF64(s.geo, s.app, lg, la)
    for t, ids in enumerate(_vis_sequence(n, steps, 0.3, 13, first_all=False), start=1):
        g = gi.step_grads(0, t, ids)
        for mdl in (o3, o4, od, dense):
            mdl.step(t, ids, *g)
    for mdl in (o3, o4, od):
        mdl.flush(steps)
    check_bound(o4.w, o4, dense, steps, (lg, la), "bf16")
    for k, tau in ((0, TAU_GEO), (1, TAU_APP)):
        assert np.max(rel_err(od.w[k], dense.w[k], tau)) < 1e-6
    m4, v4 = o4.moments_f32(1)
    assert np.max(np.abs(m4 - o3.m[1])) < 0.02 * np.max(np.abs(o3.m[1]))
    assert np.max(np.abs(v4 - o3.v[1]) / np.maximum(o3.v[1], 1e-30)) < 0.05


def test_e4m3_codes_follow_the_ocp_definition():
    """E4M3FN: bias 7, 3 mantissa bits, subnormals m*2^-9, max 448, NaN S.1111.111."""
    dec = orc.e4m3_decode(np.arange(256, dtype=np.uint8))
    assert dec[0x38] == 1.0 and dec[0x40] == 2.0 and dec[0x7E] == 448.0 and dec[0xFE] == -448.0
    assert dec[0x08] == 2.0 ** -6 and dec[0x01] == 2.0 ** -9 and dec[0x07] == 7 * 2.0 ** -9
    assert np.isnan(dec[0x7F]) and np.isnan(dec[0xFF])
    finite = np.sort(np.unique(dec[np.isfinite(dec)]))
    assert finite.shape[0] == 253 and finite.max() == 448.0     # +-0 share a value
    f = orc.lib().orc_e4m3_sr
    for c in range(256):
        if np.isfinite(dec[c]) and c != 0x80:
            assert f(float(dec[c]), 0) == c and f(float(dec[c]), 65535) == c
    assert f(1e6, 0) == 0x7E and f(-1e6, 0) == 0xFE                 # saturation
    assert f(float("nan"), 0) == 0x7F


def test_e4m3_decode_matches_torch_float8():
    """All 256 codes: the oracle's E4M3FN decoding equals torch's float8_e4m3fn
    cast to FP32 (an independent implementation of the OCP format), NaN codes
    included."""
    codes = np.arange(256, dtype=np.uint8)
    ref = torch.from_numpy(codes).view(torch.float8_e4m3fn).to(torch.float32).numpy()
    dec = orc.e4m3_decode(codes)
    nan = np.isnan(ref)
    assert np.array_equal(nan, np.isnan(dec))
    assert np.array_equal(ref[~nan].view(np.uint32), dec[~nan].view(np.uint32))
    # and round-to-nearest encoding of every finite value gives back its code (+0 for -0)
    enc = torch.from_numpy(dec[~nan]).to(torch.float8_e4m3fn).view(torch.uint8).numpy()
    assert np.array_equal(enc[codes[~nan] != 0x80], codes[~nan][codes[~nan] != 0x80])


def test_quantised_bound_holds_under_long_deferral_and_subnormal_codes():
    """The a-posteriori bound of the quantised models holds element by element
    where the moments of rarely visible rows decay far below their block's
    scale (E4M3 subnormal codes, a lost second moment) and with the saturating
    counter; a mistake planted in the model's result is caught by it."""
    n, steps = 2048, 160
    s, lg, la = _scene(n, 31)
    for state, K in (("fp8", 0), ("fp8", 15), ("bf16", 0)):
        o4 = orc.DeferredF32(s.geo, s.app, lg, la, state=state, sr_seed=6, max_defer=K, track_bound=True)
        dense = orc.DenseAdamF64(s.geo, s.app, lg, la)
        rng = np.random.default_rng(77)
        # a few rows are visible at almost every step (they set the block
        # scales), the rest rarely
        busy = rng.random(n) < 0.05
        for t in range(1, steps + 1):
            ids = np.nonzero(busy | (rng.random(n) < 0.01))[0]
            g = gi.step_grads(2, t, ids)
            o4.step(t, ids, *g)
            dense.step(t, ids, *g)
        o4.flush(steps)
        if state == "fp8":
            codes = np.concatenate([o4.m[0].ravel(), o4.m[1].ravel()])
            assert np.count_nonzero((codes & 0x78) == 0) > 0, "no subnormal codes exercised"
        check_bound(o4.w, o4, dense, steps, (lg, la), f"{state} K={K}")
        # a planted error of twice an element's bound is detected
        k, i, j = 1, int(np.argmax(o4.bw[1].max(1))), 0
        o4.w[k][i, j] = np.float32(dense.w[k][i, j] + 2.0 * o4.bw[k][i, j] + 1e-6)
        with pytest.raises(AssertionError):
            check_bound(o4.w, o4, dense, steps, (lg, la), "planted")


def test_e4m3_stochastic_rounding_is_unbiased_and_brackets():
    rng = np.random.default_rng(5)
    f = orc.lib().orc_e4m3_sr
    ys = np.concatenate([rng.uniform(-440, 440, 8), rng.uniform(-1e-2, 1e-2, 6), [3e-3, 0.3, 17.0]])
    for y in ys.astype(np.float32):
        outs = np.array([f(float(y), r) for r in range(65536)], np.uint8)
        vals = orc.e4m3_decode(outs).astype(np.float64)
        assert np.unique(vals).shape[0] <= 2
        lo, hi = vals.min(), vals.max()
        assert lo <= y <= hi
        assert vals.mean() == pytest.approx(float(y), abs=(hi - lo) * 2.0 ** -15 + 1e-30)


def test_fp8_scale_rule():
    f = orc.lib().orc_fp8_scale_for
    for amax in [1e-9, 3e-4, 0.7, 448.0, 449.0, 1e5]:
        s = f(amax)
        assert s > 0 and np.log2(s) == np.round(np.log2(s))
        assert amax / s <= 448.0 * (1 + 1e-6) and amax / (s / 2) > 448.0 * (1 - 1e-6)
    assert f(0.0) == 0.0 and f(float("inf")) == 0.0


def test_fp8_state_tracks_dense_and_keeps_codes_in_range():
    n, steps = 1500, 30
    s, lg, la = _scene(n, 21)
    o8 = orc.DeferredF32(s.geo, s.app, lg, la, state="fp8", sr_seed=4, max_defer=15, track_bound=True)
    dense = orc.DenseAdamF64(s.geo, s.app, lg, la)
    for t, ids in enumerate(_vis_sequence(n, steps, 0.3, 22, first_all=False), start=1):
        g = gi.step_grads(0, t, ids)
        o8.step(t, ids, *g)
        dense.step(t, ids, *g)
        for k in range(2):
            mm, vv = o8.moments_f32(k)
            blk = np.arange(n) // orc.FP8_BLOCK
            assert np.all(np.abs(mm) <= 448.0 * o8.ms[k][blk][:, None])
            assert np.all(vv >= 0) and np.all(np.sqrt(vv) <= 448.0 * o8.vs[k][blk][:, None])
    o8.flush(steps)
    check_bound(o8.w, o8, dense, steps, (lg, la), "fp8")


def _schedule(steps, seed):
    """A learning-rate multiplier per step: exponential decay with noise, the
    shape of the position-rate schedule of 3DGS training, kept adversarial."""
    rng = np.random.default_rng(seed)
    t = np.arange(steps + 2, dtype=np.float64)
    return 0.01 ** (t / (steps + 1)) * rng.uniform(0.5, 2.0, steps + 2)


@pytest.mark.parametrize("max_defer", [0, 15])
def test_deferred_f64_with_schedule_equals_dense(max_defer):
    """With a per-step rate the skipped step k contributes s[k] c(k) and the
    method stays exact at eps = 0 (each term of Eq. 3 carries its own rate)."""
    n, steps = 400, 60
    s, lg, la = _scene(n, 13)
    sc = _schedule(steps, 14)
    dense = orc.DenseAdamF64(s.geo, s.app, lg, la, eps=0.0, sched=sc)
    o2 = orc.DeferredF64(s.geo, s.app, lg, la, eps=0.0, max_defer=max_defer, sched=sc)
    plain = orc.DenseAdamF64(s.geo, s.app, lg, la, eps=0.0)
    for t, ids in enumerate(_vis_sequence(n, steps, 0.05, 15), start=1):
        g = _gauss_grads(t, ids, 16)
        dense.step(t, ids, *g)
        o2.step(t, ids, *g)
        plain.step(t, ids, *g)
    o2.flush(steps)
    for k in range(2):
        assert np.max(rel_err(o2.w[k], dense.w[k], 1e-3)) < 1e-12
    # the schedule really changes the trajectory (a dropped s[k] would fail above)
    assert np.max(rel_err(plain.w[0], dense.w[0], 1e-3)) > 1e-5


def test_spec_lut_with_schedule_within_one_rounding_of_paper_lut():
    sc = _schedule(200, 3)
    for t in (2, 50, 201):
        lut, _, _ = orc.restore_coeff(B1, B2, t, t - 1, sc)
        Wf, _, _, ss, _ = orc.lut_spec(B1, B2, t, t - 1, sc)
        ulp = np.spacing(np.abs(lut).astype(np.float32)).astype(np.float64)
        assert np.all(np.abs(Wf.astype(np.float64) - lut) <= ulp)
        assert abs(float(ss) - sc[t] / (1 - B1 ** t)) <= np.spacing(np.float32(ss))
    # a constant schedule of 1 gives the unscheduled tables bit for bit
    one = np.ones(202)
    a = orc.lut_spec(B1, B2, 100, 99, one)
    b = orc.lut_spec(B1, B2, 100, 99)
    assert all(np.array_equal(np.asarray(x).view(np.uint32), np.asarray(y).view(np.uint32))
               for x, y in zip(a, b))


def test_f32_model_with_schedule_within_fp32_rounding_of_dense():
    n, steps = 2000, 20
    s, lg, la = _scene(n, 17)
    sc = _schedule(steps, 18)
    o3 = orc.DeferredF32(s.geo, s.app, lg, la, max_defer=15, sched=sc)
    dense = orc.DenseAdamF64(s.geo, s.app, lg, la, sched=sc)
    for t, ids in enumerate(_vis_sequence(n, steps, 0.3, 19, first_all=False), start=1):
        g = gi.step_grads(0, t, ids)
        o3.step(t, ids, *g)
        dense.step(t, ids, *g)
    o3.flush(steps)
    for k, tau in ((0, TAU_GEO), (1, TAU_APP)):
        assert np.max(rel_err(o3.w[k], dense.w[k], tau)) < 1e-6


def test_e4m3_exponent_shift_is_exact_stochastic_rounding():
    """Growing a block scale by 2^k re-encodes each code as SR(x / 2^k).  For a
    normal code whose exponent stays normal the value is exactly representable,
    so every random draw gives the code with k taken off the exponent field
    (the rescale kernel's fast path); all other codes need the full rounding."""
    f = orc.lib().orc_e4m3_sr
    for code in range(256):
        e, m = (code >> 3) & 15, code & 7
        if e == 0 or (e == 15 and m == 7):
            continue
        x = float(orc.e4m3_decode(np.array([code], np.uint8))[0])
        for k in range(1, 12):
            y = np.float32(x * 2.0 ** -k)
            got = {f(float(y), r) for r in (0, 1, 0x7fff, 0xfffe, 0xffff)}
            if e - k >= 1:
                assert got == {(code & 0x80) | ((e - k) << 3) | m}, (code, k)
