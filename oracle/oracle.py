"""Python driver of the CPU oracle (TEST INFRASTRUCTURE ONLY).

Only the tests, the smoke check and the CPU-baseline leg of the benchmark may
import this module.  It loads ``liboracle.so`` built from ``gs_oracle.c`` (plain
C, ``-O2 -ffp-contract=off -fno-fast-math``) and never touches the HIP library.

Models
  DenseAdamF64     Eq. 1 stepped on every row every step (the definition).
  DeferredF64      the deferred-update figure in FP64 (model O2): restore with
                   the paper's LUTs, Adam on update_ids = valid_ids U saturated.
  DeferredF32      the same algorithm with FP32 state and the implementation's
                   fixed operation order (model O3); its cull of the *current*
                   geometry gives the visible sets.
Every simulation may run on a subset of rows (``keys`` = the rows' Gaussian
ids): rows are independent given their own visibility, so a row sample is
exact for the sampled rows.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "gs_oracle.c")
LIB = os.path.join(HERE, "liboracle.so")

GEO_DIM, APP_DIM = 10, 49


def build(force: bool = True) -> str:
    """Compile liboracle.so with gcc (no contraction, no fast-math, OpenMP)."""
    if force or not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
        tmp = LIB + ".tmp%d" % os.getpid()
        cmd = ["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fopenmp", "-fPIC",
               "-shared", "-std=c11", "-Wall", "-o", tmp, SRC, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, LIB)
    return LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
            build(force=True)
        L = C.CDLL(LIB)
        vp, i64, i32, f64, f32 = C.c_void_p, C.c_int64, C.c_int, C.c_double, C.c_float
        sig = {
            "orc_exp_gs": (f32, [f32]),
            "orc_cull_v1": (None, [i64, vp, vp, vp, vp]),
            "orc_compact": (i64, [i64, vp, vp]),
            "orc_adam_dense_f64": (None, [i64, i32, vp, vp, vp, vp, vp, f64, f64, f64, i64]),
            "orc_adam_dense_sparse_grad_f64": (None, [i64, i32, vp, vp, vp, i64, vp, vp, vp,
                                                       f64, f64, f64, i64]),
            "orc_restore_coeff_f64": (None, [f64, f64, i64, i32, vp, vp, vp, vp]),
            "orc_deferred_rows_f64": (None, [i32, vp, vp, vp, i64, vp, vp, vp, vp, f64, f64, f64,
                                             i64, f64, vp, vp, vp]),
            "orc_restore_rows_f64": (None, [i32, vp, vp, vp, i64, vp, vp, vp, f64, vp, vp]),
            "orc_flush_rows_f64": (None, [i32, vp, vp, vp, i64, vp, vp, vp, f64, f64, f64, vp]),
            "orc_lut_spec": (None, [f64, f64, i64, i32, vp, vp, vp, vp, vp, vp]),
            "orc_restore_bound": (f32, [f64, f64]),
            "orc_bf16_sr": (C.c_uint16, [f32, C.c_uint32]),
            "orc_e4m3_sr": (C.c_uint8, [f32, C.c_uint32]),
            "orc_fp8_scale_for": (f32, [f32]),
            "orc_deferred_rows_fp8": (None, [i32, vp, vp, vp, vp, vp, i64, i64, i64, vp, vp, vp, i64, vp,
                                             f64, f64, f64, vp, vp, vp, f32, f32, f32, C.c_uint64, i64, i32, vp]),
            "orc_restore_rows_fp8": (None, [i32, vp, vp, vp, vp, vp, i64, i64, vp, vp, vp, f64, vp, f32, vp]),
            "orc_flush_rows_fp8": (None, [i32, vp, vp, vp, vp, vp, i64, i64, vp, vp, vp, f64, vp, vp, vp, f32,
                                          C.c_uint64, i64, i32, f64, vp]),
            "orc_deferred_rows_f32": (None, [i32, vp, vp, vp, i32, i64, i64, vp, vp, vp, i64, vp,
                                             f64, f64, f64, vp, vp, vp, f32, f32, f32, C.c_uint64, i64, i32, vp]),
            "orc_restore_rows_f32": (None, [i32, vp, vp, vp, i32, i64, i64, vp, vp, vp, f64, vp, f32, vp]),
            "orc_flush_rows_f32": (None, [i32, vp, vp, vp, i32, i64, i64, vp, vp, vp, f64, vp, vp, vp, f32,
                                          C.c_uint64, i64, i32, f64, vp]),
            "orc_sgdm_dense_sparse_grad_f64": (None, [i64, i32, vp, vp, i64, vp, vp, vp, f64, f64]),
            "orc_lut_sgdm_f64": (None, [f64, i64, i32, vp, vp, vp]),
            "orc_lut_sgdm_spec": (None, [f64, i64, i32, vp, vp, vp, vp]),
            "orc_sgdm_deferred_rows_f64": (None, [i32, vp, vp, i64, vp, vp, vp, vp, f64, vp, vp]),
            "orc_sgdm_flush_rows_f64": (None, [i32, vp, vp, i64, vp, vp, vp, vp, f64]),
            "orc_sgdm_rows_f32": (None, [i32, vp, vp, i32, i64, i64, vp, vp, vp, i64, vp, vp, vp, f32,
                                         C.c_uint64, i64, i32]),
            "orc_sgdm_restore_rows_f32": (None, [i32, vp, vp, i32, i64, i64, vp, vp, vp, vp, vp]),
            "orc_sgdm_flush_rows_f32": (None, [i32, vp, vp, i32, i64, i64, vp, vp, vp, vp, vp, C.c_uint64,
                                               i64, i32]),
            "orc_adamw_dense_sparse_grad_f64": (None, [i64, i32, vp, vp, vp, i64, vp, vp, vp, f64, f64, f64, f64,
                                                        i64]),
            "orc_lut_adamw_f64": (None, [f64, f64, f64, f64, i64, i32, vp, vp, vp]),
            "orc_lut_adamw_spec": (None, [f64, f64, f64, f64, i64, i32, vp, vp, vp, vp]),
            "orc_adamw_deferred_rows_f64": (None, [i32, vp, vp, vp, i64, vp, vp, vp, vp, f64, f64, f64, i64, f64,
                                                   f64, vp, vp, i64, vp, vp]),
            "orc_adamw_restore_rows_f64": (None, [i32, vp, vp, vp, i64, vp, vp, vp, f64, vp, vp, i64, vp]),
            "orc_adamw_flush_rows_f64": (None, [i32, vp, vp, vp, i64, vp, vp, vp, f64, f64, f64, vp, vp, i64]),
            "orc_adamw_rows_f32": (None, [i32, vp, vp, vp, i32, i64, i64, vp, vp, vp, i64, vp, f64, f64, f64,
                                          vp, vp, i64, vp, vp, vp, f32, f32, f32, C.c_uint64, i64, i32]),
            "orc_adamw_restore_rows_f32": (None, [i32, vp, vp, vp, i32, i64, i64, vp, vp, vp, f64, vp, vp, i64,
                                                  f32, vp]),
            "orc_adamw_flush_rows_f32": (None, [i32, vp, vp, vp, i32, i64, i64, vp, vp, vp, f64, vp, vp, i64, vp,
                                                vp, f32, C.c_uint64, i64, i32]),
            "orc_densify": (i64, [i64, i32, vp, vp, vp, vp, vp, f32, f32, i32, f32, f32, f32, f32, C.c_uint64,
                                  i64, vp, vp, vp, vp, vp]),
            "orc_densify_thresholds": (None, [f64, f64, f64, vp]),
            "orc_set_threads": (i32, [i32]),
        }
        for name, (res, args) in sig.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def set_threads(n: int) -> int:
    """Thread count of the oracle's OpenMP loops; returns the previous one."""
    return int(lib().orc_set_threads(int(n)))


def _p(a, dtype=None):
    if a is None:
        return None
    if dtype is not None:
        assert a.dtype == dtype, (a.dtype, dtype)
    assert a.flags["C_CONTIGUOUS"]
    return a.ctypes.data


# ---------------------------------------------------------------------------
# cull
# ---------------------------------------------------------------------------
def cam_floats(cam) -> np.ndarray:
    """R(9), t(3), fx, fy, cx, cy, W, H, near, far as float32."""
    if isinstance(cam, np.ndarray):
        out = cam.astype(np.float32)
    else:
        out = cam.as_floats()
    assert out.shape == (20,)
    return np.ascontiguousarray(out)


def exp_gs(x: np.ndarray) -> np.ndarray:
    f = lib().orc_exp_gs
    x = np.asarray(x, np.float32).ravel()
    return np.array([f(float(v)) for v in x], np.float32)


def cull(geo: np.ndarray, cam, detail: bool = False):
    """keep mask (bool [n]) of cull_v1 on FP32 geometry [n,10]; optional detail [n,11]."""
    geo = np.ascontiguousarray(geo, np.float32)
    n = geo.shape[0]
    keep = np.zeros(n, np.uint8)
    det = np.zeros((n, 11), np.float32) if detail else None
    lib().orc_cull_v1(n, _p(geo), _p(cam_floats(cam)), _p(keep), _p(det))
    return (keep.astype(bool), det) if detail else keep.astype(bool)


def compact(keep: np.ndarray) -> np.ndarray:
    k = np.ascontiguousarray(keep, np.uint8)
    ids = np.empty(k.shape[0], np.uint32)
    m = lib().orc_compact(k.shape[0], _p(k), _p(ids))
    return ids[:m].copy()


# ---------------------------------------------------------------------------
# LUTs
# ---------------------------------------------------------------------------
def _sched(sched):
    return None if sched is None else np.ascontiguousarray(sched, np.float64)


def restore_coeff(b1: float, b2: float, step: int, dmax: int, sched=None):
    """(coef, m_dec, v_dec), FP64, unit rate, d = 0..dmax: the restore
    coefficient of Eq. 3 summed over a row's skipped steps, and the moments'
    decay b1^(d+1), b2^(d+1) to update `step`; sched: optional per-step
    learning-rate multiplier (index = step)."""
    coef = np.zeros(dmax + 1); mdec = np.zeros(dmax + 1); vdec = np.zeros(dmax + 1)
    sc = _sched(sched)
    lib().orc_restore_coeff_f64(b1, b2, step, dmax, _p(sc), _p(coef), _p(mdec), _p(vdec))
    return coef, mdec, vdec


def lut_spec(b1: float, b2: float, step: int, dmax: int, sched=None):
    """FP32 tables (Wf, Mf, Vf, ss, bc) of the implementation spec for update `step`."""
    Wf = np.zeros(dmax + 1, np.float32); Mf = np.zeros(dmax + 1, np.float32)
    Vf = np.zeros(dmax + 1, np.float32)
    ss = C.c_float(); bc = C.c_float()
    sc = _sched(sched)
    lib().orc_lut_spec(b1, b2, step, dmax, _p(sc), _p(Wf), _p(Mf), _p(Vf), C.addressof(ss), C.addressof(bc))
    return Wf, Mf, Vf, np.float32(ss.value), np.float32(bc.value)


# ---------------------------------------------------------------------------
# dense Adam (Eq. 1)
# ---------------------------------------------------------------------------
class DenseAdamF64:
    """FP64 Adam on every row every step; rows without a gradient use g = 0."""

    def __init__(self, geo, app, lr_geo, lr_app, b1=0.9, b2=0.999, eps=1e-15, sched=None):
        self.w = [np.array(geo, np.float64), np.array(app, np.float64)]
        self.m = [np.zeros_like(x) for x in self.w]
        self.v = [np.zeros_like(x) for x in self.w]
        self.lr = [np.asarray(lr_geo, np.float64), np.asarray(lr_app, np.float64)]
        self.b1, self.b2, self.eps = b1, b2, eps
        self.sched = _sched(sched)

    def step(self, t: int, ids: np.ndarray, g_geo: np.ndarray, g_app: np.ndarray):
        ids = np.ascontiguousarray(ids, np.uint32)
        s = 1.0 if self.sched is None else float(self.sched[t])
        for k, g in enumerate((g_geo, g_app)):
            g = np.ascontiguousarray(g, np.float32)
            w, m, v = self.w[k], self.m[k], self.v[k]
            lr = np.ascontiguousarray(self.lr[k] * s)
            lib().orc_adam_dense_sparse_grad_f64(w.shape[0], w.shape[1], _p(w), _p(m), _p(v),
                                                 ids.shape[0], _p(ids), _p(g), _p(lr),
                                                 self.b1, self.b2, self.eps, t)


class DenseAdamF32:
    """Eq. 1 in FP32 on every row every step (numpy float32 arithmetic, one
    operation at a time; bias corrections rounded once from FP64).  It is the
    yardstick of FP32 rounding: an FP32-state deferred run is judged against
    dense FP64 Adam relative to the error this plain FP32 Adam makes."""

    def __init__(self, geo, app, lr_geo, lr_app, b1=0.9, b2=0.999, eps=1e-15):
        self.w = [np.array(geo, np.float32), np.array(app, np.float32)]
        self.m = [np.zeros_like(x) for x in self.w]
        self.v = [np.zeros_like(x) for x in self.w]
        self.lr = [np.asarray(lr_geo, np.float32), np.asarray(lr_app, np.float32)]
        self.b1, self.b2, self.eps = np.float32(b1), np.float32(b2), np.float32(eps)
        self.omb1, self.omb2 = np.float32(1.0 - b1), np.float32(1.0 - b2)
        self.B1, self.B2 = b1, b2

    def step(self, t: int, ids: np.ndarray, g_geo: np.ndarray, g_app: np.ndarray):
        ids = np.asarray(ids, np.int64)
        bc1 = np.float32(1.0 - self.B1 ** t)
        bc2 = np.float32(1.0 - self.B2 ** t)
        for k, g in enumerate((g_geo, g_app)):
            gd = np.zeros_like(self.w[k])
            gd[ids] = np.asarray(g, np.float32)
            m = self.b1 * self.m[k] + self.omb1 * gd
            v = self.b2 * self.v[k] + (self.omb2 * gd) * gd
            self.m[k], self.v[k] = m, v
            den = np.sqrt(v / bc2) + self.eps
            self.w[k] = self.w[k] - (self.lr[k] * (m / bc1)) / den


# ---------------------------------------------------------------------------
# deferred models
# ---------------------------------------------------------------------------
class _Deferred:
    """Common bookkeeping of the deferred-update figure: a per-row counter of
    deferred steps, update_ids = union(valid_ids, where(counter == MAX)),
    counters of updated rows reset and all others incremented.  max_defer = 0
    means no saturation (the counter never forces an update)."""

    def __init__(self, n, max_defer):
        self.counter = np.zeros(n, np.int64)
        self.max_defer = int(max_defer)

    def update_set(self, valid):
        valid = np.asarray(valid, np.int64)
        if self.max_defer > 0:
            sat = np.nonzero(self.counter == self.max_defer)[0]
            sat = np.setdiff1d(sat, valid, assume_unique=True)
        else:
            sat = np.zeros(0, np.int64)
        return valid, sat

    def bump(self, valid, sat):
        self.counter += 1
        self.counter[valid] = 0
        self.counter[sat] = 0

    def dmax(self, t):
        return min(t - 1, self.max_defer) if self.max_defer > 0 else t - 1

    def last_step(self, t_done: int) -> np.ndarray:
        """last update step of every row after update t_done (0 = never)."""
        return (t_done - self.counter).astype(np.int32)


class DeferredF64(_Deferred):
    """Model O2: the deferred update of Sec. 4.3 (restore with the stored
    moments, decayed moments, Adam step; Eq. 1-3) with FP64 state."""

    def __init__(self, geo, app, lr_geo, lr_app, b1=0.9, b2=0.999, eps=1e-15, max_defer=0, sched=None):
        super().__init__(geo.shape[0], max_defer)
        self.w = [np.array(geo, np.float64), np.array(app, np.float64)]
        self.m = [np.zeros_like(x) for x in self.w]
        self.v = [np.zeros_like(x) for x in self.w]
        self.lr = [np.asarray(lr_geo, np.float64), np.asarray(lr_app, np.float64)]
        self.b1, self.b2, self.eps = b1, b2, eps
        self.sched = _sched(sched)

    def current(self, t: int, rows=None):
        """Restored values of rows (default all) before update t: (geo, app)."""
        rows = np.arange(self.counter.shape[0]) if rows is None else np.asarray(rows)
        rows32 = np.ascontiguousarray(rows, np.uint32)
        d = np.ascontiguousarray(self.counter[rows], np.int64)
        coef, _, _ = restore_coeff(self.b1, self.b2, t, max(self.dmax(t), 0), self.sched)
        out = []
        for k in range(2):
            o = np.zeros((rows.shape[0], self.w[k].shape[1]))
            lib().orc_restore_rows_f64(self.w[k].shape[1], _p(self.w[k]), _p(self.m[k]), _p(self.v[k]),
                                       rows.shape[0], _p(rows32), _p(d), _p(self.lr[k]), self.eps,
                                       _p(coef), _p(o))
            out.append(o)
        return out[0], out[1]

    def step(self, t, valid, g_geo, g_app):
        valid, sat = self.update_set(valid)
        rows = np.ascontiguousarray(np.concatenate([valid, sat]), np.uint32)
        d = np.ascontiguousarray(self.counter[rows.astype(np.int64)], np.int64)
        coef, m_dec, v_dec = restore_coeff(self.b1, self.b2, t, max(self.dmax(t), 0), self.sched)
        s_t = 1.0 if self.sched is None else float(self.sched[t])
        for k, g in enumerate((g_geo, g_app)):
            dim = self.w[k].shape[1]
            gg = np.zeros((rows.shape[0], dim))
            gg[:valid.shape[0]] = np.asarray(g, np.float64)
            lib().orc_deferred_rows_f64(dim, _p(self.w[k]), _p(self.m[k]), _p(self.v[k]), rows.shape[0],
                                        _p(rows), _p(d), _p(gg), _p(self.lr[k]), self.b1, self.b2,
                                        self.eps, t, s_t, _p(coef), _p(m_dec), _p(v_dec))
        self.bump(valid, sat)
        return valid, sat

    def flush(self, t_done: int):
        rows = np.nonzero(self.counter > 0)[0]
        if rows.shape[0] == 0:
            return
        delta = np.ascontiguousarray(self.counter[rows], np.int64)
        coef, _, _ = restore_coeff(self.b1, self.b2, t_done + 1, int(delta.max()), self.sched)
        rows32 = np.ascontiguousarray(rows, np.uint32)
        for k in range(2):
            lib().orc_flush_rows_f64(self.w[k].shape[1], _p(self.w[k]), _p(self.m[k]), _p(self.v[k]),
                                     rows.shape[0], _p(rows32), _p(delta), _p(self.lr[k]),
                                     self.b1, self.b2, self.eps, _p(coef))
        self.counter[:] = 0


def restore_bound(b1: float, b2: float) -> np.float32:
    """Clamp of the restore factor m/(sqrt(v)+eps) (1.03 x the Adam ratio bound)."""
    return np.float32(lib().orc_restore_bound(b1, b2))


STATES = {"f32": (0, np.float32), "bf16": (1, np.uint16), "fp8": (2, np.uint8)}
FP8_BLOCK = 128


def e4m3_decode(codes: np.ndarray) -> np.ndarray:
    """FP32 values of E4M3FN codes (bias 7, max 448, NaN = S.1111.111)."""
    c = np.asarray(codes, np.uint8).astype(np.int32)
    e, m = (c >> 3) & 15, c & 7
    a = np.where(e == 0, m * 2.0 ** -9, (8 + m) * 2.0 ** (e - 10.0))
    a = np.where((e == 15) & (m == 7), np.nan, a)
    return np.where(c & 0x80, -a, a).astype(np.float32)


class _Track(C.Structure):
    """Mirror of orc_track: stochastic-rounding keys of the rows and the
    per-element error-bound arrays of the quantised models."""
    _fields_ = [("keys", C.c_void_p), ("em", C.c_void_p), ("ev", C.c_void_p), ("bw", C.c_void_p),
                ("cs", C.c_double)]


def adam_ratio_bound(b1: float, b2: float) -> float:
    """Cauchy-Schwarz bound of |m| / sqrt(v) for Adam moments grown from zero."""
    return (1.0 - b1) / np.sqrt((1.0 - b2) * (1.0 - b1 * b1 / b2)) * (1.0 + 1e-12)


class DeferredF32(_Deferred):
    """Model O3 (state='f32') / O4 (state='bf16'): deferred algorithm with FP32
    math, moments stored in FP32 or in BF16 with stochastic rounding (random
    bits from SplitMix64 of (sr_seed, step, row key, global column)), and the
    implementation's op order.  `keys` are the Gaussian ids of the rows (for
    the rounding stream); default 0..n-1."""

    def __init__(self, geo, app, lr_geo, lr_app, b1=0.9, b2=0.999, eps=1e-15, max_defer=0,
                 state="f32", sr_seed=0, keys=None, app_state=None, geo_dense=False, sched=None,
                 track_bound=False):
        super().__init__(geo.shape[0], max_defer)
        self.sched = _sched(sched)
        # geo_dense: the geometric group takes a plain Adam step on every row
        # every step (the split of Sec. 4.2.2); only the appearance is deferred
        self.geo_dense = bool(geo_dense)
        states = [state, app_state or state]
        self.sid = [STATES[x][0] for x in states]
        self.w = [np.array(geo, np.float32), np.array(app, np.float32)]
        self.m = [np.zeros(x.shape, STATES[st][1]) for x, st in zip(self.w, states)]
        self.v = [np.zeros(x.shape, STATES[st][1]) for x, st in zip(self.w, states)]
        nb = (geo.shape[0] + FP8_BLOCK - 1) // FP8_BLOCK
        self.ms = [np.zeros(nb, np.float32), np.zeros(nb, np.float32)]
        self.vs = [np.zeros(nb, np.float32), np.zeros(nb, np.float32)]
        self.lr = [np.asarray(lr_geo, np.float32), np.asarray(lr_app, np.float32)]
        self.b1, self.b2, self.eps = b1, b2, eps
        self.rb = float(restore_bound(b1, b2))
        self.sr_seed = int(sr_seed)
        self.col0 = [0, self.w[0].shape[1]]
        # keys: the Gaussian ids of the rows, which key the stochastic rounding
        # (a sample of whole 128-row blocks keeps FP8 block scales exact)
        self.keys = None if keys is None else np.ascontiguousarray(keys, np.uint32)
        if self.keys is not None:
            assert self.keys.shape[0] == geo.shape[0]
        # track_bound: carry the a-posteriori bound of |w - w64| (dense FP64
        # Adam on the same visible sets and gradients) per element
        self.bw = self.em = self.ev = None
        if track_bound:
            self.bw = [np.zeros(x.shape, np.float64) for x in self.w]
            self.em = [np.zeros(x.shape, np.float64) for x in self.w]
            self.ev = [np.zeros(x.shape, np.float64) for x in self.w]
        cs = adam_ratio_bound(b1, b2)
        self._trk = []
        for k in range(2):
            tr = _Track()
            tr.keys = None if self.keys is None else self.keys.ctypes.data
            if track_bound:
                tr.em, tr.ev, tr.bw = self.em[k].ctypes.data, self.ev[k].ctypes.data, self.bw[k].ctypes.data
            tr.cs = cs
            self._trk.append(tr)

    def moments_f32(self, k):
        """FP32 view of the stored moments of group k."""
        if self.sid[k] == 0:
            return self.m[k], self.v[k]
        if self.sid[k] == 2:
            blk = np.arange(self.m[k].shape[0]) // FP8_BLOCK
            # the second moment is stored as its square root
            return (e4m3_decode(self.m[k]) * self.ms[k][blk][:, None],
                    (e4m3_decode(self.v[k]) * self.vs[k][blk][:, None]) ** 2)
        conv = lambda a: (a.astype(np.uint32) << 16).view(np.float32)
        return conv(self.m[k]), conv(self.v[k])

    def _restore(self, k, t, rows):
        rows32 = np.ascontiguousarray(rows, np.uint32)
        d = np.ascontiguousarray(self.counter[np.asarray(rows, np.int64)], np.int64)
        if k == 0 and self.geo_dense:
            d = np.zeros_like(d)
        Wf, _, _, _, _ = lut_spec(self.b1, self.b2, t, max(self.dmax(t), 0), self.sched)
        dim = self.w[k].shape[1]
        out = np.zeros((rows32.shape[0], dim), np.float32)
        if self.sid[k] == 2:
            lib().orc_restore_rows_fp8(dim, _p(self.w[k]), _p(self.m[k]), _p(self.v[k]), _p(self.ms[k]),
                                       _p(self.vs[k]), dim, rows32.shape[0], _p(rows32), _p(d), _p(self.lr[k]),
                                       self.eps, _p(Wf), self.rb, _p(out))
            return out
        lib().orc_restore_rows_f32(dim, _p(self.w[k]), _p(self.m[k]), _p(self.v[k]), self.sid[k], dim,
                                   rows32.shape[0], _p(rows32), _p(d), _p(self.lr[k]), self.eps,
                                   _p(Wf), self.rb, _p(out))
        return out

    def current(self, t: int, rows=None):
        """FP32 restored (geo, app) of rows (default all) before update t."""
        rows = np.arange(self.counter.shape[0]) if rows is None else np.asarray(rows)
        return self._restore(0, t, rows), self._restore(1, t, rows)

    def current_geo(self, t: int):
        return self._restore(0, t, np.arange(self.counter.shape[0]))

    def cull_current(self, t: int, cam):
        """valid_ids (local row indices, ascending) of the current geometry."""
        return compact(cull(self.current_geo(t), cam))

    def step(self, t, valid, g_geo, g_app):
        valid, sat = self.update_set(valid)
        rows = np.ascontiguousarray(np.concatenate([valid, sat]), np.uint32)
        d = np.ascontiguousarray(self.counter[rows.astype(np.int64)], np.int64)
        Wf, Mf, Vf, ss, bc = lut_spec(self.b1, self.b2, t, max(self.dmax(t), 0), self.sched)
        for k, g in enumerate((g_geo, g_app)):
            dim = self.w[k].shape[1]
            if k == 0 and self.geo_dense:
                krows = np.arange(self.counter.shape[0], dtype=np.uint32)
                kd = np.zeros(krows.shape[0], np.int64)
                gg = np.zeros((krows.shape[0], dim), np.float32)
                gg[valid] = g
            else:
                krows, kd = rows, d
                gg = np.zeros((rows.shape[0], dim), np.float32)
                gg[:valid.shape[0]] = g
            if self.sid[k] == 2:
                lib().orc_deferred_rows_fp8(dim, _p(self.w[k]), _p(self.m[k]), _p(self.v[k]), _p(self.ms[k]),
                                            _p(self.vs[k]), dim, self.w[k].shape[0], krows.shape[0], _p(krows),
                                            _p(kd), _p(gg), dim, _p(self.lr[k]), self.b1, self.b2, self.eps,
                                            _p(Wf), _p(Mf), _p(Vf), float(ss), float(bc), self.rb,
                                            self.sr_seed, t, self.col0[k], C.byref(self._trk[k]))
                continue
            lib().orc_deferred_rows_f32(dim, _p(self.w[k]), _p(self.m[k]), _p(self.v[k]), self.sid[k], dim,
                                        krows.shape[0], _p(krows), _p(kd), _p(gg), dim, _p(self.lr[k]),
                                        self.b1, self.b2, self.eps, _p(Wf), _p(Mf), _p(Vf),
                                        float(ss), float(bc), self.rb, self.sr_seed, t, self.col0[k],
                                        C.byref(self._trk[k]))
        self.bump(valid, sat)
        return valid, sat

    def flush(self, t_done: int):
        rows = np.nonzero(self.counter > 0)[0]
        if rows.shape[0] == 0:
            return
        delta = np.ascontiguousarray(self.counter[rows], np.int64)
        # table of step t_done+1 at index delta <= t_done; Mf/Vf do not depend on t
        Wn, Mf, Vf, _, _ = lut_spec(self.b1, self.b2, t_done + 1, int(delta.max()), self.sched)
        rows32 = np.ascontiguousarray(rows, np.uint32)
        for k in range(2):
            if k == 0 and self.geo_dense:
                continue
            dim = self.w[k].shape[1]
            if self.sid[k] == 2:
                lib().orc_flush_rows_fp8(dim, _p(self.w[k]), _p(self.m[k]), _p(self.v[k]), _p(self.ms[k]),
                                         _p(self.vs[k]), dim, rows.shape[0], _p(rows32), _p(delta),
                                         _p(self.lr[k]), self.eps, _p(Wn), _p(Mf), _p(Vf), self.rb,
                                         self.sr_seed, t_done, self.col0[k], self.b2, C.byref(self._trk[k]))
                continue
            lib().orc_flush_rows_f32(dim, _p(self.w[k]), _p(self.m[k]), _p(self.v[k]), self.sid[k], dim,
                                     rows.shape[0], _p(rows32), _p(delta), _p(self.lr[k]), self.eps,
                                     _p(Wn), _p(Mf), _p(Vf), self.rb, self.sr_seed, t_done, self.col0[k],
                                     self.b2, C.byref(self._trk[k]))
        self.counter[:] = 0


# ---------------------------------------------------------------------------
# SGD with momentum (the momentum-optimizer extension of Sec. 4.3)
# ---------------------------------------------------------------------------
def lut_sgdm(mu: float, t: int, dmax: int, sched=None):
    """FP64 (Ws, Mf) of update t: Ws[d] = sum_{i=1..d} s_{t-i} mu^(d+1-i), Mf[d] = mu^(d+1)."""
    W = np.zeros(dmax + 1); M = np.zeros(dmax + 1)
    lib().orc_lut_sgdm_f64(mu, t, dmax, _p(_sched(sched)), _p(W), _p(M))
    return W, M


def lut_sgdm_spec(mu: float, t: int, dmax: int, sched=None):
    """The same tables rounded once to FP32, and the step multiplier s_t."""
    Wf = np.zeros(dmax + 1, np.float32); Mf = np.zeros(dmax + 1, np.float32)
    ss = C.c_float()
    lib().orc_lut_sgdm_spec(mu, t, dmax, _p(_sched(sched)), _p(Wf), _p(Mf), C.addressof(ss))
    return Wf, Mf, np.float32(ss.value)


class DenseSGDMF64:
    """FP64 SGD with momentum on every row every step (g = 0 without a gradient)."""

    def __init__(self, geo, app, lr_geo, lr_app, mu=0.9, sched=None):
        self.w = [np.array(geo, np.float64), np.array(app, np.float64)]
        self.m = [np.zeros_like(x) for x in self.w]
        self.lr = [np.asarray(lr_geo, np.float64), np.asarray(lr_app, np.float64)]
        self.mu = mu
        self.sched = _sched(sched)

    def step(self, t, ids, g_geo, g_app):
        ids = np.ascontiguousarray(ids, np.uint32)
        s = 1.0 if self.sched is None else float(self.sched[t])
        for k, g in enumerate((g_geo, g_app)):
            g = np.ascontiguousarray(g, np.float32)
            lib().orc_sgdm_dense_sparse_grad_f64(self.w[k].shape[0], self.w[k].shape[1], _p(self.w[k]),
                                                 _p(self.m[k]), ids.shape[0], _p(ids), _p(g),
                                                 _p(self.lr[k]), self.mu, s)


class DeferredSGDMF64(_Deferred):
    """Deferred SGD with momentum in FP64, catch-up then step (paper order)."""

    def __init__(self, geo, app, lr_geo, lr_app, mu=0.9, max_defer=0, sched=None):
        super().__init__(geo.shape[0], max_defer)
        self.w = [np.array(geo, np.float64), np.array(app, np.float64)]
        self.m = [np.zeros_like(x) for x in self.w]
        self.lr = [np.asarray(lr_geo, np.float64), np.asarray(lr_app, np.float64)]
        self.mu = mu
        self.sched = _sched(sched)

    def step(self, t, valid, g_geo, g_app):
        valid, sat = self.update_set(valid)
        rows = np.ascontiguousarray(np.concatenate([valid, sat]), np.uint32)
        d = np.ascontiguousarray(self.counter[rows.astype(np.int64)], np.int64)
        W, M = lut_sgdm(self.mu, t, max(self.dmax(t), 0), self.sched)
        s_t = 1.0 if self.sched is None else float(self.sched[t])
        for k, g in enumerate((g_geo, g_app)):
            dim = self.w[k].shape[1]
            gg = np.zeros((rows.shape[0], dim))
            gg[:valid.shape[0]] = np.asarray(g, np.float64)
            lib().orc_sgdm_deferred_rows_f64(dim, _p(self.w[k]), _p(self.m[k]), rows.shape[0], _p(rows), _p(d),
                                             _p(gg), _p(self.lr[k]), s_t, _p(W), _p(M))
        self.bump(valid, sat)
        return valid, sat

    def flush(self, t_done):
        rows = np.nonzero(self.counter > 0)[0]
        if rows.shape[0] == 0:
            return
        delta = np.ascontiguousarray(self.counter[rows], np.int64)
        W, _ = lut_sgdm(self.mu, t_done + 1, int(delta.max()), self.sched)
        rows32 = np.ascontiguousarray(rows, np.uint32)
        for k in range(2):
            lib().orc_sgdm_flush_rows_f64(self.w[k].shape[1], _p(self.w[k]), _p(self.m[k]), rows.shape[0],
                                          _p(rows32), _p(delta), _p(self.lr[k]), _p(W), self.mu)
        self.counter[:] = 0


class DeferredSGDMF32(_Deferred):
    """Deferred SGD with momentum with FP32 math and the implementation's op
    order; the momentum buffer stored FP32 or BF16 (stochastic rounding with
    the same random stream as the Adam models)."""

    def __init__(self, geo, app, lr_geo, lr_app, mu=0.9, max_defer=0, state="f32", app_state=None,
                 sr_seed=0, sched=None):
        super().__init__(geo.shape[0], max_defer)
        states = [state, app_state or state]
        assert all(x in ("f32", "bf16") for x in states)
        self.sid = [STATES[x][0] for x in states]
        self.w = [np.array(geo, np.float32), np.array(app, np.float32)]
        self.m = [np.zeros(x.shape, STATES[st][1]) for x, st in zip(self.w, states)]
        self.lr = [np.asarray(lr_geo, np.float32), np.asarray(lr_app, np.float32)]
        self.mu = mu
        self.sched = _sched(sched)
        self.sr_seed = int(sr_seed)
        self.col0 = [0, self.w[0].shape[1]]

    def _restore(self, k, t, rows):
        rows32 = np.ascontiguousarray(rows, np.uint32)
        d = np.ascontiguousarray(self.counter[np.asarray(rows, np.int64)], np.int64)
        Wf, _, _ = lut_sgdm_spec(self.mu, t, max(self.dmax(t), 0), self.sched)
        dim = self.w[k].shape[1]
        out = np.zeros((rows32.shape[0], dim), np.float32)
        lib().orc_sgdm_restore_rows_f32(dim, _p(self.w[k]), _p(self.m[k]), self.sid[k], dim, rows32.shape[0],
                                        _p(rows32), _p(d), _p(self.lr[k]), _p(Wf), _p(out))
        return out

    def current(self, t, rows=None):
        rows = np.arange(self.counter.shape[0]) if rows is None else np.asarray(rows)
        return self._restore(0, t, rows), self._restore(1, t, rows)

    def cull_current(self, t, cam):
        return compact(cull(self._restore(0, t, np.arange(self.counter.shape[0])), cam))

    def step(self, t, valid, g_geo, g_app):
        valid, sat = self.update_set(valid)
        rows = np.ascontiguousarray(np.concatenate([valid, sat]), np.uint32)
        d = np.ascontiguousarray(self.counter[rows.astype(np.int64)], np.int64)
        Wf, Mf, ss = lut_sgdm_spec(self.mu, t, max(self.dmax(t), 0), self.sched)
        for k, g in enumerate((g_geo, g_app)):
            dim = self.w[k].shape[1]
            gg = np.zeros((rows.shape[0], dim), np.float32)
            gg[:valid.shape[0]] = g
            lib().orc_sgdm_rows_f32(dim, _p(self.w[k]), _p(self.m[k]), self.sid[k], dim, rows.shape[0], _p(rows),
                                    _p(d), _p(gg), dim, _p(self.lr[k]), _p(Wf), _p(Mf), float(ss), self.sr_seed,
                                    t, self.col0[k])
        self.bump(valid, sat)
        return valid, sat

    def flush(self, t_done):
        rows = np.nonzero(self.counter > 0)[0]
        if rows.shape[0] == 0:
            return
        delta = np.ascontiguousarray(self.counter[rows], np.int64)
        Wn, Mf, _ = lut_sgdm_spec(self.mu, t_done + 1, int(delta.max()), self.sched)
        rows32 = np.ascontiguousarray(rows, np.uint32)
        for k in range(2):
            dim = self.w[k].shape[1]
            lib().orc_sgdm_flush_rows_f32(dim, _p(self.w[k]), _p(self.m[k]), self.sid[k], dim, rows.shape[0],
                                          _p(rows32), _p(delta), _p(self.lr[k]), _p(Wn), _p(Mf), self.sr_seed,
                                          t_done, self.col0[k])
        self.counter[:] = 0


# ---------------------------------------------------------------------------
# AdamW (decoupled weight decay, the other optimizer named in Sec. 4.3)
# ---------------------------------------------------------------------------
def lut_adamw(b1, b2, lam, lr, t, dmax, sched=None):
    """FP64 (Wl, P) of update t for one column rate (paper form)."""
    W = np.zeros(dmax + 1); P = np.zeros(dmax + 1)
    lib().orc_lut_adamw_f64(b1, b2, lam, float(lr), t, dmax, _p(_sched(sched)), _p(W), _p(P))
    return W, P


def lut_adamw_spec(b1, b2, lam, lr, t, dmax, sched=None):
    """FP32 (Wf, Pf, q_t) of update t for one FP32 column rate."""
    Wf = np.zeros(dmax + 1, np.float32); Pf = np.zeros(dmax + 1, np.float32)
    q = C.c_float()
    lib().orc_lut_adamw_spec(b1, b2, lam, float(lr), t, dmax, _p(_sched(sched)), _p(Wf), _p(Pf), C.addressof(q))
    return Wf, Pf, np.float32(q.value)


def _col_tables(fn, lr, *args):
    """Per-column tables [dim, dmax+1] (one table per distinct rate)."""
    cache, W, P, Q = {}, [], [], []
    for r in np.asarray(lr).tolist():
        if r not in cache:
            cache[r] = fn(*args[:3], r, *args[3:])
        w_, p_, *q_ = cache[r]
        W.append(w_); P.append(p_); Q.append(q_[0] if q_ else 0.0)
    return np.ascontiguousarray(np.stack(W)), np.ascontiguousarray(np.stack(P)), np.asarray(Q, np.float32)


class DenseAdamWF64:
    """FP64 AdamW on every row every step: w *= 1 - lr_t lambda, then Adam."""

    def __init__(self, geo, app, lr_geo, lr_app, b1=0.9, b2=0.999, eps=1e-15, weight_decay=0.01, sched=None):
        self.w = [np.array(geo, np.float64), np.array(app, np.float64)]
        self.m = [np.zeros_like(x) for x in self.w]
        self.v = [np.zeros_like(x) for x in self.w]
        self.lr = [np.asarray(lr_geo, np.float64), np.asarray(lr_app, np.float64)]
        self.b1, self.b2, self.eps, self.lam = b1, b2, eps, weight_decay
        self.sched = _sched(sched)

    def step(self, t, ids, g_geo, g_app):
        ids = np.ascontiguousarray(ids, np.uint32)
        s = 1.0 if self.sched is None else float(self.sched[t])
        for k, g in enumerate((g_geo, g_app)):
            g = np.ascontiguousarray(g, np.float32)
            lr = np.ascontiguousarray(self.lr[k] * s)
            lib().orc_adamw_dense_sparse_grad_f64(self.w[k].shape[0], self.w[k].shape[1], _p(self.w[k]),
                                                  _p(self.m[k]), _p(self.v[k]), ids.shape[0], _p(ids), _p(g),
                                                  _p(lr), self.b1, self.b2, self.eps, self.lam, t)


class DeferredAdamWF64(_Deferred):
    """Deferred AdamW in FP64 (paper order, paper-form tables)."""

    def __init__(self, geo, app, lr_geo, lr_app, b1=0.9, b2=0.999, eps=1e-15, weight_decay=0.01, max_defer=0,
                 sched=None):
        super().__init__(geo.shape[0], max_defer)
        self.w = [np.array(geo, np.float64), np.array(app, np.float64)]
        self.m = [np.zeros_like(x) for x in self.w]
        self.v = [np.zeros_like(x) for x in self.w]
        self.lr = [np.asarray(lr_geo, np.float64), np.asarray(lr_app, np.float64)]
        self.b1, self.b2, self.eps, self.lam = b1, b2, eps, weight_decay
        self.sched = _sched(sched)

    def _tabs(self, k, t, dmax):
        return _col_tables(lut_adamw, self.lr[k], self.b1, self.b2, self.lam, t, dmax, self.sched)

    def step(self, t, valid, g_geo, g_app):
        valid, sat = self.update_set(valid)
        rows = np.ascontiguousarray(np.concatenate([valid, sat]), np.uint32)
        d = np.ascontiguousarray(self.counter[rows.astype(np.int64)], np.int64)
        dmax = max(self.dmax(t), 0)
        _, m_dec, v_dec = restore_coeff(self.b1, self.b2, t, dmax, self.sched)
        s_t = 1.0 if self.sched is None else float(self.sched[t])
        for k, g in enumerate((g_geo, g_app)):
            dim = self.w[k].shape[1]
            W, P, _ = self._tabs(k, t, dmax)
            gg = np.zeros((rows.shape[0], dim))
            gg[:valid.shape[0]] = np.asarray(g, np.float64)
            lib().orc_adamw_deferred_rows_f64(dim, _p(self.w[k]), _p(self.m[k]), _p(self.v[k]), rows.shape[0],
                                              _p(rows), _p(d), _p(gg), _p(self.lr[k]), self.b1, self.b2, self.eps,
                                              t, s_t, self.lam, _p(W), _p(P), dmax + 1, _p(m_dec), _p(v_dec))
        self.bump(valid, sat)
        return valid, sat

    def flush(self, t_done):
        rows = np.nonzero(self.counter > 0)[0]
        if rows.shape[0] == 0:
            return
        delta = np.ascontiguousarray(self.counter[rows], np.int64)
        dm = int(delta.max())
        rows32 = np.ascontiguousarray(rows, np.uint32)
        for k in range(2):
            W, P, _ = self._tabs(k, t_done + 1, dm)
            lib().orc_adamw_flush_rows_f64(self.w[k].shape[1], _p(self.w[k]), _p(self.m[k]), _p(self.v[k]),
                                           rows.shape[0], _p(rows32), _p(delta), _p(self.lr[k]), self.b1, self.b2,
                                           self.eps, _p(W), _p(P), dm + 1)
        self.counter[:] = 0


class DeferredAdamWF32(_Deferred):
    """Deferred AdamW with FP32 math in the implementation's op order;
    moments FP32 or BF16 (stochastic rounding as the Adam models)."""

    def __init__(self, geo, app, lr_geo, lr_app, b1=0.9, b2=0.999, eps=1e-15, weight_decay=0.01, max_defer=0,
                 state="f32", app_state=None, sr_seed=0, sched=None):
        super().__init__(geo.shape[0], max_defer)
        states = [state, app_state or state]
        assert all(x in ("f32", "bf16") for x in states)
        self.sid = [STATES[x][0] for x in states]
        self.w = [np.array(geo, np.float32), np.array(app, np.float32)]
        self.m = [np.zeros(x.shape, STATES[st][1]) for x, st in zip(self.w, states)]
        self.v = [np.zeros(x.shape, STATES[st][1]) for x, st in zip(self.w, states)]
        self.lr = [np.asarray(lr_geo, np.float32), np.asarray(lr_app, np.float32)]
        self.b1, self.b2, self.eps, self.lam = b1, b2, eps, weight_decay
        self.rb = float(restore_bound(b1, b2))
        self.sched = _sched(sched)
        self.sr_seed = int(sr_seed)
        self.col0 = [0, self.w[0].shape[1]]

    def _tabs(self, k, t, dmax):
        return _col_tables(lut_adamw_spec, self.lr[k], self.b1, self.b2, self.lam, t, dmax, self.sched)

    def _restore(self, k, t, rows):
        rows32 = np.ascontiguousarray(rows, np.uint32)
        d = np.ascontiguousarray(self.counter[np.asarray(rows, np.int64)], np.int64)
        dmax = max(self.dmax(t), 0)
        W, P, _ = self._tabs(k, t, dmax)
        dim = self.w[k].shape[1]
        out = np.zeros((rows32.shape[0], dim), np.float32)
        lib().orc_adamw_restore_rows_f32(dim, _p(self.w[k]), _p(self.m[k]), _p(self.v[k]), self.sid[k], dim,
                                         rows32.shape[0], _p(rows32), _p(d), _p(self.lr[k]), self.eps, _p(W), _p(P),
                                         dmax + 1, self.rb, _p(out))
        return out

    def current(self, t, rows=None):
        rows = np.arange(self.counter.shape[0]) if rows is None else np.asarray(rows)
        return self._restore(0, t, rows), self._restore(1, t, rows)

    def cull_current(self, t, cam):
        return compact(cull(self._restore(0, t, np.arange(self.counter.shape[0])), cam))

    def step(self, t, valid, g_geo, g_app):
        valid, sat = self.update_set(valid)
        rows = np.ascontiguousarray(np.concatenate([valid, sat]), np.uint32)
        d = np.ascontiguousarray(self.counter[rows.astype(np.int64)], np.int64)
        dmax = max(self.dmax(t), 0)
        _, Mf, Vf, ss, bc = lut_spec(self.b1, self.b2, t, dmax, self.sched)
        for k, g in enumerate((g_geo, g_app)):
            dim = self.w[k].shape[1]
            W, P, Q = self._tabs(k, t, dmax)
            gg = np.zeros((rows.shape[0], dim), np.float32)
            gg[:valid.shape[0]] = g
            lib().orc_adamw_rows_f32(dim, _p(self.w[k]), _p(self.m[k]), _p(self.v[k]), self.sid[k], dim,
                                     rows.shape[0], _p(rows), _p(d), _p(gg), dim, _p(self.lr[k]), self.b1, self.b2,
                                     self.eps, _p(W), _p(P), dmax + 1, _p(Q), _p(Mf), _p(Vf), float(ss), float(bc),
                                     self.rb, self.sr_seed, t, self.col0[k])
        self.bump(valid, sat)
        return valid, sat

    def flush(self, t_done):
        rows = np.nonzero(self.counter > 0)[0]
        if rows.shape[0] == 0:
            return
        delta = np.ascontiguousarray(self.counter[rows], np.int64)
        dm = int(delta.max())
        _, Mf, Vf, _, _ = lut_spec(self.b1, self.b2, t_done + 1, dm, self.sched)
        rows32 = np.ascontiguousarray(rows, np.uint32)
        for k in range(2):
            dim = self.w[k].shape[1]
            W, P, _ = self._tabs(k, t_done + 1, dm)
            lib().orc_adamw_flush_rows_f32(dim, _p(self.w[k]), _p(self.m[k]), _p(self.v[k]), self.sid[k], dim,
                                           rows.shape[0], _p(rows32), _p(delta), _p(self.lr[k]), self.eps, _p(W),
                                           _p(P), dm + 1, _p(Mf), _p(Vf), self.rb, self.sr_seed, t_done, self.col0[k])
        self.counter[:] = 0


# ---------------------------------------------------------------------------
# densification (Sec. 2.4 step 7, the 3DGS procedure)
# ---------------------------------------------------------------------------
def densify_thresholds(percent_dense, extent, min_opacity):
    """FP32 (log_dense, log_big, logit_min, log_split) from FP64 logs."""
    out = np.zeros(4, np.float32)
    lib().orc_densify_thresholds(percent_dense, extent, min_opacity, _p(out))
    return out


def densify(geo, app, accum, denom, radii=None, grad_thr=2e-4, percent_dense=0.01, extent=100.0,
            min_opacity=0.005, prune_big=True, max_screen=0.0, seed=0):
    """Densify current FP32 rows.  Returns (geo_out, app_out, src, kind, counts):
    src = source row, kind 0 original, 1 clone, 2/3 split child 0/1."""
    geo = np.ascontiguousarray(geo, np.float32)
    app = np.ascontiguousarray(app, np.float32)
    n, adim = geo.shape[0], app.shape[1]
    # the library takes these parameters as FP32 values
    percent_dense, extent, min_opacity = (float(np.float32(x)) for x in (percent_dense, extent, min_opacity))
    th = densify_thresholds(percent_dense, extent, min_opacity)
    cap = 3 * n + 1
    og = np.zeros((cap, 10), np.float32); oa = np.zeros((cap, adim), np.float32)
    src = np.zeros(cap, np.int64); kind = np.zeros(cap, np.uint8); counts = np.zeros(3, np.int64)
    rad = None if radii is None else np.ascontiguousarray(radii, np.float32)
    m = lib().orc_densify(n, adim, _p(geo), _p(app), _p(np.ascontiguousarray(accum, np.float32)),
                          _p(np.ascontiguousarray(denom, np.float32)), _p(rad), np.float32(grad_thr), float(th[0]),
                          int(prune_big), float(th[1]), float(th[2]), np.float32(max_screen), float(th[3]),
                          int(seed), cap, _p(og), _p(oa), _p(src), _p(kind), _p(counts))
    return og[:m], oa[:m], src[:m], kind[:m], counts


def simulate(models, scene_geo_rows_keys, cams_for_step, grads_for, steps, t0=1):
    """Drive O3 (and optionally O2 / dense) through `steps` updates.

    models: dict with 'f32' (DeferredF32, required), optional 'f64', 'dense'.
    scene_geo_rows_keys: Gaussian ids of the simulated rows (for gradients).
    grads_for(t, keys) -> (g_geo, g_app) FP32 compact gradients.
    Returns the list of per-step valid (local) id arrays of O3.
    """
    keys = np.asarray(scene_geo_rows_keys)
    history = []
    for t in range(t0, t0 + steps):
        o3 = models["f32"]
        valid = o3.cull_current(t, cams_for_step(t))
        g_geo, g_app = grads_for(t, keys[valid])
        o3.step(t, valid, g_geo, g_app)
        if "f64" in models:
            models["f64"].step(t, valid, g_geo, g_app)
        if "dense" in models:
            models["dense"].step(t, valid, g_geo, g_app)
        history.append(valid)
    return history


if __name__ == "__main__":
    print(build(force=True), file=sys.stderr)


# ---------------------------------------------------------------------------
# batched form: several scenes (row ranges), several cameras per scene
# ---------------------------------------------------------------------------
def cull_multi(geo_current: np.ndarray, scene_row0, cams_per_scene):
    """Union and per-camera lists of a batch, from the FP32 cull of each row
    of scene s against each camera of scene s.
    Returns (union_ids ascending, [cam_pos[c]] union positions ascending,
    scene_start [S, 1+C])."""
    n = geo_current.shape[0]
    row0 = np.asarray(scene_row0, np.int64)
    S = row0.shape[0] - 1
    Cc = len(cams_per_scene[0])
    masks = np.zeros(n, np.uint64)
    for s in range(S):
        a, b = int(row0[s]), int(row0[s + 1])
        for c, cam in enumerate(cams_per_scene[s]):
            keep = cull(geo_current[a:b], cam)
            masks[a:b] |= keep.astype(np.uint64) << np.uint64(c)
    union = np.nonzero(masks)[0]
    pos_of = np.full(n, -1, np.int64)
    pos_of[union] = np.arange(union.shape[0])
    cam_rows = [np.nonzero((masks >> np.uint64(c)) & np.uint64(1))[0] for c in range(Cc)]
    cam_pos = [pos_of[r] for r in cam_rows]
    start = np.zeros((S, 1 + Cc), np.int64)
    for s in range(S):
        start[s, 0] = np.searchsorted(union, row0[s])
        for c in range(Cc):
            start[s, 1 + c] = np.searchsorted(cam_rows[c], row0[s])
    return union, cam_pos, start


def grad_sum_multi(cam_pos, g_cam, n_union: int) -> np.ndarray:
    """out[p] = sum over cameras c in order of the gradient of the entry of
    camera c at union position p (FP32 additions starting from 0)."""
    D = g_cam[0].shape[1]
    out = np.zeros((n_union, D), np.float32)
    for c, pos in enumerate(cam_pos):
        out[pos] = out[pos] + np.asarray(g_cam[c], np.float32)
    return out


# ---------------------------------------------------------------------------
# balance-aware image split (Sec. 4.4)
# ---------------------------------------------------------------------------
def crop_camera(cam, x0: int, x1: int) -> np.ndarray:
    """The camera of image columns [x0, x1): same rotation, translation and
    focal lengths, principal point moved left by x0, width x1 - x0 (as the 20
    floats the cull takes)."""
    f = cam_floats(cam).copy()
    f[14] = np.float32(f[14] - np.float32(x0))
    f[16] = np.float32(x1 - x0)
    return f


def image_split_plan(geo_current: np.ndarray, cam, mem_limit: float, search_steps: int = 5):
    """Where to split an image whose visible set is too large (Sec. 4.4; the
    paper gives the idea, not the search): no split (x = 0) when at most
    mem_limit * n rows are visible; otherwise start at the middle column and
    move toward the side with fewer visible rows by halving, search_steps
    times.  Returns (x, (visible in the whole image, left crop, right crop))."""
    n = geo_current.shape[0]
    width = int(cam_floats(cam)[16])
    full = int(cull(geo_current, cam).sum())
    if full <= mem_limit * n:
        return 0, (full, 0, 0)

    def sides(x):
        left = int(cull(geo_current, crop_camera(cam, 0, x)).sum())
        right = int(cull(geo_current, crop_camera(cam, x, width)).sum())
        return left, right

    lo, hi, x = 1, width - 1, width // 2
    for _ in range(search_steps):
        left, right = sides(x)
        if left > right:
            hi = x
        else:
            lo = x
        x = (lo + hi) // 2
    left, right = sides(x)
    return x, (full, left, right)
