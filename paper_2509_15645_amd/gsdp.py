"""Thin ctypes binding of libgsdp (argument marshalling only).

Every step of the path runs in the HIP kernels of ``libgsdp.so``; this module
only turns torch tensors into device pointers and the current HIP stream into
a stream handle, and raises when the library reports an error.  If the
library has not been built the import of this module fails: there is no
fallback implementation.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np
import torch

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "libgsdp.so")

GS_OK, GS_EINVAL, GS_EHIP, GS_EUNSUPPORTED, GS_ESPACE = 0, -1, -2, -3, -4
GS_F32, GS_BF16, GS_FP8E4M3 = 0, 1, 2
GS_OPT_ADAM, GS_OPT_ADAMW, GS_OPT_SGD_MOMENTUM = 0, 1, 2
GS_CHUNK_ROWS = 1024

# exported C symbols (kept in sync with include/gsdp.h)
SYMBOLS = ("gs_lut_bytes", "gs_lut_build", "gs_lut_build_host", "gs_lut_build_schedule",
           "gs_lut_build_schedule_host", "gs_workspace_bytes", "gs_cull",
           "gs_gather", "gs_scatter_grad", "gs_adam_step_deferred", "gs_adam_flush", "gs_synth_grad",
           "gs_device_cu_count", "gs_status_string", "gs_last_hip_error", "gs_step_advance", "gs_stream_read_probe",
           "gs_camera_pack_bytes", "gs_camera_pack", "gs_multi_workspace_bytes", "gs_cull_multi",
           "gs_cull_multi_autotune", "gs_grad_sum_multi", "gs_plan_image_split", "gs_lut_build_sgd_momentum",
           "gs_lut_build_sgd_momentum_host", "gs_lut_bytes_adamw", "gs_lut_build_adamw", "gs_lut_build_adamw_host",
           "gs_densify_workspace_bytes", "gs_densify_plan", "gs_densify_apply", "gs_cull_noalloc",
           "gs_lut_seek", "gs_lut_seek_host", "gs_cull_summary_build", "gs_cull_table", "gs_row_probe",
           "gs_cull_chunk_flags")


class GsCamera(C.Structure):
    _fields_ = [("R", C.c_float * 9), ("t", C.c_float * 3), ("fx", C.c_float), ("fy", C.c_float),
                ("cx", C.c_float), ("cy", C.c_float), ("width", C.c_int32), ("height", C.c_int32),
                ("near_plane", C.c_float), ("far_plane", C.c_float)]


class GsGroup(C.Structure):
    _fields_ = [("w", C.c_void_p), ("m", C.c_void_p), ("v", C.c_void_p), ("dim", C.c_int32),
                ("w_ld", C.c_int32), ("m_ld", C.c_int32), ("v_ld", C.c_int32), ("state", C.c_int32),
                ("pad_", C.c_int32), ("m_scale", C.c_void_p), ("v_scale", C.c_void_p),
                ("lr", C.c_float * 64)]


class GsModel(C.Structure):
    _fields_ = [("n", C.c_int64), ("geo", GsGroup), ("app", GsGroup), ("last_step", C.c_void_p),
                ("lut", C.c_void_p), ("lut_max_steps", C.c_int32), ("max_defer", C.c_int32),
                ("beta1", C.c_double), ("beta2", C.c_double), ("eps", C.c_double),
                ("cull_mode", C.c_int32), ("geo_mode", C.c_int32), ("sr_seed", C.c_uint64),
                ("step_dev", C.c_void_p), ("optimizer", C.c_int32), ("reserved_", C.c_int32),
                ("cull_sum", C.c_void_p), ("cull_chunk", C.c_void_p)]


class GsMulti(C.Structure):
    _fields_ = [("n_scenes", C.c_int32), ("cams_per_scene", C.c_int32), ("n_sets", C.c_int32),
                ("variant", C.c_int32), ("scene_row0", C.c_void_p), ("cams", C.c_void_p),
                ("union_ids", C.c_void_p), ("union_count", C.c_void_p), ("cam_pos", C.c_void_p),
                ("cam_count", C.c_void_p), ("cap_union", C.c_uint32), ("cap_cam", C.c_uint32),
                ("scene_start", C.c_void_p), ("chunk_start", C.c_void_p)]


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is not built; run __graft_entry__.build() (hipcc, gfx950)")
    L = C.CDLL(LIB_PATH)
    vp, i32, i64, u32, u64, f64, sz = (C.c_void_p, C.c_int32, C.c_int64, C.c_uint32, C.c_uint64,
                                       C.c_double, C.c_size_t)
    P = C.POINTER
    sig = {
        "gs_lut_bytes": (C.c_int, [i32, i32, P(sz)]),
        "gs_lut_build": (C.c_int, [f64, f64, i32, i32, vp, sz]),
        "gs_lut_build_host": (C.c_int, [f64, f64, i32, i32, vp, sz]),
        "gs_lut_seek": (C.c_int, [P(GsModel), i64, vp]),
        "gs_lut_seek_host": (C.c_int, [vp, sz, i64]),
        "gs_lut_build_schedule": (C.c_int, [f64, f64, i32, i32, vp, vp, sz]),
        "gs_lut_build_schedule_host": (C.c_int, [f64, f64, i32, i32, vp, vp, sz]),
        "gs_lut_build_sgd_momentum": (C.c_int, [f64, i32, i32, vp, vp, sz]),
        "gs_lut_build_sgd_momentum_host": (C.c_int, [f64, i32, i32, vp, vp, sz]),
        "gs_lut_bytes_adamw": (C.c_int, [P(GsModel), P(sz)]),
        "gs_lut_build_adamw": (C.c_int, [P(GsModel), f64, vp, vp, sz]),
        "gs_lut_build_adamw_host": (C.c_int, [P(GsModel), f64, vp, vp, sz]),
        "gs_workspace_bytes": (C.c_int, [P(GsModel), P(sz)]),
        "gs_densify_workspace_bytes": (C.c_int, [P(GsModel), P(sz)]),
        "gs_densify_plan": (C.c_int, [P(GsModel), vp, vp, vp, vp, vp, sz, vp, P(C.c_int64), vp]),
        "gs_densify_apply": (C.c_int, [P(GsModel), vp, P(GsModel), i64, vp, sz, vp]),
        "gs_cull": (C.c_int, [P(GsModel), P(GsCamera), i64, vp, vp, u32, vp, sz, vp]),
        "gs_cull_noalloc": (C.c_int, [P(GsModel), P(GsCamera), i64, vp, vp, u32, vp]),
        "gs_cull_summary_build": (C.c_int, [P(GsModel), vp]),
        "gs_cull_chunk_flags": (C.c_int, [P(GsModel), P(GsCamera), i64, vp, vp]),
        "gs_cull_table": (C.c_int, [P(GsModel), vp, i32, i64, vp, vp, u32, vp, sz, vp]),
        "gs_row_probe": (C.c_int, [vp, u32, vp, u64, u32, i32, vp, vp]),
        "gs_gather": (C.c_int, [P(GsModel), i64, vp, vp, u32, vp, vp, vp]),
        "gs_scatter_grad": (C.c_int, [vp, vp, u32, i32, vp, vp, i32, vp]),
        "gs_adam_step_deferred": (C.c_int, [P(GsModel), i64, vp, vp, u32, vp, vp, vp, vp, vp, sz, vp]),
        "gs_adam_flush": (C.c_int, [P(GsModel), i64, vp]),
        "gs_synth_grad": (C.c_int, [u64, i64, vp, vp, u32, i32, i32, f64, vp, vp]),
        "gs_device_cu_count": (C.c_int, []),
        "gs_step_advance": (C.c_int, [vp, vp]),
        "gs_stream_read_probe": (C.c_int, [vp, C.c_size_t, vp, vp]),
        "gs_camera_pack_bytes": (C.c_int, [P(sz)]),
        "gs_camera_pack": (C.c_int, [P(GsModel), vp, i32, vp]),
        "gs_multi_workspace_bytes": (C.c_int, [P(GsModel), P(sz)]),
        "gs_cull_multi": (C.c_int, [P(GsModel), P(GsMulti), i64, vp, sz, vp]),
        "gs_cull_multi_autotune": (C.c_int, [P(GsModel), P(GsMulti), i64, vp, sz, vp, vp, P(i32)]),
        "gs_grad_sum_multi": (C.c_int, [P(GsMulti), i32, vp, vp, vp, vp]),
        "gs_plan_image_split": (C.c_int, [P(GsModel), P(GsCamera), i64, f64, P(GsMulti), vp, sz, vp, P(i32), vp]),
        "gs_status_string": (C.c_char_p, [C.c_int]),
        "gs_last_hip_error": (C.c_char_p, []),
    }
    for name, (res, args) in sig.items():
        fn = getattr(L, name)
        fn.restype = res
        fn.argtypes = args
    return L


lib = _load()


class GsError(RuntimeError):
    pass


def _check(rc: int, what: str):
    if rc != GS_OK:
        msg = lib.gs_status_string(rc).decode()
        if rc == GS_EHIP:
            msg += ": " + lib.gs_last_hip_error().decode()
        raise GsError(f"{what}: {msg}")


def _ptr(t):
    return None if t is None else C.c_void_p(t.data_ptr())


def _stream(stream):
    if stream is None:
        stream = torch.cuda.current_stream()
    return C.c_void_p(stream.cuda_stream)


def camera_struct(cam) -> GsCamera:
    """gs_camera from an object with R, t, fx, fy, cx, cy, width, height, near, far."""
    c = GsCamera()
    R = np.asarray(cam.R, np.float32).ravel()
    t = np.asarray(cam.t, np.float32).ravel()
    for i in range(9):
        c.R[i] = float(R[i])
    for i in range(3):
        c.t[i] = float(t[i])
    c.fx, c.fy, c.cx, c.cy = float(cam.fx), float(cam.fy), float(cam.cx), float(cam.cy)
    c.width, c.height = int(cam.width), int(cam.height)
    c.near_plane, c.far_plane = float(cam.near), float(cam.far)
    return c


# ---------------------------------------------------------------------------
# tables and workspace
# ---------------------------------------------------------------------------
def gs_lut_bytes(max_steps: int, max_defer: int) -> int:
    b = C.c_size_t()
    _check(lib.gs_lut_bytes(max_steps, max_defer, C.byref(b)), "gs_lut_bytes")
    return b.value


def gs_lut_build(beta1, beta2, max_steps, max_defer, lut: torch.Tensor):
    _check(lib.gs_lut_build(beta1, beta2, max_steps, max_defer, _ptr(lut), lut.numel() * lut.element_size()),
           "gs_lut_build")


def _host_image(nbytes: int) -> np.ndarray:
    """A zeroed, 8-byte aligned host buffer of nbytes bytes (uint8 view)."""
    return np.zeros((nbytes + 7) // 8, np.float64).view(np.uint8)[:nbytes]


def gs_lut_build_host(beta1, beta2, max_steps, max_defer, lr_scale=None) -> np.ndarray:
    """Host image (uint8) of the tables at step 1."""
    nbytes = gs_lut_bytes(max_steps, max_defer)
    out = _host_image(nbytes)
    sc = None if lr_scale is None else np.ascontiguousarray(lr_scale, np.float64)
    _check(lib.gs_lut_build_schedule_host(beta1, beta2, max_steps, max_defer,
                                          None if sc is None else sc.ctypes.data, out.ctypes.data, nbytes),
           "gs_lut_build_host")
    return out


def gs_lut_seek_host(img: np.ndarray, step: int):
    """Advance a host image of the tables (in place) to `step`."""
    _check(lib.gs_lut_seek_host(img.ctypes.data, img.nbytes, int(step)), "gs_lut_seek_host")


def gs_lut_seek(model, step: int, stream=None):
    _check(lib.gs_lut_seek(C.byref(model.c), int(step), _stream(stream)), "gs_lut_seek")


def gs_lut_build_schedule(beta1, beta2, max_steps, max_defer, lr_scale, lut: torch.Tensor):
    sc = np.ascontiguousarray(lr_scale, np.float64)
    assert sc.shape[0] >= max_steps + 2
    _check(lib.gs_lut_build_schedule(beta1, beta2, max_steps, max_defer, sc.ctypes.data, _ptr(lut),
                                     lut.numel() * lut.element_size()), "gs_lut_build_schedule")


def gs_lut_build_sgd_momentum(momentum, max_steps, max_defer, lr_scale, lut: torch.Tensor):
    sc = None if lr_scale is None else np.ascontiguousarray(lr_scale, np.float64)
    assert sc is None or sc.shape[0] >= max_steps + 2
    _check(lib.gs_lut_build_sgd_momentum(momentum, max_steps, max_defer, None if sc is None else sc.ctypes.data,
                                         _ptr(lut), lut.numel() * lut.element_size()), "gs_lut_build_sgd_momentum")


def gs_lut_build_sgd_momentum_host(momentum, max_steps, max_defer, lr_scale=None) -> np.ndarray:
    nbytes = gs_lut_bytes(max_steps, max_defer)
    out = _host_image(nbytes)
    sc = None if lr_scale is None else np.ascontiguousarray(lr_scale, np.float64)
    _check(lib.gs_lut_build_sgd_momentum_host(momentum, max_steps, max_defer,
                                              None if sc is None else sc.ctypes.data, out.ctypes.data, nbytes),
           "gs_lut_build_sgd_momentum_host")
    return out


def gs_workspace_bytes(model) -> int:
    b = C.c_size_t()
    _check(lib.gs_workspace_bytes(C.byref(model.c), C.byref(b)), "gs_workspace_bytes")
    return b.value


# ---------------------------------------------------------------------------
# model state (device memory owned by torch)
# ---------------------------------------------------------------------------
class Model:
    """Device-resident parameters, Adam moments, per-row last step, tables and
    workspace of one set of Gaussians, plus the gs_model struct describing them.

    geo_state / app_state: "f32" or "bf16" storage of the Adam moments.
    app_layout "separate": w, m, v of A are three [n, dim] tensors.
               "interleaved": one byte row per Gaussian holding w | m | v
               (padded to a multiple of 64 bytes), so the random row accesses of
               gather and Adam touch one contiguous span.
    """

    def __init__(self, geo, app, lr_geo, lr_app, *, beta1=0.9, beta2=0.999, eps=1e-15, max_defer=0,
                 max_steps=1000, cull_mode=0, app_layout="separate", geo_state="f32", app_state="f32",
                 sr_seed=0, geo_mode=0, lr_scale=None, optimizer="adam", weight_decay=0.0, device=None,
                 cull_summary=None, cull_chunks=False):
        device = device or torch.device("cuda")
        # constructor settings, reused by densify() for the resized model
        self._kw = dict(beta1=beta1, beta2=beta2, eps=eps, max_defer=max_defer, max_steps=max_steps,
                        cull_mode=cull_mode, app_layout=app_layout, geo_state=geo_state, app_state=app_state,
                        sr_seed=sr_seed, geo_mode=geo_mode, lr_scale=lr_scale, optimizer=optimizer,
                        weight_decay=weight_decay, device=device, cull_summary=cull_summary,
                        cull_chunks=cull_chunks)
        geo = torch.as_tensor(geo, dtype=torch.float32)
        app = torch.as_tensor(app, dtype=torch.float32)
        n, adim = geo.shape[0], app.shape[1]
        assert geo.shape == (n, 10) and app.shape[0] == n
        self.n, self.adim, self.device = n, adim, device
        sdt = {"f32": (torch.float32, GS_F32, 4), "bf16": (torch.bfloat16, GS_BF16, 2),
               "fp8": (torch.uint8, GS_FP8E4M3, 1)}
        gdt, gcode, _ = sdt[geo_state]
        adt, acode, asz = sdt[app_state]
        self.geo_state, self.app_state = geo_state, app_state
        _, _, gsz = sdt[geo_state]
        self.geo_w = geo.to(device).contiguous()
        self.app_layout = app_layout
        gld = (10, 10, 10)
        if app_layout != "fused":
            self.geo_m = torch.zeros((n, 10), dtype=gdt, device=device)
            self.geo_v = torch.zeros((n, 10), dtype=gdt, device=device)
        if app_layout == "fused":
            # one byte row per Gaussian: A w | G m, A m | G v, A v, padded to 64 bytes,
            # so a visible row's state is a single contiguous span and each moment
            # of all 10 + dim columns is one run (lane c of a row kernel at c)
            wbytes, mbytes, gbytes = 4 * adim, asz * adim, gsz * 10
            o_gm = wbytes
            o_am = o_gm + gbytes
            o_gv = o_am + mbytes
            o_gv = (o_gv + gsz - 1) // gsz * gsz
            o_av = o_gv + gbytes
            row = (o_av + mbytes + 63) // 64 * 64
            assert row % 4 == 0 and row % asz == 0 and row % gsz == 0
            self.app_state_bytes = torch.zeros((n, row), dtype=torch.uint8, device=device)
            st = self.app_state_bytes
            self.app_w = st[:, 0:wbytes].view(torch.float32)
            self.app_m = st[:, o_am:o_am + mbytes].view(adt)
            self.app_v = st[:, o_av:o_av + mbytes].view(adt)
            self.geo_m = st[:, o_gm:o_gm + gbytes].view(gdt)
            self.geo_v = st[:, o_gv:o_gv + gbytes].view(gdt)
            self.app_w.copy_(app.to(device))
            ld = (row // 4, row // asz, row // asz)
            gld = (10, row // gsz, row // gsz)
        elif app_layout == "separate":
            self.app_w = app.to(device).contiguous()
            self.app_m = torch.zeros((n, adim), dtype=adt, device=device)
            self.app_v = torch.zeros((n, adim), dtype=adt, device=device)
            ld = (adim, adim, adim)
        elif app_layout == "interleaved":
            wbytes, mbytes = 4 * adim, asz * adim
            row = (wbytes + 2 * mbytes + 63) // 64 * 64
            self.app_state_bytes = torch.zeros((n, row), dtype=torch.uint8, device=device)
            st = self.app_state_bytes
            self.app_w = st[:, 0:wbytes].view(torch.float32)
            self.app_m = st[:, wbytes:wbytes + mbytes].view(adt)
            self.app_v = st[:, wbytes + mbytes:wbytes + 2 * mbytes].view(adt)
            self.app_w.copy_(app.to(device))
            ld = (row // 4, row // asz, row // asz)
        else:
            raise ValueError(app_layout)
        nb = (n + 127) // 128
        zs = lambda code: torch.zeros(nb, dtype=torch.float32, device=device) if code == GS_FP8E4M3 else None
        self.geo_ms, self.geo_vs = zs(gcode), zs(gcode)
        self.app_ms, self.app_vs = zs(acode), zs(acode)
        self.last_step = torch.zeros(n, dtype=torch.int32, device=device)
        self.max_steps, self.max_defer = int(max_steps), int(max_defer)
        self.optimizer = optimizer
        if optimizer not in ("adam", "adamw", "sgd_momentum"):
            raise ValueError(optimizer)
        self.lr_geo = np.asarray(lr_geo, np.float32)
        self.lr_app = np.asarray(lr_app, np.float32)

        c = GsModel()
        c.n = n
        for grp, w, m, v, lds, lr, dim, code, ms, vs in (
                (c.geo, self.geo_w, self.geo_m, self.geo_v, gld, self.lr_geo, 10, gcode,
                 self.geo_ms, self.geo_vs),
                (c.app, self.app_w, self.app_m, self.app_v, ld, self.lr_app, adim, acode,
                 self.app_ms, self.app_vs)):
            grp.w, grp.m, grp.v = w.data_ptr(), m.data_ptr(), v.data_ptr()
            grp.m_scale = ms.data_ptr() if ms is not None else None
            grp.v_scale = vs.data_ptr() if vs is not None else None
            grp.dim = dim
            grp.w_ld, grp.m_ld, grp.v_ld = lds
            grp.state = code
            for k in range(dim):
                grp.lr[k] = float(lr[k])
        c.last_step = self.last_step.data_ptr()
        c.lut_max_steps = self.max_steps
        c.max_defer = self.max_defer
        c.beta1, c.beta2, c.eps = float(beta1), float(beta2), float(eps)
        c.cull_mode = int(cull_mode)
        c.sr_seed = int(sr_seed)
        c.geo_mode = int(geo_mode)
        c.optimizer = {"adam": GS_OPT_ADAM, "adamw": GS_OPT_ADAMW, "sgd_momentum": GS_OPT_SGD_MOMENTUM}[optimizer]
        if optimizer == "adamw":
            b = C.c_size_t()
            _check(lib.gs_lut_bytes_adamw(C.byref(c), C.byref(b)), "gs_lut_bytes_adamw")
            self.lut = torch.empty(b.value // 4, dtype=torch.float32, device=device)
            sc = None if lr_scale is None else np.ascontiguousarray(lr_scale, np.float64)
            _check(lib.gs_lut_build_adamw(C.byref(c), float(weight_decay), None if sc is None else sc.ctypes.data,
                                          _ptr(self.lut), b.value), "gs_lut_build_adamw")
        else:
            self.lut = torch.empty(gs_lut_bytes(self.max_steps, self.max_defer) // 4, dtype=torch.float32,
                                   device=device)
            if optimizer == "sgd_momentum":
                # beta1 is the momentum; the v buffers are allocated but unused
                gs_lut_build_sgd_momentum(beta1, self.max_steps, self.max_defer, lr_scale, self.lut)
            elif lr_scale is None:
                gs_lut_build(beta1, beta2, self.max_steps, self.max_defer, self.lut)
            else:
                gs_lut_build_schedule(beta1, beta2, self.max_steps, self.max_defer, lr_scale, self.lut)
        c.lut = self.lut.data_ptr()
        # device step counter for graph replay (calls with step == 0 read it)
        self.step_dev = torch.zeros(1, dtype=torch.int32, device=device)
        c.step_dev = self.step_dev.data_ptr()
        # cull summaries (16 bytes a row, read by the band cull instead of the
        # 40-byte geometry rows): by default wherever the band cull runs
        if cull_summary is None:
            cull_summary = cull_mode == 1 and geo_mode == 0 and optimizer == "adam"
        self.cull_sum = None
        if cull_summary:
            self.cull_sum = torch.empty((max(n, 1), 4), dtype=torch.float32, device=device)
            c.cull_sum = self.cull_sum.data_ptr()
        # their chunk records (32 bytes per GS_CHUNK_ROWS rows): worth it when
        # the rows are in a spatial order (the cull then skips most chunks);
        # with rows in no order every chunk's box spans the scene
        self.cull_chunk = None
        if cull_chunks and self.cull_sum is not None:
            self.cull_chunk = torch.empty((max((n + GS_CHUNK_ROWS - 1) // GS_CHUNK_ROWS, 1), 8),
                                          dtype=torch.float32, device=device)
            c.cull_chunk = self.cull_chunk.data_ptr()
        self.c = c
        self.ws = torch.zeros(gs_workspace_bytes(self) // 4, dtype=torch.int32, device=device)
        if self.cull_sum is not None:
            self.cull_summary_build()

    def cull_summary_build(self, stream=None):
        """Recompute every row's cull summary from geo_w (and the chunk
        records from the summaries): needed after geo_w is written other than
        by this library's calls (which keep them current)."""
        _check(lib.gs_cull_summary_build(C.byref(self.c), _stream(stream)), "gs_cull_summary_build")

    @property
    def ws_bytes(self) -> int:
        return self.ws.numel() * 4

    def ws_header(self) -> dict:
        """Diagnostic counters of the workspace; "error" is the tables' error
        word (bit 0: a call's step was not the one the tables held; bit 1: a
        step outside [1, max_steps])."""
        h = self.ws[:8].cpu().numpy().view(np.uint32)
        q = h[4:8].view(np.uint64)
        return {"vis_total": int(h[0]), "sat_total": int(h[1]), "restored_last": int(h[2]),
                "error": int(h[3]) | self.lut_header()["error"],
                "vis_accum": int(q[0]), "restored_accum": int(q[1])}

    def lut_header(self) -> dict:
        """The tables' header: the step each row slot holds and the error word."""
        h = self.lut[:16].view(torch.int32).cpu().numpy()
        return {"t_row": (int(h[0]), int(h[1])), "T": int(h[2]), "K": int(h[3]), "nclass": int(h[4]),
                "error": int(h[5]), "kind": int(h[6])}

    def lut_seek(self, step: int):
        """Move the tables forward to `step` (to start a model at a later step)."""
        gs_lut_seek(self, step)

    def state(self):
        """Host copies: geo/app w (float32), m, v (float32 or raw uint16 BF16 bits) and last_step."""
        out = {}
        for name in ("geo_w", "geo_m", "geo_v", "app_w", "app_m", "app_v"):
            t = getattr(self, name).contiguous()
            if t.dtype == torch.bfloat16:
                out[name] = t.view(torch.int16).cpu().numpy().view(np.uint16)
            else:
                out[name] = t.cpu().numpy()
        out["last_step"] = self.last_step.cpu().numpy()
        for name in ("geo_ms", "geo_vs", "app_ms", "app_vs"):
            t = getattr(self, name)
            if t is not None:
                out[name] = t.cpu().numpy()
        return out

    def load_state(self, st, step=None):
        """Write host arrays in the form state() returns (any subset) into the
        model, recompute the cull summaries, and with `step` move the tables to
        that update step (a model resumed after a flush at step - 1)."""
        for name, a in st.items():
            t = getattr(self, name)
            src = torch.from_numpy(np.ascontiguousarray(a))
            if t.dtype == torch.bfloat16:
                src = src.view(torch.int16).view(torch.bfloat16)
            t.copy_(src.to(t.device).view(t.shape))
        if self.cull_sum is not None:
            self.cull_summary_build()
        if step is not None:
            self.lut_seek(step)


# ---------------------------------------------------------------------------
# the path (same names as the C ABI)
# ---------------------------------------------------------------------------
def gs_cull(model: Model, cam, step: int, ids: torch.Tensor, count: torch.Tensor, capacity=None, stream=None):
    cap = ids.numel() if capacity is None else int(capacity)
    camc = cam if isinstance(cam, GsCamera) else camera_struct(cam)
    _check(lib.gs_cull(C.byref(model.c), C.byref(camc), int(step), _ptr(ids), _ptr(count), cap,
                       _ptr(model.ws), model.ws_bytes, _stream(stream)), "gs_cull")


def gs_cull_noalloc(model: Model, cam, step: int, ids: torch.Tensor, count: torch.Tensor, capacity=None,
                    stream=None):
    cap = ids.numel() if capacity is None else int(capacity)
    camc = cam if isinstance(cam, GsCamera) else camera_struct(cam)
    _check(lib.gs_cull_noalloc(C.byref(model.c), C.byref(camc), int(step), _ptr(ids), _ptr(count), cap,
                               _stream(stream)), "gs_cull_noalloc")


def gs_cull_chunk_flags(model: Model, cam, step: int, flags: torch.Tensor, stream=None):
    """flags (uint8, one per chunk of GS_CHUNK_ROWS rows) = 1 where the summary
    cull skips the chunk for this camera."""
    camc = cam if isinstance(cam, GsCamera) else camera_struct(cam)
    _check(lib.gs_cull_chunk_flags(C.byref(model.c), C.byref(camc), int(step), _ptr(flags), _stream(stream)),
           "gs_cull_chunk_flags")


def camera_table(model: Model, cams):
    """Device table of camera records (gs_camera_pack) for gs_cull_table."""
    rb = C.c_size_t()
    _check(lib.gs_camera_pack_bytes(C.byref(rb)), "gs_camera_pack_bytes")
    flat = (GsCamera * len(cams))()
    for i, cam in enumerate(cams):
        flat[i] = cam if isinstance(cam, GsCamera) else camera_struct(cam)
    recs = np.zeros(len(cams) * rb.value, np.uint8)
    _check(lib.gs_camera_pack(C.byref(model.c), flat, len(cams), recs.ctypes.data), "gs_camera_pack")
    return torch.from_numpy(recs).to(model.device)


def gs_cull_table(model: Model, table, step: int, ids: torch.Tensor, count: torch.Tensor, capacity=None,
                  stream=None):
    """gs_cull with camera (t - 1) % len of a camera_table (step 0: the model's
    device step counter)."""
    cap = ids.numel() if capacity is None else int(capacity)
    rb = C.c_size_t()
    _check(lib.gs_camera_pack_bytes(C.byref(rb)), "gs_camera_pack_bytes")
    _check(lib.gs_cull_table(C.byref(model.c), _ptr(table), table.numel() // rb.value, int(step), _ptr(ids),
                             _ptr(count), cap, _ptr(model.ws), model.ws_bytes, _stream(stream)), "gs_cull_table")


def gs_gather(model: Model, step: int, ids, count, out_geo, out_app, capacity=None, stream=None):
    cap = ids.numel() if capacity is None else int(capacity)
    _check(lib.gs_gather(C.byref(model.c), int(step), _ptr(ids), _ptr(count), cap, _ptr(out_geo),
                         _ptr(out_app), _stream(stream)), "gs_gather")


def gs_scatter_grad(ids, count, g_compact, g_dense, accumulate=False, capacity=None, stream=None):
    cap = ids.numel() if capacity is None else int(capacity)
    dim = g_compact.shape[1]
    _check(lib.gs_scatter_grad(_ptr(ids), _ptr(count), cap, dim, _ptr(g_compact), _ptr(g_dense),
                               1 if accumulate else 0, _stream(stream)), "gs_scatter_grad")


def gs_adam_step_deferred(model: Model, step: int, ids, count, g_geo=None, g_app=None, g_geo_dense=None,
                          g_app_dense=None, capacity=None, stream=None):
    cap = ids.numel() if capacity is None else int(capacity)
    _check(lib.gs_adam_step_deferred(C.byref(model.c), int(step), _ptr(ids), _ptr(count), cap, _ptr(g_geo),
                                     _ptr(g_app), _ptr(g_geo_dense), _ptr(g_app_dense), _ptr(model.ws),
                                     model.ws_bytes, _stream(stream)), "gs_adam_step_deferred")


def gs_adam_flush(model: Model, step: int, stream=None):
    _check(lib.gs_adam_flush(C.byref(model.c), int(step), _stream(stream)), "gs_adam_flush")


def gs_synth_grad(seed: int, step: int, ids, count, out, col0: int, sigma=1e-3, capacity=None, stream=None):
    cap = out.shape[0] if capacity is None else int(capacity)
    _check(lib.gs_synth_grad(int(seed), int(step), _ptr(ids), _ptr(count), cap, out.shape[1], int(col0),
                             float(sigma), _ptr(out), _stream(stream)), "gs_synth_grad")


# ---------------------------------------------------------------------------
# densification
# ---------------------------------------------------------------------------
class GsDensifyParams(C.Structure):
    _fields_ = [("grad_threshold", C.c_float), ("percent_dense", C.c_float), ("scene_extent", C.c_float),
                ("min_opacity", C.c_float), ("max_screen_size", C.c_float), ("prune_big", C.c_int32),
                ("seed", C.c_uint64)]


def densify(model: Model, step: int, grad_accum, grad_denom, max_radii2d=None, *, grad_threshold=2e-4,
            percent_dense=0.01, scene_extent=1.0, min_opacity=0.005, max_screen_size=0.0, prune_big=True,
            seed=0, stream=None):
    """Clone / split / prune the rows of a flushed `model` (gs_adam_flush at
    `step` first) into a new Model of the planned size with the same
    settings.  Returns (new_model, counts[originals, clones, children])."""
    p = GsDensifyParams(grad_threshold, percent_dense, scene_extent, min_opacity, max_screen_size,
                        int(bool(prune_big)), int(seed))
    b = C.c_size_t()
    _check(lib.gs_densify_workspace_bytes(C.byref(model.c), C.byref(b)), "gs_densify_workspace_bytes")
    ws = torch.zeros(max(b.value // 4, 64), dtype=torch.int32, device=model.device)
    n_out = C.c_int64()
    counts = (C.c_int64 * 3)()
    _check(lib.gs_densify_plan(C.byref(model.c), _ptr(grad_accum), _ptr(grad_denom), _ptr(max_radii2d),
                               C.byref(p), _ptr(ws), ws.numel() * 4, _stream(stream), C.byref(n_out), counts),
           "gs_densify_plan")
    n = int(n_out.value)
    dev = model.device
    new = Model(torch.zeros((n, 10), dtype=torch.float32, device=dev),
                torch.zeros((n, model.adim), dtype=torch.float32, device=dev), model.lr_geo, model.lr_app,
                **model._kw)
    _check(lib.gs_densify_apply(C.byref(model.c), C.byref(p), C.byref(new.c), int(step), _ptr(ws), ws.numel() * 4,
                                _stream(stream)), "gs_densify_apply")
    # the resized model continues at the next update: it takes over the tables
    new.lut.copy_(model.lut)
    return new, [int(x) for x in counts]


def gs_step_advance(step_dev, stream=None):
    _check(lib.gs_step_advance(_ptr(step_dev), _stream(stream)), "gs_step_advance")


def gs_row_probe(ids, count: int, rows, write: bool, sink, stream=None):
    """Load (and with write, store back unchanged) rows ids[0..count) of the
    2-D tensor `rows` (measurement helper)."""
    _check(lib.gs_row_probe(_ptr(ids), int(count), _ptr(rows), rows.shape[0], rows.shape[1] * rows.element_size(),
                            int(bool(write)), _ptr(sink), _stream(stream)), "gs_row_probe")


def gs_stream_read_probe(buf, sink, stream=None):
    """One streaming read of the whole tensor `buf` (measurement helper)."""
    _check(lib.gs_stream_read_probe(_ptr(buf), buf.numel() * buf.element_size(), _ptr(sink), _stream(stream)),
           "gs_stream_read_probe")


def gs_device_cu_count() -> int:
    return int(lib.gs_device_cu_count())


# ---------------------------------------------------------------------------
# batched form
# ---------------------------------------------------------------------------
MULTI_ALIGN = 1024


class Multi:
    """Device buffers of the batched cull of one model whose scenes are row
    ranges [scene_row0[s], scene_row0[s+1]) (multiples of 1024).
    camera_sets[k][s][c] is camera slot c of scene s in set k; update t uses
    set (t-1) % len(camera_sets)."""

    def __init__(self, model: Model, scene_row0, camera_sets, cap_union=None, cap_cam=None, variant=0):
        dev = model.device
        row0 = np.asarray(scene_row0, np.int64)
        assert np.all(row0[:-1] % MULTI_ALIGN == 0) and row0[-1] == model.n
        S = row0.shape[0] - 1
        n_sets = len(camera_sets)
        Cc = len(camera_sets[0][0])
        self.S, self.C, self.n_sets = S, Cc, n_sets
        self.cap_union = int(cap_union or model.n)
        self.cap_cam = int(cap_cam or model.n)
        self.scene_row0 = torch.from_numpy(row0).to(dev)
        rb = C.c_size_t()
        _check(lib.gs_camera_pack_bytes(C.byref(rb)), "gs_camera_pack_bytes")
        recs = np.zeros(n_sets * S * Cc * rb.value, np.uint8)
        flat = (GsCamera * (n_sets * S * Cc))()
        i = 0
        for k in range(n_sets):
            for sc in range(S):
                assert len(camera_sets[k][sc]) == Cc
                for cam in camera_sets[k][sc]:
                    flat[i] = camera_struct(cam)
                    i += 1
        _check(lib.gs_camera_pack(C.byref(model.c), flat, i, recs.ctypes.data), "gs_camera_pack")
        self.cams = torch.from_numpy(recs).to(dev)
        self.union_ids = torch.zeros(max(self.cap_union, 1), dtype=torch.int32, device=dev)
        self.union_count = torch.zeros(1, dtype=torch.int32, device=dev)
        self.cam_pos = torch.zeros((Cc, max(self.cap_cam, 1)), dtype=torch.int32, device=dev)
        self.cam_count = torch.zeros(Cc, dtype=torch.int32, device=dev)
        self.scene_start = torch.zeros((S, 1 + Cc), dtype=torch.int32, device=dev)
        self.chunk_start = torch.zeros(((max(self.cap_union, 1) + 127) // 128 + 1, Cc), dtype=torch.int32,
                                       device=dev)
        wb = C.c_size_t()
        _check(lib.gs_multi_workspace_bytes(C.byref(model.c), C.byref(wb)), "gs_multi_workspace_bytes")
        self.ws = torch.zeros((wb.value + 3) // 4, dtype=torch.int32, device=dev)
        d = GsMulti()
        d.n_scenes, d.cams_per_scene, d.n_sets, d.variant = S, Cc, n_sets, int(variant)
        d.scene_row0 = self.scene_row0.data_ptr()
        d.cams = self.cams.data_ptr()
        d.union_ids = self.union_ids.data_ptr()
        d.union_count = self.union_count.data_ptr()
        d.cam_pos = self.cam_pos.data_ptr()
        d.cam_count = self.cam_count.data_ptr()
        d.cap_union, d.cap_cam = self.cap_union, self.cap_cam
        d.scene_start = self.scene_start.data_ptr()
        d.chunk_start = self.chunk_start.data_ptr()
        self.c = d

    def lists(self):
        """Host copies: union ids, per-camera position lists, scene starts."""
        u = int(self.union_count.item())
        cc = self.cam_count.cpu().numpy()
        ids = self.union_ids[:min(u, self.cap_union)].cpu().numpy().view(np.uint32)
        pos = self.cam_pos.cpu().numpy().view(np.uint32)
        cams = [pos[c, :min(int(cc[c]), self.cap_cam)].copy() for c in range(self.C)]
        return u, ids, [int(x) for x in cc], cams, self.scene_start.cpu().numpy().view(np.uint32)


def gs_cull_multi(model: Model, multi: Multi, step: int, stream=None):
    _check(lib.gs_cull_multi(C.byref(model.c), C.byref(multi.c), int(step), _ptr(multi.ws), multi.ws.numel() * 4,
                             _stream(stream)), "gs_cull_multi")


def gs_cull_multi_autotune(model: Model, multi: Multi, step: int, stream=None):
    times = (C.c_float * 32)()
    nv = C.c_int32()
    _check(lib.gs_cull_multi_autotune(C.byref(model.c), C.byref(multi.c), int(step), _ptr(multi.ws),
                                      multi.ws.numel() * 4, _stream(stream), times, C.byref(nv)),
           "gs_cull_multi_autotune")
    return [times[i] for i in range(nv.value)]


def gs_grad_sum_multi(multi: Multi, adim: int, g_cam, out_geo, out_app, stream=None):
    _check(lib.gs_grad_sum_multi(C.byref(multi.c), int(adim), _ptr(g_cam), _ptr(out_geo), _ptr(out_app),
                                 _stream(stream)), "gs_grad_sum_multi")


def gs_plan_image_split(model: Model, cam, step: int, mem_limit: float, stream=None):
    """(split_x, (visible_full, visible_left, visible_right)); split_x = 0: no split."""
    multi = Multi(model, [0, model.n], [[[cam, cam]]], cap_union=0, cap_cam=0)
    x = C.c_int32()
    counts = (C.c_uint32 * 3)()
    _check(lib.gs_plan_image_split(C.byref(model.c), C.byref(camera_struct(cam)), int(step), float(mem_limit),
                                   C.byref(multi.c), _ptr(multi.ws), multi.ws.numel() * 4, _stream(stream),
                                   C.byref(x), counts), "gs_plan_image_split")
    return x.value, (counts[0], counts[1], counts[2])
