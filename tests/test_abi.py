"""The C ABI without a GPU: the library loads, exports every declared symbol,
rejects bad arguments before touching the device, and its host-built tables
equal the oracle's independently computed FP32 tables bit for bit."""
import ctypes as C
import os
import re
import shutil
import subprocess

import numpy as np
import pytest

import lut_layout as LL
from oracle import oracle as orc

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "gsdp.h")


@pytest.fixture(scope="module")
def gsdp():
    from paper_2509_15645_amd import build
    if not os.path.exists(build.LIB):
        build.build(force=True)
    from paper_2509_15645_amd import gsdp as g
    return g


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(gs_[a-z0-9_]+)\s*\(", text)))


def test_every_declared_symbol_is_exported(gsdp):
    names = declared_functions()
    assert len(names) >= 12
    lib = C.CDLL(gsdp.LIB_PATH)
    for n in names:
        assert hasattr(lib, n), n
    assert sorted(gsdp.SYMBOLS) == names


def test_struct_layouts(gsdp):
    assert C.sizeof(gsdp.GsCamera) == 80
    assert C.sizeof(gsdp.GsGroup) == 3 * 8 + 6 * 4 + 2 * 8 + 64 * 4
    assert gsdp.GsModel.lut_max_steps.offset == 8 + 2 * C.sizeof(gsdp.GsGroup) + 16


@pytest.mark.skipif(shutil.which("gcc") is None, reason="needs gcc")
def test_struct_layouts_match_the_c_header(gsdp, tmp_path):
    """Sizes and field offsets of the binding's structures equal those a C
    compiler gives the header's."""
    fields = {"gs_model": (gsdp.GsModel, ["n", "last_step", "lut", "lut_max_steps", "max_defer", "beta1",
                                          "cull_mode", "sr_seed", "step_dev", "optimizer", "cull_sum",
                                          "cull_chunk"]),
              "gs_group": (gsdp.GsGroup, ["w", "lr"]),
              "gs_camera": (gsdp.GsCamera, [])}
    src = ["#include <stdio.h>", "#include <stddef.h>", '#include "gsdp.h"', "int main(void) {"]
    for cname, (_, names) in fields.items():
        src.append(f'printf("{cname} %zu\\n", sizeof({cname}));')
        for f in names:
            src.append(f'printf("{cname}.{f} %zu\\n", offsetof({cname}, {f}));')
    src.append('printf("GS_CHUNK_ROWS %d\\n", GS_CHUNK_ROWS); return 0; }')
    c = tmp_path / "layout.c"
    c.write_text("\n".join(src) + "\n")
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-std=c11", "-I", os.path.join(ROOT, "include"), "-o", str(exe), str(c)], check=True)
    got = dict(line.split() for line in subprocess.run([str(exe)], capture_output=True, text=True,
                                                           check=True).stdout.splitlines())
    for cname, (cls, names) in fields.items():
        assert int(got[cname]) == C.sizeof(cls), cname
        for f in names:
            assert int(got[f"{cname}.{f}"]) == getattr(cls, f).offset, f"{cname}.{f}"
    assert int(got["GS_CHUNK_ROWS"]) == gsdp.GS_CHUNK_ROWS


def test_status_strings(gsdp):
    for code in (0, -1, -2, -3, -4):
        assert gsdp.lib.gs_status_string(code).decode().startswith("GS_")


def test_argument_checks_need_no_device(gsdp):
    L = gsdp.lib
    b = C.c_size_t()
    assert L.gs_lut_bytes(0, 0, C.byref(b)) == gsdp.GS_EINVAL
    assert L.gs_lut_bytes(10, -1, C.byref(b)) == gsdp.GS_EINVAL
    assert L.gs_lut_bytes(10, 0, C.byref(b)) == 0 and b.value > 0
    assert L.gs_cull(None, None, 1, None, None, 0, None, 0, None) == gsdp.GS_EINVAL
    m = gsdp.GsModel()
    m.n = 10
    assert L.gs_cull(C.byref(m), None, 1, None, None, 0, None, 0, None) == gsdp.GS_EINVAL
    assert L.gs_adam_flush(C.byref(m), 1, None) == gsdp.GS_EINVAL
    assert L.gs_workspace_bytes(None, C.byref(b)) == gsdp.GS_EINVAL
    m.max_defer = 0
    assert L.gs_workspace_bytes(C.byref(m), C.byref(b)) == 0 and b.value >= 256
    # a host buffer that is too small is reported, not overrun
    small = np.zeros(4, np.float32)
    assert L.gs_lut_build_host(0.9, 0.999, 10, 0, small.ctypes.data, 16) == gsdp.GS_ESPACE
    assert L.gs_lut_build_host(1.5, 0.999, 10, 0, small.ctypes.data, 16) == gsdp.GS_EINVAL


@pytest.mark.parametrize("max_defer", [0, 15])
def test_host_tables_equal_oracle_tables_bitwise(gsdp, max_defer):
    """The library's tables, advanced step by step from step 1 as the update
    calls advance them, against the oracle's independently computed FP32
    tables of each step; the size is O(max_steps + max_defer)."""
    T, K = 300, max_defer
    img = gsdp.gs_lut_build_host(0.9, 0.999, T, K)
    assert img.nbytes == LL.layout(T, K)["total"]
    v = LL.views(img, T, K)
    assert tuple(v["hdr"][:5]) == (0, 1, T, K, 0)
    for t in [1, 2, 3, 16, 17, 100, T, T + 1]:
        gsdp.gs_lut_seek_host(img, t)
        dmax = min(t - 1, K) if K else t - 1
        slot = t & 1
        assert v["hdr"][slot] == t and v["hdr"][5] == 0
        Wf, Mf, Vf, ss, bc = orc.lut_spec(0.9, 0.999, t, dmax)
        assert np.array_equal(v["Wf"][slot, :dmax + 1].view(np.uint32), Wf.view(np.uint32)), t
        assert np.array_equal(v["Mf"][:dmax + 1].view(np.uint32), Mf.view(np.uint32))
        assert np.array_equal(v["Vf"][:dmax + 1].view(np.uint32), Vf.view(np.uint32))
        assert v["SS"][t].view(np.uint32) == np.float32(ss).view(np.uint32)
        assert v["BC"][t].view(np.uint32) == np.float32(bc).view(np.uint32)
    # moving backwards or past T + 1 is refused
    with pytest.raises(RuntimeError):
        gsdp.gs_lut_seek_host(img, T)
    with pytest.raises(RuntimeError):
        gsdp.gs_lut_seek_host(img, T + 2)


def test_tables_of_a_long_run_are_small(gsdp):
    """30000 steps with unbounded deferral fit in about 1.7 MB."""
    b = C.c_size_t()
    assert gsdp.lib.gs_lut_bytes(30000, 0, C.byref(b)) == 0
    assert b.value == LL.layout(30000, 0)["total"] and b.value < 2_000_000
    assert gsdp.lib.gs_lut_bytes(30000, 15, C.byref(b)) == 0 and b.value < 600_000


def test_batched_entry_points_check_arguments(gsdp):
    L = gsdp.lib
    b = C.c_size_t()
    assert L.gs_camera_pack_bytes(C.byref(b)) == 0 and b.value == 256
    m = gsdp.GsModel()
    m.n = 5000
    assert L.gs_multi_workspace_bytes(C.byref(m), C.byref(b)) == 0
    assert b.value >= 256 + 8 * (5000 // 128)
    assert L.gs_cull_multi(None, None, 1, None, 0, None) == gsdp.GS_EINVAL
    assert L.gs_grad_sum_multi(None, 49, None, None, None, None) == gsdp.GS_EINVAL
    d = gsdp.GsMulti()
    d.cams_per_scene = 40                       # more than 32 camera slots
    buf = np.zeros(16, np.float32)
    assert L.gs_grad_sum_multi(C.byref(d), 49, buf.ctypes.data, buf.ctypes.data, buf.ctypes.data,
                               None) == gsdp.GS_EINVAL
    assert L.gs_step_advance(None, None) == gsdp.GS_EINVAL
    assert L.gs_plan_image_split(None, None, 1, 0.3, None, None, 0, None, None, None) == gsdp.GS_EINVAL
    cams = (gsdp.GsCamera * 2)()
    out = np.zeros(256, np.uint8)
    # fx = 0 is rejected before anything is written
    assert L.gs_camera_pack(C.byref(m), cams, 2, out.ctypes.data) == gsdp.GS_EINVAL


def test_camera_pack_layout(gsdp):
    """Packed camera records hold the camera and rounded-up band constants."""
    import gs_inputs as gi
    m = gsdp.GsModel()
    m.n = 10
    m.beta1, m.beta2 = 0.9, 0.999
    for k in range(10):
        m.geo.lr[k] = 1.6e-4 if k < 3 else 5e-3
    cam = gi.orbit_cameras(1, seed=3)[0]
    b = C.c_size_t()
    assert gsdp.lib.gs_camera_pack_bytes(C.byref(b)) == 0 and b.value == 256
    rec = np.zeros(b.value // 4, np.float32)
    assert gsdp.lib.gs_camera_pack(C.byref(m), C.byref(gsdp.camera_struct(cam)), 1, rec.ctypes.data) == 0
    assert np.array_equal(rec[:9], cam.R.ravel()) and np.array_equal(rec[9:12], cam.t)
    assert rec[12] == cam.fx and rec[16] == cam.width and rec[17] == cam.height
    rows = np.abs(cam.R.astype(np.float64)).sum(1)
    assert np.all(rec[20:23] >= rows) and np.all(rec[20:23] <= rows * (1 + 1e-5))
    rb = 1.03 * 0.1 / np.sqrt(0.001 * (1 - 0.81 / 0.999))
    assert rec[24] >= rb * 1.6e-4 and rec[25] >= rb * 5e-3 and rec[26] >= rb * 5e-3
    # side-test constants: the left plane fx R_0 + (cx + 3.93) R_2, fx T_0 + (cx + 3.93) T_2, and
    # ksig >= 3.003 sqrt(1.001 jf2)
    R, t = cam.R.astype(np.float64), cam.t.astype(np.float64)
    cl = cam.cx + 3.93
    assert np.allclose(rec[27:30], cam.fx * R[0] + cl * R[2], rtol=1e-6, atol=1e-3)
    assert np.isclose(rec[39], cam.fx * t[0] + cl * t[2], rtol=1e-6, atol=1e-3)
    assert rec[47] >= 3.003 * np.sqrt(1.001 * float(rec[23]))


@pytest.mark.parametrize("max_defer", [0, 15])
def test_host_schedule_tables_equal_oracle_tables_bitwise(gsdp, max_defer):
    T, K = 120, max_defer
    rng = np.random.default_rng(5)
    sc = 0.01 ** (np.arange(T + 2) / (T + 1)) * rng.uniform(0.5, 2.0, T + 2)
    img = gsdp.gs_lut_build_host(0.9, 0.999, T, K, lr_scale=sc)
    v = LL.views(img, T, K)
    for t in [1, 2, 17, 60, T, T + 1]:
        gsdp.gs_lut_seek_host(img, t)
        dmax = min(t - 1, K) if K else t - 1
        Wf, _, _, ss, _ = orc.lut_spec(0.9, 0.999, t, dmax, sc)
        assert np.array_equal(v["Wf"][t & 1, :dmax + 1].view(np.uint32), Wf.view(np.uint32)), t
        assert v["SS"][t].view(np.uint32) == np.float32(ss).view(np.uint32)


@pytest.mark.parametrize("max_defer,sched", [(0, False), (15, True)])
def test_host_sgd_momentum_tables_equal_oracle_bitwise(gsdp, max_defer, sched):
    T, mu, K = 90, 0.9, max_defer
    sc = None
    if sched:
        rng = np.random.default_rng(8)
        sc = 0.01 ** (np.arange(T + 2) / (T + 1)) * rng.uniform(0.5, 2.0, T + 2)
    img = gsdp.gs_lut_build_sgd_momentum_host(mu, T, K, lr_scale=sc)
    v = LL.views(img, T, K)
    assert v["hdr"][6] == 1
    for t in [1, 2, 16, 17, 50, T, T + 1]:
        gsdp.gs_lut_seek_host(img, t)
        dmax = min(t - 1, K) if K else t - 1
        Wf, Mf, ss = orc.lut_sgdm_spec(mu, t, dmax, sc)
        assert np.array_equal(v["Wf"][t & 1, :dmax + 1].view(np.uint32), Wf.view(np.uint32)), t
        assert np.array_equal(v["Mf"][:dmax + 1].view(np.uint32), Mf.view(np.uint32))
        assert v["SS"][t].view(np.uint32) == np.float32(ss).view(np.uint32)
    small = np.zeros(4, np.float64)
    assert gsdp.lib.gs_lut_build_sgd_momentum_host(1.0, 10, 0, None, small.ctypes.data, 32) == gsdp.GS_EINVAL


@pytest.mark.parametrize("max_defer,sched", [(0, False), (15, True)])
def test_host_adamw_tables_equal_oracle_bitwise(gsdp, max_defer, sched):
    import gs_inputs as gi
    T, lam = 70, 0.05
    lg, la = gi.lr_columns()
    m = gsdp.GsModel()
    m.n = 10
    m.geo.dim, m.app.dim = 10, 49
    for k in range(10):
        m.geo.lr[k] = float(lg[k])
    for k in range(49):
        m.app.lr[k] = float(la[k])
    m.lut_max_steps, m.max_defer = T, max_defer
    m.beta1, m.beta2 = 0.9, 0.999
    m.optimizer = gsdp.GS_OPT_ADAMW
    sc = None
    if sched:
        rng = np.random.default_rng(3)
        sc = 0.01 ** (np.arange(T + 2) / (T + 1)) * rng.uniform(0.5, 2.0, T + 2)
    b = C.c_size_t()
    assert gsdp.lib.gs_lut_bytes_adamw(C.byref(m), C.byref(b)) == 0
    K = max_defer
    rates = [np.float32(lg[0]), np.float32(lg[3])]          # classes in order of first appearance
    assert b.value == LL.layout(T, K, len(rates))["total"]
    out = np.zeros(b.value // 8, np.float64).view(np.uint8)
    scp = None if sc is None else np.ascontiguousarray(sc).ctypes.data
    assert gsdp.lib.gs_lut_build_adamw_host(C.byref(m), lam, scp, out.ctypes.data, b.value) == 0
    v = LL.views(out, T, K, len(rates))
    assert v["hdr"][4] == len(rates) and v["hdr"][6] == 2
    for t in [1, 2, 16, 17, 40, T, T + 1]:
        gsdp.gs_lut_seek_host(out, t)
        dmax = min(t - 1, K) if K else t - 1
        for c, r in enumerate(rates):
            Wf, Pf, qt = orc.lut_adamw_spec(0.9, 0.999, lam, r, t, dmax, sc)
            cv = v["cls"][c]
            assert np.array_equal(cv["Wlf"][t & 1, :dmax + 1].view(np.uint32), Wf.view(np.uint32)), (c, t)
            assert np.array_equal(cv["Pf"][t & 1, :dmax + 1].view(np.uint32), Pf.view(np.uint32)), (c, t)
            assert cv["qf"][t].view(np.uint32) == np.float32(qt).view(np.uint32)
    # too many distinct rates are rejected
    for k in range(10):
        m.geo.lr[k] = 1e-3 * (k + 1)
    assert gsdp.lib.gs_lut_bytes_adamw(C.byref(m), C.byref(b)) == gsdp.GS_EUNSUPPORTED


def _host_model(gsdp, n=8, state=0, opt=0):
    """A gs_model over host buffers, only for argument checks that return
    before any device work."""
    bufs = {k: np.zeros(n * 64, np.float32) for k in ("gw", "gm", "gv", "aw", "am", "av", "last", "lut", "sc")}
    m = gsdp.GsModel()
    m.n = n
    for grp, pre, dim in ((m.geo, "g", 10), (m.app, "a", 49)):
        grp.w, grp.m, grp.v = (bufs[pre + x].ctypes.data for x in "wmv")
        grp.dim = dim
        grp.w_ld = grp.m_ld = grp.v_ld = dim
        grp.state = state
        grp.m_scale = grp.v_scale = bufs["sc"].ctypes.data
        for k in range(dim):
            grp.lr[k] = 1e-3
    m.last_step = bufs["last"].ctypes.data
    m.lut = bufs["lut"].ctypes.data
    m.lut_max_steps = 8
    m.beta1, m.beta2, m.eps = 0.9, 0.999, 1e-15
    m.optimizer = opt
    return m, bufs


def test_densify_and_optimizer_checks_need_no_device(gsdp):
    L = gsdp.lib
    b = C.c_size_t()
    assert L.gs_densify_workspace_bytes(None, C.byref(b)) == gsdp.GS_EINVAL
    m, keep = _host_model(gsdp)
    assert L.gs_densify_workspace_bytes(C.byref(m), C.byref(b)) == 0 and b.value >= 256 + 8
    p = gsdp.GsDensifyParams(2e-4, 0.01, 10.0, 0.005, 0.0, 1, 0)
    n_out = C.c_int64()
    raw = np.zeros(2048, np.float32)
    ws = raw[(-raw.ctypes.data % 256) // 4:]            # 256-byte aligned view
    assert ws.ctypes.data % 256 == 0
    # missing parameters / statistics, bad parameters, unsupported FP8 state
    assert L.gs_densify_plan(C.byref(m), None, None, None, None, ws.ctypes.data, 4096, None, C.byref(n_out),
                             None) == gsdp.GS_EINVAL
    assert L.gs_densify_plan(C.byref(m), None, None, None, C.byref(p), ws.ctypes.data, 4096, None,
                             C.byref(n_out), None) == gsdp.GS_EINVAL
    bad = gsdp.GsDensifyParams(2e-4, 0.01, -1.0, 0.005, 0.0, 1, 0)
    acc = np.zeros(8, np.float32)
    assert L.gs_densify_plan(C.byref(m), acc.ctypes.data, acc.ctypes.data, None, C.byref(bad), ws.ctypes.data,
                             4096, None, C.byref(n_out), None) == gsdp.GS_EINVAL
    m8, keep8 = _host_model(gsdp, state=gsdp.GS_FP8E4M3)
    assert L.gs_densify_plan(C.byref(m8), acc.ctypes.data, acc.ctypes.data, None, C.byref(p), ws.ctypes.data,
                             4096, None, C.byref(n_out), None) == gsdp.GS_EUNSUPPORTED
    # optimizer extensions: FP8 state and the batched form are rejected
    for opt in (gsdp.GS_OPT_SGD_MOMENTUM, gsdp.GS_OPT_ADAMW):
        mo, keepo = _host_model(gsdp, state=gsdp.GS_FP8E4M3, opt=opt)
        assert L.gs_workspace_bytes(C.byref(mo), C.byref(b)) == 0
        assert L.gs_adam_flush(C.byref(mo), 1, None) == gsdp.GS_EUNSUPPORTED
    mu, keepu = _host_model(gsdp, opt=7)
    assert L.gs_adam_flush(C.byref(mu), 1, None) == gsdp.GS_EINVAL


def _fake_model(gsdp, n):
    """A model that passes the argument checks; its pointers are never
    dereferenced because every call below fails a check first."""
    m = gsdp.GsModel()
    m.n = n
    fake = 1 << 20
    for g, dim in ((m.geo, 10), (m.app, 49)):
        g.w = g.m = g.v = fake
        g.dim = g.w_ld = g.m_ld = g.v_ld = dim
        g.state = gsdp.GS_F32
    m.last_step = fake
    m.lut = fake
    m.lut_max_steps = 10
    m.beta1, m.beta2, m.eps = 0.9, 0.999, 1e-15
    return m


def test_cull_noalloc_checks_need_no_device(gsdp):
    L = gsdp.lib
    cam = gsdp.GsCamera()
    cam.fx = cam.fy = 1000.0
    cam.width, cam.height = 64, 64
    ids = C.c_void_p(1 << 20)
    m = _fake_model(gsdp, 1000)
    m.max_defer = 15
    assert L.gs_cull_noalloc(C.byref(m), C.byref(cam), 1, ids, ids, 16, None) == gsdp.GS_EUNSUPPORTED
    m.max_defer = 0
    m.geo_mode = 1
    assert L.gs_cull_noalloc(C.byref(m), C.byref(cam), 1, ids, ids, 16, None) == gsdp.GS_EUNSUPPORTED
    m.geo_mode = 0
    assert L.gs_cull_noalloc(C.byref(m), C.byref(cam), 11, ids, ids, 16, None) == gsdp.GS_EINVAL
    assert L.gs_cull_noalloc(C.byref(m), C.byref(cam), 1, ids, None, 16, None) == gsdp.GS_EINVAL
    # a model whose workspace exceeds the library's array is refused with a message
    big = _fake_model(gsdp, 0x7FFFFFFF)
    b = C.c_size_t()
    assert L.gs_workspace_bytes(C.byref(big), C.byref(b)) == 0 and b.value > (16 << 20)
    assert L.gs_cull_noalloc(C.byref(big), C.byref(cam), 1, ids, ids, 16, None) == gsdp.GS_ESPACE
    assert b"workspace" in L.gs_last_hip_error()


def test_cull_summary_checks_need_no_device(gsdp):
    """gs_cull_summary_build without summaries, misaligned summaries, and
    summaries with dense geometry are refused before anything is launched."""
    L = gsdp.lib
    m = _fake_model(gsdp, 1000)
    assert L.gs_cull_summary_build(C.byref(m), None) == gsdp.GS_EINVAL
    m.cull_sum = (1 << 20) + 4
    assert L.gs_cull_summary_build(C.byref(m), None) == gsdp.GS_EINVAL
    m.cull_sum = 1 << 20
    m.geo_mode = 1
    assert L.gs_cull_summary_build(C.byref(m), None) == gsdp.GS_EUNSUPPORTED
    m.geo_mode = 0
    # chunk records need summaries and 32-byte alignment
    m.cull_chunk = 1 << 21
    m.cull_sum = None
    assert L.gs_cull_summary_build(C.byref(m), None) == gsdp.GS_EINVAL
    m.cull_sum = 1 << 20
    m.cull_chunk = (1 << 21) + 16
    assert L.gs_cull_summary_build(C.byref(m), None) == gsdp.GS_EINVAL
    m.cull_chunk = None
    m.geo_mode = 1
    cam = gsdp.GsCamera()
    cam.fx = cam.fy = 1000.0
    cam.width, cam.height = 64, 64
    ids = C.c_void_p(1 << 20)
    assert L.gs_cull_noalloc(C.byref(m), C.byref(cam), 1, ids, ids, 16, None) == gsdp.GS_EUNSUPPORTED
    # chunk decisions: only where the summary cull runs with chunk records
    # (cull_mode 0 here, then no records, then a deferral limit); missing
    # camera or flags
    m.geo_mode = 0
    m.cull_chunk = 1 << 21
    assert L.gs_cull_chunk_flags(C.byref(m), C.byref(cam), 1, ids, None) == gsdp.GS_EUNSUPPORTED
    m.cull_mode = 1
    m.cull_chunk = None
    assert L.gs_cull_chunk_flags(C.byref(m), C.byref(cam), 1, ids, None) == gsdp.GS_EUNSUPPORTED
    m.cull_chunk = 1 << 21
    m.max_defer = 15
    assert L.gs_cull_chunk_flags(C.byref(m), C.byref(cam), 1, ids, None) == gsdp.GS_EUNSUPPORTED
    m.max_defer = 0
    assert L.gs_cull_chunk_flags(C.byref(m), None, 1, ids, None) == gsdp.GS_EINVAL
    assert L.gs_cull_chunk_flags(C.byref(m), C.byref(cam), 1, None, None) == gsdp.GS_EINVAL
    assert L.gs_cull_chunk_flags(C.byref(m), C.byref(cam), 11, ids, None) == gsdp.GS_EINVAL


@pytest.mark.parametrize("kind,max_defer,sched", [("adam", 0, False), ("adam", 15, False), ("adam", 0, True),
                                                   ("sgdm", 15, True)])
def test_table_bound_covers_every_restore_coefficient(gsdp, kind, max_defer, sched):
    """The header's wbound (word 7) is at least every FP32 restore coefficient
    the tables hold at every step up to max_steps + 1."""
    T = 300
    rng = np.random.default_rng(3)
    sc = (0.01 ** (np.arange(T + 2) / (T + 1)) * rng.uniform(0.5, 2.0, T + 2)) if sched else None
    if kind == "adam":
        img = gsdp.gs_lut_build_host(0.9, 0.999, T, max_defer, lr_scale=sc)
    else:
        img = gsdp.gs_lut_build_sgd_momentum_host(0.9, T, max_defer, lr_scale=sc)
    v = LL.views(img, T, max_defer)
    wb = float(v["hdr"][7:8].view(np.float32)[0])
    top = 0.0
    for t in range(2, T + 2):
        gsdp.gs_lut_seek_host(img, t)
        top = max(top, float(v["Wf"][t & 1].max()))
        assert v["Wf"][t & 1].max() <= wb, t
    # not vacuous, and within a modest factor of the largest coefficient held
    assert 0.0 < top <= wb < 4.0 * top


def test_row_probe_checks_need_no_device(gsdp):
    L = gsdp.lib
    fake = C.c_void_p(1 << 20)
    assert L.gs_row_probe(None, 10, fake, 100, 48, 1, fake, None) == gsdp.GS_EINVAL
    assert L.gs_row_probe(fake, 10, fake, 100, 40, 1, fake, None) == gsdp.GS_EINVAL      # not a multiple of 16
    assert L.gs_row_probe(fake, 10, fake, 100, 2048, 0, fake, None) == gsdp.GS_EINVAL    # more than 1024 bytes
    assert L.gs_row_probe(fake, 0, fake, 100, 48, 0, fake, None) == gsdp.GS_OK          # nothing to do
