"""Train-step throughput of the Gaussian-parameter path on one MI355X.

One step = gs_cull (cull + ordered compaction of every Gaussian) ->
gs_gather (restored visible rows) -> gs_adam_step_deferred (fused scatter +
deferred Adam), on the 40M-Gaussian aerial workload (3000x3000x200 box, 4000
nadir/oblique cameras 1152x864 f=1100, one camera per step), FP32 moment
state; the same steps with BF16 moment state on the same scene are reported
beside it.
Synthetic gradients are generated on the device before the timed region (a
pool of compact gradient buffers, one per step mod pool size) and stand in
for the renderer's backward pass.

Prints one JSON line: value = Gaussians/s = N / (ms per step), with a
roofline object for the dominant call (HIP events on the launch stream,
algorithmic bytes per launch), the whole step's algorithmic bytes over its
median time, step-time percentiles, and the CPU oracle timed on a row sample
with all host cores and with one thread.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
METRIC = "train-step Gaussians/s (cull+gather+Adam), HBM % of peak, fp32 vs bf16-state"


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=100)
    p.add_argument("--warmup", type=int, default=10)
    p.add_argument("--workload", default="aerial40m",
                   choices=["small", "aerial4m", "aerial18m", "aerial40m", "aerial40m_f8", "batched16"])
    p.add_argument("--scenes", type=int, default=16, help="batched16: number of scenes")
    p.add_argument("--cams", type=int, default=32, help="batched16: cameras per scene per step")
    p.add_argument("--scale", type=float, default=1.0, help="batched16: multiply every scene size")
    p.add_argument("--copy-probe", type=int, default=0,
                   help="only copy this many MiB device-to-device 5 times (calibrates HBM byte counters)")
    p.add_argument("--n", type=int, default=None, help="override the Gaussian count")
    p.add_argument("--layout", default="fused", choices=["separate", "interleaved", "fused"])
    p.add_argument("--max-defer", type=int, default=0)
    p.add_argument("--cull-mode", type=int, default=1)
    p.add_argument("--cull-summary", type=int, default=1, choices=[0, 1],
                   help="1: the band cull reads the 16-byte cull summaries; 0: the geometry rows")
    p.add_argument("--cull-chunks", type=int, default=-1, choices=[-1, 0, 1],
                   help="chunk records of the summaries (the cull skips chunks whose box is culled): 1 on, "
                        "0 off, -1 on with rows in Morton order")
    p.add_argument("--other-order", type=int, default=1, choices=[0, 1],
                   help="also time the first state with the rows in the other order (reported as "
                        "generation_order or spatial_order)")
    p.add_argument("--state", default="f32", choices=["f32", "bf16", "fp8"], help="Adam moment storage (both groups)")
    p.add_argument("--compare-state", default="bf16", choices=["", "f32", "bf16", "fp8"],
                   help="a second moment storage timed on the same scene and reported beside the first")
    p.add_argument("--geo-state", default=None, choices=["f32", "bf16", "fp8"])
    p.add_argument("--graph", action="store_true",
                   help="also time the step captured in a hipGraph (camera table + device step counter)")
    p.add_argument("--geo-mode", type=int, default=0, help="1 = dense geometric Adam every step")
    p.add_argument("--tilt", default="20,45", help="oblique tilt range in degrees")
    p.add_argument("--pool", type=int, default=4)
    p.add_argument("--device-scene", type=int, default=None,
                   help="1 = draw the scene on the device (default for more than 8M Gaussians)")
    p.add_argument("--order", default="morton", choices=["generated", "morton"],
                   help="row order of the scene: sorted by the Morton code of the position, as the scene is laid "
                        "out at load (default; a camera's visible rows then form contiguous runs), or as generated "
                        "(spatially random)")
    p.add_argument("--metrics-jsonl", default=None,
                   help="append one JSON record per timed step (HIP event times per call) to this file")
    p.add_argument("--no-cpu-baseline", action="store_true")
    p.add_argument("--cpu-sample", type=int, default=1 << 20)
    p.add_argument("--cpu-steps", type=int, default=6)
    return p.parse_args()


def cpu_baseline(w, geo_all, app_all, sample, steps, lg, la):
    """The oracle as it stands, on a seeded row sample of the same workload:
    FP32 cull of the sample's geometry + ids + synthetic grads + dense FP64
    Adam on every sampled row (Eq. 1), per step, with all host cores and with
    one thread.  Gaussians/s = sample / median step time (the first step is
    not counted); p10 / p90 of the step times beside it."""
    from oracle import oracle as orc
    import gs_inputs as gi
    rng = np.random.default_rng(123)
    rows = np.sort(rng.choice(w.n, min(sample, w.n), replace=False))

    def take(x):
        if isinstance(x, np.ndarray):
            return np.ascontiguousarray(x[rows])
        import torch
        return x.index_select(0, torch.from_numpy(rows).to(x.device)).cpu().numpy()
    geo, app = take(geo_all), take(app_all)

    def leg(nsteps):
        dense = orc.DenseAdamF64(geo, app, lg, la)
        times = []
        for t in range(1, nsteps + 1):
            t0 = time.perf_counter()
            keep = orc.cull(dense.w[0].astype(np.float32), w.camera_for_step(t))
            valid = orc.compact(keep)
            gg, ga = gi.step_grads(0, t, rows[valid])
            dense.step(t, valid, gg, ga)
            times.append(time.perf_counter() - t0)
        ts = np.array(times[1:] if len(times) > 1 else times)
        med = float(np.median(ts))
        return med, float(np.percentile(ts, 10)), float(np.percentile(ts, 90))

    def paper_leg(nsteps):
        # the paper's own CPU method on this host: the deferred update (FP32
        # state, OpenMP) of the visible rows only, after the cull of the
        # sample's current geometry
        model = orc.DeferredF32(geo, app, lg, la)
        times = []
        for t in range(1, nsteps + 1):
            t0 = time.perf_counter()
            valid = model.cull_current(t, w.camera_for_step(t))
            gg, ga = gi.step_grads(0, t, rows[valid])
            model.step(t, valid, gg, ga)
            times.append(time.perf_counter() - t0)
        ts = np.array(times[1:] if len(times) > 1 else times)
        return float(np.median(ts))

    cores = orc.set_threads(0)
    med, p10, p90 = leg(steps)
    med_paper = paper_leg(steps)
    orc.set_threads(1)
    med1, p10_1, p90_1 = leg(max(3, steps // 2))
    orc.set_threads(cores)
    model, numa = host_cpu()
    what = (f"{rows.shape[0]} seeded rows of the {w.n}-Gaussian workload: FP32 cull + ids + synthetic grads + "
            f"dense FP64 Adam per step")
    return {"value": rows.shape[0] / med, "unit": "Gaussians/s", "cores": cores, "kind": "oracle",
            "sample": f"{what}; {steps} steps, median {med * 1e3:.1f} ms (p10 {p10 * 1e3:.1f}, p90 {p90 * 1e3:.1f})",
            "step_ms": {"p10": p10 * 1e3, "p50": med * 1e3, "p90": p90 * 1e3},
            "single_thread": {"value": rows.shape[0] / med1, "unit": "Gaussians/s", "cores": 1,
                              "step_ms": {"p10": p10_1 * 1e3, "p50": med1 * 1e3, "p90": p90_1 * 1e3}},
            "paper_method_on_host": {"value": rows.shape[0] / med_paper, "unit": "Gaussians/s", "cores": cores,
                                     "what": "the paper's deferred update (FP32 state, OpenMP) of the visible rows "
                                             "after the cull of the sample's current geometry, median step "
                                             f"{med_paper * 1e3:.1f} ms"},
            "cpu_model": model, "numa_nodes": numa}


# the launches behind each timed call (the cull is three launches: tile cull,
# group sums, prefixes + id scatter; with chunk records: chunk scan, tile
# cull, prefixes + id scatter; the batched cull four)
KERNEL_SYMBOLS = {"cull": ["k_cull", "k_tile_reduce", "k_tile_ids"],
                  "cull_sum": ["k_cull_sum", "k_tile_reduce", "k_tile_ids"],
                  "cull_chunks": ["k_chunk_scan", "k_cull_sum", "k_tile_ids"], "gather": ["k_rows_fz<0"],
                  "adam": ["k_rows_fz<1"], "cull_multi": ["k_cull_multi", "k_multi_reduce", "k_multi_gscan", "k_multi_offsets",
                                                      "k_multi_ids"],
                  "grad_sum": ["k_grad_sum"], "adam_bf16": ["k_rows_fz<1"]}


def source_digest():
    import hashlib
    h = hashlib.sha256()
    for name in ("gsdp.hip", "gsdp_internal.h", "gsdp_lut.cpp"):
        with open(os.path.join(ROOT, "paper_2509_15645_amd", "csrc", name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def measured_traffic(kernel, config_key):
    """HBM bytes per launch of `kernel` from the committed counter summary
    (FETCH_SIZE + WRITE_SIZE per dispatch, scaled by the plain-copy
    calibration), or None when no summary matches this configuration or the
    kernel sources changed since the counters were taken."""
    path = os.path.join(ROOT, "profiles", "hbm_traffic.txt")
    if not os.path.exists(path):
        return None
    digest, cur, found = source_digest(), None, {}
    for line in open(path):
        f = line.split()
        if len(f) >= 2 and f[0] == "source_digest":
            cur = f[1]
        elif len(f) >= 4 and f[0] == "bytes_per_launch" and cur == digest and f[1] == config_key:
            found[f[2]] = float(f[3])
    syms = KERNEL_SYMBOLS.get(kernel, [kernel])
    if not all(x in found for x in syms):
        return None
    return sum(found[x] for x in syms)


def morton_sorted(geo, app, box, on_dev):
    """The scene's rows sorted by the Morton code of their position (tensors
    on the device, or numpy arrays for a host scene)."""
    import torch
    g_t = torch.as_tensor(geo)
    perm = morton_order(g_t[:, :3], box)
    g_s = g_t[perm].contiguous()
    a_t = torch.as_tensor(app)
    a_s = a_t[perm.to(a_t.device)].contiguous()
    if not on_dev:
        return g_s.numpy(), a_s.numpy()
    return g_s, a_s


def morton_order(pos, box):
    """Permutation sorting rows by the 63-bit Morton code of their position
    quantised to 21 bits per axis inside `box` (a torch tensor in, out)."""
    import torch
    lo = torch.tensor([b[0] for b in box], dtype=torch.float64, device=pos.device)
    hi = torch.tensor([b[1] for b in box], dtype=torch.float64, device=pos.device)
    q = ((pos.double() - lo) / (hi - lo) * (2 ** 21 - 1)).clamp(0, 2 ** 21 - 1).long()
    code = torch.zeros(pos.shape[0], dtype=torch.int64, device=pos.device)
    for b in range(21):
        for a in range(3):
            code |= ((q[:, a] >> b) & 1) << (3 * b + a)
    return torch.argsort(code)


def run_batched(args):
    """16 scenes of log-uniform size (0.5M-8M) x 32 cameras per step: the
    batched cull + compaction, the gather of the union's current rows (once
    for all cameras), the deterministic per-camera gradient sum and the
    BF16-moment deferred Adam on the union; the step is captured in a hipGraph
    with a device step counter and replayed."""
    import torch

    import gs_inputs as gi
    from paper_2509_15645_amd import gsdp
    dev = torch.device("cuda")
    t_setup = time.perf_counter()
    sizes = [max(1024, int(x * args.scale)) for x in gi.batched_scene_sizes(args.scenes)]
    C = args.cams
    n_sets = 10
    geos, apps, row0, sets = [], [], [0], [[] for _ in range(n_sets)]
    for sidx, n in enumerate(sizes):
        box, half = gi.aerial_box_for(n)
        g_, a_ = gi.device_scene(n, box, 1000 + sidx, dev)
        if args.order == "morton":
            perm = morton_order(g_[:, :3], box)
            g_, a_ = g_[perm], a_[perm]
            del perm
        pad = (-n) % gsdp.MULTI_ALIGN
        if pad:
            gp = torch.full((pad, 10), float("nan"), device=dev)
            gp[:, 6] = 1.0
            g_ = torch.cat([g_, gp])
            a_ = torch.cat([a_, torch.zeros((pad, 49), device=dev)])
        geos.append(g_)
        apps.append(a_)
        row0.append(row0[-1] + n + pad)
        cams = gi.aerial_cameras(C * n_sets, half, half, seed=sidx)
        for k in range(n_sets):
            sets[k].append(cams[k * C:(k + 1) * C])
    geo = torch.cat(geos)
    app = torch.cat(apps)
    del geos, apps
    N = int(geo.shape[0])
    n_real = sum(sizes)
    lg, la = gi.lr_columns()
    total_steps = args.warmup + args.steps + 2
    # (the batched cull reads the geometry rows: no summaries to keep)
    model = gsdp.Model(geo, app, lg, la, max_steps=total_steps + 4, cull_mode=args.cull_mode,
                       app_layout=args.layout, geo_state=args.geo_state or "bf16", app_state="bf16", sr_seed=9,
                       cull_summary=False)
    del geo, app
    cap_cam = max(1, int(N * 0.08))      # one camera slot over all scenes sees up to ~5% of the rows
    multi = gsdp.Multi(model, row0, sets, cap_union=N, cap_cam=cap_cam)
    D = 59
    g_cam = torch.empty((C, cap_cam, D), dtype=torch.float32, device=dev)
    g_cam.normal_(0.0, 1e-3, generator=torch.Generator(device=dev).manual_seed(5))
    out_g = torch.zeros((N, 10), dtype=torch.float32, device=dev)
    out_a = torch.zeros((N, 49), dtype=torch.float32, device=dev)
    gath_g = torch.zeros((N, 10), dtype=torch.float32, device=dev)
    gath_a = torch.zeros((N, 49), dtype=torch.float32, device=dev)
    model.step_dev.fill_(1)
    setup_s = time.perf_counter() - t_setup

    def step_dev_only():
        gsdp.gs_cull_multi(model, multi, 0)
        gsdp.gs_gather(model, 0, multi.union_ids, multi.union_count, gath_g, gath_a, capacity=multi.cap_union)
        gsdp.gs_grad_sum_multi(multi, 49, g_cam, out_g, out_a)
        gsdp.gs_adam_step_deferred(model, 0, multi.union_ids, multi.union_count, out_g, out_a,
                                   capacity=multi.cap_union)
        gsdp.gs_step_advance(model.step_dev)

    for _ in range(args.warmup):
        step_dev_only()
    # autotune the batched cull on the next step's cameras and state (deferred
    # rows to restore, as in every timed step); the cull only reads the model
    t_next = args.warmup + 1
    times = gsdp.gs_cull_multi_autotune(model, multi, t_next)
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        step_dev_only()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        graph.replay()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms_step = (t1 - t0) * 1e3 / args.steps
    # per-kernel attribution: the same steps eagerly with HIP events
    stream = torch.cuda.current_stream()
    ev = [[torch.cuda.Event(enable_timing=True) for _ in range(5)] for _ in range(3)]
    U_tot, cc_tot = 0, 0
    for k in range(3):
        ev[k][0].record(stream)
        gsdp.gs_cull_multi(model, multi, 0)
        ev[k][1].record(stream)
        gsdp.gs_gather(model, 0, multi.union_ids, multi.union_count, gath_g, gath_a, capacity=multi.cap_union)
        ev[k][2].record(stream)
        gsdp.gs_grad_sum_multi(multi, 49, g_cam, out_g, out_a)
        ev[k][3].record(stream)
        gsdp.gs_adam_step_deferred(model, 0, multi.union_ids, multi.union_count, out_g, out_a,
                                   capacity=multi.cap_union)
        ev[k][4].record(stream)
        gsdp.gs_step_advance(model.step_dev)
        torch.cuda.synchronize()
        U_tot += int(multi.union_count.item())
        cc_tot += int(multi.cam_count.sum().item())
    if int(multi.cam_count.max().item()) > cap_cam:
        raise RuntimeError("camera list capacity exceeded")
    hdr = model.lut_header()
    if hdr["error"]:
        raise RuntimeError(f"deferred-update tables report an error: {hdr}")
    # rows behind the current step (deferred) and their mean defer count
    t_now = int(model.step_dev.item())
    lag = (t_now - 1) - model.last_step.long()
    deferred = {"step": t_now, "rows_deferred_frac": float((lag > 0).double().mean().item()),
                "mean_defer": float(lag.clamp(min=0).double().mean().item())}
    k_ms = np.array([[e[i].elapsed_time(e[i + 1]) for i in range(4)] for e in ev]).mean(0)
    U, CC = U_tot / 3.0, cc_tot / 3.0
    sg = 4 if (args.geo_state or "bf16") == "f32" else 2
    cull_bytes = 44.0 * N + 4.0 * U + 4.0 * CC
    # gather: id + last step + G w and A w, m, v (+ G m, v) + the 236-byte output row
    gather_bytes = U * (4 + 4 + 40 + 2 * 10 * sg + 49 * (4 + 2 * 2) + 236)
    sum_bytes = CC * (D * 4 + 4) + U * D * 4
    adam_bytes = U * (12 + 10 * (12 + 4 * sg) + 49 * (12 + 4 * 2))
    kern = {"cull_multi": (k_ms[0], cull_bytes), "gather": (k_ms[1], gather_bytes), "grad_sum": (k_ms[2], sum_bytes),
            "adam_bf16": (k_ms[3], adam_bytes)}
    dom = max(kern, key=lambda k: kern[k][0])
    achieved = kern[dom][1] / (kern[dom][0] * 1e-3) / 1e9
    out = {
        "metric": "train-step Gaussians/s (cull+gather+Adam), BF16 moment state, batched scenes x cameras",
        "value": n_real / (ms_step * 1e-3), "unit": "Gaussians/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms_step, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32 math, bf16 moments", "data": "synthetic",
        "config": {"workload": "batched16", "scenes": len(sizes), "scene_sizes": sizes, "n_gaussians": n_real,
                   "row_order": args.order,
                   "rows_padded": N, "cameras_per_scene": C, "union_per_step": U, "camera_entries_per_step": CC,
                   "geo_state": args.geo_state or "bf16", "app_state": "bf16",
                   "autotune_ms": times, "variant": int(multi.c.variant), "hipgraph": True,
                   "deferral": deferred},
        "kernels_ms": {k: float(v[0]) for k, v in kern.items()},
        "kernels_gbs": {k: v[1] / (v[0] * 1e-3) / 1e9 for k, v in kern.items()},
        "roofline": {"kernel": dom, "bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": None},
        "setup_s": setup_s,
    }
    print(json.dumps(out), flush=True)


def chunks_on(args):
    """Chunk records: as asked, or by default with rows in Morton order."""
    return bool(args.cull_chunks) if args.cull_chunks >= 0 else args.order == "morton"


def config_key(args, workload, state=None):
    """Names the launch configuration a counter summary was taken with."""
    st = state or args.state
    summ = args.cull_summary and args.cull_mode == 1 and args.geo_mode == 0
    return (f"{workload}/{st}/{args.geo_state or st}/{args.layout}/cull{args.cull_mode}"
            f"/geo{args.geo_mode}/K{args.max_defer}/tilt{args.tilt.replace(',', '-')}/{args.order}"
            f"/sum{int(bool(summ))}" + ("/chunks" if summ and chunks_on(args) else ""))


def host_cpu():
    """CPU model name and NUMA node count of this host."""
    model = "unknown"
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    try:
        nodes = len([d for d in os.listdir("/sys/devices/system/node") if d.startswith("node") and d[4:].isdigit()])
    except OSError:
        nodes = None
    return model, nodes


def step_bytes(n, M, R, geo_state, app_state, geo_mode, summary=0, chunk_skip=None):
    """Algorithmic bytes of one step per call (sg / sa: bytes per stored moment
    of G / A): cull 44 per Gaussian (geometry row + last step) + 20 sg per
    restored row + 4 per visible id, or with cull summaries `summary` bytes per
    Gaussian (16, or 20 with the last step past 2^16 steps) + (4 + 40 + 20 sg)
    per restored row (last step, geometry row and moments; undecided rows that
    need no restore are not counted) + 4 per visible id; with chunk records
    (chunk_skip: the fraction of chunks skipped) 32 per 1024-row chunk + the
    summaries of the chunks not skipped; gather id + last step
    + G w, m, v + A w, m, v + the 236-byte output row; Adam id + last step
    read and write + per column w, g read, w written and m, v read and written
    (+ the 16-byte summary written)."""
    msz = {"f32": 4, "bf16": 2, "fp8": 1}
    sg, sa = msz[geo_state], msz[app_state]
    gcols = 0 if geo_mode else 10                       # G columns handled by the sparse kernels
    if summary and chunk_skip is not None:
        cull = 32.0 * math.ceil(n / 1024) + float(summary) * n * (1.0 - chunk_skip) + (44.0 + 20.0 * sg) * R + 4.0 * M
    elif summary:
        cull = float(summary) * n + (44.0 + 20.0 * sg) * R + 4.0 * M
    else:
        cull = 44.0 * n + 20.0 * sg * R + 4.0 * M
    gather = M * (4 + 4 + 8 * 10 + 2 * sg * gcols + 8 * 49 + 2 * sa * 49)
    adam = M * (4 + 4 + 4 + gcols * (12 + 4 * sg) + 49 * (12 + 4 * sa) + (16 if summary else 0))
    if geo_mode:                                        # dense G Adam over every row
        adam += n * 10 * (8 + 4 * sg) + n / 8.0 + M * 40
    return {"cull": cull, "gather": gather, "adam": adam}


def run_single(args, w, geo0, app0, state, tilt, on_dev):
    """Times K steps of one moment-state configuration; returns its result
    record (the scene tensors are not modified)."""
    import torch

    import gs_inputs as gi
    from paper_2509_15645_amd import gsdp
    dev = torch.device("cuda")
    t_setup = time.perf_counter()
    lg, la = gi.lr_columns()
    total_steps = args.warmup + args.steps
    geo_state = args.geo_state or state
    geo_in = geo0.clone() if torch.is_tensor(geo0) else geo0
    model = gsdp.Model(geo_in, app0, lg, la, max_steps=2 * total_steps + 8, max_defer=args.max_defer,
                       cull_mode=args.cull_mode, app_layout=args.layout, geo_state=geo_state,
                       app_state=state, geo_mode=args.geo_mode, sr_seed=9,
                       cull_summary=None if args.cull_summary else False,
                       cull_chunks=chunks_on(args))
    summ = model.cull_sum is not None
    sum_bytes = (16 if model.max_steps <= 65536 else 20) if summ else 0
    del geo_in
    n = w.n
    cap = max(1, n // 2)             # a high oblique camera of the 8% workload sees up to 27%
    ids = torch.zeros(cap, dtype=torch.int32, device=dev)
    count = torch.zeros(1, dtype=torch.int32, device=dev)
    out_g = torch.zeros((cap, 10), dtype=torch.float32, device=dev)
    out_a = torch.zeros((cap, 49), dtype=torch.float32, device=dev)
    full = torch.tensor([cap], dtype=torch.int32, device=dev)
    pool = []
    for p in range(args.pool):
        gg = torch.empty((cap, 10), dtype=torch.float32, device=dev)
        ga = torch.empty((cap, 49), dtype=torch.float32, device=dev)
        gsdp.gs_synth_grad(1000 + p, 0, None, full, gg, 0)
        gsdp.gs_synth_grad(1000 + p, 0, None, full, ga, 10)
        pool.append((gg, ga))
    cams = [gsdp.camera_struct(w.camera_for_step(t)) for t in range(1, total_steps + 1)]
    torch.cuda.synchronize()
    setup_s = time.perf_counter() - t_setup
    stream = torch.cuda.current_stream()

    def step(t, ev=None):
        if ev is not None:
            ev[0].record(stream)
        gsdp.gs_cull(model, cams[t - 1], t, ids, count, stream=stream)
        if ev is not None:
            ev[1].record(stream)
        gsdp.gs_gather(model, t, ids, count, out_g, out_a, stream=stream)
        if ev is not None:
            ev[2].record(stream)
        gg, ga = pool[t % len(pool)]
        gsdp.gs_adam_step_deferred(model, t, ids, count, gg, ga, stream=stream)
        if ev is not None:
            ev[3].record(stream)

    for t in range(1, args.warmup + 1):
        step(t)
    torch.cuda.synchronize()
    h0 = model.ws_header()
    evs = [[torch.cuda.Event(enable_timing=True) for _ in range(4)] for _ in range(args.steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        step(args.warmup + 1 + k, evs[k])
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    h1 = model.ws_header()
    if h1["error"]:
        raise RuntimeError(f"cull reported an error flag: {h1}")
    ms_step = (t1 - t0) * 1e3 / args.steps
    # the chunks the summary cull skipped at each timed step (decided again
    # after the timed steps, from the records as they are then)
    chunk_skip = None
    if summ and model.cull_chunk is not None and args.max_defer == 0:
        fl = torch.zeros(model.cull_chunk.shape[0], dtype=torch.uint8, device=dev)
        fr = []
        for k in range(args.steps):
            t = args.warmup + 1 + k
            gsdp.gs_cull_chunk_flags(model, cams[t - 1], t, fl, stream=stream)
            fr.append(fl.float().mean())
        chunk_skip = float(torch.stack(fr).mean().item())

    # the hardware's bandwidth for the last step's visible rows of the fused
    # state: loads, and loads with unchanged stores (gs_row_probe)
    row_probe = None
    fz = getattr(model, "app_state_bytes", None)
    if fz is not None and fz.shape[1] <= 1024 and fz.shape[1] % 16 == 0:
        m_last = min(int(count.item()), cap)
        sink = torch.zeros(1, dtype=torch.float32, device=dev)
        row_probe = {"what": "the last step's visible rows of the fused state (one byte row per Gaussian): "
                             "loads, then loads with the same bytes stored back", "rows": m_last,
                     "row_bytes": int(fz.shape[1])}
        for name, wr in (("read", False), ("read_write", True)):
            pe = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
            for _ in range(2):
                gsdp.gs_row_probe(ids, m_last, fz, wr, sink, stream=stream)
            pe[0].record(stream)
            reps = 10
            for _ in range(reps):
                gsdp.gs_row_probe(ids, m_last, fz, wr, sink, stream=stream)
            pe[1].record(stream)
            torch.cuda.synchronize()
            us = pe[0].elapsed_time(pe[1]) * 1e3 / reps
            moved = m_last * fz.shape[1] * (2 if wr else 1)
            row_probe[name] = {"us": us, "gbs": moved / (us * 1e-6) / 1e9}

    graph_ms = None
    if args.graph:
        # the same step as one hipGraph, the camera of step t read from a device
        # table (gs_cull_table, the summary cull); without summaries the
        # single-camera cull runs as the batched cull with one scene and one
        # camera per set (set k = the camera of step k+1)
        ntab = total_steps + args.steps + 2
        gg, ga = pool[0]
        t_next = args.warmup + args.steps + 1
        model.step_dev.fill_(t_next)
        if summ:
            table = gsdp.camera_table(model, [w.camera_for_step(k + 1) for k in range(ntab)])

            def gstep():
                gsdp.gs_cull_table(model, table, 0, ids, count, capacity=cap)
                gsdp.gs_gather(model, 0, ids, count, out_g, out_a, capacity=cap)
                gsdp.gs_adam_step_deferred(model, 0, ids, count, gg, ga, capacity=cap)
                gsdp.gs_step_advance(model.step_dev)
        else:
            cam_sets = [[[w.camera_for_step(k + 1)]] for k in range(ntab)]
            multi = gsdp.Multi(model, [0, n], cam_sets, cap_union=cap, cap_cam=1)

            def gstep():
                gsdp.gs_cull_multi(model, multi, 0)
                gsdp.gs_gather(model, 0, multi.union_ids, multi.union_count, out_g, out_a, capacity=cap)
                gsdp.gs_adam_step_deferred(model, 0, multi.union_ids, multi.union_count, gg, ga, capacity=cap)
                gsdp.gs_step_advance(model.step_dev)

        gstep()
        torch.cuda.synchronize()
        graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(graph):
            gstep()
        torch.cuda.synchronize()
        reps = min(args.steps, ntab - (t_next + 1) - 1)
        g0 = time.perf_counter()
        for _ in range(reps):
            graph.replay()
        torch.cuda.synchronize()
        graph_ms = (time.perf_counter() - g0) * 1e3 / reps
    k_ms = np.array([[e[0].elapsed_time(e[1]), e[1].elapsed_time(e[2]), e[2].elapsed_time(e[3])]
                     for e in evs])
    if args.metrics_jsonl:
        with open(args.metrics_jsonl, "a") as fh:
            for k, row in enumerate(k_ms):
                fh.write(json.dumps({"workload": w.name, "state": state, "step": args.warmup + 1 + k,
                                     "cull_ms": float(row[0]), "gather_ms": float(row[1]),
                                     "adam_ms": float(row[2]), "step_ms": float(row.sum())}) + "\n")
    cull_ms, gather_ms, adam_ms = k_ms.mean(0)
    step_ev = k_ms.sum(1)
    vis_total = h1["vis_accum"] - h0["vis_accum"]
    rest_total = h1["restored_accum"] - h0["restored_accum"]
    M = vis_total / args.steps
    R = rest_total / args.steps
    f = M / n
    by = step_bytes(n, M, R, geo_state, state, args.geo_mode, sum_bytes, chunk_skip)
    kernels = {k: (float(ms), by[k]) for k, ms in (("cull", cull_ms), ("gather", gather_ms), ("adam", adam_ms))}
    dom = max(kernels, key=lambda k: kernels[k][0])
    # the launches of the dominant call
    sym = dom if dom != "cull" or not summ else ("cull_chunks" if chunk_skip is not None else "cull_sum")
    dms, dbytes = kernels[dom]
    achieved = dbytes / (dms * 1e-3) / 1e9
    tot_bytes = sum(by.values())
    p10, p50, p90 = (float(x) for x in np.percentile(step_ev, [10, 50, 90]))
    step_gbs = tot_bytes / (p50 * 1e-3) / 1e9
    rec = {
        "value": n / (ms_step * 1e-3), "ms_per_step": ms_step,
        "step_ms": {"p10": p10, "p50": p50, "p90": p90, "from": "HIP events around the three calls of each step"},
        "value_p50": n / (p50 * 1e-3),
        "config": {"workload": w.name, "n_gaussians": n, "scene_drawn_on": "device" if on_dev else "host",
                   "row_order": args.order, "cameras": len(w.cameras),
                   "image": f"{w.cameras[0].width}x{w.cameras[0].height}", "oblique_tilt_deg": list(tilt),
                   "visible_fraction": f, "visible_per_step": M, "restored_per_step": R,
                   "state": state, "geo_state": geo_state, "app_layout": args.layout,
                   "max_defer": args.max_defer, "cull_mode": args.cull_mode, "geo_mode": args.geo_mode,
                   "cull_summary": summ, "cull_bytes_per_row": sum_bytes or 44,
                   "cull_chunks": model.cull_chunk is not None, "chunks_skipped": chunk_skip},
        "kernels_ms": {k: v[0] for k, v in kernels.items()},
        "graph_ms_per_step": graph_ms,
        "kernels_gbs": {k: v[1] / (v[0] * 1e-3) / 1e9 for k, v in kernels.items()},
        "roofline": {"kernel": dom, "launches": KERNEL_SYMBOLS[sym], "bound": "hbm", "achieved": achieved,
                     "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
                     "traffic": measured_traffic(sym, config_key(args, w.name, state)),
                     "traffic_from": "profiles/hbm_traffic.txt (rocprofv3 FETCH_SIZE, WRITE_SIZE), "
                                     "used only while the library sources match its digest",
                     "algorithmic_bytes": dbytes},
        "step_roofline": {"bound": "hbm", "algorithmic_bytes": tot_bytes, "ms": p50, "achieved": step_gbs,
                          "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": step_gbs / HBM_PEAK_GBS,
                          "what": "all three calls' algorithmic bytes over the median step time"},
        "setup_s": setup_s,
        "row_probe": row_probe,
    }
    del model, pool, out_g, out_a
    torch.cuda.empty_cache()
    return rec


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU; multi-GPU sharding is a design note only",
                          "n_gpus": args.gpus}))
        sys.exit(2)
    if args.copy_probe:
        import torch
        n = args.copy_probe * (1 << 20) // 4
        a = torch.ones(n, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        for _ in range(5):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_probe_mib": args.copy_probe, "launches": 5}))
        return
    if args.workload == "batched16":
        run_batched(args)
        return
    import torch

    import gs_inputs as gi
    from paper_2509_15645_amd import gsdp

    torch.cuda.set_device(0)
    tilt = tuple(float(x) for x in args.tilt.split(","))
    w = gi.workload(args.workload, n=args.n, tilt_deg=tilt)
    dev = torch.device("cuda")
    on_dev = args.device_scene if args.device_scene is not None else int(w.n > 8_000_000)
    if on_dev:
        geo0, app0 = gi.device_scene(w.n, w.scene_box, 0, dev)
    else:
        sc = gi.make_scene(w.n, seed=0, box=w.scene_box)
        geo0, app0 = sc.geo, sc.app
    geo_gen, app_gen = geo0, app0
    if args.order == "morton":
        geo0, app0 = morton_sorted(geo0, app0, w.scene_box, on_dev)
    main_rec = run_single(args, w, geo0, app0, args.state, tilt, on_dev)
    second = None
    if args.compare_state and args.compare_state != args.state:
        second = run_single(args, w, geo0, app0, args.compare_state, tilt, on_dev)
    # achievable read bandwidth of the cull's main stream: a plain streaming
    # read of the [n][10] geometry array, timed the same way
    gflat = torch.as_tensor(geo0).to(dev).reshape(-1)
    flat = gflat[: (gflat.numel() // 4) * 4]
    sink = torch.zeros(1, dtype=torch.float32, device="cuda")
    pe = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
    gsdp.gs_stream_read_probe(flat, sink)
    pe[0].record()
    for _ in range(5):
        gsdp.gs_stream_read_probe(flat, sink)
    pe[1].record()
    torch.cuda.synchronize()
    probe_gbs = flat.numel() * 4 * 5 / (pe[0].elapsed_time(pe[1]) * 1e-3) / 1e9
    out = {
        "metric": METRIC,
        "value": main_rec["value"],
        "unit": "Gaussians/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": main_rec["ms_per_step"],
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32", "data": "synthetic",
    }
    out.update({k: v for k, v in main_rec.items() if k not in ("value", "ms_per_step")})
    if second is not None:
        out[f"{args.compare_state}_state"] = second
    out["stream_probe"] = {"what": "streaming read of the [n][10] geometry array", "bytes": flat.numel() * 4,
                           "gbs": probe_gbs, "frac_of_peak": probe_gbs / HBM_PEAK_GBS}
    del gflat, flat
    if args.other_order:
        # the same scene and cameras, the first state, with the rows in the
        # other order (chunk records with the Morton order only)
        op = argparse.Namespace(**vars(args))
        op.order = "generated" if args.order == "morton" else "morton"
        op.cull_chunks = -1
        if op.order == "morton":
            g_o, a_o = morton_sorted(geo_gen, app_gen, w.scene_box, on_dev)
        else:
            g_o, a_o = geo_gen, app_gen
        rec = run_single(op, w, g_o, a_o, args.state, tilt, on_dev)
        del g_o, a_o
        keep = ("value", "ms_per_step", "step_ms", "value_p50", "kernels_ms", "kernels_gbs", "roofline",
                "step_roofline")
        name = "spatial_order" if op.order == "morton" else "generation_order"
        what = ("the rows sorted by the Morton code of their position, chunk records on" if op.order == "morton"
                else "the rows in generation order (spatially random), no chunk records")
        out[name] = {"what": "the same scene and cameras with " + what, **{k: rec[k] for k in keep},
                     "config": {k: rec["config"][k] for k in ("row_order", "state", "cull_chunks", "chunks_skipped",
                                                              "visible_per_step", "restored_per_step")}}
        torch.cuda.empty_cache()
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(w, geo_gen, app_gen, args.cpu_sample, args.cpu_steps, *gi.lr_columns())
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
