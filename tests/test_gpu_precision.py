"""The precision form at full size (40M Gaussians, the aerial 40M workload):
BF16 or FP8 moment state on the GPU path, T steps of cull -> gather ->
deferred Adam with synthetic compact gradients, then a flush.  A seeded
sample of rows is replayed on the host with dense FP64 Adam (the oracle):
Adam is per row once the visible sets and gradients are fixed, so the sample
is exact.  Reports the per-group error |w - w64| / (lr T), over the sample
and over the sampled rows the cameras touched, and checks the bounds derived
for one stochastic rounding per stored moment (BF16: max 2e-2; FP8: max 0.3,
mean 2e-2)."""
import sys

import numpy as np
import pytest
import torch

import gs_inputs as gi
from oracle import oracle as orc

pytestmark = pytest.mark.gpu

STEPS = 100
SAMPLE = 1 << 16


def say(*a):
    print(*a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def g():
    from paper_2509_15645_amd import gsdp
    return gsdp


@pytest.mark.parametrize("state", ["bf16", "fp8"])
def test_precision_form_40m_sampled(g, state):
    w = gi.workload("aerial40m")
    n, dev = w.n, torch.device("cuda")
    geo0, app0 = gi.device_scene(n, w.scene_box, 7, dev)
    lg, la = gi.lr_columns()
    model = g.Model(geo0, app0, lg, la, max_steps=STEPS + 4, cull_mode=1, app_layout="fused",
                    geo_state=state, app_state=state, sr_seed=11)
    rng = np.random.default_rng(5)
    sample = np.sort(rng.choice(n, SAMPLE, replace=False)).astype(np.int64)
    sidx = torch.from_numpy(sample).to(dev)
    dense = orc.DenseAdamF64(geo0[sidx].cpu().numpy(), app0[sidx].cpu().numpy(), lg, la)
    del geo0, app0
    cap = n // 4
    ids = torch.zeros(cap, dtype=torch.int32, device=dev)
    count = torch.zeros(1, dtype=torch.int32, device=dev)
    out_g = torch.zeros((cap, 10), dtype=torch.float32, device=dev)
    out_a = torch.zeros((cap, 49), dtype=torch.float32, device=dev)
    touched = np.zeros(SAMPLE, bool)
    for t in range(1, STEPS + 1):
        g.gs_cull(model, w.camera_for_step(t), t, ids, count)
        g.gs_gather(model, t, ids, count, out_g, out_a)
        m = int(count.item())
        assert m <= cap
        gg = torch.empty((m, 10), dtype=torch.float32, device=dev)
        ga = torch.empty((m, 49), dtype=torch.float32, device=dev)
        mt = torch.tensor([m], dtype=torch.int32, device=dev)
        g.gs_synth_grad(31, t, None, mt, gg, 0)
        g.gs_synth_grad(31, t, None, mt, ga, 10)
        g.gs_adam_step_deferred(model, t, ids, count, gg, ga)
        # the sampled rows among this step's visible rows, with their compact gradients
        vis = ids[:m].long().cpu().numpy()
        pos_in_sample = np.searchsorted(sample, vis)
        hit = (pos_in_sample < SAMPLE) & (sample[np.minimum(pos_in_sample, SAMPLE - 1)] == vis)
        local = pos_in_sample[hit]
        rows = torch.from_numpy(np.nonzero(hit)[0]).to(dev)
        dense.step(t, local.astype(np.uint32), gg[rows].cpu().numpy(), ga[rows].cpu().numpy())
        touched[local] = True
    g.gs_adam_flush(model, STEPS)
    torch.cuda.synchronize()
    assert model.ws_header()["error"] == 0
    got = (model.geo_w[sidx].double().cpu().numpy(), model.app_w[sidx].double().cpu().numpy())
    say(f"[precision 40M {state}] {STEPS} steps, {touched.sum()} of {SAMPLE} sampled rows touched")
    for k, lr in ((0, lg), (1, la)):
        err = np.abs(got[k] - dense.w[k]) / (lr.astype(np.float64) * STEPS)
        et = err[touched]
        say(f"[precision 40M {state}] group {k}: |w - w64| / (lr T) max {err.max():.3e} "
            f"mean(all) {err.mean():.3e} mean(touched) {et.mean() if et.size else 0.0:.3e}")
        if state == "bf16":
            assert err.max() <= 2e-2
        else:
            assert err.max() <= 0.3 and (et.mean() if et.size else 0.0) <= 2e-2
