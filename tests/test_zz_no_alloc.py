"""gs_cull_noalloc (the cull whose workspace is the library's own per-GPU
array) against gs_cull on the caller's workspace: ids and counts bit-exact on
two calls in a row, the second on a smaller model; also with chunk records
on rows in a spatial order, whose chunk scan writes into the array too, at
a size whose compaction reads group sums and then at one that does not (run
with -m gpu)."""
import sys

import numpy as np
import pytest
import torch

import gs_inputs as gi

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def g():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2509_15645_amd import gsdp
    return gsdp


def _model(g, n, seed, chunks):
    lg, la = gi.lr_columns()
    if chunks:
        from test_gpu_chunks import _scene
        geo, app, _ = _scene(n, seed)
        return g.Model(geo, app, lg, la, max_steps=8, cull_mode=1, cull_chunks=True)
    sc = gi.make_scene(n, seed=seed)
    return g.Model(sc.geo, sc.app, lg, la, max_steps=8, cull_mode=1)


@pytest.mark.parametrize("order", ["large_then_small", "small_again", "chunks_large_then_small",
                                   "chunks_grouped_then_small"])
def test_cull_noalloc_matches_cull(g, order):
    chunks = order.startswith("chunks")
    cams = gi.aerial_cameras(4, 1000.0, 1000.0, seed=3) if chunks else gi.orbit_cameras(4, seed=3)
    sizes = (300_007, 40_001) if order.endswith("large_then_small") else (40_001, 12_345)
    if order == "chunks_grouped_then_small":
        # more than 16384 tiles: the group sums the summary cull adds to sit in
        # the array too; then a model small enough to sum its tiles directly
        sizes = (9_000_000, 300_007)
    for call, n in enumerate(sizes):
        say(f"[noalloc] {order} call {call}: n={n}")
        model = _model(g, n, 20 + call, chunks)
        assert (model.cull_chunk is not None) == chunks
        # take one deferred step first so the cull restores rows (band classifier path)
        ids = torch.zeros(n, dtype=torch.int32, device="cuda")
        count = torch.zeros(1, dtype=torch.int32, device="cuda")
        g.gs_cull(model, cams[0], 1, ids, count)
        gg = torch.empty((n, 10), dtype=torch.float32, device="cuda")
        ga = torch.empty((n, 49), dtype=torch.float32, device="cuda")
        g.gs_synth_grad(0, 1, ids, count, gg, 0)
        g.gs_synth_grad(0, 1, ids, count, ga, 10)
        g.gs_adam_step_deferred(model, 1, ids, count, gg, ga)
        for t, cam in ((2, cams[1]), (3, cams[2])):
            ref_ids = torch.full((n,), -1, dtype=torch.int32, device="cuda")
            ref_cnt = torch.zeros(1, dtype=torch.int32, device="cuda")
            got_ids = torch.full((n,), -1, dtype=torch.int32, device="cuda")
            got_cnt = torch.zeros(1, dtype=torch.int32, device="cuda")
            g.gs_cull(model, cam, t, ref_ids, ref_cnt)
            g.gs_cull_noalloc(model, cam, t, got_ids, got_cnt)
            # a capacity below the count: only that many ids, the true count
            cap = max(1, int(ref_cnt.item()) // 3)
            part_ids = torch.full((n,), -1, dtype=torch.int32, device="cuda")
            part_cnt = torch.zeros(1, dtype=torch.int32, device="cuda")
            g.gs_cull_noalloc(model, cam, t, part_ids, part_cnt, capacity=cap)
            torch.cuda.synchronize()
            m = int(ref_cnt.item())
            assert 0 < m < n
            assert int(got_cnt.item()) == m
            assert np.array_equal(got_ids.cpu().numpy(), ref_ids.cpu().numpy())
            assert int(part_cnt.item()) == m
            pi = part_ids.cpu().numpy()
            assert np.array_equal(pi[:cap], ref_ids.cpu().numpy()[:cap]) and np.all(pi[cap:] == -1)
            say(f"[noalloc] {order} call {call} step {t}: M={m} ids bit-exact")
        del model
