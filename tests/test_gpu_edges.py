"""Degenerate inputs of the update path (run with -m gpu): an empty model, an
empty visible list, a zero capacity, ids past the rows and a capacity below
the count.  Every call succeeds, stores exactly what its contract says, and
the tables still advance one step per update."""
import sys

import numpy as np
import pytest
import torch

import gs_inputs as gi
from oracle import oracle as orc

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def g():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2509_15645_amd import gsdp
    return gsdp


def bits(a):
    return np.ascontiguousarray(a, np.float32).view(np.uint32)


@pytest.mark.parametrize("layout,state", [("fused", "f32"), ("fused", "bf16"), ("interleaved", "fp8")])
def test_empty_model_and_empty_lists(g, layout, state):
    lg, la = gi.lr_columns()
    empty = g.Model(np.zeros((0, 10), np.float32), np.zeros((0, 49), np.float32), lg, la, max_steps=4,
                    app_layout=layout, geo_state=state, app_state=state)
    ids = torch.zeros(1, dtype=torch.int32, device="cuda")
    count = torch.zeros(1, dtype=torch.int32, device="cuda")
    gg = torch.zeros((1, 10), device="cuda")
    ga = torch.zeros((1, 49), device="cuda")
    cam = gi.orbit_cameras(1, seed=1)[0]
    for t in (1, 2):
        g.gs_cull(empty, cam, t, ids, count)
        g.gs_gather(empty, t, ids, count, gg, ga)
        g.gs_adam_step_deferred(empty, t, ids, count, gg, ga)
    g.gs_adam_flush(empty, 2)
    torch.cuda.synchronize()
    assert int(count.item()) == 0
    assert sorted(empty.lut_header()["t_row"]) == [2, 3] and empty.ws_header()["error"] == 0

    # a model whose visible list is empty (a camera that sees nothing): no row
    # changes, the tables advance
    n = 5000
    sc = gi.make_scene(n, seed=2)
    model = g.Model(sc.geo, sc.app, lg, la, max_steps=4, app_layout=layout, geo_state=state, app_state=state)
    before = model.state()
    g.gs_adam_step_deferred(model, 1, ids, count, gg, ga)          # count = 0
    g.gs_adam_step_deferred(model, 2, ids, count, gg, ga, capacity=0)
    torch.cuda.synchronize()
    after = model.state()
    for k in before:
        assert before[k].tobytes() == after[k].tobytes(), k
    assert sorted(model.lut_header()["t_row"]) == [2, 3] and model.ws_header()["error"] == 0


def test_ids_past_the_rows_are_skipped_and_capacity_bounds_the_list(g):
    """Ids >= n in the list are skipped by the gather and the update; a
    capacity below the count makes them use the first `capacity` entries."""
    n = 20_000
    sc = gi.make_scene(n, seed=3)
    lg, la = gi.lr_columns()
    model = g.Model(sc.geo, sc.app, lg, la, max_steps=8, app_layout="fused")
    o3 = orc.DeferredF32(sc.geo, sc.app, lg, la)
    rng = np.random.default_rng(4)
    rows = np.sort(rng.choice(n, 300, replace=False)).astype(np.uint32)
    lst = np.concatenate([rows[:200], np.array([n, n + 5, 0xFFFFFFF0], np.uint32), rows[200:]])
    ids = torch.from_numpy(lst.view(np.int32)).cuda()
    count = torch.tensor([lst.shape[0]], dtype=torch.int32, device="cuda")
    cap = 250                                   # 200 valid + 3 past the rows + 47 valid
    gg = torch.from_numpy(rng.normal(0, 1e-3, (cap, 10)).astype(np.float32)).cuda()
    ga = torch.from_numpy(rng.normal(0, 1e-3, (cap, 49)).astype(np.float32)).cuda()
    out_g = torch.full((cap, 10), 7.0, device="cuda")
    out_a = torch.full((cap, 49), 7.0, device="cuda")
    g.gs_gather(model, 1, ids, count, out_g, out_a, capacity=cap)
    g.gs_adam_step_deferred(model, 1, ids, count, gg, ga, capacity=cap)
    torch.cuda.synchronize()
    used = np.concatenate([np.arange(200), np.arange(203, cap)])
    valid = lst[used]
    cg, ca = o3.current(1, valid)
    og, oa = out_g.cpu().numpy(), out_a.cpu().numpy()
    assert np.array_equal(bits(og[used]), bits(cg)) and np.array_equal(bits(oa[used]), bits(ca))
    assert np.all(og[200:203] == 7.0) and np.all(oa[200:203] == 7.0)   # skipped positions untouched
    o3.step(1, valid, gg.cpu().numpy()[used], ga.cpu().numpy()[used])
    st = model.state()
    for k, name in ((0, "geo"), (1, "app")):
        for part, ref in (("w", o3.w[k]), ("m", o3.m[k]), ("v", o3.v[k])):
            assert np.array_equal(bits(st[f"{name}_{part}"]), bits(ref)), f"{name}_{part}"
    assert np.array_equal(st["last_step"], o3.last_step(1))
    say(f"[edges] {valid.shape[0]} rows updated, 3 ids past the rows skipped, {lst.shape[0] - cap} beyond capacity")
