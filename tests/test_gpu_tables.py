"""The deferred-update tables on the device (run with -m gpu): each update
moves the restore rows to the next step on the GPU, bit for bit as the host
advance (and so as the oracle's tables, test_abi); calls out of sequence, or
graph replays past the last step the tables cover, set the tables' error word
and store nothing."""
import sys

import numpy as np
import pytest
import torch

import gs_inputs as gi
import lut_layout as LL

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def g():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2509_15645_amd import gsdp
    return gsdp


def _run_steps(g, model, n, steps, seed=0):
    cams = gi.orbit_cameras(steps, seed=seed)
    ids = torch.zeros(n, dtype=torch.int32, device="cuda")
    count = torch.zeros(1, dtype=torch.int32, device="cuda")
    gg = torch.empty((n, 10), dtype=torch.float32, device="cuda")
    ga = torch.empty((n, model.adim), dtype=torch.float32, device="cuda")
    for t in range(1, steps + 1):
        g.gs_cull(model, cams[t - 1], t, ids, count)
        g.gs_synth_grad(seed, t, ids, count, gg, 0)
        g.gs_synth_grad(seed, t, ids, count, ga, 10)
        g.gs_adam_step_deferred(model, t, ids, count, gg, ga)
    torch.cuda.synchronize()
    return ids, count, gg, ga


@pytest.mark.parametrize("optimizer,max_defer", [("adam", 0), ("adam", 15), ("adamw", 0), ("sgd_momentum", 15)])
def test_device_advance_equals_host_advance(g, optimizer, max_defer):
    n, T, steps = 20_000, 40, 23
    sc = gi.make_scene(n, seed=3)
    lg, la = gi.lr_columns()
    kw = dict(weight_decay=0.02) if optimizer == "adamw" else {}
    model = g.Model(sc.geo, sc.app, lg, la, max_steps=T, max_defer=max_defer, optimizer=optimizer, **kw)
    host = model.lut.cpu().numpy().view(np.uint8).copy()      # the tables of step 1
    _run_steps(g, model, n, steps)
    dev = model.lut.cpu().numpy().view(np.uint8)
    g.gs_lut_seek_host(host, steps + 1)
    nclass = int(host[16:20].view(np.int32)[0])
    vd, vh = LL.views(dev, T, max_defer, nclass), LL.views(host, T, max_defer, nclass)
    t = steps + 1
    dmax = min(t - 1, max_defer) if max_defer else t - 1
    assert vd["hdr"][t & 1] == t and vd["hdr"][5] == 0
    for key in ("Wf", "Wd"):
        assert np.array_equal(vd[key][t & 1, :dmax + 1], vh[key][t & 1, :dmax + 1]), key
    for c in range(nclass):
        for key in ("Wlf", "Pf"):
            assert np.array_equal(vd["cls"][c][key][t & 1, :dmax + 1], vh["cls"][c][key][t & 1, :dmax + 1])
    say(f"[tables] {optimizer} K={max_defer}: device rows of step {t} equal the host advance")


def test_calls_out_of_sequence_set_the_error_and_store_nothing(g):
    n = 20_000
    sc = gi.make_scene(n, seed=4)
    lg, la = gi.lr_columns()
    model = g.Model(sc.geo, sc.app, lg, la, max_steps=8)
    ids, count, gg, ga = _run_steps(g, model, n, 2)
    assert model.ws_header()["error"] == 0
    before = model.state()
    # the tables hold step 3: an update or a flush of another step is refused on the device
    g.gs_adam_step_deferred(model, 5, ids, count, gg, ga)
    g.gs_adam_flush(model, 4)
    torch.cuda.synchronize()
    assert model.lut_header()["error"] == 1
    after = model.state()
    for key in before:
        assert before[key].tobytes() == after[key].tobytes(), key
    assert sorted(model.lut_header()["t_row"]) == [2, 3]


def test_graph_replay_past_the_tables_sets_the_error_and_stores_nothing(g):
    """A device step counter beyond max_steps (a captured step replayed too
    often) is flagged, not clamped: nothing is stored."""
    n = 20_000
    sc = gi.make_scene(n, seed=5)
    lg, la = gi.lr_columns()
    model = g.Model(sc.geo, sc.app, lg, la, max_steps=4)
    ids, count, gg, ga = _run_steps(g, model, n, 4)
    before = model.state()
    model.step_dev.fill_(5)
    g.gs_adam_step_deferred(model, 0, ids, count, gg, ga)
    torch.cuda.synchronize()
    assert model.lut_header()["error"] & 2
    after = model.state()
    for key in before:
        assert before[key].tobytes() == after[key].tobytes(), key
