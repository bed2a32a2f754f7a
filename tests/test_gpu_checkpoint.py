"""Save -> flush -> load -> resume (run with -m gpu): a model flushed after
update t and rebuilt from its host copy (weights, moments, last steps, the
tables moved to step t+1 with gs_lut_seek) continues bit for bit like the
original; with chunk records too, which the load rebuilds tight."""
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


def _steps(g, model, n, t0, t1, cams, seed):
    ids = torch.zeros(n, dtype=torch.int32, device="cuda")
    count = torch.zeros(1, dtype=torch.int32, device="cuda")
    gg = torch.empty((n, 10), dtype=torch.float32, device="cuda")
    ga = torch.empty((n, 49), dtype=torch.float32, device="cuda")
    for t in range(t0, t1 + 1):
        g.gs_cull(model, cams[t - 1], t, ids, count)
        g.gs_synth_grad(seed, t, ids, count, gg, 0)
        g.gs_synth_grad(seed, t, ids, count, ga, 10)
        g.gs_adam_step_deferred(model, t, ids, count, gg, ga)
    torch.cuda.synchronize()


@pytest.mark.parametrize("layout,state,max_defer", [("fused", "f32", 0), ("fused", "bf16", 0), ("separate", "f32", 0),
                                                    ("fused", "f32", 15)])
def test_flush_save_load_resume_is_bit_exact(g, layout, state, max_defer):
    n, T, t_save = 60_000, 32, 7
    sc = gi.make_scene(n, seed=41)
    lg, la = gi.lr_columns()
    cams = gi.orbit_cameras(T, seed=42)
    kw = dict(max_steps=T, cull_mode=1, app_layout=layout, geo_state=state, app_state=state, sr_seed=3,
              max_defer=max_defer)
    a = g.Model(sc.geo, sc.app, lg, la, **kw)
    _steps(g, a, n, 1, t_save, cams, 5)
    g.gs_adam_flush(a, t_save)
    torch.cuda.synchronize()
    # checkpoint: host copies of every array of the state
    ckpt = a.state()
    # the original continues
    _steps(g, a, n, t_save + 1, T, cams, 5)
    # a new model (initial scene) loaded from the checkpoint: its arrays, its
    # cull summaries recomputed, the tables moved to the next update
    b = g.Model(sc.geo, sc.app, lg, la, **kw)
    b.load_state(ckpt, step=t_save + 1)
    _steps(g, b, n, t_save + 1, T, cams, 5)
    sa, sb = a.state(), b.state()
    for k in sa:
        assert sa[k].tobytes() == sb[k].tobytes(), k
    assert a.ws_header()["error"] == 0 and b.ws_header()["error"] == 0
    say(f"[checkpoint] {layout} {state} K={max_defer}: resumed at {t_save + 1}, bit-exact after step {T}")


def test_resume_with_chunk_records(g):
    """Rows in Morton order with chunk records: the loaded model's records are
    rebuilt tight from its summaries, and it continues bit for bit like the
    original, whose records were widened by every update since the start."""
    from test_gpu_chunks import CH, _scene, host_chunks, same_records
    n, T, t_save = 200_000, 24, 9
    geo, app, half = _scene(n, seed=43)
    lg, la = gi.lr_columns()
    lg = lg.copy()
    lg[0:3] = 2.0
    cams = gi.aerial_cameras(T, half, half, seed=44)
    kw = dict(max_steps=T, cull_mode=1, app_layout="fused", sr_seed=3, cull_chunks=True)
    a = g.Model(geo, app, lg, la, **kw)
    _steps(g, a, n, 1, t_save, cams, 5)
    g.gs_adam_flush(a, t_save)
    ckpt = a.state()
    _steps(g, a, n, t_save + 1, T, cams, 5)
    b = g.Model(geo, app, lg, la, **kw)
    b.load_state(ckpt, step=t_save + 1)
    torch.cuda.synchronize()
    assert b.cull_chunk is not None and b.cull_chunk.shape[0] == (n + CH - 1) // CH
    assert same_records(b.cull_chunk.cpu().numpy(), host_chunks(b.cull_sum[:n].cpu().numpy()))
    _steps(g, b, n, t_save + 1, T, cams, 5)
    sa, sb = a.state(), b.state()
    for k in sa:
        assert sa[k].tobytes() == sb[k].tobytes(), k
    assert a.ws_header()["error"] == 0 and b.ws_header()["error"] == 0
    say(f"[checkpoint chunks] resumed at {t_save + 1}, bit-exact after step {T}")
