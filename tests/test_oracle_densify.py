"""Pins of the oracle's densification (Sec. 2.4 step 7, the 3DGS procedure):

  * a staged torch reference in 3DGS's own order -- append clones, append
    split children and drop their parents, then prune -- gives the same rows
    in the same order (ids and kinds exact; values to FP32 rounding, with the
    child rotation taken from scipy);
  * identities: with no gradient above threshold and nothing to prune the
    output is the input bit for bit; clones are bit copies of their parents;
  * split children: scale = parent / 1.6, and over many draws the child
    offsets have mean 0 and covariance R diag(sigma^2) R^T (scipy rotation);
  * the normal-approximation draws have mean 0 and variance 1.
"""
import numpy as np
import pytest
import torch
from scipy.spatial.transform import Rotation

import gs_inputs as gi
from oracle import oracle as orc

INV_SD = 1.0 / np.sqrt(4.0 * (65536.0 * 65536.0 - 1.0) / 12.0)


def draws(seed, rows, child):
    """z[len(rows), 3] of the split children, from the SplitMix64 stream."""
    out = np.zeros((len(rows), 3), np.float32)
    for a in range(3):
        h = gi.splitmix_at(gi.splitmix_at(gi.splitmix_at(np.uint64(seed), np.asarray(rows, np.uint64)),
                                          np.uint64(child)), np.uint64(a))
        u = sum(((h >> np.uint64(16 * k)) & np.uint64(0xffff)).astype(np.float64) for k in range(4))
        out[:, a] = ((u - 131070.0) * INV_SD).astype(np.float32)
    return out


def _stats(n, seed, frac=0.3):
    rng = np.random.default_rng(seed)
    accum = np.where(rng.random(n) < frac, rng.uniform(3e-4, 1e-3, n), rng.uniform(0, 1e-4, n)).astype(np.float32)
    denom = rng.integers(0, 3, n).astype(np.float32)
    return accum * np.maximum(denom, 1), denom


def _scene(n, seed):
    s = gi.make_scene(n, seed=seed, box=((-10, 10), (-10, 10), (-10, 10)))
    geo, app = s.geo.copy(), s.app.copy()
    rng = np.random.default_rng(seed + 1)
    app[:, 0] = rng.normal(-2.0, 3.0, n).astype(np.float32)      # some below logit(0.005)
    geo[:, 3:6] += rng.normal(0, 1.0, (n, 3)).astype(np.float32)  # some large scales
    return geo, app


def staged_3dgs(geo, app, accum, denom, extent, pd=0.01, min_op=0.005, seed=0):
    """3DGS's densify-and-prune in its own order, with torch tensors."""
    G = torch.tensor(geo, dtype=torch.float64)
    A = torch.tensor(app, dtype=torch.float64)
    ids = torch.arange(G.shape[0])
    kind = torch.zeros(G.shape[0], dtype=torch.int64)
    grads = torch.tensor(np.where(denom > 0, accum / np.where(denom > 0, denom, 1), 0.0), dtype=torch.float64)
    smax = torch.exp(G[:, 3:6]).max(1).values
    # clone
    sel = (grads >= 2e-4) & (smax <= pd * extent)
    G, A = torch.cat([G, G[sel]]), torch.cat([A, A[sel]])
    ids, kind = torch.cat([ids, ids[sel]]), torch.cat([kind, torch.ones(int(sel.sum()), dtype=torch.int64)])
    # split (padded gradients: the clones have none)
    gpad = torch.cat([grads, torch.zeros(int(sel.sum()), dtype=torch.float64)])
    smax = torch.exp(G[:, 3:6]).max(1).values
    sel = (gpad >= 2e-4) & (smax > pd * extent)
    parents = ids[sel].numpy()
    kids_g, kids_a, kids_id, kids_k = [], [], [], []
    for j in range(2):
        z = torch.tensor(draws(seed, parents, j), dtype=torch.float64)
        sig = torch.exp(G[sel][:, 3:6])
        rot = torch.tensor(Rotation.from_quat(G[sel][:, [7, 8, 9, 6]].numpy()).as_matrix())
        off = torch.einsum("nab,nb->na", rot, sig * z)
        kg = G[sel].clone()
        kg[:, :3] = kg[:, :3] + off
        kg[:, 3:6] = torch.log(sig / 1.6)
        kids_g.append(kg); kids_a.append(A[sel]); kids_id.append(ids[sel])
        kids_k.append(torch.full((int(sel.sum()),), 2 + j, dtype=torch.int64))
    # children interleave per parent: child 0 then child 1
    kg = torch.stack(kids_g, 1).reshape(-1, 10)
    ka = torch.stack(kids_a, 1).reshape(-1, A.shape[1])
    kid = torch.stack(kids_id, 1).reshape(-1)
    kk = torch.stack(kids_k, 1).reshape(-1)
    keep = ~sel
    G = torch.cat([G[keep], kg]); A = torch.cat([A[keep], ka])
    ids = torch.cat([ids[keep], kid]); kind = torch.cat([kind[keep], kk])
    # prune: low opacity, large in world space
    low = torch.sigmoid(A[:, 0]) < min_op
    big = torch.exp(G[:, 3:6]).max(1).values > 0.1 * extent
    keep = ~(low | big)
    return G[keep].numpy(), A[keep].numpy(), ids[keep].numpy(), kind[keep].numpy()


@pytest.mark.parametrize("seed", [0, 1])
def test_matches_staged_3dgs_reference(seed):
    n, extent = 3000, 30.0
    geo, app = _scene(n, seed)
    accum, denom = _stats(n, seed + 10)
    og, oa, src, kind, counts = orc.densify(geo, app, accum, denom, extent=extent, seed=seed + 5)
    rg, ra, rid, rk = staged_3dgs(geo, app, accum, denom, extent, seed=seed + 5)
    assert counts[0] > 0 and counts[1] > 0 and counts[2] > 0
    assert og.shape[0] == rg.shape[0] == counts.sum()
    assert np.array_equal(src, rid) and np.array_equal(kind, rk)
    assert np.allclose(og, rg, rtol=2e-6, atol=2e-6)
    assert np.array_equal(oa, ra.astype(np.float32))


def test_identity_and_clone_copies():
    n = 2000
    geo, app = _scene(n, 3)
    zero = np.zeros(n, np.float32)
    og, oa, src, kind, c = orc.densify(geo, app, zero, zero, extent=1e9, min_opacity=1e-38, prune_big=False)
    assert np.array_equal(src, np.arange(n)) and not kind.any()
    assert np.array_equal(og.view(np.uint32), geo.view(np.uint32)) and np.array_equal(oa, app)
    accum, denom = _stats(n, 4)
    og, oa, src, kind, c = orc.densify(geo, app, accum, denom, extent=1e9, min_opacity=1e-38, prune_big=False)
    cl = kind == 1
    assert cl.any() and np.array_equal(og[cl].view(np.uint32), geo[src[cl]].view(np.uint32))


def test_split_children_distribution():
    n = 40000
    rng = np.random.default_rng(7)
    g0 = np.array([1.0, -2.0, 3.0, -1.0, -0.5, -2.0, 0.0, 0.0, 0.0, 0.0], np.float32)
    q = rng.normal(size=4)
    g0[6:10] = q / np.linalg.norm(q)
    geo = np.tile(g0, (n, 1))
    app = np.zeros((n, 49), np.float32)
    accum = np.ones(n, np.float32); denom = np.ones(n, np.float32)
    og, oa, src, kind, c = orc.densify(geo, app, accum, denom, extent=1.0, prune_big=False, seed=11)
    assert c[2] == 2 * n and og.shape[0] == 2 * n
    off = og[:, :3].astype(np.float64) - g0[:3]
    sig = np.exp(g0[3:6].astype(np.float64))
    R = Rotation.from_quat(g0[[7, 8, 9, 6]]).as_matrix()
    cov = R @ np.diag(sig ** 2) @ R.T
    emp = np.cov(off.T)
    se = np.sqrt(2.0 / off.shape[0]) * np.sqrt(np.outer(np.diag(cov), np.diag(cov)))
    assert np.all(np.abs(emp - cov) < 6 * se)
    assert np.all(np.abs(off.mean(0)) < 6 * np.sqrt(np.diag(cov) / off.shape[0]))
    assert np.allclose(np.exp(og[:, 3:6].astype(np.float64)), sig / 1.6, rtol=1e-6)


def test_draws_have_unit_variance():
    z = draws(3, np.arange(200000), 1)
    assert abs(z.mean()) < 0.01 and abs(z.var() - 1.0) < 0.01
