"""The near-tie rule of the parity helper (tests/parity.py), on the CPU.

The GPU keeps its path state in FP64 and rounds only the current ray to FP32
for traversal, so it can leave the oracle's path only where an FP32 decision
on that ray differs from the FP64 one.  Here such decisions are produced on
purpose: rays aimed within 1e-8..3e-7 m of edges shared by two triangles, and
shadow segments grazing an occluder's edge, decided once in FP64 (the
oracle's brute force) and once by a float32 Moller-Trumbore on the FP32
rounding of the ray.  Every disagreement must be a near-tie by the rule's
margins, and a planted genuine mismatch must not be.
"""
import numpy as np
import pytest

import oracle as ora
import scenegen as sg
from parity import ParityCtx, _hit_margin, _shadow_margin, assert_parity, classify, matching_pixels


def _fp32_hits(tv32, o, d, t_max=None):
    """float32 Moller-Trumbore of one ray against every triangle: (hit mask, t)."""
    o = np.asarray(o, np.float32)
    d = np.asarray(d, np.float32)
    v0 = tv32[:, 0]
    e1 = tv32[:, 1] - v0
    e2 = tv32[:, 2] - v0
    p = np.cross(d[None, :], e2)
    det = np.einsum("kj,kj->k", e1, p)
    with np.errstate(divide="ignore", invalid="ignore"):
        inv = np.float32(1.0) / det
        s = o[None, :] - v0
        u = np.einsum("kj,kj->k", s, p) * inv
        q = np.cross(s, e1)
        v = (q @ d) * inv
        t = np.einsum("kj,kj->k", e2, q) * inv
    ok = (det != 0) & (u >= 0) & (u <= 1) & (v >= 0) & (u + v <= 1) & (t > 0)
    if t_max is not None:
        ok &= t < np.float32(t_max)
    return ok, t


def _shared_edges(tris):
    edges = {}
    for i, tri in enumerate(tris):
        for a, b in ((0, 1), (1, 2), (2, 0)):
            key = tuple(sorted((int(tri[a]), int(tri[b]))))
            edges.setdefault(key, []).append(i)
    return [(k, v) for k, v in edges.items() if len(v) == 2]


@pytest.fixture(scope="module")
def room():
    sc = sg.tiny_room(0, 16)
    ctx = ParityCtx(sc, 16, 16, 1, 4)
    tv32 = np.asarray(sc["verts"], np.float32)[np.asarray(sc["tris"])]
    return sc, ctx, tv32


def test_fp32_edge_decisions_are_near_ties(room):
    sc, ctx, tv32 = room
    rng = np.random.default_rng(1)
    verts = np.asarray(sc["verts"], np.float64)
    pairs = _shared_edges(sc["tris"])
    O, Dd = [], []
    for _ in range(3000):
        (a, b), (t0, t1) = pairs[rng.integers(len(pairs))]
        P = verts[a] + rng.uniform(0.05, 0.95) * (verts[b] - verts[a])
        n = ctx.tv[t0]
        nrm = np.cross(n[1] - n[0], n[2] - n[0])
        nrm /= np.linalg.norm(nrm)
        side = np.cross(nrm, verts[b] - verts[a])
        side /= np.linalg.norm(side)
        P = P + side * rng.choice([-1, 1]) * 10 ** rng.uniform(-8, -6.5)   # just off the shared edge
        w = nrm * rng.choice([-1, 1]) + 0.6 * rng.normal(size=3)
        w /= np.linalg.norm(w)
        org = P + w * rng.uniform(0.5, 3.0)
        O.append(org)
        Dd.append((P - org) / np.linalg.norm(P - org))
    O, Dd = np.array(O), np.array(Dd)
    t64, p64 = ora.trace_rays(sc, O, Dd, use_bvh=False, oscene=ctx.osc)
    n_diff, worst = 0, 0.0
    for i in range(len(O)):
        ok, t = _fp32_hits(tv32, O[i].astype(np.float32), Dd[i].astype(np.float32))
        tt = np.where(ok, t, np.inf)
        p32 = int(np.argmin(tt)) if ok.any() else -1
        if p32 == int(p64[i]):
            continue
        n_diff += 1
        pr = np.concatenate([O[i], Dd[i], [-1.0]])
        r = _hit_margin(ctx, pr, p32, int(p64[i]))
        worst = max(worst, r)
        assert r <= 1.0, (i, p32, int(p64[i]), r)
    print(f"[parity rule] {n_diff} of {len(O)} edge rays decided differently in FP32; worst ratio {worst:.3f}")
    assert n_diff >= 20


def test_fp32_grazing_shadow_segments_are_near_ties(room):
    sc, ctx, tv32 = room
    rng = np.random.default_rng(2)
    verts = np.asarray(sc["verts"], np.float64)
    opaque = np.flatnonzero(ctx.tmat == 0)
    X, Wv, R = [], [], []
    for _ in range(3000):
        k = int(opaque[rng.integers(len(opaque))])
        tri = ctx.tv[k]
        a, b = rng.choice(3, 2, replace=False)
        P = tri[a] + rng.uniform(0.05, 0.95) * (tri[b] - tri[a])
        nrm = np.cross(tri[1] - tri[0], tri[2] - tri[0])
        nrm /= np.linalg.norm(nrm)
        side = np.cross(nrm, tri[b] - tri[a])
        side /= np.linalg.norm(side)
        P = P + side * rng.choice([-1, 1]) * 10 ** rng.uniform(-8, -6.5)
        w = nrm + 0.5 * rng.normal(size=3)
        w /= np.linalg.norm(w)
        x0 = P - w * rng.uniform(0.3, 1.5)
        r = np.linalg.norm(P - x0) + rng.uniform(0.3, 1.5)
        X.append(x0)
        Wv.append(w)
        R.append(r)
    X, Wv, R = np.array(X), np.array(Wv), np.array(R)
    T = ora.shadow_rays(sc, X, Wv, R, use_bvh=False, oscene=ctx.osc)
    vis64 = T.max(axis=1) > 0          # panes transmit; only an opaque triangle makes T zero
    glass_or_light = ctx.tmat != 0
    n_diff, worst = 0, 0.0
    for i in range(len(X)):
        ok, _ = _fp32_hits(tv32, X[i].astype(np.float32), Wv[i].astype(np.float32), R[i])
        vis32 = not (ok & ~glass_or_light).any()
        if vis32 == bool(vis64[i]):
            continue
        n_diff += 1
        pr = np.full(18, np.nan)
        pr[9:12], pr[12:15], pr[15], pr[16], pr[17] = X[i], Wv[i], R[i], 1.0, 1.0
        r = _shadow_margin(ctx, pr, -1, int(vis32), int(vis64[i]))
        worst = max(worst, r)
        assert r <= 1.0, (i, vis32, bool(vis64[i]), r)
    print(f"[parity rule] {n_diff} of {len(X)} grazing segments decided differently in FP32; worst ratio {worst:.3f}")
    assert n_diff >= 20


def test_a_genuine_mismatch_is_not_a_near_tie():
    sc = sg.tiny_room(0, 16)
    W = H = 16
    spp, D = 2, 4
    o = ora.render(sc, W, H, spp, D, logs=True)
    ctx = ParityCtx(sc, W, H, spp, D)
    g = {k: np.array(v, copy=True) for k, v in o.items() if isinstance(v, np.ndarray)}
    assert matching_pixels(g, o).all()
    # two paths that take a far-away triangle at their second vertex
    live = np.argwhere(o["hit_log"][:, :, 1] >= 0)
    for (p, s) in live[[3, 40]]:
        h = o["hit_log"][p, s, 1]
        g["hit_log"][p, s, 1] = (h + 500) % len(sc["tris"])
    items = classify(ctx, g, o, np.flatnonzero(~matching_pixels(g, o)))
    assert len(items) == 2 and all(x[4] > 1.0 for x in items), items
    with pytest.raises(AssertionError):
        assert_parity(g, o, ctx)          # two unexplained pixels: above max(1, 1e-4 n)
