"""Parity metrics between the HIP path and the FP64 oracle (test helpers).

Hit agreement: fraction of (pixel, sample, depth) slots whose hit ids (and,
separately, shadow verdicts) are equal; slots after a divergence count as
mismatches unless both paths have ended.  Radiance: on pixels whose every
sample has identical hit and shadow logs, per-wavelength relative error of
the GPU's FP64-resolved mean against the oracle's FP64 mean; 0 == 0 exactly.

Excluded pixels (some sample's logs differ) are held to at most
max(1, 1e-4 n) of the n compared pixels.  A divergence that a near-tie
explains does not count against that bound: with a context (ParityCtx) the
oracle replays each diverged sample to its first differing depth and the
FP64 margin of the decision that split is measured there:

* a different hit: the distance (metres) from the ray's point on each
  candidate triangle's plane to that triangle's boundary, or the gap between
  the two candidates' t -- a near-tie when it is within the FP32 rounding
  bound 64 u32 S of the ray's and triangle's scale S = |o|_inf + t + the
  longest edge (u32 = 2^-24); or, if the previous vertex is a pane, the
  reflect/transmit draw within 1e-4 P_R + 1e-6 of P_R (P_R is an FP32 sum of
  per-wavelength terms each within 2e-5 of the FP64 ones);
* a different shadow verdict: the light-sample cosines within 64 u32 of 0 (a
  ray shot on one side only), or an opaque triangle whose crossing by the
  shadow segment is decided within 64 u32 S (grazing an edge, or t within
  that distance of either end).

The report also gives the largest relative error over all pixels, excluded
ones included.
"""
import numpy as np

HIT_AGREE_MIN = 0.9999       # >= 99.99% identical hit ids
REL_TOL = 1e-4               # per-pixel spectral radiance, relative to FP64
EXCLUDED_MAX_FRAC = 1e-4     # unexplained excluded pixels, of all compared pixels
U32 = 2.0 ** -24
TIE_ULPS = 64.0              # FP32 decision bound, in units of u32 times the operands' scale
BRANCH_REL, BRANCH_ABS = 1e-4, 1e-6
DIFFUSE, EMITTER = 0, 2


def hit_agreement(a, b):
    a = np.asarray(a)
    b = np.asarray(b)
    assert a.shape == b.shape, (a.shape, b.shape)
    return float((a == b).mean())


def matching_pixels(g, o):
    """Pixels whose every sample has identical hit and shadow logs."""
    hl = (g["hit_log"] == o["hit_log"]).reshape(len(g["hit_log"]), -1).all(1)
    sl = (g["shadow_log"] == o["shadow_log"]).reshape(len(g["shadow_log"]), -1).all(1)
    return hl & sl


def rel_err(gpu, ora):
    gpu = np.asarray(gpu, np.float64)
    ora = np.asarray(ora, np.float64)
    err = np.abs(gpu - ora)
    den = np.abs(ora)
    out = np.where(den > 0, err / np.where(den > 0, den, 1.0), np.where(err == 0, 0.0, np.inf))
    return out


def report(g, o):
    hits = hit_agreement(g["hit_log"], o["hit_log"])
    sh = hit_agreement(g["shadow_log"], o["shadow_log"])
    m = matching_pixels(g, o)
    re = rel_err(g["spectral"][m], o["spectral"][m]) if m.any() else np.zeros(1)
    rex = rel_err(g["xyz"][m], o["xyz"][m]) if m.any() else np.zeros(1)
    # all pixels, relative to the pixel's largest value (a diverged path changes a pixel by a sample's share)
    sc = np.maximum(np.abs(o["spectral"]).max(axis=1, keepdims=True), 1e-300)
    re_all = np.abs(g["spectral"] - o["spectral"]) / sc
    return dict(hit_agree=hits, shadow_agree=sh, excluded=int((~m).sum()), n_pix=int(len(m)),
                max_rel=float(re.max()), max_rel_xyz=float(rex.max()),
                n_over=int((re > REL_TOL).sum()), max_err_all_pixels=float(re_all.max()))


# ---------------------------------------------------------------------------
# near-tie classification of divergences
# ---------------------------------------------------------------------------

class ParityCtx:
    """What the oracle needs to replay a comparison's path samples: the scene
    (as rendered, e.g. with a photochromic substitution applied), the frame,
    the Philox key, the first sample index and, for a subset of pixels, the
    frame pixel index of each compared row."""

    def __init__(self, scene, W, H, spp, D, camera=None, seed=0, render_id=0, sample_offset=0, pix=None,
                 oscene=None):
        import oracle as ora
        self.ora = ora
        self.scene, self.W, self.H, self.spp, self.D = scene, W, H, spp, D
        self.camera = camera or scene["camera"]
        self.seed, self.render_id, self.sample_offset = seed, render_id, sample_offset
        self.pix = None if pix is None else np.asarray(pix, np.int64)
        self.osc = oscene or ora.OracleScene(scene)
        v = np.asarray(scene["verts"], np.float64)
        self.tv = v[np.asarray(scene["tris"])]                       # [T, 3, 3]
        self.tmat = np.asarray(scene["mat_type"])[np.asarray(scene["tri_mat"])]

    def frame_pixel(self, i):
        return int(self.pix[i]) if self.pix is not None else int(i)


def _plane_margins(tv, o, d):
    """For triangles tv [k, 3, 3] and a ray (o, d): t of the ray's point on each
    triangle's plane and the signed distance (metres) from that point to the
    triangle's boundary (> 0 inside, < 0 outside); the longest edges."""
    e1 = tv[:, 1] - tv[:, 0]
    e2 = tv[:, 2] - tv[:, 0]
    n = np.cross(e1, e2)
    den = n @ d
    with np.errstate(divide="ignore", invalid="ignore"):
        t = np.einsum("kj,kj->k", n, tv[:, 0] - o) / den
    P = o + t[:, None] * d
    dist = np.full(len(tv), np.inf)
    for a, b, c in ((0, 1, 2), (1, 2, 0), (2, 0, 1)):
        eb = tv[:, b] - tv[:, a]
        m = np.cross(n, eb)
        sgn = np.sign(np.einsum("kj,kj->k", m, tv[:, c] - tv[:, a]))
        with np.errstate(divide="ignore", invalid="ignore"):
            dd = sgn * np.einsum("kj,kj->k", m, P - tv[:, a]) / np.linalg.norm(m, axis=1)
        dist = np.minimum(dist, dd)
    edge = np.max(np.stack([np.linalg.norm(tv[:, 1] - tv[:, 0], axis=1), np.linalg.norm(tv[:, 2] - tv[:, 1], axis=1),
                            np.linalg.norm(tv[:, 0] - tv[:, 2], axis=1)]), axis=0)
    t = np.where(np.abs(den) > 0, t, np.inf)
    dist = np.where(np.isfinite(dist), dist, -np.inf)
    return t, dist, edge


def _hit_margin(ctx, pr, gp, op):
    """Margin / bound of a differing closest hit (ratio <= 1: a near-tie)."""
    o, d = pr[0:3], pr[3:6]
    cand = [p for p in (gp, op) if p >= 0]
    if not cand:
        return np.inf
    t, dist, edge = _plane_margins(ctx.tv[cand], o, d)
    S = np.max(np.abs(o)) + np.abs(t) + edge
    eps = TIE_ULPS * U32 * S
    ratio = np.minimum(np.abs(dist), np.abs(t)) / eps   # grazing an edge, or a hit at the ray's start
    best = float(np.min(np.where(np.isfinite(ratio), ratio, np.inf)))
    if len(cand) == 2 and np.all(dist > -eps) and np.all(np.isfinite(t)):
        best = min(best, float(abs(t[0] - t[1]) / max(eps)))     # two candidates at (nearly) the same t
    return best


def _branch_margin(pr_prev):
    u, PR = pr_prev[7], pr_prev[8]
    if not (np.isfinite(u) and np.isfinite(PR)):
        return np.inf
    return float(abs(u - PR) / (BRANCH_REL * PR + BRANCH_ABS))


def _shadow_margin(ctx, pr, prim, g_sh, o_sh):
    xo, w, r, cx, cy = pr[9:12], pr[12:15], pr[15], pr[16], pr[17]
    if not np.isfinite(r):
        return np.inf
    eps_c = TIE_ULPS * U32
    if g_sh == -2 or o_sh == -2:                    # a ray on one side only: a cosine at 0
        return float(min(abs(cx), abs(cy)) / eps_c)
    opaque = np.flatnonzero(ctx.tmat == DIFFUSE)
    opaque = opaque[opaque != prim]
    t, dist, edge = _plane_margins(ctx.tv[opaque], xo, w)
    S = np.max(np.abs(xo)) + r + edge
    eps = TIE_ULPS * U32 * S
    flip = np.minimum(np.minimum(np.abs(dist), np.abs(t)), np.abs(r - t)) / eps  # distance to a changed verdict
    if o_sh == 0:                                   # blocked for the oracle: every blocker must be marginal
        blocking = np.isfinite(t) & (t > 0) & (t < r) & (dist >= 0)
        return float(np.max(flip[blocking])) if blocking.any() else np.inf
    near = np.isfinite(t) & (t > -eps) & (t < r + eps) & (dist > -eps)
    return float(np.min(flip[near])) if near.any() else np.inf   # visible: some triangle barely missed


def classify(ctx, g, o, rows):
    """For the excluded rows, the list of (row, sample, depth, kind, margin /
    bound) of every diverged sample at its first differing depth."""
    items = []
    for i in rows:
        for s in range(g["hit_log"].shape[1]):
            gh, oh = g["hit_log"][i, s], o["hit_log"][i, s]
            gs, os_ = g["shadow_log"][i, s], o["shadow_log"][i, s]
            diff = np.flatnonzero((gh != oh) | (gs != os_))
            if len(diff):
                items.append((int(i), s, int(diff[0])))
    if not items:
        return []
    pix = np.array([ctx.frame_pixel(i) for i, _, _ in items], np.int32)
    smp = np.array([ctx.sample_offset + s for _, s, _ in items], np.int32)
    probe = ctx.ora.probe_paths(ctx.scene, ctx.W, ctx.H, ctx.D, pix, smp, camera=ctx.camera, seed=ctx.seed,
                                render_id=ctx.render_id, oscene=ctx.osc)
    out = []
    for n, (i, s, k) in enumerate(items):
        gh, oh = int(g["hit_log"][i, s, k]), int(o["hit_log"][i, s, k])
        if gh != oh:
            m = _hit_margin(ctx, probe[n, k], gh, oh) if min(gh, oh) >= -1 else np.inf
            if k >= 1:
                m = min(m, _branch_margin(probe[n, k - 1]))
            out.append((i, s, k, "hit", m))
        else:
            m = _shadow_margin(ctx, probe[n, k], oh, int(g["shadow_log"][i, s, k]), int(o["shadow_log"][i, s, k]))
            out.append((i, s, k, "shadow", m))
    return out


def assert_parity(g, o, ctx=None, excluded_max=None):
    r = report(g, o)
    assert r["hit_agree"] >= HIT_AGREE_MIN, r
    assert r["shadow_agree"] >= HIT_AGREE_MIN, r
    lim = excluded_max if excluded_max is not None else max(1, int(EXCLUDED_MAX_FRAC * r["n_pix"]))
    unexplained = r["excluded"]
    if ctx is not None and r["excluded"]:
        m = matching_pixels(g, o)
        items = classify(ctx, g, o, np.flatnonzero(~m))
        bad_rows = sorted({i for (i, _, _, _, ratio) in items if not ratio <= 1.0})
        unexplained = len(bad_rows)
        r["near_tie_pixels"] = r["excluded"] - unexplained
        r["max_margin_ratio"] = float(max(x[4] for x in items)) if items else 0.0
        r["divergences"] = [(i, s, k, kind, round(float(x), 4)) for (i, s, k, kind, x) in items[:12]]
    r["unexplained"] = unexplained
    print("parity:", r, flush=True)
    assert unexplained <= lim, r
    assert r["max_rel"] <= REL_TOL, r
    assert r["max_rel_xyz"] <= REL_TOL, r
    return r
