"""Pins of the oracle's estimator where it is not a textbook formula.

Two parts of the FP64 oracle are iterations rather than closed forms, and
each is pinned here against what the mathematics fixes, not against itself:

* next-event estimation through glass (Eq. 3 with the shadow ray's pane
  transmittances): a point light seen by a diffuse wall only through two
  panes, one tilted, gives L = (rho / pi) I cos_x / r^2 * T_A * T_B per pixel,
  with the panes' T at the shadow ray's own cosine on each pane (Sec. 6, the
  Fresnel definition of the pane) and everything else computed here from the
  camera and the Philox numbers;
* the radiance-cache estimator (a path that is not a training path ends at
  its first diffuse vertex of depth >= 2, after that vertex's emission and
  light sample, adding beta * L_cache; a training path is traced in full and
  each continuing diffuse vertex of depth >= 2 gives a row whose target is
  the radiance its continuation carries back, at one wavelength):
  - furnace room (closed, every surface Lambertian rho and emitting L_e):
    constant cache c0 gives L_e (1 + rho) + rho^2 c0 on every non-training
    path, which is L_e / (1 - rho) when c0 = L_e / (1 - rho); the row of
    depth d carries L_e sum_{j < D - d} rho^j;
  - lit room with a pane: the zero cache equals the plain tracer stopped at
    the path's first diffuse vertex of depth >= 2 (same hits, same light
    samples); a constant cache adds exactly (product of the path's rho) * c0;
    a row's target equals (plain estimate at D - plain estimate at its depth)
    / (product of rho up to its vertex); every path training gives the plain
    render; training paths equal their plain paths.

Each check is chosen to fail on a plausible slip: R in place of T, one pane
dropped, the wall's cosine used at the tilted pane, the cache taken one vertex
early or before the light sample, beta missing on the cache term, the target
divided by the wrong throughput.
"""
import math

import numpy as np
import pytest

import oracle as ora
import scenegen as sg


# ---------------------------------------------------------------------------
# NEE through panes
# ---------------------------------------------------------------------------

def _pane_T(sc, m, l, c, coated_side):
    """Transmittance of glass material m at wavelength index l, incidence cosine c."""
    n, k = float(sc["mat_n"][m, l]), float(sc["mat_k"][m, l])
    th, lam = float(sc["mat_thick"][m]), float(sc["lambda_nm"][l])
    if "mat_n_layers" in sc and int(sc["mat_n_layers"][m]) > 0:
        L = int(sc["mat_n_layers"][m])
        return ora.coated_pane(n, k, th, sc["mat_layer_d"][m, :L], sc["mat_layer_n"][m, :L, l],
                               sc["mat_layer_k"][m, :L, l], lam, c, coated_side)[1]
    return ora.slab(n, k, th, lam, c)[1]


def _pane_planes(sc):
    """(point, unit geometric normal) of each pane quad, from its first triangle."""
    out = []
    glass = np.flatnonzero(sc["mat_type"][sc["tri_mat"]] == sg.GLASS)
    for t in glass[::2]:
        v = sc["verts"][sc["tris"][t]].astype(np.float64)
        n = np.cross(v[1] - v[0], v[2] - v[0])
        out.append((v[0], n / np.linalg.norm(n)))
    return out


@pytest.mark.parametrize("coating", [None, 0.7])
def test_nee_through_two_panes_is_eq3_times_slab_transmittances(coating):
    sc = sg.point_light_panes(16, seed=3, coating_state=coating)
    W = H = 12
    o = ora.render(sc, W, H, 1, 1, logs=True)
    assert (o["shadow_log"][:, 0, 0] == 1).all()          # every wall point sees the light
    nl = len(sc["lambda_nm"])
    rho = sc["mat_rho"][0].astype(np.float64)
    I = sc["mat_le"][sc["light_mat"]].astype(np.float64)
    light = sc["light_p0"].astype(np.float64)
    pane_m = int(np.flatnonzero(sc["mat_type"] == sg.GLASS)[0])
    planes = _pane_planes(sc)
    assert len(planes) == 2
    tilt_gap = 0.0
    for p in range(W * H):
        px, py = p % W, p // W
        u = [ora.u01(x) for x in ora.philox([p, 0, 0, 0], [0, 0])]
        org, d = ora.camera_ray(sc["camera"], W, H, px + u[0], py + u[1])
        t = -org[0] / d[0]                                  # the wall x = 0
        x = org + t * d
        xo = x + 1e-4 * np.array([1.0, 0.0, 0.0])           # origin offset toward the light's side
        wv = light - xo
        r2 = float(wv @ wv)
        om = wv / math.sqrt(r2)
        cos_x = om[0]
        T = np.ones(nl)
        for (q, n) in planes:
            c = abs(float(om @ n))
            for l in range(nl):
                T[l] *= _pane_T(sc, pane_m, l, c, float(om @ n) < 0.0)
        tilt_gap = max(tilt_gap, abs(abs(float(om @ planes[0][1])) - cos_x))
        expect = rho / math.pi * I * cos_x / r2 * T
        np.testing.assert_allclose(o["spectral"][p], expect, rtol=1e-12, atol=0)
    assert tilt_gap > 0.2          # the tilted pane's cosine differs from the wall's


# ---------------------------------------------------------------------------
# radiance-cache estimator: furnace room
# ---------------------------------------------------------------------------

def _flat_furnace(rho=0.625, le=1.5, n_lambda=16):
    sc = sg.furnace_room(0, n_lambda)
    sc["mat_rho"][:] = np.float32(rho)
    sc["mat_le"][:] = np.float32(le)
    return sc


def _nrc(stride, c0=0.0, c=(0, 0, 0), cn=(0, 0, 0)):
    return dict(stride=stride, c=[c0, *c, *cn], lo=(0.0, 0.0, 0.0), hi=sg.ROOM)


W8 = H8 = 8
SPP = 4


def _training(stride, W, H, spp):
    s, p = np.meshgrid(np.arange(spp), np.arange(W * H))
    return (s * W * H + p) % stride == 0                    # [pixel, sample]


@pytest.mark.parametrize("D", [2, 3, 6])
def test_furnace_constant_cache_returns_the_infinite_bounce_value(D):
    rho, le = 0.625, 1.5                                   # binary fractions: the tables hold them exactly
    sc = _flat_furnace(rho, le)
    stride = 7
    o = ora.render(sc, W8, H8, SPP, D, path_L=True, nrc=_nrc(stride, le / (1 - rho)))
    tr = _training(stride, W8, H8, SPP)
    full = le / (1 - rho)
    # a cache path: Le at vertex 1, rho Le at vertex 2, then rho^2 * Le / (1 - rho)
    np.testing.assert_allclose(o["path_L"][~tr], full, rtol=1e-14, atol=0)
    # a training path is the plain estimator: Le sum_{i<D} rho^i
    np.testing.assert_allclose(o["path_L"][tr], le * sum(rho ** i for i in range(D)), rtol=1e-14, atol=0)


def test_furnace_spectral_cache_term_carries_the_throughput():
    sc = sg.furnace_room(0, 16)
    rho = sc["mat_rho"][0].astype(np.float64)
    le = sc["mat_le"][0].astype(np.float64)
    c0 = 2.75
    o = ora.render(sc, W8, H8, SPP, 5, path_L=True, nrc=_nrc(5, c0))
    tr = _training(5, W8, H8, SPP)
    np.testing.assert_allclose(o["path_L"][~tr], (le * (1 + rho) + rho * rho * c0)[None, :].repeat((~tr).sum(), 0),
                               rtol=1e-13, atol=0)


@pytest.mark.parametrize("D", [3, 6])
def test_furnace_training_rows_carry_the_continuation(D):
    sc = sg.furnace_room(0, 16)
    rho = sc["mat_rho"][0].astype(np.float64)
    le = sc["mat_le"][0].astype(np.float64)
    lam = sc["lambda_nm"]
    stride = 3
    o = ora.render(sc, W8, H8, SPP, D, path_L=True, nrc=_nrc(stride, 1.0))
    tr = _training(stride, W8, H8, SPP)
    rows = o["nrc_rows"]                                    # [pix, spp, D-1, 9]
    n_rows = 0
    for p in range(W8 * H8):
        for s in range(SPP):
            for k in range(D - 1):
                r = rows[p, s, k]
                d = k + 2
                if not tr[p, s] or d >= D:
                    assert r[0] == 0.0
                    continue
                assert r[0] == 1.0                          # the furnace is closed: every path continues
                l = int(np.flatnonzero(lam == np.float32(r[4]))[0])
                want = le[l] * sum(rho[l] ** j for j in range(D - d))
                # the target is a difference of two path sums over rho^d: a few ulp of the sum, amplified
                tol = 64 * np.finfo(float).eps * le[l] * sum(rho[l] ** j for j in range(D)) / rho[l] ** d
                assert abs(r[8] - want) <= tol, (p, s, d, r[8], want)
                n_rows += 1
    assert n_rows == int(tr.sum()) * (D - 2)


# ---------------------------------------------------------------------------
# radiance-cache estimator: lit room with a pane
# ---------------------------------------------------------------------------

D_ROOM = 4
WR = HR = 16
SPPR = 2


@pytest.fixture(scope="module")
def room():
    sc = sg.tiny_room(0, 16)
    osc = ora.OracleScene(sc)
    plain = {Dp: ora.render(sc, WR, HR, SPPR, Dp, path_L=True, logs=True, oscene=osc) for Dp in (1, 2, 3, D_ROOM)}
    mt = sc["mat_type"][sc["tri_mat"]]
    return sc, osc, plain, mt


def _first_cache_depth(hl, mt):
    """Depth (1-based) of the first diffuse vertex of depth >= 2 in a hit log, or 0."""
    for d in range(2, len(hl) + 1):
        h = hl[d - 1]
        if h < 0:
            return 0
        if mt[h] == sg.DIFFUSE:
            return d
    return 0


def test_zero_cache_is_the_plain_tracer_stopped_at_the_cache_vertex(room):
    sc, osc, plain, mt = room
    stride = 1 << 30                                        # only path 0 trains
    o = ora.render(sc, WR, HR, SPPR, D_ROOM, path_L=True, logs=True, nrc=_nrc(stride, 0.0), oscene=osc)
    hl = plain[D_ROOM]["hit_log"]
    n_cut = 0
    for p in range(WR * HR):
        for s in range(SPPR):
            if p == 0 and s == 0:
                continue
            v = _first_cache_depth(hl[p, s], mt)
            if v:
                ref = plain[v]
                n_cut += 1
                assert (o["hit_log"][p, s, :v] == hl[p, s, :v]).all()
                assert (o["hit_log"][p, s, v:] == -2).all()
            else:
                ref = plain[D_ROOM]
                assert (o["hit_log"][p, s] == hl[p, s]).all()
            vd = v or D_ROOM
            assert (o["shadow_log"][p, s, :vd] == ref["shadow_log"][p, s, :vd]).all()
            assert (o["shadow_log"][p, s, vd:] == -2).all()
            assert np.array_equal(o["path_L"][p, s], ref["path_L"][p, s]), (p, s, v)
    assert n_cut > WR * HR * SPPR // 2
    # the light sample at the cache vertex matters: stopping before it would change these paths
    lit2 = (plain[2]["path_L"] != plain[1]["path_L"]).any(-1)
    assert lit2.sum() > 20


def test_constant_cache_adds_the_path_throughput_times_c(room):
    sc, osc, plain, mt = room
    stride = 1 << 30
    c0 = 1.7
    o0 = ora.render(sc, WR, HR, SPPR, D_ROOM, path_L=True, nrc=_nrc(stride, 0.0), oscene=osc)
    oc = ora.render(sc, WR, HR, SPPR, D_ROOM, path_L=True, nrc=_nrc(stride, c0), oscene=osc)
    hl = plain[D_ROOM]["hit_log"]
    rho = sc["mat_rho"].astype(np.float64)
    checked = 0
    for p in range(WR * HR):
        for s in range(SPPR):
            if p == 0 and s == 0:
                continue
            v = _first_cache_depth(hl[p, s], mt)
            prims = hl[p, s, :v]
            if not v or not (mt[prims] == sg.DIFFUSE).all():
                continue                                    # only all-diffuse prefixes: beta = prod rho
            beta = np.prod(rho[sc["tri_mat"][prims]], axis=0)
            np.testing.assert_allclose(oc["path_L"][p, s] - o0["path_L"][p, s], beta * c0, rtol=1e-12, atol=1e-300)
            checked += 1
    assert checked > WR * HR * SPPR // 2


def test_training_targets_are_the_continuation_over_the_throughput(room):
    sc, osc, plain, mt = room
    stride = 3
    o = ora.render(sc, WR, HR, SPPR, D_ROOM, path_L=True, logs=True, nrc=_nrc(stride, 5.0), oscene=osc)
    tr = _training(stride, WR, HR, SPPR)
    hl = plain[D_ROOM]["hit_log"]
    rho = sc["mat_rho"].astype(np.float64)
    lam = sc["lambda_nm"]
    checked = 0
    for p in range(WR * HR):
        for s in range(SPPR):
            if not tr[p, s]:
                continue
            # a training path is the plain path
            assert np.array_equal(o["path_L"][p, s], plain[D_ROOM]["path_L"][p, s])
            assert (o["hit_log"][p, s] == hl[p, s]).all()
            for d in range(2, D_ROOM):
                r = o["nrc_rows"][p, s, d - 2]
                h = hl[p, s, d - 1]
                cont = h >= 0 and mt[h] == sg.DIFFUSE and hl[p, s, d] != -2
                assert r[0] == (1.0 if cont else 0.0), (p, s, d)
                prims = hl[p, s, :d]
                if not cont or not (mt[prims] == sg.DIFFUSE).all():
                    continue
                l = int(np.flatnonzero(lam == np.float32(r[4]))[0])
                beta = float(np.prod(rho[sc["tri_mat"][prims], l]))
                want = (plain[D_ROOM]["path_L"][p, s, l] - plain[d]["path_L"][p, s, l]) / beta
                tol = 64 * np.finfo(float).eps * abs(plain[D_ROOM]["path_L"][p, s, l]) / beta
                assert abs(r[8] - want) <= tol, (p, s, d, r[8], want)
                checked += 1
    assert checked > 20


def test_every_path_training_is_the_plain_render(room):
    sc, osc, plain, _ = room
    o = ora.render(sc, WR, HR, SPPR, D_ROOM, path_L=True, logs=True, nrc=_nrc(1, 3.0), oscene=osc)
    assert np.array_equal(o["path_L"], plain[D_ROOM]["path_L"])
    assert np.array_equal(o["spectral"], plain[D_ROOM]["spectral"])
    assert np.array_equal(o["hit_log"], plain[D_ROOM]["hit_log"])


def test_window_render_traces_the_frame_pixels():
    """A window render (crop) traces each of its pixels as the frame does (same
    camera ray and random numbers); with the cache its training paths are
    numbered over the window: sample s of window pixel i is path s * n + i."""
    sc = sg.tiny_room(0, 16)
    W, H, spp, D = 32, 24, 3, 4
    crop = (5, 7, 11, 6)
    ys, xs = np.meshgrid(np.arange(7, 13), np.arange(5, 16), indexing="ij")
    pix = (ys * W + xs).ravel()
    a = ora.render(sc, W, H, spp, D, crop=crop, logs=True, path_L=True)
    b = ora.render(sc, W, H, spp, D, pix=pix, logs=True, path_L=True)
    assert np.array_equal(a["path_L"], b["path_L"]) and np.array_equal(a["hit_log"], b["hit_log"])
    n = len(pix)
    stride = 7
    c = ora.render(sc, W, H, spp, D, crop=crop, path_L=True, logs=True, nrc=_nrc(stride, 0.0))
    s, i = np.meshgrid(np.arange(spp), np.arange(n))
    train = (s * n + i) % stride == 0                     # [pixel, sample]
    # training paths are the plain ones; the others end at their cache vertex (zero cache here)
    assert np.array_equal(c["path_L"][train], a["path_L"][train])
    mt = sc["mat_type"][sc["tri_mat"]]
    cut = [(p, q) for p in range(n) for q in range(spp)
           if not train[p, q] and _first_cache_depth(a["hit_log"][p, q], mt) and
           _first_cache_depth(a["hit_log"][p, q], mt) < D]
    assert cut and all((c["hit_log"][p, q, _first_cache_depth(a["hit_log"][p, q], mt):] == -2).all() for p, q in cut)
