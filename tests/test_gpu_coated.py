"""GPU parity of coated (electrochromic) panes: the device characteristic-matrix
evaluation against the FP64 oracle, fixture and room renders, and the
4M-triangle, 81-wavelength electrochromic room on 8 x 4 x 4 subdomains: its
full 3840 x 2160 frame at 1 spp (sampled pixels), and a 256 x 144 window of
that frame at the workload's 64 spp, plain and with the radiance cache,
against the oracle element by element."""
import numpy as np
import pytest

import oracle as ora
import scenegen as sg
from parity import ParityCtx, assert_parity, rel_err

pytestmark = pytest.mark.gpu

# FP32 evaluation of a five-layer characteristic-matrix product (complex
# square roots, sin/cos/exp of complex phases up to ~3 rad of absorption)
# against FP64: each of the ~60 rounded operations per layer and polarisation
# contributes ~6e-8 relative, amplified at most ~10x by the cancellation in
# 1 - R^2 tau^2 and the ratio forms; 2e-5 bounds it with margin and stays
# five times inside the 1e-4 radiance tolerance (measured: <= 5e-6).
GLASS_RTOL = 2e-5


@pytest.fixture(scope="module")
def tracer():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1912_06474_amd as m
    return m.Tracer()


def gpu_render(tracer, scene, W, H, spp, D, grid, seed=0):
    print(f"[gpu_render] {scene['name']} {W}x{H} spp={spp} D={D} grid={grid}", flush=True)
    tracer.load_scene(scene)
    tracer.build_bvh(*grid)
    hl = tracer.new_log(W, H, spp, D)
    sl = tracer.new_log(W, H, spp, D)
    tracer.trace_spectral(scene["camera"], W, H, spp, D, seed=seed, render_id=0, hit_log=hl, shadow_log=sl)
    s, x = tracer.resolve_image(0, W, H)
    out = dict(spectral=s.cpu().numpy(), xyz=x.cpu().numpy(), hit_log=hl.cpu().numpy(), shadow_log=sl.cpu().numpy())
    tracer.reset_render(0)
    return out


@pytest.mark.parametrize("state", [0.0, 0.5, 1.0])
def test_device_coated_glass_vs_oracle(tracer, state):
    sc = sg.lone_pane(n_lambda=41, coating_state=state)
    tracer.load_scene(sc)
    nl = len(sc["lambda_nm"])
    cos = np.array([1.0, 0.93, 0.7, 0.45, 0.2, 0.05, 0.01])
    L, C, S = np.meshgrid(np.arange(nl), cos, [1.0, -1.0], indexing="ij")
    lam_idx, cs = L.ravel().astype(np.int32), (C * S).ravel().astype(np.float32)
    R, T = tracer.debug_glass(np.zeros(len(cs), np.int32), lam_idx, cs)
    d = sc["mat_layer_d"][0].astype(np.float64)
    Ro = np.zeros(len(cs))
    To = np.zeros(len(cs))
    for i in range(len(cs)):
        l = int(lam_idx[i])
        Ro[i], To[i] = ora.coated_pane(float(sc["mat_n"][0, l]), float(sc["mat_k"][0, l]), float(sc["mat_thick"][0]),
                                       d, sc["mat_layer_n"][0, :, l].astype(np.float64),
                                       sc["mat_layer_k"][0, :, l].astype(np.float64), float(sc["lambda_nm"][l]),
                                       abs(float(cs[i])), bool(cs[i] > 0))
    er, et = rel_err(R, Ro), rel_err(T, To)
    print(f"[coated] state {state}: max rel R {er.max():.3e}, T {et.max():.3e}", flush=True)
    assert er.max() <= GLASS_RTOL
    assert et.max() <= GLASS_RTOL
    # the side matters for R (absorbing coating), not for T
    if state > 0:
        assert np.abs(R[cs > 0] - R[cs < 0]).max() > 1e-3


def test_device_uncoated_glass_unchanged(tracer):
    # a scene with no coating takes the slab terms (the same as sdd_debug_pane)
    sc = sg.lone_pane(n_lambda=16)
    tracer.load_scene(sc)
    cs = np.array([1.0, -0.6, 0.3], np.float32)
    R, T = tracer.debug_glass(np.zeros(3, np.int32), np.array([0, 5, 15], np.int32), cs)
    params = np.array([[sc["mat_n"][0, l], sc["mat_k"][0, l], sc["mat_thick"][0], sc["lambda_nm"][l], abs(c)]
                       for l, c in zip((0, 5, 15), cs)], np.float32)
    Rp, Tp = tracer.debug_pane(params)
    assert np.array_equal(R, Rp) and np.array_equal(T, Tp)


def test_coated_lone_pane_parity(tracer):
    sc = sg.lone_pane(n_lambda=41, coating_state=0.8)
    g = gpu_render(tracer, sc, 32, 32, 8, 2, (2, 2, 1))
    o = ora.render(sc, 32, 32, 8, 2, logs=True)
    assert_parity(g, o, ParityCtx(sc, 32, 32, 8, 2))


def test_coated_tiny_room_parity(tracer):
    sc = sg.tiny_room(coating_state=0.6)
    g = gpu_render(tracer, sc, 64, 64, 2, 6, (2, 2, 1), seed=3)
    o = ora.render(sc, 64, 64, 2, 6, logs=True, seed=3)
    assert_parity(g, o, ParityCtx(sc, 64, 64, 2, 6, seed=3))


@pytest.fixture(scope="module")
def c4():
    """The large electrochromic workload's scene and the oracle's view of it
    (its BVH is built once for every test here)."""
    sc = sg.electrochromic_room()
    print(f"[electrochromic] {len(sc['tris'])} tris, {len(sc['lambda_nm'])} lambda", flush=True)
    return sc, ora.OracleScene(sc)


C4_FRAME = (3840, 2160)
C4_CROP = (1376, 912, 256, 144)   # a window of the frame whose paths reach the panes
C4_GRID = (8, 4, 4)


def _crop_pixels(crop, W):
    x0, y0, cw, ch = crop
    ys, xs = np.meshgrid(np.arange(y0, y0 + ch), np.arange(x0, x0 + cw), indexing="ij")
    return (ys * W + xs).ravel().astype(np.int32)


def test_electrochromic_room_full_frame_sampled(tracer, c4):
    # the large workload's geometry, wavelengths, grid and frame; 1 spp keeps
    # the logs of every pixel within memory
    sc, osc = c4
    (W, H), spp, D = C4_FRAME, 1, 8
    g = gpu_render(tracer, sc, W, H, spp, D, C4_GRID)
    st = tracer.stats()
    assert st["overflow"] == 0
    rng = np.random.default_rng(11)
    pix = np.sort(rng.choice(W * H, 4096, replace=False)).astype(np.int32)
    o = ora.render(sc, W, H, spp, D, pix=pix, logs=True, oscene=osc)
    assert (o["spectral"].max(1) > 0).mean() > 0.03            # the sky reaches part of the frame
    assert_parity({k: v[pix] for k, v in g.items()}, o, ParityCtx(sc, W, H, spp, D, pix=pix, oscene=osc))
    assert np.isfinite(g["spectral"]).all() and (g["spectral"] >= 0).all()


def _crop_render(tracer, sc, spp, D, nrc=False):
    (W, H), (x0, y0, cw, ch) = C4_FRAME, C4_CROP
    hl = tracer.new_log(cw, ch, spp, D)
    sl = tracer.new_log(cw, ch, spp, D)
    print(f"[electrochromic] crop {C4_CROP} of {W}x{H}, {spp} spp, D={D}, cache={nrc}", flush=True)
    tracer.trace_spectral(sc["camera"], W, H, spp, D, render_id=0, hit_log=hl, shadow_log=sl, crop=C4_CROP,
                          nrc=nrc)
    s, x = tracer.resolve_image(0, cw, ch)
    out = dict(spectral=s.cpu().numpy(), xyz=x.cpu().numpy(), hit_log=hl.cpu().numpy(), shadow_log=sl.cpu().numpy())
    tracer.reset_render(0)
    return out


def test_electrochromic_crop_64spp_plain(tracer, c4):
    """The 256 x 144 window of the 3840 x 2160 frame at the workload's 64 spp,
    81 wavelengths, 4M triangles, 8 x 4 x 4 subdomains, against the oracle
    element by element."""
    sc, osc = c4
    (W, H), spp, D = C4_FRAME, 64, 8
    tracer.load_scene(sc)
    tracer.build_bvh(*C4_GRID)
    g = _crop_render(tracer, sc, spp, D)
    assert tracer.stats()["overflow"] == 0
    o = ora.render(sc, W, H, spp, D, crop=C4_CROP, logs=True, oscene=osc)
    glass = np.flatnonzero(np.asarray(sc["mat_type"])[np.asarray(sc["tri_mat"])] == sg.GLASS)
    n_glass = int(np.isin(o["hit_log"], glass).sum())
    lit = float((o["spectral"].max(1) > 0).mean())
    print(f"[electrochromic] crop: {n_glass} pane hits, {lit:.3f} of pixels lit", flush=True)
    assert n_glass > 0 and lit > 0.2
    assert_parity(g, o, ParityCtx(sc, W, H, spp, D, pix=_crop_pixels(C4_CROP, W), oscene=osc))


def test_electrochromic_crop_64spp_cache(tracer, c4):
    """The same window rendered with the radiance cache (a network built to
    evaluate a closed-form cache, so the oracle's estimator sees the same
    cache): logs, radiance and training rows against the oracle."""
    from test_gpu_nrc_render import COEF, HI, LO, _oracle_rows, affine_net
    sc, osc = c4
    (W, H), spp, D = C4_FRAME, 64, 8
    cw, ch = C4_CROP[2], C4_CROP[3]
    train_paths = 1 << 14
    tracer.load_scene(sc)
    tracer.build_bvh(*C4_GRID)
    params, tables = affine_net(COEF)
    tracer.nrc_init(params, tables, LO, HI, train_paths=train_paths, train_steps=0, precision="fp32")
    g = _crop_render(tracer, sc, spp, D, nrc=True)
    rows, _, _ = tracer.nrc_last_rows()
    stride = -(-(cw * ch * spp) // train_paths)
    o = ora.render(sc, W, H, spp, D, crop=C4_CROP, logs=True, oscene=osc,
                   nrc=dict(stride=stride, c=COEF, lo=LO, hi=HI))
    assert_parity(g, o, ParityCtx(sc, W, H, spp, D, pix=_crop_pixels(C4_CROP, W), oscene=osc))
    orows = _oracle_rows(o, cw, ch, spp)
    print(f"[electrochromic] cache crop: stride {stride}, {len(rows)} training rows (oracle {len(orows)})",
          flush=True)
    assert len(rows) == len(orows) and len(rows) > 0
    assert np.array_equal(rows[:, 3], orows[:, 4].astype(np.float32))
    assert np.abs(rows[:, 0:3] - orows[:, 1:4]).max() <= 1e-5
    t, to = rows[:, 7].astype(np.float64), orows[:, 8]
    assert (np.abs(t - to) / (np.abs(to) + 1e-6)).max() <= 1e-4
