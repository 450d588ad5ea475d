"""GPU parity at the room-scale workload, in the launch configuration the
benchmark times: about 200k triangles, three 4 mm panes, 41 wavelengths,
512 x 512 pixels, 16 samples per pixel, up to 8 vertices, 4 x 4 x 2
subdomains, one batch of 4.19M paths.

The whole frame is traced once on the GPU with hit and shadow logs; the FP64
oracle then renders (a) a seeded sample of pixels spread over the frame and
(b) a contiguous crop around the window panes, and both are held to the same
rules as the small scenes.  Properties that hold at any size (log structure,
ray counts against the logs, finite non-negative radiance, the XYZ reduction)
are checked on every pixel.
"""
import numpy as np
import pytest

import oracle as ora
import scenegen as sg
from parity import ParityCtx, assert_parity, rel_err

pytestmark = pytest.mark.gpu

W = H = 512
SPP, D = 16, 8
GRID = (4, 4, 2)


@pytest.fixture(scope="module")
def frame():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1912_06474_amd as m
    sc = sg.furnished_room(seed=1, n_lambda=41)
    tr = m.Tracer()
    tr.load_scene(sc)
    tr.build_bvh(*GRID)
    print(f"[room_scale] {len(sc['tris'])} tris, {W}x{H} x {SPP} spp, D={D}, grid={GRID}", flush=True)
    hl = tr.new_log(W, H, SPP, D)
    sl = tr.new_log(W, H, SPP, D)
    tr.reset_stats()
    tr.trace_spectral(sc["camera"], W, H, SPP, D, render_id=0, hit_log=hl, shadow_log=sl)
    s, x = tr.resolve_image(0, W, H)
    st = tr.stats()
    g = dict(spectral=s.cpu().numpy(), xyz=x.cpu().numpy(), hit_log=hl.cpu().numpy(), shadow_log=sl.cpu().numpy())
    del hl, sl, s, x
    tr.reset_render(0)
    print(f"[room_scale] traced: {st['ext_rays']} extension + {st['shadow_rays']} shadow rays, "
          f"batches {st['batches']}, overflow {st['overflow']}", flush=True)
    return sc, g, st


def _sub(g, pix):
    return {k: v[pix] for k, v in g.items()}


def test_room_scale_sampled_pixels_parity(frame):
    sc, g, st = frame
    assert st["overflow"] == 0 and st["batches"] == 1
    rng = np.random.default_rng(7)
    pix = np.sort(rng.choice(W * H, 8192, replace=False)).astype(np.int32)
    o = ora.render(sc, W, H, SPP, D, pix=pix, logs=True)
    assert_parity(_sub(g, pix), o, ParityCtx(sc, W, H, SPP, D, pix=pix))


def test_room_scale_window_crop_parity(frame):
    sc, g, _ = frame
    # 64 x 64 crop on the far wall, around the few pixels that see a pane directly
    ys, xs = np.meshgrid(np.arange(252, 316), np.arange(268, 332), indexing="ij")
    pix = (ys * W + xs).ravel().astype(np.int32)
    o = ora.render(sc, W, H, SPP, D, pix=pix, logs=True)
    n_glass = int(np.isin(o["hit_log"], np.flatnonzero(
        np.asarray(sc["mat_type"])[np.asarray(sc["tri_mat"])] == sg.GLASS)).sum())
    print(f"[room_scale] crop: {n_glass} pane hits", flush=True)
    assert n_glass > 0
    assert_parity(_sub(g, pix), o, ParityCtx(sc, W, H, SPP, D, pix=pix))


def test_room_scale_log_structure_and_ray_counts(frame):
    sc, g, st = frame
    hl, sl = g["hit_log"], g["shadow_log"]
    T = len(sc["tris"])
    assert hl.min() >= -2 and hl.max() < T
    assert set(np.unique(sl)).issubset({-2, 0, 1})
    # a path that has ended stays ended; a miss ends it
    ended = hl == -2
    assert not (ended[..., :-1] & ~ended[..., 1:]).any()
    assert not ((hl[..., :-1] == -1) & ~ended[..., 1:]).any()
    assert (hl[..., 0] != -2).all()
    # every live slot is one traced extension ray, every verdict one shadow ray
    assert st["ext_rays"] == int((hl != -2).sum())
    assert st["shadow_rays"] == int((sl >= 0).sum())
    # a shadow verdict only at a surface vertex that was hit
    assert not ((sl >= 0) & (hl < 0)).any()


def test_room_scale_radiance_properties(frame):
    sc, g, _ = frame
    s, x = g["spectral"], g["xyz"]
    assert np.isfinite(s).all() and (s >= 0).all()
    # the sky is seen only through three small panes behind dense furniture, so
    # most pixels stay dark at 16 spp; a lit minority must exist
    assert (s.max(1) > 0).mean() > 0.05
    w = np.asarray(sc["lambda_w"], np.float64)
    cmf = np.asarray(sc["cmf"], np.float64)
    expect = s @ (w[:, None] * cmf)
    err = rel_err(x, expect)
    assert float(np.where(np.abs(expect) > 1e-12, err, 0).max()) <= 1e-12
