"""The precision split, measured: the same renders through the library (FP64
per-path ray state and shading geometry, FP32 traversal and per-wavelength
transport) and through the FP32-path-state measurement build
(libsdd_f32state.so: state and shading geometry in FP32 too), each against
the FP64 oracle.  The library must meet the parity bar; the FP32-state
build's figures are what FP64 state buys.  Each build runs in a child process
of its own (tests/precision_split_render.py)."""
import os
import subprocess
import sys

import numpy as np
import pytest

import oracle as ora
from parity import ParityCtx, assert_parity, classify, report

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, HERE)
from precision_split_render import CASES, make_scene  # noqa: E402


def _render(case, state, path):
    env = dict(os.environ)
    env.pop("SDD_PATH_STATE", None)
    if state == "f32":
        env["SDD_PATH_STATE"] = "f32"
    print(f"[precision_split] {case}: {state} path state", flush=True)
    subprocess.run([sys.executable, os.path.join(HERE, "precision_split_render.py"), case, path], env=env,
                   check=True, timeout=400)
    d = np.load(path)
    return {k: d[k] for k in ("spectral", "xyz", "hit_log", "shadow_log")}, str(d["lib"])


@pytest.mark.parametrize("case", list(CASES))
def test_precision_split(case, tmp_path):
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    c = CASES[case]
    W, H, spp, D = c["W"], c["H"], c["spp"], c["D"]
    g64, lib64 = _render(case, "f64", str(tmp_path / "f64.npz"))
    g32, lib32 = _render(case, "f32", str(tmp_path / "f32.npz"))
    assert lib64.endswith("libsdd.so") and lib32.endswith("libsdd_f32state.so")
    sc = make_scene(case)
    osc = ora.OracleScene(sc)
    o = ora.render(sc, W, H, spp, D, crop=c["crop"], logs=True, oscene=osc)
    if c["crop"]:
        x0, y0, cw, ch = c["crop"]
        ys, xs = np.meshgrid(np.arange(y0, y0 + ch), np.arange(x0, x0 + cw), indexing="ij")
        pix = (ys * W + xs).ravel().astype(np.int32)
    else:
        pix = None
    r32 = report(g32, o)
    m = o["spectral"] > 1e-12
    rel32 = np.abs(g32["spectral"] - o["spectral"])[m] / o["spectral"][m]
    print(f"[precision_split] {case} FP32 state: hits {r32['hit_agree']:.6f}, shadows {r32['shadow_agree']:.6f}, "
          f"pixels with a differing slot {r32['excluded']} of {r32['n_pix']}, max rel error on matching pixels "
          f"{r32['max_rel']:.3e}, over 1e-4 {r32['n_over']}, max over all pixels {r32['max_err_all_pixels']:.3e}, "
          f"median rel error {float(np.median(rel32)):.3e}", flush=True)
    ctx = ParityCtx(sc, W, H, spp, D, pix=pix, oscene=osc)
    # where the FP32-state paths leave the oracle's, and by what FP64 margin
    diff = (g32["hit_log"] != o["hit_log"]) | (g32["shadow_log"] != o["shadow_log"])
    gone = diff.any(axis=2)
    if gone.any():
        first = np.bincount(np.argmax(diff, axis=2)[gone], minlength=D)
        rows = np.flatnonzero(gone.any(axis=1))[:60]
        ratios = np.array([x[4] for x in classify(ctx, g32, o, rows)])
        print(f"[precision_split] {case} FP32 state: {float(gone.mean()):.4f} of samples diverge; first differing "
              f"depth {first.tolist()}; FP64 margin / FP32 bound of the first divergence (quartiles of "
              f"{len(ratios)}) {np.quantile(ratios, [0.25, 0.5, 0.75]).round(3).tolist()}", flush=True)
    r64 = assert_parity(g64, o, ctx)
    rel64 = np.abs(g64["spectral"] - o["spectral"])[m] / o["spectral"][m]
    print(f"[precision_split] {case} FP64 state: hits {r64['hit_agree']:.6f}, shadows {r64['shadow_agree']:.6f}, "
          f"pixels with a differing slot {r64['excluded']} of {r64['n_pix']}, max rel error on matching pixels "
          f"{r64['max_rel']:.3e}, max over all pixels {r64['max_err_all_pixels']:.3e}, "
          f"median rel error {float(np.median(rel64)):.3e}", flush=True)
    # the builds differ in the path state only: the camera rays find the same
    # triangles, and the FP32-state image is finite and non-negative.  Its paths
    # leave the oracle's at later vertices: on faces whose normal has no z
    # component the FP32 cross product leaves rounding noise of either sign in
    # n.z, which picks the other branch of the cosine-sampling basis (its sign
    # s is +1 for n.z >= 0), so the same random numbers give another direction
    assert np.array_equal(g32["hit_log"][:, :, 0], o["hit_log"][:, :, 0])
    assert np.isfinite(g32["spectral"]).all() and (g32["spectral"] >= 0).all()
