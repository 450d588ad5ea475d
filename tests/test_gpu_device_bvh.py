"""GPU-built subdomain BVHs (sdd_bvh_desc.device_build): a linear BVH per cell
from Morton-sorted reference centroids.  Closest hits do not depend on the
BVH, so the device build is pinned by hits equal to brute force and to the
host SAH build, and by the render parity the host build already meets."""
import time

import numpy as np
import pytest

import oracle as ora
import scenegen as sg
from parity import ParityCtx, assert_parity, hit_agreement

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def tracer():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1912_06474_amd as m
    return m.Tracer()


def _rays(n, seed, lo=(0.1, 0.1, 0.1), hi=(3.9, 2.9, 2.4)):
    rng = np.random.default_rng(seed)
    o = rng.uniform(lo, hi, size=(n, 3))
    d = rng.normal(size=(n, 3))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    return o.astype(np.float32), d.astype(np.float32)


@pytest.mark.parametrize("grid,leaf", [((1, 1, 1), 4), ((2, 2, 1), 4), ((4, 4, 2), 1), ((5, 3, 3), 8)])
def test_device_bvh_hits_equal_brute_force(tracer, grid, leaf):
    sc = sg.tiny_room()
    tracer.load_scene(sc)
    tracer.build_bvh(*grid, leaf_max=leaf, device=True)
    st = tracer.stats()
    print(f"[device_bvh] grid {grid} leaf {leaf}: refs {st['n_refs']}, nodes {st['n_nodes']}, "
          f"depth {st['max_bvh_depth']}", flush=True)
    o, d = _rays(20000, 1)
    t, prim = tracer.debug_trace_rays(o, d)
    tb, pb = ora.trace_rays(sc, o.astype(np.float64), d.astype(np.float64), use_bvh=False)
    agree = hit_agreement(prim, pb)
    assert agree >= 0.9999, agree
    tracer.build_bvh(*grid, leaf_max=leaf)
    th, ph = tracer.debug_trace_rays(o, d)
    assert np.array_equal(prim, ph)
    assert np.array_equal(t, th)


def test_device_bvh_render_parity(tracer):
    sc = sg.tiny_room()
    W = H = 64
    tracer.load_scene(sc)
    tracer.build_bvh(2, 2, 1, device=True)
    hl = tracer.new_log(W, H, 2, 5)
    sl = tracer.new_log(W, H, 2, 5)
    tracer.trace_spectral(sc["camera"], W, H, 2, 5, seed=2, render_id=0, hit_log=hl, shadow_log=sl)
    s, x = tracer.resolve_image(0, W, H)
    tracer.reset_render(0)
    g = dict(spectral=s.cpu().numpy(), xyz=x.cpu().numpy(), hit_log=hl.cpu().numpy(), shadow_log=sl.cpu().numpy())
    o = ora.render(sc, W, H, 2, 5, logs=True, seed=2)
    assert_parity(g, o, ParityCtx(sc, W, H, 2, 5, seed=2))


@pytest.mark.parametrize("which", ["furnished_room", "electrochromic_room"])
def test_device_bvh_room_scale_hits_and_build_time(tracer, which):
    sc = getattr(sg, which)()
    grid = (4, 4, 2) if which == "furnished_room" else (8, 4, 4)
    tracer.load_scene(sc)
    t0 = time.perf_counter()
    tracer.build_bvh(*grid)
    host_s = time.perf_counter() - t0
    o, d = _rays(200000, 7)
    th, ph = tracer.debug_trace_rays(o, d)
    st_h = tracer.stats()
    tracer.build_bvh(*grid, device=True)  # first device build also loads the code objects
    t0 = time.perf_counter()
    tracer.build_bvh(*grid, device=True)
    dev_s = time.perf_counter() - t0
    st_d = tracer.stats()
    td, pd = tracer.debug_trace_rays(o, d)
    print(f"[device_bvh] {which}: host build {host_s:.3f} s ({st_h['n_refs']} refs, {st_h['n_nodes']} nodes, "
          f"depth {st_h['max_bvh_depth']}); device build {dev_s:.3f} s ({st_d['n_refs']} refs, "
          f"{st_d['n_nodes']} nodes, depth {st_d['max_bvh_depth']})", flush=True)
    assert st_d["n_refs"] == st_h["n_refs"]
    assert np.array_equal(pd, ph)
    assert np.array_equal(td, th)


@pytest.mark.parametrize("grid,leaf,boxes", [((8, 8, 8), 1, 0), ((8, 8, 8), 4, 3), ((6, 5, 4), 2, 1)])
def test_widened_trees_of_sparse_cells(tracer, grid, leaf, boxes):
    """Both builders' binary trees are widened to 4-wide nodes on the device.
    A fine grid over a sparse room gives the degenerate cases of the widening:
    empty cells, cells whose root is one leaf (a wrapper node), one-triangle
    leaves and trees of odd depth.  Hits must equal brute force either way."""
    sc = sg.tiny_room(0, 16, n_boxes=boxes)
    tracer.load_scene(sc)
    o, d = _rays(20000, 7)
    to, po = ora.trace_rays(sc, o.astype(np.float64), d.astype(np.float64), use_bvh=False)
    results = []
    for device in (False, True):
        tracer.build_bvh(*grid, leaf_max=leaf, device=device)
        st = tracer.stats()
        print(f"[widen] grid {grid} leaf {leaf} boxes {boxes} device {device}: refs {st['n_refs']}, "
              f"4-wide nodes {st['n_nodes']}, binary depth {st['max_bvh_depth']}", flush=True)
        assert st["n_nodes"] >= st["n_cells"]  # at least a root per cell, empty cells included
        t, prim = tracer.debug_trace_rays(o, d)
        assert hit_agreement(prim, po) >= 0.9999
        m = (prim == po) & (po >= 0)
        assert np.all(np.abs(t[m] - to[m]) <= 1e-5 * np.maximum(1.0, to[m]))
        results.append((t, prim))
    assert np.array_equal(results[0][1], results[1][1])
