"""GPU parity: the HIP path (through the C ABI) against the FP64 oracle."""
import os

import numpy as np
import pytest

import oracle as ora
import scenegen as sg
from parity import HIT_AGREE_MIN, REL_TOL, ParityCtx, assert_parity, hit_agreement, rel_err

pytestmark = pytest.mark.gpu

GOLD = os.path.join(os.path.dirname(__file__), "golden")


@pytest.fixture(scope="module")
def sdd():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1912_06474_amd as m
    return m


@pytest.fixture(scope="module")
def tracer(sdd):
    return sdd.Tracer()


def gpu_render(tracer, scene, W, H, spp, D, grid=(1, 1, 1), camera=None, seed=0, sample_offset=0, render_id=0,
               leaf_max=4):
    print(f"[gpu_render] {scene['name']} {W}x{H} spp={spp} D={D} grid={grid}", flush=True)
    tracer.load_scene(scene)
    tracer.build_bvh(*grid, leaf_max=leaf_max)
    cam = camera or scene["camera"]
    hl = tracer.new_log(W, H, spp, D)
    sl = tracer.new_log(W, H, spp, D)
    tracer.trace_spectral(cam, W, H, spp, D, seed=seed, sample_offset=sample_offset, render_id=render_id,
                          hit_log=hl, shadow_log=sl)
    s, x = tracer.resolve_image(render_id, W, H)
    return dict(spectral=s.cpu().numpy(), xyz=x.cpu().numpy(), hit_log=hl.cpu().numpy(),
                shadow_log=sl.cpu().numpy())


def test_device_philox_matches_rocrand_vectors(tracer):
    rows = [list(map(int, l.split())) for l in open(os.path.join(GOLD, "philox_kat.txt")) if not l.startswith("#")]
    for v in rows:
        out = tracer.debug_philox(np.array([v[0:4]], np.uint32), np.array(v[4:6], np.uint32))
        assert list(out[0]) == v[6:10]


def test_device_philox_equals_oracle_on_many_counters(tracer):
    rng = np.random.default_rng(1)
    ctr = rng.integers(0, 2 ** 32, size=(1 << 16, 4), dtype=np.uint64).astype(np.uint32)
    key = np.array([7, 3], np.uint32)
    out = tracer.debug_philox(ctr, key)
    for i in range(0, len(ctr), 997):
        assert list(out[i]) == list(ora.philox(ctr[i], key))


def test_device_pane_terms_vs_oracle(tracer):
    rng = np.random.default_rng(4)
    n = 4000
    params = np.column_stack([rng.uniform(1.2, 2.4, n), 10 ** rng.uniform(-8, -0.3, n), rng.uniform(0.0, 0.01, n),
                              rng.uniform(380, 780, n), rng.uniform(0.0, 1.0, n)]).astype(np.float32)
    params[:50, 1] = 0.0                       # lossless
    params[50:100, 4] = 1.0                    # normal incidence
    params[100:150, 4] = 0.0                   # grazing
    params[150:200, 0], params[150:200, 1] = 0.2, 3.0   # conductor-like
    R, T = tracer.debug_pane(params)
    for i in range(n):
        q = [float(x) for x in params[i]]
        Ro, To = ora.slab(*q)
        assert abs(R[i] - Ro) <= 2e-6 + 2e-5 * Ro, (i, q, R[i], Ro)
        assert abs(T[i] - To) <= 2e-6 + 2e-5 * To, (i, q, T[i], To)


@pytest.mark.parametrize("grid", [(1, 1, 1), (2, 2, 1), (4, 4, 2), (3, 5, 2)])
def test_closest_hits_vs_brute_force(tracer, grid):
    sc = sg.tiny_room()
    tracer.load_scene(sc)
    tracer.build_bvh(*grid)
    rng = np.random.default_rng(2)
    n = 20000
    o = rng.uniform([0.05, 0.05, 0.05], [3.95, 2.95, 2.45], size=(n, 3)).astype(np.float32)
    d = rng.normal(size=(n, 3))
    d = (d / np.linalg.norm(d, axis=1, keepdims=True)).astype(np.float32)
    t, prim = tracer.debug_trace_rays(o, d)
    to, po = ora.trace_rays(sc, o.astype(np.float64), d.astype(np.float64), use_bvh=False)
    agree = float((prim == po).mean())
    print("closest-hit agreement", grid, agree, flush=True)
    assert agree >= HIT_AGREE_MIN
    m = (prim == po) & (po >= 0)
    assert np.all(np.abs(t[m] - to[m]) <= 1e-5 * np.maximum(1.0, to[m]))


def test_ray_plane_analytic_hits_gpu(tracer):
    sc = sg.floor_plane()
    tracer.load_scene(sc)
    tracer.build_bvh(2, 2, 1)
    rng = np.random.default_rng(11)
    n = 20000
    o = np.column_stack([rng.uniform(-1, 5, n), rng.uniform(-1, 4, n), rng.uniform(0.2, 3, n)])
    tgt = np.column_stack([rng.uniform(0.02, 3.98, n), rng.uniform(0.02, 2.98, n), np.zeros(n)])
    d = tgt - o
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    t, prim = tracer.debug_trace_rays(o.astype(np.float32), d.astype(np.float32))
    of, df = o.astype(np.float32).astype(np.float64), d.astype(np.float32).astype(np.float64)
    t_plane = -of[:, 2] / df[:, 2]
    assert np.all(prim >= 0)
    assert np.allclose(t, t_plane, rtol=2e-6)
    x = of + t_plane[:, None] * df
    i, j = np.floor(x[:, 0]).astype(int), np.floor(x[:, 1]).astype(int)
    fx, fy = x[:, 0] - i, x[:, 1] - j
    away = (np.abs(fx - fy) > 1e-5) & (fx > 1e-5) & (fx < 1 - 1e-5) & (fy > 1e-5) & (fy < 1 - 1e-5)
    expect = 2 * (j * 4 + i) + (fy > fx).astype(int)
    assert np.array_equal(prim[away], expect[away])


def test_tiny_room_parity(tracer):
    sc = sg.tiny_room()
    g = gpu_render(tracer, sc, 64, 64, 1, 4, grid=(2, 2, 1))
    o = ora.render(sc, 64, 64, 1, 4, logs=True)
    assert_parity(g, o, ParityCtx(sc, 64, 64, 1, 4))


def test_tiny_room_parity_more_samples(tracer):
    sc = sg.tiny_room()
    g = gpu_render(tracer, sc, 48, 40, 4, 6, grid=(2, 2, 1), seed=5)
    o = ora.render(sc, 48, 40, 4, 6, logs=True, seed=5)
    assert_parity(g, o, ParityCtx(sc, 48, 40, 4, 6, seed=5))


def test_decomposition_invariance(tracer):
    sc = sg.tiny_room()
    ref = None
    for grid in [(1, 1, 1), (2, 2, 1), (4, 4, 2), (5, 3, 3)]:
        g = gpu_render(tracer, sc, 48, 48, 2, 4, grid=grid)
        if ref is None:
            ref = g
            continue
        same = hit_agreement(g["hit_log"], ref["hit_log"])
        print("decomposition", grid, same, flush=True)
        assert same >= 0.9999
        if same == 1.0:
            assert np.array_equal(g["spectral"], ref["spectral"])


def test_furnace_gpu_closed_form(tracer):
    sc = sg.furnace_room()
    D = 5
    g = gpu_render(tracer, sc, 32, 32, 2, D, grid=(2, 2, 1))
    rho = sc["mat_rho"][0].astype(np.float64)
    le = sc["mat_le"][0].astype(np.float64)
    expect = le * (1 - rho ** D) / (1 - rho)
    ok = (g["hit_log"] >= 0).reshape(len(g["hit_log"]), -1).all(1)
    assert ok.mean() >= 0.999
    err = rel_err(g["spectral"][ok], np.broadcast_to(expect, g["spectral"][ok].shape))
    assert err.max() <= 1e-5


@pytest.mark.parametrize("which", ["point_light_plane", "area_light_plane", "lone_pane"])
def test_fixture_parity(tracer, which):
    sc = getattr(sg, which)()
    W = H = 32
    spp, D = 4, 2
    g = gpu_render(tracer, sc, W, H, spp, D, grid=(2, 2, 1))
    o = ora.render(sc, W, H, spp, D, logs=True)
    assert_parity(g, o, ParityCtx(sc, W, H, spp, D))


@pytest.mark.parametrize("coating", [None, 0.7])
def test_point_light_through_panes_parity(tracer, coating):
    """Light samples through two panes (one tilted), plain and coated: the
    oracle's result here is pinned to Eq. 3 times the panes' transmittances."""
    sc = sg.point_light_panes(16, seed=3, coating_state=coating)
    W = H = 32
    spp, D = 2, 3
    g = gpu_render(tracer, sc, W, H, spp, D, grid=(2, 2, 2))
    o = ora.render(sc, W, H, spp, D, logs=True)
    assert (g["shadow_log"][:, :, 0] == 1).all()
    assert_parity(g, o, ParityCtx(sc, W, H, spp, D))


def test_sample_split_and_batching_are_bitwise_identical(tracer):
    sc = sg.tiny_room()
    W = H = 32
    tracer.load_scene(sc)
    tracer.build_bvh(2, 2, 1)
    cam = sc["camera"]
    # render_id keys Philox, so every variant reuses render 1 after a reset
    tracer.trace_spectral(cam, W, H, 3, 4, render_id=1)
    a, _ = tracer.resolve_image(1, W, H)
    tracer.reset_render(1)
    tracer.trace_spectral(cam, W, H, 1, 4, render_id=1)
    tracer.trace_spectral(cam, W, H, 2, 4, render_id=1, sample_offset=1)
    b, _ = tracer.resolve_image(1, W, H)
    assert np.array_equal(a.cpu().numpy(), b.cpu().numpy())
    tracer.reset_render(1)
    old = os.environ.get("SDD_MEM_BUDGET_GB")
    os.environ["SDD_MEM_BUDGET_GB"] = "0.0005"
    try:
        tracer.reset_stats()
        tracer.trace_spectral(cam, W, H, 3, 4, render_id=1)
        c, _ = tracer.resolve_image(1, W, H)
        assert tracer.stats()["batches"] > 3
    finally:
        if old is None:
            del os.environ["SDD_MEM_BUDGET_GB"]
        else:
            os.environ["SDD_MEM_BUDGET_GB"] = old
    assert np.array_equal(a.cpu().numpy(), c.cpu().numpy())


def test_run_to_run_bitwise(tracer):
    sc = sg.tiny_room()
    a = gpu_render(tracer, sc, 40, 40, 2, 4, grid=(2, 2, 1))
    b = gpu_render(tracer, sc, 40, 40, 2, 4, grid=(2, 2, 1))
    for k in ("spectral", "xyz", "hit_log", "shadow_log"):
        assert np.array_equal(a[k], b[k])


def test_work_counters_leave_the_render_unchanged(tracer):
    """Counting traversal work changes only the counters; every lane-level
    count lies between its wave-level step count and 64 times it.  A frame
    several times the wave count makes lanes refill from their work items."""
    sc = sg.tiny_room()
    W, H, spp, D = 96, 64, 4, 4
    a = gpu_render(tracer, sc, W, H, spp, D, grid=(2, 2, 1))
    tracer.reset_render(0)  # the same render again (its random numbers are keyed by the render id)
    hl = tracer.new_log(W, H, spp, D)
    sl = tracer.new_log(W, H, spp, D)
    tracer.reset_stats()
    tracer.trace_spectral(sc["camera"], W, H, spp, D, render_id=0, hit_log=hl, shadow_log=sl, count_work=True)
    s, x = tracer.resolve_image(0, W, H)
    st = tracer.stats()
    tracer.reset_render(0)
    assert np.array_equal(a["spectral"], s.cpu().numpy()) and np.array_equal(a["xyz"], x.cpu().numpy())
    assert np.array_equal(a["hit_log"], hl.cpu().numpy()) and np.array_equal(a["shadow_log"], sl.cpu().numpy())
    for lanes, steps in (("node_visits", "wave_node_steps"), ("tri_tests", "wave_tri_steps")):
        assert 0 < st[steps] <= st[lanes] <= 64 * st[steps], (lanes, st[lanes], st[steps])
    print(f"[count] node loop {st['node_visits'] / (64 * st['wave_node_steps']):.3f}, "
          f"leaf loop {st['tri_tests'] / (64 * st['wave_tri_steps']):.3f} of lanes busy", flush=True)


def test_xyz_is_weighted_cmf_sum(tracer):
    sc = sg.tiny_room()
    g = gpu_render(tracer, sc, 16, 16, 1, 3, grid=(2, 2, 1))
    w = sc["lambda_w"][:, None] * sc["cmf"]
    assert np.allclose(g["xyz"], g["spectral"] @ w, rtol=1e-12, atol=1e-15)


def test_edge_shapes(tracer):
    sc = sg.tiny_room()
    for (W, H, spp, D) in [(1, 1, 1, 1), (3, 1, 2, 1), (1, 7, 1, 3), (65, 33, 1, 2)]:
        g = gpu_render(tracer, sc, W, H, spp, D, grid=(2, 2, 1))
        o = ora.render(sc, W, H, spp, D, logs=True)
        assert_parity(g, o, ParityCtx(sc, W, H, spp, D))


def test_error_paths(sdd):
    t = sdd.Tracer()
    cam = dict(eye=(2, 0.5, 1.2), target=(2, 3, 1.2), fov_deg=70.0)
    with pytest.raises(sdd.SddError) as e:
        t.trace_spectral(cam, 8, 8, 1, 2)
    assert e.value.status == -2
    with pytest.raises(sdd.SddError) as e:
        t.build_bvh(2, 2, 1)
    assert e.value.status == -2
    t.load_scene(sg.tiny_room())
    with pytest.raises(sdd.SddError) as e:
        t.build_bvh(0, 1, 1)
    assert e.value.status == -1
    t.build_bvh(2, 2, 1)
    with pytest.raises(sdd.SddError) as e:
        t.trace_spectral(cam, 0, 8, 1, 2)
    assert e.value.status == -1
    with pytest.raises(sdd.SddError) as e:
        t.trace_spectral(dict(eye=(2, 0.5, 1.2), target=(2, 0.5, 3.0), fov_deg=70.0), 8, 8, 1, 2)
    assert e.value.status == -1
    with pytest.raises(sdd.SddError) as e:
        t.resolve_image(42, 8, 8)
    assert e.value.status == -2
    t.close()


def test_overflow_flag_is_per_render_and_names_its_cause(sdd):
    """A shadow segment through five panes (more than the four tracked) marks
    the renders of that call only: another render of the same context, and a
    render after a new scene, resolve cleanly; the statistics keep the bit
    until they are reset."""
    t = sdd.Tracer()
    sc = sg.point_light_panes(16, seed=3, extra_panes=3)   # every wall point's shadow segment crosses 5 panes
    t.load_scene(sc)
    t.build_bvh(2, 2, 1)
    W = H = 16
    print("[overflow] 5-pane render, D=1", flush=True)
    t.trace_spectral(sc["camera"], W, H, 1, 1, render_id=5)
    with pytest.raises(sdd.SddError, match="more than 4 glass panes") as e:
        t.resolve_image(5, W, H)
    assert e.value.status == -5
    assert t.stats()["overflow"] == 1
    # looking down onto the pane stack with one vertex per path: no shadow rays
    top = dict(eye=(1.5, 1.5, 4.5), target=(1.5, 1.6, 0.0), fov_deg=20.0)
    t.trace_spectral(top, W, H, 1, 1, render_id=6)
    s6, _ = t.resolve_image(6, W, H)
    assert np.isfinite(s6.cpu().numpy()).all()
    with pytest.raises(sdd.SddError, match="more than 4 glass panes"):
        t.resolve_image(5, W, H)                            # still marked
    t.reset_stats()
    assert t.stats()["overflow"] == 0
    # a new scene: its renders start clean
    t.load_scene(sg.point_light_panes(16, seed=3))
    t.build_bvh(2, 2, 1)
    t.trace_spectral(sc["camera"], W, H, 1, 1, render_id=5)
    s5, _ = t.resolve_image(5, W, H)
    assert (s5.cpu().numpy() > 0).any()
    assert t.stats()["overflow"] == 0
    t.close()


def test_window_render_equals_the_frame_render(tracer):
    """A window of the frame (sdd_trace_desc crop) traces its pixels exactly as
    the whole-frame render does: same camera rays and random numbers, so the
    same logs and the same radiance bit for bit; and it matches the oracle's
    window render."""
    sc = sg.tiny_room()
    W, H, spp, D = 64, 48, 2, 4
    crop = (9, 17, 23, 13)
    full = gpu_render(tracer, sc, W, H, spp, D, grid=(2, 2, 1))
    tracer.reset_render(0)          # the window render takes the same render id (the same Philox key)
    hl = tracer.new_log(crop[2], crop[3], spp, D)
    sl = tracer.new_log(crop[2], crop[3], spp, D)
    tracer.trace_spectral(sc["camera"], W, H, spp, D, render_id=0, hit_log=hl, shadow_log=sl, crop=crop)
    s, x = tracer.resolve_image(0, crop[2], crop[3])
    tracer.reset_render(0)
    ys, xs = np.meshgrid(np.arange(crop[1], crop[1] + crop[3]), np.arange(crop[0], crop[0] + crop[2]), indexing="ij")
    pix = (ys * W + xs).ravel()
    assert np.array_equal(s.cpu().numpy(), full["spectral"][pix])
    assert np.array_equal(hl.cpu().numpy(), full["hit_log"][pix])
    assert np.array_equal(sl.cpu().numpy(), full["shadow_log"][pix])
    o = ora.render(sc, W, H, spp, D, crop=crop, logs=True)
    g = dict(spectral=s.cpu().numpy(), xyz=x.cpu().numpy(), hit_log=hl.cpu().numpy(), shadow_log=sl.cpu().numpy())
    assert_parity(g, o, ParityCtx(sc, W, H, spp, D, pix=pix))
    import paper_1912_06474_amd as m
    for bad in ((60, 0, 5, 5), (0, 0, 0, 5), (-1, 0, 4, 4)):
        with pytest.raises(m.SddError, match="INVALID_ARG"):
            tracer.trace_spectral(sc["camera"], W, H, 1, D, render_id=4, crop=bad)


@pytest.mark.parametrize("below,extra", [(64, 2), (100000, 4)])
def test_deferral_leaves_the_render_unchanged(tracer, below, extra):
    """Small queues waiting a sweep (the paper's load-balancing rule): the
    same images, logs and per-kind visit counts, on a grid with many sweeps
    (below = 100000 defers every queue whose rays can still drain)."""
    import paper_1912_06474_amd as m
    sc = sg.tiny_room()
    W, H, spp, D, grid = 64, 48, 3, 5, (4, 4, 2)
    tracer.reset_stats()
    a = gpu_render(tracer, sc, W, H, spp, D, grid=grid)
    sa = tracer.stats()
    tracer.reset_render(0)
    tracer.set_deferral(below, extra)
    try:
        tracer.reset_stats()
        b = gpu_render(tracer, sc, W, H, spp, D, grid=grid)
        sb = tracer.stats()
        tracer.reset_render(0)
    finally:
        tracer.set_deferral(0, 0)
    for k in ("spectral", "xyz", "hit_log", "shadow_log"):
        assert np.array_equal(a[k], b[k]), k
    for k in ("ext_rays", "shadow_rays", "ext_cell_visits", "shadow_cell_visits", "overflow"):
        assert sa[k] == sb[k], (k, sa[k], sb[k])
    assert sb["launches_trace"] == sa["launches_trace"] + extra * (sa["launches_trace"] // 8)
    with pytest.raises(m.SddError, match="INVALID_ARG"):
        tracer.set_deferral(-1, 2)
    with pytest.raises(m.SddError, match="INVALID_ARG"):
        tracer.set_deferral(64, 5)
