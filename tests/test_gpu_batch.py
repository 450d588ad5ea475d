"""GPU: several renders in one pipeline pass (sdd_trace_batch) and
photochromic glass states.

A batched render must equal the same render traced alone, bit for bit (the
random numbers are addressed by render, pixel and sample, never by queue
position); a photochromic state is a glass material substitution, checked
against the FP64 oracle on a scene whose pane triangles carry the state's
material.  The last test runs the batched workload at full size: 64 renders of
uneven resolution (128^2 .. 1024^2, 8 spp) with 8 darkening states in one call.
"""
import os

import numpy as np
import pytest

import oracle as ora
import scenegen as sg
from parity import ParityCtx, assert_parity

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def tracer():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1912_06474_amd as m
    return m.Tracer()


def _resolve_all(tr, renders):
    out = []
    for r in renders:
        s, _ = tr.resolve_image(r["render_id"], r["W"], r["H"], xyz=False)
        out.append(s.cpu().numpy())
        tr.reset_render(r["render_id"])
    return out


def _small_renders(base, states):
    cam = sg.tiny_room()["camera"]
    side = dict(eye=(0.6, 0.4, 1.0), target=(3.0, 2.6, 1.4), fov_deg=55.0, ortho=False, ortho_half_h=1.0)
    ortho = dict(eye=(2.0, 0.2, 1.25), target=(2.0, 3.0, 1.25), fov_deg=60.0, ortho=True, ortho_half_h=1.2)
    return [
        dict(camera=cam, W=64, H=48, spp=2, render_id=3, glass_swap=None),
        dict(camera=side, W=17, H=9, spp=3, render_id=8, glass_swap=(base, states[5])),
        dict(camera=ortho, W=33, H=33, spp=1, render_id=1, glass_swap=(base, states[7])),
        dict(camera=cam, W=40, H=40, spp=4, render_id=5, sample_offset=6, glass_swap=(base, states[2])),
    ]


@pytest.mark.parametrize("budget", [None, "0.0006"])
def test_batch_equals_single_renders(tracer, budget):
    sc, base, states = sg.photochromic_states(sg.tiny_room())
    D = 5
    tracer.load_scene(sc)
    tracer.build_bvh(2, 2, 1)
    old = os.environ.get("SDD_MEM_BUDGET_GB")
    if budget is not None:
        os.environ["SDD_MEM_BUDGET_GB"] = budget  # small batches that split renders
    try:
        renders = _small_renders(base, states)
        logs = {}
        for r in renders:
            r["hit_log"] = tracer.new_log(r["W"], r["H"], r["spp"], D)
            r["shadow_log"] = tracer.new_log(r["W"], r["H"], r["spp"], D)
        tracer.trace_batch(renders, D, seed=4)
        batched = _resolve_all(tracer, renders)
        for r in renders:
            logs[r["render_id"]] = (r["hit_log"].cpu().numpy(), r["shadow_log"].cpu().numpy())
        single = []
        for r in renders:
            hl = tracer.new_log(r["W"], r["H"], r["spp"], D)
            sl = tracer.new_log(r["W"], r["H"], r["spp"], D)
            tracer.trace_spectral(r["camera"], r["W"], r["H"], r["spp"], D, seed=4, render_id=r["render_id"],
                                  sample_offset=r.get("sample_offset", 0), hit_log=hl, shadow_log=sl,
                                  glass_swap=r["glass_swap"])
            single.append(_resolve_all(tracer, [r])[0])
            assert np.array_equal(hl.cpu().numpy(), logs[r["render_id"]][0])
            assert np.array_equal(sl.cpu().numpy(), logs[r["render_id"]][1])
        for a, b in zip(batched, single):
            assert np.array_equal(a, b)
        st = tracer.stats()
        print(f"[batch] budget {budget}: batches so far {st['batches']}", flush=True)
    finally:
        if budget is not None:
            if old is None:
                del os.environ["SDD_MEM_BUDGET_GB"]
            else:
                os.environ["SDD_MEM_BUDGET_GB"] = old


def test_photochromic_state_parity(tracer):
    sc, base, states = sg.photochromic_states(sg.tiny_room(n_lambda=41))
    W, H, spp, D = 48, 48, 2, 6
    tracer.load_scene(sc)
    tracer.build_bvh(2, 2, 1)
    for k in (0, 7):
        hl = tracer.new_log(W, H, spp, D)
        sl = tracer.new_log(W, H, spp, D)
        tracer.trace_spectral(sc["camera"], W, H, spp, D, seed=9, render_id=0, hit_log=hl, shadow_log=sl,
                              glass_swap=(base, states[k]))
        s, x = tracer.resolve_image(0, W, H)
        tracer.reset_render(0)
        g = dict(spectral=s.cpu().numpy(), xyz=x.cpu().numpy(), hit_log=hl.cpu().numpy(), shadow_log=sl.cpu().numpy())
        # the oracle sees the state's material on the pane triangles directly
        so = dict(sc)
        so["tri_mat"] = np.where(sc["tri_mat"] == base, states[k], sc["tri_mat"]).astype(np.int32)
        o = ora.render(so, W, H, spp, D, logs=True, seed=9)
        assert_parity(g, o, ParityCtx(so, W, H, spp, D, seed=9))
        if k == 7:
            # the darkest state transmits less through the pane than the clearest
            assert g["spectral"].sum() < prev
        prev = g["spectral"].sum()


def test_photochromic_batch_full_size(tracer):
    sc, base, states = sg.photochromic_states(sg.furnished_room(seed=1, n_lambda=41))
    renders = sg.batch_renders()
    D = 8
    tracer.load_scene(sc)
    tracer.build_bvh(4, 4, 2)
    checked = [r for r in renders if r["W"] == 128][:2] + [r for r in renders if r["W"] == 1024][:1]
    for r in renders:
        r["glass_swap"] = (base, states[r["state"]])
    for r in checked:
        r["hit_log"] = tracer.new_log(r["W"], r["H"], r["spp"], D)
        r["shadow_log"] = tracer.new_log(r["W"], r["H"], r["spp"], D)
    tracer.reset_stats()
    tracer.trace_batch(renders, D)
    st = tracer.stats()
    n_paths = sum(r["W"] * r["H"] * r["spp"] for r in renders)
    print(f"[batch] {len(renders)} renders, {n_paths} paths, {st['batches']} batches, "
          f"{st['ext_rays'] + st['shadow_rays']} rays", flush=True)
    assert st["overflow"] == 0
    res = {}
    for r in renders:
        s, x = tracer.resolve_image(r["render_id"], r["W"], r["H"])
        if r in checked:
            res[r["render_id"]] = (s.cpu().numpy(), x.cpu().numpy())
        tracer.reset_render(r["render_id"])
    rng = np.random.default_rng(5)
    for r in checked:
        WH = r["W"] * r["H"]
        pix = np.sort(rng.choice(WH, min(WH, 1024), replace=False)).astype(np.int32)
        so = dict(sc)
        so["tri_mat"] = np.where(sc["tri_mat"] == base, r["glass_swap"][1], sc["tri_mat"]).astype(np.int32)
        o = ora.render(so, r["W"], r["H"], r["spp"], D, camera=r["camera"], pix=pix, logs=True,
                       render_id=r["render_id"])
        s, x = res[r["render_id"]]
        g = dict(spectral=s[pix], xyz=x[pix], hit_log=r["hit_log"].cpu().numpy()[pix],
                 shadow_log=r["shadow_log"].cpu().numpy()[pix])
        assert_parity(g, o, ParityCtx(so, r["W"], r["H"], r["spp"], D, camera=r["camera"],
                                      render_id=r["render_id"], pix=pix))
