"""Graph replay (SDD_TRACE_GRAPH): a trace call's launch sequence is captured
into a HIP graph once and replayed by later calls that differ only in their
sample range.  Every replay must give what the eager launches give, bit for
bit, with eager work and synchronisations between the replays."""
import numpy as np
import pytest

import scenegen as sg

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def tracer():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1912_06474_amd as m
    return m.Tracer(stream=torch.cuda.Stream())  # capture needs a stream other than the null stream


def _frames(tracer, sc, W, H, spp, D, n, graph, batch=False):
    out = []
    hl = tracer.new_log(W, H, spp, D)
    for f in range(n):
        if batch:
            renders = [dict(camera=sc["camera"], W=W, H=H, spp=spp, render_id=0, sample_offset=f * spp, hit_log=hl),
                       dict(camera=dict(sc["camera"], eye=(1.0, 0.6, 1.4)), W=W // 2, H=H // 2, spp=spp,
                            render_id=1, sample_offset=f * spp)]
            tracer.trace_batch(renders, D, seed=3, graph=graph)
            s0, _ = tracer.resolve_image(0, W, H)
            s1, _ = tracer.resolve_image(1, W // 2, H // 2)
            out.append((s0.cpu().numpy(), s1.cpu().numpy(), hl.cpu().numpy()))
        else:
            tracer.trace_spectral(sc["camera"], W, H, spp, D, seed=3, render_id=0, sample_offset=f * spp,
                                  hit_log=hl, graph=graph)
            s, x = tracer.resolve_image(0, W, H)
            out.append((s.cpu().numpy(), x.cpu().numpy(), hl.cpu().numpy()))
    tracer.reset_render(0)
    if batch:
        tracer.reset_render(1)
    return out


@pytest.mark.parametrize("grid", [(1, 1, 1), (2, 2, 1)])
def test_graph_replays_equal_eager_frames(tracer, grid):
    sc = sg.tiny_room(0, 16)
    tracer.load_scene(sc)
    tracer.build_bvh(*grid)
    W, H, spp, D = 48, 40, 2, 5
    eager = _frames(tracer, sc, W, H, spp, D, 5, graph=False)
    tracer.reset_stats()
    graph = _frames(tracer, sc, W, H, spp, D, 5, graph=True)
    for f, (a, b) in enumerate(zip(eager, graph)):
        for u, v in zip(a, b):
            assert np.array_equal(u, v), f"frame {f}"
    st = tracer.stats()
    assert st["ext_rays"] > 0 and st["batches"] == 5


def test_graph_replays_of_a_batch_call(tracer):
    sc = sg.tiny_room(0, 16)
    tracer.load_scene(sc)
    tracer.build_bvh(2, 2, 1)
    W, H, spp, D = 64, 48, 2, 4
    eager = _frames(tracer, sc, W, H, spp, D, 4, graph=False, batch=True)
    graph = _frames(tracer, sc, W, H, spp, D, 4, graph=True, batch=True)
    for f, (a, b) in enumerate(zip(eager, graph)):
        for u, v in zip(a, b):
            assert np.array_equal(u, v), f"frame {f}"


def test_graph_refuses_timing_and_null_stream():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1912_06474_amd as m
    sc = sg.tiny_room(0, 16)
    t0 = m.Tracer(stream=torch.cuda.Stream())
    t0.load_scene(sc)
    t0.build_bvh(1, 1, 1)
    with pytest.raises(m.SddError, match="UNSUPPORTED"):
        t0.trace_spectral(sc["camera"], 16, 16, 1, 3, graph=True, time_kernels=True)
    t0.close()
