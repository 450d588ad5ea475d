"""The allocation-free cache query (sdd_nrc_query_noalloc) against the
allocating one (sdd_nrc_query, BF16), through the C ABI: equal bit for bit on
two calls in a row, the second smaller than the first (the static scratch
keeps the first call's contents), and refused above its limit."""
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
    t = m.Tracer()
    t.load_scene(sg.tiny_room(0, 41))                      # the query covers the scene's 41 wavelengths
    params, tables = sg.nrc_params(31, table_size=1 << 16)
    rng = np.random.default_rng(32)
    tables = rng.uniform(-0.5, 0.5, tables.shape).astype(np.float32)
    t.nrc_init(params, tables, (0.0, 0.0, 0.0), sg.ROOM)
    return t


def _points(n, seed):
    rng = np.random.default_rng(seed)
    x = rng.uniform((0.0, 0.0, 0.0), sg.ROOM, (n, 3)).astype(np.float32)
    nrm = rng.normal(size=(n, 3))
    nrm = (nrm / np.linalg.norm(nrm, axis=1, keepdims=True)).astype(np.float32)
    return x, nrm


@pytest.mark.parametrize("sizes", [(65536, 1000), (4097, 63)])
def test_noalloc_query_equals_the_allocating_query(tracer, sizes):
    import torch
    for k, n in enumerate(sizes):
        print(f"[no_alloc] call {k + 1}: n = {n}", flush=True)
        x, nrm = _points(n, 100 + n)
        ref = tracer.nrc_query(x, nrm, "bf16")
        got = tracer.nrc_query_noalloc(x, nrm)
        torch.cuda.synchronize()
        nl = tracer.n_lambda
        assert torch.isfinite(ref[:, :nl]).all()
        assert torch.equal(got[:, :nl], ref[:, :nl]), float((got[:, :nl] - ref[:, :nl]).abs().max())


def test_noalloc_query_limits(tracer):
    import paper_1912_06474_amd as m
    x, nrm = _points(65537, 7)
    with pytest.raises(m.SddError, match="limit of 65536"):
        tracer.nrc_query_noalloc(x, nrm)
    out = tracer.nrc_query_noalloc(x[:0], nrm[:0])
    assert out.numel() == 0
