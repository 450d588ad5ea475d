"""HIP API trace of the allocation-free cache query (not a pytest module).

Run as ``rocprofv3 --hip-trace --output-format csv -d DIR -- python3
tests/trace_noalloc_query.py``.  After one allocating BF16 query (which sizes
its own buffers), three calls of sdd_nrc_query_noalloc (65536, 1000 and 777
points) run between two device synchronisations: the trace between those two
hipDeviceSynchronize calls must hold kernel launches only (no hipMalloc,
hipFree or memset).  The last line tells whether the 777-point result equals
the allocating query's.
"""
import os
import sys

import numpy as np
import torch

sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
import paper_1912_06474_amd as m  # noqa: E402
import scenegen as sg  # noqa: E402

N = 65536
t = m.Tracer()
t.load_scene(sg.tiny_room(0, 41))
params, tables = sg.nrc_params(31, table_size=1 << 16)
t.nrc_init(params, tables, (0.0, 0.0, 0.0), sg.ROOM)
rng = np.random.default_rng(1)
x = rng.uniform((0.0, 0.0, 0.0), sg.ROOM, (N, 3)).astype(np.float32)
nrm = np.tile(np.array([[0.0, 0.0, 1.0]], np.float32), (N, 1))
ref = t.nrc_query(x, nrm, "bf16")
x4 = torch.zeros((N, 4), device="cuda")
x4[:, :3] = torch.tensor(x, device="cuda")
n4 = torch.zeros((N, 4), device="cuda")
n4[:, :3] = torch.tensor(nrm, device="cuda")
out = torch.zeros((N, 44), device="cuda")
torch.cuda.synchronize()
for n in (N, 1000, 777):
    assert m.lib().sdd_nrc_query_noalloc(t.h, n, x4.data_ptr(), n4.data_ptr(), out.data_ptr()) == 0
torch.cuda.synchronize()
print("equal:", bool(torch.equal(out[:777, :41], ref[:777, :41])), flush=True)
