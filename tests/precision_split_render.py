"""Render one precision-split case through the library the environment selects
(SDD_PATH_STATE=f32: the FP32-path-state measurement build; unset: libsdd.so)
and save images and logs: python precision_split_render.py <case> <out.npz>.

Run as a child process by tests/test_gpu_precision_split.py, one process per
build, so each loads exactly one library."""
import os
import sys

import numpy as np

sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))  # the repository root

CASES = {
    # the tiny parity room, whole frame
    "tiny_room": dict(scene=("tiny_room", {}), W=64, H=64, spp=1, D=4, grid=(2, 2, 1), crop=None),
    # the room-scale frame: a 64 x 64 window around the panes
    "furnished_room_crop": dict(scene=("furnished_room", dict(seed=1, n_lambda=41)), W=512, H=512, spp=16, D=8,
                                grid=(4, 4, 2), crop=(268, 252, 64, 64)),
    # the 4M-triangle electrochromic frame: a 64 x 36 window in the lit region
    "electrochromic_crop": dict(scene=("electrochromic_room", {}), W=3840, H=2160, spp=64, D=8, grid=(8, 4, 4),
                                crop=(1472, 966, 64, 36)),
}


def make_scene(case):
    import scenegen as sg
    name, kw = CASES[case]["scene"]
    return getattr(sg, name)(**kw)


def main():
    case, out = sys.argv[1], sys.argv[2]
    import paper_1912_06474_amd as m
    c = CASES[case]
    sc = make_scene(case)
    tr = m.Tracer()
    tr.load_scene(sc)
    tr.build_bvh(*c["grid"])
    W, H, spp, D = c["W"], c["H"], c["spp"], c["D"]
    w, h = (c["crop"][2], c["crop"][3]) if c["crop"] else (W, H)
    hl = tr.new_log(w, h, spp, D)
    sl = tr.new_log(w, h, spp, D)
    print(f"[precision_split] {case} through {m.LIB_PATH}", flush=True)
    tr.trace_spectral(sc["camera"], W, H, spp, D, render_id=0, hit_log=hl, shadow_log=sl, crop=c["crop"])
    s, x = tr.resolve_image(0, w, h)
    np.savez(out, spectral=s.cpu().numpy(), xyz=x.cpu().numpy(), hit_log=hl.cpu().numpy(),
             shadow_log=sl.cpu().numpy(), lib=m.LIB_PATH)


if __name__ == "__main__":
    main()
