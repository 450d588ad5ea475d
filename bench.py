#!/usr/bin/env python
"""Throughput of the spectral domain-decomposition path tracer on one MI355X.

A step renders one full frame of the room-scale workload (about 200k
triangles, three 4 mm panes, 512 x 512 pixels, 16 samples per pixel,
41 wavelengths, up to 8 surface vertices per path, 4 x 4 x 2 subdomains)
with sdd_trace_spectral and resolves it with sdd_resolve_image.  Successive
steps trace new sample ranges of the same progressive render.  The metric is
(extension rays + shadow rays) * n_lambda / second.

One JSON line is printed (rank 0); progress goes to stderr.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0          # MI355X HBM3E, GB/s
REC_BYTES = 40                 # queue record: (o, t_enter) 16 B + (d, path) 16 B + (excl, t_max) 8 B
HIT_BYTES = 8
COPY_FLOATS = 1 << 28          # plain device copy of 1 GiB, for scaling FETCH_SIZE / WRITE_SIZE

# HBM bytes of the dominant kernel measured with rocprofv3 --pmc FETCH_SIZE /
# WRITE_SIZE, valid only while that kernel's sources are unchanged
TRAFFIC = {
    "furnished_room": (os.path.join(ROOT, "profiles", "k_trace_traffic_furnished_room_512x512_16spp.txt"),
                       ["kernels.hip", "layout.h", "device_math.h"]),
    "nrc_room": (os.path.join(ROOT, "profiles", "k_query_mfma_traffic_nrc_room_1920x1080_4spp.txt"),
                 ["nrc.hip", "nrc.h"]),
}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


WORKLOADS = {
    "furnished_room": dict(scene=("furnished_room", dict(seed=1, n_lambda=41)), W=512, H=512, spp=16, D=8,
                           grid=(4, 4, 2)),
    "tiny_room": dict(scene=("tiny_room", dict(seed=0, n_lambda=16)), W=64, H=64, spp=1, D=4, grid=(2, 2, 1)),
    # 64 renders of uneven resolution (128^2 .. 1024^2, 8 spp) with 8 photochromic
    # states, traced together in one sdd_trace_batch call per step
    "photochromic_batch": dict(scene=("furnished_room", dict(seed=1, n_lambda=41)), W=1024, H=1024, spp=8, D=8,
                               grid=(4, 4, 2), batch=dict(n=64, seed=2, n_states=8, spp=8)),
    # 4M triangles, coated (electrochromic) panes, 81 wavelengths, 128 subdomains
    "electrochromic_room": dict(scene=("electrochromic_room", dict(seed=4, n_lambda=81)), W=3840, H=2160, spp=64,
                                D=8, grid=(8, 4, 4)),
    # radiance cache vs plain at equal image quality: 1M triangles, 1920 x 1080,
    # 4 spp per frame, 41 wavelengths, paths end in the cache after vertex 2
    "nrc_room": dict(scene=("nrc_room", dict(seed=3, n_lambda=41)), W=1920, H=1080, spp=4, D=8, grid=(4, 4, 2),
                     nrc=dict(ref_frames=48, train_paths=1 << 16, train_steps=4, train_batch=1 << 14)),
}

# Multiply-adds of one cache query launch, two flops each, as the network is
# evaluated: per (path, wavelength) hidden layers 1..4 (64 x 64) and the output
# (64); per path layer 0's 48 position and direction inputs (x 64); per
# wavelength layer 0's 16 one-blob inputs (x 64).
def nrc_query_flops(rows, nl):
    return 2 * (rows * (4 * 64 * 64 + 64) + rows // nl * 48 * 64 + nl * 16 * 64)
MFMA_BF16_PEAK_TFLOPS = 2500.0  # MI355X dense BF16
ROOM_LO, ROOM_HI = (0.0, 0.0, 0.0), (4.0, 3.0, 2.5)


def source_hash(sources):
    import hashlib
    h = hashlib.sha256()
    for f in sources:
        with open(os.path.join(ROOT, "paper_1912_06474_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def measured_traffic(workload, grid):
    """HBM bytes per launch of the workload's dominant kernel from the committed
    counter summary, or None if it was taken on other kernel sources or another
    workload."""
    if workload not in TRAFFIC:
        return None
    path, sources = TRAFFIC[workload]
    try:
        with open(path) as fh:
            kv = dict(l.strip().split("=", 1) for l in fh if "=" in l and not l.lstrip().startswith("#"))
    except OSError:
        return None
    if kv.get("source_sha256") != source_hash(sources):
        return None
    if kv.get("workload") != workload or kv.get("grid") != "x".join(map(str, grid)):
        return None
    fetch = float(kv["fetch_kib_per_dispatch"]) * float(kv["fetch_scale"])
    write = float(kv["write_kib_per_dispatch"]) * float(kv["write_scale"])
    return (fetch + write) * 1024.0


def copy_calibration():
    """A plain device copy of known size: what FETCH_SIZE / WRITE_SIZE read for it
    scales the counters of the trace kernel to bytes."""
    import torch
    a = torch.ones(COPY_FLOATS, device="cuda", dtype=torch.float32)
    b = torch.empty_like(a)
    torch.cuda.synchronize()
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes_per_launch": 4 * COPY_FLOATS, "launches": 3}))


def cpu_baseline(scene, wl, target_s=15.0):
    """The FP64 oracle on a bounded, strided pixel sample of the same frame (1 spp)."""
    import numpy as np

    import oracle

    threads = int(os.environ.get("OMP_NUM_THREADS", "0") or 0) or (os.cpu_count() or 1)
    osc = oracle.OracleScene(scene)
    _ = osc.accel  # build excluded from the timing
    W, H, D = wl["W"], wl["H"], wl["D"]
    nl = len(scene["lambda_nm"])
    n, spp = 512, 1
    while True:
        stride = max(1, (W * H) // n)
        pix = np.arange(0, W * H, stride, dtype=np.int32)[:n]
        t0 = time.perf_counter()
        r = oracle.render(scene, W, H, spp, D, pix=pix, oscene=osc, n_threads=threads)
        dt = time.perf_counter() - t0
        log(f"[cpu_baseline] {len(pix)} px x {spp} spp: {dt:.2f} s")
        if dt >= target_s / 3 or (len(pix) >= W * H and spp >= wl["spp"]):
            break
        grow = max(2.0, target_s / max(dt, 1e-3))
        if n < W * H:
            n = min(W * H, int(n * grow))
        else:
            spp = min(wl["spp"], max(spp + 1, int(spp * grow)))
    rays = r["n_ext_rays"] + r["n_shadow_rays"]
    return {"value": rays * nl / dt, "unit": "rays*lambda/s", "cores": threads, "kind": "oracle",
            "sample": f"{len(pix)} pixels (every {stride}th of the {W}x{H} frame) x {spp} spp, depth {D}, "
                      f"{nl} wavelengths, FP64, {rays} rays in {dt:.2f} s"}


def nrc_comparison(args, tr, scene, wl):
    """Plain tracer and radiance-cache tracer on the same frame sequence until
    equal image quality.  Quality: rel-MSE = mean over pixels and wavelengths
    of ((I - R)^2 - var R) / (R^2 + 0.01 mean(R)^2) against a plain reference
    R = (A + B) / 2 of two independent halves, var R = (A - B)^2 / 4 (removes
    the reference's own noise from the estimate).  The plain run traces
    ``steps`` frames; its final rel-MSE q is the target; the cache run (after
    ``warmup`` training frames, timed) traces frames until it reaches q.  Both
    times are whole-frame wall times (trace + resolve), synchronised."""
    import numpy as np
    import torch

    import scenegen

    W, H, spp, D = wl["W"], wl["H"], wl["spp"], wl["D"]
    cfg = dict(wl["nrc"])
    if args.ref_frames:
        cfg["ref_frames"] = args.ref_frames
    if args.nrc_train_steps is not None:
        cfg["train_steps"] = args.nrc_train_steps
    if args.nrc_train_batch is not None:
        cfg["train_batch"] = args.nrc_train_batch
    cfg["lr"] = args.nrc_lr if args.nrc_lr is not None else 1e-2
    nl = len(scene["lambda_nm"])
    cam = scene["camera"]

    def trace(rid, off, nrc):
        tr.trace_spectral(cam, W, H, spp, D, seed=0, render_id=rid, sample_offset=off, nrc=nrc, time_kernels=True)
        s, _ = tr.resolve_image(rid, W, H, spectral=True, xyz=True)
        return s

    t0 = time.perf_counter()
    for f in range(cfg["ref_frames"]):
        trace(10, 1_000_000 + f * spp, False)
        trace(11, 2_000_000 + f * spp, False)
    A, _ = tr.resolve_image(10, W, H, spectral=True, xyz=False)
    B, _ = tr.resolve_image(11, W, H, spectral=True, xyz=False)
    tr.reset_render(10)
    tr.reset_render(11)
    R = 0.5 * (A + B)
    varR = 0.25 * (A - B) ** 2
    den = R * R + 0.01 * R.mean() ** 2
    ref_self = float((varR / den).mean())
    log(f"[bench] reference: {2 * cfg['ref_frames'] * spp} spp in {time.perf_counter() - t0:.1f} s, "
        f"its own rel-MSE {ref_self:.3e}")

    def relmse(img):
        return float((((img - R) ** 2 - varR) / den).mean())

    def run(rid, nrc, n_frames, target=None, warm=0):
        tt, hist = 0.0, []
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        for f in range(warm):  # cache training frames, not accumulated
            trace(3, 3_000_000 + f * spp, True)
        torch.cuda.synchronize()
        if warm:
            tr.reset_render(3)
        tt = time.perf_counter() - t1
        warm_s = tt
        for f in range(n_frames):
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            img = trace(rid, f * spp, nrc)
            torch.cuda.synchronize()
            tt += time.perf_counter() - t1
            hist.append((f + 1, tt, relmse(img)))
            if f % 10 == 9:
                log(f"[bench] {'cache' if nrc else 'plain'} frame {f + 1}: {tt:.2f} s, rel-MSE {hist[-1][2]:.4f}")
            if target is not None and hist[-1][2] <= target:
                break
        tr.reset_render(rid)
        return hist, warm_s

    def fit(hist):
        """rel-MSE(n) ~ a + b / n over the second half of the run; frames to 1%."""
        h = np.array(hist[len(hist) // 2:])
        X = np.stack([np.ones(len(h)), 1.0 / h[:, 0]], 1)
        a, b = np.linalg.lstsq(X, h[:, 2], rcond=None)[0]
        n1 = b / (0.01 - a) if 0.01 - a > 0 and b > 0 else None
        return float(a), float(b), (float(n1) if n1 is not None else None)

    tr.reset_stats()
    hp, _ = run(1, False, args.steps)
    stp = tr.stats()
    q = hp[-1][2]
    t_plain = hp[-1][1]
    log(f"[bench] plain: {args.steps} frames, {t_plain:.2f} s, rel-MSE {q:.4f}")

    params, tables = scenegen.nrc_params(0)
    tr.nrc_init(params, tables, ROOM_LO, ROOM_HI, lr=cfg["lr"], train_paths=cfg["train_paths"],
                train_steps=cfg["train_steps"], train_batch=cfg["train_batch"], precision="bf16")
    tr.reset_stats()
    hn, warm_s = run(2, True, 4 * args.steps, target=q, warm=args.warmup)
    stn = tr.stats()
    reached = hn[-1][2] <= q
    t_nrc = hn[-1][1]
    log(f"[bench] cache: warm-up {args.warmup} frames {warm_s:.2f} s, then {len(hn)} frames, {t_nrc:.2f} s, "
        f"rel-MSE {hn[-1][2]:.4f} ({'reached' if reached else 'did not reach'} {q:.4f})")
    fp, fn = fit(hp), fit(hn)
    nrc_frames = args.warmup + len(hn)
    fr_plain = t_plain / len(hp)
    fr_nrc = (t_nrc - warm_s) / len(hn)
    samples_plain = len(hp) * W * H * spp
    # roofline of the cache query (BF16 matrix cores) over the cache run
    launches = max(1, stn["nrc_query_launches"])
    avg_ms = stn["ms_nrc_query"] / launches
    flops = nrc_query_flops(stn["nrc_query_rows"] // launches, nl)
    achieved = flops / (avg_ms * 1e-3) / 1e12 if avg_ms > 0 else 0.0
    value = samples_plain * nl / t_nrc if reached else None
    return {
        "metric": "spectral path samples/s (rays x lambda/s) at equal rel-MSE, radiance cache vs plain, one MI355X",
        "value": value,
        "unit": "plain-equivalent path samples*lambda/s",
        "ms_per_step": fr_nrc * 1e3,
        "dtype": "bf16 cache (f32 transport)",
        "comparison": {
            "target_rel_mse": q, "reference_own_rel_mse": ref_self,
            "plain": {"frames": len(hp), "seconds": t_plain, "ms_per_frame": fr_plain * 1e3,
                      "path_samples_lambda_per_s": W * H * spp * nl / fr_plain,
                      "rays_lambda_per_s": (stp["ext_rays"] + stp["shadow_rays"]) * nl / t_plain,
                      "fit_a_b": fp[:2], "frames_to_1pct_extrapolated": fp[2]},
            "cache": {"warmup_frames": args.warmup, "frames": len(hn), "seconds_incl_warmup": t_nrc,
                      "ms_per_frame": fr_nrc * 1e3, "path_samples_lambda_per_s": W * H * spp * nl / fr_nrc,
                      "rays_lambda_per_s": (stn["ext_rays"] + stn["shadow_rays"]) * nl / t_nrc,
                      "rel_mse": hn[-1][2], "reached_target": reached,
                      "fit_a_b": fn[:2], "frames_to_1pct_extrapolated": fn[2],
                      "ms_query_mfma_per_frame": stn["ms_nrc_query"] / nrc_frames,
                      "ms_train_per_frame": stn["ms_nrc_train"] / nrc_frames},
            "speedup_at_equal_quality": (t_plain / t_nrc) if reached else None,
            "cache_settings": {k: cfg[k] for k in ("train_paths", "train_steps", "train_batch", "lr")},
        },
        "roofline": {"bound": "mfma", "kernel": "k_query_mfma", "achieved": achieved,
                     "peak": MFMA_BF16_PEAK_TFLOPS, "unit": "TFLOP/s", "frac": achieved / MFMA_BF16_PEAK_TFLOPS,
                     "traffic": measured_traffic(args.workload, wl["grid"]), "flops_per_launch": flops,
                     "avg_launch_ms": avg_ms, "launches": launches},
    }


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="furnished_room", choices=sorted(WORKLOADS))
    ap.add_argument("--grid", default=None, help="override subdomain grid, e.g. 1x1x1")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--count-work", action="store_true",
                    help="trace one extra (untimed) frame counting BVH node visits and triangle tests")
    ap.add_argument("--device-bvh", action="store_true",
                    help="build the subdomain BVHs on the GPU (linear BVH per cell) instead of the host SAH build")
    ap.add_argument("--graph", action="store_true",
                    help="also time the same steps replayed from a captured HIP graph (no per-launch events)")
    ap.add_argument("--ref-frames", type=int, default=None,
                    help="nrc_room: frames in each half of the plain reference (default 48)")
    ap.add_argument("--nrc-train-steps", type=int, default=None, help="nrc_room: Adam steps per frame (default 4)")
    ap.add_argument("--nrc-train-batch", type=int, default=None, help="nrc_room: rows per Adam step (default 2^14)")
    ap.add_argument("--nrc-lr", type=float, default=None, help="nrc_room: Adam learning rate (default 1e-2)")
    ap.add_argument("--autotune", nargs="?", const="", default=None, metavar="FILE",
                    help="search the launch settings on the step's own call before the warmup (results file "
                         "FILE is read first and written after a search)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain 1 GiB device copy (counter calibration) and exit")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path (run with --gpus 1)",
              file=sys.stderr)
        sys.exit(2)

    if args.copy_calibration:
        copy_calibration()
        return

    import torch

    import paper_1912_06474_amd as sdd
    import scenegen

    wl = dict(WORKLOADS[args.workload])
    if args.grid:
        wl["grid"] = tuple(int(x) for x in args.grid.lower().split("x"))
    name, kw = wl["scene"]
    t0 = time.perf_counter()
    scene = getattr(scenegen, name)(**kw)
    renders = None
    if "batch" in wl:
        bw = wl["batch"]
        scene, base, states = scenegen.photochromic_states(scene, bw["n_states"])
        renders = scenegen.batch_renders(bw["n"], bw["seed"], bw["n_states"], spp=bw["spp"])
        for r in renders:
            r["glass_swap"] = (base, states[r["state"]])
    log(f"[bench] scene {scene['name']}: {len(scene['tris'])} tris, {len(scene['lambda_nm'])} lambda "
        f"({time.perf_counter() - t0:.1f} s)")
    W, H, spp, D = wl["W"], wl["H"], wl["spp"], wl["D"]
    nl = len(scene["lambda_nm"])
    cam = scene["camera"]

    tr = sdd.Tracer()
    tr.load_scene(scene)
    t0 = time.perf_counter()
    tr.build_bvh(*wl["grid"], device=args.device_bvh)
    build_s = time.perf_counter() - t0
    st0 = tr.stats()
    log(f"[bench] build_bvh {wl['grid']}: {build_s:.2f} s, refs {st0['n_refs']}, nodes {st0['n_nodes']}, "
        f"depth {st0['max_bvh_depth']}")

    if "nrc" in wl:
        res = nrc_comparison(args, tr, scene, wl)
        res.update({"n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "higher_is_better": True,
                    "scaling": "weak", "vs_baseline": None, "data": "synthetic"})
        res["config"] = {"workload": f"{args.workload}: {len(scene['tris'])} tris, {W}x{H}, {spp} spp per frame, "
                                     f"{nl} lambda, depth {D}, cache after vertex 2, grid "
                                     f"{'x'.join(map(str, wl['grid']))}"}
        res["build_bvh_s"] = build_s
        if not args.no_cpu_baseline:
            res["cpu_baseline"] = cpu_baseline(scene, wl, args.cpu_seconds)
        print(json.dumps(res))
        return

    step = 0

    def frame(graph=False):
        nonlocal step
        # every launch is bracketed by HIP events on the library's stream (not in graph replays)
        if renders is None:
            tr.trace_spectral(cam, W, H, spp, D, sample_offset=step * spp, render_id=0, time_kernels=not graph,
                              graph=graph)
            tr.resolve_image(0, W, H, spectral=True, xyz=True)
        else:
            for r in renders:
                r["sample_offset"] = step * r["spp"]
            tr.trace_batch(renders, D, time_kernels=not graph, graph=graph)
            for r in renders:
                tr.resolve_image(r["render_id"], r["W"], r["H"], spectral=True, xyz=True)
        step += 1

    tuned = None
    if args.autotune is not None:
        t0 = time.perf_counter()
        call = renders if renders is not None else [dict(camera=cam, W=W, H=H, spp=spp, render_id=0)]
        tuned = tr.autotune(call, D, reps=2, cache=args.autotune or None)
        log(f"[bench] autotune {tuned} ({time.perf_counter() - t0:.1f} s)")

    for i in range(args.warmup):
        frame()
        torch.cuda.synchronize()
        log(f"[bench] warmup {i + 1}/{args.warmup}")

    # timed region
    tr.reset_stats()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        frame()
        log(f"[bench] step {i + 1}/{args.steps}")
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    st = tr.stats()
    rays = st["ext_rays"] + st["shadow_rays"]
    value = rays * nl / dt

    # roofline of k_trace over the timed region: every closest-hit and shadow
    # sweep; per cell visit a 40 B queue record is read, per crossing a 40 B
    # record is written to the neighbour's queue, per extension ray an 8 B hit
    launches = max(1, st["launches_trace"])
    ms_trace = st["ms_trace_ext"] + st["ms_trace_shadow"]
    visits = st["ext_cell_visits"] + st["shadow_cell_visits"]
    crossings = max(0, visits - rays)
    alg_bytes = REC_BYTES * visits + REC_BYTES * crossings + HIT_BYTES * st["ext_rays"]
    avg_ms = ms_trace / launches
    achieved = alg_bytes / launches / (avg_ms * 1e-3) / 1e9 if avg_ms > 0 else 0.0
    traffic = measured_traffic(args.workload, wl["grid"])
    kern_ms = {"trace_ext": st["ms_trace_ext"], "trace_shadow": st["ms_trace_shadow"], "shade": st["ms_shade"],
               "other": st["ms_other"]}
    log(f"[bench] timed {dt:.3f} s; kernel ms {kern_ms}")
    log(f"[bench] stats {json.dumps(st)}")

    if renders is None:
        paths_per_step = W * H * spp
        frame_desc = f"{W}x{H}, {spp} spp"
    else:
        paths_per_step = sum(r["W"] * r["H"] * r["spp"] for r in renders)
        frame_desc = (f"{len(renders)} renders {min(r['W'] for r in renders)}^2..{max(r['W'] for r in renders)}^2 "
                      f"({sum(r['W'] * r['H'] for r in renders)} px), {renders[0]['spp']} spp, "
                      f"{wl['batch']['n_states']} photochromic states")
    workload_desc = (f"{args.workload}: {len(scene['tris'])} tris, {frame_desc}, {nl} lambda, depth {D}, "
                     f"grid {'x'.join(map(str, wl['grid']))}")
    res = {
        "metric": "spectral path samples/s (rays x lambda/s), plain tracer, one MI355X",
        "value": value,
        "unit": "rays*lambda/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": dt / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": workload_desc, "paths_per_step": paths_per_step, "rays_per_step": rays / args.steps,
                   "path_samples_lambda_per_s": paths_per_step * nl * args.steps / dt},
        "roofline": {"bound": "hbm", "kernel": "k_trace", "achieved": achieved,
                     "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                     "alg_bytes_per_launch": alg_bytes / launches, "avg_launch_ms": avg_ms,
                     "launches": launches},
        "kernel_ms_per_step": {k: v / args.steps for k, v in kern_ms.items()},
        "build_bvh_s": build_s,
        "bvh": "device LBVH" if args.device_bvh else "host binned SAH",
        "tuning": dict(tr.get_tuning(), paths_per_pass=st["paths_per_batch"],
                       autotuned=None if tuned is None else {"from_cache": tuned["from_cache"],
                                                             "search_ms_per_call": tuned["ms"]}),
    }
    if args.count_work:
        tr.reset_stats()
        tr.trace_spectral(cam, W, H, spp, D, sample_offset=step * spp, render_id=1 << 30, count_work=True)
        torch.cuda.synchronize()
        sw = tr.stats()
        visits = sw["ext_cell_visits"] + sw["shadow_cell_visits"]
        res["work"] = {"node_visits_per_cell_visit": sw["node_visits"] / max(1, visits),
                       "tri_tests_per_cell_visit": sw["tri_tests"] / max(1, visits),
                       "cell_visits_per_ray": visits / max(1, sw["ext_rays"] + sw["shadow_rays"]),
                       "scene_bytes_per_frame": 64 * sw["node_visits"] + 48 * sw["tri_tests"]}
    if args.graph:
        gt = sdd.Tracer(stream=torch.cuda.Stream())  # graph capture needs a stream other than the null stream
        gt.load_scene(scene)
        gt.build_bvh(*wl["grid"], device=args.device_bvh)
        tr_main, tr = tr, gt
        frame(graph=True)  # capture
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            frame(graph=True)
        torch.cuda.synchronize()
        dtg = time.perf_counter() - t0
        res["graph_replay"] = {"ms_per_step": dtg / args.steps * 1e3, "value": rays * nl / dtg,
                               "note": "same steps replayed from one captured HIP graph, without per-launch events"}
        log(f"[bench] graph replay: {dtg / args.steps * 1e3:.2f} ms per step")
        tr = tr_main
        gt.close()
    if not args.no_cpu_baseline:
        res["cpu_baseline"] = cpu_baseline(scene, wl, args.cpu_seconds)
    print(json.dumps(res))


if __name__ == "__main__":
    main()
