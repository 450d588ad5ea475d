#!/usr/bin/env python
"""Radiance cache against the plain tracer at 1% rel-MSE, and plain throughput, on one MI355X.

Default (``--workload nrc_room``): the learned-radiance-cache workload (1M
triangles, 1920 x 1080, 4 samples per pixel per frame, 41 wavelengths, up to
8 vertices, 4 x 4 x 2 subdomains).  The plain tracer and the cache tracer each
accumulate frames of the same view; a step is 10 frames of each.  Their
rel-MSE curves against an unbiased estimate of the converged image give each
method's time to 1% rel-MSE, and the line's value is the plain-equivalent
rate at that quality: the plain path samples x wavelengths that reach 1%
divided by the cache's time to reach it.  The room-scale plain workload
(200k triangles, 512 x 512, 16 spp, 41 wavelengths, depth 8, 4 x 4 x 2) is
measured in the same run as a sub-object with its traversal kernel's HBM
roofline.  Other workloads (``--workload furnished_room`` ...) print the plain
throughput line alone: (extension rays + shadow rays) * n_lambda / second.

One JSON line is printed; progress goes to stderr.
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
# key: (counter summary, the kernel sources it holds for, the workload it was taken on)
TRAFFIC = {
    "furnished_room": (os.path.join(ROOT, "profiles", "k_trace_traffic_furnished_room_512x512_16spp.txt"),
                       ["kernels.hip", "layout.h", "device_math.h"], "furnished_room"),
    "nrc_room": (os.path.join(ROOT, "profiles", "k_query_mfma_traffic_nrc_room_1920x1080_4spp.txt"),
                 ["nrc.hip", "nrc.h"], "nrc_room"),
    # k_trace in the radiance-cache frames (the cache line's dominant kernel)
    "nrc_room_trace": (os.path.join(ROOT, "profiles", "k_trace_traffic_nrc_room_1920x1080_4spp.txt"),
                       ["kernels.hip", "layout.h", "device_math.h"], "nrc_room"),
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
                     nrc=dict(ref_frames=64, train_paths=1 << 16, train_steps=8, train_batch=1 << 14,
                              train_warmup=100)),
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


def measured_traffic(key, grid):
    """HBM bytes per launch of a kernel (TRAFFIC[key]) from the committed
    counter summary, or None if it was taken on other kernel sources, another
    workload or another grid."""
    if key not in TRAFFIC:
        return None
    path, sources, workload = TRAFFIC[key]
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


def cpu_model():
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(scene, wl, target_s=15.0):
    """The FP64 oracle on a bounded pixel sample of the same frame, spread
    evenly over it (1 spp; more samples per pixel only once every pixel is
    in), grown until one run takes at least 0.7 target_s."""
    import numpy as np

    import oracle

    threads = int(os.environ.get("OMP_NUM_THREADS", "0") or 0) or (os.cpu_count() or 1)
    osc = oracle.OracleScene(scene)
    _ = osc.accel  # build excluded from the timing
    W, H, D = wl["W"], wl["H"], wl["D"]
    nl = len(scene["lambda_nm"])
    n, spp = 512, 1
    while True:
        pix = (np.arange(n, dtype=np.int64) * (W * H) // n).astype(np.int32)  # n distinct, evenly spread
        t0 = time.perf_counter()
        r = oracle.render(scene, W, H, spp, D, pix=pix, oscene=osc, n_threads=threads)
        dt = time.perf_counter() - t0
        log(f"[cpu_baseline] {len(pix)} px x {spp} spp: {dt:.2f} s")
        if dt >= 0.7 * target_s or (len(pix) >= W * H and spp >= wl["spp"]):
            break
        grow = max(2.0, target_s / max(dt, 1e-3))
        if n < W * H:
            n = min(W * H, int(n * grow))
        else:
            spp = min(wl["spp"], max(spp + 1, int(spp * grow)))
    rays = r["n_ext_rays"] + r["n_shadow_rays"]
    return {"value": rays * nl / dt, "unit": "rays*lambda/s", "cores": threads, "kind": "oracle",
            "cpu_model": cpu_model(),
            "sample": f"{len(pix)} pixels spread evenly over the {W}x{H} frame x {spp} spp, depth {D}, "
                      f"{nl} wavelengths, FP64, {rays} rays in {dt:.2f} s"}


def cpu_oracle_cases():
    """The FP64 oracle on the comparison cases it is held against: the tiny
    parity room's whole frame, and the 4M-triangle electrochromic frame at its
    64 spp on the 64 x 36 centre of the 256 x 144 window the GPU is compared
    on (the whole window, 16 times the pixels, takes about two minutes on 8
    cores; its time is extrapolated).  Scene generation and the oracle's BVH
    are not timed."""
    import oracle
    import scenegen

    threads = int(os.environ.get("OMP_NUM_THREADS", "0") or 0) or (os.cpu_count() or 1)
    cases = []
    for name, make, W, H, spp, D, crop in (
            ("tiny_room whole frame", lambda: scenegen.tiny_room(), 64, 64, 1, 4, None),
            ("electrochromic_room 64x36 centre of the 256x144 window", lambda: scenegen.electrochromic_room(), 3840,
             2160, 64, 8, (1472, 966, 64, 36))):
        sc = make()
        osc = oracle.OracleScene(sc)
        _ = osc.accel
        t0 = time.perf_counter()
        r = oracle.render(sc, W, H, spp, D, crop=crop, oscene=osc, n_threads=threads)
        dt = time.perf_counter() - t0
        rays = r["n_ext_rays"] + r["n_shadow_rays"]
        nl = len(sc["lambda_nm"])
        px = crop[2] * crop[3] if crop else W * H
        log(f"[cpu_baseline] {name}: {dt:.2f} s")
        c = {"case": f"{name}: {len(sc['tris'])} tris, {px} px x {spp} spp, depth {D}, {nl} lambda",
             "seconds": dt, "rays": rays, "rays_lambda_per_s": rays * nl / dt, "cores": threads}
        if crop:
            c["seconds_whole_256x144_window_est"] = dt * (256 * 144) / px
        cases.append(c)
    return cases


def relmse_fit(hist, floor=True):
    """Least-squares fit of rel-MSE(n) ~ a + b / n over frames n (a = 0 if not floor)."""
    import numpy as np
    h = np.asarray(hist, np.float64)
    n, y = h[:, 0], h[:, 2]
    if floor:
        X = np.stack([np.ones(len(n)), 1.0 / n], 1)
        a, b = np.linalg.lstsq(X, y, rcond=None)[0]
    else:
        a, b = 0.0, float(np.sum(y / n) / np.sum(1.0 / n ** 2))
    return float(a), float(b)


def error_split(Ia, Ib, R, varR, wgt):
    """Weighted squared error of I = (Ia + Ib) / 2 split into bias and variance,
    from two independent halves Ia, Ib of equal sample counts and an
    independent reference R with variance estimate varR (all [pixels, lambda]):
    var I = (Ia - Ib)^2 / 4 estimates Var I without bias, so
    w ((I - R)^2 - var R - var I) estimates w bias_I^2.  Returns the mean
    weighted squared bias, its standard error over pixels (wavelengths averaged
    per pixel) and the mean weighted variance of I."""
    I = 0.5 * (Ia + Ib)
    varI = 0.25 * (Ia - Ib) ** 2
    term = (((I - R) ** 2 - varR - varI) * wgt).mean(dim=1)
    return float(term.mean()), float(term.std() / term.numel() ** 0.5), float((varI * wgt).mean())


def frames_to(target, a, b):
    """Frames n with a + b / n = target (None if the floor a is at or above it)."""
    return b / (target - a) if target > a and b > 0 else None


def trace_roofline(st, traffic):
    """HBM roofline of k_trace over the launches counted in st: per cell visit a
    40 B queue record is read, per crossing a 40 B record is written to the
    neighbour's queue, per extension ray an 8 B hit."""
    launches = max(1, st["launches_trace"])
    rays = st["ext_rays"] + st["shadow_rays"]
    visits = st["ext_cell_visits"] + st["shadow_cell_visits"]
    crossings = max(0, visits - rays)
    alg = REC_BYTES * visits + REC_BYTES * crossings + HIT_BYTES * st["ext_rays"]
    avg_ms = (st["ms_trace_ext"] + st["ms_trace_shadow"]) / launches
    achieved = alg / launches / (avg_ms * 1e-3) / 1e9 if avg_ms > 0 else 0.0
    return {"bound": "hbm", "kernel": "k_trace", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS, "traffic": traffic, "alg_bytes_per_launch": alg / launches,
            "avg_launch_ms": avg_ms, "launches": launches}


def query_roofline(st, nl, traffic):
    """BF16 matrix-core roofline of k_query_mfma: the network's flops on the
    launch's cache paths (nrc_query_flops)."""
    launches = max(1, st["nrc_query_launches"])
    avg_ms = st["ms_nrc_query"] / launches
    flops = nrc_query_flops(st["nrc_query_rows"] // launches, nl)
    achieved = flops / (avg_ms * 1e-3) / 1e12 if avg_ms > 0 else 0.0
    return {"bound": "mfma", "kernel": "k_query_mfma", "achieved": achieved, "peak": MFMA_BF16_PEAK_TFLOPS,
            "unit": "TFLOP/s", "frac": achieved / MFMA_BF16_PEAK_TFLOPS, "traffic": traffic,
            "flops_per_launch": flops, "avg_launch_ms": avg_ms, "launches": launches}


FRAMES_PER_STEP = 20
TARGET_REL_MSE = 0.01


def nrc_comparison(args, tr, scene, wl):
    """Plain tracer against the radiance-cache tracer at 1% rel-MSE.

    rel-MSE of an image I = mean over pixels and wavelengths of
    (I - T)^2 / (T^2 + 0.01 mean(T)^2) against the converged image T.  It is
    estimated without bias from three independent plain references (disjoint
    sample ranges): R = (R1 + R2) / 2 and var R = (R1 - R2)^2 / 4 (``ref_frames``
    frames each) make (I - R)^2 - var R an unbiased estimate of (I - T)^2; the
    weights 1 / (T3^2 + 0.01 mean(T3)^2) come from the third reference (twice
    the frames, box-filtered over 3 x 3 pixels to tame its noise), so they are
    fixed per element and independent of I and R.

    Each method traces ``frames_per_step`` frames per step into two interleaved halves (even
    and odd frames).  The plain estimator is unbiased: its rel-MSE after n
    frames is b / n.  The cache's is a + b / n with a the squared bias of its
    accumulated image, measured at the end as the mean of
    w ((I - R)^2 - var R - var I), var I = (I_even - I_odd)^2 / 4; later frames
    of a trained cache are no more biased than earlier ones, so a is an upper
    estimate for longer runs.  b is fitted over the second half of each curve
    (with the floor fixed at 0 and at a), and the time to 1% is read from the
    fits: frames n = b / (0.01 - a) at the method's measured time per frame,
    plus the cache's training warm-up.  Warm-up steps (one plain and one cache
    frame each, discarded) precede the timed runs."""
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
    if args.nrc_warmup is not None:
        cfg["train_warmup"] = args.nrc_warmup
    if args.nrc_table_fp16 is not None:
        cfg["table_fp16"] = bool(args.nrc_table_fp16)
    nl = len(scene["lambda_nm"])
    cam = scene["camera"]
    frames = args.frames_per_step * max(args.steps, 2)

    def trace(rid, off, nrc):
        tr.trace_spectral(cam, W, H, spp, D, seed=0, render_id=rid, sample_offset=off, nrc=nrc, time_kernels=True)
        s, _ = tr.resolve_image(rid, W, H, spectral=True, xyz=True)
        return s

    def init_cache():
        params, tables = scenegen.nrc_params(0)
        tr.nrc_init(params, tables, ROOM_LO, ROOM_HI, lr=cfg["lr"], train_paths=cfg["train_paths"],
                    train_steps=cfg["train_steps"], train_batch=cfg["train_batch"], precision="bf16",
                    table_fp16=cfg.get("table_fp16", False))

    if args.cache_only:
        return cache_frames_only(args, tr, wl, cfg, nl, frames, trace, init_cache)

    t0 = time.perf_counter()
    refs = []
    for k in range(3):
        for f in range(cfg["ref_frames"] * (2 if k == 2 else 1)):
            trace(10 + k, (k + 1) * 1_000_000 + f * spp, False)
        refs.append(tr.resolve_image(10 + k, W, H, spectral=True, xyz=False)[0])
        tr.reset_render(10 + k)
    R = 0.5 * (refs[0] + refs[1])
    varR = 0.25 * (refs[0] - refs[1]) ** 2
    # the weights: the third reference (twice the samples), box-filtered over 3 x 3 pixels per wavelength
    T3 = torch.nn.functional.avg_pool2d(refs[2].T.reshape(1, nl, H, W), 3, stride=1, padding=1,
                                        count_include_pad=False).reshape(nl, H * W).T
    wgt = 1.0 / (T3 * T3 + 0.01 * T3.mean() ** 2)
    del refs, T3
    ref_spp = 2 * cfg["ref_frames"] * spp
    ref_rel = float((varR * wgt).mean())   # the reference's own rel-MSE
    log(f"[bench] references: 3 x {cfg['ref_frames'] * spp} spp in {time.perf_counter() - t0:.1f} s; "
        f"R's own rel-MSE {ref_rel:.3e}")

    def relmse(img):
        return float((((img - R) ** 2 - varR) * wgt).mean())

    init_cache()
    for i in range(args.warmup):
        trace(20, 5_000_000 + i * spp, False)
        trace(21, 6_000_000 + i * spp, True)
        torch.cuda.synchronize()
        log(f"[bench] warmup {i + 1}/{args.warmup}")
    tr.reset_render(20)
    tr.reset_render(21)

    def run(rids, nrc, n_frames, warm=0):
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        for f in range(warm):  # cache training frames, not accumulated
            trace(3, 3_000_000 + f * spp, True)
        torch.cuda.synchronize()
        if warm:
            tr.reset_render(3)
        warm_s = time.perf_counter() - t1
        tt, hist = 0.0, []
        mean, cnt = {}, {rids[0]: 0, rids[1]: 0}
        for f in range(n_frames):
            rid = rids[f % 2]
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            mean[rid] = trace(rid, f * spp, nrc)
            torch.cuda.synchronize()
            tt += time.perf_counter() - t1
            cnt[rid] += 1
            img = sum(mean[r] * cnt[r] for r in mean) / (f + 1)
            hist.append((f + 1, tt, relmse(img)))
            if f % 20 == 19 or f == n_frames - 1:
                log(f"[bench] {'cache' if nrc else 'plain'} frame {f + 1}: {tt:.2f} s, rel-MSE {hist[-1][2]:.4f}")
        bias2, bias2_se, var_w = error_split(mean[rids[0]], mean[rids[1]], R, varR, wgt)
        b_direct = n_frames * var_w
        for r in rids:
            tr.reset_render(r)
        return dict(hist=hist, warm_s=warm_s, t=tt, bias2=bias2, bias2_se=bias2_se, b_direct=b_direct)

    tr.reset_stats()
    P = run((1, 4), False, frames)
    stp = tr.stats()
    init_cache()
    tr.reset_stats()
    C = run((2, 5), True, frames, warm=cfg["train_warmup"])
    stn = tr.stats()

    def second_half(h):
        return h[len(h) // 2:]

    ap_free, bp_free = relmse_fit(second_half(P["hist"]), floor=True)
    _, bp = relmse_fit(second_half(P["hist"]), floor=False)
    a_c = max(0.0, C["bias2"])
    hc = np.asarray(second_half(C["hist"]))
    bc = float(np.sum((hc[:, 2] - a_c) / hc[:, 0]) / np.sum(1.0 / hc[:, 0] ** 2))
    ac_free, bc_free = relmse_fit(second_half(C["hist"]), floor=True)
    fr_plain = P["t"] / frames
    fr_nrc = C["t"] / frames
    n_plain = frames_to(TARGET_REL_MSE, 0.0, bp)
    n_nrc = frames_to(TARGET_REL_MSE, a_c, bc)
    t1_plain = n_plain * fr_plain if n_plain else None
    t1_nrc = C["warm_s"] + n_nrc * fr_nrc if n_nrc else None
    log(f"[bench] plain: {fr_plain * 1e3:.1f} ms/frame, rel-MSE {P['hist'][-1][2]:.4f} after {frames} frames; "
        f"bias^2 {P['bias2']:.4f} +- {P['bias2_se']:.4f} (control: the plain estimator is unbiased), b {bp:.2f} "
        f"(direct {P['b_direct']:.2f}; free fit a {ap_free:.4f}): 1% after {n_plain:.0f} frames, {t1_plain:.1f} s")
    log(f"[bench] cache: {fr_nrc * 1e3:.1f} ms/frame, warm-up {C['warm_s']:.2f} s, rel-MSE {C['hist'][-1][2]:.4f} "
        f"after {frames} frames; bias^2 {C['bias2']:.4f} +- {C['bias2_se']:.4f}, b {bc:.2f} "
        f"(direct {C['b_direct']:.2f}; free fit a {ac_free:.4f} b {bc_free:.2f}): "
        + (f"1% after {n_nrc:.0f} frames, {t1_nrc:.1f} s" if n_nrc else "floor at or above 1%"))
    value = n_plain * W * H * spp * nl / t1_nrc if (t1_nrc and n_plain) else None
    kern = {"trace": stn["ms_trace_ext"] + stn["ms_trace_shadow"], "nrc_query": stn["ms_nrc_query"]}
    dominant = max(kern, key=kern.get)
    traffic_q = measured_traffic("nrc_room", wl["grid"])
    rq = query_roofline(stn, nl, traffic_q)
    rt = trace_roofline(stn, measured_traffic("nrc_room_trace", wl["grid"]))
    return {
        "metric": "spectral path samples/s (rays x lambda/s) at <=1% rel-MSE; radiance cache vs plain, one MI355X",
        "value": value,
        "unit": "plain-equivalent path samples*lambda/s",
        "ms_per_step": (P["t"] + C["warm_s"] + C["t"]) / max(args.steps, 2) * 1e3,
        "dtype": "bf16 cache network, f32 traversal and per-lambda transport, f64 path state and resolve",
        "comparison": {
            "target_rel_mse": TARGET_REL_MSE, "frames_per_step": args.frames_per_step, "frames_per_method": frames,
            "estimator": "unbiased: (I-R)^2 - var R over two independent plain references, weights 1/(T3^2 + "
                         "0.01 mean(T3)^2) from a third (T3: 3x3 box filter of it, twice the samples)",
            "reference": {"spp_in_R": ref_spp, "spp_in_weight_reference": 2 * cfg["ref_frames"] * spp,
                          "own_rel_mse": ref_rel,
                          "spp_for_own_rel_mse_1e-4": ref_spp * ref_rel / 1e-4},
            "plain": {"ms_per_frame": fr_plain * 1e3, "path_samples_lambda_per_s": W * H * spp * nl / fr_plain,
                      "rays_lambda_per_s": (stp["ext_rays"] + stp["shadow_rays"]) * nl / P["t"],
                      "rel_mse_reached": P["hist"][-1][2], "bias2": [P["bias2"], P["bias2_se"]],
                      "fit_b": bp, "b_direct": P["b_direct"], "fit_a_b_free": [ap_free, bp_free],
                      "frames_to_1pct": n_plain, "seconds_to_1pct": t1_plain},
            "cache": {"train_warmup_frames": cfg["train_warmup"], "warmup_s": C["warm_s"],
                      "ms_per_frame": fr_nrc * 1e3, "path_samples_lambda_per_s": W * H * spp * nl / fr_nrc,
                      "rays_lambda_per_s": (stn["ext_rays"] + stn["shadow_rays"]) * nl / (C["t"] + C["warm_s"]),
                      "rel_mse_reached": C["hist"][-1][2], "bias2": [C["bias2"], C["bias2_se"]],
                      "fit_a_b": [a_c, bc], "b_direct": C["b_direct"], "fit_a_b_free": [ac_free, bc_free],
                      "frames_to_1pct": n_nrc, "seconds_to_1pct": t1_nrc,
                      "ms_query_mfma_per_frame": stn["ms_nrc_query"] / (frames + cfg["train_warmup"]),
                      "ms_train_per_frame": stn["ms_nrc_train"] / (frames + cfg["train_warmup"])},
            "speedup_to_1pct": (t1_plain / t1_nrc) if (t1_nrc and t1_plain) else None,
            "cache_settings": {k: cfg.get(k) for k in ("train_paths", "train_steps", "train_batch", "lr",
                                                       "table_fp16")},
        },
        "roofline": rt if dominant == "trace" else rq,
        "roofline_query": rq,
        "kernel_ms_per_cache_frame": {k: v / (frames + cfg["train_warmup"]) for k, v in kern.items()},
    }


def cache_frames_only(args, tr, wl, cfg, nl, frames, trace, init_cache):
    """The cache side of the comparison alone, for profiling: the cache's
    training warm-up and its frames, as in the comparison, without the
    references and the plain frames, so that a kernel trace or counter run of
    this command covers exactly the launches the cache line's roofline
    averages over."""
    import torch

    init_cache()
    tr.reset_stats()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    for f in range(cfg["train_warmup"]):
        trace(3, 3_000_000 + f * wl["spp"], True)
    tr.reset_render(3)
    for f in range(frames):
        trace(2, f * wl["spp"], True)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t1
    stn = tr.stats()
    n = frames + cfg["train_warmup"]
    return {"metric": "radiance-cache frames only (profiling run of the cache line's kernels)",
            "frames": n, "ms_per_frame": dt / n * 1e3,
            "roofline": trace_roofline(stn, measured_traffic("nrc_room_trace", wl["grid"])),
            "roofline_query": query_roofline(stn, nl, measured_traffic("nrc_room", wl["grid"])),
            "kernel_ms_per_cache_frame": {"trace": (stn["ms_trace_ext"] + stn["ms_trace_shadow"]) / n,
                                          "nrc_query": stn["ms_nrc_query"] / n}}


def plain_line(args, workload, wl, scene, tr, build_s, cpu_s):
    """Plain throughput of one workload: warm-up steps, then K timed frames."""
    import torch

    import scenegen

    W, H, spp, D = wl["W"], wl["H"], wl["spp"], wl["D"]
    nl = len(scene["lambda_nm"])
    cam = scene["camera"]
    renders = None
    if "batch" in wl:
        bw = wl["batch"]
        scene, base, states = scenegen.photochromic_states(scene, bw["n_states"])
        renders = scenegen.batch_renders(bw["n"], bw["seed"], bw["n_states"], spp=bw["spp"])
        for r in renders:
            r["glass_swap"] = (base, states[r["state"]])
        tr.load_scene(scene)
        tr.build_bvh(*wl["grid"], device=args.device_bvh)
    step = 0

    def frame(graph=False, t=None):
        nonlocal step
        t = t or tr
        # every launch is bracketed by HIP events on the library's stream (not in graph replays)
        if renders is None:
            t.trace_spectral(cam, W, H, spp, D, sample_offset=step * spp, render_id=0, time_kernels=not graph,
                             graph=graph)
            t.resolve_image(0, W, H, spectral=True, xyz=True)
        else:
            for r in renders:
                r["sample_offset"] = step * r["spp"]
            t.trace_batch(renders, D, time_kernels=not graph, graph=graph)
            for r in renders:
                t.resolve_image(r["render_id"], r["W"], r["H"], spectral=True, xyz=True)
        step += 1

    if args.defer_rays:
        tr.set_deferral(args.defer_rays, args.defer_extra)
    tuned = None
    if args.autotune is not None:
        t0 = time.perf_counter()
        call = renders if renders is not None else [dict(camera=cam, W=W, H=H, spp=spp, render_id=0)]
        tuned = tr.autotune(call, D, reps=2, cache=args.autotune or None)
        log(f"[bench] autotune {tuned} ({time.perf_counter() - t0:.1f} s)")

    for i in range(args.warmup):
        frame()
        torch.cuda.synchronize()
        log(f"[bench] {workload} warmup {i + 1}/{args.warmup}")

    tr.reset_stats()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        frame()
        log(f"[bench] {workload} step {i + 1}/{args.steps}")
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    st = tr.stats()
    rays = st["ext_rays"] + st["shadow_rays"]
    kern_ms = {"trace_ext": st["ms_trace_ext"], "trace_shadow": st["ms_trace_shadow"], "shade": st["ms_shade"],
               "other": st["ms_other"]}
    log(f"[bench] {workload} timed {dt:.3f} s; kernel ms {kern_ms}")
    if renders is None:
        paths_per_step = W * H * spp
        frame_desc = f"{W}x{H}, {spp} spp"
    else:
        paths_per_step = sum(r["W"] * r["H"] * r["spp"] for r in renders)
        frame_desc = (f"{len(renders)} renders {min(r['W'] for r in renders)}^2..{max(r['W'] for r in renders)}^2 "
                      f"({sum(r['W'] * r['H'] for r in renders)} px), {renders[0]['spp']} spp, "
                      f"{wl['batch']['n_states']} photochromic states")
    res = {
        "metric": "spectral path samples/s (rays x lambda/s), plain tracer, one MI355X",
        "value": rays * nl / dt,
        "unit": "rays*lambda/s",
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": dt / args.steps * 1e3,
        "dtype": ("f32 traversal, path state and per-lambda transport, f64 resolve (FP32-path-state measurement "
                  "build)" if os.environ.get("SDD_PATH_STATE") == "f32"
                  else "f32 traversal and per-lambda transport, f64 path state and resolve"),
        "config": {"workload": f"{workload}: {len(scene['tris'])} tris, {frame_desc}, {nl} lambda, depth {D}, "
                               f"grid {'x'.join(map(str, wl['grid']))}",
                   "paths_per_step": paths_per_step, "rays_per_step": rays / args.steps,
                   "path_samples_lambda_per_s": paths_per_step * nl * args.steps / dt},
        "roofline": trace_roofline(st, measured_traffic(workload, wl["grid"])),
        "kernel_ms_per_step": {k: v / args.steps for k, v in kern_ms.items()},
        "build_bvh_s": build_s,
        "bvh": "device LBVH" if args.device_bvh else "host binned SAH",
        "deferral": {"below_rays": args.defer_rays, "extra_sweeps": args.defer_extra} if args.defer_rays else None,
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
                       "scene_bytes_per_frame": 64 * sw["node_visits"] + 48 * sw["tri_tests"],
                       # lanes busy per wave step of the traversal's node loop and triangle loop
                       "node_loop_lane_utilisation": sw["node_visits"] / max(1, 64 * sw["wave_node_steps"]),
                       "tri_loop_lane_utilisation": sw["tri_tests"] / max(1, 64 * sw["wave_tri_steps"])}
    if args.graph:
        import paper_1912_06474_amd as sdd
        gt = sdd.Tracer(stream=torch.cuda.Stream())  # graph capture needs a stream other than the null stream
        gt.load_scene(scene)
        gt.build_bvh(*wl["grid"], device=args.device_bvh)
        frame(graph=True, t=gt)  # capture
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            frame(graph=True, t=gt)
        torch.cuda.synchronize()
        dtg = time.perf_counter() - t0
        res["graph_replay"] = {"ms_per_step": dtg / args.steps * 1e3, "value": rays * nl / dtg,
                               "note": "same steps replayed from one captured HIP graph, without per-launch events"}
        log(f"[bench] graph replay: {dtg / args.steps * 1e3:.2f} ms per step")
        gt.close()
    if cpu_s > 0:
        res["cpu_baseline"] = cpu_baseline(scene, wl, cpu_s)
    return res


def load(workload, args):
    import paper_1912_06474_amd as sdd
    import scenegen

    wl = dict(WORKLOADS[workload])
    if args.grid:
        wl["grid"] = tuple(int(x) for x in args.grid.lower().split("x"))
    name, kw = wl["scene"]
    t0 = time.perf_counter()
    scene = getattr(scenegen, name)(**kw)
    log(f"[bench] scene {scene['name']}: {len(scene['tris'])} tris, {len(scene['lambda_nm'])} lambda "
        f"({time.perf_counter() - t0:.1f} s)")
    tr = sdd.Tracer()
    tr.load_scene(scene)
    t0 = time.perf_counter()
    tr.build_bvh(*wl["grid"], device=args.device_bvh)
    build_s = time.perf_counter() - t0
    st0 = tr.stats()
    log(f"[bench] build_bvh {wl['grid']}: {build_s:.2f} s, refs {st0['n_refs']}, nodes {st0['n_nodes']}, "
        f"depth {st0['max_bvh_depth']}")
    return wl, scene, tr, build_s


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="nrc_room", choices=sorted(WORKLOADS))
    ap.add_argument("--grid", default=None, help="override subdomain grid, e.g. 1x1x1")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-plain-line", action="store_true",
                    help="nrc_room: skip the room-scale plain sub-line")
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--count-work", action="store_true",
                    help="trace one extra (untimed) frame counting BVH node visits and triangle tests")
    ap.add_argument("--device-bvh", action="store_true",
                    help="build the subdomain BVHs on the GPU (linear BVH per cell) instead of the host SAH build")
    ap.add_argument("--graph", action="store_true",
                    help="also time the same steps replayed from a captured HIP graph (no per-launch events)")
    ap.add_argument("--ref-frames", type=int, default=None,
                    help="nrc_room: frames in each of the two plain references (the weights' reference takes twice "
                         "as many; default 64)")
    ap.add_argument("--frames-per-step", type=int, default=FRAMES_PER_STEP,
                    help="nrc_room: frames of each method per step (default %(default)s)")
    ap.add_argument("--nrc-train-steps", type=int, default=None, help="nrc_room: Adam steps per frame (default 8)")
    ap.add_argument("--nrc-train-batch", type=int, default=None, help="nrc_room: rows per Adam step (default 2^14)")
    ap.add_argument("--nrc-lr", type=float, default=None, help="nrc_room: Adam learning rate (default 1e-2)")
    ap.add_argument("--nrc-table-fp16", type=int, choices=[0, 1], default=None,
                    help="nrc_room: 1 = BF16 queries gather from an FP16 copy of the hash tables")
    ap.add_argument("--nrc-warmup", type=int, default=None,
                    help="nrc_room: cache training frames before accumulation (default 100; their time counts)")
    ap.add_argument("--autotune", nargs="?", const="", default=None, metavar="FILE",
                    help="search the launch settings on the step's own call before the warmup (results file "
                         "FILE is read first and written after a search)")
    ap.add_argument("--defer-rays", type=int, default=0,
                    help="plain workloads: queues with fewer rays wait a sweep (the paper's deferral rule; 0: off)")
    ap.add_argument("--defer-extra", type=int, default=2, help="extra sweeps per depth for --defer-rays")
    ap.add_argument("--path-state", choices=["f64", "f32"], default="f64",
                    help="f32: load the FP32-path-state measurement build (libsdd_f32state.so) to time what FP64 "
                         "path state costs; the library itself keeps FP64 path state")
    ap.add_argument("--cache-only", action="store_true",
                    help="nrc_room: only the cache's warm-up and frames (profiling the cache line's kernels)")
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
    if args.path_state == "f32":
        os.environ["SDD_PATH_STATE"] = "f32"  # read when the package is first imported

    cpu_s = 0.0 if args.no_cpu_baseline else args.cpu_seconds
    wl, scene, tr, build_s = load(args.workload, args)
    common = {"n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "higher_is_better": True,
              "scaling": "weak", "vs_baseline": None, "data": "synthetic"}
    if "nrc" in wl:
        W, H, spp, D = wl["W"], wl["H"], wl["spp"], wl["D"]
        res = nrc_comparison(args, tr, scene, wl)
        if args.cache_only:
            tr.close()
            print(json.dumps(res))
            return
        res.update(common)
        res["config"] = {"workload": f"{args.workload}: {len(scene['tris'])} tris, {W}x{H}, {spp} spp per frame, "
                                     f"{len(scene['lambda_nm'])} lambda, depth {D}, cache after vertex 2, grid "
                                     f"{'x'.join(map(str, wl['grid']))}; plain vs radiance cache to 1% rel-MSE"}
        res["build_bvh_s"] = build_s
        if cpu_s > 0:
            res["cpu_baseline"] = cpu_baseline(scene, wl, cpu_s)
            res["cpu_oracle_cases"] = cpu_oracle_cases()
        tr.close()
        del scene
        if not args.no_plain_line:
            wl1, scene1, tr1, build1 = load("furnished_room", args)
            res["plain_room_scale"] = plain_line(args, "furnished_room", wl1, scene1, tr1, build1, cpu_s)
            tr1.close()
        print(json.dumps(res))
        return

    res = plain_line(args, args.workload, wl, scene, tr, build_s, cpu_s)
    res.update(common)
    print(json.dumps(res))


if __name__ == "__main__":
    main()
