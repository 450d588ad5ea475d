"""Spectral domain-decomposition ray tracing on MI355X (gfx950).

Thin ctypes binding of ``libsdd.so`` (C ABI in ``include/sdd.h``).  It only
marshals arguments: every step of the rendering runs in the library's HIP
kernels.  PyTorch supplies device memory (outputs, debug logs) and the HIP
stream.  There is no CPU fallback: if the library is missing or no GPU is
present, the calls raise.

    t = Tracer()                        # context on cuda:0, torch's current stream
    t.load_scene(scene)                 # dict of arrays (see scenegen)
    t.build_bvh(4, 4, 2)                # subdomain grid + per-subdomain BVHs
    t.trace_spectral(camera, 512, 512, spp=16, max_depth=8)
    spec, xyz = t.resolve_image()       # FP64 torch tensors on the device
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
# SDD_PATH_STATE=f32 selects the FP32-path-state measurement build (the same
# kernels with the per-path ray state and shading geometry in FP32), which
# exists to state what FP64 path state buys in accuracy and costs in time
LIB_PATH = os.path.join(HERE, "libsdd_f32state.so" if os.environ.get("SDD_PATH_STATE") == "f32" else "libsdd.so")

SDD_OK = 0
STATUS = {0: "SDD_OK", -1: "SDD_ERR_INVALID_ARG", -2: "SDD_ERR_STATE", -3: "SDD_ERR_OOM", -4: "SDD_ERR_HIP",
          -5: "SDD_ERR_OVERFLOW", -6: "SDD_ERR_UNSUPPORTED"}
TRACE_ORTHO, TRACE_TIME_KERNELS, TRACE_COUNT_WORK, TRACE_NRC, TRACE_GRAPH = 1, 2, 4, 8, 16

EXPORTS = ("sdd_create", "sdd_destroy", "sdd_last_error", "sdd_load_scene", "sdd_validate_scene", "sdd_build_bvh",
           "sdd_trace_spectral", "sdd_resolve_image", "sdd_reset_render", "sdd_get_stats", "sdd_reset_stats",
           "sdd_debug_philox", "sdd_debug_pane", "sdd_debug_trace_rays", "sdd_debug_glass", "sdd_trace_batch",
           "sdd_nrc_param_count", "sdd_nrc_init", "sdd_nrc_infer", "sdd_nrc_train_step", "sdd_nrc_get_params",
           "sdd_nrc_last_rows", "sdd_nrc_query", "sdd_nrc_query_noalloc", "sdd_set_deferral")
NRC_LEVELS, NRC_FEAT, NRC_HID, NRC_LAYERS = 16, 2, 64, 5


class SddError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status


class SceneDesc(C.Structure):
    _fields_ = [
        ("n_verts", C.c_int32), ("verts", C.c_void_p),
        ("n_tris", C.c_int32), ("tris", C.c_void_p), ("tri_mat", C.c_void_p),
        ("n_lambda", C.c_int32), ("lambda_nm", C.c_void_p), ("lambda_w", C.c_void_p), ("cmf", C.c_void_p),
        ("n_mats", C.c_int32), ("mat_type", C.c_void_p), ("mat_rho", C.c_void_p), ("mat_n", C.c_void_p),
        ("mat_k", C.c_void_p), ("mat_thick", C.c_void_p), ("mat_le", C.c_void_p),
        ("light_type", C.c_int32), ("light_p0", C.c_float * 3), ("light_e1", C.c_float * 3),
        ("light_e2", C.c_float * 3), ("light_mat", C.c_int32),
        ("max_layers", C.c_int32), ("mat_n_layers", C.c_void_p), ("mat_layer_d", C.c_void_p),
        ("mat_layer_n", C.c_void_p), ("mat_layer_k", C.c_void_p),
    ]


class BvhDesc(C.Structure):
    _fields_ = [("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32), ("leaf_max", C.c_int32),
                ("sah_bins", C.c_int32), ("device_build", C.c_int32)]


class TraceDesc(C.Structure):
    _fields_ = [
        ("eye", C.c_double * 3), ("target", C.c_double * 3), ("fov_deg", C.c_double), ("ortho_half_h", C.c_double),
        ("W", C.c_int32), ("H", C.c_int32), ("spp", C.c_int32), ("sample_offset", C.c_int32),
        ("max_depth", C.c_int32), ("seed", C.c_uint32), ("render_id", C.c_int32), ("flags", C.c_uint32),
        ("hit_log", C.c_void_p), ("shadow_log", C.c_void_p), ("glass_from", C.c_int32), ("glass_to", C.c_int32),
        ("crop_x0", C.c_int32), ("crop_y0", C.c_int32), ("crop_w", C.c_int32), ("crop_h", C.c_int32),
    ]


class NrcDesc(C.Structure):
    _fields_ = [("table_log2", C.c_int32), ("aabb_lo", C.c_float * 3), ("aabb_hi", C.c_float * 3),
                ("lambda_lo", C.c_float), ("lambda_hi", C.c_float), ("lr", C.c_float), ("beta1", C.c_float),
                ("beta2", C.c_float), ("eps", C.c_float), ("params", C.c_void_p),
                ("train_paths", C.c_int32), ("train_steps", C.c_int32), ("train_batch", C.c_int32),
                ("precision", C.c_int32), ("table_fp16", C.c_int32)]


class Tuning(C.Structure):
    _fields_ = [("batch_paths", C.c_int64), ("trace_grid", C.c_int32), ("dir_bins", C.c_int32)]

    def as_dict(self):
        return {"batch_paths": int(self.batch_paths), "trace_grid": int(self.trace_grid),
                "dir_bins": int(self.dir_bins)}


class Stats(C.Structure):
    _fields_ = [
        ("ext_rays", C.c_int64), ("shadow_rays", C.c_int64), ("ext_cell_visits", C.c_int64),
        ("shadow_cell_visits", C.c_int64), ("node_visits", C.c_int64), ("tri_tests", C.c_int64),
        ("batches", C.c_int64), ("launches_trace", C.c_int64),
        ("ms_trace_ext", C.c_double), ("ms_trace_shadow", C.c_double), ("ms_shade", C.c_double),
        ("ms_other", C.c_double),
        ("n_refs", C.c_int64), ("n_nodes", C.c_int64), ("max_bvh_depth", C.c_int32), ("n_cells", C.c_int32),
        ("device_bytes", C.c_int64), ("paths_per_batch", C.c_int64), ("overflow", C.c_int32), ("pad_", C.c_int32),
        ("ms_nrc_query", C.c_double), ("ms_nrc_train", C.c_double), ("nrc_query_rows", C.c_int64),
        ("nrc_query_launches", C.c_int64), ("nrc_train_rows", C.c_int64),
        ("wave_node_steps", C.c_int64), ("wave_tri_steps", C.c_int64),
    ]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_ if k != "pad_"}


_LIB = None


def lib():
    """Load libsdd.so (raises if it has not been built)."""
    global _LIB
    if _LIB is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -m paper_1912_06474_amd.build` "
                               "(there is no CPU fallback)")
        L = C.CDLL(LIB_PATH)
        vp, i32 = C.c_void_p, C.c_int32
        L.sdd_create.argtypes = [C.c_int, vp, C.POINTER(vp)]
        L.sdd_destroy.argtypes = [vp]
        L.sdd_destroy.restype = None
        L.sdd_last_error.argtypes = [vp]
        L.sdd_last_error.restype = C.c_char_p
        L.sdd_load_scene.argtypes = [vp, C.POINTER(SceneDesc)]
        L.sdd_validate_scene.argtypes = [C.POINTER(SceneDesc), C.c_char_p, C.c_int]
        L.sdd_build_bvh.argtypes = [vp, C.POINTER(BvhDesc)]
        L.sdd_trace_spectral.argtypes = [vp, C.POINTER(TraceDesc)]
        L.sdd_resolve_image.argtypes = [vp, i32, vp, vp, i32]
        L.sdd_reset_render.argtypes = [vp, i32]
        L.sdd_get_stats.argtypes = [vp, C.POINTER(Stats)]
        L.sdd_reset_stats.argtypes = [vp]
        L.sdd_debug_philox.argtypes = [vp, i32, vp, vp, vp]
        L.sdd_debug_pane.argtypes = [vp, i32, vp, vp, vp]
        L.sdd_debug_trace_rays.argtypes = [vp, i32, vp, vp, vp, vp]
        L.sdd_debug_glass.argtypes = [vp, i32, vp, vp, vp, vp, vp]
        L.sdd_trace_batch.argtypes = [vp, i32, C.POINTER(TraceDesc)]
        L.sdd_nrc_param_count.argtypes = [i32]
        L.sdd_nrc_param_count.restype = C.c_int64
        L.sdd_nrc_init.argtypes = [vp, C.POINTER(NrcDesc)]
        L.sdd_nrc_infer.argtypes = [vp, i32, vp, vp, vp, vp, i32]
        L.sdd_nrc_train_step.argtypes = [vp, i32, vp, vp, vp, vp, i32, C.POINTER(C.c_float)]
        L.sdd_nrc_get_params.argtypes = [vp, i32, vp]
        L.sdd_nrc_query.argtypes = [vp, i32, vp, vp, vp, i32]
        L.sdd_nrc_query_noalloc.argtypes = [vp, i32, vp, vp, vp]
        L.sdd_nrc_last_rows.argtypes = [vp, i32, vp, C.POINTER(C.c_int32), C.POINTER(C.c_int32),
                                        C.POINTER(C.c_float)]
        tp = C.POINTER(Tuning)
        L.sdd_validate_tuning.argtypes = [tp, C.c_char_p, C.c_int]
        L.sdd_set_tuning.argtypes = [vp, tp]
        L.sdd_set_deferral.argtypes = [vp, i32, i32]
        L.sdd_get_tuning.argtypes = [vp, tp]
        L.sdd_autotune.argtypes = [vp, i32, C.POINTER(TraceDesc), i32, C.c_char_p, tp, C.POINTER(C.c_double),
                                   C.POINTER(C.c_int32)]
        L.sdd_tune_key.argtypes = [vp, i32, C.POINTER(TraceDesc), C.c_char_p, i32]
        L.sdd_tune_cache_lookup.argtypes = [C.c_char_p, C.c_char_p, tp, C.POINTER(C.c_double), C.POINTER(C.c_int32)]
        L.sdd_tune_cache_store.argtypes = [C.c_char_p, C.c_char_p, tp, C.c_double]
        _LIB = L
    return _LIB


def _ptr(a):
    return a.ctypes.data_as(C.c_void_p)


class _SceneArrays:
    """Contiguous host copies of a scene dict and the C descriptor over them."""

    def __init__(self, scene):
        self.keep = {}

        def arr(key, dt):
            a = np.ascontiguousarray(scene[key], dtype=dt)
            self.keep[key] = a
            return a

        verts, tris, tri_mat = arr("verts", np.float32), arr("tris", np.int32), arr("tri_mat", np.int32)
        lam, w, cmf = arr("lambda_nm", np.float32), arr("lambda_w", np.float64), arr("cmf", np.float64)
        mt = arr("mat_type", np.int32)
        rho, mn, mk, le = (arr(k, np.float32) for k in ("mat_rho", "mat_n", "mat_k", "mat_le"))
        th = arr("mat_thick", np.float32)
        d = SceneDesc()
        d.n_verts, d.verts = len(verts), _ptr(verts)
        d.n_tris, d.tris, d.tri_mat = len(tris), _ptr(tris), _ptr(tri_mat)
        d.n_lambda, d.lambda_nm, d.lambda_w, d.cmf = len(lam), _ptr(lam), _ptr(w), _ptr(cmf)
        d.n_mats, d.mat_type = len(mt), _ptr(mt)
        d.mat_rho, d.mat_n, d.mat_k, d.mat_thick, d.mat_le = _ptr(rho), _ptr(mn), _ptr(mk), _ptr(th), _ptr(le)
        d.light_type = int(scene["light_type"])
        d.light_p0[:] = [float(x) for x in np.asarray(scene["light_p0"]).reshape(3)]
        d.light_e1[:] = [float(x) for x in np.asarray(scene["light_e1"]).reshape(3)]
        d.light_e2[:] = [float(x) for x in np.asarray(scene["light_e2"]).reshape(3)]
        d.light_mat = int(scene["light_mat"])
        if "mat_n_layers" in scene:
            nlay = arr("mat_n_layers", np.int32)
            ld = arr("mat_layer_d", np.float32)
            ln, lk = arr("mat_layer_n", np.float32), arr("mat_layer_k", np.float32)
            d.max_layers = int(ld.shape[1]) if ld.ndim == 2 else 0
            d.mat_n_layers, d.mat_layer_d, d.mat_layer_n, d.mat_layer_k = _ptr(nlay), _ptr(ld), _ptr(ln), _ptr(lk)
        self.desc = d
        self.n_lambda = len(lam)


def validate_scene(scene):
    """Host-only validation (no GPU needed).  Returns (ok, message)."""
    sa = _SceneArrays(scene)
    buf = C.create_string_buffer(512)
    st = lib().sdd_validate_scene(C.byref(sa.desc), buf, 512)
    return st == SDD_OK, buf.value.decode()


def validate_tuning(batch_paths=0, trace_grid=0, dir_bins=0):
    """Host-only check of launch settings.  Returns (ok, message)."""
    buf = C.create_string_buffer(256)
    st = lib().sdd_validate_tuning(C.byref(Tuning(batch_paths, trace_grid, dir_bins)), buf, 256)
    return st == SDD_OK, buf.value.decode()


def tune_cache_lookup(path, key):
    """(settings dict with "ms", or None) for key in a results file (host only)."""
    t, ms, found = Tuning(), C.c_double(0.0), C.c_int32(0)
    st = lib().sdd_tune_cache_lookup(str(path).encode(), key.encode(), C.byref(t), C.byref(ms), C.byref(found))
    if st != SDD_OK:
        raise SddError(st, "sdd_tune_cache_lookup failed")
    if not found.value:
        return None
    return dict(t.as_dict(), ms=ms.value)


def tune_cache_store(path, key, batch_paths=0, trace_grid=0, dir_bins=0, ms=0.0):
    """Replace key's entry of a results file (host only)."""
    st = lib().sdd_tune_cache_store(str(path).encode(), key.encode(),
                                    C.byref(Tuning(batch_paths, trace_grid, dir_bins)), float(ms))
    if st != SDD_OK:
        raise SddError(st, "sdd_tune_cache_store failed")


class Tracer:
    """One library context on one HIP device (torch's current stream by default)."""

    def __init__(self, device: int = 0, stream=None):
        import torch
        if not torch.cuda.is_available():
            raise RuntimeError("no HIP device visible: the spectral tracer runs only on the GPU")
        self.torch = torch
        self.device = torch.device("cuda", device)
        if stream is None:
            stream = torch.cuda.current_stream(self.device)
        self.stream = stream
        h = C.c_void_p()
        st = lib().sdd_create(int(device), C.c_void_p(stream.cuda_stream), C.byref(h))
        if st != SDD_OK:
            raise SddError(st, "sdd_create failed")
        self.h = h
        self.n_lambda = 0

    def close(self):
        if getattr(self, "h", None):
            lib().sdd_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, st):
        if st != SDD_OK:
            raise SddError(st, lib().sdd_last_error(self.h).decode())

    def load_scene(self, scene):
        sa = _SceneArrays(scene)
        self._check(lib().sdd_load_scene(self.h, C.byref(sa.desc)))
        self.n_lambda = sa.n_lambda

    def build_bvh(self, nx=1, ny=1, nz=1, leaf_max=3, sah_bins=16, device=False):
        """Subdomain grid and per-cell BVHs: host binned SAH, or with device=True a
        linear BVH per cell built on the GPU."""
        self._check(lib().sdd_build_bvh(self.h, C.byref(BvhDesc(nx, ny, nz, leaf_max, sah_bins, int(bool(device))))))

    def _desc(self, camera, W, H, spp, max_depth, seed=0, render_id=0, sample_offset=0, time_kernels=False,
              count_work=False, hit_log=None, shadow_log=None, glass_swap=None, nrc=False, graph=False, crop=None):
        d = TraceDesc()
        d.eye[:] = [float(x) for x in camera["eye"]]
        d.target[:] = [float(x) for x in camera["target"]]
        d.fov_deg = float(camera.get("fov_deg", 60.0))
        d.ortho_half_h = float(camera.get("ortho_half_h", 1.0))
        d.W, d.H, d.spp, d.sample_offset, d.max_depth = int(W), int(H), int(spp), int(sample_offset), int(max_depth)
        d.seed, d.render_id = int(seed), int(render_id)
        fl = 0
        if camera.get("ortho", False):
            fl |= TRACE_ORTHO
        if time_kernels:
            fl |= TRACE_TIME_KERNELS
        if count_work:
            fl |= TRACE_COUNT_WORK
        if nrc:
            fl |= TRACE_NRC
        if graph:
            fl |= TRACE_GRAPH
        d.flags = fl
        if crop is not None:
            d.crop_x0, d.crop_y0, d.crop_w, d.crop_h = (int(v) for v in crop)
        npix = int(W) * int(H) if crop is None else int(crop[2]) * int(crop[3])
        n_slots = npix * int(spp) * int(max_depth)
        for name, t in (("hit_log", hit_log), ("shadow_log", shadow_log)):
            if t is not None:
                if not (t.is_cuda and t.dtype == self.torch.int32 and t.is_contiguous() and t.numel() == n_slots):
                    raise ValueError(f"{name} must be a contiguous int32 CUDA tensor of {n_slots} elements")
                setattr(d, name, t.data_ptr())
        d.glass_from, d.glass_to = (-1, -1) if glass_swap is None else (int(glass_swap[0]), int(glass_swap[1]))
        return d

    def trace_spectral(self, camera, W, H, spp, max_depth, *, seed=0, render_id=0, sample_offset=0,
                       time_kernels=False, count_work=False, hit_log=None, shadow_log=None, glass_swap=None,
                       nrc=False, graph=False, crop=None):
        """Trace spp samples of every pixel; glass_swap = (from_material, to_material) substitutes a
        glass material for this render (photochromic state); nrc=True uses the radiance cache
        (paths end in the cache, training paths train it after the call); graph=True captures the
        call's launches in a HIP graph replayed by later calls that differ only in sample_offset; crop =
        (x0, y0, w, h) traces only that window of the W x H frame (logs and resolve_image then cover the
        window: pass w, h there)."""
        d = self._desc(camera, W, H, spp, max_depth, seed, render_id, sample_offset, time_kernels, count_work,
                       hit_log, shadow_log, glass_swap, nrc, graph, crop)
        self._check(lib().sdd_trace_spectral(self.h, C.byref(d)))

    def trace_batch(self, renders, max_depth, *, seed=0, time_kernels=False, count_work=False, graph=False):
        """Several renders in one pipeline pass.  renders: list of dicts with keys camera, W, H, spp,
        render_id and optionally sample_offset, hit_log, shadow_log, glass_swap."""
        arr = (TraceDesc * len(renders))()
        for i, r in enumerate(renders):
            arr[i] = self._desc(r["camera"], r["W"], r["H"], r["spp"], max_depth, seed, r["render_id"],
                                r.get("sample_offset", 0), time_kernels, count_work, r.get("hit_log"),
                                r.get("shadow_log"), r.get("glass_swap"), graph=graph)
        self._check(lib().sdd_trace_batch(self.h, len(renders), arr))

    def _batch_descs(self, renders, max_depth, seed=0, count_work=False, graph=False):
        arr = (TraceDesc * len(renders))()
        for i, r in enumerate(renders):
            arr[i] = self._desc(r["camera"], r["W"], r["H"], r["spp"], max_depth, seed, r["render_id"],
                                r.get("sample_offset", 0), False, count_work, None, None, r.get("glass_swap"),
                                graph=graph)
        return arr

    def set_tuning(self, batch_paths=0, trace_grid=0, dir_bins=0):
        """Launch settings for later calls (0 = the library's choice); images do not change."""
        self._check(lib().sdd_set_tuning(self.h, C.byref(Tuning(batch_paths, trace_grid, dir_bins))))

    def set_deferral(self, below_rays, extra_sweeps=2):
        """Small queues (fewer than below_rays rays) wait a sweep while their rays can still drain;
        extra_sweeps sweeps per depth are added (0 turns deferral off)."""
        self._check(lib().sdd_set_deferral(self.h, int(below_rays), int(extra_sweeps)))

    def get_tuning(self):
        t = Tuning()
        self._check(lib().sdd_get_tuning(self.h, C.byref(t)))
        return t.as_dict()

    def tune_key(self, renders, max_depth, *, count_work=False, graph=False):
        arr = self._batch_descs(renders, max_depth, count_work=count_work, graph=graph)
        buf = C.create_string_buffer(1024)
        self._check(lib().sdd_tune_key(self.h, len(renders), arr, buf, 1024))
        return buf.value.decode()

    def autotune(self, renders, max_depth, *, seed=0, reps=2, cache=None, count_work=False, graph=False):
        """Time a call shaped like trace_batch(renders, max_depth) under candidate launch settings,
        apply the fastest and return it (with "ms" and "from_cache").  cache: path of a results file
        read first and written after a search.  The search's samples are discarded: the render ids
        must be unused."""
        arr = self._batch_descs(renders, max_depth, seed, count_work, graph)
        t, ms, fc = Tuning(), C.c_double(0.0), C.c_int32(0)
        self._check(lib().sdd_autotune(self.h, len(renders), arr, int(reps),
                                       None if cache is None else str(cache).encode(), C.byref(t), C.byref(ms),
                                       C.byref(fc)))
        return dict(t.as_dict(), ms=ms.value, from_cache=bool(fc.value))

    def new_log(self, W, H, spp, max_depth):
        return self.torch.empty((W * H, spp, max_depth), dtype=self.torch.int32, device=self.device)

    def resolve_image(self, render_id=0, W=None, H=None, spectral=True, xyz=True):
        """FP64 [H*W, n_lambda] spectral mean and [H*W, 3] XYZ as device tensors."""
        if W is None or H is None:
            raise ValueError("resolve_image needs W and H")
        torch = self.torch
        s = torch.empty((H * W, self.n_lambda), dtype=torch.float64, device=self.device) if spectral else None
        x = torch.empty((H * W, 3), dtype=torch.float64, device=self.device) if xyz else None
        self._check(lib().sdd_resolve_image(self.h, int(render_id), s.data_ptr() if s is not None else None,
                                            x.data_ptr() if x is not None else None, 1))
        return s, x

    def reset_render(self, render_id=0):
        self._check(lib().sdd_reset_render(self.h, int(render_id)))

    def stats(self):
        s = Stats()
        self._check(lib().sdd_get_stats(self.h, C.byref(s)))
        return s.as_dict()

    def reset_stats(self):
        self._check(lib().sdd_reset_stats(self.h))

    def debug_philox(self, ctr, key):
        ctr = np.ascontiguousarray(ctr, np.uint32).reshape(-1, 4)
        key = np.ascontiguousarray(key, np.uint32).reshape(2)
        out = np.zeros_like(ctr)
        self._check(lib().sdd_debug_philox(self.h, len(ctr), _ptr(ctr), _ptr(key), _ptr(out)))
        return out

    def debug_pane(self, params):
        """params [n, 5] = (n, k, thickness m, wavelength nm, cos): returns (R, T) float32."""
        params = np.ascontiguousarray(params, np.float32).reshape(-1, 5)
        R = np.zeros(len(params), np.float32)
        T = np.zeros(len(params), np.float32)
        self._check(lib().sdd_debug_pane(self.h, len(params), _ptr(params), _ptr(R), _ptr(T)))
        return R, T

    def debug_glass(self, mat, lam_idx, cs):
        """Glass R, T of the loaded scene: material indices, wavelength indices and
        signed incidence cosines (> 0: the coated, normal-side face).  float32 arrays."""
        mat = np.ascontiguousarray(mat, np.int32).reshape(-1)
        lam_idx = np.ascontiguousarray(lam_idx, np.int32).reshape(-1)
        cs = np.ascontiguousarray(cs, np.float32).reshape(-1)
        if not (len(mat) == len(lam_idx) == len(cs)):
            raise ValueError("mat, lam_idx and cs must have the same length")
        R = np.zeros(len(cs), np.float32)
        T = np.zeros(len(cs), np.float32)
        self._check(lib().sdd_debug_glass(self.h, len(cs), _ptr(mat), _ptr(lam_idx), _ptr(cs), _ptr(R), _ptr(T)))
        return R, T

    def debug_trace_rays(self, o, d):
        o = np.ascontiguousarray(o, np.float32).reshape(-1, 3)
        d = np.ascontiguousarray(d, np.float32).reshape(-1, 3)
        t = np.zeros(len(o), np.float32)
        prim = np.zeros(len(o), np.int32)
        self._check(lib().sdd_debug_trace_rays(self.h, len(o), _ptr(o), _ptr(d), _ptr(t), _ptr(prim)))
        return t, prim


    # ---- learned radiance cache -------------------------------------------------
    def nrc_init(self, params, tables, aabb_lo, aabb_hi, lambda_range=(380.0, 780.0), lr=1e-2, betas=(0.9, 0.99),
                 eps=1e-8, train_paths=1 << 16, train_steps=4, train_batch=1 << 14, precision="bf16",
                 table_fp16=False):
        """Create the cache from a parameter dict (W [5][64][64], b [5][64], wo [64], bo) and hash
        tables [16][T][2] (T a power of two); train_* and precision apply to renders with nrc=True;
        table_fp16: BF16 queries gather from an FP16 copy of the tables."""
        T = int(np.asarray(tables).shape[1])
        log2 = T.bit_length() - 1
        if T != 1 << log2:
            raise ValueError("table size must be a power of two")
        flat = nrc_flatten(params, tables)
        self._nrc_T = T
        d = NrcDesc()
        d.table_log2 = log2
        d.aabb_lo[:] = [float(v) for v in aabb_lo]
        d.aabb_hi[:] = [float(v) for v in aabb_hi]
        d.lambda_lo, d.lambda_hi = float(lambda_range[0]), float(lambda_range[1])
        d.lr, d.beta1, d.beta2, d.eps = float(lr), float(betas[0]), float(betas[1]), float(eps)
        d.params = flat.ctypes.data
        d.train_paths, d.train_steps, d.train_batch = int(train_paths), int(train_steps), int(train_batch)
        d.precision = {"fp32": 0, "bf16": 1}[precision]
        d.table_fp16 = int(bool(table_fp16))
        self._check(lib().sdd_nrc_init(self.h, C.byref(d)))

    def _rows(self, *arrays):
        out = []
        for a in arrays:
            t = self.torch.as_tensor(a, dtype=self.torch.float32, device=self.device).contiguous()
            out.append(t)
        return out

    def nrc_infer(self, x, w, lam, precision="fp32"):
        """Network outputs for rows (x [n,3], w [n,3], lambda [n]); a float32 device tensor."""
        x, w, lam = self._rows(x, w, lam)
        n = lam.numel()
        y = self.torch.empty(n, dtype=self.torch.float32, device=self.device)
        prec = {"fp32": 0, "bf16": 1}[precision]
        self._check(lib().sdd_nrc_infer(self.h, n, x.data_ptr(), w.data_ptr(), lam.data_ptr(), y.data_ptr(), prec))
        return y

    def nrc_train_step(self, x, w, lam, target, apply=True):
        """One gradient (and, if apply, Adam) step; returns the batch loss before the update."""
        x, w, lam, target = self._rows(x, w, lam, target)
        loss = C.c_float()
        self._check(lib().sdd_nrc_train_step(self.h, lam.numel(), x.data_ptr(), w.data_ptr(), lam.data_ptr(),
                                             target.data_ptr(), int(bool(apply)), C.byref(loss)))
        return float(loss.value)

    def nrc_query(self, x, nrm, precision="fp32"):
        """Cache values of points (x [n,3], normal [n,3]) at every scene wavelength: [n, nlp] device tensor."""
        torch = self.torch
        x = torch.as_tensor(x, dtype=torch.float32, device=self.device).reshape(-1, 3)
        nrm = torch.as_tensor(nrm, dtype=torch.float32, device=self.device).reshape(-1, 3)
        n = x.shape[0]
        x4 = torch.zeros((n, 4), dtype=torch.float32, device=self.device)
        n4 = torch.zeros((n, 4), dtype=torch.float32, device=self.device)
        x4[:, :3] = x
        n4[:, :3] = nrm
        nlp = (self.n_lambda + 3) // 4 * 4
        out = torch.zeros((n, nlp), dtype=torch.float32, device=self.device)
        self._check(lib().sdd_nrc_query(self.h, n, x4.data_ptr(), n4.data_ptr(), out.data_ptr(),
                                        {"fp32": 0, "bf16": 1}[precision]))
        return out

    def nrc_query_noalloc(self, x, nrm):
        """sdd_nrc_query_noalloc: the BF16 query with its scratch in the library's static array (no allocation
        inside the library; this wrapper allocates the operand and output tensors)."""
        torch = self.torch
        x = torch.as_tensor(x, dtype=torch.float32, device=self.device).reshape(-1, 3)
        nrm = torch.as_tensor(nrm, dtype=torch.float32, device=self.device).reshape(-1, 3)
        n = x.shape[0]
        x4 = torch.zeros((n, 4), dtype=torch.float32, device=self.device)
        n4 = torch.zeros((n, 4), dtype=torch.float32, device=self.device)
        x4[:, :3] = x
        n4[:, :3] = nrm
        nlp = (self.n_lambda + 3) // 4 * 4
        out = torch.zeros((n, nlp), dtype=torch.float32, device=self.device)
        self._check(lib().sdd_nrc_query_noalloc(self.h, n, x4.data_ptr(), n4.data_ptr(), out.data_ptr()))
        return out

    def nrc_last_rows(self, max_rows=None):
        """(rows [n][8] = x, y, z, lambda, n_x, n_y, n_z, target; Adam steps; last loss) of the last cache render."""
        n, steps, loss = C.c_int32(), C.c_int32(), C.c_float()
        self._check(lib().sdd_nrc_last_rows(self.h, 0, None, C.byref(n), C.byref(steps), C.byref(loss)))
        m = n.value if max_rows is None else min(n.value, int(max_rows))
        rows = np.zeros((m, 8), np.float32)
        if m:
            self._check(lib().sdd_nrc_last_rows(self.h, m, _ptr(rows), None, None, None))
        return rows, steps.value, loss.value

    def nrc_get(self, which="params"):
        """(dict, tables) of the parameters, last gradient, or Adam moments ('m', 'v')."""
        n = lib().sdd_nrc_param_count(self._nrc_T.bit_length() - 1)
        out = np.empty(n, np.float32)
        self._check(lib().sdd_nrc_get_params(self.h, {"params": 0, "grad": 1, "m": 2, "v": 3}[which], _ptr(out)))
        return nrc_unflatten(out, self._nrc_T)


def nrc_flatten(params, tables):
    """Parameter dict + tables -> the library's flat float32 layout."""
    tables = np.ascontiguousarray(tables, np.float32)
    if tables.ndim != 3 or tables.shape[0] != NRC_LEVELS or tables.shape[2] != NRC_FEAT:
        raise ValueError("tables must be [16][T][2]")
    parts = [tables.reshape(-1),
             np.ascontiguousarray(params["W"], np.float32).reshape(-1),
             np.ascontiguousarray(params["b"], np.float32).reshape(-1),
             np.ascontiguousarray(params["wo"], np.float32).reshape(-1),
             np.asarray([params["bo"]], np.float32)]
    flat = np.ascontiguousarray(np.concatenate(parts))
    if flat.size != NRC_LEVELS * tables.shape[1] * NRC_FEAT + NRC_LAYERS * NRC_HID * (NRC_HID + 1) + NRC_HID + 1:
        raise ValueError("parameter shapes do not match the network")
    return flat


def nrc_unflatten(flat, T):
    nt = NRC_LEVELS * T * NRC_FEAT
    o = nt
    W = flat[o:o + NRC_LAYERS * NRC_HID * NRC_HID].reshape(NRC_LAYERS, NRC_HID, NRC_HID)
    o += NRC_LAYERS * NRC_HID * NRC_HID
    b = flat[o:o + NRC_LAYERS * NRC_HID].reshape(NRC_LAYERS, NRC_HID)
    o += NRC_LAYERS * NRC_HID
    wo = flat[o:o + NRC_HID]
    bo = float(flat[o + NRC_HID])
    return dict(W=list(W), b=list(b), wo=wo, bo=bo), flat[:nt].reshape(NRC_LEVELS, T, NRC_FEAT)


def render(scene, W, H, spp, max_depth, grid=(1, 1, 1), *, camera=None, seed=0, logs=False, tracer=None):
    """Convenience: one render; returns numpy spectral [H*W, nl], xyz, and optional logs."""
    t = tracer or Tracer()
    t.load_scene(scene)
    t.build_bvh(*grid)
    cam = camera or scene["camera"]
    hl = sl = None
    if logs:
        hl = t.new_log(W, H, spp, max_depth)
        sl = t.new_log(W, H, spp, max_depth)
    t.trace_spectral(cam, W, H, spp, max_depth, seed=seed, hit_log=hl, shadow_log=sl)
    s, x = t.resolve_image(0, W, H)
    out = dict(spectral=s.cpu().numpy(), xyz=x.cpu().numpy())
    if logs:
        out["hit_log"] = hl.cpu().numpy()
        out["shadow_log"] = sl.cpu().numpy()
    out["stats"] = t.stats()
    return out
