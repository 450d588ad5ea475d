"""ctypes front end of the FP64 CPU oracle -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  The product library never calls it:
it exists to check the HIP path against (plain FP64 definitions, see ``oracle.h``).
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

from . import build as _build

_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_build.LIB):
            _build.build()
        _lib = C.CDLL(_build.LIB)
        _declare(_lib)
    return _lib


class Scene(C.Structure):
    _fields_ = [
        ("n_verts", C.c_int), ("verts", C.c_void_p),
        ("n_tris", C.c_int), ("tris", C.c_void_p), ("tri_mat", C.c_void_p),
        ("n_lambda", C.c_int), ("lambda_nm", C.c_void_p), ("lambda_w", C.c_void_p), ("cmf", C.c_void_p),
        ("n_mats", C.c_int), ("mat_type", C.c_void_p), ("mat_rho", C.c_void_p), ("mat_n", C.c_void_p),
        ("mat_k", C.c_void_p), ("mat_thick", C.c_void_p), ("mat_le", C.c_void_p),
        ("light_type", C.c_int), ("light_p0", C.c_void_p), ("light_e1", C.c_void_p),
        ("light_e2", C.c_void_p), ("light_mat", C.c_int),
        ("max_layers", C.c_int), ("mat_n_layers", C.c_void_p), ("mat_layer_d", C.c_void_p),
        ("mat_layer_n", C.c_void_p), ("mat_layer_k", C.c_void_p),
    ]


class Args(C.Structure):
    _fields_ = [
        ("eye", C.c_double * 3), ("target", C.c_double * 3), ("fov_deg", C.c_double),
        ("ortho", C.c_int), ("ortho_half_h", C.c_double),
        ("W", C.c_int), ("H", C.c_int), ("spp", C.c_int), ("sample_offset", C.c_int), ("max_depth", C.c_int),
        ("seed", C.c_uint32), ("render_id", C.c_uint32), ("use_bvh", C.c_int), ("n_threads", C.c_int),
        ("n_pix", C.c_int), ("pix", C.c_void_p), ("window", C.c_int),
        ("nrc", C.c_int), ("nrc_stride", C.c_uint32), ("nrc_c", C.c_double * 7), ("nrc_lo", C.c_double * 3),
        ("nrc_hi", C.c_double * 3),
    ]


class Out(C.Structure):
    _fields_ = [
        ("spectral", C.c_void_p), ("xyz", C.c_void_p), ("hit_log", C.c_void_p),
        ("shadow_log", C.c_void_p), ("path_L", C.c_void_p), ("first_hit", C.c_void_p), ("nrc_rows", C.c_void_p),
        ("n_ext_rays", C.c_int64), ("n_shadow_rays", C.c_int64),
    ]


def _declare(L):
    L.ora_build.restype = C.c_void_p
    L.ora_build.argtypes = [C.POINTER(Scene)]
    L.ora_free.argtypes = [C.c_void_p]
    L.ora_accel_nodes.argtypes = [C.c_void_p]
    L.ora_render.argtypes = [C.POINTER(Scene), C.c_void_p, C.POINTER(Args), C.POINTER(Out)]
    L.ora_trace_rays.argtypes = [C.POINTER(Scene), C.c_void_p, C.c_int, C.c_void_p, C.c_void_p,
                                 C.c_void_p, C.c_void_p, C.c_void_p]
    L.ora_shadow_rays.argtypes = [C.POINTER(Scene), C.c_void_p, C.c_int, C.c_void_p, C.c_void_p,
                                  C.c_void_p, C.c_void_p, C.c_void_p]
    L.ora_probe_paths.argtypes = [C.POINTER(Scene), C.c_void_p, C.POINTER(Args), C.c_int, C.c_void_p, C.c_void_p,
                                  C.c_void_p]
    L.ora_philox4x32_10.argtypes = [C.c_void_p, C.c_void_p, C.c_void_p]
    L.ora_u01.restype = C.c_double
    L.ora_u01.argtypes = [C.c_uint32]
    dp = C.POINTER(C.c_double)
    L.ora_fresnel_sp.argtypes = [C.c_double, C.c_double, C.c_double, dp, dp]
    L.ora_slab_sp.argtypes = [C.c_double] * 5 + [dp] * 4
    L.ora_slab.argtypes = [C.c_double] * 5 + [dp] * 2
    L.ora_tmm_sp.argtypes = [C.c_int, C.c_void_p, C.c_void_p, C.c_void_p] + [C.c_double] * 6 + [dp] * 4
    L.ora_coated_pane.argtypes = ([C.c_double] * 3 + [C.c_int, C.c_void_p, C.c_void_p, C.c_void_p]
                                  + [C.c_double] * 2 + [C.c_int] + [dp] * 2)
    L.ora_cosine_hemisphere.argtypes = [C.c_void_p, C.c_double, C.c_double, C.c_void_p]
    L.ora_camera_ray.argtypes = [C.POINTER(Args), C.c_double, C.c_double, C.c_void_p, C.c_void_p]


def _ptr(a):
    return a.ctypes.data_as(C.c_void_p) if a is not None else None


class OracleScene:
    """Holds contiguous copies of a scene's arrays and the C view onto them."""

    def __init__(self, scene):
        self.keep = {}

        def arr(key, dt):
            a = np.ascontiguousarray(scene[key], dtype=dt)
            self.keep[key] = a
            return a

        verts = arr("verts", np.float32)
        tris = arr("tris", np.int32)
        arr("tri_mat", np.int32)
        lam = arr("lambda_nm", np.float32)
        arr("lambda_w", np.float64)
        arr("cmf", np.float64)
        mt = arr("mat_type", np.int32)
        for k in ("mat_rho", "mat_n", "mat_k", "mat_le"):
            arr(k, np.float32)
        arr("mat_thick", np.float32)
        for k in ("light_p0", "light_e1", "light_e2"):
            arr(k, np.float32)
        k = self.keep
        self.n_lambda = len(lam)
        self.c = Scene(len(verts), _ptr(verts), len(tris), _ptr(tris), _ptr(k["tri_mat"]),
                       len(lam), _ptr(lam), _ptr(k["lambda_w"]), _ptr(k["cmf"]),
                       len(mt), _ptr(mt), _ptr(k["mat_rho"]), _ptr(k["mat_n"]), _ptr(k["mat_k"]),
                       _ptr(k["mat_thick"]), _ptr(k["mat_le"]),
                       int(scene["light_type"]), _ptr(k["light_p0"]), _ptr(k["light_e1"]),
                       _ptr(k["light_e2"]), int(scene["light_mat"]))
        if "mat_n_layers" in scene:
            nlay = arr("mat_n_layers", np.int32)
            ld = arr("mat_layer_d", np.float32)
            arr("mat_layer_n", np.float32)
            arr("mat_layer_k", np.float32)
            self.c.max_layers = int(ld.shape[1]) if ld.ndim == 2 else 0
            self.c.mat_n_layers = _ptr(nlay)
            self.c.mat_layer_d = _ptr(ld)
            self.c.mat_layer_n = _ptr(k["mat_layer_n"])
            self.c.mat_layer_k = _ptr(k["mat_layer_k"])
        self._accel = None

    @property
    def accel(self):
        if self._accel is None:
            self._accel = lib().ora_build(C.byref(self.c))
        return self._accel

    def __del__(self):
        if self._accel is not None and _lib is not None:
            _lib.ora_free(self._accel)
            self._accel = None


def make_args(camera, W, H, spp, max_depth, seed=0, render_id=0, sample_offset=0, use_bvh=True,
              n_threads=0, pix=None):
    a = Args()
    a.eye[:] = [float(x) for x in camera["eye"]]
    a.target[:] = [float(x) for x in camera["target"]]
    a.fov_deg = float(camera["fov_deg"])
    a.ortho = int(bool(camera.get("ortho", False)))
    a.ortho_half_h = float(camera.get("ortho_half_h", 1.0))
    a.W, a.H, a.spp, a.max_depth = int(W), int(H), int(spp), int(max_depth)
    a.sample_offset = int(sample_offset)
    a.seed, a.render_id = int(seed), int(render_id)
    a.use_bvh = int(bool(use_bvh))
    a.n_threads = int(n_threads)
    a.n_pix, a.pix = 0, None
    return a


def render(scene, W, H, spp, max_depth, *, camera=None, seed=0, render_id=0, sample_offset=0,
           use_bvh=True, n_threads=0, pix=None, logs=False, path_L=False, first_hit=False,
           oscene=None, nrc=None, crop=None):
    """Render with the oracle.  Returns a dict of numpy arrays.

    ``pix``: optional list of pixel indices p = py*W + px (outputs follow it).
    ``crop``: optional window (x0, y0, w, h) of the frame: its pixels in row-major
    order, with the render's paths numbered over the window (as a window
    render numbers them); excludes ``pix``.
    ``nrc``: optional dict(stride, c (7 coefficients), lo, hi) selecting the
    radiance-cache estimator with the closed-form cache c0 + c[1:4].xn + c[4:7].n;
    the result then also holds ``nrc_rows`` [n_out][spp][D-1][9].
    """
    osc = oscene or OracleScene(scene)
    cam = camera or scene["camera"]
    a = make_args(cam, W, H, spp, max_depth, seed, render_id, sample_offset, use_bvh, n_threads)
    pix_arr = None
    if crop is not None:
        x0, y0, cw, ch = (int(v) for v in crop)
        ys, xs = np.meshgrid(np.arange(y0, y0 + ch), np.arange(x0, x0 + cw), indexing="ij")
        pix = (ys * W + xs).ravel()
        a.window = 1
    if pix is not None:
        pix_arr = np.ascontiguousarray(pix, dtype=np.int32)
        a.n_pix, a.pix = len(pix_arr), _ptr(pix_arr)
    n_out = len(pix_arr) if pix_arr is not None else W * H
    nl = osc.n_lambda
    res = dict(spectral=np.zeros((n_out, nl)), xyz=np.zeros((n_out, 3)))
    if logs:
        res["hit_log"] = np.zeros((n_out, spp, max_depth), np.int32)
        res["shadow_log"] = np.zeros((n_out, spp, max_depth), np.int32)
    if path_L:
        res["path_L"] = np.zeros((n_out, spp, nl))
    if first_hit:
        res["first_hit"] = np.zeros((n_out, spp, 3))
    if nrc is not None:
        a.nrc, a.nrc_stride = 1, int(nrc["stride"])
        a.nrc_c[:] = [float(v) for v in nrc["c"]]
        a.nrc_lo[:] = [float(v) for v in nrc["lo"]]
        a.nrc_hi[:] = [float(v) for v in nrc["hi"]]
        res["nrc_rows"] = np.zeros((n_out, spp, max(1, max_depth - 1), 9))
    o = Out(_ptr(res["spectral"]), _ptr(res["xyz"]), _ptr(res.get("hit_log")), _ptr(res.get("shadow_log")),
            _ptr(res.get("path_L")), _ptr(res.get("first_hit")), _ptr(res.get("nrc_rows")), 0, 0)
    acc = osc.accel if use_bvh else None
    rc = lib().ora_render(C.byref(osc.c), acc, C.byref(a), C.byref(o))
    if rc != 0:
        raise RuntimeError(f"ora_render failed ({rc})")
    res["n_ext_rays"] = int(o.n_ext_rays)
    res["n_shadow_rays"] = int(o.n_shadow_rays)
    return res


PROBE_STRIDE = 18


def probe_paths(scene, W, H, max_depth, pix, samples, *, camera=None, seed=0, render_id=0, use_bvh=True,
                oscene=None):
    """Replay path samples (pix[i], samples[i]) and return [n, D, 18] per-depth
    state (see ora_probe_paths in oracle.h): ray, glass draw and P_R, light sample."""
    osc = oscene or OracleScene(scene)
    cam = camera or scene["camera"]
    a = make_args(cam, W, H, 1, max_depth, seed, render_id, 0, use_bvh)
    pix = np.ascontiguousarray(pix, np.int32)
    samples = np.ascontiguousarray(samples, np.int32)
    out = np.zeros((len(pix), max_depth, PROBE_STRIDE))
    rc = lib().ora_probe_paths(C.byref(osc.c), osc.accel if use_bvh else None, C.byref(a), len(pix), _ptr(pix),
                               _ptr(samples), _ptr(out))
    if rc != 0:
        raise RuntimeError("ora_probe_paths failed")
    return out


def trace_rays(scene, o, d, exclude=None, use_bvh=True, oscene=None):
    osc = oscene or OracleScene(scene)
    o = np.ascontiguousarray(o, np.float64).reshape(-1, 3)
    d = np.ascontiguousarray(d, np.float64).reshape(-1, 3)
    n = len(o)
    ex = None if exclude is None else np.ascontiguousarray(exclude, np.int32)
    t = np.zeros(n)
    prim = np.zeros(n, np.int32)
    lib().ora_trace_rays(C.byref(osc.c), osc.accel if use_bvh else None, n, _ptr(o), _ptr(d), _ptr(ex),
                         _ptr(t), _ptr(prim))
    return t, prim


def shadow_rays(scene, o, d, r, exclude=None, use_bvh=True, oscene=None):
    osc = oscene or OracleScene(scene)
    o = np.ascontiguousarray(o, np.float64).reshape(-1, 3)
    d = np.ascontiguousarray(d, np.float64).reshape(-1, 3)
    r = np.ascontiguousarray(r, np.float64)
    n = len(o)
    ex = None if exclude is None else np.ascontiguousarray(exclude, np.int32)
    out = np.zeros((n, osc.n_lambda))
    lib().ora_shadow_rays(C.byref(osc.c), osc.accel if use_bvh else None, n, _ptr(o), _ptr(d), _ptr(r),
                          _ptr(ex), _ptr(out))
    return out


def philox(ctr, key):
    c = np.ascontiguousarray(ctr, np.uint32)
    k = np.ascontiguousarray(key, np.uint32)
    out = np.zeros(4, np.uint32)
    lib().ora_philox4x32_10(_ptr(c), _ptr(k), _ptr(out))
    return out


def u01(x):
    return lib().ora_u01(int(x))


def fresnel_sp(n, k, c):
    rs, rp = C.c_double(), C.c_double()
    lib().ora_fresnel_sp(n, k, c, C.byref(rs), C.byref(rp))
    return rs.value, rp.value


def slab_sp(n, k, thick_m, lam_nm, c):
    v = [C.c_double() for _ in range(4)]
    lib().ora_slab_sp(n, k, thick_m, lam_nm, c, *[C.byref(x) for x in v])
    return tuple(x.value for x in v)


def slab(n, k, thick_m, lam_nm, c):
    R, T = C.c_double(), C.c_double()
    lib().ora_slab(n, k, thick_m, lam_nm, c, C.byref(R), C.byref(T))
    return R.value, T.value


def tmm_sp(d_m, n, k, n_in, k_in, n_out, k_out, lam_nm, beta):
    """Coherent stack between two media: (Rs, Rp, Ts, Tp)."""
    d = np.ascontiguousarray(d_m, np.float64)
    nn = np.ascontiguousarray(n, np.float64)
    kk = np.ascontiguousarray(k, np.float64)
    v = [C.c_double() for _ in range(4)]
    lib().ora_tmm_sp(len(d), _ptr(d), _ptr(nn), _ptr(kk), n_in, k_in, n_out, k_out, lam_nm, beta,
                     *[C.byref(x) for x in v])
    return tuple(x.value for x in v)


def coated_pane(n_s, k_s, thick_m, d_m, n, k, lam_nm, c, coated_side=True):
    """Coated incoherent pane: (R, T), polarisation-averaged."""
    d = np.ascontiguousarray(d_m, np.float64)
    nn = np.ascontiguousarray(n, np.float64)
    kk = np.ascontiguousarray(k, np.float64)
    R, T = C.c_double(), C.c_double()
    lib().ora_coated_pane(n_s, k_s, thick_m, len(d), _ptr(d), _ptr(nn), _ptr(kk), lam_nm, c, int(bool(coated_side)),
                          C.byref(R), C.byref(T))
    return R.value, T.value


def cosine_hemisphere(n, u0, u1):
    nn = np.ascontiguousarray(n, np.float64)
    out = np.zeros(3)
    lib().ora_cosine_hemisphere(_ptr(nn), u0, u1, _ptr(out))
    return out


def camera_ray(camera, W, H, x, y):
    a = make_args(camera, W, H, 1, 1)
    o, d = np.zeros(3), np.zeros(3)
    lib().ora_camera_ray(C.byref(a), x, y, _ptr(o), _ptr(d))
    return o, d
