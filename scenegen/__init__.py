"""Seeded synthetic scene generator: the inputs shared by the oracle and the GPU path.

This module produces *inputs only*: geometry, per-wavelength optical tables,
the light and the camera.  It holds none of the rendering method's arithmetic
(no intersection, no Fresnel, no sampling, no transport).  Both the FP64 CPU
oracle (``oracle/``) and the HIP library (``paper_1912_06474_amd``) read the
same arrays produced here.

The paper's hotel-room model, its measured spectra and its BK7 data are not
available, so rooms are synthesised with the shape of the paper's workload
(Sec. 6: an interior with glass windows lit by daylight through the panes):

* an axis-aligned room 4 x 3 x 2.5 m (z up) whose rectangles are tessellated
  into ceil(Lu) x ceil(Lv) equal quads (2 triangles each);
* window panes cut into the y = 3 wall, each a zero-thickness double-sided
  quad whose material carries a slab thickness (4 mm) and a complex index
  n(lambda) + i k(lambda) (Eq. 1) -- here a Cauchy law stands in for BK7;
* a one-sided parallelogram sky emitter outside the window facing -y, with a
  daylight-shaped spectrum (Planck at 6504 K, normalised at 560 nm);
* diffuse furniture: seeded axis-aligned boxes (and, for the room-scale case,
  capped z-axis cylinders) with reflectances that are seeded sums of three
  Gaussians clipped to [0.05, 0.9].

Randomness uses numpy's PCG64 keyed by the scene seed.  Every table is stored
as float32 already sampled on the wavelength grid (weights and CMFs as
float64), so both consumers read identical numbers.

Scene dictionary keys (all numpy arrays unless noted)::

    verts     f32 [V,3]      tris      i32 [T,3]     tri_mat  i32 [T]
    lambda_nm f32 [nl]       lambda_w  f64 [nl]      cmf      f64 [nl,3]
    mat_type  i32 [M]  (0 diffuse, 1 glass slab, 2 emitter)
    mat_rho   f32 [M,nl]     mat_n f32 [M,nl]        mat_k    f32 [M,nl]
    mat_thick f32 [M] (m)    mat_le f32 [M,nl]
    light_type int (0 none, 1 parallelogram, 2 point)
    light_p0, light_e1, light_e2  f32 [3]           light_mat int
    camera    dict(eye, target, fov_deg, ortho, ortho_half_h)
    name, seed, cmf_provenance (str / int)
"""
from __future__ import annotations

import math

import numpy as np

DIFFUSE, GLASS, EMITTER = 0, 1, 2
LIGHT_NONE, LIGHT_PARALLELOGRAM, LIGHT_POINT = 0, 1, 2

ROOM = (4.0, 3.0, 2.5)
EYE = (2.0, 0.5, 1.2)
TARGET = (2.0, 3.0, 1.2)
FOV_DEG = 70.0
# Outside sky emitter: plane y = 4, x in [-1, 5], z in [-0.5, 3], facing -y.
LIGHT_P0 = (-1.0, 4.0, -0.5)
LIGHT_E1 = (6.0, 0.0, 0.0)
LIGHT_E2 = (0.0, 0.0, 3.5)
L0_SKY = 10.0
T_DAYLIGHT = 6504.0


# ----------------------------------------------------------------------------
# wavelength grids and spectra (inputs)
# ----------------------------------------------------------------------------

def lambda_grid(n: int):
    """Wavelength samples (nm) and integration weights (nm).

    * n == 16: bin centres 392.5 .. 767.5 nm, 25 nm bins, weight 25 each.
    * otherwise: n points spanning 380 .. 780 nm inclusive with trapezoid
      weights (half a step at both ends).
    """
    if n == 16:
        lam = 392.5 + 25.0 * np.arange(16)
        w = np.full(16, 25.0)
    else:
        if n < 2:
            raise ValueError("need at least 2 wavelengths")
        lam = np.linspace(380.0, 780.0, n)
        step = 400.0 / (n - 1)
        w = np.full(n, step)
        w[0] = w[-1] = step / 2
    return lam.astype(np.float32), w.astype(np.float64)


def _lobe(lam, mu, s_lo, s_hi):
    s = np.where(lam < mu, s_lo, s_hi)
    return np.exp(-0.5 * ((lam - mu) / s) ** 2)


def cmf_proxy(lam_nm):
    """Approximate CIE-1931-like colour matching functions.

    The official CIE tables are not available to this project, so the
    per-wavelength weights used for the spectral -> XYZ reduction are a
    multi-lobe piecewise-Gaussian fit in the form published by Wyman, Sloan
    and Shirley (JCGT 2013).  It is labelled a *proxy*: parity between the
    GPU path and the oracle does not depend on these values (both read this
    same table), but absolute colorimetry does.
    """
    lam = np.asarray(lam_nm, dtype=np.float64)
    x = (1.056 * _lobe(lam, 599.8, 37.9, 31.0) + 0.362 * _lobe(lam, 442.0, 16.0, 26.7)
         - 0.065 * _lobe(lam, 501.1, 20.4, 26.2))
    y = 0.821 * _lobe(lam, 568.8, 46.9, 40.5) + 0.286 * _lobe(lam, 530.9, 16.3, 31.1)
    z = 1.217 * _lobe(lam, 437.0, 11.8, 36.0) + 0.681 * _lobe(lam, 459.0, 26.0, 13.8)
    return np.stack([x, y, z], axis=1)


def planck_shape(lam_nm, temp=T_DAYLIGHT, norm_nm=560.0, scale=L0_SKY):
    """Daylight-shaped emission: Planck B(lambda, T) / B(560 nm, T) * scale."""
    h, c, kb = 6.62607015e-34, 2.99792458e8, 1.380649e-23

    def b(l_nm):
        l = np.asarray(l_nm, dtype=np.float64) * 1e-9
        return 1.0 / (l ** 5 * (np.exp(h * c / (l * kb * temp)) - 1.0))

    return (scale * b(lam_nm) / b(norm_nm)).astype(np.float32)


def cauchy_n(lam_nm, a=1.5, b_um2=0.0042):
    """Cauchy dispersion n(lambda) = A + B / lambda^2 (lambda in micrometres)."""
    l_um = np.asarray(lam_nm, dtype=np.float64) / 1000.0
    return (a + b_um2 / l_um ** 2).astype(np.float32)


def gaussian_reflectance(rng, lam_nm):
    """Seeded sum of 3 Gaussians over [380, 780] nm, clipped to [0.05, 0.9]."""
    lam = np.asarray(lam_nm, dtype=np.float64)
    r = np.zeros_like(lam)
    for _ in range(3):
        a = rng.uniform(0.1, 0.6)
        mu = rng.uniform(380.0, 780.0)
        sg = rng.uniform(20.0, 80.0)
        r += a * np.exp(-0.5 * ((lam - mu) / sg) ** 2)
    return np.clip(r, 0.05, 0.9).astype(np.float32)


# ----------------------------------------------------------------------------
# geometry builders
# ----------------------------------------------------------------------------

class _Mesh:
    def __init__(self):
        self.v: list[tuple[float, float, float]] = []
        self.t: list[tuple[int, int, int]] = []
        self.m: list[int] = []

    def vert(self, p):
        self.v.append((float(p[0]), float(p[1]), float(p[2])))
        return len(self.v) - 1

    def tri(self, a, b, c, mat):
        self.t.append((a, b, c))
        self.m.append(mat)

    def ntri(self):
        return len(self.t)


def _rect(mesh, origin, du, dv, nu, nv, mat, skip=()):
    """Tessellate origin + a*du + b*dv, (a, b) in [0,1]^2, into nu x nv quads.

    Quad (i, j) -> triangles A = (P00, P10, P11) and B = (P00, P11, P01),
    emitted in row-major order (j outer, i inner), so the prim id of quad
    (i, j) is base + 2*(j*nu + i) (+1 for B) when nothing is skipped.
    """
    o = np.asarray(origin, dtype=np.float64)
    du = np.asarray(du, dtype=np.float64)
    dv = np.asarray(dv, dtype=np.float64)
    idx = np.empty((nv + 1, nu + 1), dtype=np.int64)
    for j in range(nv + 1):
        for i in range(nu + 1):
            idx[j, i] = mesh.vert(o + du * (i / nu) + dv * (j / nv))
    for j in range(nv):
        for i in range(nu):
            if (i, j) in skip:
                continue
            p00, p10, p11, p01 = idx[j, i], idx[j, i + 1], idx[j + 1, i + 1], idx[j + 1, i]
            mesh.tri(p00, p10, p11, mat)
            mesh.tri(p00, p11, p01, mat)
    return idx


def _box(mesh, lo, hi, s, mat):
    """Axis-aligned box, every face split into s x s quads (12 s^2 triangles)."""
    lo = np.asarray(lo, dtype=np.float64)
    hi = np.asarray(hi, dtype=np.float64)
    ext = hi - lo
    ex, ey, ez = np.array([ext[0], 0, 0]), np.array([0, ext[1], 0]), np.array([0, 0, ext[2]])
    _rect(mesh, lo, ex, ey, s, s, mat)                      # z = lo
    _rect(mesh, lo + ez, ex, ey, s, s, mat)                 # z = hi
    _rect(mesh, lo, ex, ez, s, s, mat)                      # y = lo
    _rect(mesh, lo + ey, ex, ez, s, s, mat)                 # y = hi
    _rect(mesh, lo, ey, ez, s, s, mat)                      # x = lo
    _rect(mesh, lo + ex, ey, ez, s, s, mat)                 # x = hi


def _cylinder(mesh, centre, radius, half_h, nseg, nstack, mat):
    """Capped z-axis cylinder: 2*nseg*nstack side + 2*nseg cap triangles."""
    cx, cy, cz = centre
    rings = []
    for j in range(nstack + 1):
        z = cz - half_h + 2.0 * half_h * j / nstack
        ring = []
        for i in range(nseg):
            a = 2.0 * math.pi * i / nseg
            ring.append(mesh.vert((cx + radius * math.cos(a), cy + radius * math.sin(a), z)))
        rings.append(ring)
    for j in range(nstack):
        for i in range(nseg):
            i1 = (i + 1) % nseg
            a, b, c, d = rings[j][i], rings[j][i1], rings[j + 1][i1], rings[j + 1][i]
            mesh.tri(a, b, c, mat)
            mesh.tri(a, c, d, mat)
    bot = mesh.vert((cx, cy, cz - half_h))
    top = mesh.vert((cx, cy, cz + half_h))
    for i in range(nseg):
        i1 = (i + 1) % nseg
        mesh.tri(bot, rings[0][i1], rings[0][i], mat)
        mesh.tri(top, rings[-1][i], rings[-1][i1], mat)


def _room_shell(mesh, mats_for_rect, window_cells=(), pane_mat=None):
    """Six tessellated rectangles of the 4 x 3 x 2.5 m room.

    ``window_cells`` lists (ix, iz) quads of the y = 3 wall (4 x 3 quads)
    that are removed; each contiguous horizontal run of removed quads in a row
    is closed by one 2-triangle pane made of ``pane_mat`` on the same corner
    vertices.
    """
    lx, ly, lz = ROOM
    nx, ny, nz = math.ceil(lx), math.ceil(ly), math.ceil(lz)
    _rect(mesh, (0, 0, 0), (lx, 0, 0), (0, ly, 0), nx, ny, mats_for_rect[0])         # floor
    _rect(mesh, (0, 0, lz), (lx, 0, 0), (0, ly, 0), nx, ny, mats_for_rect[1])        # ceiling
    _rect(mesh, (0, 0, 0), (lx, 0, 0), (0, 0, lz), nx, nz, mats_for_rect[2])         # wall y = 0
    skip = set(window_cells)
    idx = _rect(mesh, (0, ly, 0), (lx, 0, 0), (0, 0, lz), nx, nz, mats_for_rect[3],
                skip=skip)                                                           # wall y = 3
    _rect(mesh, (0, 0, 0), (0, ly, 0), (0, 0, lz), ny, nz, mats_for_rect[4])         # wall x = 0
    _rect(mesh, (lx, 0, 0), (0, ly, 0), (0, 0, lz), ny, nz, mats_for_rect[5])        # wall x = 4
    # panes: group removed cells row by row into horizontal runs
    rows: dict[int, list[int]] = {}
    for (i, j) in sorted(skip):
        rows.setdefault(j, []).append(i)
    for j, cols in sorted(rows.items()):
        cols.sort()
        runs, start, prev = [], cols[0], cols[0]
        for c in cols[1:]:
            if c != prev + 1:
                runs.append((start, prev))
                start = c
            prev = c
        runs.append((start, prev))
        for (i0, i1) in runs:
            p00, p10 = idx[j, i0], idx[j, i1 + 1]
            p11, p01 = idx[j + 1, i1 + 1], idx[j + 1, i0]
            mesh.tri(p00, p10, p11, pane_mat)
            mesh.tri(p00, p11, p01, pane_mat)


def _add_sky_light(mesh, mat):
    p0 = np.asarray(LIGHT_P0)
    e1 = np.asarray(LIGHT_E1)
    e2 = np.asarray(LIGHT_E2)
    a = mesh.vert(p0)
    b = mesh.vert(p0 + e1)
    c = mesh.vert(p0 + e1 + e2)
    d = mesh.vert(p0 + e2)
    # wound so that the geometric normal (v1-v0) x (v2-v0) equals e1 x e2
    mesh.tri(a, b, c, mat)
    mesh.tri(a, c, d, mat)


def _box_clear_of_camera(lo, hi, eye, margin=0.1):
    q = np.clip(eye, lo, hi)
    return float(np.linalg.norm(np.asarray(eye) - q)) >= margin


class _Materials:
    def __init__(self, nl):
        self.nl = nl
        self.type: list[int] = []
        self.rho: list[np.ndarray] = []
        self.n: list[np.ndarray] = []
        self.k: list[np.ndarray] = []
        self.thick: list[float] = []
        self.le: list[np.ndarray] = []
        self.layers: list[list] = []

    def add(self, typ, rho=None, n=None, k=None, thick=0.0, le=None, layers=None):
        z = np.zeros(self.nl, dtype=np.float32)
        self.type.append(typ)
        self.rho.append(z if rho is None else np.asarray(rho, dtype=np.float32))
        self.n.append(np.ones(self.nl, dtype=np.float32) if n is None else np.asarray(n, dtype=np.float32))
        self.k.append(z if k is None else np.asarray(k, dtype=np.float32))
        self.thick.append(float(thick))
        self.le.append(z if le is None else np.asarray(le, dtype=np.float32))
        self.layers.append(list(layers or []))
        return len(self.type) - 1


def _finish(mesh, mats, lam, w, *, light_type, light_mat, name, seed,
            light_p0=LIGHT_P0, light_e1=LIGHT_E1, light_e2=LIGHT_E2, camera=None):
    scene = dict(
        verts=np.asarray(mesh.v, dtype=np.float32).reshape(-1, 3),
        tris=np.asarray(mesh.t, dtype=np.int32).reshape(-1, 3),
        tri_mat=np.asarray(mesh.m, dtype=np.int32),
        lambda_nm=lam,
        lambda_w=w,
        cmf=cmf_proxy(lam),
        mat_type=np.asarray(mats.type, dtype=np.int32),
        mat_rho=np.stack(mats.rho).astype(np.float32),
        mat_n=np.stack(mats.n).astype(np.float32),
        mat_k=np.stack(mats.k).astype(np.float32),
        mat_thick=np.asarray(mats.thick, dtype=np.float32),
        mat_le=np.stack(mats.le).astype(np.float32),
        light_type=int(light_type),
        light_p0=np.asarray(light_p0, dtype=np.float32),
        light_e1=np.asarray(light_e1, dtype=np.float32),
        light_e2=np.asarray(light_e2, dtype=np.float32),
        light_mat=int(light_mat),
        camera=camera or dict(eye=EYE, target=TARGET, fov_deg=FOV_DEG, ortho=False, ortho_half_h=1.0),
        name=name,
        seed=int(seed),
        cmf_provenance="proxy: multi-lobe Gaussian fit (Wyman-Sloan-Shirley 2013), not the CIE table",
    )
    n_lay = [len(x) for x in mats.layers]
    if any(n_lay):
        M, Lm, nl = len(mats.type), max(n_lay), len(lam)
        d = np.zeros((M, Lm), np.float32)
        n = np.ones((M, Lm, nl), np.float32)
        k = np.zeros((M, Lm, nl), np.float32)
        for m, lay in enumerate(mats.layers):
            for j, (dj, nj, kj) in enumerate(lay):
                d[m, j], n[m, j], k[m, j] = dj, nj, kj
        scene.update(mat_n_layers=np.asarray(n_lay, np.int32), mat_layer_d=d, mat_layer_n=n, mat_layer_k=k)
    return scene


def electrochromic_layers(lam_nm, state: float):
    """Synthetic five-layer electrochromic coating, listed from the air side:
    transparent conductor / electrochromic / ion conductor / counter electrode /
    transparent conductor, thicknesses 50-400 nm, n(lambda) in [1.4, 2.4] from
    Cauchy laws and k(lambda) in [0, 0.5].  ``state`` in [0, 1] is the
    colouring level: it scales the absorption bands of the electrochromic and
    counter-electrode layers.  Returns [(thickness_m, n[nl], k[nl]), ...]."""
    lam = np.asarray(lam_nm, dtype=np.float64)
    l_um = lam / 1000.0
    state = float(np.clip(state, 0.0, 1.0))

    def layer(d_nm, a, b, k):
        n = np.clip(a + b / l_um ** 2, 1.4, 2.4)
        return (d_nm * 1e-9, n.astype(np.float32), np.clip(k, 0.0, 0.5).astype(np.float32))

    tco = layer(150.0, 1.85, 0.012, np.full_like(lam, 0.004))
    ec = layer(300.0, 2.05, 0.020, 0.5 * state * np.exp(-0.5 * ((lam - 760.0) / 160.0) ** 2) + 0.002)
    ion = layer(200.0, 1.45, 0.004, np.zeros_like(lam))
    ce = layer(100.0, 2.15, 0.015, 0.2 * state * np.exp(-0.5 * ((lam - 450.0) / 90.0) ** 2) + 0.002)
    return [tco, ec, ion, ce, tco]


def _glass_material(mats, lam, k=1e-7, thick=0.004, coating_state=None):
    layers = None if coating_state is None else electrochromic_layers(lam, coating_state)
    return mats.add(GLASS, n=cauchy_n(lam), k=np.full(mats.nl, k, dtype=np.float32), thick=thick, layers=layers)


# ----------------------------------------------------------------------------
# the workloads
# ----------------------------------------------------------------------------

def tiny_room(seed: int = 0, n_lambda: int = 16, n_boxes: int = 20, window=((1, 1), (2, 1)), coating_state=None):
    """Tiny plain-method room: 1,092 triangles, one 4 mm pane, sky light.

    132 shell triangles, minus the 4 of the two window quads, plus the
    2-triangle pane, plus the 2-triangle sky emitter, plus 20 boxes with faces
    split 2 x 2 (48 triangles each).
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    lam, w = lambda_grid(n_lambda)
    mats = _Materials(len(lam))
    rect_mats = [mats.add(DIFFUSE, rho=gaussian_reflectance(rng, lam)) for _ in range(6)]
    pane = _glass_material(mats, lam, coating_state=coating_state)
    sky = mats.add(EMITTER, le=planck_shape(lam))
    mesh = _Mesh()
    _room_shell(mesh, rect_mats, window_cells=window, pane_mat=pane)
    _add_sky_light(mesh, sky)
    eye = np.asarray(EYE)
    placed = 0
    while placed < n_boxes:
        h = rng.uniform(0.05, 0.35, size=3)
        lo_c = h + 0.01
        hi_c = np.asarray(ROOM) - h - 0.01
        c = rng.uniform(lo_c, hi_c)
        lo, hi = c - h, c + h
        if not _box_clear_of_camera(lo, hi, eye):
            continue
        m = mats.add(DIFFUSE, rho=gaussian_reflectance(rng, lam))
        _box(mesh, lo, hi, 2, m)
        placed += 1
    return _finish(mesh, mats, lam, w, light_type=LIGHT_PARALLELOGRAM, light_mat=sky,
                   name=f"tiny_room(seed={seed},nl={n_lambda})", seed=seed)


def furnished_room(seed: int = 1, n_lambda: int = 41, min_tris: int = 200_000,
                   panes=((0, 1), (2, 1), (3, 2)), coating_state=None, name=None, detail: int = 1):
    """Room-scale plain-method room: >= ``min_tris`` triangles, three 4 mm panes.

    Furniture: boxes (faces s x s, s in 2..6) and capped z-axis cylinders
    (16..64 segments, 1..8 stacks), half-sizes U[0.03, 0.25] m, centres
    uniform in the room volume (1 cm clear of the shell, 0.1 m clear of the
    camera), generated until the triangle count reaches ``min_tris``.  With
    ``coating_state`` the panes carry the electrochromic coating
    (``electrochromic_layers``) on their room-side face.  ``detail`` multiplies
    the tessellation (face splits, segments and stacks), so a larger triangle
    budget buys finer furniture instead of more of it.
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    lam, w = lambda_grid(n_lambda)
    mats = _Materials(len(lam))
    rect_mats = [mats.add(DIFFUSE, rho=gaussian_reflectance(rng, lam)) for _ in range(6)]
    pane = _glass_material(mats, lam, coating_state=coating_state)
    sky = mats.add(EMITTER, le=planck_shape(lam))
    mesh = _Mesh()
    _room_shell(mesh, rect_mats, window_cells=panes, pane_mat=pane)
    _add_sky_light(mesh, sky)
    eye = np.asarray(EYE)
    room = np.asarray(ROOM)
    while mesh.ntri() < min_tris:
        is_box = rng.uniform() < 0.5
        if is_box:
            h = rng.uniform(0.03, 0.25, size=3)
        else:
            r = rng.uniform(0.03, 0.25)
            hh = rng.uniform(0.03, 0.25)
            h = np.array([r, r, hh])
        c = rng.uniform(h + 0.01, room - h - 0.01)
        lo, hi = c - h, c + h
        if not _box_clear_of_camera(lo, hi, eye):
            continue
        m = mats.add(DIFFUSE, rho=gaussian_reflectance(rng, lam))
        if is_box:
            _box(mesh, lo, hi, int(rng.integers(2, 7)) * detail, m)
        else:
            _cylinder(mesh, c, h[0], h[2], int(rng.integers(16, 65)) * detail, int(rng.integers(1, 9)) * detail, m)
    return _finish(mesh, mats, lam, w, light_type=LIGHT_PARALLELOGRAM, light_mat=sky,
                   name=name or f"furnished_room(seed={seed},nl={n_lambda},T>={min_tris})", seed=seed)


def photochromic_k(lam_nm, k_peak: float, k0: float = 1e-7, sigma_nm: float = 50.0):
    """Darkened pane absorption k(lambda) = k0 + (k_peak - k0) exp(-(lambda - 550)^2 / (2 sigma^2))."""
    lam = np.asarray(lam_nm, dtype=np.float64)
    return (k0 + (k_peak - k0) * np.exp(-0.5 * ((lam - 550.0) / sigma_nm) ** 2)).astype(np.float32)


def photochromic_states(scene, n_states: int = 8, k_lo: float = 1e-7, k_hi: float = 5e-6):
    """Append ``n_states`` darkening states of the scene's (first) glass material
    as extra glass materials (k_peak log-spaced over [k_lo, k_hi]); returns
    (scene, base glass material, [state material indices]).  A render selects
    a state by substituting its material for the base one."""
    sc = dict(scene)
    base = int(np.flatnonzero(sc["mat_type"] == GLASS)[0])
    lam = sc["lambda_nm"]
    ks = [photochromic_k(lam, kp) for kp in np.geomspace(k_lo, k_hi, n_states)]
    M = len(sc["mat_type"])
    rep = lambda a: np.concatenate([a, np.repeat(a[base:base + 1], n_states, axis=0)])
    sc["mat_type"] = rep(sc["mat_type"])
    sc["mat_rho"] = rep(sc["mat_rho"])
    sc["mat_n"] = rep(sc["mat_n"])
    sc["mat_thick"] = rep(sc["mat_thick"])
    sc["mat_le"] = rep(sc["mat_le"])
    sc["mat_k"] = np.concatenate([sc["mat_k"], np.stack(ks).astype(np.float32)])
    for key in ("mat_n_layers", "mat_layer_d", "mat_layer_n", "mat_layer_k"):
        if key in sc:
            sc[key] = rep(sc[key])
    sc["name"] = f"{scene['name']}+{n_states} photochromic states"
    return sc, base, list(range(M, M + n_states))


def batch_renders(n: int = 64, seed: int = 2, n_states: int = 8, sizes=(128, 256, 512, 1024), spp: int = 8):
    """Seeded render list for the batched workload: square resolutions drawn
    uniformly from ``sizes``, camera poses inside the room (eye 0.3 m clear of
    the walls, heading uniform, pitch within +-15 degrees, vertical fov 60
    degrees) and a photochromic state per render."""
    rng = np.random.Generator(np.random.PCG64(seed))
    room = np.asarray(ROOM)
    out = []
    for i in range(n):
        res = int(rng.choice(sizes))
        eye = rng.uniform(0.3, room - 0.3)
        yaw = rng.uniform(0.0, 2.0 * math.pi)
        pitch = math.radians(rng.uniform(-15.0, 15.0))
        look = np.array([math.cos(pitch) * math.cos(yaw), math.cos(pitch) * math.sin(yaw), math.sin(pitch)])
        cam = dict(eye=tuple(float(x) for x in eye), target=tuple(float(x) for x in eye + look), fov_deg=60.0,
                   ortho=False, ortho_half_h=1.0)
        out.append(dict(camera=cam, W=res, H=res, spp=spp, render_id=i, state=int(rng.integers(0, n_states))))
    return out


def nrc_params(seed: int = 0, table_size: int = 1 << 19, levels: int = 16, features: int = 2, n_in: int = 64,
               n_hid: int = 64, n_layers: int = 5):
    """Seeded initial parameters of the radiance-cache network (inputs of both
    the oracle and the GPU path): He-uniform weights U(-sqrt(6/fan_in),
    sqrt(6/fan_in)), zero biases, hash-table entries U(-1e-4, 1e-4).  float32."""
    rng = np.random.Generator(np.random.PCG64(seed))
    W, b = [], []
    fan = n_in
    for _ in range(n_layers):
        lim = math.sqrt(6.0 / fan)
        W.append(rng.uniform(-lim, lim, size=(n_hid, fan)).astype(np.float32))
        b.append(np.zeros(n_hid, np.float32))
        fan = n_hid
    lim = math.sqrt(6.0 / n_hid)
    wo = rng.uniform(-lim, lim, size=n_hid).astype(np.float32)
    tables = rng.uniform(-1e-4, 1e-4, size=(levels, table_size, features)).astype(np.float32)
    return dict(W=W, b=b, wo=wo, bo=np.float32(0.0)), tables


def nrc_rows(n: int, seed: int, aabb_lo=(0.0, 0.0, 0.0), aabb_hi=(4.0, 3.0, 2.5), lam=(380.0, 780.0)):
    """Seeded query rows (position in the box, unit direction, wavelength) and
    positive targets, for network tests."""
    rng = np.random.Generator(np.random.PCG64(seed))
    x = rng.uniform(aabb_lo, aabb_hi, size=(n, 3))
    w = rng.normal(size=(n, 3))
    w /= np.linalg.norm(w, axis=1, keepdims=True)
    lam_nm = rng.uniform(lam[0], lam[1], size=n)
    t = rng.gamma(2.0, 0.5, size=n)
    return x.astype(np.float32), w.astype(np.float32), lam_nm.astype(np.float32), t.astype(np.float32)


def nrc_room(seed: int = 3, n_lambda: int = 41, min_tris: int = 1_000_000, detail: int = 3):
    """Radiance-cache workload: the furnished-room recipe at >= 1M triangles,
    the furniture tessellated ``detail`` times finer (so the room holds about
    half as many pieces as the 200k room rather than five times as many)."""
    return furnished_room(seed=seed, n_lambda=n_lambda, min_tris=min_tris, detail=detail,
                          name=f"nrc_room(seed={seed},nl={n_lambda},T>={min_tris},detail={detail})")


def electrochromic_room(seed: int = 4, n_lambda: int = 81, min_tris: int = 4_000_000, coating_state: float = 0.6,
                        detail: int = 6):
    """Large electrochromic workload: the furnished-room recipe grown to
    >= 4M triangles with the furniture tessellated ``detail`` times finer (about
    370 pieces, as many as the room-scale workload has), 81 wavelengths, panes
    with the five-layer coating.  Reaching 4M triangles with more pieces
    instead walls off the windows: at the room-scale detail the camera's image
    is black."""
    return furnished_room(seed=seed, n_lambda=n_lambda, min_tris=min_tris, coating_state=coating_state,
                          detail=detail,
                          name=f"electrochromic_room(seed={seed},nl={n_lambda},T>={min_tris},state={coating_state},"
                               f"detail={detail})")


# ----------------------------------------------------------------------------
# closed-form fixtures
# ----------------------------------------------------------------------------

def floor_plane(n_lambda: int = 16, seed: int = 0):
    """Tessellated floor z = 0, x in [0,4], y in [0,3] (4 x 3 quads, 24 tris).

    Quad (i, j) covers x in [i, i+1], y in [j, j+1]; its triangles are
    2*(j*4 + i) (below the diagonal, local y-j <= x-i) and 2*(j*4 + i) + 1.
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    lam, w = lambda_grid(n_lambda)
    mats = _Materials(len(lam))
    m = mats.add(DIFFUSE, rho=gaussian_reflectance(rng, lam))
    mesh = _Mesh()
    _rect(mesh, (0, 0, 0), (4, 0, 0), (0, 3, 0), 4, 3, m)
    cam = dict(eye=(2.0, 1.5, 2.0), target=(2.0, 2.5, 0.0), fov_deg=60.0, ortho=False, ortho_half_h=1.0)
    return _finish(mesh, mats, lam, w, light_type=LIGHT_NONE, light_mat=-1,
                   name="floor_plane", seed=seed, camera=cam)


def point_light_plane(n_lambda: int = 16, seed: int = 0, pos=(2.0, 1.5, 1.5)):
    """Floor plane lit by one isotropic point light of intensity I(lambda) (Eq. 3)."""
    sc = floor_plane(n_lambda, seed)
    lam = sc["lambda_nm"]
    # the point light's intensity spectrum lives in an extra (unreferenced) emitter material
    le = planck_shape(lam, scale=5.0)
    for key, val in (("mat_type", EMITTER), ("mat_thick", 0.0)):
        sc[key] = np.append(sc[key], np.asarray([val], dtype=sc[key].dtype))
    sc["mat_rho"] = np.vstack([sc["mat_rho"], np.zeros((1, len(lam)), np.float32)])
    sc["mat_n"] = np.vstack([sc["mat_n"], np.ones((1, len(lam)), np.float32)])
    sc["mat_k"] = np.vstack([sc["mat_k"], np.zeros((1, len(lam)), np.float32)])
    sc["mat_le"] = np.vstack([sc["mat_le"], le[None, :]])
    sc["light_type"] = LIGHT_POINT
    sc["light_p0"] = np.asarray(pos, dtype=np.float32)
    sc["light_e1"] = np.zeros(3, np.float32)
    sc["light_e2"] = np.zeros(3, np.float32)
    sc["light_mat"] = len(sc["mat_type"]) - 1
    sc["name"] = "point_light_plane"
    sc["camera"] = dict(eye=(2.0, 1.5, 3.0), target=(2.0, 1.5001, 0.0), fov_deg=40.0, ortho=True,
                        ortho_half_h=1.2)
    return sc


PANE_A_CENTRE = (1.0, 1.5, 2.7)
PANE_A_TILT_DEG = 35.0
PANE_B_Z = 3.35
WALL_LIGHT_POS = (1.5, 1.5, 3.6)


def point_light_panes(n_lambda: int = 16, seed: int = 0, coating_state=None, extra_panes: int = 0):
    """A diffuse wall x = 0 lit by a point light (Eq. 3) that it sees only
    through two 4 mm panes, and a camera that sees the wall but no pane.

    * wall: x = 0, y in [-1, 4], z in [-1, 3.5], 5 x 5 quads, reflectance
      rho(lambda), facing +x;
    * pane A: 2 x 2 m, centred at PANE_A_CENTRE, tilted PANE_A_TILT_DEG about
      the y axis (geometric normal -(sin a, 0, cos a), facing down), so a
      shadow ray meets it at a cosine unlike its cosine at the wall;
    * pane B: horizontal, z = PANE_B_Z, x and y in [0.5, 2.5], geometric
      normal +z (facing up);
    * point light at WALL_LIGHT_POS, above both panes;
    * camera: eye (3, 1.5, 1.25) looking along -x at the wall, 30 degrees,
      whose rays stay below z = 2.05 on their way to the wall.

    Every shadow segment from the visible wall to the light crosses pane A,
    then pane B, and nothing else.  With ``coating_state`` both panes carry
    the electrochromic coating on the face their geometric normal points out
    of.  ``extra_panes`` stacks that many more horizontal panes 5 cm apart
    above pane B (each shadow segment then crosses 2 + extra_panes panes).
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    lam, w = lambda_grid(n_lambda)
    mats = _Materials(len(lam))
    wall = mats.add(DIFFUSE, rho=gaussian_reflectance(rng, lam))
    pane = _glass_material(mats, lam, coating_state=coating_state)
    point = mats.add(EMITTER, le=planck_shape(lam, scale=5.0))  # the point light's intensity I(lambda)
    mesh = _Mesh()
    _rect(mesh, (0, -1, -1), (0, 5, 0), (0, 0, 4.5), 5, 5, wall)
    a = math.radians(PANE_A_TILT_DEG)
    ca = np.asarray(PANE_A_CENTRE)
    du = np.array([0.0, 2.0, 0.0])
    dv = np.array([2.0 * math.cos(a), 0.0, -2.0 * math.sin(a)])
    _rect(mesh, ca - 0.5 * du - 0.5 * dv, du, dv, 1, 1, pane)   # geometric normal du x dv: -(sin a, 0, cos a)
    _rect(mesh, (0.5, 0.5, PANE_B_Z), (2, 0, 0), (0, 2, 0), 1, 1, pane)  # normal +z
    for i in range(extra_panes):
        _rect(mesh, (0.5, 0.5, PANE_B_Z + 0.05 * (i + 1)), (2, 0, 0), (0, 2, 0), 1, 1, pane)
    cam = dict(eye=(3.0, 1.5, 1.25), target=(0.0, 1.5, 1.25), fov_deg=30.0, ortho=False, ortho_half_h=1.0)
    return _finish(mesh, mats, lam, w, light_type=LIGHT_POINT, light_mat=point, name="point_light_panes",
                   seed=seed, light_p0=WALL_LIGHT_POS, light_e1=(0.0, 0.0, 0.0), light_e2=(0.0, 0.0, 0.0),
                   camera=cam)


def area_light_plane(n_lambda: int = 16, seed: int = 0):
    """Floor plane under a 1 x 0.8 m parallelogram emitter at z = 1.2 facing -z."""
    rng = np.random.Generator(np.random.PCG64(seed))
    lam, w = lambda_grid(n_lambda)
    mats = _Materials(len(lam))
    m = mats.add(DIFFUSE, rho=gaussian_reflectance(rng, lam))
    sky = mats.add(EMITTER, le=planck_shape(lam, scale=3.0))
    mesh = _Mesh()
    _rect(mesh, (0, 0, 0), (4, 0, 0), (0, 3, 0), 4, 3, m)
    p0, e1, e2 = np.array([1.5, 1.1, 1.2]), np.array([0.0, 0.8, 0.0]), np.array([1.0, 0.0, 0.0])
    # e1 x e2 = (0,0,-0.8): faces the floor
    a, b = mesh.vert(p0), mesh.vert(p0 + e1)
    c, d = mesh.vert(p0 + e1 + e2), mesh.vert(p0 + e2)
    mesh.tri(a, b, c, sky)
    mesh.tri(a, c, d, sky)
    cam = dict(eye=(2.0, 1.5, 0.9), target=(2.0, 1.5001, 0.0), fov_deg=40.0, ortho=True, ortho_half_h=1.0)
    return _finish(mesh, mats, lam, w, light_type=LIGHT_PARALLELOGRAM, light_mat=sky,
                   name="area_light_plane", seed=seed, light_p0=p0, light_e1=e1, light_e2=e2,
                   camera=cam)


def furnace_room(seed: int = 0, n_lambda: int = 16, n_boxes: int = 20):
    """Closed room (no window, no light) with C0-style boxes; every surface is
    the same diffuse material with reflectance rho(lambda) and two-sided
    emission Le(lambda).  Every path of depth D returns Le * sum_{i<D} rho^i.
    """
    sc = tiny_room(seed=seed, n_lambda=n_lambda, n_boxes=n_boxes, window=())
    lam = sc["lambda_nm"]
    rng = np.random.Generator(np.random.PCG64(seed + 1000))
    rho = gaussian_reflectance(rng, lam)
    le = planck_shape(lam, scale=1.0)
    # drop the sky emitter triangles: the furnace is closed and has no NEE light
    keep = sc["mat_type"][sc["tri_mat"]] != EMITTER
    sc["tris"] = sc["tris"][keep]
    sc["tri_mat"] = np.zeros(int(keep.sum()), dtype=np.int32)
    sc["mat_type"] = np.asarray([DIFFUSE], dtype=np.int32)
    sc["mat_rho"] = rho[None, :].astype(np.float32)
    sc["mat_n"] = np.ones((1, len(lam)), np.float32)
    sc["mat_k"] = np.zeros((1, len(lam)), np.float32)
    sc["mat_thick"] = np.zeros(1, np.float32)
    sc["mat_le"] = le[None, :].astype(np.float32)
    sc["light_type"] = LIGHT_NONE
    sc["light_mat"] = -1
    sc["name"] = "furnace_room"
    return sc


def lone_pane(n_lambda: int = 16, seed: int = 0, k: float = 1e-7, thick: float = 0.004, coating_state=None):
    """A single 1 x 1 m pane at y = 1 with a large emitter behind it (y = 2,
    facing -y) and an orthographic camera looking along +y at normal incidence.
    With ``coating_state`` the pane carries the electrochromic coating on its
    camera-side face (the face its geometric normal, -y, points out of)."""
    lam, w = lambda_grid(n_lambda)
    mats = _Materials(len(lam))
    pane = _glass_material(mats, lam, k=k, thick=thick, coating_state=coating_state)
    sky = mats.add(EMITTER, le=planck_shape(lam))
    mesh = _Mesh()
    _rect(mesh, (0, 1, 0), (1, 0, 0), (0, 0, 1), 1, 1, pane)
    p0, e1, e2 = np.array([-2.0, 2.0, -2.0]), np.array([5.0, 0.0, 0.0]), np.array([0.0, 0.0, 5.0])
    a, b = mesh.vert(p0), mesh.vert(p0 + e1)
    c, d = mesh.vert(p0 + e1 + e2), mesh.vert(p0 + e2)
    mesh.tri(a, b, c, sky)
    mesh.tri(a, c, d, sky)
    cam = dict(eye=(0.5, 0.0, 0.5), target=(0.5, 1.0, 0.5), fov_deg=40.0, ortho=True, ortho_half_h=0.4)
    return _finish(mesh, mats, lam, w, light_type=LIGHT_PARALLELOGRAM, light_mat=sky,
                   name="lone_pane", seed=seed, light_p0=p0, light_e1=e1, light_e2=e2, camera=cam)


def save_npz(scene, path):
    flat = {k: v for k, v in scene.items() if isinstance(v, np.ndarray)}
    for k in ("light_type", "light_mat", "seed"):
        flat[k] = np.asarray(scene[k])
    cam = scene["camera"]
    flat["cam_eye"] = np.asarray(cam["eye"], np.float64)
    flat["cam_target"] = np.asarray(cam["target"], np.float64)
    flat["cam_fov_deg"] = np.asarray(cam["fov_deg"], np.float64)
    flat["cam_ortho"] = np.asarray(int(cam["ortho"]))
    flat["cam_ortho_half_h"] = np.asarray(cam["ortho_half_h"], np.float64)
    np.savez(path, **flat)


def load_npz(path):
    z = np.load(path, allow_pickle=False)
    sc = {k: z[k] for k in z.files if not k.startswith("cam_")}
    for k in ("light_type", "light_mat", "seed"):
        sc[k] = int(sc[k])
    sc["camera"] = dict(eye=tuple(z["cam_eye"]), target=tuple(z["cam_target"]),
                        fov_deg=float(z["cam_fov_deg"]), ortho=bool(int(z["cam_ortho"])),
                        ortho_half_h=float(z["cam_ortho_half_h"]))
    sc["name"] = str(path)
    sc["cmf_provenance"] = "loaded"
    return sc


WORKLOADS = {
    "tiny_room": dict(build=lambda: tiny_room(0, 16), W=64, H=64, spp=1, max_depth=4, grid=(2, 2, 1), seed=0),
    "furnished_room": dict(build=lambda: furnished_room(1, 41), W=512, H=512, spp=16, max_depth=8,
                           grid=(4, 4, 2), seed=0),
    "electrochromic_room": dict(build=lambda: electrochromic_room(4, 81), W=3840, H=2160, spp=64, max_depth=8,
                                grid=(8, 4, 4), seed=0),
    "nrc_room": dict(build=lambda: nrc_room(3, 41), W=1920, H=1080, spp=4, max_depth=8, grid=(4, 4, 2), seed=0),
}
