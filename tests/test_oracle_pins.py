"""Pins of the FP64 oracle against what the paper and mathematics fix.

None of these re-type the oracle's own formulas: each checks a closed form,
a special case, an invariant, a brute-force sum, or a third-party library
(rocRAND) output.  They run on the CPU.
"""
import math
import os

import numpy as np
import pytest

import oracle as ora
import scenegen as sg

GOLD = os.path.join(os.path.dirname(__file__), "golden")


# --------------------------------------------------------------------------
# Philox4x32-10 and the uniform mapping
# --------------------------------------------------------------------------

def _kat():
    rows = []
    with open(os.path.join(GOLD, "philox_kat.txt")) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            rows.append([int(x) for x in line.split()])
    return rows


def test_philox_matches_rocrand_vectors():
    rows = _kat()
    assert len(rows) >= 8
    for v in rows:
        assert list(ora.philox(v[0:4], v[4:6])) == v[6:10]


def test_u01_is_24_bit_exact():
    assert ora.u01(0) == 0.0
    assert ora.u01(0xFFFFFFFF) == 1.0 - 2.0 ** -24
    assert ora.u01(256) == 2.0 ** -24
    assert ora.u01(255) == 0.0
    # representable in float32 without rounding
    for x in (0x12345678, 0xDEADBEEF, 0x80000000):
        u = ora.u01(x)
        assert float(np.float32(u)) == u


# --------------------------------------------------------------------------
# Fresnel from the complex index (Eq. 1) and the pane slab (Sec. 6)
# --------------------------------------------------------------------------

@pytest.mark.parametrize("n,k", [(1.5, 0.0), (1.513884, 1e-7), (1.33, 0.0), (2.4, 0.5), (0.2, 3.0),
                                 (1.7, 5e-6), (1.0, 0.1)])
def test_normal_incidence_closed_form(n, k):
    rs, rp = ora.fresnel_sp(n, k, 1.0)
    closed = ((n - 1) ** 2 + k ** 2) / ((n + 1) ** 2 + k ** 2)
    assert rs == pytest.approx(closed, rel=1e-12, abs=1e-15)
    assert rp == pytest.approx(closed, rel=1e-12, abs=1e-15)
    assert 0.0 < rs < 1.0


def test_c0_pane_normal_incidence_value():
    # Cauchy n = 1.5 + 0.0042 / 0.55^2 at 550 nm
    n = float(sg.cauchy_n([550.0])[0])
    assert n == pytest.approx(1.513884, abs=5e-7)
    rs, _ = ora.fresnel_sp(n, 0.0, 1.0)
    assert rs == pytest.approx(0.0417869, abs=5e-7)


@pytest.mark.parametrize("n", [1.33, 1.5, 1.9, 2.4])
def test_brewster_angle_zero_p(n):
    th = math.atan(n)
    rs, rp = ora.fresnel_sp(n, 0.0, math.cos(th))
    assert rp < 1e-25
    assert rs > 0.01


@pytest.mark.parametrize("n", [1.33, 1.5, 2.0])
@pytest.mark.parametrize("deg", [5.0, 30.0, 55.0, 80.0])
def test_reciprocity_inside_outside(n, deg):
    ci = math.cos(math.radians(deg))
    st = math.sin(math.radians(deg)) / n                  # Snell
    ct = math.sqrt(1.0 - st * st)
    rs_out, rp_out = ora.fresnel_sp(n, 0.0, ci)
    rs_in, rp_in = ora.fresnel_sp(1.0 / n, 0.0, ct)        # from the glass side
    assert rs_in == pytest.approx(rs_out, rel=1e-10)
    assert rp_in == pytest.approx(rp_out, rel=1e-10)


def test_total_internal_reflection():
    n_rel = 1.0 / 1.5
    crit = math.asin(n_rel)
    for deg in (math.degrees(crit) + 0.5, 60.0, 85.0):
        rs, rp = ora.fresnel_sp(n_rel, 0.0, math.cos(math.radians(deg)))
        assert rs == pytest.approx(1.0, abs=1e-12)
        assert rp == pytest.approx(1.0, abs=1e-12)


def test_lossless_slab_closed_forms():
    rs, rp, ts, tp = ora.slab_sp(1.5, 0.0, 0.004, 550.0, 1.0)
    R = 0.04
    assert rs == pytest.approx(2 * R / (1 + R), rel=1e-12)
    assert ts == pytest.approx((1 - R) / (1 + R), rel=1e-12)
    assert rs == pytest.approx(0.076923, abs=5e-7)
    assert ts == pytest.approx(0.923077, abs=5e-7)
    Rm, Tm = ora.slab(1.5, 0.0, 0.004, 550.0, 1.0)
    assert Rm == pytest.approx(rs) and Tm == pytest.approx(ts)


def test_slab_equals_explicit_multiple_reflection_sum():
    """Brute force: follow the light bouncing inside the pane term by term."""
    rng = np.random.default_rng(3)
    for _ in range(50):
        n = rng.uniform(1.3, 2.2)
        k = 10 ** rng.uniform(-8, -5)
        lam = rng.uniform(380, 780)
        d = rng.uniform(0.001, 0.01)
        c = rng.uniform(0.05, 1.0)
        rs, rp = ora.fresnel_sp(n, k, c)
        cos_r = math.sqrt(1.0 - (1.0 - c * c) / (n * n))
        tau = math.exp(-4 * math.pi * k / (lam * 1e-9) * d / cos_r)
        got = ora.slab_sp(n, k, d, lam, c)
        for i, Rf in enumerate((rs, rp)):
            refl = Rf              # first surface reflection
            trans = 0.0
            amp = (1 - Rf) * tau   # entered, crossed once
            for _m in range(400):
                trans += amp * (1 - Rf)      # leaves through the back face
                amp *= Rf * tau              # reflects at the back face, crosses back
                refl += amp * (1 - Rf)       # leaves through the front face
                amp *= Rf * tau              # reflects at the front face, crosses again
            assert got[i] == pytest.approx(refl, rel=1e-12)
            assert got[2 + i] == pytest.approx(trans, rel=1e-12)


def test_slab_energy_balance():
    rng = np.random.default_rng(5)
    for _ in range(500):
        n = rng.uniform(1.2, 2.4)
        k = rng.choice([0.0, 10 ** rng.uniform(-8, -3)])
        lam = rng.uniform(380, 780)
        c = rng.uniform(0.0, 1.0)
        rs, rp, ts, tp = ora.slab_sp(n, k, 0.004, lam, c)
        for R, T in ((rs, ts), (rp, tp)):
            A = 1.0 - R - T
            assert A >= -1e-12
            assert 0.0 <= R <= 1.0 and 0.0 <= T <= 1.0
            if k == 0.0:
                assert abs(A) < 1e-12


def test_c0_pane_values_550nm():
    n = float(np.float64(sg.cauchy_n([550.0])[0]))
    R, T = ora.slab(n, 1e-7, 0.004, 550.0, 1.0)
    tau = math.exp(-4 * math.pi * 1e-7 / 550e-9 * 0.004)
    assert tau == pytest.approx(0.990902, abs=5e-7)
    assert R == pytest.approx(0.079524, abs=2e-6)
    assert T == pytest.approx(0.911382, abs=2e-6)
    assert 1 - R - T == pytest.approx(0.009094, abs=3e-6)


@pytest.mark.parametrize("deg", [0.0, 20.0, 45.0, 70.0])
def test_beer_lambert_limit(deg):
    c = math.cos(math.radians(deg))
    k, d, lam = 5e-6, 0.004, 550.0
    _, T = ora.slab(1.0, k, d, lam, c)   # index-matched: no interface reflection besides k^2/4
    bl = math.exp(-4 * math.pi * k * d / (lam * 1e-9 * c))
    assert T == pytest.approx(bl, rel=1e-9)
    if deg == 0.0:
        assert bl == pytest.approx(0.633206, abs=5e-7)


# --------------------------------------------------------------------------
# sampling and camera
# --------------------------------------------------------------------------

@pytest.mark.parametrize("normal", [(0, 0, 1), (0, 0, -1), (1, 0, 0), (0.3, -0.5, 0.81), (-0.6, 0.64, -0.48)])
def test_cosine_hemisphere_moments(normal):
    n = np.asarray(normal, float)
    n /= np.linalg.norm(n)
    m = 200
    us = (np.arange(m) + 0.5) / m
    cos_sum = cos2_sum = 0.0
    mean_dir = np.zeros(3)
    for u0 in us:
        for u1 in us:
            w = ora.cosine_hemisphere(n, u0, u1)
            assert abs(np.linalg.norm(w) - 1.0) < 1e-12
            c = float(w @ n)
            assert c == pytest.approx(math.sqrt(1 - u0), abs=1e-12)
            cos_sum += c
            cos2_sum += c * c
            mean_dir += w
    N = m * m
    # pdf cos(theta)/pi: E[cos] = 2/3, E[cos^2] = 1/2, mean direction = (2/3) n
    assert cos_sum / N == pytest.approx(2 / 3, abs=2e-4)
    assert cos2_sum / N == pytest.approx(1 / 2, abs=2e-4)
    assert np.allclose(mean_dir / N, (2 / 3) * n, atol=2e-4)


def test_pinhole_field_of_view_and_orientation():
    cam = dict(eye=(0, 0, 0), target=(0, 1, 0), fov_deg=70.0, ortho=False)
    W, H = 80, 60
    _, d_c = ora.camera_ray(cam, W, H, W / 2, H / 2)
    assert np.allclose(d_c, [0, 1, 0], atol=1e-15)
    _, d_top = ora.camera_ray(cam, W, H, W / 2, 0.0)
    ang = math.degrees(math.acos(d_top @ np.array([0, 1, 0])))
    assert ang == pytest.approx(35.0, abs=1e-9)          # half the vertical fov
    assert d_top[2] > 0                                   # row 0 is the top
    _, d_left = ora.camera_ray(cam, W, H, 0.0, H / 2)
    hang = math.degrees(math.atan(math.tan(math.radians(35)) * W / H))
    assert math.degrees(math.acos(d_left @ np.array([0, 1, 0]))) == pytest.approx(hang, abs=1e-9)
    assert d_left[0] < 0                                  # column 0 is the left


def test_orthographic_rays_are_parallel():
    cam = dict(eye=(0.5, 0.0, 0.5), target=(0.5, 1.0, 0.5), fov_deg=40.0, ortho=True, ortho_half_h=0.4)
    o1, d1 = ora.camera_ray(cam, 32, 32, 0.0, 0.0)
    o2, d2 = ora.camera_ray(cam, 32, 32, 32.0, 32.0)
    assert np.allclose(d1, [0, 1, 0]) and np.allclose(d2, [0, 1, 0])
    assert np.allclose(o1, [0.1, 0.0, 0.9]) and np.allclose(o2, [0.9, 0.0, 0.1])


# --------------------------------------------------------------------------
# traversal: ray-plane analytic hits, BVH == brute force
# --------------------------------------------------------------------------

def test_ray_plane_analytic_hits():
    sc = sg.floor_plane()
    rng = np.random.default_rng(11)
    n = 4000
    o = np.column_stack([rng.uniform(-1, 5, n), rng.uniform(-1, 4, n), rng.uniform(0.2, 3, n)])
    target = np.column_stack([rng.uniform(0.02, 3.98, n), rng.uniform(0.02, 2.98, n), np.zeros(n)])
    d = target - o
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    osc = ora.OracleScene(sc)
    for use_bvh in (True, False):
        t, prim = ora.trace_rays(sc, o, d, use_bvh=use_bvh, oscene=osc)
        t_plane = -o[:, 2] / d[:, 2]
        assert np.allclose(t, t_plane, rtol=1e-12)
        x = o + t[:, None] * d
        i = np.floor(x[:, 0]).astype(int)
        j = np.floor(x[:, 1]).astype(int)
        fx, fy = x[:, 0] - i, x[:, 1] - j
        away = np.abs(fx - fy) > 1e-9   # not on the diagonal
        expect = 2 * (j * 4 + i) + (fy > fx).astype(int)
        assert np.array_equal(prim[away], expect[away])
        assert np.all(prim >= 0)
    # rays pointing away miss
    t, prim = ora.trace_rays(sc, o, -d, oscene=osc)
    assert np.all(prim == -1) and np.all(np.isinf(t))


@pytest.mark.parametrize("which", ["tiny", "furnished"])
def test_bvh_equals_brute_force(which):
    sc = sg.tiny_room() if which == "tiny" else sg.furnished_room(min_tris=20_000)
    rng = np.random.default_rng(7)
    n = 3000 if which == "tiny" else 600
    o = rng.uniform([0.05, 0.05, 0.05], [3.95, 2.95, 2.45], size=(n, 3))
    d = rng.normal(size=(n, 3))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    osc = ora.OracleScene(sc)
    t1, p1 = ora.trace_rays(sc, o, d, use_bvh=True, oscene=osc)
    t0, p0 = ora.trace_rays(sc, o, d, use_bvh=False, oscene=osc)
    assert np.array_equal(p0, p1)
    assert np.array_equal(t0, t1)
    r = rng.uniform(0.1, 4.0, n)
    s1 = ora.shadow_rays(sc, o, d, r, use_bvh=True, oscene=osc)
    s0 = ora.shadow_rays(sc, o, d, r, use_bvh=False, oscene=osc)
    assert np.array_equal(s0, s1)


def test_render_bvh_equals_brute_force(tiny_scene):
    a = ora.render(tiny_scene, 32, 32, 2, 4, logs=True, use_bvh=True)
    b = ora.render(tiny_scene, 32, 32, 2, 4, logs=True, use_bvh=False)
    assert np.array_equal(a["hit_log"], b["hit_log"])
    assert np.array_equal(a["shadow_log"], b["shadow_log"])
    assert np.array_equal(a["spectral"], b["spectral"])


# --------------------------------------------------------------------------
# transport loop: furnace, point light (Eq. 3), area light, glass pane
# --------------------------------------------------------------------------

@pytest.mark.parametrize("D", [1, 3, 6])
def test_furnace_closed_form(D):
    sc = sg.furnace_room()
    rho = sc["mat_rho"][0].astype(np.float64)
    le = sc["mat_le"][0].astype(np.float64)
    expect = le * (1.0 - rho ** D) / (1.0 - rho)          # Le * sum_{i<D} rho^i
    r = ora.render(sc, 24, 24, 2, D, path_L=True, logs=True)
    pl = r["path_L"].reshape(-1, len(rho))
    assert np.all(r["hit_log"] != -1)                      # closed room: nothing escapes
    assert np.allclose(pl, expect[None, :], rtol=1e-12, atol=0)


def test_point_light_eq3():
    sc = sg.point_light_plane()
    W = H = 24
    r = ora.render(sc, W, H, 1, 1, path_L=True, first_hit=True)
    x = r["first_hit"].reshape(-1, 3)
    L = r["path_L"].reshape(-1, sc["mat_rho"].shape[1])
    rho = sc["mat_rho"][0].astype(np.float64)
    I = sc["mat_le"][sc["light_mat"]].astype(np.float64)
    pL = sc["light_p0"].astype(np.float64)
    xo = x + np.array([0, 0, 1e-4])           # origin offset along the normal toward the viewer
    w = pL - xo
    r2 = (w * w).sum(1)
    cos = w[:, 2] / np.sqrt(r2)
    expect = (rho[None, :] / math.pi) * I[None, :] * (cos / r2)[:, None]
    assert np.all(np.isfinite(x))
    assert np.allclose(L, expect, rtol=1e-12)


def _polygon_irradiance_geo(x, n, verts):
    """Lambert's formula: integral over the polygon of cos_x cos_y / r^2 dA."""
    a = [(v - x) / np.linalg.norm(v - x) for v in verts]
    tot = 0.0
    for i in range(len(a)):
        b, c = a[i], a[(i + 1) % len(a)]
        theta = math.acos(max(-1.0, min(1.0, float(b @ c))))
        g = np.cross(b, c)
        g /= np.linalg.norm(g)
        tot += theta * float(g @ n)
    return abs(0.5 * tot)


def test_area_light_matches_polygon_irradiance():
    sc = sg.area_light_plane()
    W = H = 8
    spp = 256
    r = ora.render(sc, W, H, spp, 1, path_L=True, first_hit=True)
    x = r["first_hit"].reshape(-1, 3)
    L = r["path_L"].reshape(-1, sc["mat_rho"].shape[1])
    rho = sc["mat_rho"][0].astype(np.float64)
    Le = sc["mat_le"][sc["light_mat"]].astype(np.float64)
    p0, e1, e2 = (sc[k].astype(np.float64) for k in ("light_p0", "light_e1", "light_e2"))
    poly = [p0, p0 + e1, p0 + e1 + e2, p0 + e2]
    ratios = []
    for xi, Li in zip(x, L):
        xo = xi + np.array([0, 0, 1e-4])
        geo = _polygon_irradiance_geo(xo, np.array([0, 0, 1.0]), poly)
        expect = rho / math.pi * Le * geo
        ratios.append(Li[5] / expect[5])
        # every wavelength carries the same geometric estimate
        assert np.allclose(Li / expect, Li[5] / expect[5], rtol=1e-10)
    ratios = np.asarray(ratios)
    err = ratios.std() / math.sqrt(len(ratios))
    assert abs(ratios.mean() - 1.0) < 3.5 * err + 1e-12


def test_glass_pane_transmission_branch():
    sc = sg.lone_pane()
    W = H = 16
    spp = 64
    r = ora.render(sc, W, H, spp, 2, path_L=True, logs=True)
    nl = sc["mat_rho"].shape[1]
    L = r["path_L"].reshape(-1, nl)
    Le = sc["mat_le"][1].astype(np.float64)
    R = np.zeros(nl)
    T = np.zeros(nl)
    for l in range(nl):
        R[l], T[l] = ora.slab(float(sc["mat_n"][0, l]), float(sc["mat_k"][0, l]), float(sc["mat_thick"][0]),
                              float(sc["lambda_nm"][l]), 1.0)
    PR = R.mean() / (R.mean() + T.mean())
    trans = np.all(L > 0, axis=1)
    # orthographic rays at normal incidence: each sample is 0 (reflected away) or Le * T / (1 - PR)
    assert np.allclose(L[trans], (Le * T / (1 - PR))[None, :], rtol=1e-12)
    assert np.all(L[~trans] == 0.0)
    frac = trans.mean()
    sd = math.sqrt(PR * (1 - PR) / len(L))
    assert abs(frac - (1 - PR)) < 4 * sd
    hl = r["hit_log"].reshape(-1, 2)
    assert np.all(hl[:, 0] >= 0)
    assert np.all((hl[trans, 1] >= 0))
    assert np.all(hl[~trans, 1] == -1)


def test_logs_are_consistent(tiny_scene):
    r = ora.render(tiny_scene, 16, 16, 2, 4, logs=True)
    hl = r["hit_log"].reshape(-1, 4)
    for row in hl:
        ended = False
        for v in row:
            if ended:
                assert v == -2
            if v < 0:
                ended = True
    sl = r["shadow_log"]
    assert set(np.unique(sl)) <= {-2, 0, 1}


# ---------------------------------------------------------------------------
# coherent thin-film coating (electrochromic windows): characteristic matrices
# ---------------------------------------------------------------------------
def _admittance(N, beta, p_pol):
    Nc = np.sqrt(complex(N) ** 2 - beta ** 2)
    if Nc.real < 0 or (Nc.real == 0 and Nc.imag < 0):
        Nc = -Nc
    return N * N / Nc if p_pol else Nc, Nc


def _rouard_r(layers, N_in, N_out, lam_nm, beta, p_pol):
    """Amplitude reflectance of a stack by the Rouard recursion of Airy's
    two-interface formula, from the exit medium up: r_j = (rho_j + r_{j+1} e)
    / (1 + rho_j r_{j+1} e), e = exp(2 i delta_j) (fields ~ exp(-i omega t),
    N = n + i k, so Im delta > 0 attenuates)."""
    media = [N_in] + [complex(n, k) for (_, n, k) in layers] + [N_out]
    eta = [_admittance(N, beta, p_pol)[0] for N in media]
    rho = [(eta[i] - eta[i + 1]) / (eta[i] + eta[i + 1]) for i in range(len(media) - 1)]
    r = rho[-1]
    for j in range(len(layers), 0, -1):
        d = layers[j - 1][0]
        Nc = _admittance(media[j], beta, p_pol)[1]
        e = np.exp(2j * 2 * np.pi * Nc * d / (lam_nm * 1e-9))
        r = (rho[j - 1] + r * e) / (1 + rho[j - 1] * r * e)
    return r


def _tmm(layers, n_in, k_in, n_out, k_out, lam, beta):
    d = [x[0] for x in layers]
    n = [x[1] for x in layers]
    k = [x[2] for x in layers]
    return ora.tmm_sp(d, n, k, n_in, k_in, n_out, k_out, lam, beta)


@pytest.mark.parametrize("c", [1.0, 0.6, 0.15])
def test_tmm_zero_thickness_layers_are_the_bare_interface(c):
    beta = math.sqrt(1 - c * c)
    layers = [(0.0, 2.1, 0.3), (0.0, 1.45, 0.0), (0.0, 2.3, 0.05)]
    Rs, Rp, Ts, Tp = _tmm(layers, 1.0, 0.0, 1.52, 0.0, 550.0, beta)
    Fs, Fp = ora.fresnel_sp(1.52, 0.0, c)
    assert Rs == pytest.approx(Fs, rel=1e-12, abs=1e-15)
    assert Rp == pytest.approx(Fp, rel=1e-12, abs=1e-15)
    assert Ts == pytest.approx(1 - Fs, rel=1e-12)
    assert Tp == pytest.approx(1 - Fp, rel=1e-12)


@pytest.mark.parametrize("c", [1.0, 0.7, 0.3])
@pytest.mark.parametrize("layer", [(120e-9, 1.9, 0.0), (80e-9, 2.2, 0.35)])
def test_tmm_single_layer_is_airy(c, layer):
    beta = math.sqrt(1 - c * c)
    lam = 520.0
    Rs, Rp, _, _ = _tmm([layer], 1.0, 0.0, 1.52, 0.0, lam, beta)
    # Airy: r = (r01 + r12 exp(2 i delta)) / (1 + r01 r12 exp(2 i delta)) with
    # Fresnel amplitudes written from Snell's law directly
    N1, Ns = complex(layer[1], layer[2]), 1.52
    for p_pol, R in ((False, Rs), (True, Rp)):
        c1 = np.sqrt(1 - (beta / N1) ** 2)
        cs = np.sqrt(1 - (beta / Ns) ** 2)
        if p_pol:
            r01 = (N1 * c - 1.0 * c1) / (N1 * c + 1.0 * c1)
            r12 = (Ns * c1 - N1 * cs) / (Ns * c1 + N1 * cs)
        else:
            r01 = (c - N1 * c1) / (c + N1 * c1)
            r12 = (N1 * c1 - Ns * cs) / (N1 * c1 + Ns * cs)
        e = np.exp(2j * 2 * np.pi * N1 * c1 * layer[0] / (lam * 1e-9))
        r = (r01 + r12 * e) / (1 + r01 * r12 * e)
        assert R == pytest.approx(abs(r) ** 2, rel=1e-10, abs=1e-14)


@pytest.mark.parametrize("state", [0.0, 0.5, 1.0])
@pytest.mark.parametrize("c", [1.0, 0.5, 0.1])
def test_tmm_electrochromic_stack_matches_rouard_recursion(state, c):
    lam = sg.lambda_grid(16)[0]
    lay = sg.electrochromic_layers(lam, state)
    beta = math.sqrt(1 - c * c)
    for l in (0, 7, 15):
        layers = [(float(d), float(n[l]), float(k[l])) for (d, n, k) in lay]
        Rs, Rp, Ts, Tp = _tmm(layers, 1.0, 0.0, 1.52, 0.0, float(lam[l]), beta)
        for p_pol, R in ((False, Rs), (True, Rp)):
            r = _rouard_r(layers, 1.0, 1.52, float(lam[l]), beta, p_pol)
            assert R == pytest.approx(abs(r) ** 2, rel=1e-9, abs=1e-13)
        # absorbing layers: 0 <= R, T and R + T <= 1
        for R, T in ((Rs, Ts), (Rp, Tp)):
            assert 0 <= R <= 1 and 0 <= T <= 1 and R + T <= 1 + 1e-12


def test_tmm_quarter_wave_antireflection():
    ns, lam0 = 1.52, 550.0
    n1 = math.sqrt(ns)
    layer = [(lam0 * 1e-9 / (4 * n1), n1, 0.0)]
    Rs, Rp, Ts, Tp = _tmm(layer, 1.0, 0.0, ns, 0.0, lam0, 0.0)
    assert Rs < 1e-20 and Rp < 1e-20
    assert Ts == pytest.approx(1.0, rel=1e-12)
    bare = ora.fresnel_sp(ns, 0.0, 1.0)[0]
    for lam in (400.0, 750.0):
        R = _tmm(layer, 1.0, 0.0, ns, 0.0, lam, 0.0)[0]
        assert 0 < R < bare


@pytest.mark.parametrize("c", [1.0, 0.8, 0.4, 0.05])
def test_tmm_lossless_stack_conserves_energy(c):
    beta = math.sqrt(1 - c * c)
    layers = [(150e-9, 1.85, 0.0), (300e-9, 2.05, 0.0), (200e-9, 1.45, 0.0), (100e-9, 2.15, 0.0), (150e-9, 1.85, 0.0)]
    Rs, Rp, Ts, Tp = _tmm(layers, 1.0, 0.0, 1.52, 0.0, 480.0, beta)
    assert Rs + Ts == pytest.approx(1.0, abs=1e-12)
    assert Rp + Tp == pytest.approx(1.0, abs=1e-12)


def test_thick_absorbing_layer_is_semi_infinite():
    c = math.sqrt(1 - 0.09)
    Rs, Rp, Ts, Tp = _tmm([(5e-6, 2.0, 0.5)], 1.0, 0.0, 1.5, 0.0, 500.0, 0.3)
    N = complex(2.0, 0.5)
    Nc = np.sqrt(N * N - 0.09)
    assert Rs == pytest.approx(abs((c - Nc) / (c + Nc)) ** 2, rel=1e-9)
    assert Rp == pytest.approx(abs((N * N / Nc - 1 / c) / (N * N / Nc + 1 / c)) ** 2, rel=1e-9)
    assert Ts < 1e-20 and Tp < 1e-20


@pytest.mark.parametrize("c", [1.0, 0.5])
def test_coated_pane_without_coating_is_the_slab(c):
    for side in (True, False):
        Rc, Tc = ora.coated_pane(1.52, 2e-6, 0.004, [], [], [], 600.0, c, side)
        Rsl, Tsl = ora.slab(1.52, 2e-6, 0.004, 600.0, c)
        assert Rc == pytest.approx(Rsl, rel=1e-13)
        assert Tc == pytest.approx(Tsl, rel=1e-13)
        Rz, Tz = ora.coated_pane(1.52, 2e-6, 0.004, [0.0, 0.0], [2.0, 1.5], [0.4, 0.0], 600.0, c, side)
        assert Rz == pytest.approx(Rsl, rel=1e-12)
        assert Tz == pytest.approx(Tsl, rel=1e-12)


@pytest.mark.parametrize("state", [0.2, 1.0])
def test_coated_pane_reciprocity_and_energy(state):
    lam = sg.lambda_grid(41)[0]
    lay = sg.electrochromic_layers(lam, state)
    for l in (3, 20, 38):
        d = [float(x[0]) for x in lay]
        n = [float(x[1][l]) for x in lay]
        k = [float(x[2][l]) for x in lay]
        for c in (1.0, 0.6, 0.2):
            Rf, Tf = ora.coated_pane(1.52, 1e-7, 0.004, d, n, k, float(lam[l]), c, True)
            Rb, Tb = ora.coated_pane(1.52, 1e-7, 0.004, d, n, k, float(lam[l]), c, False)
            assert Tf == pytest.approx(Tb, rel=1e-11)       # reciprocity of transmission
            assert Rf != pytest.approx(Rb, rel=1e-6)        # absorbing coating: R depends on the side
            for R, T in ((Rf, Tf), (Rb, Tb)):
                assert 0 < R < 1 and 0 < T < 1 and R + T < 1


def test_coated_pane_transmission_branch():
    sc = sg.lone_pane(coating_state=0.8)
    W = H = 8
    r = ora.render(sc, W, H, 64, 2, path_L=True)
    nl = sc["mat_rho"].shape[1]
    L = r["path_L"].reshape(-1, nl)
    Le = sc["mat_le"][1].astype(np.float64)
    R = np.zeros(nl)
    T = np.zeros(nl)
    for l in range(nl):
        d = sc["mat_layer_d"][0].astype(np.float64)
        R[l], T[l] = ora.coated_pane(float(sc["mat_n"][0, l]), float(sc["mat_k"][0, l]), float(sc["mat_thick"][0]),
                                     d, sc["mat_layer_n"][0, :, l].astype(np.float64),
                                     sc["mat_layer_k"][0, :, l].astype(np.float64), float(sc["lambda_nm"][l]), 1.0,
                                     True)
    PR = R.mean() / (R.mean() + T.mean())
    trans = np.all(L > 0, axis=1)
    # camera rays meet the coated face (the pane's normal faces the camera)
    assert np.allclose(L[trans], (Le * T / (1 - PR))[None, :], rtol=1e-12)
    assert trans.any()
