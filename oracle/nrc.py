"""FP64 reference of the learned radiance cache -- TEST INFRASTRUCTURE ONLY.

Only the test-suite, the smoke check and the benchmark's CPU-baseline leg use
this module; it shares no code with the HIP library.  Plain numpy, float64,
written from the definitions:

* multiresolution hash encoding of a position (Mueller, Evans, Schied,
  Keller, SIGGRAPH 2022): L levels of resolution N_l = floor(N_min b^l),
  b = exp((ln N_max - ln N_min) / (L - 1)); on each level the 8 lattice
  corners around the position are looked up (dense index when the level's
  (N_l + 1)^3 vertices fit the table, else the spatial hash
  (x * 1) xor (y * 2654435761) xor (z * 805459861) mod T on uint32) and
  blended trilinearly, F features per entry;
* real spherical harmonics of the direction, bands 0..3 (16 values),
  Y_l^m = K_l^m P_l^|m|(cos theta) * {sqrt2 cos(m phi), 1, sqrt2 sin(|m| phi)},
  K_l^m = sqrt((2l + 1) / (4 pi) (l - |m|)! / (l + |m|)!), P_l^m the
  associated Legendre functions without the Condon-Shortley phase;
* one-blob encoding of the wavelength: u = (lambda - lam_lo) / (lam_hi -
  lam_lo), 16 Gaussian bins exp(-(16 u - (i + 0.5))^2 / 2);
* a multilayer perceptron 64 -> 64 (ReLU) x 5 hidden layers -> 1 (linear)
  (also as BF16 matrix units evaluate it: every layer's operands rounded to
  bfloat16, round to nearest even),
  its backward pass, the relative L2 loss (y - t)^2 / (sg(y)^2 + 0.01) with
  the prediction's magnitude held constant (Mueller, Rousselle, Novak,
  Keller, SIGGRAPH 2021), and Adam (Kingma and Ba, ICLR 2015).
"""
from __future__ import annotations

import math

import numpy as np

L_LEVELS = 16
F_FEAT = 2
N_MIN = 16
N_MAX = 2048
N_SH = 16
N_BLOB = 16
N_IN = L_LEVELS * F_FEAT + N_SH + N_BLOB  # 64
N_HID = 64
N_LAYERS = 5          # hidden layers
PRIMES = (1, 2654435761, 805459861)


def level_resolution(l, levels=L_LEVELS, n_min=N_MIN, n_max=N_MAX):
    b = math.exp((math.log(n_max) - math.log(n_min)) / (levels - 1))
    return int(math.floor(n_min * b ** l))


def corner_index(c, N, T):
    """Table index of integer lattice corners c [n, 3] on a level of resolution N."""
    c = np.asarray(c, dtype=np.int64)
    if (N + 1) ** 3 <= T:
        return c[:, 0] + c[:, 1] * (N + 1) + c[:, 2] * (N + 1) ** 2
    h = np.zeros(len(c), dtype=np.uint64)
    for a in range(3):
        h ^= (c[:, a].astype(np.uint64) * np.uint64(PRIMES[a])) & np.uint64(0xFFFFFFFF)
    return (h % np.uint64(T)).astype(np.int64)


def hash_encode(xn, tables, levels=L_LEVELS):
    """xn [n, 3] positions normalised to [0, 1]; tables [L, T, F]."""
    xn = np.asarray(xn, dtype=np.float64)
    T = tables.shape[1]
    out = np.zeros((len(xn), levels * tables.shape[2]))
    for l in range(levels):
        N = level_resolution(l, levels)
        p = xn * N
        i0 = np.clip(np.floor(p), 0, N - 1).astype(np.int64)
        f = p - i0
        acc = np.zeros((len(xn), tables.shape[2]))
        for dz in (0, 1):
            for dy in (0, 1):
                for dx in (0, 1):
                    d = np.array([dx, dy, dz])
                    w = np.prod(np.where(d == 1, f, 1.0 - f), axis=1)
                    idx = corner_index(i0 + d, N, T)
                    acc += w[:, None] * tables[l, idx, :]
        out[:, l * tables.shape[2]:(l + 1) * tables.shape[2]] = acc
    return out


def _assoc_legendre(l, m, x):
    """P_l^m(x), m >= 0, without the Condon-Shortley phase (recurrences in l)."""
    pmm = np.ones_like(x)
    if m > 0:
        s = np.sqrt(np.maximum(0.0, 1.0 - x * x))
        fact = 1.0
        for _ in range(m):
            pmm = pmm * fact * s
            fact += 2.0
    if l == m:
        return pmm
    pmmp1 = x * (2 * m + 1) * pmm
    if l == m + 1:
        return pmmp1
    pll = None
    for ll in range(m + 2, l + 1):
        pll = ((2 * ll - 1) * x * pmmp1 - (ll + m - 1) * pmm) / (ll - m)
        pmm, pmmp1 = pmmp1, pll
    return pll


def sh_encode(w):
    """Real spherical harmonics of unit directions w [n, 3], bands 0..3, ordered
    (l, m) = (0,0), (1,-1), (1,0), (1,1), (2,-2), ..., (3,3)."""
    w = np.asarray(w, dtype=np.float64)
    ct = w[:, 2]
    phi = np.arctan2(w[:, 1], w[:, 0])
    out = []
    for l in range(4):
        for m in range(-l, l + 1):
            am = abs(m)
            K = math.sqrt((2 * l + 1) / (4 * math.pi) * math.factorial(l - am) / math.factorial(l + am))
            P = _assoc_legendre(l, am, ct)
            if m > 0:
                out.append(math.sqrt(2.0) * K * np.cos(m * phi) * P)
            elif m < 0:
                out.append(math.sqrt(2.0) * K * np.sin(am * phi) * P)
            else:
                out.append(K * P)
    return np.stack(out, axis=1)


def blob_encode(lam_nm, lam_lo=380.0, lam_hi=780.0, bins=N_BLOB):
    u = (np.asarray(lam_nm, dtype=np.float64) - lam_lo) / (lam_hi - lam_lo)
    c = np.arange(bins) + 0.5
    return np.exp(-0.5 * (u[:, None] * bins - c[None, :]) ** 2)


def encode(x, w, lam_nm, aabb_lo, aabb_hi, tables):
    """Network input [n, 64] of positions x (metres), unit directions w and wavelengths."""
    xn = (np.asarray(x, np.float64) - np.asarray(aabb_lo, np.float64)) / (
        np.asarray(aabb_hi, np.float64) - np.asarray(aabb_lo, np.float64))
    return np.concatenate([hash_encode(np.clip(xn, 0.0, 1.0), tables), sh_encode(w), blob_encode(lam_nm)], axis=1)


def mlp_forward(params, X):
    """params: dict W[k] [64, 64] (out, in), b[k] [64] for k = 0..4, wo [64], bo (scalar).
    Returns (y [n], activations list) with activations[0] = X."""
    acts = [np.asarray(X, np.float64)]
    h = acts[0]
    for k in range(N_LAYERS):
        h = np.maximum(0.0, h @ params["W"][k].T + params["b"][k])
        acts.append(h)
    y = h @ params["wo"] + params["bo"]
    return y, acts


def bf16_round(a):
    """Nearest bfloat16 (ties to even) of each value taken as float32: the
    float32 bit pattern rounded at bit 16 (IEEE round-to-nearest-even)."""
    f = np.ascontiguousarray(np.asarray(a, np.float64).astype(np.float32))
    u = f.view(np.uint32).astype(np.uint64)
    u = (u + np.uint64(0x7FFF) + ((u >> np.uint64(16)) & np.uint64(1))) & np.uint64(0xFFFF0000)
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def mlp_forward_bf16(params, X):
    """The forward pass as BF16 matrix units evaluate it: every layer's
    operands (inputs and weights, the output layer's included) rounded to
    bfloat16, products summed exactly (here in float64) onto the bias, ReLU
    between layers."""
    h = np.asarray(X, np.float64)
    for k in range(N_LAYERS):
        h = np.maximum(0.0, bf16_round(h) @ bf16_round(params["W"][k]).T + params["b"][k])
    return bf16_round(h) @ bf16_round(params["wo"]) + params["bo"]


# ---------------------------------------------------------------------------
# error bound of the network evaluated with BF16 operands
# ---------------------------------------------------------------------------
U_BF16 = 2.0 ** -8    # unit roundoff of bfloat16 (8 significand bits): |bf(x) - x| <= u |x|
U_FP32 = 2.0 ** -24   # unit roundoff of float32


def gamma(m, u=U_FP32):
    """Higham's gamma_m = m u / (1 - m u): bound on the relative error of a sum
    of m + 1 terms accumulated with m roundings of unit roundoff u."""
    return m * u / (1.0 - m * u)


def encode_error_bound(x, aabb_lo, aabb_hi, tables, n_sh_abs=4e-6, n_blob_abs=4e-6, table_u=0.0):
    """Bound on |X_fp32 - X| for the network input as an FP32 kernel encodes it.

    * position: xn = (x - lo) * (1 / (hi - lo)) in FP32 carries at most three
      roundings (|d xn| <= 3 * 2^-24 <= 2^-22 after clamping to [0, 1]); the
      lattice coordinate p = xn N then moves by at most N 2^-21.  The
      trilinear interpolant is continuous across cells and its derivative
      along an axis is a difference of two bilinear interpolants, at most
      2 max|t_l| in magnitude, so a level's features move by at most
      3 * N 2^-21 * 2 max|t_l|, plus the FP32 sum of 8 weighted corners,
      gamma_11 max|t_l|;
    * harmonics and one-blob bins: FP32 evaluation of bounded polynomials and
      of exp(-d^2 / 2) (derivative at most 0.61), a few ulp of terms below 3:
      n_sh_abs and n_blob_abs absolute;
    * table_u > 0: the kernel reads the table entries rounded to a format of
      unit roundoff table_u (FP16: 2^-11); each corner value moves by at most
      table_u |t|, so the interpolant (weights summing to 1) by at most
      table_u max|t_l|.
    """
    n = len(np.asarray(x))
    E = np.zeros((n, N_IN))
    F = tables.shape[2]
    for l in range(L_LEVELS):
        N = level_resolution(l)
        tmax = float(np.max(np.abs(tables[l])))
        E[:, l * F:(l + 1) * F] = 3.0 * N * 2.0 ** -21 * 2.0 * tmax + gamma(11) * tmax + table_u * tmax
    E[:, L_LEVELS * F:L_LEVELS * F + N_SH] = n_sh_abs
    E[:, L_LEVELS * F + N_SH:] = n_blob_abs
    return E


def mlp_bf16_error_bound(params, X, EX, u=U_BF16, lam=6.0):
    """FP64 output y of the network and a bound B on |y_hat - y| for an
    evaluation y_hat with BF16 operands in every layer (inputs, activations,
    weights, the output layer's included), FP32 accumulation and FP32 biases,
    from an FP32 input X_hat with |X_hat - X| <= EX.

    Error model (probabilistic rounding error analysis, Higham and Mary, SIAM
    J. Sci. Comput. 2019): every BF16 rounding is bf(v) = v (1 + d), |d| <= u,
    the d independent with mean zero.  To first order the output error is
    linear in them,
      dy = sum over layers k, inputs m:  (dy/da_{k-1,m}) a_{k-1,m} phi_{k,m}
         + sum over weights (i, m):      (dy/dz_{k,i}) W_k,im a_{k-1,m} theta_{k,im},
    phi the rounding of layer k's input operand, theta of its weight (layer 5 =
    the output layer, dy/dz = 1), the sensitivities dy/dz, dy/da signed
    (backpropagation of 1 through the exact ReLU masks).  By Hoeffding's
    inequality |dy| <= lam u sqrt(V) with probability at least
    1 - 2 exp(-lam^2 / 2) (3e-8 for lam = 6), V the sum of the squared
    coefficients: the layer sums of squares sum_m (dy/da_m a_m)^2 and
    sum_i (dy/dz_i)^2 sum_m (W_im a_m)^2.  Added in the worst case:
      * products' second-order term theta phi: u^2 sum |dy/dz| |W| |a|;
      * FP32 accumulation: gamma_66 (layer 0 in two partial sums) or gamma_65
        of sum |dy/dz| ((1 + u)^2 |W| |a| + |b|);
      * the input's encoding error: sum_m |dy/dX_m| EX_m;
      * ReLU kinks: a unit whose |z| lies within its own error bound e (the
        same model, carried to the unit through the signed maps between
        layers) may take the other branch; its activation then differs from
        the linear model's by |z + dz| <= e - |z|, which moves the output by
        at most |dy/da| (e - |z|).
    Returns (y, B, n_kink_units [n], u sqrt(V) [n]); under the model the error
    has standard deviation at most u sqrt(V / 3) (a rounding error uniform on
    [-u, u] has variance u^2 / 3)."""
    X = np.asarray(X, np.float64)
    n = len(X)
    Ws = [np.asarray(w, np.float64) for w in params["W"]] + [np.asarray(params["wo"], np.float64)[None, :]]
    bs = [np.asarray(b, np.float64) for b in params["b"]] + [np.array([float(params["bo"])])]
    nl = N_LAYERS + 1
    a, z = [X], []
    for k in range(nl):
        zk = a[-1] @ Ws[k].T + bs[k]
        z.append(zk)
        a.append(np.maximum(0.0, zk) if k < N_LAYERS else zk)
    y = z[-1][:, 0]
    masks = [(zk > 0.0).astype(np.float64) for zk in z[:N_LAYERS]] + [np.ones((n, 1))]
    # sensitivities: g[k] = dy/dz_k, da[k] = dy/d(input of layer k)
    g = [None] * nl
    da = [None] * nl
    g[nl - 1] = np.ones((n, 1))
    for k in range(nl - 1, -1, -1):
        da[k] = g[k] @ Ws[k]
        if k > 0:
            g[k - 1] = da[k] * masks[k - 1]
    # squared coefficients of the roundings, per layer: q[k][i] = sum_m (W_im a_m)^2
    q = [(a[k] ** 2) @ (Ws[k] ** 2).T for k in range(nl)]
    V = np.zeros(n)
    worst = np.zeros(n)
    for k in range(nl):
        V += np.sum((da[k] * a[k]) ** 2, axis=1) + np.sum(g[k] ** 2 * q[k], axis=1)
        S = np.abs(a[k]) @ np.abs(Ws[k]).T
        m = 66 if k == 0 else 65
        worst += np.sum(np.abs(g[k]) * (u * u * S + gamma(m) * ((1.0 + u) ** 2 * S + np.abs(bs[k]))), axis=1)
    EXa = np.abs(np.asarray(EX, np.float64) * np.ones_like(X))
    worst += np.sum(np.abs(da[0]) * EXa, axis=1)
    B = lam * u * np.sqrt(V) + worst
    # per-unit bounds of the hidden layers, through the signed maps P[j] (layer j -> current)
    nk = np.zeros(n, np.int64)
    P = []
    Vu = []
    for k in range(N_LAYERS):
        if k > 0:
            P = [np.matmul(Ws[k][None], masks[k - 1][:, :, None] * Pj) for Pj in P]
        P.append(np.broadcast_to(np.eye(N_HID), (n, N_HID, N_HID)))
        var = np.zeros((n, N_HID))
        wst = np.zeros((n, N_HID))
        for j, Pj in enumerate(P):
            PW = np.matmul(Pj, np.broadcast_to(Ws[j], (n,) + Ws[j].shape))
            var += np.einsum("nim,nm->ni", PW ** 2, a[j] ** 2) + np.einsum("nij,nj->ni", Pj ** 2, q[j])
            S = np.abs(a[j]) @ np.abs(Ws[j]).T
            loc = u * u * S + gamma(66 if j == 0 else 65) * ((1.0 + u) ** 2 * S + np.abs(bs[j]))
            if j == 0:
                loc = loc + EXa @ np.abs(Ws[0]).T
            wst += np.einsum("nij,nj->ni", np.abs(Pj), loc)
        e = lam * u * np.sqrt(var) + wst
        over = e - np.abs(z[k])          # how far the error bound reaches past the kink
        near = over > 0.0
        B = B + np.sum(np.where(near, np.abs(da[k + 1]) * over, 0.0), axis=1)
        nk += near.sum(axis=1)
    return y, B, nk, u * np.sqrt(V)


def rel_l2_loss(y, t, eps=0.01):
    """Mean of (y - t)^2 / (sg(y)^2 + eps) and its gradient with respect to y."""
    den = y * y + eps
    loss = np.mean((y - t) ** 2 / den)
    dy = 2.0 * (y - t) / den / len(y)
    return loss, dy


def mlp_backward(params, acts, dy):
    """Gradients of a scalar loss with respect to params and to the input, given dL/dy."""
    g = {"W": [None] * N_LAYERS, "b": [None] * N_LAYERS}
    h = acts[-1]
    g["wo"] = h.T @ dy
    g["bo"] = float(np.sum(dy))
    dh = np.outer(dy, params["wo"])
    for k in range(N_LAYERS - 1, -1, -1):
        dz = dh * (acts[k + 1] > 0.0)
        g["W"][k] = dz.T @ acts[k]
        g["b"][k] = np.sum(dz, axis=0)
        dh = dz @ params["W"][k]
    return g, dh


def hash_backward(xn, dfeat, shape, levels=L_LEVELS):
    """Gradient of the tables [L, T, F] given dL/d(hash features) [n, L * F]."""
    xn = np.asarray(xn, dtype=np.float64)
    gt = np.zeros(shape)
    T, F = shape[1], shape[2]
    for l in range(levels):
        N = level_resolution(l, levels)
        p = xn * N
        i0 = np.clip(np.floor(p), 0, N - 1).astype(np.int64)
        f = p - i0
        for dz in (0, 1):
            for dy in (0, 1):
                for dx in (0, 1):
                    d = np.array([dx, dy, dz])
                    w = np.prod(np.where(d == 1, f, 1.0 - f), axis=1)
                    idx = corner_index(i0 + d, N, T)
                    np.add.at(gt[l], idx, w[:, None] * dfeat[:, l * F:(l + 1) * F])
    return gt


class Adam:
    """Kingma and Ba (2015): m = b1 m + (1 - b1) g, v = b2 v + (1 - b2) g^2,
    p -= lr * (m / (1 - b1^t)) / (sqrt(v / (1 - b2^t)) + eps)."""

    def __init__(self, lr=1e-2, b1=0.9, b2=0.99, eps=1e-8):
        self.lr, self.b1, self.b2, self.eps = lr, b1, b2, eps
        self.t = 0
        self.m = {}
        self.v = {}

    def step(self, name, p, g):
        if name not in self.m:
            self.m[name] = np.zeros_like(p)
            self.v[name] = np.zeros_like(p)
        m = self.m[name] = self.b1 * self.m[name] + (1 - self.b1) * g
        v = self.v[name] = self.b2 * self.v[name] + (1 - self.b2) * g * g
        mh = m / (1 - self.b1 ** self.t)
        vh = v / (1 - self.b2 ** self.t)
        return p - self.lr * mh / (np.sqrt(vh) + self.eps)


def train_step(params, tables, opt, x, w, lam_nm, target, aabb_lo, aabb_hi):
    """One optimisation step on a batch of rows; returns (loss, new params, new tables)."""
    xn = np.clip((np.asarray(x, np.float64) - np.asarray(aabb_lo)) / (np.asarray(aabb_hi) - np.asarray(aabb_lo)),
                 0.0, 1.0)
    X = encode(x, w, lam_nm, aabb_lo, aabb_hi, tables)
    y, acts = mlp_forward(params, X)
    loss, dy = rel_l2_loss(y, np.asarray(target, np.float64))
    g, dX = mlp_backward(params, acts, dy)
    gt = hash_backward(xn, dX[:, :L_LEVELS * F_FEAT], tables.shape)
    opt.t += 1
    newp = {"W": [opt.step(f"W{k}", params["W"][k], g["W"][k]) for k in range(N_LAYERS)],
            "b": [opt.step(f"b{k}", params["b"][k], g["b"][k]) for k in range(N_LAYERS)],
            "wo": opt.step("wo", params["wo"], g["wo"]),
            "bo": float(opt.step("bo", np.array(params["bo"]), np.array(g["bo"])))}
    newt = opt.step("tables", tables, gt)
    return loss, newp, newt
