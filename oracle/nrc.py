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
