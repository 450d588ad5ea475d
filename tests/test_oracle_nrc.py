"""Pins of the FP64 radiance-cache reference (oracle/nrc.py): closed forms,
orthonormality, exact reproduction of affine fields, finite differences."""
import math

import numpy as np
import pytest

import scenegen as sg
from oracle import nrc


def test_sh_orthonormal():
    # Gauss-Legendre in cos(theta) x uniform phi integrates degree <= 6 products exactly
    xg, wg = np.polynomial.legendre.leggauss(24)
    phi = (np.arange(48) + 0.5) * 2 * np.pi / 48
    ct, ph = np.meshgrid(xg, phi, indexing="ij")
    st = np.sqrt(1 - ct ** 2)
    w = np.stack([st * np.cos(ph), st * np.sin(ph), ct], axis=-1).reshape(-1, 3)
    wt = (wg[:, None] * np.full(len(phi), 2 * np.pi / 48)[None, :]).reshape(-1)
    Y = nrc.sh_encode(w)
    G = (Y * wt[:, None]).T @ Y
    assert np.abs(G - np.eye(16)).max() < 1e-12


def test_sh_low_bands_closed_form():
    w = np.array([[0.6, 0.0, 0.8], [0.0, -1.0, 0.0], [0.36, 0.48, 0.8]])
    Y = nrc.sh_encode(w)
    c0, c1 = 0.5 / math.sqrt(math.pi), math.sqrt(3 / (4 * math.pi))
    assert np.allclose(Y[:, 0], c0, rtol=1e-14)
    assert np.allclose(Y[:, 1], c1 * w[:, 1], rtol=1e-13, atol=1e-15)  # (1,-1) ~ y
    assert np.allclose(Y[:, 2], c1 * w[:, 2], rtol=1e-13, atol=1e-15)  # (1, 0) ~ z
    assert np.allclose(Y[:, 3], c1 * w[:, 0], rtol=1e-13, atol=1e-15)  # (1, 1) ~ x
    # (2, 0) = sqrt(5 / 16 pi) (3 z^2 - 1)
    assert np.allclose(Y[:, 6], math.sqrt(5 / (16 * math.pi)) * (3 * w[:, 2] ** 2 - 1), rtol=1e-13, atol=1e-15)


def test_level_resolutions():
    r = [nrc.level_resolution(l) for l in range(16)]
    assert r[0] == 16 and r[-1] in (2047, 2048)
    assert all(b > a for a, b in zip(r, r[1:]))


def test_corner_index_dense_and_hashed():
    T = 1 << 19
    # a dense level is a bijection of its (N + 1)^3 lattice onto [0, (N+1)^3)
    N = 16
    g = np.stack(np.meshgrid(*[np.arange(N + 1)] * 3, indexing="ij"), -1).reshape(-1, 3)
    idx = nrc.corner_index(g, N, T)
    assert len(np.unique(idx)) == (N + 1) ** 3 and idx.max() == (N + 1) ** 3 - 1
    # a hashed level: uint32 products of the three primes, xor, modulo T
    N = 1000
    c = np.array([[1, 2, 3], [7, 0, 999]])
    expect = [(1 ^ ((2 * 2654435761) % 2 ** 32) ^ ((3 * 805459861) % 2 ** 32)) % T,
              (7 ^ 0 ^ ((999 * 805459861) % 2 ** 32)) % T]
    assert list(nrc.corner_index(c, N, T)) == expect


def test_hash_encode_reproduces_affine_fields_on_dense_levels():
    # tables holding an affine function of the lattice corner are interpolated exactly
    T, F = 1 << 16, 2
    tables = np.zeros((16, T, F))
    a = np.array([0.3, -1.2, 0.7])
    dense = [l for l in range(16) if (nrc.level_resolution(l) + 1) ** 3 <= T]
    assert dense == [0, 1, 2]
    for l in dense:
        N = nrc.level_resolution(l)
        g = np.stack(np.meshgrid(*[np.arange(N + 1)] * 3, indexing="ij"), -1).reshape(-1, 3)
        idx = nrc.corner_index(g, N, T)
        tables[l, idx, 0] = g @ a / N + 0.25
        tables[l, idx, 1] = g[:, 2] / N
    rng = np.random.default_rng(0)
    xn = rng.uniform(0, 1, size=(200, 3))
    f = nrc.hash_encode(xn, tables)
    for l in dense:
        assert np.allclose(f[:, 2 * l], xn @ a + 0.25, atol=1e-12)
        assert np.allclose(f[:, 2 * l + 1], xn[:, 2], atol=1e-12)


def test_one_blob():
    lam = np.array([381.0, 590.0, 701.0])
    B = nrc.blob_encode(lam)
    u = (lam - 380) / 400 * 16
    assert np.array_equal(np.argmax(B, axis=1), np.clip(np.floor(u), 0, 15).astype(int))
    # an interior blob sums to ~sqrt(2 pi) (sampled unit Gaussian)
    assert abs(B[1].sum() - math.sqrt(2 * math.pi)) < 1e-6


def _small_net(seed=1):
    params, tables = sg.nrc_params(seed, table_size=1 << 12)
    p = {"W": [w.astype(np.float64) for w in params["W"]], "b": [np.asarray(b, np.float64) + 0.01 for b in params["b"]],
         "wo": params["wo"].astype(np.float64), "bo": 0.1}
    return p, tables.astype(np.float64) * 1e3


def test_mlp_backward_matches_finite_differences():
    p, tables = _small_net()
    x, w, lam, t = sg.nrc_rows(16, 3)
    X = nrc.encode(x, w, lam, (0, 0, 0), (4, 3, 2.5), tables)

    def loss_of(pp, XX):
        y, _ = nrc.mlp_forward(pp, XX)
        return np.mean((y - t) ** 2)

    y, acts = nrc.mlp_forward(p, X)
    dy = 2 * (y - t) / len(y)
    g, dX = nrc.mlp_backward(p, acts, dy)
    h = 1e-6
    for k, (i, j) in ((0, (3, 5)), (2, (10, 60)), (4, (63, 0))):
        q = {"W": [w.copy() for w in p["W"]], "b": list(p["b"]), "wo": p["wo"], "bo": p["bo"]}
        q["W"][k][i, j] += h
        up = loss_of(q, X)
        q["W"][k][i, j] -= 2 * h
        dn = loss_of(q, X)
        assert g["W"][k][i, j] == pytest.approx((up - dn) / (2 * h), rel=1e-5, abs=1e-9)
    Xp = X.copy()
    Xp[2, 7] += h
    up = loss_of(p, Xp)
    Xp[2, 7] -= 2 * h
    dn = loss_of(p, Xp)
    assert dX[2, 7] == pytest.approx((up - dn) / (2 * h), rel=1e-5, abs=1e-9)


def test_hash_backward_matches_finite_differences():
    _, tables = _small_net()
    rng = np.random.default_rng(4)
    xn = rng.uniform(0, 1, size=(8, 3))
    dfeat = rng.normal(size=(8, 32))
    gt = nrc.hash_backward(xn, dfeat, tables.shape)
    f0 = nrc.hash_encode(xn, tables)
    # the loss sum(dfeat * features) is linear in the tables: its gradient is exact
    for (l, i, c) in ((0, 5, 0), (7, 100, 1), (15, 4000, 0)):
        t2 = tables.copy()
        t2[l, i, c] += 1.0
        f1 = nrc.hash_encode(xn, t2)
        assert np.sum(dfeat * (f1 - f0)) == pytest.approx(gt[l, i, c], rel=1e-12, abs=1e-14)


def test_rel_l2_gradient_holds_the_denominator():
    y = np.array([0.5, 2.0, -0.1])
    t = np.array([1.0, 1.5, 0.0])
    _, dy = nrc.rel_l2_loss(y, t)
    assert np.allclose(dy, 2 * (y - t) / (y * y + 0.01) / 3)


def test_adam_first_step_is_signed_learning_rate():
    opt = nrc.Adam(lr=1e-2)
    opt.t = 1
    p = np.array([1.0, -2.0, 0.5])
    g = np.array([0.3, -4.0, 1e-3])
    q = opt.step("p", p, g)
    assert np.allclose(q, p - 1e-2 * g / (np.abs(g) + 1e-8), rtol=1e-12)


def test_train_step_reduces_the_loss():
    p, tables = _small_net(2)
    tables = tables * 1e-3
    x, w, lam, t = sg.nrc_rows(256, 5)
    opt = nrc.Adam(lr=1e-3)
    losses = []
    for _ in range(30):
        loss, p, tables = nrc.train_step(p, tables, opt, x, w, lam, t, (0, 0, 0), (4, 3, 2.5))
        losses.append(loss)
    assert losses[-1] < 0.5 * losses[0]


def test_bf16_round_ties_to_even_and_matches_torch():
    u = 2.0 ** -8  # half an ulp of bfloat16 at 1
    got = nrc.bf16_round(np.array([1.0, 1.0 + u, 1.0 + 3 * u, 1.0 + u + 2.0 ** -20, -(1.0 + 3 * u), 0.0]))
    assert got.tolist() == [1.0, 1.0, 1.0 + 4 * u, 1.0 + 2 * u, -(1.0 + 4 * u), 0.0]
    import torch
    x = np.random.default_rng(3).normal(size=4096) * np.exp(np.random.default_rng(4).uniform(-20, 20, 4096))
    ref = torch.tensor(x, dtype=torch.float32).to(torch.bfloat16).to(torch.float64).numpy()
    assert np.array_equal(nrc.bf16_round(x), ref)


def test_bf16_forward_is_exact_on_bf16_operands():
    rng = np.random.default_rng(5)
    # operands with at most 8 significant bits are bfloat16 values: nothing rounds
    params = {"W": [rng.integers(-8, 9, (64, 64)) / 16.0] + [np.zeros((64, 64)) for _ in range(4)],
              "b": [rng.integers(-4, 5, 64) / 8.0 for _ in range(5)],
              "wo": rng.integers(-16, 17, 64) / 32.0, "bo": 0.25}
    X = rng.integers(-64, 65, (50, 64)) / 32.0
    y, _ = nrc.mlp_forward(params, X)
    assert np.array_equal(nrc.mlp_forward_bf16(params, X), y)
    # with W_1 = I the second layer consumes the first layer's outputs, which need
    # more than 8 bits: the result is relu(bf16(h1) + b1) passed on exactly
    params["W"][1] = np.eye(64)
    _, acts = nrc.mlp_forward(params, X)
    assert not np.array_equal(nrc.bf16_round(acts[1]), acts[1])
    h = np.maximum(0.0, nrc.bf16_round(acts[1]) + params["b"][1])
    for k in range(2, 5):
        h = np.maximum(0.0, 0.0 * h + params["b"][k])
    assert np.allclose(nrc.mlp_forward_bf16(params, X), h @ params["wo"] + params["bo"], rtol=0, atol=1e-12)


# ---------------------------------------------------------------------------
# the BF16 error bound the GPU network is judged by (FP64 forward +- bound)
# ---------------------------------------------------------------------------
LO3, HI3 = (0.0, 0.0, 0.0), (4.0, 3.0, 2.5)


def _test_net(seed, log2=12, table_scale=0.5):
    params, tables = sg.nrc_params(seed, table_size=1 << log2)
    rng = np.random.default_rng(seed + 1000)
    tables = rng.uniform(-table_scale, table_scale, tables.shape)
    p = {"W": [np.asarray(w, np.float64) for w in params["W"]],
         "b": [rng.uniform(-0.1, 0.1, 64) for _ in range(5)],
         "wo": np.asarray(params["wo"], np.float64), "bo": 0.05}
    return p, tables


def _torch_bf16_forward(p, X):
    """An evaluation independent of this module: torch rounds every operand to
    bfloat16 and multiplies in float32 (its own accumulation order)."""
    import torch

    def bf(a):
        return torch.tensor(np.asarray(a, np.float32)).to(torch.bfloat16).to(torch.float32)

    h = torch.tensor(np.asarray(X, np.float32))
    for k in range(5):
        h = torch.relu(bf(h) @ bf(p["W"][k]).T + torch.tensor(np.asarray(p["b"][k], np.float32)))
    return (bf(h) @ bf(p["wo"]) + np.float32(p["bo"])).double().numpy()


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_bf16_bound_holds_and_is_informative(seed):
    p, tables = _test_net(seed)
    x, w, lam, _ = sg.nrc_rows(2000, seed)
    X = nrc.encode(x, w, lam, LO3, HI3, tables)
    X32 = X.astype(np.float32).astype(np.float64)          # the kernel's input is FP32
    y, B, nk, s = nrc.mlp_bf16_error_bound(p, X, np.abs(X32 - X))
    scale = np.abs(y) + np.sqrt(np.mean(y ** 2))
    for name, yb in (("torch", _torch_bf16_forward(p, X32)), ("emulation", nrc.mlp_forward_bf16(p, X32))):
        err = np.abs(yb - y)
        assert np.all(err <= B), (name, float(np.max(err / B)))
        # the error model's scale: uniform roundings of +-u give a standard
        # deviation of at most u sqrt(V / 3); a wrong u (2x) moves this ratio out
        r = float(np.sqrt(np.mean((err / (s / np.sqrt(3.0))) ** 2)))
        assert 0.4 <= r <= 1.2, (name, r)
        # and the bound is not inflated: the worst row reaches a tenth of it
        assert float(np.max(err / B)) >= 0.05, name
    assert float(np.median(B / scale)) <= 0.25
    assert nk.max() < 64                                   # few ReLU decisions are in doubt


def test_bf16_bound_catches_a_wrong_operand():
    """A layout slip (one input feature fed to the wrong slot) breaks the bound."""
    p, tables = _test_net(4)
    x, w, lam, _ = sg.nrc_rows(500, 4)
    X = nrc.encode(x, w, lam, LO3, HI3, tables)
    y, B, _, _ = nrc.mlp_bf16_error_bound(p, X, np.zeros_like(X))
    Xs = X.copy()
    Xs[:, [3, 40]] = Xs[:, [40, 3]]                         # one pair of slots exchanged
    assert np.mean(np.abs(_torch_bf16_forward(p, Xs) - y) > B) > 0.1
    Xs = X.copy()
    Xs[:, 32:48] = np.roll(Xs[:, 32:48], 4, axis=1)         # a lane group's slots rotated
    assert np.mean(np.abs(_torch_bf16_forward(p, Xs) - y) > B) > 0.5


def test_bf16_bound_encoding_term():
    """The encoding allowance covers FP32 lattice coordinates of general
    positions: features recomputed from positions rounded to FP32 relative
    steps stay within it."""
    p, tables = _test_net(5)
    x, w, lam, _ = sg.nrc_rows(400, 5)
    X = nrc.encode(x, w, lam, LO3, HI3, tables)
    EX = nrc.encode_error_bound(x, LO3, HI3, tables)
    xp = np.asarray(x, np.float64) * (1.0 + 3.0 * 2.0 ** -24)
    Xp = nrc.encode(xp, w, lam, LO3, HI3, tables)
    assert np.all(np.abs(Xp - X)[:, :32] <= EX[:, :32])


def test_bf16_bound_fp16_table_term():
    """The table term covers tables read in FP16: features encoded from the
    FP16 rounding of the tables stay within table_u = 2^-11 of max |t| per
    level, and that term is needed (without it the bound fails)."""
    p, tables = _test_net(6)
    x, w, lam, _ = sg.nrc_rows(2000, 6)
    X = nrc.encode(x, w, lam, LO3, HI3, tables)
    t16 = tables.astype(np.float16).astype(np.float64)
    X16 = nrc.encode(x, w, lam, LO3, HI3, t16)
    d = np.abs(X16 - X)[:, :32]
    E16 = nrc.encode_error_bound(x, LO3, HI3, tables, table_u=2.0 ** -11)
    E0 = nrc.encode_error_bound(x, LO3, HI3, tables)
    assert np.all(d <= E16[:, :32] - E0[:, :32])   # the table term alone covers it
    assert np.any(d > E0[:, :32])                  # and the FP32 terms do not
