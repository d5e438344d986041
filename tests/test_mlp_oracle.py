"""Pins of the network reference (oracle/mlp.py) against facts that do not
come from its own formulas: the bit-level definition of bfloat16 rounding,
finite differences, Adam's first-step closed form, the published SplitMix64
outputs, and an FP32-accumulating re-implementation for the error bounds."""
from __future__ import annotations

import os

import numpy as np
import pytest

from oracle import mlp

HERE = os.path.dirname(os.path.abspath(__file__))


def bf16_bits_rne(x32: np.ndarray) -> np.ndarray:
    """Round FP32 values to bfloat16 on their bit patterns: add 0x7FFF plus the
    lowest kept bit, then clear the low 16 bits (round to nearest, ties to even)."""
    b = x32.astype(np.float32).view(np.uint32).astype(np.uint64)
    b = (b + 0x7FFF + ((b >> 16) & 1)) >> 16 << 16
    return b.astype(np.uint32).view(np.float32).astype(np.float64)


def test_bf16_matches_bit_rounding():
    rng = np.random.default_rng(1)
    x = rng.standard_normal(200_000).astype(np.float32) * np.exp2(rng.integers(-30, 30, 200_000))
    x = x.astype(np.float32)
    np.testing.assert_array_equal(mlp.bf16(x.astype(np.float64)), bf16_bits_rne(x))


def test_bf16_ties_to_even():
    one = 1.0
    assert mlp.bf16(one + 2.0 ** -8) == 1.0                   # halfway, 1.0 is even
    assert mlp.bf16(one + 3 * 2.0 ** -8) == 1.0 + 2.0 ** -6   # halfway, rounds up to even
    assert mlp.bf16(one + 2.0 ** -8 + 2.0 ** -30) == 1.0 + 2.0 ** -7
    assert mlp.bf16(-3.0) == -3.0 and mlp.bf16(0.0) == 0.0
    assert mlp.bf16_ulp(1.0) == 2.0 ** -7 and mlp.bf16_ulp(1.99) == 2.0 ** -7 and mlp.bf16_ulp(2.0) == 2.0 ** -6


def test_splitmix64_published_vector():
    with open(os.path.join(HERE, "golden", "splitmix64_seed0.txt")) as f:
        vals = [int(line.split()[1], 16) for line in f if line.strip() and not line.startswith("#")]
    assert [mlp.splitmix64(0, i) for i in range(len(vals))] == vals


def test_init_ranges():
    p = mlp.unflatten(mlp.init_params(7))
    assert np.all(np.abs(p["W1"]) <= np.sqrt(6 / 16)) and np.all(np.abs(p["W2"]) <= np.sqrt(6 / 64))
    assert np.all(np.abs(p["W3"]) <= np.sqrt(6 / 64))
    assert not p["b1"].any() and not p["b2"].any() and not p["b3"].any()
    # uniform on [-lim, lim]: mean ~ 0, variance lim^2/3
    w2 = p["W2"].ravel()
    assert abs(w2.mean()) < 0.02 and abs(w2.var() - (6 / 64) / 3) < 0.005
    assert np.all(np.float32(mlp.init_params(7)) == mlp.init_params(7))


def _batch(seed, B=24):
    rng = np.random.default_rng(seed)
    X = rng.uniform(-1, 1, (B, 16))
    t = rng.uniform(0, 1, B)
    flat = mlp.init_params(seed)
    flat[1024:1088] = rng.uniform(-0.1, 0.1, 64)   # nonzero biases so their gradients are exercised
    flat[5248:5312] = rng.uniform(-0.1, 0.1, 64)
    flat[5312] = 0.05
    return flat, X, t


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_gradient_finite_differences(seed):
    flat, X, t = _batch(seed)
    g, _ = mlp.backward(flat, X, t, emulate=False)
    rng = np.random.default_rng(100 + seed)
    idx = np.concatenate([rng.choice(np.arange(0, 1024), 30, replace=False),
                          rng.choice(np.arange(1024, 1088), 8, replace=False),
                          rng.choice(np.arange(1088, 5184), 30, replace=False),
                          rng.choice(np.arange(5184, 5248), 8, replace=False),
                          rng.choice(np.arange(5248, 5312), 8, replace=False), [5312]])
    h = 1e-6
    for p in idx:
        fp, fm = flat.copy(), flat.copy()
        fp[p] += h
        fm[p] -= h
        fd = (mlp.loss(fp, X, t) - mlp.loss(fm, X, t)) / (2 * h)
        assert abs(fd - g[p]) <= 1e-6 * max(1.0, abs(g[p])) + 1e-8, (p, fd, g[p])


def test_emulation_close_to_fp64():
    flat, X, t = _batch(3, B=64)
    ge, ye = mlp.backward(flat, X, t, emulate=True)
    gx, yx = mlp.backward(flat, X, t, emulate=False)
    assert np.max(np.abs(ye - yx)) < 0.05 * np.max(np.abs(yx)) + 1e-3
    assert np.linalg.norm(ge - gx) < 0.05 * np.linalg.norm(gx)


def _fp32_forward_backward(flat, X, t, order_seed):
    """Kernel stand-in: bfloat16 operands, FP32 sums accumulated in a random
    order (a different order for every output)."""
    rng = np.random.default_rng(order_seed)
    P = mlp.unflatten(flat)
    f32 = np.float32

    def acc(terms, bias=0.0):
        terms = np.asarray(terms, dtype=np.float64)
        s = f32(bias)
        for k in rng.permutation(terms.shape[0]):
            s = f32(s + f32(terms[k]))
        return float(s)

    B = X.shape[0]
    Xb = mlp.bf16(X)
    W1, W2, W3 = mlp.bf16(P["W1"]), mlp.bf16(P["W2"]), mlp.bf16(P["W3"])
    z1 = np.array([[acc(Xb[b] * W1[o], P["b1"][o]) for o in range(64)] for b in range(B)])
    h1 = mlp.bf16(np.maximum(z1, 0))
    z2 = np.array([[acc(h1[b] * W2[o], P["b2"][o]) for o in range(64)] for b in range(B)])
    h2 = mlp.bf16(np.maximum(z2, 0))
    y = np.array([acc(h2[b] * W3, P["b3"][0]) for b in range(B)])
    g3 = np.array([float(f32(f32(2.0 * f32(y[b] - t[b])) / f32(B))) for b in range(B)])
    dW3 = np.array([acc(g3 * h2[:, i]) for i in range(64)])
    db3 = np.array([acc(g3)])
    g2 = np.array([[float(f32(g3[b] * W3[o])) if z2[b, o] > 0 else 0.0 for o in range(64)] for b in range(B)])
    g2b = mlp.bf16(g2)
    dW2 = np.array([[acc(g2b[:, o] * h1[:, i]) for i in range(64)] for o in range(64)])
    db2 = np.array([acc(g2[:, o]) for o in range(64)])
    dh1 = np.array([[acc(g2b[b] * W2[:, i]) for i in range(64)] for b in range(B)])
    g1 = dh1 * (z1 > 0)
    g1b = mlp.bf16(g1)
    dW1 = np.array([[acc(g1b[:, o] * Xb[:, i]) for i in range(16)] for o in range(64)])
    db1 = np.array([acc(g1[:, o]) for o in range(64)])
    return y, mlp.flatten(dict(W1=dW1, b1=db1, W2=dW2, b2=db2, W3=dW3, b3=db3))


def tensor_rel_errors(g, ref):
    """Relative Frobenius error of each parameter tensor."""
    G, R = mlp.unflatten(g), mlp.unflatten(ref)
    return {k: float(np.linalg.norm(G[k] - R[k]) / max(np.linalg.norm(R[k]), 1e-30)) for k in R}


@pytest.mark.parametrize("seed,offset", [(0, 0.0), (1, 0.0), (2, 3.0)])
def test_bounds_cover_fp32_accumulation(seed, offset):
    flat, X, t = _batch(seed, B=12)
    X = X * 3.0
    t = t + offset
    y32, g32 = _fp32_forward_backward(flat, X, t, seed)
    ye, _ = mlp.forward(flat, X, True)
    ge, _ = mlp.backward(flat, X, t, True)
    ey, _ = mlp.forward_bound(flat, X)
    eg = mlp.backward_bound(flat, X, t)
    assert np.all(np.abs(y32 - ye) <= ey)
    assert np.all(np.abs(g32 - ge) <= eg)
    # the worst case assumes every hidden value rounds the other way; in
    # practice a few do, so whole tensors agree far more closely
    assert max(tensor_rel_errors(g32, ge).values()) < 2.0 ** -6
    assert np.linalg.norm(y32 - ye) < 2.0 ** -6 * np.linalg.norm(ye)
    # a planted mistake (dW2 transposed) breaks that criterion
    bad = g32.copy()
    bad[1088:5184] = g32[1088:5184].reshape(64, 64).T.ravel()
    assert tensor_rel_errors(bad, ge)["W2"] > 2.0 ** -6


def test_adam_first_step_closed_form():
    rng = np.random.default_rng(5)
    flat = rng.standard_normal(mlp.NPARAM)
    g = rng.standard_normal(mlp.NPARAM)
    z = np.zeros(mlp.NPARAM)
    new, m, v = mlp.adam_step(flat, z, z, g, 1, 1e-3)
    # bias-corrected moments equal g and g^2 after the first step
    np.testing.assert_allclose(new, flat - 1e-3 * g / (np.abs(g) + 1e-8), rtol=0, atol=1e-15)
    np.testing.assert_allclose(m, 0.1 * g)
    np.testing.assert_allclose(v, 0.001 * g * g)
