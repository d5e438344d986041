"""Proposal network on the GPU (matrix-core forward, backward and Adam) against
the CPU reference in oracle/mlp.py.

Inputs are seeded synthetic feature rows of bfloat16 values. The criteria are
the rigorous per-element bounds of oracle.mlp (FP32 accumulation order and
bfloat16 re-rounding of hidden values) and, per parameter tensor, a relative
Frobenius error below 2^-6, which a wrong index or transposition exceeds."""
from __future__ import annotations

import numpy as np
import pytest

from oracle import mlp
import helpers

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

NP = mlp.NPARAM


def bf16_bits(x):
    """bfloat16 bit patterns (int16) of values already representable in bfloat16."""
    x32 = np.asarray(x, dtype=np.float32)
    assert np.array_equal(mlp.bf16(x32.astype(np.float64)), x32.astype(np.float64))
    return (x32.view(np.uint32) >> 16).astype(np.uint16).view(np.int16)


def features(n, seed, scale=1.0):
    rng = np.random.default_rng(seed)
    X = rng.uniform(-1.0, 1.0, (n, 16)) * scale
    X[:, 5:8] = rng.integers(0, 2, (n, 3))   # indicator-like inputs as in the proposal features
    return mlp.bf16(X)


def params(seed):
    rng = np.random.default_rng(1000 + seed)
    flat = mlp.init_params(seed)
    flat[mlp.NPARAM - 1] = 0.03
    flat[1024:1088] = rng.uniform(-0.2, 0.2, 64)
    flat[5184:5248] = rng.uniform(-0.2, 0.2, 64)
    return flat.astype(np.float32).astype(np.float64)


def model_with(flat):
    import paper_2605_05086_amd as chap
    M = chap.Model(0)
    M.set_params(flat.astype(np.float32))
    return M


def dev(a, dtype):
    return torch.from_numpy(np.ascontiguousarray(a)).to(device="cuda", dtype=dtype)


def rel_errors(g, ref):
    G, R = mlp.unflatten(g), mlp.unflatten(ref)
    return {k: float(np.linalg.norm(G[k] - R[k]) / max(np.linalg.norm(R[k]), 1e-30)) for k in R}


def test_init_matches_reference():
    import paper_2605_05086_amd as chap
    for seed in (0, 7, 123456789):
        M = chap.Model(seed)
        np.testing.assert_array_equal(M.get_params().astype(np.float64), mlp.init_params(seed))


@pytest.mark.parametrize("n,seed,scale", [(1, 0, 1.0), (17, 1, 1.0), (1000, 2, 1.0), (4099, 3, 4.0),
                                          (100_003, 4, 1.0)])
def test_forward_parity(n, seed, scale):
    flat = params(seed)
    X = features(n, seed, scale)
    M = model_with(flat)
    y = M.forward(dev(bf16_bits(X), torch.int16)).cpu().numpy().astype(np.float64)
    torch.cuda.synchronize()
    ye, _ = mlp.forward(flat, X, True)
    ey, _ = mlp.forward_bound(flat, X)
    bad = np.nonzero(np.abs(y - ye) > ey)[0]
    assert bad.size == 0, (bad[:5], y[bad[:5]], ye[bad[:5]], ey[bad[:5]])
    assert np.linalg.norm(y - ye) <= 2.0 ** -6 * np.linalg.norm(ye)


@pytest.mark.parametrize("n,seed,offset", [(16, 0, 0.0), (1000, 1, 0.0), (4099, 2, 3.0), (20_000, 3, 0.0)])
def test_gradient_parity(n, seed, offset):
    flat = params(seed)
    X = features(n, seed + 10)
    t = np.random.default_rng(seed + 20).uniform(0.0, 1.0, n) + offset
    t = t.astype(np.float32).astype(np.float64)
    M = model_with(flat)
    feat = dev(bf16_bits(X), torch.int16)
    tgt = dev(t, torch.float32)
    g = M.grad(feat, tgt).cpu().numpy().astype(np.float64)
    g2 = M.grad(feat, tgt).cpu().numpy().astype(np.float64)
    np.testing.assert_array_equal(g, g2)   # fixed summation order
    ge, _ = mlp.backward(flat, X, t, True)
    eg = mlp.backward_bound(flat, X, t)
    bad = np.nonzero(np.abs(g - ge) > eg)[0]
    assert bad.size == 0, (bad[:5], g[bad[:5]], ge[bad[:5]], eg[bad[:5]])
    errs = rel_errors(g, ge)
    assert max(errs.values()) < 2.0 ** -6, errs


def test_adam_step_parity():
    n, B, lr, seed = 3000, 512, 1e-3, 77
    flat = params(5)
    X = features(n, 50)
    t = np.random.default_rng(51).uniform(0.0, 1.0, n).astype(np.float32).astype(np.float64)
    M = model_with(flat)
    M.train(dev(bf16_bits(X), torch.int16), dev(t, torch.float32), steps=1, batch=B, lr=lr, seed=seed)
    new = M.get_params().astype(np.float64)
    rows = np.array([helpers.splitmix64_py(seed, i) % n for i in range(B)])
    ge, _ = mlp.backward(flat, X[rows], t[rows], True)
    eg = mlp.backward_bound(flat, X[rows], t[rows])
    z = np.zeros(NP)
    ref, _, _ = mlp.adam_step(flat, z, z, ge, 1, lr)
    step = new - flat
    # the first Adam step is lr * g / (|g| + eps): +-lr wherever the gradient
    # sign is certain, somewhere in [-lr, lr] otherwise
    sure = np.abs(ge) > eg + 1e-6
    assert np.all(np.abs(new[sure] - ref[sure]) <= 1e-6 * lr + 2.0 ** -23 * np.abs(flat[sure]))
    assert np.all(np.abs(step) <= lr * (1 + 1e-5) + 2.0 ** -23 * np.abs(flat))
    assert sure.mean() > 0.3


def test_training_reduces_loss():
    n = 8192
    X = features(n, 60)
    # a smooth target of the inputs the network can fit
    t = np.tanh(X[:, 0] - 0.5 * X[:, 1] + 0.25 * X[:, 2] * X[:, 3]) + 0.5 * X[:, 5]
    t = t.astype(np.float32).astype(np.float64)
    flat = mlp.init_params(3)
    M = model_with(flat)
    l0 = mlp.loss(flat, X, t)
    M.train(dev(bf16_bits(X), torch.int16), dev(t, torch.float32), steps=300, batch=256, lr=3e-3, seed=9)
    l1 = mlp.loss(M.get_params().astype(np.float64), X, t)
    assert l1 < 0.1 * l0, (l0, l1)
