"""CPU reference of the candidate-proposal network: a 16-64-64-1 ReLU MLP.

TEST INFRASTRUCTURE ONLY: used by the tests and the smoke check; the product
library never imports it. It shares no code with the HIP kernels.

The paper evaluates every variable exactly in every iteration (section 3.1,
"Scoring Functions": scores are computed from scratch each iteration); the
learned proposal is an addition beside that method, so this file follows the
textbook definitions instead of a passage of the paper:

* forward  z1 = W1 x + b1, h1 = relu(z1), z2 = W2 h1 + b2, h2 = relu(z2),
  y = W3 h2 + b3;
* loss     L = mean_b (y_b - t_b)^2 (mean squared error over the batch);
* backward by the chain rule, in the same order;
* Adam     (Kingma & Ba 2015, Algorithm 1) with bias-corrected moments.

Precision model of the kernels it checks: every operand of a product is a
bfloat16 value (weights, inputs and hidden activations rounded to nearest,
ties to even), products are accumulated in FP32, biases and master weights
are FP32. `emulate=True` reproduces the bfloat16 roundings and accumulates in
FP64 (so the only difference to the kernels is FP32 accumulation order);
`emulate=False` is plain FP64 and is the function the finite-difference
check pins. `forward_bound` / `backward_bound` propagate a rigorous per-output
bound on |kernel - emulated reference| through the layers.

Flat parameter order (5313 FP32 values): W1[64][16] (row = output unit),
b1[64], W2[64][64], b2[64], W3[64], b3[1].
"""
from __future__ import annotations

import numpy as np

H = 64
F = 16
SIZES = (("W1", (H, F)), ("b1", (H,)), ("W2", (H, H)), ("b2", (H,)), ("W3", (H,)), ("b3", (1,)))
NPARAM = sum(int(np.prod(s)) for _, s in SIZES)
U32 = 2.0 ** -24  # unit roundoff of FP32 (round to nearest)
MASK64 = (1 << 64) - 1


def bf16(x):
    """Round FP64 values to the nearest bfloat16 value (8 significant bits,
    ties to even), returned as FP64. bfloat16 keeps FP32's exponent range;
    magnitudes below 2^-126 are outside what the network sees and are not
    treated as subnormals here."""
    x = np.asarray(x, dtype=np.float64)
    f, e = np.frexp(x)  # x = f * 2^e, 0.5 <= |f| < 1
    return np.ldexp(np.rint(f * 256.0), e - 8)


def bf16_ulp(x):
    """Spacing of bfloat16 values at |x| (2^(floor(log2|x|) - 7)); 0 at 0."""
    x = np.abs(np.asarray(x, dtype=np.float64))
    _, e = np.frexp(x)
    return np.where(x > 0, np.ldexp(1.0, e - 8), 0.0)


def splitmix64(seed: int, index: int) -> int:
    """(index+1)-th output of SplitMix64 started at state `seed` (Steele, Lea
    and Flood, "Fast splittable pseudorandom number generators", 2014)."""
    z = (seed + (index + 1) * 0x9E3779B97F4A7C15) & MASK64
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & MASK64
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & MASK64
    return z ^ (z >> 31)


def unflatten(flat):
    flat = np.asarray(flat, dtype=np.float64)
    assert flat.shape == (NPARAM,)
    out, o = {}, 0
    for name, shape in SIZES:
        k = int(np.prod(shape))
        out[name] = flat[o:o + k].reshape(shape).copy()
        o += k
    return out


def flatten(params):
    return np.concatenate([np.asarray(params[name], dtype=np.float64).reshape(-1) for name, _ in SIZES])


def init_params(seed: int):
    """He-uniform initialisation: weight with flat index p of a layer with
    fan-in k is (2u - 1) * sqrt(6 / k), u = (splitmix64(seed, p) >> 11) * 2^-53,
    rounded to FP32; biases are zero."""
    flat = np.zeros(NPARAM)
    o = 0
    for name, shape in SIZES:
        k = int(np.prod(shape))
        if name.startswith("W"):
            fan_in = shape[-1] if len(shape) == 2 else H
            lim = np.sqrt(6.0 / fan_in)
            for p in range(o, o + k):
                u = (splitmix64(seed, p) >> 11) * 2.0 ** -53
                flat[p] = float(np.float32((2.0 * u - 1.0) * lim))
        o += k
    return flat


def forward(flat, X, emulate: bool = True):
    """Network outputs for inputs X (batch x 16); returns (y, cache)."""
    P = unflatten(flat)
    r = bf16 if emulate else (lambda a: np.asarray(a, dtype=np.float64))
    Xb = r(X)
    W1, W2, W3 = r(P["W1"]), r(P["W2"]), r(P["W3"])
    z1 = Xb @ W1.T + P["b1"]
    h1 = r(np.maximum(z1, 0.0))
    z2 = h1 @ W2.T + P["b2"]
    h2 = r(np.maximum(z2, 0.0))
    y = h2 @ W3 + P["b3"][0]
    return y, dict(Xb=Xb, W1=W1, W2=W2, W3=W3, z1=z1, h1=h1, z2=z2, h2=h2, P=P)


def loss(flat, X, t, emulate: bool = False):
    y, _ = forward(flat, X, emulate)
    return float(np.mean((y - np.asarray(t, dtype=np.float64)) ** 2))


def backward(flat, X, t, emulate: bool = True):
    """Gradient of the mean squared error with respect to the flat
    parameters. With `emulate`, the operands of every product are rounded to
    bfloat16 as the kernels do: hidden activations (already in the forward),
    the output-layer weights, and the back-propagated signals g2 and g1."""
    t = np.asarray(t, dtype=np.float64)
    y, c = forward(flat, X, emulate)
    r = bf16 if emulate else (lambda a: np.asarray(a, dtype=np.float64))
    B = y.shape[0]
    g3 = 2.0 * (y - t) / B                       # dL/dy
    dW3 = c["h2"].T @ g3
    db3 = np.array([g3.sum()])
    g2 = np.outer(g3, c["W3"]) * (c["z2"] > 0)   # dL/dz2
    g2b = r(g2)
    dW2 = g2b.T @ c["h1"]
    db2 = g2.sum(axis=0)
    g1 = (g2b @ c["W2"]) * (c["z1"] > 0)         # dL/dz1
    g1b = r(g1)
    dW1 = g1b.T @ c["Xb"]
    db1 = g1.sum(axis=0)
    return flatten(dict(W1=dW1, b1=db1, W2=dW2, b2=db2, W3=dW3, b3=db3)), y


def _relu_round_error(z, e):
    """Bound on |bf16(relu(z')) - bf16(relu(z))| when |z' - z| <= e: zero where
    both are clearly negative, e plus one bfloat16 spacing elsewhere."""
    return np.where(z < -e, 0.0, e + bf16_ulp(np.abs(z) + e))


def forward_bound(flat, X):
    """Per-sample bound on |y_kernel - y_emulated| and the layer bounds used by
    backward_bound. A K-term FP32 accumulation (bias included as one more
    term) differs from the exact sum by at most (K+1) u sum|terms|; a hidden
    value whose FP32 result differs by e from the reference may round to a
    different bfloat16 value, at most e + one bfloat16 spacing away."""
    y, c = forward(flat, X, True)
    P = c["P"]
    aW1, aW2, aW3 = np.abs(c["W1"]), np.abs(c["W2"]), np.abs(c["W3"])
    e1 = (F + 2) * U32 * (np.abs(c["Xb"]) @ aW1.T + np.abs(P["b1"]))
    r1 = _relu_round_error(c["z1"], e1)
    e2 = r1 @ aW2.T + (H + 2) * U32 * (np.abs(c["h1"]) @ aW2.T + np.abs(P["b2"]))
    r2 = _relu_round_error(c["z2"], e2)
    ey = r2 @ aW3 + (H + 2) * U32 * (np.abs(c["h2"]) @ aW3 + abs(P["b3"][0]))
    return ey, dict(e1=e1, r1=r1, e2=e2, r2=r2, ey=ey, c=c, y=y)


def backward_bound(flat, X, t):
    """Per-parameter bound on |gradient_kernel - gradient_emulated| for a
    kernel that follows the precision model above and sums the batch in FP32
    (in any order): forward errors are carried into the output signal, ReLU
    gates whose pre-activation lies within its error bound of zero count with
    their full magnitude, and every product over the batch gets the FP32
    accumulation term."""
    t = np.asarray(t, dtype=np.float64)
    ey, b = forward_bound(flat, X)
    c, y = b["c"], b["y"]
    B = y.shape[0]
    Bt = B + 2
    g3 = 2.0 * (y - t) / B
    eg3 = 2.0 * ey / B + 4 * U32 * np.abs(g3)
    aW2, aW3 = np.abs(c["W2"]), np.abs(c["W3"])
    ah1, ah2, aX = np.abs(c["h1"]), np.abs(c["h2"]), np.abs(c["Xb"])
    dW3 = eg3 @ (ah2 + b["r2"]) + np.abs(g3) @ b["r2"] + Bt * U32 * (np.abs(g3) @ ah2)
    db3 = np.array([eg3.sum() + Bt * U32 * np.abs(g3).sum()])
    g2 = np.outer(g3, c["W3"]) * (c["z2"] > 0)
    unsure2 = np.abs(c["z2"]) <= b["e2"]
    eg2 = np.outer(eg3, aW3) + 2 * U32 * np.abs(g2)
    eg2 = np.where(unsure2, np.outer(np.abs(g3) + eg3, aW3), eg2)
    rg2 = eg2 + bf16_ulp(np.abs(g2) + eg2)
    ag2 = np.abs(bf16(g2))
    dW2 = rg2.T @ (ah1 + b["r1"]) + ag2.T @ b["r1"] + Bt * U32 * (ag2.T @ ah1)
    db2 = eg2.sum(axis=0) + Bt * U32 * np.abs(g2).sum(axis=0)
    dh1 = bf16(g2) @ c["W2"]
    edh1 = rg2 @ aW2 + (H + 2) * U32 * (ag2 @ aW2)
    unsure1 = np.abs(c["z1"]) <= b["e1"]
    eg1 = np.where(unsure1, np.abs(dh1) + edh1, edh1)
    g1 = dh1 * (c["z1"] > 0)
    rg1 = eg1 + bf16_ulp(np.abs(g1) + eg1)
    ag1 = np.abs(bf16(g1))
    dW1 = rg1.T @ aX + Bt * U32 * (ag1.T @ aX)
    db1 = eg1.sum(axis=0) + Bt * U32 * np.abs(g1).sum(axis=0)
    return flatten(dict(W1=dW1, b1=db1, W2=dW2, b2=db2, W3=dW3, b3=db3))


def adam_step(flat, m, v, grad, step: int, lr: float, beta1: float = 0.9, beta2: float = 0.999,
              eps: float = 1e-8):
    """One Adam update (step counts from 1); returns (params, m, v)."""
    m = beta1 * m + (1.0 - beta1) * grad
    v = beta2 * v + (1.0 - beta2) * grad * grad
    mhat = m / (1.0 - beta1 ** step)
    vhat = v / (1.0 - beta2 ** step)
    return flat - lr * mhat / (np.sqrt(vhat) + eps), m, v
