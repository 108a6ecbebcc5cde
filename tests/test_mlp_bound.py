"""CPU checks of the element-wise FP32 error bounds used by the network's GPU
parity tests (tests/mlp_bound.py): an FP32 evaluation of the network and of
its gradients (numpy, BLAS summation order) stays inside them, element by
element, and the bounds are tight enough to see a mistake of a small fraction
of any one element."""
import numpy as np

import oracle
from tests import mlp_bound


def _params(seed, D=32, H1=256, H2=256):
    rng = np.random.default_rng(seed)
    W1 = oracle.to_bf16(rng.standard_normal((H1, D)) * np.sqrt(2.0 / D))
    W2 = oracle.to_bf16(rng.standard_normal((H2, H1)) * np.sqrt(2.0 / H1))
    W3 = oracle.to_bf16(rng.standard_normal(H2) * np.sqrt(1.0 / H2))
    b1 = rng.standard_normal(H1).astype(np.float32).astype(np.float64) * 0.1
    b2 = rng.standard_normal(H2).astype(np.float32).astype(np.float64) * 0.1
    return oracle.MLPParams(W1, b1, W2, b2, W3, np.float32(0.7))


def _f32_network(p, x, t):
    """The network and its gradients with every operation rounded to FP32."""
    from scipy.special import erf
    f = np.float32

    def g(z):
        return (f(0.5) * z * (f(1) + erf(z.astype(np.float64) / np.sqrt(2.0)).astype(f))).astype(f)

    def gp(z):
        z64 = z.astype(np.float64)
        return (0.5 * (1 + erf(z64 / np.sqrt(2))) + z64 * np.exp(-0.5 * z64 * z64) / np.sqrt(2 * np.pi)).astype(f)

    W1, W2, W3 = (a.astype(f) for a in (p.W1, p.W2, p.W3))
    b1, b2, b3 = p.b1.astype(f), p.b2.astype(f), f(p.b3)
    z1 = x @ W1.T + b1
    a1 = g(z1)
    z2 = a1 @ W2.T + b2
    a2 = g(z2)
    y = a2 @ W3 + b3
    B = x.shape[0]
    dy = (f(2) * (y - t) / f(B)).astype(f)
    dz2 = dy[:, None] * W3[None, :] * gp(z2)
    dz1 = (dz2 @ W2) * gp(z1)
    grads = [dz1.T @ x, dz1.sum(0), dz2.T @ a1, dz2.sum(0), a2.T @ dy, np.array([dy.sum()], dtype=f)]
    return y, np.concatenate([a.ravel() for a in grads]).astype(np.float64)


def test_fp32_network_stays_inside_the_bounds():
    p = _params(1)
    rng = np.random.default_rng(2)
    x = rng.standard_normal((257, 32)).astype(np.float32)
    t = (rng.standard_normal(257) * 0.5 + 1.0).astype(np.float32)
    y_ref = oracle.mlp_forward(p, x)
    y, e_y, v = mlp_bound.forward_bound(p, x)
    assert np.allclose(y, y_ref, rtol=1e-12, atol=1e-12)  # the helper reads the oracle's parameters alike
    y32, g32 = _f32_network(p, x, t)
    assert np.all(np.abs(y32.astype(np.float64) - y_ref) <= e_y)
    loss_ref, rg = oracle.mlp_backward(p, x, t)
    g_ref = np.concatenate([rg[k].ravel() for k in ("W1", "b1", "W2", "b2", "W3", "b3")])
    g, e_g, loss, e_loss = mlp_bound.gradient_bound(p, x, t)
    assert np.allclose(g, g_ref, rtol=1e-9, atol=1e-15)
    assert abs(loss - loss_ref) <= 1e-12 * loss_ref
    assert np.all(np.abs(g32 - g_ref) <= e_g)
    # the bounds are element-wise and tight: a mistake of 1% of an element is
    # visible on 95% of the gradient elements (the old test allowed 1e-3 of
    # the largest element of each block), and y is held to 1e-4
    ratio = e_g / np.maximum(np.abs(g_ref), 1e-30)
    assert np.median(ratio) < 1e-3 and np.percentile(ratio, 95) < 1e-2
    assert np.max(e_y / (1 + np.abs(y_ref))) < 1e-4
    # the worst-case first-order bound holds too, and is far wider
    assert np.all(np.abs(y32.astype(np.float64) - y_ref) <= v["worst_y"])
    assert np.median(v["worst_y"] / e_y) > 10
