"""Element-wise error bounds for the learned-radius network evaluated in FP32.

The GPU evaluates y = W3 g(W2 g(W1 xs + b1) + b2) + b3 and the gradients of
mean_b (y_b - t_b)^2 in FP32.  The weights lie on the BF16 grid, so they are
exact.  The functions here compute, for every output and gradient element, a
bound on |FP32 result - exact result| derived from the arithmetic.

Model (Higham and Mary, "A new approach to probabilistic rounding error
analysis", SIAM J. Sci. Comput. 41(5), 2019).  Every FP32 operation returns
its exact result times (1 + d) with |d| <= u = 2^-24.  The d of distinct
operations are independent with mean zero.  An error is a sum of such terms
c_k d_k, each bounded by u |c_k|, so it is sub-Gaussian with variance proxy
sigma^2 = u^2 sum_k c_k^2.  Then P(|error| > lam sigma) <= 2 exp(-lam^2 / 2).
With lam = 8 that is 2.5e-14 per element, and below 2e-9 over the 74,497
parameters.  Errors of the network's intermediate values are propagated to
first order with the same proxies:
  * independent sources add in quadrature;
  * dependent groups (several functions of one sample's forward errors) add
    their sigmas (Minkowski), which stays a valid proxy whatever the
    correlation;
  * a chain of K fused multiply-adds (or adds) over terms t_k has at most K
    roundings, each of size <= u |partial sum| <= u sum|t_k|, so its
    sigma is at most u sqrt(K) sum|t_k|; K follows the library's reduction
    orders (stated per line);
  * g(z) = 0.5 z (1 + erf(z / sqrt 2)) in FP32 counts as CG = 8 roundings of
    size u|z| (the argument, erff within 2 ulp, 1 + erf and the product take
    about 4; the approximation errors of erff and expf are treated as
    independent of one another like roundings);
  * g'(z) = Phi(z) + z phi(z) in FP32 counts as CGP = 8 roundings of size u.

A worst-case first-order bound (gamma_K sum|terms| propagated through every
layer) is also returned.  It holds with no probabilistic assumption, but it
compounds K u through the layers and is about 1e-3 of the output; the
probabilistic bound is what a parity test can use to see small mistakes.
"""
import numpy as np
from scipy.special import erf

U = 2.0 ** -24
LAM = 8.0
CG = 8.0
CGP = 8.0


def gamma(k):
    k = np.asarray(k, dtype=np.float64)
    return k * U / (1.0 - k * U)


def _g(z):
    return 0.5 * z * (1.0 + erf(z / np.sqrt(2.0)))


def _phi(z):
    return np.exp(-0.5 * z * z) / np.sqrt(2.0 * np.pi)


def _gp(z):
    return 0.5 * (1.0 + erf(z / np.sqrt(2.0))) + z * _phi(z)


def _gpp(z):
    return _phi(z) * (2.0 - z * z)


def forward(p, xs, xs_rounded=False):
    """FP64 forward pass of the oracle's network and the error proxies of an
    FP32 evaluation.  xs: B x D FP32 inputs as both sides receive them.
    xs_rounded: the GPU forms xs itself as (x - mu) / sd (two roundings; the
    test forms it in FP32 too, so each element may differ by four).
    Returns a dict of FP64 values, sigmas and the worst-case bound of y."""
    x = xs.astype(np.float64)
    D, H1, H2 = p.dims
    W1, W2, W3 = p.W1, p.W2, p.W3
    v = {"x": x}
    s2x = 4.0 * U * U * x * x if xs_rounded else np.zeros_like(x)
    # layer 1: an FMA chain over the D inputs from zero, then + b1
    z1 = x @ W1.T + p.b1
    S1 = np.abs(x) @ np.abs(W1).T + np.abs(p.b1)
    s2c1 = U * U * (D + 1) * S1 * S1
    a1 = _g(z1)
    gp1 = _gp(z1)
    # local error of a1 (independent across j): chain 1 and the evaluation of g
    s2a1 = gp1 * gp1 * s2c1 + CG * U * U * z1 * z1
    # layer 2: an FMA chain over H1, then + b2
    z2 = a1 @ W2.T + p.b2
    S2 = np.abs(a1) @ np.abs(W2).T + np.abs(p.b2)
    s2c2 = U * U * (H1 + 1) * S2 * S2
    s2z2 = s2a1 @ (W2 * W2).T + s2c2          # the a1 errors are independent across j
    a2 = _g(z2)
    gp2 = _gp(z2)
    # output: per lane an FMA chain over ceil(H2/64) values, a 6-level
    # butterfly across the wave, then + b3
    y = a2 @ W3 + p.b3
    S3 = np.abs(a2) @ np.abs(W3) + abs(p.b3)
    s2c3 = U * U * (-(-H2 // 64) + 6 + 1) * S3 * S3
    # y's error written over its independent sources: w_j = dy/da1_j
    v2 = gp2 * W3[None, :]
    w = v2 @ W2
    s2y = (w * w * s2a1).sum(1) + (v2 * v2 * s2c2).sum(1) + CG * U * U * (W3[None, :] ** 2 * z2 * z2).sum(1) \
        + s2c3
    if xs_rounded:
        wx = (w * gp1) @ W1
        s2y = s2y + (wx * wx * s2x).sum(1)
    # worst case: gamma_K sum|terms| carried through every layer
    e_x = 4.0 * U * np.abs(x) if xs_rounded else np.zeros_like(x)
    e_z1 = gamma(D + 1) * S1 + e_x @ np.abs(W1).T
    e_a1 = np.abs(gp1) * e_z1 + CG * U * np.abs(z1)
    e_z2 = gamma(H1 + 1) * S2 + e_a1 @ np.abs(W2).T
    e_a2 = np.abs(gp2) * e_z2 + CG * U * np.abs(z2)
    e_y = gamma(-(-H2 // 64) + 7) * S3 + e_a2 @ np.abs(W3)
    v.update(z1=z1, a1=a1, gp1=gp1, s2c1=s2c1, s2a1=s2a1, z2=z2, a2=a2, gp2=gp2, s2c2=s2c2, s2z2=s2z2,
             w=w, y=y, s2y=s2y, S3=S3, worst_y=1.01 * e_y)
    return v


def forward_bound(p, xs, xs_rounded=False):
    """(y, bound) with bound = LAM sigma_y plus the FP64 oracle's own rounding."""
    v = forward(p, xs, xs_rounded)
    return v["y"], LAM * np.sqrt(v["s2y"]) + 2.0 ** -50 * v["S3"], v


def gradient_bound(p, xs, t):
    """Gradients of mean_b (y_b - t_b)^2 in the flat order W1, b1, W2, b2,
    W3, b3 (FP64), the element-wise bounds LAM sigma, the loss, its bound.
    xs are the FP32 network inputs (standardisation mu = 0, sd = 1)."""
    v = forward(p, xs)
    D, H1, H2 = p.dims
    B = xs.shape[0]
    W2, W3 = p.W2, p.W3
    x, z1, a1, z2, a2 = v["x"], v["z1"], v["a1"], v["z2"], v["a2"]
    gp1, gp2 = v["gp1"], v["gp2"]
    t = t.astype(np.float64)
    r = v["y"] - t
    s2r = v["s2y"] + U * U * r * r
    dy = 2.0 * r / B
    s2dy = (2.0 / B) ** 2 * s2r + U * U * dy * dy
    sdy = np.sqrt(s2dy)
    # loss: per thread an FMA chain over ceil(B/256) rows, an 8-level tree, / B
    loss = float(np.mean(r * r))
    s2loss = float(np.sum((2 * r / B) ** 2 * s2r) + U * U * (-(-B // 256) + 9) * (np.sum(r * r) / B) ** 2 +
                   U * U * loss * loss)
    # column sums over the batch: FMA chains of ceil(B/64) rows in 16 x 4
    # slices, 3 adds across 4 waves, 16 adds across slices
    kcol = -(-B // 64) + 3 + 16
    # split-K weight gradients: 8 slices of ceil(B/8) rows, 8 adds
    ksk = -(-B // 8) + 8
    sa1 = np.sqrt(v["s2a1"])                      # local error of a1 (chain 1 and g)
    sz2 = np.sqrt(v["s2z2"])
    sa2 = np.abs(gp2) * sz2 + np.sqrt(CG) * U * np.abs(z2)
    # output layer: gW3_i = sum_b dy_b a2_bi
    per = np.abs(a2) * sdy[:, None] + np.abs(dy)[:, None] * sa2   # dependent within a sample
    s_W3 = np.sqrt((per * per).sum(0) + U * U * kcol * (np.abs(dy) @ np.abs(a2)) ** 2)
    s_b3 = np.sqrt([s2dy.sum() + U * U * kcol * np.abs(dy).sum() ** 2])
    # dz2 = (dy w3) g'(z2), two roundings
    gpp2 = _gpp(z2)
    dz2 = dy[:, None] * W3[None, :] * gp2
    sdz2 = np.abs(W3[None, :] * gp2) * sdy[:, None] + np.abs(dy[:, None] * W3[None, :]) * (
        np.abs(gpp2) * sz2 + np.sqrt(CGP) * U) + np.sqrt(2.0) * U * np.abs(dz2)
    # gW2_ij = sum_b dz2_bi a1_bj (split-K)
    s2_W2 = (sdz2 ** 2).T @ (a1 * a1) + 2.0 * (np.abs(dz2) * sdz2).T @ (np.abs(a1) * sa1) + \
        (dz2 * dz2).T @ (sa1 * sa1) + U * U * ksk * (np.abs(dz2).T @ np.abs(a1)) ** 2
    s_b2 = np.sqrt((sdz2 ** 2).sum(0) + U * U * kcol * np.abs(dz2).sum(0) ** 2)
    # sd_bj = sum_i dz2_bi W2_ij (FMA chain over H2), its error split into
    #  A: through dy_b (coefficient w_bj, exactly as in the forward pass)
    #  B: through z2's errors, rewritten over the independent a1 and chain-2 errors
    #  C, D: g' evaluation and the two roundings of dz2 (independent over i)
    #  E: the chain itself
    c = W3[None, :] * gpp2                                          # B x H2
    M = np.einsum("ij,bi,ik->bjk", W2, c, W2, optimize=True)       # W2^T diag(c_b) W2
    s2B = dy[:, None] ** 2 * (np.einsum("bjk,bk->bj", M * M, v["s2a1"]) +
                              (c * c * v["s2c2"]) @ (W2 * W2))
    del M
    s2C = dy[:, None] ** 2 * (CGP * U * U * (W3 * W3)[None, :]) @ (W2 * W2)
    s2D = (2.0 * U * U * dz2 * dz2) @ (W2 * W2)
    sdv = dz2 @ W2
    s2E = U * U * H2 * (np.abs(dz2) @ np.abs(W2)) ** 2
    ssd = np.abs(v["w"]) * sdy[:, None] + np.sqrt(s2B) + np.sqrt(s2C + s2D + s2E)
    # dz1 = sd g'(z1), one rounding
    gpp1 = _gpp(z1)
    dz1 = sdv * gp1
    sdz1 = np.abs(gp1) * ssd + np.abs(sdv) * np.abs(gpp1) * np.sqrt(v["s2c1"]) + \
        np.sqrt(CGP * U * U * sdv * sdv + U * U * dz1 * dz1)
    # gW1_jd = sum_b dz1_bj x_bd (x exact), gb1_j = sum_b dz1_bj
    s2_W1 = (sdz1 ** 2).T @ (x * x) + U * U * ksk * (np.abs(dz1).T @ np.abs(x)) ** 2
    s_b1 = np.sqrt((sdz1 ** 2).sum(0) + U * U * kcol * np.abs(dz1).sum(0) ** 2)
    g = np.concatenate([(dz1.T @ x).ravel(), dz1.sum(0), (dz2.T @ a1).ravel(), dz2.sum(0), a2.T @ dy,
                        [dy.sum()]])
    s = np.concatenate([np.sqrt(s2_W1).ravel(), s_b1, np.sqrt(s2_W2).ravel(), s_b2, s_W3, s_b3])
    return g, LAM * s + 2.0 ** -50 * np.abs(g).max(), loss, LAM * np.sqrt(s2loss) + 2.0 ** -50 * loss
