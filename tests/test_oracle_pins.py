"""Pins of the FP64 oracle against facts the paper and the mathematics fix.

None of these re-types an oracle formula: each checks the oracle against a
closed form, an identity, a library routine in a special case, brute force on
tiny inputs, or a constructed input whose answer is known.
"""
import math

import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.filterwarnings("ignore::RuntimeWarning")


# --------------------------------------------------------------------------- #
# DFT (Section IV-E, Eq. 1): Parseval, closed forms, numpy.fft special case
@pytest.mark.parametrize("n", [8, 64, 256, 1024])
def test_parseval_full_spectrum(n):
    rng = np.random.default_rng(n)
    x = rng.standard_normal(n).astype(np.float32)
    total = 0.0
    for k in range(0, n // 2 + 1):
        re, im = oracle.dft_coef(x, k)
        total += oracle.weight(k, n) * (re * re + im * im)
    energy = float(np.sum(x.astype(np.float64) ** 2))
    assert abs(total - energy) <= 1e-12 * energy


@pytest.mark.parametrize("n,f,A,phi", [(256, 3, 1.5, 0.3), (256, 16, 2.0, -1.2),
                                       (128, 1, 0.7, 2.9), (1024, 100, 1.0, -math.pi / 2)])
def test_dft_closed_form_sinusoid(n, f, A, phi):
    t = np.arange(n)
    x = (A * np.cos(2 * np.pi * f * t / n + phi)).astype(np.float32)
    tol = 4 * A * math.sqrt(n) * 2.0 ** -24  # FP32 rounding of the input
    for k in range(1, n // 2):
        re, im = oracle.dft_coef(x, k)
        if k == f:
            assert abs(re - A * math.sqrt(n) / 2 * math.cos(phi)) <= tol
            assert abs(im - A * math.sqrt(n) / 2 * math.sin(phi)) <= tol
        else:
            assert abs(re) <= tol and abs(im) <= tol


def test_dft_sign_convention_sine():
    # sin(2 pi f t / n) has X_f = -i sqrt(n)/2 under exp(-i...) with n^-1/2 scaling
    n, f = 256, 5
    x = np.sin(2 * np.pi * f * np.arange(n) / n).astype(np.float32)
    re, im = oracle.dft_coef(x, f)
    assert abs(re) < 1e-5 and abs(im + math.sqrt(n) / 2) < 1e-5


def test_dft_pool_matches_numpy_fft():
    X = synth.collection(20, 256, "mix", seed=11)
    pool = oracle.dft_pool(X, 16)
    F = np.fft.fft(X.astype(np.float64), axis=1) / math.sqrt(256)
    ref = np.empty_like(pool)
    ref[:, 0::2] = F[:, 1:17].real
    ref[:, 1::2] = F[:, 1:17].imag
    assert np.max(np.abs(pool - ref)) < 1e-12


# --------------------------------------------------------------------------- #
# Lower bounds (Eq. 1, Eq. 2, Eq. 3; Definition of LBD)
@pytest.mark.parametrize("n", [16, 64, 256])
def test_dft_lb_full_spectrum_equals_distance(n):
    """Eq. 1 with every non-DC value (weights 2, Nyquist 1) is the distance."""
    X = synth.collection(6, n, "mix", seed=5)
    coefs = []
    for x in X:
        c = []
        for k in range(1, n // 2 + 1):
            re, im = oracle.dft_coef(x, k)
            c += [re, im]
        coefs.append(np.array(c))
    w = np.array([oracle.weight(k, n) for k in range(1, n // 2 + 1) for _ in (0, 1)])
    for a in range(len(X)):
        for b in range(len(X)):
            d2 = oracle.dist2(X[a], X[b])
            lb = oracle.dft_lb2(coefs[a], coefs[b], w)
            assert abs(lb - d2) <= 1e-10 * max(d2, 1.0)


@pytest.mark.parametrize("n", [8, 16, 64, 256])
@pytest.mark.parametrize("binning", [0, 1])
@pytest.mark.parametrize("alpha", [1, 4, 256])
def test_sfa_lb_below_distance_every_pair(n, binning, alpha):
    """Definition of LBD: the SFA lower bound never exceeds the distance."""
    P = min(16, n // 2 - 1)
    l = min(16, 2 * P)
    X = np.concatenate([synth.collection(100, n, "rw", seed=21),
                        synth.collection(100, n, "hf", seed=22)])
    var, sel, beta = oracle.learn_bins(X, X.shape[0], P=P, l=l, alpha=alpha, binning=binning)
    W, C = oracle.words(X, sel, beta, P=P)
    # pairwise distances in FP64 from the oracle, every ordered pair
    worst = -np.inf
    for qi in range(0, X.shape[0], 3):
        for xi in range(X.shape[0]):
            lb = oracle.sfa_lb2(C[qi], W[xi], beta)
            d2 = oracle.dist2(X[qi], X[xi])
            worst = max(worst, lb - d2 * (1 + 1e-12))
            if alpha == 1:
                assert lb == 0.0
    assert worst <= 0.0


def test_sfa_lb_fine_bins_approach_dft_lb():
    """Very fine equi-width bins: the SFA bound tends to the DFT bound (Eq. 2 -> Eq. 1)."""
    n = 256
    X = synth.collection(300, n, "mix", seed=31)
    for alpha in (16, 256):
        var, sel, beta = oracle.learn_bins(X, 300, alpha=alpha, binning=1)
        W, C = oracle.words(X, sel, beta)
        width = (beta[:, -1] - beta[:, 0]) / (alpha - 2)
        slack = math.sqrt(float(np.sum(2.0 * width ** 2)))
        for qi in range(0, 300, 37):
            for xi in range(0, 300, 7):
                lb = oracle.sfa_lb2(C[qi], W[xi], beta)
                dl = oracle.dft_lb2(C[qi], C[xi], np.full(16, 2.0))
                assert lb <= dl * (1 + 1e-12) + 1e-12
                assert math.sqrt(dl) - math.sqrt(lb) <= slack + 1e-9


def test_mind_cases():
    beta = np.array([-1.0, 0.0, 2.0])  # alpha = 4 bins: (-inf,-1) [-1,0) [0,2) [2,inf)
    assert oracle.mind(-0.5, 1, beta) == 0.0
    assert oracle.mind(-3.0, 1, beta) == pytest.approx(2.0)
    assert oracle.mind(5.0, 2, beta) == pytest.approx(3.0)
    assert oracle.mind(-1e9, 0, beta) == 0.0
    assert oracle.mind(1e9, 3, beta) == 0.0
    assert oracle.mind(-5.0, 3, beta) == pytest.approx(7.0)


# --------------------------------------------------------------------------- #
# MCB (Algorithm 1): breakpoints and variance selection on constructed samples
def test_equi_depth_on_permutation():
    M, alpha = 1000, 256
    vals = np.random.default_rng(0).permutation(M).astype(np.float64)
    beta = oracle.breakpoints(vals, alpha, binning=0)
    expect = np.array([(a * M) // alpha for a in range(1, alpha)], dtype=np.float64)
    assert np.array_equal(beta, expect)


def test_equi_width_known_range():
    vals = np.array([3.0, -1.0, 7.0, 0.5, 2.0])
    beta = oracle.breakpoints(vals, 4, binning=1)
    assert np.allclose(beta, [1.0, 3.0, 5.0], atol=0, rtol=0)


def test_symbol_half_open_bins():
    beta = np.array([-1.0, 0.0, 2.0])
    assert oracle.symbol(-1.0, beta) == 1  # a value on a breakpoint goes up
    assert oracle.symbol(-1.0000001, beta) == 0
    assert oracle.symbol(0.0, beta) == 2
    assert oracle.symbol(1.999, beta) == 2
    assert oracle.symbol(2.0, beta) == 3
    assert oracle.symbol(float("-inf"), beta) == 0


def test_variance_selection_constructed():
    """Sinusoids with amplitude A_f and uniform random phase have
    Var(Re X_f) = Var(Im X_f) = A_f^2 n / 8, so the top-16 values are the Re/Im
    pairs of the 8 largest amplitudes, in decreasing amplitude order."""
    n, m = 256, 4000
    rng = np.random.default_rng(7)
    amps = rng.permutation(np.linspace(0.2, 3.2, 16))  # amplitude of f = 1..16
    t = np.arange(n)
    X = np.zeros((m, n))
    for f in range(1, 17):
        ph = rng.uniform(0, 2 * np.pi, size=(m, 1))
        X += amps[f - 1] * np.cos(2 * np.pi * f * t / n + ph)
    X = X.astype(np.float32)
    var, sel, beta = oracle.learn_bins(X, m, P=16, l=16, alpha=4)
    expect_var = np.repeat(amps ** 2 * n / 8, 2)
    assert np.allclose(var, expect_var, rtol=0.12)
    top = np.argsort(-amps, kind="stable")[:8] + 1  # frequencies by amplitude
    got_freqs = sel // 2 + 1
    assert sorted(got_freqs.tolist()) == sorted(np.repeat(top, 2).tolist())
    # pairs appear in decreasing amplitude order
    order = [got_freqs[2 * i] for i in range(8)]
    assert order == top.tolist()


def test_select_tie_lower_index_first():
    var = np.array([1.0, 3.0, 3.0, 2.0, 3.0])
    assert oracle.select(var, 4).tolist() == [1, 2, 4, 3]


def test_learn_bins_stride_sample():
    """Rows floor(i*N/m) form the sample: a sample of all rows equals m = N."""
    X = synth.collection(64, 64, "mix", seed=3)
    v1, s1, b1 = oracle.learn_bins(X, 64, P=8, l=8, alpha=8)
    v2, s2, b2 = oracle.learn_bins(X[::4], 16, P=8, l=8, alpha=8)
    v3, s3, b3 = oracle.learn_bins(X, 16, P=8, l=8, alpha=8)
    assert np.array_equal(v2, v3) and np.array_equal(s2, s3) and np.array_equal(b2, b3)
    assert v1.shape == (16,)


# --------------------------------------------------------------------------- #
# Distances, z-normalisation, brute-force k-NN
def test_znorm_population_sigma_closed_form():
    rng = np.random.default_rng(1)
    for n in (16, 256):
        x = rng.standard_normal(n) * 3 + 5
        y = rng.standard_normal(n) + 0.5 * x
        zx, zy = oracle.znorm(x), oracle.znorm(y)
        assert abs(np.sum(zx ** 2) - n) < 1e-10
        rho = np.corrcoef(x, y)[0, 1]
        d2 = float(np.sum((zx - zy) ** 2))
        assert abs(d2 - 2 * n * (1 - rho)) < 1e-9 * n
    assert np.all(oracle.znorm(np.full(8, 3.0)) == 0.0)


def test_dist2_matches_numpy_exact_cases():
    # small integers: every partial sum is exact, so any order gives the same bits
    q = np.array([1, -2, 3, 0, 5], dtype=np.float32)
    x = np.array([0, 2, -1, 4, 5], dtype=np.float32)
    assert oracle.dist2(q, x) == 1 + 16 + 16 + 16 + 0


@pytest.mark.parametrize("k", [1, 3, 10])
def test_knn_matches_numpy_lexsort(k):
    X = synth.collection(3000, 64, "mix", seed=41)
    X[100] = X[7]      # exact duplicates: ties resolved to the lower row id
    X[2500] = X[7]
    X[1234] = X[999]
    Q, src = synth.queries(X, 12, sigma=0.1, seed=42)
    Q[3] = X[7]        # a query equal to three rows
    Q[5] = X[999]
    ids, d2 = oracle.knn(X, Q, k)
    Xd = X.astype(np.float64)
    for b in range(Q.shape[0]):
        dd = np.sum((Xd - Q[b].astype(np.float64)) ** 2, axis=1)
        order = np.lexsort((np.arange(X.shape[0]), dd))[:k]
        assert ids[b].tolist() == order.tolist()
        assert np.allclose(d2[b], dd[order], rtol=1e-12, atol=0)
    assert ids[3, 0] == 7 and d2[3, 0] == 0.0
    if k >= 3:
        assert ids[3, :3].tolist() == [7, 100, 2500]


def test_knn_k_larger_than_needed_padding():
    X = synth.collection(5, 32, "rw", seed=1)
    ids, d2 = oracle.knn(X, X[:1], 7)
    assert ids[0, :5].tolist()[0] == 0 and ids[0, 5] == -1 and np.isinf(d2[0, 6])


# --------------------------------------------------------------------------- #
# Learned-radius network: gradients, Adam, GELU form
def _tiny_mlp(seed=0, D=3, H1=4, H2=5):
    rng = np.random.default_rng(seed)
    return oracle.MLPParams(rng.standard_normal((H1, D)) * 0.7, rng.standard_normal(H1) * 0.1,
                            rng.standard_normal((H2, H1)) * 0.5, rng.standard_normal(H2) * 0.1,
                            rng.standard_normal(H2) * 0.5, 0.3)


def test_mlp_gradients_central_differences():
    p = _tiny_mlp()
    rng = np.random.default_rng(5)
    x = rng.standard_normal((7, 3)).astype(np.float32)
    t = rng.standard_normal(7).astype(np.float32)
    loss, g = oracle.mlp_backward(p, x, t)
    yb = oracle.mlp_forward(p, x)
    assert abs(loss - np.mean((yb - t.astype(np.float64)) ** 2)) < 1e-12
    h = 1e-6
    for name in ("W1", "b1", "W2", "b2", "W3"):
        arr = getattr(p, name)
        flat = arr.reshape(-1)
        for i in range(flat.shape[0]):
            old = flat[i]
            flat[i] = old + h
            lp = np.mean((oracle.mlp_forward(p, x) - t) ** 2)
            flat[i] = old - h
            lm = np.mean((oracle.mlp_forward(p, x) - t) ** 2)
            flat[i] = old
            num = (lp - lm) / (2 * h)
            assert abs(num - g[name].reshape(-1)[i]) <= 1e-6 * max(1.0, abs(num))
    old = p.b3
    p.b3 = old + h
    lp = np.mean((oracle.mlp_forward(p, x) - t) ** 2)
    p.b3 = old - h
    lm = np.mean((oracle.mlp_forward(p, x) - t) ** 2)
    p.b3 = old
    assert abs((lp - lm) / (2 * h) - g["b3"][0]) < 1e-6


def test_mlp_gelu_is_erf_form():
    # W2 = 0: the output is W3 . GELU(b2) + b3; GELU(1) = Phi(1) = 0.841344746...
    p = _tiny_mlp()
    p.W2[:] = 0.0
    p.b2[:] = 1.0
    p.W3[:] = 0.0
    p.W3[0] = 1.0
    p.b3 = 0.0
    y = oracle.mlp_forward(p, np.zeros((1, 3), dtype=np.float32))
    assert abs(y[0] - 0.8413447460685429) < 1e-14


def test_adam_first_step():
    rng = np.random.default_rng(9)
    p = rng.standard_normal(50)
    g = rng.standard_normal(50)
    p0 = p.copy()
    m, v = np.zeros(50), np.zeros(50)
    oracle.adam(p, g, m, v, 1, lr=1e-3)
    assert np.allclose(p - p0, -1e-3 * g / (np.abs(g) + 1e-8), rtol=1e-12, atol=1e-18)


def test_adam_constant_gradient_many_steps():
    """Kingma & Ba, Algorithm 1, with the same gradient g at every step: the
    moments are m_t = (1 - b1^t) g and v_t = (1 - b2^t) g^2, so the
    bias-corrected ratio is g / (|g| + eps) at every t and the parameter moves
    by the same amount each step.  Resetting the moments between steps, or a
    wrong power in either correction, makes the steps unequal."""
    rng = np.random.default_rng(19)
    g = rng.standard_normal(40) * np.logspace(-6, 2, 40)
    p = rng.standard_normal(40)
    p0 = p.copy()
    m, v = np.zeros(40), np.zeros(40)
    lr, eps = 2e-3, 1e-8
    step = -lr * g / (np.abs(g) + eps)
    for t in range(1, 31):
        prev = p.copy()
        oracle.adam(p, g, m, v, t, lr=lr, eps=eps)
        assert np.allclose(p - prev, step, rtol=1e-9, atol=1e-20), t
        assert np.allclose(m, (1 - 0.9 ** t) * g, rtol=1e-12, atol=0)
        assert np.allclose(v, (1 - 0.999 ** t) * g * g, rtol=1e-12, atol=0)
    assert np.allclose(p - p0, 30 * step, rtol=1e-9, atol=1e-20)


def test_adam_two_steps_worked_by_hand():
    """Kingma & Ba, Algorithm 1, b1 = 0.9, b2 = 0.999, two steps worked by
    hand with different gradients.

    g1 = 2, g2 = 1:  m2 = 0.9*0.1*2 + 0.1*1 = 0.28, v2 = 0.999*0.001*4 +
    0.001*1 = 0.004996; the corrections are 1 - 0.9^2 = 0.19 and
    1 - 0.999^2 = 0.001999, so the second step is
    -lr * (28/19) / (sqrt(4996/1999) + eps).

    g1 = 1, g2 = -1: m2 = 0.09 - 0.1 = -0.01 and v2 = 0.000999 + 0.001 =
    0.001999, so m2/0.19 = -1/19 and v2/0.001999 = 1: the second step is
    +lr / (19 (1 + eps)), against -lr/(1 + eps) for the first."""
    lr, eps = 1e-3, 1e-8
    p = np.zeros(2)
    m, v = np.zeros(2), np.zeros(2)
    oracle.adam(p, np.array([2.0, 1.0]), m, v, 1, lr=lr, eps=eps)
    first = p.copy()
    assert np.allclose(first, [-lr * 2 / (2 + eps), -lr / (1 + eps)], rtol=1e-13, atol=0)
    oracle.adam(p, np.array([1.0, -1.0]), m, v, 2, lr=lr, eps=eps)
    assert np.allclose(m, [0.28, -0.01], rtol=1e-12, atol=0)
    assert np.allclose(v, [0.004996, 0.001999], rtol=1e-12, atol=0)
    expect = [-lr * (28 / 19) / (np.sqrt(4996 / 1999) + eps), lr / (19 * (1 + eps))]
    assert np.allclose(p - first, expect, rtol=1e-11, atol=0)


# --------------------------------------------------------------------------- #
# Reduced-precision grids (definitions of BF16 and OCP E4M3)
def test_bf16_rounding_grid():
    assert oracle.to_bf16(1 + 2 ** -8) == 1.0             # tie to even
    assert oracle.to_bf16(1 + 3 * 2 ** -8) == 1 + 2 ** -6  # tie to even (up)
    assert oracle.to_bf16(1 + 2 ** -8 + 2 ** -20) == 1 + 2 ** -7
    torch = pytest.importorskip("torch")
    v = np.random.default_rng(3).standard_normal(2000).astype(np.float32) * 10
    ref = torch.from_numpy(v).to(torch.bfloat16).to(torch.float64).numpy()
    assert np.array_equal(oracle.to_bf16(v.astype(np.float64)), ref)


def test_e4m3_rounding_grid():
    assert oracle.to_e4m3(448.0) == 448.0
    assert oracle.to_e4m3(1000.0) == 448.0
    assert oracle.to_e4m3(2.0 ** -9) == 2.0 ** -9            # smallest subnormal
    assert oracle.to_e4m3(1.0625) == 1.0                      # tie to even
    assert oracle.to_e4m3(1.1875) == 1.25
    torch = pytest.importorskip("torch")
    if not hasattr(torch, "float8_e4m3fn"):
        pytest.skip("no float8 in this torch")
    v = (np.random.default_rng(4).standard_normal(2000) * 40).astype(np.float32)
    v = np.clip(v, -440, 440)
    ref = torch.from_numpy(v).to(torch.float8_e4m3fn).to(torch.float64).numpy()
    assert np.array_equal(oracle.to_e4m3(v.astype(np.float64)), ref)


def test_tlb_hand_computed_and_equality():
    """Section V-E: TLB is the bound over the true distance (distances, not
    their squares), averaged over the pairs, and it is one where the two are
    equal.  The pairs at distance zero have no ratio and are left out.  The
    values below are worked by hand: a squared ratio would give 0.4375, a
    count that kept the zero pair 0.5."""
    lb2 = np.array([1.0, 4.0, 0.0, 9.0, 2.0])
    d2 = np.array([4.0, 16.0, 0.0, 9.0, 8.0])
    # ratios 1/2, 2/4, (none), 3/3, sqrt(2)/sqrt(8) = 1/2
    assert oracle.tlb(lb2, d2) == pytest.approx(0.625, abs=1e-15)
    d = np.random.default_rng(5).uniform(0.1, 40.0, 1000)
    assert oracle.tlb(d, d) == pytest.approx(1.0, abs=1e-15)
    assert oracle.tlb(np.zeros(1000), d) == 0.0
    # linear in the bound's distance: four times the squared bound doubles it
    assert oracle.tlb(d / 16.0, d) == pytest.approx(0.25, abs=1e-15)
    assert oracle.tlb(d / 4.0, d) == pytest.approx(0.5, abs=1e-15)
    assert oracle.tlb(np.zeros(3), np.zeros(3)) == 0.0


def test_tlb_range_on_sfa_bounds():
    """On SFA bounds of real pairs the TLB lies in (0, 1]."""
    X = synth.collection(200, 128, "mix", seed=8)
    var, sel, beta = oracle.learn_bins(X, 200, P=16, l=16, alpha=256)
    W, C = oracle.words(X, sel, beta)
    lbs, ds = [], []
    for a in range(0, 200, 9):
        for b in range(0, 200, 5):
            if a != b:
                lbs.append(oracle.sfa_lb2(C[a], W[b], beta))
                ds.append(oracle.dist2(X[a], X[b]))
    t = oracle.tlb(np.array(lbs), np.array(ds))
    assert 0.0 < t <= 1.0


# --------------------------------------------------------------------------- #
# iSAX (Section IV-D): PAA means, N(0,1) equal-depth breakpoints, mindist.

@pytest.mark.parametrize("alpha", [2, 3, 4, 8, 64, 256])
def test_isax_breakpoints_are_normal_quantiles(alpha):
    """Equal-depth bins of N(0,1): breakpoint a is the a/alpha quantile.
    Pinned to scipy's inverse normal CDF and to symmetry about 0."""
    from scipy.special import ndtri
    b = oracle.isax_breakpoints(alpha)
    assert b.shape == (alpha - 1,)
    assert np.all(np.diff(b) > 0)
    assert np.allclose(b, ndtri(np.arange(1, alpha) / alpha), rtol=0, atol=1e-12)
    assert np.allclose(b, -b[::-1], rtol=0, atol=1e-12)


def test_isax_quartiles_textbook_value():
    """alpha = 4: the quartiles of N(0,1) are 0 and +-0.6744897501960817."""
    b = oracle.isax_breakpoints(4)
    assert abs(b[1]) < 1e-12
    assert abs(b[2] - 0.6744897501960817) < 1e-12 and abs(b[0] + 0.6744897501960817) < 1e-12


@pytest.mark.parametrize("n,l", [(16, 4), (64, 8), (256, 16), (256, 1)])
def test_paa_exact_on_piecewise_constant_series(n, l):
    """A series constant on each of the l segments is its own PAA, and the PAA
    distance of two such series equals their Euclidean distance."""
    rng = np.random.default_rng(n + l)
    seg = n // l
    a = np.repeat(rng.standard_normal(l), seg).astype(np.float32)
    b = np.repeat(rng.standard_normal(l), seg).astype(np.float32)
    assert np.array_equal(oracle.paa(a, l), a[::seg].astype(np.float64))
    d = oracle.dist2(a, b)
    assert abs(oracle.paa_dist2(a, b, l) - d) <= 1e-12 * d


@pytest.mark.parametrize("n,l", [(64, 8), (256, 16)])
@pytest.mark.parametrize("alpha", [4, 256])
def test_isax_lb_below_paa_below_distance_every_pair(n, l, alpha):
    """On every pair of a small z-normalised mix set: the quantised iSAX bound
    <= the PAA distance <= the Euclidean distance."""
    X = synth.collection(48, n, "mix", seed=7 * n + alpha)
    W, M = oracle.isax_words(X, l, alpha)
    for i in range(48):
        for j in range(48):
            lb = oracle.isax_lb2(M[i], W[j], n, alpha)
            pd = oracle.paa_dist2(X[i], X[j], l)
            d = oracle.dist2(X[i], X[j])
            assert lb <= pd * (1 + 1e-12) + 1e-12, (i, j)
            assert pd <= d * (1 + 1e-12) + 1e-12, (i, j)


def test_isax_words_half_open_and_single_symbol():
    """A PAA mean on a breakpoint takes the upper bin; one symbol gives the
    all-zero word and a zero bound."""
    b = oracle.isax_breakpoints(4)
    x = np.repeat(np.array([b[2], b[0] - 1.0, 0.1, 2.0]), 4).astype(np.float32)
    beta_f32 = oracle.isax_breakpoints(4)
    W, M = oracle.isax_words(x, 4, 4)
    expect = [oracle.symbol(m, beta_f32) for m in M[0]]
    assert list(W[0]) == expect and W[0][1] == 0 and W[0][3] == 3
    W1, M1 = oracle.isax_words(x, 4, 1)
    assert np.all(W1 == 0)
    assert oracle.isax_lb2(M1[0] + 5.0, W1[0], 16, 1) == 0.0


@pytest.mark.parametrize("binning", [0, 1])
def test_learn_bins_first_values(binning):
    """selection = 1 keeps pool values 0..l-1 and learns their breakpoints
    exactly as for the same columns chosen by variance: each column's
    breakpoints equal orc_breakpoints of that column of the stride sample."""
    X = synth.collection(900, 64, "mix", seed=61)
    m, P, l, alpha = 300, 8, 6, 16
    var, sel, beta = oracle.learn_bins(X, m, P=P, l=l, alpha=alpha, binning=binning, selection=1)
    assert sel.tolist() == list(range(l))
    rows = (np.arange(m, dtype=np.int64) * X.shape[0]) // m
    F = oracle.dft_pool(X[rows], P)
    for j in range(l):
        assert np.array_equal(beta[j], oracle.breakpoints(F[:, j], alpha, binning))
