"""Pins of the FP64 oracle against what the paper and the mathematics fix.

None of these tests re-evaluates the oracle's own formula: each compares the
oracle with an independent route (exact binomial expansion, closed forms,
integral-image box means, brute force with exact integer weights, a NumPy
moving-sum evaluation of the expansion, finite differences) or checks an
invariant of eq. (3).  The paper prints no worked numerical example.
"""
import math

import numpy as np
import pytest

from paper_1107_4617_amd import workloads as wl

T = 255.0


def _binom_kernel(t, sigma_r, N):
    """phi(t) through the binomial expansion cos^N a = 2^-N sum_n C(N,n) cos((2n-N) a),
    with exact integer binomials and exactly rounded weights (Section 1: a sum of
    exponentials; Section 3: q_N has order N+1)."""
    if N == 0:
        return 1.0
    a = t / (sigma_r * math.sqrt(N))
    return math.fsum((math.comb(N, n) / 2 ** N) * math.cos((2 * n - N) * a) for n in range(N + 1))


# ---------------------------------------------------------------- P1 ---------
def test_shift_identity():
    """cos(x - tau) = cos(tau) cos(x) + sin(tau) sin(x) (Section 1): the rule that
    recombines per-order box sums into the kernel at f(x)."""
    rng = np.random.default_rng(11)
    x = rng.uniform(-50, 50, 10000)
    tau = rng.uniform(-50, 50, 10000)
    lhs = np.cos(x - tau)
    rhs = np.cos(tau) * np.cos(x) + np.sin(tau) * np.sin(x)
    assert np.max(np.abs(lhs - rhs)) < 1e-13


# ---------------------------------------------------------------- P2 ---------
@pytest.mark.parametrize("N", [0, 1, 2, 3, 30, 43, 117, 264])
def test_kernel_matches_binomial_expansion(oracle, N):
    """The oracle's cos^N (repeated squaring) equals the exact finite exponential sum."""
    rng = np.random.default_rng(100 + N)
    sigma = 30.0
    s = sigma * math.sqrt(max(N, 1))
    # |a| <= pi/2, plus a few arguments beyond it where cos < 0 (odd N keeps the sign)
    ts = np.concatenate([rng.uniform(-math.pi / 2, math.pi / 2, 200) * s,
                         rng.uniform(-3.0, 3.0, 50) * s])
    err = max(abs(oracle.kernel(t, sigma, N) - _binom_kernel(t, sigma, N)) for t in ts)
    assert err <= 1e-13, err


def test_kernel_derivative_matches_difference_quotient(oracle):
    for N in (1, 2, 30, 43):
        for t in (-200.0, -31.0, 0.0, 7.5, 120.0):
            h = 1e-4
            fd = (_binom_kernel(t + h, 25.0, N) - _binom_kernel(t - h, 25.0, N)) / (2 * h)
            assert abs(oracle.kernel_deriv(t, 25.0, N) - fd) < 1e-9


# ---------------------------------------------------------------- P3 ---------
def test_gaussian_convergence_rate(oracle):
    """Theorem 3.3, eq. (6): cos^N(t/(sigma sqrt N)) -> exp(-t^2/(2 sigma^2)).
    From log cos u = -u^2/2 - u^4/12 - ..., N * sup_t |phi_N - G| -> 16 e^-2 / 12 = 4/(3 e^2)."""
    sigma = 30.0
    t = np.linspace(0.0, 8 * sigma, 4001)
    G = np.exp(-t ** 2 / (2 * sigma ** 2))
    limit = 4.0 / (3.0 * math.e ** 2)
    prev = None
    for N in (10, 30, 100, 300, 1000, 3000):
        phi = np.array([oracle.kernel(x, sigma, N) for x in t])
        sup = np.max(np.abs(phi - G))
        if prev is not None:
            assert sup < prev  # monotone decrease
        prev = sup
        if N >= 300:
            assert abs(N * sup - limit) / limit < 0.02, (N, N * sup)


# ---------------------------------------------------------------- N_0 --------
@pytest.mark.parametrize("sigma,expect", [(30.0, 30), (25.0, 43), (15.0, 118), (10.0, 264), (60.0, 8)])
def test_order_threshold(oracle, sigma, expect):
    """Section 3.1: N_0 = O(T^2/sigma^2) is the smallest order for which the kernel is
    non-negative and unimodal on [-T, T]; with the eq. (6) scaling that is the smallest N
    with T/(sigma sqrt N) <= pi/2."""
    N0 = oracle.order_for(sigma, T)
    assert N0 == expect
    assert T / (sigma * math.sqrt(N0)) <= math.pi / 2
    assert T / (sigma * math.sqrt(N0 - 1)) > math.pi / 2
    # non-negative on [-T, T] at N_0 (even or odd N)
    ts = np.linspace(-T, T, 2001)
    assert min(oracle.kernel(t, sigma, N0) for t in ts) >= 0.0


# ---------------------------------------------------------------- P4 ---------
@pytest.mark.parametrize("r,N", [(0, 30), (2, 1), (3, 30), (5, 117), (40, 8)])
def test_constant_image_is_fixed(oracle, r, N):
    for c in (0.0, 17.25, 255.0):
        f = np.full((9, 14), c, np.float32)
        out = oracle.bilateral(f, r, 30.0, N)
        assert np.max(np.abs(out - c)) <= 1e-14 * max(c, 1.0)


# ---------------------------------------------------------------- P5 ---------
def _box_mean(f, r):
    """Truncated-window mean through an integral image (Section 2: Sum(F, x, T))."""
    H, W = f.shape
    S = np.zeros((H + 1, W + 1))
    S[1:, 1:] = np.cumsum(np.cumsum(f.astype(np.float64), 0), 1)
    i = np.arange(H)[:, None]
    j = np.arange(W)[None, :]
    y0, y1 = np.maximum(i - r, 0), np.minimum(i + r, H - 1) + 1
    x0, x1 = np.maximum(j - r, 0), np.minimum(j + r, W - 1) + 1
    tot = S[y1, x1] - S[y0, x1] - S[y1, x0] + S[y0, x0]
    cnt = (y1 - y0) * (x1 - x0)
    return tot / cnt


def test_radius_zero_is_identity(oracle):
    f = wl.random_image(11, 13, 3)
    out = oracle.bilateral(f, 0, 30.0, 30)
    assert np.array_equal(out, f.astype(np.float64))


@pytest.mark.parametrize("r", [1, 3, 8, 30])
def test_order_zero_is_box_mean(oracle, r):
    """N = 0 (allowed in Section 3) makes the range kernel constant: eq. (3) becomes the
    normalised moving sum of eq. (2) with a box."""
    f = wl.random_image(15, 21, 4)
    out = oracle.bilateral(f, r, 30.0, 0)
    assert np.max(np.abs(out - _box_mean(f, r))) < 1e-11


def test_wide_range_kernel_is_box_mean(oracle):
    f = wl.random_image(12, 10, 5)
    out = oracle.bilateral(f, 3, 1e9, 30)
    assert np.max(np.abs(out - _box_mean(f, 3))) < 1e-9


# ---------------------------------------------------------------- P6 ---------
def test_shift_scale_and_symmetry_covariance(oracle):
    rng = np.random.default_rng(6)
    f = rng.uniform(0, 200, (13, 17))
    base = oracle.bilateral(f, 3, 25.0, 43)
    # shift: phi depends on differences only
    assert np.max(np.abs(oracle.bilateral(f + 40.0, 3, 25.0, 43) - (base + 40.0))) < 1e-10
    # scale: phi(a t; a sigma) = phi(t; sigma); a = 2 is exact in binary
    assert np.max(np.abs(oracle.bilateral(2.0 * f, 3, 50.0, 43) - 2.0 * base)) < 1e-11
    # transpose and flips: the square window is symmetric
    assert np.max(np.abs(oracle.bilateral(np.ascontiguousarray(f.T), 3, 25.0, 43) - base.T)) < 1e-11
    assert np.max(np.abs(oracle.bilateral(np.ascontiguousarray(f[::-1]), 3, 25.0, 43) - base[::-1])) < 1e-11
    assert np.max(np.abs(oracle.bilateral(np.ascontiguousarray(f[:, ::-1]), 3, 25.0, 43) - base[:, ::-1])) < 1e-11


# ---------------------------------------------------------------- P7 ---------
def test_two_level_closed_form(oracle):
    """Levels a (left block of columns) and b (right): at a pixel of level a whose window
    holds n_a pixels of a and n_b of b, eq. (3) gives
    (n_a a + n_b b phi(b-a)) / (n_a + n_b phi(b-a)), with n_a, n_b counted by hand."""
    H, W, split, r = 10, 12, 5, 2
    a, b = 60.0, 100.0
    sigma, N = 30.0, 30
    f = np.full((H, W), a)
    f[:, split:] = b
    out = oracle.bilateral(f, r, sigma, N)
    phi_ab = _binom_kernel(b - a, sigma, N)
    for i in range(H):
        for j in range(W):
            rows = min(H - 1, i + r) - max(0, i - r) + 1
            c0, c1 = max(0, j - r), min(W - 1, j + r)
            na = rows * max(0, min(c1, split - 1) - c0 + 1)
            nb = rows * max(0, c1 - max(c0, split) + 1)
            if f[i, j] == a:
                expect = (na * a + nb * b * phi_ab) / (na + nb * phi_ab)
            else:
                expect = (nb * b + na * a * phi_ab) / (nb + na * phi_ab)
            assert abs(out[i, j] - expect) < 1e-12


# ---------------------------------------------------------------- P8 ---------
def test_convex_combination_bounds(oracle):
    """With N >= N_0 and data in [0, T] the kernel is non-negative (Section 3), so each output
    is a convex combination of its window."""
    f = wl.random_image(20, 23, 8)
    N0 = oracle.order_for(20.0, T)
    out = oracle.bilateral(f, 4, 20.0, N0)
    from numpy.lib.stride_tricks import sliding_window_view
    pad_lo = np.pad(f.astype(np.float64), 4, constant_values=np.inf)
    pad_hi = np.pad(f.astype(np.float64), 4, constant_values=-np.inf)
    mn = sliding_window_view(pad_lo, (9, 9)).min(axis=(-1, -2))
    mx = sliding_window_view(pad_hi, (9, 9)).max(axis=(-1, -2))
    assert np.all(out >= mn - 1e-12) and np.all(out <= mx + 1e-12)


# ---------------------------------------------------------------- P9 ---------
def _brute(f, r, sigma, N):
    """Pure-Python eq. (3) with the kernel taken as the exact binomial sum of exponentials."""
    H, W = f.shape
    P = np.empty((H, W))
    Q = np.empty((H, W))
    if N == 0:
        w = [1.0]
        om = [0.0]
    else:
        s = sigma * math.sqrt(N)
        w = [math.comb(N, n) / 2 ** N for n in range(N + 1)]
        om = [(2 * n - N) / s for n in range(N + 1)]
    for i in range(H):
        for j in range(W):
            fx = float(f[i, j])
            ps, qs = [], []
            for y in range(max(0, i - r), min(H - 1, i + r) + 1):
                for x in range(max(0, j - r), min(W - 1, j + r) + 1):
                    fy = float(f[y, x])
                    k = math.fsum(wn * math.cos(o * (fy - fx)) for wn, o in zip(w, om))
                    ps.append(k * fy)
                    qs.append(k)
            P[i, j] = math.fsum(ps)
            Q[i, j] = math.fsum(qs)
    return P, Q


@pytest.mark.parametrize("r,N,shape", [(0, 2, (7, 5)), (1, 1, (13, 17)), (3, 30, (16, 16)),
                                       (7, 2, (11, 16)), (20, 30, (9, 13)), (2, 117, (6, 9))])
def test_brute_force_small(oracle, r, N, shape):
    """P and Q are compared (below N_0 the kernel changes sign and the ratio can be
    ill-conditioned); the ratio is compared where Q is bounded away from zero."""
    f = wl.random_image(*shape, seed=9 + r)
    Pr, Qr = _brute(f, r, 30.0, N)
    out, P, Q = oracle.bilateral(f, r, 30.0, N, return_pq=True)
    nwin = (2 * r + 1) ** 2
    assert np.max(np.abs(P - Pr)) <= 1e-13 * nwin * T
    assert np.max(np.abs(Q - Qr)) <= 1e-13 * nwin
    ok = np.abs(Qr) > 0.5
    assert np.max(np.abs(out - Pr / Qr)[ok]) <= 1e-12 * T


# ---------------------------------------------------------------- P10 --------
def _folded_shiftable(f, r, sigma, N):
    """Algorithm 2 with one spatial basis function (the box), in NumPy FP64: fold terms n and
    N-n, form cos/sin channels and their f-weighted copies, box-sum each through an
    integral image, recombine with the shift identity, take the ratio."""
    f = f.astype(np.float64)
    H, W = f.shape

    def box(X):
        S = np.zeros((H + 1, W + 1))
        S[1:, 1:] = np.cumsum(np.cumsum(X, 0), 1)
        i = np.arange(H)[:, None]
        j = np.arange(W)[None, :]
        y0, y1 = np.maximum(i - r, 0), np.minimum(i + r, H - 1) + 1
        x0, x1 = np.maximum(j - r, 0), np.minimum(j + r, W - 1) + 1
        return S[y1, x1] - S[y0, x1] - S[y1, x0] + S[y0, x0]

    P = np.zeros((H, W))
    Q = np.zeros((H, W))
    s = sigma * math.sqrt(N)
    for n in range((N + 1) // 2):
        v = 2.0 * math.comb(N, n) / 2 ** N
        om = (N - 2 * n) / s
        C, S_ = np.cos(om * f), np.sin(om * f)
        P += v * (C * box(f * C) + S_ * box(f * S_))
        Q += v * (C * box(C) + S_ * box(S_))
    if N % 2 == 0:
        v = math.comb(N, N // 2) / 2 ** N
        P += v * box(f)
        Q += v * box(np.ones_like(f))
    return P / Q


@pytest.mark.parametrize("r,N", [(2, 30), (5, 43), (4, 117), (6, 7)])
def test_folded_moving_sum_evaluation(oracle, r, N):
    f = wl.smooth_image(40, 56, seed=1)
    ref = _folded_shiftable(f, r, 30.0, N)
    out = oracle.bilateral(f, r, 30.0, N)
    assert np.max(np.abs(out - ref)) <= 1e-11 * T


# ---------------------------------------------------------------- P11 --------
@pytest.mark.parametrize("shape,r,sigma,N", [((9, 11), 2, 30.0, 30), ((8, 10), 3, 25.0, 43), ((7, 6), 1, 40.0, 5)])
def test_gradient_matches_central_differences(oracle, shape, r, sigma, N):
    rng = np.random.default_rng(12)
    f = rng.uniform(20, 230, shape)
    g = rng.normal(size=shape)
    gf, gs, u = oracle.bilateral_grad(f, g, r, sigma, N)
    assert np.max(np.abs(u - oracle.bilateral(f, r, sigma, N))) < 1e-12

    def L(ff, ss):
        return float(np.sum(g * oracle.bilateral(ff, r, ss, N)))

    h = 1e-3
    fd = np.empty(shape)
    for i in range(shape[0]):
        for j in range(shape[1]):
            fp = f.copy(); fp[i, j] += h
            fm = f.copy(); fm[i, j] -= h
            fd[i, j] = (L(fp, sigma) - L(fm, sigma)) / (2 * h)
    assert np.max(np.abs(gf - fd)) <= 1e-6 * np.max(np.abs(fd))
    fds = (L(f, sigma + h) - L(f, sigma - h)) / (2 * h)
    assert abs(gs - fds) <= 1e-6 * abs(fds)


# ---------------------------------------------------------------- P12 --------
@pytest.mark.parametrize("N,eps", [(30, 1e-7), (117, 1e-7), (264, 1e-7), (43, 1e-4)])
def test_truncation_bound_and_counts(oracle, N, eps):
    """Discarding basis functions with w_n < eps (Section 3.1) changes the kernel by at most
    the dropped weight mass, everywhere."""
    kept, dropped = oracle.trunc_terms(N, eps)
    exact_w = [math.comb(N, n) / 2 ** N for n in range(N + 1)]
    assert kept == sum(1 for w in exact_w if w >= eps)
    assert abs(dropped - math.fsum(w for w in exact_w if w < eps)) <= 1e-12 * max(dropped, 1e-300)
    sigma = 15.0
    ts = np.linspace(-T, T, 1001)
    dev = max(abs(oracle.kernel(t, sigma, N) - oracle.trunc_kernel(t, sigma, N, eps)) for t in ts)
    # plus the rounding of log-gamma weights, |lgamma(N+1)| * 2^-52 ~ 3e-13 at N = 264
    assert dev <= dropped + 1e-12


def test_truncated_filter_reduces_to_exact_when_nothing_dropped(oracle):
    f = wl.random_image(10, 12, 13)
    a = oracle.bilateral(f, 2, 30.0, 30)
    b = oracle.bilateral(f, 2, 30.0, 30, eps=0.0, truncated=True)
    assert np.max(np.abs(a - b)) < 1e-11


def _brute_truncated(f, r, sigma, N, eps, pixels):
    """The truncated filter by brute force, independent of the oracle: the kernel of
    Section 3.1 after discarding every unfolded basis function whose exact weight
    w_n = C(N, n) / 2^N is strictly below eps (the comparison in exact rationals),
    summed per window element with math.fsum."""
    H, W = f.shape
    s = sigma * math.sqrt(N)
    eps_q = Fraction(eps)
    kept = [(math.comb(N, n) / 2 ** N, (2 * n - N) / s) for n in range(N + 1)
            if Fraction(math.comb(N, n), 2 ** N) >= eps_q]
    out = []
    for (i, j) in pixels:
        fx = float(f[i, j])
        ps, qs = [], []
        for y in range(max(0, i - r), min(H - 1, i + r) + 1):
            for x in range(max(0, j - r), min(W - 1, j + r) + 1):
                fy = float(f[y, x])
                k = math.fsum(w * math.cos(om * (fy - fx)) for w, om in kept)
                ps.append(k * fy)
                qs.append(k)
        out.append(math.fsum(ps) / math.fsum(qs))
    return np.array(out), len(kept)


def _eps_cases(N):
    """Thresholds for N: the precision form's 1e-7; one equal to a kept weight (exactly
    representable for N <= 50, so only a strict drop keeps it); and one at 1.5 times a
    weight, which the unfolded rule drops but a rule on the folded weights 2 w_n keeps."""
    w = [Fraction(math.comb(N, n), 2 ** N) for n in range(N + 1)]
    k = next(n for n in range(N + 1) if w[n] >= Fraction(1, 10 ** 4))   # a mid-sized weight
    cases = [1e-7, 1.5 * float(w[k - 1])]
    if N <= 50:
        assert Fraction(float(w[k])) == w[k]
        cases.append(float(w[k]))
    return cases


@pytest.mark.parametrize("N", [30, 117])
def test_truncated_filter_matches_brute_force(oracle, N):
    """Pins the oracle's truncated filter (Section 3.1, less significant basis functions
    discarded) at eps > 0: whole-image and per-pixel entry points against a brute force
    with exact binomial weights and the strict drop w_n < eps, on a non-square image with
    a window that reaches every border."""
    f = wl.rect_image(9, 11, seed=17, n_rect=4)
    sigma, r = (30.0, 3) if N == 30 else (15.0, 2)
    pixels = [(i, j) for i in range(9) for j in range(11)]
    idx = np.array([i * 11 + j for i, j in pixels], dtype=np.int64)
    for eps in _eps_cases(N):
        ref, nkept = _brute_truncated(f, r, sigma, N, eps, pixels)
        kept, _ = oracle.trunc_terms(N, eps)
        assert kept == nkept, (N, eps)
        full = oracle.bilateral(f, r, sigma, N, eps=eps, truncated=True).ravel()
        at = oracle.bilateral_at(f, idx, r, sigma, N, eps=eps, truncated=True)
        assert np.max(np.abs(full - ref)) <= 1e-11 * T, (N, eps)
        assert np.max(np.abs(at - ref)) <= 1e-11 * T, (N, eps)


def test_truncation_threshold_is_strict_and_unfolded(oracle):
    """At eps equal to a kept weight that weight stays (drop only w_n < eps); at 1.5 times
    a weight that weight goes although its folded pair weight 2 w_n exceeds eps."""
    N = 30
    w = [math.comb(N, n) / 2 ** N for n in range(N + 1)]
    k = 9
    assert oracle.trunc_terms(N, w[k])[0] == sum(1 for x in w if x >= w[k]) == N + 1 - 2 * k
    assert oracle.trunc_terms(N, 1.5 * w[k])[0] == N + 1 - 2 * (k + 1)
    sigma = 30.0
    s = sigma * math.sqrt(N)
    for t in (0.0, 13.0, 77.0, 200.0):
        exact_keep = math.fsum(w[n] * math.cos((2 * n - N) * t / s) for n in range(k, N + 1 - k))
        assert abs(oracle.trunc_kernel(t, sigma, N, w[k]) - exact_keep) <= 1e-15
        drop_k = math.fsum(w[n] * math.cos((2 * n - N) * t / s) for n in range(k + 1, N - k))
        assert abs(oracle.trunc_kernel(t, sigma, N, 1.5 * w[k]) - drop_k) <= 1e-15


def test_sampled_matches_full(oracle):
    f = wl.rect_image(40, 50, seed=2)
    full, P, Q = oracle.bilateral(f, 6, 30.0, 30, return_pq=True)
    idx = np.array([0, 7, 49, 50, 1999, 1234, 999])
    o, p, q = oracle.bilateral_at(f, idx, 6, 30.0, 30, return_pq=True)
    assert np.array_equal(o, full.ravel()[idx])
    assert np.array_equal(p, P.ravel()[idx]) and np.array_equal(q, Q.ravel()[idx])


def test_huge_radius_covers_whole_image(oracle):
    f = wl.random_image(6, 9, 14)
    a = oracle.bilateral(f, 9, 30.0, 30)
    b = oracle.bilateral(f, 2 ** 30, 30.0, 30)
    assert np.array_equal(a, b)
    # every pixel sees every pixel: compare with direct whole-image sums
    ff = f.astype(np.float64).ravel()
    for x in (0, 17, 53):
        k = np.array([_binom_kernel(fy - ff[x], 30.0, 30) for fy in ff])
        assert abs(a.ravel()[x] - (k * ff).sum() / k.sum()) < 1e-10


# ---------------------------------------------------------------- P13 --------
# The separable raised-cosine spatial kernel of Algorithms 1 and 2 with M > 1.
def _binom_spatial(d, sigma_s, Ns):
    """w(d) = cos^Ns(d / (sigma_s sqrt Ns)) as the exact binomial sum of cosines: order of
    shiftability Ns + 1 per axis (Section 3), M = (Ns + 1)^2 in two dimensions."""
    return _binom_kernel(d, sigma_s, Ns)


@pytest.mark.parametrize("Ns", [0, 1, 2, 3, 4, 9])
def test_spatial_weight_matches_binomial_expansion(oracle, Ns):
    for d in range(-12, 13):
        assert abs(oracle.spatial_weight(d, 3.0, Ns) - _binom_spatial(d, 3.0, Ns)) <= 1e-14


def test_spatial_weight_gaussian_limit(oracle):
    """Eq. (6) applied to the spatial kernel: w_Ns(d) -> exp(-d^2 / (2 sigma_s^2)) with the
    error decaying like 1/Ns (the same constant 4/(3e^2) as the range kernel)."""
    sigma_s = 2.5
    for Ns in (400, 1600):
        d = np.linspace(-4 * sigma_s, 4 * sigma_s, 801)
        w = np.array([oracle.spatial_weight(x, sigma_s, Ns) for x in d])
        sup = np.max(np.abs(w - np.exp(-d * d / (2 * sigma_s ** 2))))
        assert abs(Ns * sup - 4 / (3 * math.e ** 2)) < 0.02 * 4 / (3 * math.e ** 2)


def test_spatial_order_zero_is_the_box(oracle):
    """Ns = 0 makes every spatial weight 1: the *_sp entry points equal the box ones."""
    f = wl.random_image(19, 23, 31)
    for r, N in ((0, 30), (2, 30), (4, 0), (30, 7)):
        assert np.array_equal(oracle.bilateral_sp(f, r, 30.0, N, 2.0, 0), oracle.bilateral(f, r, 30.0, N))


@pytest.mark.parametrize("r,sigma_s,Ns", [(1, 1.0, 1), (3, 2.0, 2), (5, 2.25, 2), (6, 3.0, 4), (9, 2.0, 7)])
def test_algorithm1_is_normalised_separable_correlation(oracle, r, sigma_s, Ns):
    """N = 0 (range kernel 1) is Algorithm 1: the normalised linear filter
    sum_y w(y-x) f(y) / sum_y w(y-x) over the truncated window.  With zero padding this is
    a separable correlation of f and of the indicator of the image, done here with
    scipy.ndimage along each axis."""
    from scipy import ndimage
    f = wl.random_image(37, 41, 40 + r).astype(np.float64)
    k1 = np.array([_binom_spatial(d, sigma_s, Ns) for d in range(-r, r + 1)])
    def sep(a):
        a = ndimage.correlate1d(a, k1, axis=0, mode="constant", cval=0.0)
        return ndimage.correlate1d(a, k1, axis=1, mode="constant", cval=0.0)
    ref = sep(f) / sep(np.ones_like(f))
    out = oracle.bilateral_sp(f, r, 30.0, 0, sigma_s, Ns)
    assert np.max(np.abs(out - ref)) <= 1e-11 * T


def _brute_sp(f, r, sigma, N, sigma_s, Ns):
    """Pure-Python Algorithm 2 definition with the spatial weights and the range kernel both
    taken as exact binomial sums of cosines."""
    H, W = f.shape
    P = np.empty((H, W))
    Q = np.empty((H, W))
    ws = {d: _binom_spatial(d, sigma_s, Ns) for d in range(-r, r + 1)}
    for i in range(H):
        for j in range(W):
            fx = float(f[i, j])
            ps, qs = [], []
            for y in range(max(0, i - r), min(H - 1, i + r) + 1):
                for x in range(max(0, j - r), min(W - 1, j + r) + 1):
                    fy = float(f[y, x])
                    k = ws[y - i] * ws[x - j] * _binom_kernel(fy - fx, sigma, N)
                    ps.append(k * fy)
                    qs.append(k)
            P[i, j] = math.fsum(ps)
            Q[i, j] = math.fsum(qs)
    return P, Q


@pytest.mark.parametrize("r,N,sigma_s,Ns,shape", [(1, 4, 1.0, 1, (7, 9)), (2, 30, 2.0, 2, (11, 8)),
                                                   (4, 5, 2.5, 3, (9, 12)), (3, 117, 1.5, 4, (6, 10))])
def test_spatial_brute_force_small(oracle, r, N, sigma_s, Ns, shape):
    f = wl.random_image(*shape, seed=70 + r)
    sig = 30.0 if N >= 30 else 200.0
    Pr, Qr = _brute_sp(f, r, sig, N, sigma_s, Ns)
    out, P, Q = oracle.bilateral_sp(f, r, sig, N, sigma_s, Ns, return_pq=True)
    nwin = (2 * r + 1) ** 2
    assert np.max(np.abs(P - Pr)) <= 1e-13 * nwin * T
    assert np.max(np.abs(Q - Qr)) <= 1e-13 * nwin
    ok = np.abs(Qr) > 0.1
    assert np.max(np.abs(out - Pr / Qr)[ok]) <= 1e-12 * T


def test_spatial_filter_invariants(oracle):
    """Constant images are fixed; transposing or flipping the image transposes or flips
    the result (the spatial kernel is separable, symmetric and the same on both axes);
    adding a constant shifts the result (the range kernel sees differences only)."""
    f = wl.random_image(14, 19, 77)
    a = oracle.bilateral_sp(f, 3, 30.0, 30, 2.0, 2)
    assert np.max(np.abs(oracle.bilateral_sp(np.full((9, 8), 99.0), 3, 30.0, 30, 2.0, 2) - 99.0)) < 1e-12
    assert np.max(np.abs(oracle.bilateral_sp(np.ascontiguousarray(f.T), 3, 30.0, 30, 2.0, 2) - a.T)) < 1e-11
    assert np.max(np.abs(oracle.bilateral_sp(np.ascontiguousarray(f[::-1, ::-1]), 3, 30.0, 30, 2.0, 2)
                         - a[::-1, ::-1])) < 1e-11
    b = oracle.bilateral_sp(f.astype(np.float64) + 17.0, 3, 30.0, 30, 2.0, 2)
    assert np.max(np.abs(b - (a + 17.0))) < 1e-10


def test_spatial_sampled_matches_full(oracle):
    f = wl.rect_image(30, 40, seed=2)
    full = oracle.bilateral_sp(f, 5, 30.0, 30, 2.25, 2)
    idx = np.array([0, 7, 39, 40, 1199, 345, 777])
    assert np.array_equal(oracle.bilateral_sp_at(f, idx, 5, 30.0, 30, 2.25, 2), full.ravel()[idx])


# ------------------------------------------------ polynomial range kernel ----
# Section 3's p_N(t) = (1 - t^2/T^2)^N in the scaling of eq. (5), with T = sqrt(2) sigma_r:
# phi(t) = (1 - t^2 / (2 N sigma_r^2))^N.
from fractions import Fraction


def _poly_exact(t, sigma, N):
    """phi(t) as an exact rational through the binomial theorem,
    (1 - u)^N = sum_m C(N, m) (-u)^m with u = t^2 / (2 N sigma^2); t and sigma rational."""
    if N == 0:
        return Fraction(1)
    u = Fraction(t) ** 2 / (2 * N * Fraction(sigma) ** 2)
    return sum(math.comb(N, m) * (-u) ** m for m in range(N + 1))


@pytest.mark.parametrize("N", [0, 1, 2, 5, 37, 145])
def test_poly_kernel_matches_exact_binomial_expansion(oracle, N):
    for t in [0, 1, 7, 30, 99, 180, 255]:
        exact = _poly_exact(t, 30, N)
        got = oracle.poly_kernel(float(t), 30.0, N)
        assert abs(got - float(exact)) <= 1e-14 * max(1.0, abs(float(exact))), (t, N)


def test_poly_gaussian_limit_rate(oracle):
    """Eq. (5): p_N(t / sqrt N) tends to the Gaussian; the error decays like 1/N
    (log(1 - u/N) N = -u - u^2/(2N) - ...)."""
    sigma = 30.0
    ts = np.linspace(0.0, 120.0, 241)

    def err(N):
        return max(abs(oracle.poly_kernel(t, sigma, N) - math.exp(-t * t / (2 * sigma * sigma))) for t in ts)

    e1, e2, e4 = err(50), err(100), err(200)
    assert e4 < 1e-2
    assert 1.8 < e1 / e2 < 2.2 and 1.8 < e2 / e4 < 2.2


@pytest.mark.parametrize("sigma,expect", [(30.0, 37), (60.0, 10), (15.0, 145), (25.0, 53), (255.0, 1)])
def test_poly_order_threshold(oracle, sigma, expect):
    """N_p is the smallest order with the kernel non-negative and non-increasing on [0, T];
    one order less puts the polynomial's zero sigma sqrt(2N) inside [0, T), past which
    (1 - u)^N changes sign (odd N) or grows again (even N)."""
    assert oracle.poly_order_for(sigma, T) == expect
    ts = np.linspace(0.0, T, 4001)
    v = np.array([oracle.poly_kernel(t, sigma, expect) for t in ts])
    assert np.all(v >= 0.0) and np.all(np.diff(v) <= 0.0)
    base = lambda N: 1 - Fraction(T) ** 2 / (2 * N * Fraction(sigma) ** 2)   # 1 - u at t = T
    assert base(expect) >= 0
    if expect > 1:
        assert base(expect - 1) < 0


@pytest.mark.parametrize("r", [1, 4, 11])
def test_poly_order_zero_is_box_mean(oracle, r):
    f = wl.random_image(15, 19, 3)
    assert np.max(np.abs(oracle.bilateral_poly(f, r, 30.0, 0) - _box_mean(f, r))) < 1e-9


def _brute_poly_exact(f, r, sigma, N):
    """Eq. (3) in exact rational arithmetic for an integer-valued image."""
    H, W = f.shape
    P = np.empty((H, W))
    Q = np.empty((H, W))
    cache = {}
    for i in range(H):
        for j in range(W):
            fx = int(f[i, j])
            p = q = Fraction(0)
            for y in range(max(0, i - r), min(H - 1, i + r) + 1):
                for x in range(max(0, j - r), min(W - 1, j + r) + 1):
                    fy = int(f[y, x])
                    d = fy - fx
                    if d not in cache:
                        cache[d] = _poly_exact(d, sigma, N)
                    k = cache[d]
                    p += k * fy
                    q += k
            P[i, j] = float(p)
            Q[i, j] = float(q)
    return P, Q


@pytest.mark.parametrize("r,N,sigma,shape", [(1, 1, 30, (6, 7)), (2, 37, 30, (7, 9)), (3, 10, 60, (8, 6)),
                                             (0, 4, 30, (5, 5)), (2, 145, 15, (6, 6))])
def test_poly_brute_force_exact_rationals(oracle, r, N, sigma, shape):
    rng = np.random.default_rng(40 + N)
    f = rng.integers(0, 256, shape).astype(np.float64)
    Pr, Qr = _brute_poly_exact(f, r, sigma, N)
    out, P, Q = oracle.bilateral_poly(f, r, float(sigma), N, return_pq=True)
    nwin = (2 * r + 1) ** 2
    assert np.max(np.abs(P - Pr)) <= 1e-13 * nwin * T
    assert np.max(np.abs(Q - Qr)) <= 1e-13 * nwin
    assert np.max(np.abs(out - Pr / Qr)) <= 1e-12 * T


def _monomial_shiftable(f, r, sigma, N):
    """Algorithm 2 for the polynomial kernel in the monomial basis (its shiftability,
    Section 1): phi(s - c) = sum_k a_k(c) s^k, so P = sum_k a_k(f_x) Box[f^(k+1)] and
    Q = sum_k a_k(f_x) Box[f^k].  Data are centred and scaled first (the filter is shift and
    scale covariant), and the expansion is only well conditioned for small N."""
    from numpy.polynomial import polynomial as Pl
    f = f.astype(np.float64)
    H, W = f.shape
    mu, rho = 0.5 * (f.min() + f.max()), 0.5 * (f.max() - f.min())
    g = (f - mu) / rho
    a2 = 2.0 * N * (sigma / rho) ** 2

    def box(X):
        S = np.zeros((H + 1, W + 1))
        S[1:, 1:] = np.cumsum(np.cumsum(X, 0), 1)
        i = np.arange(H)[:, None]
        j = np.arange(W)[None, :]
        y0, y1 = np.maximum(i - r, 0), np.minimum(i + r, H - 1) + 1
        x0, x1 = np.maximum(j - r, 0), np.minimum(j + r, W - 1) + 1
        return S[y1, x1] - S[y0, x1] - S[y1, x0] + S[y0, x0]

    M = [box(g ** k) for k in range(2 * N + 2)]
    P = np.zeros((H, W))
    Q = np.zeros((H, W))
    for i in range(H):
        for j in range(W):
            c = g[i, j]
            a = Pl.polypow([1.0 - c * c / a2, 2.0 * c / a2, -1.0 / a2], N)
            Q[i, j] = sum(a[k] * M[k][i, j] for k in range(len(a)))
            P[i, j] = sum(a[k] * M[k + 1][i, j] for k in range(len(a)))
    return mu + rho * P / Q


@pytest.mark.parametrize("r,N,sigma", [(2, 1, 60.0), (3, 3, 60.0), (4, 6, 80.0), (2, 10, 60.0)])
def test_poly_monomial_moving_sum_evaluation(oracle, r, N, sigma):
    f = wl.smooth_image(30, 41, seed=2)
    ref = _monomial_shiftable(f, r, sigma, N)
    out = oracle.bilateral_poly(f, r, sigma, N)
    assert np.max(np.abs(out - ref)) <= 1e-9 * T


def test_poly_invariants(oracle):
    rng = np.random.default_rng(16)
    f = rng.uniform(0, 200, (13, 17))
    base = oracle.bilateral_poly(f, 3, 30.0, 37)
    # constant image, shift, scale (a = 2 exact in binary), transpose and flips
    assert np.max(np.abs(oracle.bilateral_poly(np.full((9, 8), 77.0), 2, 30.0, 37) - 77.0)) < 1e-12
    assert np.max(np.abs(oracle.bilateral_poly(f + 40.0, 3, 30.0, 37) - (base + 40.0))) < 1e-10
    assert np.max(np.abs(oracle.bilateral_poly(2.0 * f, 3, 60.0, 37) - 2.0 * base)) < 1e-11
    assert np.max(np.abs(oracle.bilateral_poly(np.ascontiguousarray(f.T), 3, 30.0, 37) - base.T)) < 1e-11
    assert np.max(np.abs(oracle.bilateral_poly(np.ascontiguousarray(f[::-1]), 3, 30.0, 37) - base[::-1])) < 1e-11
    # N >= N_p on data in [0, T]: a convex combination of the window
    g = wl.random_image(20, 23, 8)
    out = oracle.bilateral_poly(g, 4, 20.0, oracle.poly_order_for(20.0, T))
    from numpy.lib.stride_tricks import sliding_window_view
    mn = sliding_window_view(np.pad(g.astype(np.float64), 4, constant_values=np.inf), (9, 9)).min(axis=(-1, -2))
    mx = sliding_window_view(np.pad(g.astype(np.float64), 4, constant_values=-np.inf), (9, 9)).max(axis=(-1, -2))
    assert np.all(out >= mn - 1e-12) and np.all(out <= mx + 1e-12)


def test_poly_two_level_closed_form(oracle):
    """Two levels a | b: (n_a a + n_b b phi(b-a)) / (n_a + n_b phi(b-a)) with phi exact."""
    H, W, split, r = 9, 11, 4, 2
    a, b, sigma, N = 60.0, 100.0, 30, 37
    f = np.full((H, W), a)
    f[:, split:] = b
    out = oracle.bilateral_poly(f, r, float(sigma), N)
    phi = float(_poly_exact(b - a, sigma, N))
    for i in range(H):
        for j in range(W):
            rows = min(H - 1, i + r) - max(0, i - r) + 1
            c0, c1 = max(0, j - r), min(W - 1, j + r)
            na = rows * max(0, min(c1, split - 1) - c0 + 1)
            nb = rows * max(0, c1 - max(c0, split) + 1)
            if f[i, j] == a:
                expect = (na * a + nb * b * phi) / (na + nb * phi)
            else:
                expect = (nb * b + na * a * phi) / (nb + na * phi)
            assert abs(out[i, j] - expect) < 1e-12


def test_poly_gaussian_bilateral_limit(oracle):
    """As N grows the filter approaches the Gaussian-range bilateral (eq. (5)), here by
    direct NumPy window sums; the gap shrinks about in proportion to 1/N."""
    f = wl.smooth_image(24, 28, seed=5).astype(np.float64)
    r, sigma = 3, 30.0
    H, W = f.shape
    g = np.empty_like(f)
    for i in range(H):
        for j in range(W):
            w = f[max(0, i - r):i + r + 1, max(0, j - r):j + r + 1]
            k = np.exp(-((w - f[i, j]) ** 2) / (2 * sigma * sigma))
            g[i, j] = (k * w).sum() / k.sum()
    gaps = [np.max(np.abs(oracle.bilateral_poly(f, r, sigma, N) - g)) for N in (40, 80, 160)]
    assert gaps[2] < 0.1
    assert 1.6 < gaps[0] / gaps[1] < 2.4 and 1.6 < gaps[1] / gaps[2] < 2.4


def test_poly_sampled_matches_full(oracle):
    f = wl.rect_image(40, 50, seed=7)
    full = oracle.bilateral_poly(f, 5, 30.0, 37)
    idx = np.array([0, 49, 50 * 39, 40 * 50 - 1, 777, 1234, 1500])
    assert np.array_equal(oracle.bilateral_poly_at(f, idx, 5, 30.0, 37), full.ravel()[idx])


# ------------------------------------ two-pixel-patch non-local means (Section 5) ----
@pytest.mark.parametrize("offset", [(0, 1), (1, 0), (-2, 3)])
def test_nlm2_second_order_zero_is_bilateral(oracle, offset):
    """N2 = 0 drops the second patch pixel: the bilateral filter of eq. (3)."""
    f = wl.random_image(14, 17, 2)
    a = oracle.nlm2(f, 3, 30.0, 30, 40.0, 0, offset)
    assert np.max(np.abs(a - oracle.bilateral(f, 3, 30.0, 30))) < 1e-12


def test_nlm2_zero_offset_closed_form(oracle):
    """u = 0 compares each pixel twice: cos^N(t / (s sqrt N))^2 = cos^2N(t / ((s / sqrt 2) sqrt 2N)),
    the bilateral filter of order 2N at sigma_r / sqrt 2."""
    f = wl.random_image(12, 15, 3)
    a = oracle.nlm2(f, 2, 50.0, 9, 50.0, 9, (0, 0))
    b = oracle.bilateral(f, 2, 50.0 / math.sqrt(2.0), 18)
    assert np.max(np.abs(a - b)) < 1e-10


def _nlm2_brute(f, r, s1, N1, s2, N2, off):
    """Eq. (NL) with p = 2 in pure Python, each factor as its exact binomial sum of cosines."""
    H, W = f.shape
    uy, ux = off
    fe = lambda i, j: float(f[min(max(i, 0), H - 1), min(max(j, 0), W - 1)])
    out = np.empty((H, W))
    for i in range(H):
        for j in range(W):
            fx, gx = float(f[i, j]), fe(i + uy, j + ux)
            ps, qs = [], []
            for y in range(max(0, i - r), min(H - 1, i + r) + 1):
                for x in range(max(0, j - r), min(W - 1, j + r) + 1):
                    k = _binom_kernel(float(f[y, x]) - fx, s1, N1) * _binom_kernel(fe(y + uy, x + ux) - gx, s2, N2)
                    ps.append(k * float(f[y, x]))
                    qs.append(k)
            out[i, j] = math.fsum(ps) / math.fsum(qs)
    return out


@pytest.mark.parametrize("r,N1,N2,off,shape", [(1, 30, 14, (0, 1), (7, 9)), (2, 30, 20, (1, 0), (9, 8)),
                                               (3, 31, 15, (-1, 2), (8, 11))])
def test_nlm2_brute_force_small(oracle, r, N1, N2, off, shape):
    """Orders at or above N_0 of each factor (30 at sigma 30, 14 at sigma 45), so the kernel
    is non-negative and the ratio well conditioned."""
    f = wl.random_image(*shape, seed=21 + r)
    ref = _nlm2_brute(f, r, 30.0, N1, 45.0, N2, off)
    assert np.max(np.abs(oracle.nlm2(f, r, 30.0, N1, 45.0, N2, off) - ref)) <= 1e-11 * T


def _nlm2_shiftable(f, r, s1, N1, s2, N2, off):
    """Algorithm 2 with the two-pixel patch in NumPy FP64: the product kernel expands into
    cos(w1 t1 + w2 t2) terms (all w1, folded w2), each giving the channels cos(psi), sin(psi),
    f cos(psi), f sin(psi) of the patch phase psi(z) = w1 f(z) + w2 fe(z + u), box-summed through
    integral images and recombined by the shift identity."""
    f = f.astype(np.float64)
    H, W = f.shape
    uy, ux = off
    ii = np.clip(np.arange(H) + uy, 0, H - 1)
    jj = np.clip(np.arange(W) + ux, 0, W - 1)
    g = f[ii][:, jj]

    def box(X):
        S = np.zeros((H + 1, W + 1))
        S[1:, 1:] = np.cumsum(np.cumsum(X, 0), 1)
        i = np.arange(H)[:, None]
        j = np.arange(W)[None, :]
        y0, y1 = np.maximum(i - r, 0), np.minimum(i + r, H - 1) + 1
        x0, x1 = np.maximum(j - r, 0), np.minimum(j + r, W - 1) + 1
        return S[y1, x1] - S[y0, x1] - S[y1, x0] + S[y0, x0]

    terms1 = [(math.comb(N1, n) / 2 ** N1, (2 * n - N1) / (s1 * math.sqrt(N1)) if N1 else 0.0)
              for n in range(N1 + 1)]
    terms2 = []
    for n in range((N2 + 1) // 2):
        terms2.append((2.0 * math.comb(N2, n) / 2 ** N2, (N2 - 2 * n) / (s2 * math.sqrt(N2))))
    if N2 % 2 == 0:
        terms2.append((math.comb(N2, N2 // 2) / 2 ** N2, 0.0))
    P = np.zeros((H, W))
    Q = np.zeros((H, W))
    for w1, om1 in terms1:
        for w2, om2 in terms2:
            psi = om1 * f + om2 * g
            C, S_ = np.cos(psi), np.sin(psi)
            P += w1 * w2 * (C * box(f * C) + S_ * box(f * S_))
            Q += w1 * w2 * (C * box(C) + S_ * box(S_))
    return P / Q


@pytest.mark.parametrize("r,N1,N2,off", [(2, 8, 8, (0, 1)), (3, 10, 6, (2, -1)), (4, 5, 9, (1, 1))])
def test_nlm2_moving_sum_evaluation(oracle, r, N1, N2, off):
    f = wl.smooth_image(30, 37, seed=4)
    ref = _nlm2_shiftable(f, r, 60.0, N1, 70.0, N2, off)
    assert np.max(np.abs(oracle.nlm2(f, r, 60.0, N1, 70.0, N2, off) - ref)) <= 1e-10 * T


def test_nlm2_invariants(oracle):
    rng = np.random.default_rng(26)
    f = rng.uniform(0, 200, (13, 16))
    base = oracle.nlm2(f, 3, 30.0, 30, 40.0, 20, (1, 2))
    assert np.max(np.abs(oracle.nlm2(np.full((9, 8), 77.0), 2, 30.0, 30, 40.0, 20, (1, 2)) - 77.0)) < 1e-12
    assert np.max(np.abs(oracle.nlm2(f + 40.0, 3, 30.0, 30, 40.0, 20, (1, 2)) - (base + 40.0))) < 1e-10
    assert np.max(np.abs(oracle.nlm2(2.0 * f, 3, 60.0, 30, 80.0, 20, (1, 2)) - 2.0 * base)) < 1e-11
    # transposing the image transposes the offset; flipping the rows negates its row part
    assert np.max(np.abs(oracle.nlm2(np.ascontiguousarray(f.T), 3, 30.0, 30, 40.0, 20, (2, 1)) - base.T)) < 1e-11
    assert np.max(np.abs(oracle.nlm2(np.ascontiguousarray(f[::-1]), 3, 30.0, 30, 40.0, 20, (-1, 2))
                         - base[::-1])) < 1e-11


def test_nlm2_sampled_matches_full(oracle):
    f = wl.rect_image(40, 50, seed=7)
    full = oracle.nlm2(f, 5, 30.0, 30, 40.0, 20, (0, 1))
    idx = np.array([0, 49, 50 * 39, 40 * 50 - 1, 777, 1234])
    assert np.array_equal(oracle.nlm2_at(f, idx, 5, 30.0, 30, 40.0, 20, (0, 1)), full.ravel()[idx])
