"""Pins of the CPU oracle against facts fixed by the paper and by mathematics
(hand-enumerated cases, textbook reductions, closed forms, invariants), so that
the oracle is trusted before any GPU result is compared with it."""
import math

import numpy as np
import pytest

import oracle


# ---------------------------------------------------------------- ECDF / ESF
def test_hand_points_d2(golden):
    g = golden["points_d2"]
    x = np.array(g["x"], dtype=float)
    y = np.array(g["y"], dtype=float)
    assert list(oracle.ecdf(x, x)) == g["ecdf_counts"]
    assert list(oracle.esf(x, x)) == g["esf_counts"]
    s, _ = oracle.dominance_sums(x, x, y)
    assert list(s) == g["ecdf_weighted_sums"]
    s, _ = oracle.dominance_sums(x, x, y, survival=True)
    assert list(s) == g["esf_weighted_sums"]
    f, _ = oracle.ecdf(x, x, y)
    np.testing.assert_array_equal(f, np.array(g["ecdf_weighted_sums"]) / 5.0)


def test_hand_grid_d2(golden):
    g = golden["grid_d2"]
    x = np.array(g["x"], dtype=float)
    z = oracle.grid_points(g["nodes"])
    assert oracle.ecdf(x, z).reshape(3, 3).tolist() == g["ecdf_counts"]
    assert oracle.esf(x, z).reshape(3, 3).tolist() == g["esf_counts"]


def test_d1_matches_searchsorted():
    """d = 1: the ECDF count is the upper-bound rank in the sorted sample."""
    g = np.random.default_rng(1)
    x = np.round(g.normal(size=3000), 2)  # ties on purpose
    z = np.concatenate([np.round(g.normal(size=500), 2), x[:200], [-np.inf, np.inf]])
    xs = np.sort(x)
    want = np.searchsorted(xs, z, side="right")
    np.testing.assert_array_equal(oracle.ecdf(x, z), want)
    np.testing.assert_array_equal(oracle.esf(x, z), x.size - want)


def test_inclusion_exclusion_d2_d3():
    """ESF(z) = sum over subsets S of (-1)^|S| ECDF_S(z_S) for counts, where
    ECDF_S only constrains the coordinates in S (ECDF of the empty set = N)."""
    g = np.random.default_rng(2)
    for d in (2, 3):
        x = np.round(g.normal(size=(d, 800)), 1)
        z = np.concatenate([np.round(g.normal(size=(d, 300)), 1), x[:, :50]], axis=1)
        n = x.shape[1]
        total = np.zeros(z.shape[1], dtype=np.int64)
        for mask in range(1 << d):
            ks = [k for k in range(d) if mask >> k & 1]
            term = np.full(z.shape[1], n, dtype=np.int64) if not ks else oracle.ecdf(x[ks], z[ks])
            total += (-1) ** len(ks) * term
        np.testing.assert_array_equal(oracle.esf(x, z), total)


def test_grid_invariants():
    g = np.random.default_rng(3)
    x = g.normal(size=(3, 2000))
    y = g.integers(-3, 4, size=2000).astype(float)
    nodes = [np.linspace(x[k].min(), x[k].max(), 7) for k in range(3)]
    for k in range(3):
        nodes[k][-1] = x[k].max()
    z = oracle.grid_points(nodes)
    cnt = oracle.ecdf(x, z).reshape(7, 7, 7)
    bar = oracle.esf(x, z).reshape(7, 7, 7)
    for ax in range(3):
        assert np.all(np.diff(cnt, axis=ax) >= 0)
        assert np.all(np.diff(bar, axis=ax) <= 0)
    assert cnt[-1, -1, -1] == x.shape[1]      # top corner dominates every point
    assert bar[-1, -1, -1] == 0
    f, a = oracle.ecdf(x, z, y)
    assert f.reshape(7, 7, 7)[-1, -1, -1] == pytest.approx(y.sum() / x.shape[1], abs=0)
    # integer weights: exact multiples of 1/N (Remark on the 1/N scaling)
    s, _ = oracle.dominance_sums(x, z, y)
    assert np.all(s == np.round(s))
    # ESF below every data point is the total
    zlow = np.full((3, 1), -1e300)
    assert oracle.esf(x, zlow)[0] == x.shape[1]


def test_ties_and_strictness():
    x = np.array([[1.0, 1.0, 2.0], [5.0, 6.0, 5.0]])
    z = np.array([[1.0], [5.0]])
    assert oracle.ecdf(x, z)[0] == 1          # (1,5) itself, <= in both
    assert oracle.esf(x, z)[0] == 0           # (2,5): x2 = 5 is not > 5
    z2 = np.array([[0.5], [4.0]])
    assert oracle.esf(x, z2)[0] == 3


def test_nan_semantics():
    x = np.array([[0.0, np.nan, 1.0], [0.0, 0.0, 1.0]])
    z = np.array([[2.0, np.nan], [2.0, 2.0]])
    np.testing.assert_array_equal(oracle.ecdf(x, z), [2, 0])
    np.testing.assert_array_equal(oracle.esf(x, np.array([[-1.0], [-1.0]])), [2])


def test_permutation_and_monotone_transform_invariance():
    g = np.random.default_rng(4)
    x = np.round(g.normal(size=(3, 1500)), 1)
    z = np.round(g.normal(size=(3, 200)), 1)
    c = oracle.ecdf(x, z)
    p = g.permutation(x.shape[1])
    np.testing.assert_array_equal(oracle.ecdf(x[:, p], z), c)
    # a strictly increasing map applied to both data and queries
    np.testing.assert_array_equal(oracle.ecdf(np.exp(x) ** 3, np.exp(z) ** 3), c)
    e = oracle.esf(x, z)
    np.testing.assert_array_equal(oracle.esf(np.arctan(x), np.arctan(z)), e)


def test_additivity_in_y():
    g = np.random.default_rng(5)
    x = g.normal(size=(2, 1000))
    z = g.normal(size=(2, 100))
    y1 = g.integers(-5, 6, 1000).astype(float)
    y2 = g.integers(-5, 6, 1000).astype(float)
    s1, _ = oracle.dominance_sums(x, z, y1)
    s2, _ = oracle.dominance_sums(x, z, y2)
    s12, _ = oracle.dominance_sums(x, z, y1 + y2)
    np.testing.assert_array_equal(s1 + s2, s12)


def test_compensated_sum_is_near_exact():
    """Weighted sums with heavy cancellation agree with math.fsum (exactly
    rounded) to a couple of ulps of the magnitude scale."""
    g = np.random.default_rng(6)
    n = 20000
    x = g.random((2, n))
    big = g.normal(size=n) * 1e12
    y = np.concatenate([big, -big]) + np.concatenate([g.normal(size=n), g.normal(size=n)])
    x2 = np.concatenate([x, x], axis=1)
    z = g.random((2, 40))
    s, a = oracle.dominance_sums(x2, z, y)
    for q in range(z.shape[1]):
        sel = np.all(x2 <= z[:, q:q + 1], axis=0)
        exact = math.fsum(y[sel])
        assert abs(s[q] - exact) <= 4 * np.finfo(float).eps * abs(exact) + 1e-30 * a[q]


# ---------------------------------------------------------------- Laplacian KDE
def test_kde_hand_d1(golden):
    g = golden["kde_d1"]
    x = np.array([g["x"]])
    f, _ = oracle.kde_laplace(x, np.array([[g["z"]]]), g["h"])
    assert f[0, 0] == pytest.approx(g["f"], rel=1e-15)
    floo, _ = oracle.kde_laplace_loo(x, g["h"])
    assert floo[0, 0] == pytest.approx(g["f_loo_point0"], rel=1e-15)


@pytest.mark.parametrize("d", [1, 2, 3])
def test_kde_single_point_closed_form(d):
    g = np.random.default_rng(7)
    x = g.normal(size=(d, 1))
    z = g.normal(size=(d, 5))
    h = g.uniform(0.2, 2.0, size=(1, d))
    f, _ = oracle.kde_laplace(x, z, h, w=np.array([2.5]))
    want = 2.5 * np.exp(-np.sum(np.abs(x - z) / h[0][:, None], axis=0)) / (2 ** d * np.prod(h))
    np.testing.assert_allclose(f[0], want, rtol=1e-15)


def test_kde_d1_two_sided_recursion():
    """d = 1: on sorted data the kernel sum splits into a forward and a backward
    exponentially-decayed running sum (the recursion behind the 1-D
    decomposition of Section 3.1)."""
    g = np.random.default_rng(8)
    x = np.sort(g.normal(size=2000))
    w = g.uniform(0.5, 2.0, size=2000)
    h = 0.3
    n = x.size
    fwd = np.zeros(n)
    bwd = np.zeros(n)
    fwd[0] = w[0]
    for j in range(1, n):
        fwd[j] = np.exp(-(x[j] - x[j - 1]) / h) * fwd[j - 1] + w[j]
    for j in range(n - 2, -1, -1):
        bwd[j] = np.exp(-(x[j + 1] - x[j]) / h) * (bwd[j + 1] + w[j + 1])
    want = (fwd + bwd) / (2 * h * n)
    f, _ = oracle.kde_laplace(x[None, :], x[None, :], h, w=w)
    np.testing.assert_allclose(f[0], want, rtol=1e-12)


def test_kde_product_set_separates():
    """Data on a Cartesian product with product weights: the d-dimensional
    Laplacian KDE is the product of the 1-D ones."""
    g = np.random.default_rng(9)
    a = g.normal(size=30)
    b = g.normal(size=20)
    wa = g.uniform(0.5, 1.5, 30)
    wb = g.uniform(0.5, 1.5, 20)
    x = np.stack([np.repeat(a, 20), np.tile(b, 30)])
    w = np.repeat(wa, 20) * np.tile(wb, 30)
    z = g.normal(size=(2, 25))
    h = np.array([[0.4, 0.7]])
    f2, _ = oracle.kde_laplace(x, z, h, w=w)
    fa, _ = oracle.kde_laplace(a[None, :], z[:1], 0.4, w=wa)
    fb, _ = oracle.kde_laplace(b[None, :], z[1:], 0.7, w=wb)
    np.testing.assert_allclose(f2[0], fa[0] * fb[0], rtol=1e-13)


def test_kde_large_h_limit_and_multi_h():
    g = np.random.default_rng(10)
    x = g.normal(size=(2, 300))
    z = g.normal(size=(2, 10))
    hs = np.array([1e6, 2e6])
    f, _ = oracle.kde_laplace(x, z, hs)
    np.testing.assert_allclose(f, 1.0 / (4 * hs[:, None] ** 2) * np.ones((2, 10)), rtol=1e-5)


def test_loo_and_lcv_two_points():
    x = np.array([[0.0, 0.5], [0.0, 1.0]])
    h = 0.5
    k = np.exp(-(0.5 + 1.0) / h)
    # each point's LOO density is the other point's kernel with N-1 = 1
    want = k / (4 * h * h)
    floo, _ = oracle.kde_laplace_loo(x, h)
    np.testing.assert_allclose(floo[0], [want, want], rtol=1e-15)
    assert oracle.lcv(x, [h])[0] == pytest.approx(np.log(want), rel=1e-15)


def test_nw_constant_and_cv():
    g = np.random.default_rng(11)
    x = g.normal(size=(2, 400))
    y = np.full(400, 3.25)
    m = oracle.nw_regression(x, y, g.normal(size=(2, 30)), [0.2, 1.0])
    np.testing.assert_allclose(m, 3.25, rtol=1e-14)
    assert np.allclose(oracle.nw_cv(x, y, [0.3]), 0.0, atol=1e-25)
    # two points: the LOO estimate at one point is the other point's response
    x2 = np.array([[0.0, 1.0]])
    y2 = np.array([1.0, 3.0])
    assert oracle.nw_cv(x2, y2, [0.7])[0] == pytest.approx(4.0, rel=1e-15)


def test_far_points_underflow_exactly():
    """x = (7, 7) vs (-7, -7) with h = 0.01: exp(-2800) is 0 in FP64."""
    x = np.array([[7.0, -7.0], [7.0, -7.0]])
    s, _ = oracle.laplace_sums(x, x, 0.01)
    np.testing.assert_array_equal(s[0, 0], [1.0, 1.0])


# ------------------------------------------- leave-one-out scores under underflow
def test_lcv_two_far_points_closed_form():
    """Two points 8 apart at h = 0.01: every leave-one-out kernel term is
    exp(-800), which is 0 in FP64, yet log fhat_{-j} is finite:
    log(exp(-800) / (2 h (N - 1))) = -800 - log(2 * 0.01)."""
    x = np.array([[0.0, 8.0]])
    want = -800.0 - math.log(2 * 0.01)
    got = oracle.lcv(x, [0.01])[0]
    assert got == pytest.approx(want, rel=1e-15)
    # the plain (unshifted) sum does underflow here
    floo, _ = oracle.kde_laplace_loo(x, 0.01)
    assert np.all(floo == 0.0)


def test_lcv_three_points_hand_values():
    """x = (0, 1, 3) in d = 1, h = 0.5, N - 1 = 2: the leave-one-out density
    at x_j is (1 / (2 h 2)) sum_{i != j} exp(-|x_i - x_j| / h)."""
    x = np.array([[0.0, 1.0, 3.0]])
    terms = [math.log((math.exp(-2) + math.exp(-6)) / 2.0),
             math.log((math.exp(-2) + math.exp(-4)) / 2.0),
             math.log((math.exp(-6) + math.exp(-4)) / 2.0)]
    got = oracle.log_kde_loo(x, [0.5])[0]
    np.testing.assert_allclose(got, terms, rtol=1e-15)
    assert oracle.lcv(x, [0.5])[0] == pytest.approx(sum(terms) / 3, rel=1e-15)


def test_lcv_brute_force_logsumexp_tiny():
    """Tiny random samples at bandwidths from moderate down to where every
    kernel term underflows, against scipy's logsumexp over i != j."""
    from scipy.special import logsumexp

    g = np.random.default_rng(12)
    for d in (1, 2, 3):
        x = g.normal(size=(d, 7)) * 3
        hs = np.array([1.0, 0.05, 0.002])
        got = oracle.log_kde_loo(x, hs)
        for b, h in enumerate(hs):
            for j in range(7):
                e = np.sum(np.abs(x - x[:, j:j + 1]), axis=0) / h
                e = np.delete(e, j)
                want = logsumexp(-e) - math.log(2 ** d * 6 * h ** d)
                assert got[b, j] == pytest.approx(want, rel=1e-13, abs=1e-12)
    # where nothing underflows the shifted form equals the plain logarithm
    x = g.normal(size=(2, 300))
    floo, _ = oracle.kde_laplace_loo(x, [0.2, 0.9])
    np.testing.assert_allclose(oracle.lcv(x, [0.2, 0.9]), np.log(floo).mean(axis=1),
                               rtol=1e-14)


def test_nw_loo_ratio_under_underflow():
    """x = (0, 10, 10.5), y = (1, 2, 4), h = 0.01: at point 0 the other two
    terms are exp(-1000) and exp(-1050) (both 0 in FP64); their ratio is
    (2 + 4 e^-50) / (1 + e^-50).  At point 2 the terms are exp(-1050) and
    exp(-50): m = (e^-1000 + 2) / (e^-1000 + 1) = 2 to double precision."""
    x = np.array([[0.0, 10.0, 10.5]])
    y = np.array([1.0, 2.0, 4.0])
    m, _, _, _ = oracle.nw_loo(x, y, [0.01])
    e = math.exp(-50)
    assert m[0, 0] == pytest.approx((2 + 4 * e) / (1 + e), rel=1e-15)
    assert m[0, 1] == pytest.approx(4.0, rel=1e-15)
    assert m[0, 2] == pytest.approx(2.0, rel=1e-15)
    cv = oracle.nw_cv(x, y, [0.01])[0]
    assert cv == pytest.approx(((1 - m[0, 0]) ** 2 + 4 + 4) / 3, rel=1e-15)


# ------------------------------------------------- grid -> point interpolation
def test_interp_reproduces_multilinear_functions():
    """Multilinear interpolation is exact for functions that are affine in
    each coordinate separately (a + sum b_k z_k + c z_0 z_1 + e z_0 z_1 z_2)."""
    g = np.random.default_rng(21)
    nodes = [np.sort(g.uniform(-2, 2, 7)), np.sort(g.uniform(-1, 3, 5)),
             np.sort(g.uniform(0, 1, 4))]
    Z = np.meshgrid(*nodes, indexing="ij")
    f = lambda a, b, c: 0.3 + 1.5 * a - 2.0 * b + 0.7 * c + 0.9 * a * b - 1.1 * a * b * c
    G = f(*Z)
    q = np.stack([g.uniform(z[0], z[-1], 200) for z in nodes])
    np.testing.assert_allclose(oracle.grid_interp(nodes, G, q), f(*q), rtol=1e-12, atol=1e-12)


def test_interp_nodes_clamping_and_1d():
    g = np.random.default_rng(22)
    z = np.sort(g.uniform(0, 1, 9))
    v = g.normal(size=9)
    q = np.concatenate([z, [-1.0, 2.0], g.uniform(-0.5, 1.5, 50)])
    # one dimension: numpy's interp clamps outside the nodes in the same way
    np.testing.assert_allclose(oracle.grid_interp([z], v, q[None]), np.interp(q, z, v),
                               rtol=1e-14, atol=1e-15)
    # at the nodes the node values, in two dimensions, and a one-node axis
    z2 = np.sort(g.uniform(0, 1, 4))
    G = g.normal(size=(9, 4))
    Zq = np.array([[z[i], z2[j]] for i in range(9) for j in range(4)]).T
    np.testing.assert_allclose(oracle.grid_interp([z, z2], G, Zq), G.reshape(-1), rtol=1e-14)
    G1 = g.normal(size=(9, 1))
    qq = np.stack([g.uniform(0, 1, 20), g.uniform(-5, 5, 20)])
    np.testing.assert_allclose(oracle.grid_interp([z, [0.5]], G1, qq),
                               np.interp(qq[0], z, G1[:, 0]), rtol=1e-14)
    # a NaN coordinate gives NaN, the other points are unaffected
    qn = qq.copy()
    qn[1, 3] = np.nan
    r = oracle.grid_interp([z, [0.5]], G1, qn)
    assert np.isnan(r[3]) and not np.any(np.isnan(np.delete(r, 3)))


# ------------------------------------------ matrix bandwidth and local linear
def test_matrix_bandwidth_diagonal_and_rotation_invariance():
    g = np.random.default_rng(51)
    x = g.normal(size=(2, 60))
    z = g.normal(size=(2, 9))
    # a diagonal H is the per-axis bandwidth h = sqrt(diag)
    f, _ = oracle.kde_laplace_H(x, z, [np.diag([0.09, 0.25])])
    want, _ = oracle.kde_laplace(x, z, np.array([[0.3, 0.5]]))
    np.testing.assert_allclose(f, want, rtol=1e-13)
    # rotating the data, the points and H together changes nothing
    th = 0.7
    Q = np.array([[np.cos(th), -np.sin(th)], [np.sin(th), np.cos(th)]])
    H = np.array([[0.2, 0.05], [0.05, 0.1]])
    a, _ = oracle.kde_laplace_H(x, z, [H])
    b, _ = oracle.kde_laplace_H(Q @ x, Q @ z, [Q @ H @ Q.T])
    np.testing.assert_allclose(a, b, rtol=1e-12)


def test_matrix_bandwidth_two_points_by_hand():
    """H with eigenvectors at 45 degrees, eigenvalues 0.25 and 1: one data
    point at the origin seen from (1, 1): R^T (x - z) = (0, -sqrt 2) up to
    signs, so the kernel is exp(-sqrt(2) / 1) / 4 and f = that / (N h1 h2)."""
    c = 1 / np.sqrt(2)
    R = np.array([[c, -c], [c, c]])
    H = R @ np.diag([1.0, 0.25]) @ R.T
    f, _ = oracle.kde_laplace_H(np.zeros((2, 1)), np.ones((2, 1)), [H])
    want = np.exp(-np.sqrt(2.0) / 1.0) / 4.0 / (1.0 * 0.5)
    assert f[0, 0] == pytest.approx(want, rel=1e-13)


def test_local_linear_reproduces_linear_functions():
    g = np.random.default_rng(52)
    for d in (1, 2, 3):
        x = g.normal(size=(d, 80))
        b = g.normal(size=d)
        y = 0.4 + b @ x
        z = g.normal(size=(d, 7))
        got = oracle.local_linear(x, y, z, np.full(d, 0.6))
        np.testing.assert_allclose(got, 0.4 + b @ z, rtol=1e-10, atol=1e-10)


def test_local_linear_large_bandwidth_is_least_squares():
    g = np.random.default_rng(53)
    x = g.normal(size=(2, 50))
    y = np.sin(x[0]) + x[1] ** 2
    z = g.normal(size=(2, 5))
    got = oracle.local_linear(x, y, z, np.full(2, 1e7))
    X = np.vstack([np.ones(50), x]).T
    coef = np.linalg.lstsq(X, y, rcond=None)[0]
    np.testing.assert_allclose(got, coef[0] + coef[1:] @ z, rtol=1e-6, atol=1e-6)


# --------------------------------------------------------------------------
# eq. (ECDFdelta) at arbitrary points, the uniform kernel (Section 3.2) and
# the additive Matern-3/2 kernel (Appendix C)
# --------------------------------------------------------------------------
def test_ecdf_delta_hand_ties():
    """x = 0, 1, 2 on one axis, z = 1: <= counts 2 points, < counts 1."""
    x = np.array([[0.0, 1.0, 2.0]])
    z = np.array([[1.0, 1.0, -1.0, 2.5]])
    got = oracle.ecdf_delta(x, z, np.array([0, 1, 1, 1], np.uint8))
    assert got.tolist() == [2, 1, 0, 3]


def test_ecdf_delta_strict_is_half_step_below_on_integer_data():
    """For integer-valued data, x < z equals x <= z - 1/2 on that axis, so each
    strict axis of eq. (ECDFdelta) moves the query half a step down."""
    g = np.random.default_rng(71)
    for d in (1, 2, 3):
        x = g.integers(-3, 4, size=(d, 400)).astype(float)
        z = g.integers(-3, 4, size=(d, 60)).astype(float)
        y = g.uniform(-1.0, 2.0, 400)
        delta = g.integers(0, 1 << d, size=60).astype(np.uint8)
        zs = z.copy()
        for k in range(d):
            zs[k] -= 0.5 * ((delta >> k) & 1)
        assert np.array_equal(oracle.ecdf_delta(x, z, delta), oracle.ecdf(x, zs))
        s, _ = oracle.ecdf_delta(x, z, delta, y)
        w, _ = oracle.dominance_sums(x, zs, y)
        assert np.array_equal(s, w)


def test_ecdf_delta_all_strict_on_reflected_data_is_the_esf():
    """1{-x < -z} on every axis is 1{x > z}: eq. (ECDFdelta) with delta = -1
    everywhere on the reflected sample is eq. (ESF)."""
    g = np.random.default_rng(72)
    x = np.round(g.normal(size=(3, 500)), 1)
    z = np.round(g.normal(size=(3, 80)), 1)
    got = oracle.ecdf_delta(-x, -z, np.full(80, 7, np.uint8))
    assert np.array_equal(got, oracle.esf(x, z))


def test_uniform_box_hand_and_closed_ends():
    """d = 1, x = 0, .25, .5, .75, 1, z = .5, h = .25: the closed box [.25, .75]
    holds three points (dyadic values, so the ends are exact)."""
    x = np.array([[0.0, 0.25, 0.5, 0.75, 1.0]])
    s, _ = oracle.kernel_sums("uniform", x, np.array([[0.5]]), [0.25])
    assert s[0, 0, 0] == 3.0
    f, _ = oracle.kde_uniform(x, np.array([[0.5]]), [0.25])
    assert f[0, 0] == pytest.approx(3.0 / (2 * 5 * 0.25), rel=1e-15)


def test_uniform_is_the_signed_sum_of_shifted_ecdfs():
    """eq. (uniform_decomposition_nD): the box count at z equals
    sum_delta (prod_k delta_k) F_N(z + delta h, delta), with the corner
    coordinates z + delta h rounded to doubles, bit for bit on counts."""
    g = np.random.default_rng(73)
    for d in (1, 2, 3):
        x = np.round(g.normal(size=(d, 600)), 1)
        z = np.round(g.normal(size=(d, 40)), 1)
        h = np.round(g.uniform(0.1, 0.8, d), 1)
        want = np.zeros(40, dtype=np.int64)
        for dl in range(1 << d):
            sign = (-1) ** bin(dl).count("1")
            zc = np.stack([z[k] - h[k] if (dl >> k) & 1 else z[k] + h[k] for k in range(d)])
            want += sign * oracle.ecdf_delta(x, zc, np.full(40, dl, np.uint8))
        s, _ = oracle.kernel_sums("uniform", x, z, h[None, :])
        assert np.array_equal(s[0, 0], want.astype(float))


def _matern_general(u, p):
    """eq. (Matern_kernel) with eq. (Matern_constant), h = 1."""
    from math import comb, factorial

    norm = sum(factorial(p) // factorial(p - k) * factorial(2 * p - k) / factorial(2 * p)
               * 2 ** k for k in range(p + 1))
    gam = math.sqrt(2 * p + 1) / (2 * norm)
    poly = sum(comb(p, k) * factorial(2 * p - k) / factorial(2 * p)
               * (2 * math.sqrt(2 * p + 1)) ** k * np.abs(u) ** k for k in range(p + 1))
    return gam * poly * np.exp(-math.sqrt(2 * p + 1) * np.abs(u))


def test_matern32_d1_is_the_papers_univariate_kernel():
    """In d = 1 the additive kernel is eq. (Matern32) (the p = 1 member of eq.
    (Matern_kernel)) with its bandwidth sqrt(3) h."""
    g = np.random.default_rng(74)
    x = g.normal(size=(1, 300))
    z = np.linspace(-3, 3, 41)[None, :]
    h = 0.4
    f, _ = oracle.kde_matern32(x, z, [h])
    H = math.sqrt(3.0) * h
    u = (x[0][None, :] - z[0][:, None]) / H
    want = _matern_general(u, 1).mean(axis=1) / H
    assert np.max(np.abs(f[0] - want)) <= 1e-14 * np.max(want)


def test_matern32_integrates_to_one():
    """eq. (Matern32_average) is a density: for one point in d = 2 the
    estimate integrates to 1 (trapezoid rule on a fine, wide grid)."""
    t = np.linspace(-30, 30, 1201)
    zz = np.stack(np.meshgrid(t, t, indexing="ij")).reshape(2, -1)
    f, _ = oracle.kde_matern32(np.zeros((2, 1)), zz, [[1.0, 2.0]])
    tot = np.trapezoid(np.trapezoid(f[0].reshape(1201, 1201), t, axis=1), t)
    assert abs(tot - 1.0) < 1e-3


def test_matern32_is_the_papers_decomposition():
    """eq. (Matern32_decomposition_nD): the additive kernel sum at z equals
    sum_delta e^{-sum_k delta_k z_k/h_k} ((1 + sum_l delta_l z_l/h_l)
    F(delta z, delta; delta x, y0) - sum_l (delta_l/h_l) F(delta z, delta;
    delta x, y_l)) with y0 = w e^{sum_k delta_k x_k/h_k} and y_l = x_l y0
    (F without its 1/N; small coordinates, so the exponential weights stay
    in range)."""
    g = np.random.default_rng(75)
    for d in (1, 2, 3):
        x = g.uniform(-1.0, 1.0, size=(d, 300))
        z = g.uniform(-1.0, 1.0, size=(d, 25))
        w = g.uniform(0.5, 2.0, 300)
        h = g.uniform(0.4, 0.9, d)
        want = np.zeros(25)
        for dl in range(1 << d):
            sg = np.array([-1.0 if (dl >> k) & 1 else 1.0 for k in range(d)])
            y0 = w * np.exp((sg[:, None] * x / h[:, None]).sum(0))
            mask = np.full(25, dl, np.uint8)
            f0, _ = oracle.ecdf_delta(sg[:, None] * x, sg[:, None] * z, mask, y0)
            acc = (1.0 + (sg[:, None] * z / h[:, None]).sum(0)) * f0
            for l in range(d):
                fl, _ = oracle.ecdf_delta(sg[:, None] * x, sg[:, None] * z, mask, x[l] * y0)
                acc -= sg[l] / h[l] * fl
            want += np.exp(-(sg[:, None] * z / h[:, None]).sum(0)) * acc
        s, _ = oracle.kernel_sums("matern32", x, z, h[None, :], w)
        assert np.max(np.abs(s[0, 0] - want)) <= 1e-12 * np.max(np.abs(want))
