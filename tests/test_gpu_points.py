"""Parity of the points path (ecdf_points / esf_points) with the brute-force
oracle: counts bit-exact, float64 within 1e-12 and float32 within 1e-5 of the
|y|-weighted scale, ties and duplicates included."""
import numpy as np
import pytest
import torch

import oracle
from paper_2005_03246_amd import datagen

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def lib():
    from paper_2005_03246_amd import mecdf

    return mecdf


@pytest.fixture(params=["direct", "recursion"])
def path(request, monkeypatch):
    """Small samples go to the direct (all pairs) kernel unless
    MECDF_POINTS_DIRECT_MAX is 0; each small case runs on both paths."""
    if request.param == "recursion":
        monkeypatch.setenv("MECDF_POINTS_DIRECT_MAX", "0")
    else:
        monkeypatch.delenv("MECDF_POINTS_DIRECT_MAX", raising=False)
    return request.param


def dev(a, dtype=torch.float64):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=dtype).cuda()


def check_weighted(got, want, scale, tol):
    got = np.asarray(got, dtype=np.float64).reshape(-1)
    zero = scale == 0
    assert np.all(got[zero] == 0.0)
    nz = ~zero
    err = np.abs(got[nz] - want[nz]) / scale[nz]
    assert err.size == 0 or err.max() <= tol, err.max()


CASES = [
    (1, 1, 1), (1, 2000, 2), (2, 1, 1), (2, 2, 3), (2, 513, 1), (2, 3000, 2),
    (3, 700, 1), (3, 2500, 2), (4, 1500, 1), (4, 3000, 2), (5, 1200, 1),
    (6, 900, 1),
]


@pytest.mark.parametrize("case", CASES)
def test_points_random(lib, path, case):
    d, n, dec = case
    g = np.random.default_rng(77 + 13 * d + n)
    x = np.round(g.normal(size=(d, n)), dec)   # ties on purpose
    xt = dev(x)
    np.testing.assert_array_equal(lib.ecdf_points(xt).cpu().numpy(), oracle.ecdf(x, x))
    np.testing.assert_array_equal(lib.esf_points(xt).cpu().numpy(), oracle.esf(x, x))
    yi = g.integers(-3, 4, size=n).astype(np.float64)
    np.testing.assert_array_equal(lib.ecdf_points(xt, dev(yi)).cpu().numpy(),
                                  oracle.ecdf(x, x, yi)[0])
    np.testing.assert_array_equal(lib.esf_points(xt, dev(yi)).cpu().numpy(),
                                  oracle.esf(x, x, yi)[0])
    y = g.normal(size=n)
    w, a = oracle.ecdf(x, x, y)
    check_weighted(lib.ecdf_points(xt, dev(y)).cpu().numpy(), w, a, 1e-12)
    w, a = oracle.esf(x, x, y)
    check_weighted(lib.esf_points(xt, dev(y)).cpu().numpy(), w, a, 1e-12)
    y32 = y.astype(np.float32)
    f = lib.ecdf_points(xt, dev(y32, torch.float32), prec="f32c")
    assert f.dtype == torch.float32
    w, a = oracle.ecdf(x, x, y32.astype(np.float64))
    check_weighted(f.cpu().numpy(), w, a, 1e-5)


def test_hand_points(lib, path, golden):
    g = golden["points_d2"]
    x = np.array(g["x"], dtype=float)
    y = np.array(g["y"], dtype=float)
    assert lib.ecdf_points(dev(x)).cpu().numpy().tolist() == g["ecdf_counts"]
    assert lib.esf_points(dev(x)).cpu().numpy().tolist() == g["esf_counts"]
    got = lib.ecdf_points(dev(x), dev(y)).cpu().numpy()
    np.testing.assert_array_equal(got, np.array(g["ecdf_weighted_sums"]) / 5.0)
    got = lib.esf_points(dev(x), dev(y)).cpu().numpy()
    np.testing.assert_array_equal(got, np.array(g["esf_weighted_sums"]) / 5.0)


def test_all_equal_points_and_nan(lib, path):
    x = np.ones((3, 1000))
    np.testing.assert_array_equal(lib.ecdf_points(dev(x)).cpu().numpy(), np.full(1000, 1000))
    np.testing.assert_array_equal(lib.esf_points(dev(x)).cpu().numpy(), np.zeros(1000))
    g = np.random.default_rng(3)
    x = np.round(g.normal(size=(2, 600)), 1)
    x[0, ::7] = np.nan
    x[1, 3::11] = np.nan
    np.testing.assert_array_equal(lib.ecdf_points(dev(x)).cpu().numpy(), oracle.ecdf(x, x))
    np.testing.assert_array_equal(lib.esf_points(dev(x)).cpu().numpy(), oracle.esf(x, x))


def test_config1_uniform_d2_full(lib, path):
    """d = 2, N = 4096 uniform points: bit-exact counts against the full brute force."""
    x = datagen.config1()
    xt = dev(x)
    np.testing.assert_array_equal(lib.ecdf_points(xt).cpu().numpy(), oracle.ecdf(x, x))
    np.testing.assert_array_equal(lib.esf_points(xt).cpu().numpy(), oracle.esf(x, x))


def test_config3_reduced_full(lib, path):
    """The d = 4 tied t(3)-copula workload at N = 2^15, every point checked."""
    x = datagen.config3(n=1 << 15)
    xt = dev(x)
    np.testing.assert_array_equal(lib.ecdf_points(xt).cpu().numpy(), oracle.ecdf(x, x))
    np.testing.assert_array_equal(lib.esf_points(xt).cpu().numpy(), oracle.esf(x, x))


def test_config3_full_size_sampled(lib):
    """N = 2^22, d = 4: sampled points plus the coordinate-wise extreme points."""
    x = datagen.config3()
    xt = dev(x)
    F = lib.ecdf_points(xt).cpu().numpy()
    Fb = lib.esf_points(xt).cpu().numpy()
    g = np.random.default_rng(8)
    idx = np.concatenate([g.choice(x.shape[1], 600, replace=False),
                          np.argmax(x, axis=1), np.argmin(x, axis=1)])
    z = x[:, idx]
    np.testing.assert_array_equal(F[idx], oracle.ecdf(x, z))
    np.testing.assert_array_equal(Fb[idx], oracle.esf(x, z))
    # invariants at full size: the ECDF count includes the point itself
    assert F.min() >= 1
    assert Fb.max() < x.shape[1]


def test_points_deterministic(lib, path):
    g = np.random.default_rng(9)
    x = dev(np.round(g.normal(size=(3, 20000)), 2))
    y = dev(g.normal(size=20000))
    a = lib.ecdf_points(x, y)
    b = lib.ecdf_points(x, y)
    assert torch.equal(a, b)


@pytest.mark.parametrize("d", [1, 3, 4])
def test_nan_points_weighted(lib, path, d):
    """Points with a NaN coordinate count for nothing and get 0, with
    weights too, in d = 1, 3, 4 (the recursion keeps them as items that only
    receive, and discards what they receive)."""
    g = np.random.default_rng(60 + d)
    n = 1500
    x = np.round(g.normal(size=(d, n)), 1)
    x[d - 1, ::9] = np.nan
    x[0, 5::13] = np.nan
    y = g.integers(-3, 4, size=n).astype(np.float64)
    for fn, ofn in ((lib.ecdf_points, oracle.ecdf), (lib.esf_points, oracle.esf)):
        np.testing.assert_array_equal(fn(dev(x)).cpu().numpy(), ofn(x, x))
        want, _ = ofn(x, x, y)
        np.testing.assert_array_equal(fn(dev(x), dev(y)).cpu().numpy(), want)


# Largest sample sizes of the direct (all pairs) kernel for d = 1 .. 6 when
# MECDF_POINTS_DIRECT_MAX is not set; one point more takes the recursion.
DIRECT_MAX = {1: 20000, 2: 24000, 3: 32000, 4: 46000, 5: 80000, 6: 150000}


@pytest.mark.parametrize("d", [1, 2, 3, 4, 5, 6])
def test_points_at_the_path_switch(lib, monkeypatch, d):
    """Both sides of the size where the default path changes, for each d:
    counts at sampled points (and the extreme points) equal to the brute
    force, weights within 1e-12 of the |y| scale; the direct and the
    recursive evaluation of the same sample give the same counts at every
    point."""
    monkeypatch.delenv("MECDF_POINTS_DIRECT_MAX", raising=False)
    g = np.random.default_rng(500 + d)
    for n in (DIRECT_MAX[d], DIRECT_MAX[d] + 1):
        x = np.round(g.normal(size=(d, n)), 2)   # ties on purpose
        y = g.normal(size=n)
        xt, yt = dev(x), dev(y)
        idx = np.concatenate([g.choice(n, 150, replace=False), [0, n - 1],
                              np.argmax(x, axis=1), np.argmin(x, axis=1)])
        z = x[:, idx]
        F = lib.ecdf_points(xt).cpu().numpy()
        Fb = lib.esf_points(xt).cpu().numpy()
        np.testing.assert_array_equal(F[idx], oracle.ecdf(x, z))
        np.testing.assert_array_equal(Fb[idx], oracle.esf(x, z))
        w, a = oracle.ecdf(x, z, y)
        check_weighted(lib.ecdf_points(xt, yt).cpu().numpy()[idx], w, a, 1e-12)
        w, a = oracle.esf(x, z, y)
        check_weighted(lib.esf_points(xt, yt).cpu().numpy()[idx], w, a, 1e-12)
        # the other path on the same sample
        other = "0" if n <= DIRECT_MAX[d] else str(1 << 30)
        monkeypatch.setenv("MECDF_POINTS_DIRECT_MAX", other)
        np.testing.assert_array_equal(lib.ecdf_points(xt).cpu().numpy(), F)
        np.testing.assert_array_equal(lib.esf_points(xt).cpu().numpy(), Fb)
        monkeypatch.delenv("MECDF_POINTS_DIRECT_MAX")
