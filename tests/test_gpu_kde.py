"""Parity of the kernel path (kde_laplace / kreg_laplace) with the brute-force
oracle: densities and NW estimates within 1e-12 (float64) / 1e-5 (float32) of
the |w|-weighted scale, LCV / CV scores within 1e-12."""
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


def dev(a, dtype=torch.float64):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=dtype).cuda()


def rel_err(got, want, scale):
    got = np.asarray(got, dtype=np.float64)
    return np.max(np.abs(got - want) / scale)


def hmat(hs, d):
    return np.repeat(np.asarray(hs, dtype=float)[:, None], d, 1)


CASES = [(1, 2), (1, 700), (1, 5000), (2, 2), (2, 63), (2, 64), (2, 65), (2, 1000),
         (2, 3000), (3, 2), (3, 64), (3, 200), (3, 900), (3, 3000)]


@pytest.mark.parametrize("case", CASES)
def test_kde_random(lib, case):
    d, n = case
    g = np.random.default_rng(500 + 7 * d + n)
    x = np.round(g.normal(size=(d, n)), 2)
    w = g.uniform(0.2, 2.0, n)
    hs = hmat([0.01, 0.07, 0.3, 1.0, 4.0], d)
    hs[1] = g.uniform(0.05, 0.5, d)          # per-axis bandwidths
    f, lcv = lib.kde_laplace(dev(x), hs, dev(w))
    want, scale = oracle.kde_laplace(x, x, hs, w)
    assert rel_err(f.cpu().numpy(), want, scale) <= 1e-12
    f0, lcv0 = lib.kde_laplace(dev(x), hs)
    want0, scale0 = oracle.kde_laplace(x, x, hs)
    assert rel_err(f0.cpu().numpy(), want0, scale0) <= 1e-12
    ref = oracle.lcv(x, hs)
    got = lcv0.cpu().numpy()
    assert np.all(np.isfinite(got))
    assert np.all(np.abs(got - ref) <= 1e-12 * np.maximum(1.0, np.abs(ref)))
    # float32 path: densities and the LCV scores
    f32, _ = lib.kde_laplace(dev(x), hs, dev(w.astype(np.float32), torch.float32),
                             prec="f32c", want_lcv=False)
    want32, scale32 = oracle.kde_laplace(x, x, hs, w.astype(np.float32).astype(np.float64))
    assert rel_err(f32.cpu().numpy(), want32, scale32) <= 1e-5
    _, l32 = lib.kde_laplace(dev(x), hs, prec="f32c", want_f=False)
    assert np.all(np.abs(l32.cpu().numpy() - ref) <= 1e-5 * np.maximum(1.0, np.abs(ref)))


@pytest.mark.parametrize("case", [(1, 800), (2, 70), (2, 2500), (3, 600), (3, 2100)])
def test_nw_random(lib, case):
    d, n = case
    g = np.random.default_rng(900 + d + n)
    x = g.normal(size=(d, n))
    y = np.sin(x[0]) + 0.1 * g.normal(size=n)
    hs = hmat([0.05, 0.2, 0.8], d)
    m, cv = lib.kreg_laplace(dev(x), dev(y), hs)
    want = oracle.nw_regression(x, y, x, hs)
    # NW ratio: error normalised by max |y|
    assert np.max(np.abs(m.cpu().numpy() - want)) <= 1e-12 * np.max(np.abs(y))
    ref = oracle.nw_cv(x, y, hs)
    assert np.all(np.abs(cv.cpu().numpy() - ref) <= 1e-12 * np.maximum(1.0, ref))
    m32, cv32 = lib.kreg_laplace(dev(x), dev(y.astype(np.float32), torch.float32), hs,
                                 prec="f32c")
    y32 = y.astype(np.float32).astype(np.float64)
    want32 = oracle.nw_regression(x, y32, x, hs)
    assert np.max(np.abs(m32.cpu().numpy() - want32)) <= 1e-5 * np.max(np.abs(y))
    ref32 = oracle.nw_cv(x, y32, hs)
    assert np.all(np.abs(cv32.cpu().numpy() - ref32) <= 1e-5 * np.maximum(1.0, ref32))


@pytest.mark.parametrize("d", [1, 2, 3])
def test_loo_sums_below_the_float_range(lib, d):
    """Points far from every other one: at h = 0.01 their leave-one-out
    kernel sums are below the float64 range (exp(-1000)) or the float32 range,
    yet log fhat_{-j} and the NW leave-one-out ratio are finite and equal the
    oracle's values (taken relative to the nearest point)."""
    g = np.random.default_rng(40 + d)
    n = 900
    x = g.normal(size=(d, n)) * 0.3
    x[:, 5] += 10.0          # 10 / 0.01 = 1000 from everything in axis 0 alone
    x[:, 6] -= 9.0
    x[:, 7] += 0.8           # e^-80: below the float32 range only
    y = np.sin(x[0]) + 0.1 * g.normal(size=n)
    hs = hmat([0.01, 0.02, 0.5], d)
    ref = oracle.lcv(x, hs)
    refcv = oracle.nw_cv(x, y, hs)
    for prec, tol in (("f64", 1e-12), ("f32c", 1e-5)):
        yy = dev(y) if prec == "f64" else dev(y.astype(np.float32), torch.float32)
        _, lcv = lib.kde_laplace(dev(x), hs, prec=prec, want_f=False)
        got = lcv.cpu().numpy()
        assert np.all(np.isfinite(got)), prec
        assert np.all(np.abs(got - ref) <= tol * np.maximum(1.0, np.abs(ref))), prec
        _, cv = lib.kreg_laplace(dev(x), yy, hs, prec=prec, want_m=False)
        r = refcv if prec == "f64" else oracle.nw_cv(x, y.astype(np.float32).astype(np.float64), hs)
        assert np.all(np.abs(cv.cpu().numpy() - r) <= tol * np.maximum(1.0, r)), prec


@pytest.mark.parametrize("case", [(4, 2), (4, 300), (5, 257), (6, 700)])
def test_direct_sums_d4_to_d6(lib, case):
    """d = 4..6 (direct evaluation of every pair): densities, NW estimates and
    both scores against the oracle in float64 and float32."""
    d, n = case
    g = np.random.default_rng(70 + d + n)
    x = g.normal(size=(d, n))
    x[:, 0] += 6.0           # one far point: its sums are relative to its neighbour
    w = g.uniform(0.2, 2.0, n)
    y = np.cos(x[1]) + 0.1 * g.normal(size=n)
    hs = hmat([0.05, 0.3, 1.0, 2.5, 0.7], d)
    hs[2] = g.uniform(0.2, 1.5, d)
    f, _ = lib.kde_laplace(dev(x), hs, dev(w), want_lcv=False)
    want, scale = oracle.kde_laplace(x, x, hs, w)
    assert rel_err(f.cpu().numpy(), want, scale) <= 1e-12
    _, lcv = lib.kde_laplace(dev(x), hs, want_f=False)
    ref = oracle.lcv(x, hs)
    assert np.all(np.abs(lcv.cpu().numpy() - ref) <= 1e-12 * np.maximum(1.0, np.abs(ref)))
    m, cv = lib.kreg_laplace(dev(x), dev(y), hs)
    assert np.max(np.abs(m.cpu().numpy() - oracle.nw_regression(x, y, x, hs))) <= \
        1e-12 * np.max(np.abs(y))
    refcv = oracle.nw_cv(x, y, hs)
    assert np.all(np.abs(cv.cpu().numpy() - refcv) <= 1e-12 * np.maximum(1.0, refcv))
    f32, l32 = lib.kde_laplace(dev(x), hs, prec="f32c")
    want1, scale1 = oracle.kde_laplace(x, x, hs)
    assert rel_err(f32.cpu().numpy(), want1, scale1) <= 1e-5
    assert np.all(np.abs(l32.cpu().numpy() - ref) <= 1e-5 * np.maximum(1.0, np.abs(ref)))
    y32 = y.astype(np.float32)
    m32, cv32 = lib.kreg_laplace(dev(x), dev(y32, torch.float32), hs, prec="f32c")
    y32d = y32.astype(np.float64)
    assert np.max(np.abs(m32.cpu().numpy() - oracle.nw_regression(x, y32d, x, hs))) <= \
        1e-5 * np.max(np.abs(y))
    r32 = oracle.nw_cv(x, y32d, hs)
    assert np.all(np.abs(cv32.cpu().numpy() - r32) <= 1e-5 * np.maximum(1.0, r32))


def test_paper_accuracy_claim_2d(lib):
    """Section 4.2 reports the fast Laplacian KDE within 1e-14 (max absolute
    difference) of the naive sum for X ~ N(0, I_2), h = 0.1: N = 20000 here,
    every sample point, float64."""
    g = np.random.default_rng(4_2)
    x = g.normal(size=(2, 20000))
    f, _ = lib.kde_laplace(dev(x), [0.1], want_lcv=False)
    want, _ = oracle.kde_laplace(x, x, hmat([0.1], 2))
    assert np.max(np.abs(f.cpu().numpy() - want)) < 1e-14


def test_kde_hand_d1(lib, golden):
    g = golden["kde_d1"]
    x = np.array([g["x"]])
    f, lcv = lib.kde_laplace(dev(x), [g["h"]])
    assert f.cpu().numpy()[0, 0] == pytest.approx(g["f"], rel=1e-15)
    assert lcv.cpu().numpy()[0] == pytest.approx(np.log(g["f_loo_point0"]), rel=1e-15)


def test_kde_config4_lcv_full_small(lib):
    """The mixture workload at N = 2^13 with all 64 bandwidths: every LOO
    density enters the LCV score, checked against the full oracle."""
    x, y, hs = datagen.config4(n=1 << 13)
    f, lcv = lib.kde_laplace(dev(x), hs)
    ref = oracle.lcv(x, hs)
    got = lcv.cpu().numpy()
    assert np.all(np.abs(got - ref) <= 1e-12 * np.maximum(1.0, np.abs(ref)))
    assert int(np.argmax(got)) == int(np.argmax(ref))
    m, cv = lib.kreg_laplace(dev(x), dev(y), hs)
    refcv = oracle.nw_cv(x, y, hs)
    assert np.all(np.abs(cv.cpu().numpy() - refcv) <= 1e-12 * refcv)
    assert int(np.argmin(cv.cpu().numpy())) == int(np.argmin(refcv))
    # float32 path: all 64 scores within 1e-5, and the selected bandwidth's
    # oracle score within that tolerance of the best one
    _, l32 = lib.kde_laplace(dev(x), hs, prec="f32c", want_f=False)
    g32 = l32.cpu().numpy()
    assert np.all(np.abs(g32 - ref) <= 1e-5 * np.maximum(1.0, np.abs(ref)))
    assert ref[int(np.argmax(g32))] >= ref.max() - 2e-5 * max(1.0, abs(ref.max()))
    y32 = y.astype(np.float32)
    _, c32 = lib.kreg_laplace(dev(x), dev(y32, torch.float32), hs, prec="f32c", want_m=False)
    r32 = oracle.nw_cv(x, y32.astype(np.float64), hs)
    c32 = c32.cpu().numpy()
    assert np.all(np.abs(c32 - r32) <= 1e-5 * np.maximum(1.0, r32))
    assert r32[int(np.argmin(c32))] <= r32.min() + 2e-5 * max(1.0, r32.min())


def test_kde_config4_full_size_sampled(lib):
    """N = 2^22 points, the 64-bandwidth batch in one call; densities and NW
    estimates checked at sampled points for a spread of the bandwidths."""
    x, y, hs = datagen.config4()
    n = x.shape[1]
    xt = dev(x)
    f, lcv = lib.kde_laplace(xt, hs)
    m, cv = lib.kreg_laplace(xt, dev(y), hs)
    g = np.random.default_rng(10)
    idx = np.concatenate([g.choice(n, 96, replace=False), np.argmax(x, axis=1),
                          np.argmin(x, axis=1)])
    pick = [0, 21, 42, 63]
    want, scale = oracle.kde_laplace(x, x[:, idx], hs[pick])
    got = f.cpu().numpy()[pick][:, idx]
    assert rel_err(got, want, scale) <= 1e-12
    wantm = oracle.nw_regression(x, y, x[:, idx], hs[pick])
    gotm = m.cpu().numpy()[pick][:, idx]
    assert np.max(np.abs(gotm - wantm)) <= 1e-12 * np.max(np.abs(y))
    assert np.all(np.isfinite(lcv.cpu().numpy())) and np.all(np.isfinite(cv.cpu().numpy()))
    del f, m
    # float32 path at the same points and bandwidths
    f32, l32 = lib.kde_laplace(xt, hs, prec="f32c")
    assert rel_err(f32.cpu().numpy()[pick][:, idx], want, scale) <= 1e-5
    l32 = l32.cpu().numpy()
    assert np.all(np.isfinite(l32))
    assert np.all(np.abs(l32 - lcv.cpu().numpy()) <= 1e-5 * np.maximum(1.0, np.abs(l32)))
    del f32
    y32 = y.astype(np.float32)
    m32, c32 = lib.kreg_laplace(xt, dev(y32, torch.float32), hs, prec="f32c")
    want32 = oracle.nw_regression(x, y32.astype(np.float64), x[:, idx], hs[pick])
    assert np.max(np.abs(m32.cpu().numpy()[pick][:, idx] - want32)) <= 1e-5 * np.max(np.abs(y))
    assert np.all(np.isfinite(c32.cpu().numpy()))


@pytest.mark.parametrize("d,n", [(1, 300001), (2, 300001), (3, 280003)])
def test_kde_tile_carries_in_runs_sampled(lib, d, n):
    """More than 256 tiles of 1024 items: the tile carries go through groups
    of 256 tiles and a per-tile composition of the group totals before it;
    densities and NW at sampled points (ragged last tile and group) against
    the oracle, float64 and the float32 path."""
    g = np.random.default_rng(12 + d)
    x = g.normal(size=(d, n))
    y = np.sin(x[0]) + 0.1 * g.normal(size=n)
    hs = np.array([0.02, 0.15, 0.9])
    xt = dev(x)
    idx = np.concatenate([g.choice(n, 48, replace=False), np.argmax(x, axis=1),
                          np.argmin(x, axis=1)])
    want, scale = oracle.kde_laplace(x, x[:, idx], hs)
    f, _ = lib.kde_laplace(xt, hs)
    assert rel_err(f.cpu().numpy()[:, idx], want, scale) <= 1e-12
    f32, _ = lib.kde_laplace(xt, hs, prec="f32c")
    assert rel_err(f32.cpu().numpy()[:, idx], want, scale) <= 1e-5
    m, _ = lib.kreg_laplace(xt, dev(y), hs)
    wantm = oracle.nw_regression(x, y, x[:, idx], hs)
    assert np.max(np.abs(m.cpu().numpy()[:, idx] - wantm)) <= 1e-12 * np.max(np.abs(y))


def test_kde_deterministic(lib):
    g = np.random.default_rng(11)
    x = dev(g.normal(size=(2, 30000)))
    a, la = lib.kde_laplace(x, [0.05, 0.3])
    b, lb = lib.kde_laplace(x, [0.05, 0.3])
    assert torch.equal(a, b) and torch.equal(la, lb)
