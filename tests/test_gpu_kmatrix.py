"""Matrix bandwidths (kde_laplace_H / kreg_laplace_H) and local-linear
regression (kreg_loclin_laplace) at the sample points against the oracle."""
import numpy as np
import pytest
import torch

import oracle

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def lib():
    from paper_2005_03246_amd import mecdf

    return mecdf


def dev(a, dtype=torch.float64):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=dtype).cuda()


def spd(g, d, lo, hi):
    Q, _ = np.linalg.qr(g.normal(size=(d, d)))
    ev = np.sort(g.uniform(lo, hi, d))
    return Q @ np.diag(ev) @ Q.T


@pytest.mark.parametrize("case", [(2, 700), (3, 500), (4, 300)])
def test_matrix_bandwidth_kde_and_nw(lib, case):
    d, n = case
    g = np.random.default_rng(80 + d)
    x = g.normal(size=(d, n))
    w = g.uniform(0.3, 1.5, n)
    y = np.cos(x[0]) + 0.1 * g.normal(size=n)
    Hs = np.stack([spd(g, d, 0.01, 0.2), spd(g, d, 0.1, 1.0), np.diag(g.uniform(0.05, 0.4, d))])
    f, _ = lib.kde_laplace_H(dev(x), Hs, dev(w), want_lcv=False)
    want, scale = oracle.kde_laplace_H(x, x, Hs, w)
    assert np.max(np.abs(f.cpu().numpy() - want) / scale) <= 1e-12
    _, lcv = lib.kde_laplace_H(dev(x), Hs, want_f=False)
    ref = []
    for H in Hs:
        R, h = oracle.matrix_bandwidth(H)
        ref.append(oracle.lcv(R.T @ x, h[None, :])[0])
    ref = np.array(ref)
    assert np.all(np.abs(lcv.cpu().numpy() - ref) <= 1e-12 * np.maximum(1, np.abs(ref)))
    m, _ = lib.kreg_laplace_H(dev(x), dev(y), Hs, want_cv=False)
    wm = oracle.nw_regression_H(x, y, x, Hs)
    assert np.max(np.abs(m.cpu().numpy() - wm)) <= 1e-12 * np.max(np.abs(y))
    f32, _ = lib.kde_laplace_H(dev(x), Hs, prec="f32c", want_lcv=False)
    w1, s1 = oracle.kde_laplace_H(x, x, Hs)
    assert np.max(np.abs(f32.cpu().numpy() - w1) / s1) <= 1e-5
    with pytest.raises(lib.MecdfError):
        lib.kde_laplace_H(dev(x), -Hs[:1])


@pytest.mark.parametrize("case", [(1, 400), (2, 600), (3, 500)])
def test_local_linear(lib, case):
    """Against the oracle's direct weighted least squares; linear responses
    are reproduced exactly up to rounding."""
    d, n = case
    g = np.random.default_rng(90 + d)
    x = g.normal(size=(d, n))
    y = np.sin(2 * x[0]) + 0.3 * x[-1] + 0.05 * g.normal(size=n)
    hs = np.repeat(np.array([0.15, 0.4, 1.0])[:, None], d, 1)
    m = lib.kreg_loclin_laplace(dev(x), dev(y), hs).cpu().numpy()
    for b, h in enumerate(hs):
        want = oracle.local_linear(x, y, x, h)
        # the moment expansion about each x_j cancels digits (|x_j| / spread)^2
        assert np.max(np.abs(m[b] - want)) <= 1e-8 * np.max(np.abs(y)), b
    lin = 0.7 - 1.3 * x[0] + (0.5 * x[1] if d > 1 else 0)
    ml = lib.kreg_loclin_laplace(dev(x), dev(lin), hs).cpu().numpy()
    assert np.max(np.abs(ml - lin[None, :])) <= 1e-8 * np.max(np.abs(lin))
    m32 = lib.kreg_loclin_laplace(dev(x), dev(y.astype(np.float32), torch.float32), hs,
                                  prec="f32c").cpu().numpy()
    want32 = oracle.local_linear(x, y.astype(np.float32).astype(np.float64), x, hs[1])
    assert np.max(np.abs(m32[1] - want32)) <= 1e-5 * np.max(np.abs(y))
