"""Grid -> point interpolation (mecdf_grid_interp) against the oracle's
multilinear interpolation, and the interpolation-error study of Sections 4.1
and 4.2 in small: grid ECDF interpolated to the sample points against the
points path's exact values."""
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


@pytest.mark.parametrize("shape", [(7,), (1,), (2,), (9, 4), (5, 1), (6, 7, 3), (3, 4, 2, 5),
                                   (2, 2, 2, 2, 2, 3)])
def test_interp_random(lib, shape):
    d = len(shape)
    g = np.random.default_rng(sum(shape) * 7 + d)
    nodes = [np.sort(g.uniform(-2, 2, m)) if m > 1 else np.array([g.uniform(-1, 1)])
             for m in shape]
    G = g.normal(size=shape)
    Q = 3001
    q = np.stack([g.uniform(-2.5, 2.5, Q) for _ in range(d)])
    # some queries exactly at nodes, some with a NaN coordinate
    for k in range(d):
        q[k, :len(nodes[k])] = nodes[k]
    q[0, -3:] = np.nan
    want = oracle.grid_interp(nodes, G, q)
    got = lib.grid_interp(dev(G), nodes, dev(q)).cpu().numpy()
    assert np.array_equal(np.isnan(got), np.isnan(want))
    ok = ~np.isnan(want)
    assert np.max(np.abs(got[ok] - want[ok])) <= 1e-13 * np.max(np.abs(G))
    got32 = lib.grid_interp(dev(G, torch.float32), nodes, dev(q)).cpu().numpy()
    want32 = oracle.grid_interp(nodes, G.astype(np.float32).astype(np.float64), q)
    assert np.max(np.abs(got32[ok] - want32[ok])) <= 1e-6 * np.max(np.abs(G))


def test_interp_zero_queries_and_bad_nodes(lib):
    nodes = [np.array([0.0, 1.0])]
    G = dev(np.array([1.0, 2.0]))
    out = lib.grid_interp(G, nodes, torch.empty((1, 0), dtype=torch.float64, device="cuda"))
    assert out.numel() == 0
    with pytest.raises(lib.MecdfError):
        lib.grid_interp(G, [np.array([1.0, 0.0])], dev(np.zeros((1, 4))))


@pytest.mark.parametrize("d", [2, 3])
def test_grid_ecdf_interpolated_to_the_points(lib, d):
    """The route Section 4.1 studies: the ECDF on an M = N grid over the
    data, linearly interpolated to the sample points, against the exact
    values there (points path).  The error shrinks when the grid is refined;
    the interpolated values match the oracle's interpolation of the same
    grid values."""
    g = np.random.default_rng(31 + d)
    n = 20000
    x = g.normal(size=(d, n))
    xt = dev(x)
    exact = lib.ecdf_points(xt).cpu().numpy() / n
    errs = []
    for m in (int(round(n ** (1 / d))), int(round((4 * n) ** (1 / d)))):
        nodes = datagen.uniform_grid(x, m)
        F, _ = lib.ecdf_esf_grid(xt, nodes, want_esf=False)
        Fn = F.double() / n
        got = lib.grid_interp(Fn, nodes, xt).cpu().numpy()
        want = oracle.grid_interp(nodes, Fn.cpu().numpy(), x)
        assert np.max(np.abs(got - want)) <= 1e-13
        errs.append(np.max(np.abs(got - exact)))
    assert errs[1] < errs[0]
