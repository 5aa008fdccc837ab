"""The grid entry point that allocates nothing (ecdf_esf_grid_noalloc),
called through the C ABI: results equal ecdf_esf_grid's bit for bit on two
calls in a row (the second smaller, so the scratch array still holds the
first call's data), it runs while the library's growing workspace is capped
at one byte, and a problem too large for its scratch array is refused before
anything runs."""
import os

import numpy as np
import pytest
import torch

from paper_2005_03246_amd import datagen

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def lib():
    from paper_2005_03246_amd import mecdf

    return mecdf


def _case(seed, d, n, m):
    g = np.random.default_rng(seed)
    x = g.normal(size=(d, n))
    y = g.normal(size=n)
    return x, y, datagen.uniform_grid(x, m)


def _weights(y, prec):
    if prec == "counts":
        return None, "f64"
    dt = np.float64 if prec == "f64" else np.float32
    return torch.from_numpy(y.astype(dt)).cuda(), prec


@pytest.mark.parametrize("prec", ["counts", "f64", "f32c"])
@pytest.mark.parametrize("d", [1, 2, 3])
def test_noalloc_matches_grid_entry(lib, prec, d):
    sizes = {1: ([3000], [37]), 2: ([300, 400], [40, 50]), 3: ([40, 50, 60], [7, 9, 11])}[d]
    for seed, n, m in ((10 + d, 600000, sizes[0]), (20 + d, 30001, sizes[1])):
        x, y, nodes = _case(seed, d, n, m)
        xt = torch.from_numpy(x).cuda()
        yt, p = _weights(y, prec)
        want = lib.ecdf_esf_grid(xt, nodes, yt, prec=p)
        got = lib.ecdf_esf_grid(xt, nodes, yt, prec=p, noalloc=True)
        torch.cuda.synchronize()
        for a, b in zip(want, got):
            assert a.dtype == b.dtype and torch.equal(a, b), (prec, d, n)


def test_noalloc_runs_with_the_workspace_capped(lib):
    x, y, nodes = _case(5, 3, 200000, [30, 31, 32])
    xt = torch.from_numpy(x).cuda()
    yt = torch.from_numpy(y).cuda()
    want = lib.ecdf_esf_grid(xt, nodes, yt)
    out = tuple(torch.empty_like(a) for a in want)
    old = os.environ.get("MECDF_WORKSPACE_LIMIT")
    os.environ["MECDF_WORKSPACE_LIMIT"] = "1"
    try:
        lib.ecdf_esf_grid(xt, nodes, yt, out=out, noalloc=True)
        with pytest.raises(lib.MecdfError) as e:
            lib.ecdf_esf_grid(xt, nodes, yt)
        assert e.value.code == lib.MECDF_ENOMEM
    finally:
        if old is None:
            del os.environ["MECDF_WORKSPACE_LIMIT"]
        else:
            os.environ["MECDF_WORKSPACE_LIMIT"] = old
    torch.cuda.synchronize()
    for a, b in zip(want, out):
        assert torch.equal(a, b)


def test_noalloc_refuses_problems_over_its_scratch(lib):
    n = 3_000_000  # about 28.5 bytes per float64 point: above 64 MiB
    x = torch.linspace(-1.0, 1.0, n, dtype=torch.float64, device="cuda")[None, :]
    y = torch.ones(n, dtype=torch.float64, device="cuda")
    F = torch.full((16,), -7.0, dtype=torch.float64, device="cuda")
    nodes = [np.linspace(-1.0, 1.0, 16)]
    with pytest.raises(lib.MecdfError) as e:
        lib.ecdf_esf_grid(x, nodes, y, out=(F, None), want_esf=False, noalloc=True)
    assert e.value.code == lib.MECDF_EUNSUPPORTED
    assert "scratch" in str(e.value)
    torch.cuda.synchronize()
    assert torch.all(F == -7.0)  # nothing ran
