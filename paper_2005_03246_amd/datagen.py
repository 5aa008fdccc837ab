"""Seeded synthetic inputs shared by the tests, the smoke check and the
benchmark.

This module holds input recipes only (random draws, shapes, grids); none of
the method's arithmetic.  Every array is float64 numpy in the structure-of-
arrays layout the library takes: x has shape (d, N), x[k, i] = coordinate k
of sample point i.  Seeds are ``200503246 + config`` unless given.

Workloads (synthetic stand-ins for the experiments of Section 4, whose own
data are N(0, I_d) samples):

1. points ECDF, d=2, x ~ U[0,1]^2, y = 1 (int64 counts)
2. grid ECDF/ESF, d=3, x ~ N(0, 0.5 I + 0.5 J), y ~ N(0,1), uniform grid
   spanning the per-axis min..max, 256 nodes per axis
3. points ECDF/ESF, d=4, Gaussian copula with correlation 0.3 and Student-t(3)
   marginals, rounded to 1e-3 (ties), y = 1
4. Laplacian KDE / NW regression, d=2, mixture 0.5 N(+1.5(1,1), I) +
   0.5 N(-1.5(1,1), I), y = sin(x1) + 0.1 N(0,1), 64 log-spaced bandwidths in
   [0.01, 1]
5. many small datasets (Gaussian mixtures of 1-5 components, d in {1,2,3}) for
   bandwidth selection
"""
from __future__ import annotations

import numpy as np

BASE_SEED = 200503246


def rng(config: int, seed: int | None = None) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(BASE_SEED + config if seed is None else seed))


def _equicorrelated_normal(g: np.random.Generator, d: int, n: int, rho: float) -> np.ndarray:
    """(d, n) draws of N(0, (1-rho) I + rho J) as sqrt(rho) * common +
    sqrt(1-rho) * independent."""
    common = g.standard_normal(n)
    x = g.standard_normal((d, n))
    return np.sqrt(rho) * common[None, :] + np.sqrt(1.0 - rho) * x


def uniform_grid(x: np.ndarray, m: int | list[int]) -> list[np.ndarray]:
    """Per-axis uniform nodes spanning min..max of the data.  Node j is
    lo + (hi - lo) * j / (M - 1) and the last node is set to hi exactly, so
    that the grid's top corner dominates every sample point."""
    d = x.shape[0]
    ms = [m] * d if np.isscalar(m) else list(m)
    nodes = []
    for k in range(d):
        lo, hi = float(np.min(x[k])), float(np.max(x[k]))
        mk = int(ms[k])
        if mk == 1:
            nodes.append(np.array([hi]))
            continue
        z = lo + (hi - lo) * (np.arange(mk, dtype=np.float64) / (mk - 1))
        z[-1] = hi
        # strictly increasing even for a degenerate range
        if not np.all(np.diff(z) > 0):
            z = lo + np.arange(mk, dtype=np.float64)
        nodes.append(z)
    return nodes


def config1(n: int = 4096, seed: int | None = None):
    g = rng(1, seed)
    return g.random((2, n))


def config2(n: int = 1 << 24, m: int = 256, seed: int | None = None):
    """Returns x (3, n), y (n,), nodes (list of 3 arrays)."""
    g = rng(2, seed)
    x = _equicorrelated_normal(g, 3, n, 0.5)
    y = g.standard_normal(n)
    return x, y, uniform_grid(x, m)


def _t3_ppf(u: np.ndarray) -> np.ndarray:
    from scipy.stats import t as student_t

    return student_t.ppf(u, 3)


def config3(n: int = 1 << 22, d: int = 4, seed: int | None = None):
    """Gaussian copula (equicorrelation 0.3) with t(3) marginals, rounded to
    1e-3 with round-half-even so that equal values are bitwise equal."""
    from scipy.special import ndtr

    g = rng(3, seed)
    zn = _equicorrelated_normal(g, d, n, 0.3)
    x = _t3_ppf(ndtr(zn))
    return np.rint(1000.0 * x) / 1000.0


def bandwidths(nh: int = 64, lo: float = 0.01, hi: float = 1.0) -> np.ndarray:
    """nh log-spaced bandwidths h_j = lo * (hi/lo)^(j/(nh-1))."""
    if nh == 1:
        return np.array([lo])
    return lo * (hi / lo) ** (np.arange(nh) / (nh - 1))


def config4(n: int = 1 << 22, seed: int | None = None):
    """Returns x (2, n), y (n,), h (64,)."""
    g = rng(4, seed)
    comp = g.random(n) < 0.5
    mu = np.where(comp, 1.5, -1.5)
    x = g.standard_normal((2, n)) + mu[None, :]
    y = np.sin(x[0]) + 0.1 * g.standard_normal(n)
    return x, y, bandwidths(64)


def paper_normal(n: int, d: int, seed: int | None = None) -> np.ndarray:
    """The timing workload of Section 4: X ~ N(0, I_d), (d, n)."""
    g = rng(10 + d, seed)
    return g.standard_normal((d, n))


def mixture_dataset(g: np.random.Generator, n: int, d: int) -> np.ndarray:
    """One random Gaussian mixture sample: K ~ U{1..5} components, Dirichlet(1)
    weights, means U[-3,3]^d, covariances Wishart(d+2, I/(d+2))."""
    k = int(g.integers(1, 6))
    wts = g.dirichlet(np.ones(k))
    mus = g.uniform(-3.0, 3.0, (k, d))
    df = d + 2
    covs = []
    for _ in range(k):
        a = g.standard_normal((df, d)) / np.sqrt(df)
        covs.append(a.T @ a)
    lab = g.choice(k, size=n, p=wts)
    x = np.empty((d, n))
    for c in range(k):
        idx = np.nonzero(lab == c)[0]
        if idx.size == 0:
            continue
        l = np.linalg.cholesky(covs[c] + 1e-9 * np.eye(d))
        x[:, idx] = (mus[c][:, None] + l @ g.standard_normal((d, idx.size)))
    return x


def config5(count: int = 512, log2n_lo: float = 10.0, log2n_hi: float = 18.0,
            seed: int | None = None):
    """List of (d, n) arrays: n = floor(2^U(lo, hi)), d uniform on {1,2,3}."""
    g = rng(5, seed)
    out = []
    for _ in range(count):
        n = int(np.floor(2.0 ** g.uniform(log2n_lo, log2n_hi)))
        d = int(g.integers(1, 4))
        out.append(mixture_dataset(g, n, d))
    return out
