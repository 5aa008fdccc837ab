"""Brute-force CPU oracle (test infrastructure only).

Plain, slow, obviously correct evaluations of the quantities defined in
Langrene & Warin, arXiv 2005.03246:

* eq. (ECDF) and eq. (ESF), Section 1: generalized weighted ECDF / ESF at
  arbitrary evaluation points (rectilinear grid nodes or the sample points);
* eq. (Laplacian_kde_nD), Section 3.1: weighted Laplacian-kernel density
  estimate, which with w = response gives the Nadaraya-Watson ratio named in
  the same section;
* leave-one-out likelihood and squared-error cross-validation scores built
  from those sums (Section 3.2 notes that infinite-support kernels such as
  the Laplacian suit likelihood cross-validation);
* linear interpolation of grid values to arbitrary points (Sections 4.1 and
  4.2), through scipy's regular-grid interpolator.

The arithmetic lives in ``oracle.c`` (a double loop over query and data
point, Neumaier-compensated FP64 sums, OpenMP over queries).  This module only
marshals numpy arrays and applies the normalising constants of the
definitions.  Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline
leg of ``bench.py`` may import it; the GPU library never does.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None


def build(force: bool = False) -> str:
    """Compile oracle.c into liboracle.so with gcc (OpenMP, no fast-math)."""
    if force or not os.path.exists(_LIB) or (
        os.path.getmtime(_LIB) < os.path.getmtime(_SRC)
    ):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(
            ["gcc", "-O2", "-std=c11", "-fopenmp", "-fPIC", "-shared", _SRC,
             "-o", tmp, "-lm"]
        )
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        build()
        lib = ctypes.CDLL(_LIB)
        P = ctypes.c_void_p
        I64 = ctypes.c_int64
        I = ctypes.c_int
        lib.oracle_dominance.argtypes = [I, I64, P, P, I64, P, I, P, P, P, I]
        lib.oracle_dominance.restype = I
        lib.oracle_laplace_sums.argtypes = [I, I64, P, I, P, I64, P, I, P, P,
                                            P, P, I]
        lib.oracle_laplace_sums.restype = I
        lib.oracle_laplace_loo_shifted.argtypes = [I, I64, P, I, P, I, P, P,
                                                   P, P, I]
        lib.oracle_laplace_loo_shifted.restype = I
        lib.oracle_ecdf_delta.argtypes = [I, I64, P, P, I64, P, P, P, P, P, I]
        lib.oracle_ecdf_delta.restype = I
        lib.oracle_kernel_sums.argtypes = [I, I, I64, P, I, P, I64, P, I, P, P, P, I]
        lib.oracle_kernel_sums.restype = I
        lib.oracle_max_threads.argtypes = []
        lib.oracle_max_threads.restype = I
        _lib = lib
    return _lib


def max_threads() -> int:
    return int(_load().oracle_max_threads())


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.float64)


def _ptr(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def _as_2d(x) -> np.ndarray:
    x = _f64(x)
    if x.ndim == 1:
        x = x[None, :]
    return x


# --------------------------------------------------------------------------
# eq. (ECDF) / eq. (ESF)
# --------------------------------------------------------------------------
def dominance_sums(x, z, y=None, survival=False, nthreads=0):
    """Raw sums of eq. (ECDF) (survival=False) or eq. (ESF) (survival=True).

    x: (d, N) data, z: (d, Q) evaluation points, y: (N,) weights or None.
    Returns int64 counts when y is None, else (sum, abs_sum) float64 arrays.
    No 1/N factor is applied here.
    """
    x = _as_2d(x)
    z = _as_2d(z)
    d, n = x.shape
    if z.shape[0] != d:
        raise ValueError("x and z must have the same dimension")
    q = z.shape[1]
    lib = _load()
    if y is None:
        cnt = np.zeros(q, dtype=np.int64)
        rc = lib.oracle_dominance(d, n, _ptr(x), None, q, _ptr(z),
                                  int(bool(survival)), _ptr(cnt), None, None,
                                  int(nthreads))
        if rc:
            raise ValueError("oracle_dominance rejected its arguments")
        return cnt
    y = _f64(y)
    if y.shape != (n,):
        raise ValueError("y must have shape (N,)")
    s = np.zeros(q)
    a = np.zeros(q)
    rc = lib.oracle_dominance(d, n, _ptr(x), _ptr(y), q, _ptr(z),
                              int(bool(survival)), None, _ptr(s), _ptr(a),
                              int(nthreads))
    if rc:
        raise ValueError("oracle_dominance rejected its arguments")
    return s, a


def ecdf(x, z, y=None, nthreads=0):
    """F_N(z; x, y) of eq. (ECDF).  y None: int64 counts (no 1/N, y = 1).
    Otherwise returns (F_N, A_N) with A_N the same functional over |y|."""
    r = dominance_sums(x, z, y, survival=False, nthreads=nthreads)
    if y is None:
        return r
    n = _as_2d(x).shape[1]
    return r[0] / n, r[1] / n


def esf(x, z, y=None, nthreads=0):
    """Fbar_N(z; x, y) of eq. (ESF); same conventions as :func:`ecdf`."""
    r = dominance_sums(x, z, y, survival=True, nthreads=nthreads)
    if y is None:
        return r
    n = _as_2d(x).shape[1]
    return r[0] / n, r[1] / n


def ecdf_delta(x, z, delta, y=None, nthreads=0):
    """F_N(z, delta; x, y) of eq. (ECDFdelta) without the 1/N factor, at the
    points z (d, Q) with a sign pattern per point: delta (Q,) bit masks, bit
    k set for delta_k = -1 (strict < on axis k), clear for <=.  y None: int64
    counts, else (sum, abs_sum)."""
    x = _as_2d(x)
    z = _as_2d(z)
    d, n = x.shape
    q = z.shape[1]
    dl = np.ascontiguousarray(delta, dtype=np.uint8)
    if z.shape[0] != d or dl.shape != (q,):
        raise ValueError("z must be (d, Q) and delta (Q,)")
    lib = _load()
    if y is None:
        cnt = np.zeros(q, dtype=np.int64)
        rc = lib.oracle_ecdf_delta(d, n, _ptr(x), None, q, _ptr(z), _ptr(dl), _ptr(cnt),
                                   None, None, int(nthreads))
        if rc:
            raise ValueError("oracle_ecdf_delta rejected its arguments")
        return cnt
    y = _f64(y)
    s = np.zeros(q)
    a = np.zeros(q)
    rc = lib.oracle_ecdf_delta(d, n, _ptr(x), _ptr(y), q, _ptr(z), _ptr(dl), None, _ptr(s),
                               _ptr(a), int(nthreads))
    if rc:
        raise ValueError("oracle_ecdf_delta rejected its arguments")
    return s, a


def grid_points(nodes, index=None) -> np.ndarray:
    """Evaluation points of a rectilinear grid (Section 2.1): the Cartesian
    product of the per-axis node vectors, C order (last axis fastest).

    index: optional (Q, d) integer array of multi-indices to keep only those
    nodes (sampled checks at full size)."""
    nodes = [_f64(v) for v in nodes]
    d = len(nodes)
    if index is None:
        mesh = np.meshgrid(*nodes, indexing="ij")
        return np.stack([m.reshape(-1) for m in mesh])
    index = np.asarray(index, dtype=np.int64)
    return np.stack([nodes[k][index[:, k]] for k in range(d)])


# --------------------------------------------------------------------------
# eq. (Laplacian_kde_nD) and the quantities built on it
# --------------------------------------------------------------------------
def _hmat(h, d):
    """Bandwidths as an (nh, d) matrix.  A scalar is one isotropic bandwidth,
    a 1-D array is a list of isotropic bandwidths, a 2-D array is taken as
    (nh, d) per-axis bandwidths (eq. (Laplacian_kde_nD) allows h_k per axis)."""
    h = np.asarray(h, dtype=np.float64)
    if h.ndim == 0:
        return np.full((1, d), float(h))
    if h.ndim == 1:
        return np.repeat(h[:, None], d, 1)
    if h.shape[1] != d:
        raise ValueError("per-axis bandwidths must have shape (nh, d)")
    return h


def laplace_sums(x, z, h, w=None, skip=None, nthreads=0):
    """Raw kernel sums sum_i w_c,i exp(-sum_k |x_ki - z_kq| / h_bk).

    h: see _hmat; w: (nw, N) or (N,) or None.
    skip: (Q,) index of a data point to leave out per query (-1 = none).
    Returns (S, A) with shape (nw, nh, Q)."""
    x = _as_2d(x)
    z = _as_2d(z)
    d, n = x.shape
    q = z.shape[1]
    h = _f64(_hmat(h, d))
    nh = h.shape[0]
    if w is None:
        wv, nw = None, 1
    else:
        wv = _f64(w)
        if wv.ndim == 1:
            wv = wv[None, :]
        nw = wv.shape[0]
        wv = _f64(wv)
    sk = None if skip is None else np.ascontiguousarray(skip, dtype=np.int64)
    s = np.zeros((nw, nh, q))
    a = np.zeros((nw, nh, q))
    rc = _load().oracle_laplace_sums(d, n, _ptr(x), nw, _ptr(wv), q, _ptr(z),
                                     nh, _ptr(h), _ptr(sk), _ptr(s), _ptr(a),
                                     int(nthreads))
    if rc:
        raise ValueError("oracle_laplace_sums rejected its arguments")
    return s, a


def kde_laplace(x, z, h, w=None, nthreads=0):
    """f_KDE(z) of eq. (Laplacian_kde_nD): (nh, Q) values and the |w| scale."""
    x = _as_2d(x)
    d, n = x.shape
    hm = _hmat(h, d)
    s, a = laplace_sums(x, z, hm, w, None, nthreads)
    c = 1.0 / (2.0 ** d * n * np.prod(hm, axis=1))
    return s[0] * c[:, None], a[0] * c[:, None]


def kde_laplace_loo(x, h, w=None, nthreads=0):
    """Leave-one-out density at every sample point: the kernel sum over
    i != j normalised with N - 1 instead of N.  Returns (nh, N) and scale."""
    x = _as_2d(x)
    d, n = x.shape
    hm = _hmat(h, d)
    s, a = laplace_sums(x, x, hm, w, np.arange(n), nthreads)
    c = 1.0 / (2.0 ** d * (n - 1) * np.prod(hm, axis=1))
    return s[0] * c[:, None], a[0] * c[:, None]


def laplace_loo_shifted(x, h, w=None, nthreads=0):
    """Leave-one-out kernel sums at the sample points with the nearest term
    factored out: returns (m, S, A) with m of shape (nh, N) the smallest
    scaled distance min_{i != j} sum_k |x_ki - x_kj| / h_bk, and S, A of shape
    (nw, nh, N) the sums of w_c,i exp(-(e_i - m)) (and of |w_c,i| ...) over
    i != j.  The plain leave-one-out sum is exp(-m) * S."""
    x = _as_2d(x)
    d, n = x.shape
    if n < 2:
        raise ValueError("leave-one-out sums need N >= 2")
    h = _f64(_hmat(h, d))
    nh = h.shape[0]
    if w is None:
        wv, nw = None, 1
    else:
        wv = _f64(w)
        if wv.ndim == 1:
            wv = wv[None, :]
        nw = wv.shape[0]
        wv = _f64(wv)
    m = np.zeros((nh, n))
    s = np.zeros((nw, nh, n))
    a = np.zeros((nw, nh, n))
    rc = _load().oracle_laplace_loo_shifted(d, n, _ptr(x), nw, _ptr(wv), nh,
                                            _ptr(h), _ptr(m), _ptr(s), _ptr(a),
                                            int(nthreads))
    if rc:
        raise ValueError("oracle_laplace_loo_shifted rejected its arguments")
    return m, s, a


def log_kde_loo(x, h, nthreads=0):
    """log fhat_{-j}(x_j) at every sample point, (nh, N): the leave-one-out
    density of eq. (Laplacian_kde_nD) (sum over i != j, N - 1 normalisation)
    through a max-shifted log-sum-exp, -m_j + log S_j + log(1 / (2^d (N-1)
    prod_k h_k)), finite even where every kernel term underflows."""
    x = _as_2d(x)
    d, n = x.shape
    hm = _hmat(h, d)
    m, s, _ = laplace_loo_shifted(x, hm, None, nthreads)
    c = -np.log(2.0 ** d * (n - 1) * np.prod(hm, axis=1))
    return -m + np.log(s[0]) + c[:, None]


def lcv(x, h, nthreads=0):
    """Likelihood cross-validation score LCV(h) = (1/N) sum_j log fhat_{-j}(x_j)
    for each bandwidth row of h (Section 3.2 names likelihood
    cross-validation for infinite-support kernels).  Returns (nh,)."""
    return log_kde_loo(x, h, nthreads).mean(axis=1)


def nw_regression(x, y, z, h, nthreads=0):
    """Nadaraya-Watson estimate m(z) = sum_i y_i K / sum_i K (Section 3.1,
    weights w = response).  Returns (nh, Q)."""
    x = _as_2d(x)
    d = x.shape[0]
    hm = _hmat(h, d)
    s, _ = laplace_sums(x, z, hm, np.stack([np.ones_like(_f64(y)), _f64(y)]),
                        None, nthreads)
    return s[1] / s[0]


def nw_loo(x, y, h, nthreads=0):
    """Leave-one-out NW estimate at the sample points and the |y| scale of its
    numerator: (m_loo, num, den, num_abs), each (nh, N).  num and den are the
    kernel sums over i != j relative to the nearest term (both carry the same
    factor exp(m_j), which cancels in the ratio), so the ratio is defined
    wherever some other point exists."""
    x = _as_2d(x)
    y = _f64(y)
    _, s, a = laplace_loo_shifted(x, h, np.stack([np.ones_like(y), y]),
                                  nthreads)
    return s[1] / s[0], s[1], s[0], a[1]


def nw_cv(x, y, h, nthreads=0):
    """Squared-error LOO CV score CV(h) = (1/N) sum_j (y_j - m_{-j}(x_j))^2."""
    m, _, _, _ = nw_loo(x, y, h, nthreads)
    return ((_f64(y)[None, :] - m) ** 2).mean(axis=1)


# --------------------------------------------------------------------------
# the uniform kernel (Section 3.2) and the additive Matern-3/2 kernel
# (Appendix C)
# --------------------------------------------------------------------------
def kernel_sums(kind, x, z, h, w=None, nthreads=0):
    """Raw sums of the uniform ("uniform": prod_k 1{z_k - h_k <= x_k <= z_k +
    h_k}, both ends rounded to doubles) or additive Matern-3/2 ("matern32":
    (1 + e) exp(-e), e = sum_k |x_k - z_k| / h_k) kernel; conventions of
    laplace_sums without skip.  Returns (S, A) of shape (nw, nh, Q)."""
    kd = {"uniform": 0, "matern32": 1}[kind]
    x = _as_2d(x)
    z = _as_2d(z)
    d, n = x.shape
    q = z.shape[1]
    h = _f64(_hmat(h, d))
    nh = h.shape[0]
    if w is None:
        wv, nw = None, 1
    else:
        wv = _f64(w)
        if wv.ndim == 1:
            wv = wv[None, :]
        nw = wv.shape[0]
        wv = _f64(wv)
    s = np.zeros((nw, nh, q))
    a = np.zeros((nw, nh, q))
    rc = _load().oracle_kernel_sums(kd, d, n, _ptr(x), nw, _ptr(wv), q, _ptr(z), nh, _ptr(h),
                                    _ptr(s), _ptr(a), int(nthreads))
    if rc:
        raise ValueError("oracle_kernel_sums rejected its arguments")
    return s, a


def kde_uniform(x, z, h, w=None, nthreads=0):
    """f_KDE(z) of eq. (uniform_kde_nD), 1/(2^d N prod h) times the box sums:
    (nh, Q) values and the |w| scale."""
    x = _as_2d(x)
    d, n = x.shape
    hm = _hmat(h, d)
    s, a = kernel_sums("uniform", x, z, hm, w, nthreads)
    c = 1.0 / (2.0 ** d * n * np.prod(hm, axis=1))
    return s[0] * c[:, None], a[0] * c[:, None]


def kde_matern32(x, z, h, w=None, nthreads=0):
    """The kernel density estimate with the additive Matern-3/2 kernel of eq.
    (Matern32_average), K_d(u) = (1 + |u|_1) exp(-|u|_1) / (2^d (1 + d)):
    (nh, Q) values and the |w| scale."""
    x = _as_2d(x)
    d, n = x.shape
    hm = _hmat(h, d)
    s, a = kernel_sums("matern32", x, z, hm, w, nthreads)
    c = 1.0 / (2.0 ** d * (1 + d) * n * np.prod(hm, axis=1))
    return s[0] * c[:, None], a[0] * c[:, None]


def nw_matern32(x, y, z, h, nthreads=0):
    """Nadaraya-Watson ratio with the additive Matern-3/2 kernel: (nh, Q)."""
    x = _as_2d(x)
    hm = _hmat(h, x.shape[0])
    s, _ = kernel_sums("matern32", x, z, hm, np.stack([np.ones_like(_f64(y)), _f64(y)]),
                       nthreads)
    return s[1] / s[0]


# --------------------------------------------------------------------------
# grid -> point interpolation (Sections 4.1 and 4.2 interpolate grid values
# linearly to the sample points)
# --------------------------------------------------------------------------
def grid_interp(nodes, G, q):
    """Multilinear interpolation of node values G (shape (M_1..M_d)) at the
    points q (d, Q): each coordinate clipped to its axis's node range (no
    extrapolation), axes with a single node dropped (constant), then
    scipy's RegularGridInterpolator with method "linear"."""
    from scipy.interpolate import RegularGridInterpolator

    q = _as_2d(q)
    G = np.asarray(G, dtype=np.float64)
    axes, pts, keep = [], [], []
    for k, z in enumerate(nodes):
        z = np.asarray(z, dtype=np.float64)
        if len(z) == 1:
            continue
        keep.append(k)
        axes.append(z)
        qk = np.where(np.isnan(q[k]), z[0], q[k])  # NaN rows are set to NaN below
        pts.append(np.clip(qk, z[0], z[-1]))
    single = [k for k in range(len(nodes)) if k not in keep]
    Gk = G[tuple(0 if k in single else slice(None) for k in range(len(nodes)))]
    if keep:
        f = RegularGridInterpolator(tuple(axes), Gk, method="linear")
        out = f(np.stack(pts, axis=1))
    else:
        out = np.full(q.shape[1], float(Gk))
    out[np.any(np.isnan(q), axis=0)] = np.nan
    return out


# --------------------------------------------------------------------------
# general matrix bandwidth (Appendix B, eq. (kde_nD_H)) and local-linear
# regression with the Laplacian kernel
# --------------------------------------------------------------------------
def matrix_bandwidth(H):
    """H = R diag(h)^2 R^T (numpy's symmetric eigendecomposition): (R, h)."""
    H = np.asarray(H, dtype=np.float64)
    ev, R = np.linalg.eigh(H)
    if np.any(ev <= 0):
        raise ValueError("H must be positive definite")
    return R, np.sqrt(ev)


def kde_laplace_H(x, z, Hs, w=None, nthreads=0):
    """eq. (kde_nD_H) with the Laplacian kernel, read as in Appendix B: the
    estimator with diagonal bandwidth h in the rotated coordinates R^T x, R^T z
    (H = R diag(h)^2 R^T), so fhat(z) = 1/(2^d N prod h) sum_i w_i
    exp(-|| diag(1/h) R^T (x_i - z) ||_1).  Hs: (nh, d, d).  Returns (f, A)
    of shape (nh, Q) like kde_laplace."""
    x = _as_2d(x)
    z = _as_2d(z)
    fs, As = [], []
    for H in np.asarray(Hs, dtype=np.float64):
        R, h = matrix_bandwidth(H)
        f, a = kde_laplace(R.T @ x, R.T @ z, h[None, :], w, nthreads)
        fs.append(f[0])
        As.append(a[0])
    return np.array(fs), np.array(As)


def nw_regression_H(x, y, z, Hs, nthreads=0):
    """NW ratio with a matrix bandwidth, in the coordinates of kde_laplace_H."""
    x = _as_2d(x)
    z = _as_2d(z)
    out = []
    for H in np.asarray(Hs, dtype=np.float64):
        R, h = matrix_bandwidth(H)
        out.append(nw_regression(R.T @ x, y, R.T @ z, h[None, :], nthreads)[0])
    return np.array(out)


def local_linear(x, y, z, h):
    """Local-linear regression at the points z (d, Q): the intercept a of the
    weighted least-squares fit of y ~ a + b^T (x - z_j) with Laplacian weights
    exp(-sum_k |x_k - z_k| / h_k), from the moments about z_j formed directly
    (no expansion).  Where the (d+1) x (d+1) system has a pivot below 1e-10 of
    its largest diagonal entry (Gaussian elimination with partial pivoting),
    the local constant (NW) estimate.  Pure Python loops over the queries:
    small cases only."""
    x = _as_2d(x)
    z = _as_2d(z)
    y = _f64(y)
    h = np.asarray(h, dtype=np.float64).reshape(-1)
    d, n = x.shape
    out = np.empty(z.shape[1])
    for j in range(z.shape[1]):
        u = x - z[:, j:j + 1]
        k = np.exp(-np.sum(np.abs(u) / h[:, None], axis=0))
        X = np.vstack([np.ones(n), u])          # (d+1, N)
        A = (X * k) @ X.T
        rhs = (X * k) @ y
        M = np.hstack([A, rhs[:, None]])
        dmax = np.max(np.abs(np.diag(A)))
        ok = dmax > 0
        m = d + 1
        for c in range(m):
            if not ok:
                break
            p = c + int(np.argmax(np.abs(M[c:, c])))
            if not abs(M[p, c]) > 1e-10 * dmax:
                ok = False
                break
            M[[c, p]] = M[[p, c]]
            M[c + 1:] -= np.outer(M[c + 1:, c] / M[c, c], M[c])
        if ok:
            sol = np.zeros(m)
            for r in range(m - 1, -1, -1):
                sol[r] = (M[r, m] - M[r, r + 1:m] @ sol[r + 1:]) / M[r, r]
            out[j] = sol[0]
        else:
            out[j] = rhs[0] / A[0, 0]
    return out
