"""Thin Python binding of libmecdf (argument marshalling only).

Every function takes torch tensors that live on the current HIP device,
allocates the outputs with torch, and calls the C ABI of include/mecdf.h with
raw device pointers and the current torch stream.  All arithmetic happens in
the library's HIP kernels; there is no CPU fallback: if libmecdf.so is
missing, importing this module raises.
"""
from __future__ import annotations

import ctypes
import os

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "_lib", "libmecdf.so")

if not os.path.exists(LIB_PATH):
    raise ImportError(
        "libmecdf.so is not built (expected at %s); run "
        "`python -m paper_2005_03246_amd.build` first" % LIB_PATH)

_lib = ctypes.CDLL(LIB_PATH)

MECDF_OK = 0
MECDF_EINVAL = -1
MECDF_ENOMEM = -2
MECDF_EDEVICE = -3
MECDF_EUNSUPPORTED = -4
MECDF_EIO = -5
MECDF_F64 = 0
MECDF_F32C = 1

_P = ctypes.c_void_p
_I = ctypes.c_int
_I64 = ctypes.c_int64

_SIGS = {
    "ecdf_grid": [_I, _I64, _P, _P, _P, _P, _P, _I, _P],
    "esf_grid": [_I, _I64, _P, _P, _P, _P, _P, _I, _P],
    "ecdf_esf_grid": [_I, _I64, _P, _P, _P, _P, _P, _P, _I, _P],
    "ecdf_esf_grid_noalloc": [_I, _I64, _P, _P, _P, _P, _P, _P, _I, _P],
    "ecdf_points": [_I, _I64, _P, _P, _P, _I, _P],
    "esf_points": [_I, _I64, _P, _P, _P, _I, _P],
    "kde_laplace": [_I, _I64, _P, _P, _I, _P, _P, _P, _I, _P],
    "kreg_laplace": [_I, _I64, _P, _P, _I, _P, _P, _P, _I, _P],
}
for _name, _args in _SIGS.items():
    _fn = getattr(_lib, _name)
    _fn.argtypes = _args
    _fn.restype = _I
_lib.mecdf_strerror.argtypes = [_I]
_lib.mecdf_strerror.restype = ctypes.c_char_p
_lib.mecdf_last_error.argtypes = []
_lib.mecdf_last_error.restype = ctypes.c_char_p
_lib.mecdf_release.argtypes = []
_lib.mecdf_release.restype = None

# the raw C functions, for callers that marshal pointers themselves
raw = _lib


class MecdfError(RuntimeError):
    def __init__(self, code: int, where: str):
        self.code = code
        msg = _lib.mecdf_last_error().decode(errors="replace")
        super().__init__("%s failed: %s (%d): %s" % (
            where, _lib.mecdf_strerror(code).decode(), code, msg))


def _check(rc: int, where: str):
    if rc != MECDF_OK:
        raise MecdfError(rc, where)


def _prec(prec) -> int:
    if prec in (MECDF_F64, "f64", "float64", torch.float64):
        return MECDF_F64
    if prec in (MECDF_F32C, "f32c", "float32", torch.float32):
        return MECDF_F32C
    raise ValueError("prec must be 'f64' or 'f32c'")


def _stream_ptr(stream=None):
    s = torch.cuda.current_stream() if stream is None else stream
    return ctypes.c_void_p(s.cuda_stream)


def _x(x: torch.Tensor) -> torch.Tensor:
    if not (x.is_cuda and x.dtype == torch.float64 and x.dim() == 2):
        raise TypeError("x must be a (d, N) float64 tensor on the GPU")
    return x.contiguous()


def _y(y, n: int, prec: int, x: torch.Tensor):
    if y is None:
        return None
    want = torch.float64 if prec == MECDF_F64 else torch.float32
    if not (y.is_cuda and y.dtype == want and y.shape == (n,)):
        raise TypeError("y must be a (N,) %s tensor on the GPU" % want)
    if y.device != x.device:
        raise ValueError("x and y must be on the same device")
    return y.contiguous()


def _out_dtype(y, prec: int):
    if y is None:
        return torch.int64
    return torch.float64 if prec == MECDF_F64 else torch.float32


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _grid_args(nodes):
    ms = (ctypes.c_int64 * len(nodes))(*[int(len(v)) for v in nodes])
    flat = []
    for v in nodes:
        flat.extend(float(a) for a in (v.tolist() if hasattr(v, "tolist") else v))
    zs = (ctypes.c_double * max(1, len(flat)))(*flat)
    return ms, zs, tuple(int(len(v)) for v in nodes)


NOALLOC_SCRATCH_BYTES = 64 << 20


def ecdf_esf_grid(x: torch.Tensor, nodes, y=None, prec="f64", want_ecdf=True,
                  want_esf=True, stream=None, out=None, noalloc=False):
    """ECDF and/or ESF at every node of the rectilinear grid given by the
    per-axis node lists ``nodes`` (C ABI ``ecdf_esf_grid``).  Returns
    (F, Fbar), each of shape (M_1, ..., M_d) or None when not requested.
    ``out`` = (F, Fbar) writes into caller tensors; ``noalloc`` calls
    ``ecdf_esf_grid_noalloc`` (working memory in the library's fixed scratch
    array; with ``out`` given, nothing is allocated on the device)."""
    x = _x(x)
    d, n = x.shape
    if len(nodes) != d:
        raise ValueError("need one node vector per dimension")
    p = _prec(prec)
    y = _y(y, n, p, x)
    ms, zs, shape = _grid_args(nodes)
    dt = _out_dtype(y, p)
    if out is not None:
        F, Fb = out
        for t in (F, Fb):
            if t is not None and (t.dtype != dt or tuple(t.shape) != shape or
                                  not t.is_contiguous() or t.device != x.device):
                raise ValueError("out tensors must be contiguous %s of shape %s" % (dt, shape))
    else:
        F = torch.empty(shape, dtype=dt, device=x.device) if want_ecdf else None
        Fb = torch.empty(shape, dtype=dt, device=x.device) if want_esf else None
    fn = _lib.ecdf_esf_grid_noalloc if noalloc else _lib.ecdf_esf_grid
    rc = fn(d, n, _ptr(x), _ptr(y), ms, zs, _ptr(F), _ptr(Fb), p, _stream_ptr(stream))
    _check(rc, "ecdf_esf_grid_noalloc" if noalloc else "ecdf_esf_grid")
    return F, Fb


_lib.mecdf_grid_interp.argtypes = [_I, _P, _P, _P, _I64, _P, _P, _I, _P]
_lib.mecdf_grid_interp.restype = _I


def grid_interp(G: torch.Tensor, nodes, q: torch.Tensor, stream=None):
    """Multilinear interpolation of grid values G (shape (M_1, ..., M_d),
    float64 or float32 GPU tensor) at the points q (d, Q) (C ABI
    ``mecdf_grid_interp``).  Returns (Q,) of G's dtype."""
    q = _x(q)
    d, Q = q.shape
    if len(nodes) != d or G.dim() != d:
        raise ValueError("need one node vector per dimension of G and q")
    ms, zs, shape = _grid_args(nodes)
    if tuple(G.shape) != shape:
        raise ValueError("G's shape must be the node counts")
    if G.dtype == torch.float64:
        p = MECDF_F64
    elif G.dtype == torch.float32:
        p = MECDF_F32C
    else:
        raise TypeError("G must be float64 or float32")
    G = G.contiguous()
    out = torch.empty((Q,), dtype=G.dtype, device=q.device)
    _check(_lib.mecdf_grid_interp(d, ms, zs, _ptr(G), Q, _ptr(q), _ptr(out), p,
                                  _stream_ptr(stream)), "mecdf_grid_interp")
    return out


def ecdf_grid(x, nodes, y=None, prec="f64", stream=None):
    """F_N at every grid node (C ABI ``ecdf_grid``)."""
    x = _x(x)
    d, n = x.shape
    p = _prec(prec)
    y = _y(y, n, p, x)
    ms, zs, shape = _grid_args(nodes)
    F = torch.empty(shape, dtype=_out_dtype(y, p), device=x.device)
    _check(_lib.ecdf_grid(d, n, _ptr(x), _ptr(y), ms, zs, _ptr(F), p,
                          _stream_ptr(stream)), "ecdf_grid")
    return F


def esf_grid(x, nodes, y=None, prec="f64", stream=None):
    """Fbar_N at every grid node (C ABI ``esf_grid``)."""
    x = _x(x)
    d, n = x.shape
    p = _prec(prec)
    y = _y(y, n, p, x)
    ms, zs, shape = _grid_args(nodes)
    F = torch.empty(shape, dtype=_out_dtype(y, p), device=x.device)
    _check(_lib.esf_grid(d, n, _ptr(x), _ptr(y), ms, zs, _ptr(F), p,
                         _stream_ptr(stream)), "esf_grid")
    return F


def ecdf_points(x, y=None, prec="f64", stream=None):
    """F_N(x_j) at every sample point (C ABI ``ecdf_points``)."""
    x = _x(x)
    d, n = x.shape
    p = _prec(prec)
    y = _y(y, n, p, x)
    F = torch.empty((n,), dtype=_out_dtype(y, p), device=x.device)
    _check(_lib.ecdf_points(d, n, _ptr(x), _ptr(y), _ptr(F), p,
                            _stream_ptr(stream)), "ecdf_points")
    return F


def esf_points(x, y=None, prec="f64", stream=None):
    """Fbar_N(x_j) at every sample point (C ABI ``esf_points``)."""
    x = _x(x)
    d, n = x.shape
    p = _prec(prec)
    y = _y(y, n, p, x)
    F = torch.empty((n,), dtype=_out_dtype(y, p), device=x.device)
    _check(_lib.esf_points(d, n, _ptr(x), _ptr(y), _ptr(F), p,
                           _stream_ptr(stream)), "esf_points")
    return F


_lib.ecdf_delta_at.argtypes = [_I, _I64, _P, _P, _I64, _P, _P, _P, _I, _P]
_lib.ecdf_delta_at.restype = _I
_lib.kde_uniform.argtypes = [_I, _I64, _P, _P, _I64, _P, _I, _P, _P, _I, _P]
_lib.kde_uniform.restype = _I


def ecdf_delta_at(x, z, delta=None, y=None, prec="f64", stream=None):
    """F_N(z_q, delta_q) of eq. (ECDFdelta) at the points z (d, Q) (C ABI
    ``ecdf_delta_at``); delta: (Q,) uint8 masks on the device (bit k set:
    strict on axis k) or None.  int64 counts when y is None."""
    x = _x(x)
    d, n = x.shape
    z = _x(z)
    if z.shape[0] != d:
        raise ValueError("z must have the dimension of x")
    q = z.shape[1]
    p = _prec(prec)
    y = _y(y, n, p, x)
    if delta is not None:
        delta = delta.to(device=x.device, dtype=torch.uint8).contiguous()
        if delta.shape != (q,):
            raise ValueError("delta must have shape (Q,)")
    F = torch.empty((q,), dtype=_out_dtype(y, p), device=x.device)
    _check(_lib.ecdf_delta_at(d, n, _ptr(x), _ptr(y), q, _ptr(z), _ptr(delta), _ptr(F), p,
                              _stream_ptr(stream)), "ecdf_delta_at")
    return F


def kde_uniform(x, h, z=None, w=None, prec="f64", stream=None):
    """Uniform-kernel density estimate at the points z (default: the sample
    points) for each bandwidth row of h (C ABI ``kde_uniform``): (nh, Q)."""
    x = _x(x)
    d, n = x.shape
    z = x if z is None else _x(z)
    q = z.shape[1]
    p = _prec(prec)
    w = _y(w, n, p, x)
    hm = _hmat(h, d)
    hs = (ctypes.c_double * hm.size)(*hm.reshape(-1).tolist())
    dt = torch.float64 if p == MECDF_F64 else torch.float32
    f = torch.empty((hm.shape[0], q), dtype=dt, device=x.device)
    _check(_lib.kde_uniform(d, n, _ptr(x), _ptr(w), q, _ptr(z), hm.shape[0], hs, _ptr(f), p,
                            _stream_ptr(stream)), "kde_uniform")
    return f


def _hmat(h, d):
    import numpy as np

    h = np.asarray(h, dtype=np.float64)
    if h.ndim == 0:
        h = np.full((1, d), float(h))
    elif h.ndim == 1:
        h = np.repeat(h[:, None], d, 1)
    if h.ndim != 2 or h.shape[1] != d:
        raise ValueError("bandwidths must be scalar, (nh,) or (nh, d)")
    return np.ascontiguousarray(h)


def kde_laplace(x, h, w=None, prec="f64", want_f=True, want_lcv=True,
                stream=None):
    """Laplacian KDE at the sample points for each bandwidth row of h and the
    likelihood CV scores (C ABI ``kde_laplace``).  Returns (f, lcv):
    f of shape (nh, N) or None, lcv of shape (nh,) float64 or None."""
    x = _x(x)
    d, n = x.shape
    p = _prec(prec)
    w = _y(w, n, p, x)
    hm = _hmat(h, d)
    nh = hm.shape[0]
    hs = (ctypes.c_double * hm.size)(*hm.reshape(-1).tolist())
    dt = torch.float64 if p == MECDF_F64 else torch.float32
    f = torch.empty((nh, n), dtype=dt, device=x.device) if want_f else None
    lcv = torch.empty((nh,), dtype=torch.float64, device=x.device) if want_lcv else None
    _check(_lib.kde_laplace(d, n, _ptr(x), _ptr(w), nh, hs, _ptr(f), _ptr(lcv),
                            p, _stream_ptr(stream)), "kde_laplace")
    return f, lcv


def kreg_laplace(x, y, h, prec="f64", want_m=True, want_cv=True, stream=None):
    """Nadaraya-Watson regression at the sample points and squared-error LOO
    CV scores (C ABI ``kreg_laplace``).  Returns (m, cv)."""
    x = _x(x)
    d, n = x.shape
    p = _prec(prec)
    y = _y(y, n, p, x)
    if y is None:
        raise ValueError("kreg_laplace needs the response y")
    hm = _hmat(h, d)
    nh = hm.shape[0]
    hs = (ctypes.c_double * hm.size)(*hm.reshape(-1).tolist())
    dt = torch.float64 if p == MECDF_F64 else torch.float32
    m = torch.empty((nh, n), dtype=dt, device=x.device) if want_m else None
    cv = torch.empty((nh,), dtype=torch.float64, device=x.device) if want_cv else None
    _check(_lib.kreg_laplace(d, n, _ptr(x), _ptr(y), nh, hs, _ptr(m), _ptr(cv),
                             p, _stream_ptr(stream)), "kreg_laplace")
    return m, cv


_lib.kde_laplace_grid.argtypes = [_I, _I64, _P, _P, _P, _P, _I, _P, _P, _I, _P]
_lib.kde_laplace_grid.restype = _I
_lib.kreg_laplace_grid.argtypes = [_I, _I64, _P, _P, _P, _P, _I, _P, _P, _I, _P]
_lib.kreg_laplace_grid.restype = _I
_lib.kde_matern32_grid.argtypes = [_I, _I64, _P, _P, _P, _P, _I, _P, _P, _I, _P]
_lib.kde_matern32_grid.restype = _I
_lib.kreg_matern32_grid.argtypes = [_I, _I64, _P, _P, _P, _P, _I, _P, _P, _I, _P]
_lib.kreg_matern32_grid.restype = _I


def _grid_sums(fn, name, x, v, nodes, h, prec, stream):
    x = _x(x)
    d, n = x.shape
    p = _prec(prec)
    v = _y(v, n, p, x)
    ms, zs, shape = _grid_args(nodes)
    hm = _hmat(h, d)
    hs = (ctypes.c_double * hm.size)(*hm.reshape(-1).tolist())
    dt = torch.float64 if p == MECDF_F64 else torch.float32
    out = torch.empty((hm.shape[0],) + shape, dtype=dt, device=x.device)
    _check(fn(d, n, _ptr(x), _ptr(v), ms, zs, hm.shape[0], hs, _ptr(out), p,
              _stream_ptr(stream)), name)
    return out


def kde_matern32_grid(x, nodes, h, w=None, prec="f64", stream=None):
    """KDE with the additive Matern-3/2 kernel at every grid node (C ABI
    ``kde_matern32_grid``): (nh, M_1, ..., M_d) tensor."""
    return _grid_sums(_lib.kde_matern32_grid, "kde_matern32_grid", x, w, nodes, h, prec,
                      stream)


def kreg_matern32_grid(x, y, nodes, h, prec="f64", stream=None):
    """Nadaraya-Watson regression with the additive Matern-3/2 kernel at every
    grid node (C ABI ``kreg_matern32_grid``): (nh, M_1, ..., M_d) tensor."""
    if y is None:
        raise ValueError("kreg_matern32_grid needs the response y")
    return _grid_sums(_lib.kreg_matern32_grid, "kreg_matern32_grid", x, y, nodes, h, prec,
                      stream)


def kde_laplace_grid(x, nodes, h, w=None, prec="f64", stream=None):
    """Laplacian KDE at every grid node (C ABI ``kde_laplace_grid``):
    (nh, M_1, ..., M_d) tensor."""
    x = _x(x)
    d, n = x.shape
    p = _prec(prec)
    w = _y(w, n, p, x)
    ms, zs, shape = _grid_args(nodes)
    hm = _hmat(h, d)
    hs = (ctypes.c_double * hm.size)(*hm.reshape(-1).tolist())
    dt = torch.float64 if p == MECDF_F64 else torch.float32
    f = torch.empty((hm.shape[0],) + shape, dtype=dt, device=x.device)
    _check(_lib.kde_laplace_grid(d, n, _ptr(x), _ptr(w), ms, zs, hm.shape[0], hs, _ptr(f), p,
                                 _stream_ptr(stream)), "kde_laplace_grid")
    return f


def kreg_laplace_grid(x, y, nodes, h, prec="f64", stream=None):
    """Nadaraya-Watson regression at every grid node (C ABI
    ``kreg_laplace_grid``): (nh, M_1, ..., M_d) tensor."""
    x = _x(x)
    d, n = x.shape
    p = _prec(prec)
    y = _y(y, n, p, x)
    if y is None:
        raise ValueError("kreg_laplace_grid needs the response y")
    ms, zs, shape = _grid_args(nodes)
    hm = _hmat(h, d)
    hs = (ctypes.c_double * hm.size)(*hm.reshape(-1).tolist())
    dt = torch.float64 if p == MECDF_F64 else torch.float32
    m = torch.empty((hm.shape[0],) + shape, dtype=dt, device=x.device)
    _check(_lib.kreg_laplace_grid(d, n, _ptr(x), _ptr(y), ms, zs, hm.shape[0], hs, _ptr(m), p,
                                  _stream_ptr(stream)), "kreg_laplace_grid")
    return m


_lib.kde_laplace_H.argtypes = [_I, _I64, _P, _P, _I, _P, _P, _P, _I, _P]
_lib.kde_laplace_H.restype = _I
_lib.kreg_laplace_H.argtypes = [_I, _I64, _P, _P, _I, _P, _P, _P, _I, _P]
_lib.kreg_laplace_H.restype = _I
_lib.kreg_loclin_laplace.argtypes = [_I, _I64, _P, _P, _I, _P, _P, _I, _P]
_lib.kreg_loclin_laplace.restype = _I


def _hmats(Hs, d):
    import numpy as np

    H = np.ascontiguousarray(np.asarray(Hs, dtype=np.float64))
    if H.ndim == 2:
        H = H[None]
    if H.ndim != 3 or H.shape[1:] != (d, d):
        raise ValueError("bandwidth matrices must be (nh, d, d)")
    return H, (ctypes.c_double * H.size)(*H.reshape(-1).tolist())


def kde_laplace_H(x, Hs, w=None, prec="f64", want_f=True, want_lcv=True, stream=None):
    """kde_laplace with bandwidth matrices (C ABI ``kde_laplace_H``)."""
    x = _x(x)
    d, n = x.shape
    p = _prec(prec)
    w = _y(w, n, p, x)
    H, hs = _hmats(Hs, d)
    dt = torch.float64 if p == MECDF_F64 else torch.float32
    f = torch.empty((H.shape[0], n), dtype=dt, device=x.device) if want_f else None
    lcv = torch.empty((H.shape[0],), dtype=torch.float64, device=x.device) if want_lcv else None
    _check(_lib.kde_laplace_H(d, n, _ptr(x), _ptr(w), H.shape[0], hs, _ptr(f), _ptr(lcv), p,
                              _stream_ptr(stream)), "kde_laplace_H")
    return f, lcv


def kreg_laplace_H(x, y, Hs, prec="f64", want_m=True, want_cv=True, stream=None):
    """kreg_laplace with bandwidth matrices (C ABI ``kreg_laplace_H``)."""
    x = _x(x)
    d, n = x.shape
    p = _prec(prec)
    y = _y(y, n, p, x)
    H, hs = _hmats(Hs, d)
    dt = torch.float64 if p == MECDF_F64 else torch.float32
    m = torch.empty((H.shape[0], n), dtype=dt, device=x.device) if want_m else None
    cv = torch.empty((H.shape[0],), dtype=torch.float64, device=x.device) if want_cv else None
    _check(_lib.kreg_laplace_H(d, n, _ptr(x), _ptr(y), H.shape[0], hs, _ptr(m), _ptr(cv), p,
                               _stream_ptr(stream)), "kreg_laplace_H")
    return m, cv


def kreg_loclin_laplace(x, y, h, prec="f64", stream=None):
    """Local-linear regression at the sample points (C ABI
    ``kreg_loclin_laplace``): (nh, N)."""
    x = _x(x)
    d, n = x.shape
    p = _prec(prec)
    y = _y(y, n, p, x)
    hm = _hmat(h, d)
    hs = (ctypes.c_double * hm.size)(*hm.reshape(-1).tolist())
    dt = torch.float64 if p == MECDF_F64 else torch.float32
    m = torch.empty((hm.shape[0], n), dtype=dt, device=x.device)
    _check(_lib.kreg_loclin_laplace(d, n, _ptr(x), _ptr(y), hm.shape[0], hs, _ptr(m), p,
                                    _stream_ptr(stream)), "kreg_loclin_laplace")
    return m


def release():
    """Free the library's device workspaces."""
    _lib.mecdf_release()


# ---------------------------------------------------------------- profiling
_lib.mecdf_profile_enable.argtypes = [_I]
_lib.mecdf_profile_enable.restype = _I
_lib.mecdf_profile_reset.argtypes = []
_lib.mecdf_profile_reset.restype = None
_lib.mecdf_profile_collect.argtypes = [_I, _P, _P, _P]
_lib.mecdf_profile_collect.restype = _I


def profile_enable(on=True, cold: bool = False):
    """Bracket every library kernel launch with HIP events (timing only);
    with cold, a 1 GiB buffer is read before each bracketed group so that its
    inputs come from HBM rather than the infinity cache."""
    _check(_lib.mecdf_profile_enable((2 if cold else 1) if on else 0), "mecdf_profile_enable")


def profile_reset():
    _lib.mecdf_profile_reset()


def profile_collect(max_names: int = 64):
    """{kernel name: (total ms, launches)} for the launches recorded since the
    last reset; waits for the recorded events."""
    names = ctypes.create_string_buffer(64 * max_names)
    ms = (ctypes.c_double * max_names)()
    cnt = (ctypes.c_int64 * max_names)()
    n = _lib.mecdf_profile_collect(max_names, names, ms, cnt)
    if n < 0:
        raise MecdfError(n, "mecdf_profile_collect")
    out = {}
    for i in range(n):
        nm = names.raw[64 * i:64 * (i + 1)].split(b"\0", 1)[0].decode()
        out[nm] = (float(ms[i]), int(cnt[i]))
    return out


# ------------------------------------------------------- bandwidth selection
MLP_PARAMS = 20865
N_FEATURES = 32


class _Dataset(ctypes.Structure):
    _fields_ = [("d", ctypes.c_int), ("N", ctypes.c_int64), ("x", ctypes.c_void_p)]


_lib.mecdf_kde_lcv_batched.argtypes = [_P, _I, _P, _P, _P, _P, _I, _P]
_lib.mecdf_kde_lcv_batched.restype = _I
_lib.mecdf_bw_features.argtypes = [_P, _I, _P, _P]
_lib.mecdf_bw_features.restype = _I
_lib.mecdf_mlp_forward.argtypes = [_I, _P, _P, _P, _P]
_lib.mecdf_mlp_forward.restype = _I
_lib.mecdf_mlp_grad.argtypes = [_I, _P, _P, _P, _P, _P, _P]
_lib.mecdf_mlp_grad.restype = _I
_lib.mecdf_mlp_train.argtypes = [_I, _P, _P, _P, _P, _I, ctypes.c_float, ctypes.c_float, _P, _P]
_lib.mecdf_mlp_train.restype = _I
_lib.mecdf_bw_select.argtypes = [_P, _I, _P, _I, _P, _I, _P, _P, _P, _P]
_lib.mecdf_bw_select.restype = _I
_lib.mecdf_bw_train.argtypes = [_I, _P, _P, _I, _P, _I, ctypes.c_float, ctypes.c_float,
                                ctypes.c_uint64, _P, _P, _P, ctypes.c_char_p, _P, _P]
_lib.mecdf_bw_train.restype = _I


def _sets(datasets):
    arr = (_Dataset * len(datasets))()
    keep = []
    for i, x in enumerate(datasets):
        x = _x(x)
        keep.append(x)
        arr[i].d = x.shape[0]
        arr[i].N = x.shape[1]
        arr[i].x = x.data_ptr()
    return arr, keep


def kde_lcv_batched(datasets, hs, prec="f64", stream=None, want_best=False):
    """LCV scores for a list of (d, N) GPU datasets; hs[i] is the list of
    isotropic bandwidths of dataset i.  Returns a list of (len(hs[i]),) float64
    GPU tensors (C ABI ``mecdf_kde_lcv_batched``), and with want_best also the
    (nsets,) int32 GPU tensor of each dataset's best index."""
    arr, keep = _sets(datasets)
    nh = (ctypes.c_int * len(datasets))(*[len(h) for h in hs])
    flat = [float(v) for h in hs for v in h]
    hv = (ctypes.c_double * max(1, len(flat)))(*flat)
    out = torch.empty((max(1, len(flat)),), dtype=torch.float64, device=keep[0].device)
    best = torch.empty((len(datasets),), dtype=torch.int32, device=keep[0].device) \
        if want_best else None
    _check(_lib.mecdf_kde_lcv_batched(ctypes.addressof(arr), len(datasets), nh, hv,
                                      _ptr(out), _ptr(best), _prec(prec), _stream_ptr(stream)),
           "mecdf_kde_lcv_batched")
    res, off = [], 0
    for h in hs:
        res.append(out[off:off + len(h)])
        off += len(h)
    return (res, best) if want_best else res


_lib.mecdf_lcv_plan_create.argtypes = [_P, _I, _P, _P, _P, _P, _I, _P]
_lib.mecdf_lcv_plan_create.restype = _I
_lib.mecdf_lcv_plan_run.argtypes = [_P, _P]
_lib.mecdf_lcv_plan_run.restype = _I
_lib.mecdf_lcv_plan_destroy.argtypes = [_P]
_lib.mecdf_lcv_plan_destroy.restype = None
_lib.mecdf_autotune.argtypes = [ctypes.c_char_p, _P]
_lib.mecdf_autotune.restype = _I
_lib.mecdf_tuning.argtypes = [_P, ctypes.c_char_p, _I]
_lib.mecdf_tuning.restype = _I
_lib.mecdf_tuning_set.argtypes = [_P]
_lib.mecdf_tuning_set.restype = _I


class LcvPlan:
    """The batched scores of a fixed list of datasets recorded into a HIP
    graph (C ABI ``mecdf_lcv_plan_*``); ``run()`` replays it and returns the
    same outputs as :func:`kde_lcv_batched` (written in place each run)."""

    def __init__(self, datasets, hs, prec="f64", want_best=True):
        arr, self._keep = _sets(datasets)
        nh = (ctypes.c_int * len(datasets))(*[len(h) for h in hs])
        flat = [float(v) for h in hs for v in h]
        hv = (ctypes.c_double * max(1, len(flat)))(*flat)
        dev = self._keep[0].device
        self.out = torch.empty((max(1, len(flat)),), dtype=torch.float64, device=dev)
        self.best = torch.empty((len(datasets),), dtype=torch.int32, device=dev) \
            if want_best else None
        self._hs = [len(h) for h in hs]
        self._plan = ctypes.c_void_p()
        _check(_lib.mecdf_lcv_plan_create(ctypes.addressof(arr), len(datasets), nh, hv,
                                          _ptr(self.out), _ptr(self.best), _prec(prec),
                                          ctypes.byref(self._plan)), "mecdf_lcv_plan_create")

    def run(self, stream=None):
        _check(_lib.mecdf_lcv_plan_run(self._plan, _stream_ptr(stream)), "mecdf_lcv_plan_run")
        res, off = [], 0
        for k in self._hs:
            res.append(self.out[off:off + k])
            off += k
        return res, self.best

    def close(self):
        if self._plan:
            _lib.mecdf_lcv_plan_destroy(self._plan)
            self._plan = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def autotune(path=None, stream=None):
    """Time the work queue against the recursion on this GPU and store the
    choice (C ABI ``mecdf_autotune``)."""
    ck = None if path is None else os.fsencode(path)
    _check(_lib.mecdf_autotune(ck, _stream_ptr(stream)), "mecdf_autotune")


def tuning_set(queue_max_n):
    """Replace the queue sizes for this process: {"f64": [d1, d2, d3], "f32c":
    [...]} (C ABI ``mecdf_tuning_set``)."""
    v = (ctypes.c_int64 * 6)(*(list(queue_max_n["f64"]) + list(queue_max_n["f32c"])))
    _check(_lib.mecdf_tuning_set(v), "mecdf_tuning_set")


def tuning():
    """(queue_max_n as {"f64": [d1, d2, d3], "f32c": [...]}, source)."""
    v = (ctypes.c_int64 * 6)()
    src = ctypes.create_string_buffer(4096)
    _check(_lib.mecdf_tuning(v, src, 4096), "mecdf_tuning")
    return {"f64": list(v[0:3]), "f32c": list(v[3:6])}, src.value.decode()


def bw_features(datasets, stream=None):
    """(nsets, 32) float32 GPU tensor of summary features (C ABI
    ``mecdf_bw_features``)."""
    arr, keep = _sets(datasets)
    feat = torch.empty((len(datasets), N_FEATURES), dtype=torch.float32, device=keep[0].device)
    _check(_lib.mecdf_bw_features(ctypes.addressof(arr), len(datasets), _ptr(feat),
                                  _stream_ptr(stream)), "mecdf_bw_features")
    return feat


def _f32(t):
    if not (t.is_cuda and t.dtype == torch.float32):
        raise TypeError("expected a float32 GPU tensor")
    return t.contiguous()


def mlp_forward(feat, params, stream=None):
    feat = _f32(feat)
    params = _f32(params)
    out = torch.empty((feat.shape[0],), dtype=torch.float32, device=feat.device)
    _check(_lib.mecdf_mlp_forward(feat.shape[0], _ptr(feat), _ptr(params), _ptr(out),
                                  _stream_ptr(stream)), "mecdf_mlp_forward")
    return out


def mlp_grad(feat, target, params, stream=None):
    feat, target, params = _f32(feat), _f32(target), _f32(params)
    grad = torch.empty((MLP_PARAMS,), dtype=torch.float32, device=feat.device)
    loss = torch.empty((1,), dtype=torch.float32, device=feat.device)
    _check(_lib.mecdf_mlp_grad(feat.shape[0], _ptr(feat), _ptr(target), _ptr(params),
                               _ptr(grad), _ptr(loss), _stream_ptr(stream)), "mecdf_mlp_grad")
    return grad, loss


def mlp_train(feat, target, params, adam, steps, lr, wd=0.0, stream=None):
    """In-place Adam steps (decoupled weight decay wd) on params (float32 GPU
    vector); returns the losses."""
    feat, target = _f32(feat), _f32(target)
    if not (params.is_cuda and params.dtype == torch.float32 and params.is_contiguous()):
        raise TypeError("params must be a contiguous float32 GPU tensor")
    losses = torch.empty((max(1, steps),), dtype=torch.float32, device=feat.device)
    _check(_lib.mecdf_mlp_train(feat.shape[0], _ptr(feat), _ptr(target), _ptr(params),
                                _ptr(adam), int(steps), float(lr), float(wd), _ptr(losses),
                                _stream_ptr(stream)), "mecdf_mlp_train")
    return losses[:steps]


def bw_train(feat, label, hgrid, steps, lr, wd=0.0, seed=0, params=None, adam=None,
             step=0, checkpoint=None, stream=None):
    """Train the proposal network on grid labels (C ABI ``mecdf_bw_train``).
    feat: (B, 32) float32 GPU features; label: (B,) int32 GPU grid indices.
    params / adam: float32 GPU vectors (allocated when None; then step must
    be 0, so that they are initialised from the seed).  Returns (params,
    adam, losses, total steps)."""
    feat = _f32(feat)
    if not (label.is_cuda and label.dtype == torch.int32):
        raise TypeError("label must be an int32 GPU tensor")
    label = label.contiguous()
    dev = feat.device
    if params is None:
        params = torch.empty((MLP_PARAMS,), dtype=torch.float32, device=dev)
    if adam is None:
        adam = torch.empty((2 * MLP_PARAMS,), dtype=torch.float32, device=dev)
    for t in (params, adam):
        if not (t.is_cuda and t.dtype == torch.float32 and t.is_contiguous()):
            raise TypeError("params and adam must be contiguous float32 GPU tensors")
    hg = (ctypes.c_double * len(hgrid))(*[float(v) for v in hgrid])
    losses = torch.empty((max(1, steps),), dtype=torch.float32, device=dev)
    st = ctypes.c_int64(int(step))
    ck = None if checkpoint is None else os.fsencode(checkpoint)
    _check(_lib.mecdf_bw_train(feat.shape[0], _ptr(feat), _ptr(label), len(hgrid), hg,
                               int(steps), float(lr), float(wd), int(seed), _ptr(params),
                               _ptr(adam), _ptr(losses), ck, ctypes.byref(st),
                               _stream_ptr(stream)), "mecdf_bw_train")
    return params, adam, losses[:steps], int(st.value)


BW_EXTEND = 0
BW_WINDOW = 1


def bw_select(datasets, params, hgrid, mode=BW_EXTEND, stream=None):
    """Learned-proposal LCV bandwidth selection (C ABI ``mecdf_bw_select``):
    mode BW_EXTEND widens the window until its best score is interior,
    BW_WINDOW keeps the four grid points around the proposal.  Returns numpy
    arrays (grid index, exact LCV there, bandwidths evaluated)."""
    import numpy as np

    arr, keep = _sets(datasets)
    params = _f32(params)
    n = len(datasets)
    hg = (ctypes.c_double * len(hgrid))(*[float(v) for v in hgrid])
    hidx = (ctypes.c_int * n)()
    lcv = (ctypes.c_double * n)()
    ev = (ctypes.c_int * n)()
    _check(_lib.mecdf_bw_select(ctypes.addressof(arr), n, _ptr(params), len(hgrid), hg,
                                int(mode), hidx, lcv, ev, _stream_ptr(stream)),
           "mecdf_bw_select")
    return (np.array(hidx[:], dtype=np.int64), np.array(lcv[:], dtype=np.float64),
            np.array(ev[:], dtype=np.int64))
