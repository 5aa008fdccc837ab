"""Exact multivariate ECDF / ESF and Laplacian kernel sums on AMD MI355X.

The compute path is the HIP library ``_lib/libmecdf.so`` (C ABI in
``include/mecdf.h``); :mod:`paper_2005_03246_amd.mecdf` is its thin binding.
Attribute access such as ``paper_2005_03246_amd.ecdf_grid`` loads that
binding and raises if the library has not been built.
"""

_BINDING_NAMES = {
    "ecdf_grid", "esf_grid", "ecdf_esf_grid", "ecdf_points", "esf_points",
    "kde_laplace", "kreg_laplace", "release", "MecdfError",
}


def __getattr__(name):
    if name in _BINDING_NAMES:
        from . import mecdf

        return getattr(mecdf, name)
    raise AttributeError(name)
