"""CPU FP64 oracle of the implicit radiation diffusion step (TEST INFRASTRUCTURE).

Only the tests, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import this module.  The arithmetic lives in
``fld_oracle.cpp``: the flux-limited diffusion coefficient, one backward-Euler
step of the diffusion equation and its geometric multigrid V-cycle solver
(paper sections 2.2.1 and 2.2.2; the file header lists the readings).

States are oracle ``Grid`` states with the radiation field
(``Grid(..., rad=(kappa, mu))``): field 0 is rho, the last field is E_r.
"""
import ctypes
import os

import numpy as np

from . import Grid, _as_state, _dptr
from . import build as _build

EDDINGTON, LEVERMORE = 0, 1  # flux limiter: lambda = 1/3, or Levermore's lambda(R)

_lib = None


def use_library(path):
    """Load another build of fld_oracle.cpp (the mutation tests compile
    deliberately broken copies and check that the pins fail)."""
    global _lib
    _lib = None
    return lib(path)


def lib(path=None):
    global _lib
    if _lib is None:
        if path is None:
            path = os.environ.get("HARD_FLD_ORACLE_LIB") or _build.FLD_LIB
            if not os.path.exists(path):
                _build.build_fld()
        L = ctypes.CDLL(path)
        i64p = ctypes.POINTER(ctypes.c_int64)
        dp = ctypes.POINTER(ctypes.c_double)
        ip = ctypes.POINTER(ctypes.c_int)
        geo = [ctypes.c_int, i64p, dp, ip]
        L.oracle_levermore.argtypes = [ctypes.c_double]
        L.oracle_levermore.restype = ctypes.c_double
        L.oracle_gmg_levels.argtypes = geo + [ctypes.c_int, i64p]
        L.oracle_gmg_levels.restype = ctypes.c_int
        L.oracle_fld_coefficient.argtypes = geo + [ctypes.c_double, ctypes.c_int, dp,
                                                   ctypes.c_int, dp]
        L.oracle_fld_coefficient.restype = ctypes.c_int
        L.oracle_fld_apply.argtypes = geo + [ctypes.c_double, ctypes.c_int, ctypes.c_double, dp,
                                             ctypes.c_int, dp, dp]
        L.oracle_fld_apply.restype = ctypes.c_int
        L.oracle_rad_diffuse.argtypes = geo + [ctypes.c_double, ctypes.c_int, ctypes.c_double,
                                               ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                               ctypes.c_int, dp, ctypes.c_int, dp]
        L.oracle_rad_diffuse.restype = ctypes.c_int
        _lib = L
    return _lib


def _geo(g: Grid):
    a = g._args()
    return [a[0], a[1], a[2], a[4]]


def _kappa(g: Grid):
    if g.rad is None:
        raise ValueError("the grid has no radiation field")
    return float(g.rad[0])


def levermore(R):
    """Levermore's flux limiter lambda(R)."""
    return lib().oracle_levermore(float(R))


def gmg_levels(g: Grid):
    """Sizes (n_x, n_y, n_z) of every multigrid level, finest first."""
    out = (ctypes.c_int64 * (3 * 64))()
    nl = lib().oracle_gmg_levels(*_geo(g), 64, out)
    return [tuple(out[3 * l + d] for d in range(3)) for l in range(nl)]


def fld_coefficient(g: Grid, U, limiter=LEVERMORE):
    """D = c lambda / (kappa rho) per cell (array of the grid's cell shape) and
    the status (1: non-physical cell, -1: grid not supported)."""
    U = _as_state(g, U)
    D = np.empty(U.shape[1:])
    st = lib().oracle_fld_coefficient(*_geo(g), _kappa(g), int(limiter), _dptr(U), g.nvar,
                                      _dptr(D))
    return D, st


def fld_apply(g: Grid, U, dt, x, limiter=LEVERMORE):
    """y = (I - dt div D grad) x with D from U."""
    U = _as_state(g, U)
    x = np.ascontiguousarray(x, dtype=np.float64)
    assert x.shape == U.shape[1:]
    y = np.empty_like(x)
    st = lib().oracle_fld_apply(*_geo(g), _kappa(g), int(limiter), float(dt), _dptr(U), g.nvar,
                                _dptr(x), _dptr(y))
    return y, st


def rad_diffuse(g: Grid, U, dt, ncycles=4, nu1=2, nu2=2, ncoarse=8, limiter=LEVERMORE):
    """One backward-Euler diffusion step of E_r by `ncycles` V(nu1, nu2) cycles.

    Returns (U_new, status, resid) with resid[k] the finest-grid residual
    2-norm after k cycles (k = 0..ncycles).
    """
    X = _as_state(g, U).copy()
    resid = np.empty(ncycles + 1)
    st = lib().oracle_rad_diffuse(*_geo(g), _kappa(g), int(limiter), float(dt), int(ncycles),
                                  int(nu1), int(nu2), int(ncoarse), _dptr(X), g.nvar,
                                  _dptr(resid))
    return X, st, resid
