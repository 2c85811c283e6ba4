"""CPU FP64 oracle of the explicit hydro step (TEST INFRASTRUCTURE).

Only the tests, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import this package.  The product path (``libhard`` and its
Python binding) never touches it, and the two share no code.

The arithmetic lives in ``hydro_oracle.cpp`` (primitive recovery, MUSCL-minmod,
HLLC, flux difference, Heun/SSP-RK2, CFL dt; see that file's header for the
paper passages each part follows).  ``exact_riemann.py`` holds the exact
solution of the 1D Riemann problem used to pin the oracle, and ``metrics.py``
the L1 error of the paper's section 3 (equation "l1_error").

Arrays are NumPy float64 in the layout ``U[nvar][nz][ny][nx]`` (x fastest),
``nvar = ndim + 2`` with fields (rho, m_x[, m_y[, m_z]], E).
"""
import ctypes
import os
from dataclasses import dataclass, field
from typing import Sequence

import numpy as np

from . import build as _build

PERIODIC, OUTFLOW, REFLECT = 0, 1, 2
MUSCL_HLLC, WENO5Z_HLL = 0, 1  # face reconstruction + flux schemes

_lib = None


def use_library(path):
    """Load the oracle from another build of hydro_oracle.cpp (the mutation
    tests compile deliberately broken copies and check that the pins fail)."""
    global _lib
    _lib = None
    return lib(path)


def lib(path=None):
    """Load liboracle.so, compiling it only if it is not there."""
    global _lib
    if _lib is None:
        if path is None:
            path = os.environ.get("HARD_ORACLE_LIB") or _build.LIB
            if not os.path.exists(path):
                _build.build()
        L = ctypes.CDLL(path)
        i64p = ctypes.POINTER(ctypes.c_int64)
        dp = ctypes.POINTER(ctypes.c_double)
        ip = ctypes.POINTER(ctypes.c_int)
        common = [ctypes.c_int, i64p, dp, ctypes.c_double, ip, ctypes.c_int, dp]
        L.oracle_rhs.argtypes = common + [dp, dp]
        L.oracle_rhs.restype = ctypes.c_int
        L.oracle_step.argtypes = common + [ctypes.c_double, dp]
        L.oracle_step.restype = ctypes.c_int
        L.oracle_steps_fixed.argtypes = common + [ctypes.c_int64, dp, dp]
        L.oracle_steps_fixed.restype = ctypes.c_int
        L.oracle_cfl_dt.argtypes = common + [ctypes.c_double, dp, ip]
        L.oracle_cfl_dt.restype = ctypes.c_double
        L.oracle_run.argtypes = common + [ctypes.c_double, ctypes.c_double, ctypes.c_int64, dp,
                                          dp, i64p, dp]
        L.oracle_run.restype = ctypes.c_int
        L.oracle_steps_tangent.argtypes = common + [ctypes.c_int64, dp, dp, dp]
        L.oracle_steps_tangent.restype = ctypes.c_int
        L.oracle_hllc.argtypes = [ctypes.c_int, ctypes.c_double, dp, dp, dp]
        L.oracle_hllc.restype = None
        L.oracle_minmod.argtypes = [ctypes.c_double, ctypes.c_double]
        L.oracle_minmod.restype = ctypes.c_double
        L.oracle_hll.argtypes = [ctypes.c_int, ctypes.c_double, dp, dp, dp]
        L.oracle_hll.restype = None
        L.oracle_weno5z.argtypes = [dp]
        L.oracle_weno5z.restype = ctypes.c_double
        L.oracle_weno5z_indicators.argtypes = [dp, dp]
        L.oracle_weno5z_indicators.restype = None
        L.oracle_threads.argtypes = []
        L.oracle_threads.restype = ctypes.c_int
        L.oracle_steps_tangent_multi.argtypes = common + [ctypes.c_int64, dp, ctypes.c_int,
                                                               dp, dp]
        L.oracle_steps_tangent_multi.restype = ctypes.c_int
        L.oracle_branch_signature.argtypes = common + [ctypes.c_int64, dp, dp]
        L.oracle_branch_signature.restype = ctypes.c_uint64
        L.oracle_set_threads.argtypes = [ctypes.c_int]
        L.oracle_set_threads.restype = None
        L.oracle_count_ops.argtypes = common + [ctypes.c_double, dp, i64p]
        L.oracle_count_ops.restype = None
        _lib = L
    return _lib


@dataclass
class Grid:
    """Uniform Cartesian grid on [0,1]^ndim (dx = 1/n unless given)."""
    n: Sequence[int]
    gamma: float = 1.4
    bc: Sequence[int] = (OUTFLOW, OUTFLOW)  # (lo, hi) per axis, flattened
    dx: Sequence[float] = field(default=None)
    scheme: int = 0  # MUSCL_HLLC or WENO5Z_HLL
    rad: Sequence[float] = None  # (kappa, mu): radiation energy density as one more field

    def __post_init__(self):
        self.n = tuple(int(v) for v in self.n)
        if self.dx is None:
            self.dx = tuple(1.0 / v for v in self.n)
        self.dx = tuple(float(v) for v in self.dx)
        bc = tuple(int(v) for v in self.bc)
        if len(bc) == 2 and self.ndim > 1:
            bc = bc * self.ndim
        self.bc = bc
        assert len(self.bc) == 2 * self.ndim
        assert self.scheme in (MUSCL_HLLC, WENO5Z_HLL)
        ng = 3 if self.scheme == WENO5Z_HLL else 2
        assert min(self.n) >= ng, f"need at least {ng} cells per axis"

    @property
    def ndim(self):
        return len(self.n)

    @property
    def nvar(self):
        return self.ndim + 2 + (self.rad is not None)

    @property
    def shape(self):
        """Array shape (nvar, [nz, [ny,]] nx)."""
        return (self.nvar,) + tuple(reversed(self.n))

    def _args(self):
        n3 = (ctypes.c_int64 * 3)(*(list(self.n) + [1] * (3 - self.ndim)))
        dx3 = (ctypes.c_double * 3)(*(list(self.dx) + [1.0] * (3 - self.ndim)))
        bc6 = (ctypes.c_int * 6)(*(list(self.bc) + [0] * (6 - 2 * self.ndim)))
        radp = None if self.rad is None else (ctypes.c_double * 2)(*[float(v) for v in self.rad])
        return [self.ndim, n3, dx3, self.gamma, bc6, int(self.scheme), radp]


def _dptr(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _as_state(g: Grid, U):
    U = np.ascontiguousarray(U, dtype=np.float64)
    if U.shape != g.shape:
        raise ValueError(f"state shape {U.shape} != {g.shape}")
    return U


def rhs(g: Grid, U):
    """L(U) and the status bits of U."""
    U = _as_state(g, U)
    L = np.empty_like(U)
    st = lib().oracle_rhs(*g._args(), _dptr(U), _dptr(L))
    return L, st


def step(g: Grid, U, dt):
    """One SSP-RK2 step; returns (U_new, status)."""
    X = _as_state(g, U).copy()
    st = lib().oracle_step(*g._args(), float(dt), _dptr(X))
    return X, st


def steps(g: Grid, U, dts):
    """len(dts) steps with the given dt list; returns (U_new, status)."""
    X = _as_state(g, U).copy()
    d = np.ascontiguousarray(dts, dtype=np.float64)
    st = lib().oracle_steps_fixed(*g._args(), len(d), _dptr(d), _dptr(X))
    return X, st


def cfl_dt(g: Grid, U, cfl):
    """dt = cfl / max_i sum_d (|u_d| + c)/dx_d; returns (dt, status)."""
    U = _as_state(g, U)
    st = ctypes.c_int(0)
    dt = lib().oracle_cfl_dt(*g._args(), float(cfl), _dptr(U), ctypes.byref(st))
    return dt, st.value


def run(g: Grid, U, cfl, t_end, max_steps=10_000_000, record_dts=False):
    """CFL-driven run to t_end.  Returns (U, t, nsteps, status[, dts])."""
    X = _as_state(g, U).copy()
    t = ctypes.c_double(0.0)
    ns = ctypes.c_int64(0)
    dts = np.empty(max_steps if record_dts else 0)
    st = lib().oracle_run(*g._args(), float(cfl), float(t_end), int(max_steps), _dptr(X),
                          ctypes.byref(t), ctypes.byref(ns),
                          _dptr(dts) if record_dts else None)
    out = (X, t.value, ns.value, st)
    if record_dts:
        out = out + (dts[:ns.value].copy(),)
    return out


def steps_tangent(g: Grid, U, dU, dts):
    """Forward-mode derivative of len(dts) steps with frozen dts.

    Returns (U_n, dU_n, status): dU_n = (d step^n / dU) . dU exactly for the
    branches taken at U.
    """
    X = _as_state(g, U).copy()
    D = _as_state(g, dU).copy()
    d = np.ascontiguousarray(dts, dtype=np.float64)
    st = lib().oracle_steps_tangent(*g._args(), len(d), _dptr(d), _dptr(X), _dptr(D))
    return X, D, st


def steps_tangent_multi(g: Grid, U, dUs, dts):
    """Forward-mode derivatives of len(dts) steps with frozen dts along
    len(dUs) directions at once (1, 2, 4 or 8), by one evaluation with
    dual numbers of that many components.

    Returns (U_n, [dU_n per direction], status).
    """
    X = _as_state(g, U).copy()
    K = len(dUs)
    D = np.ascontiguousarray(np.stack([_as_state(g, d) for d in dUs]))
    d = np.ascontiguousarray(dts, dtype=np.float64)
    st = lib().oracle_steps_tangent_multi(*g._args(), len(d), _dptr(d), K, _dptr(X),
                                          _dptr(D))
    if st < 0:
        raise ValueError("1, 2, 4 or 8 directions")
    return X, [D[k] for k in range(K)], st


def branch_signature(g: Grid, U, dts):
    """64-bit hash of the outcome of every comparison that len(dts) steps
    from U with the step sizes dts make (minmod picks, wave-speed min/max,
    HLLC regions, |x|), in evaluation order: two inputs with the same
    signature take the same branches everywhere."""
    X = np.ascontiguousarray(_as_state(g, U), dtype=np.float64)
    d = np.ascontiguousarray(dts, dtype=np.float64)
    return int(lib().oracle_branch_signature(*g._args(), len(d), _dptr(d), _dptr(X)))


def hllc(WL, WR, gamma=1.4):
    """HLLC flux for face states (rho, un, ut..., p) -> (mass, mom_n, mom_t..., energy)."""
    WL = np.ascontiguousarray(WL, dtype=np.float64)
    WR = np.ascontiguousarray(WR, dtype=np.float64)
    nt = WL.size - 3
    F = np.empty(nt + 3)
    lib().oracle_hllc(nt, float(gamma), _dptr(WL), _dptr(WR), _dptr(F))
    return F


OP_KINDS = ("add", "mul", "div", "sqrt", "cmp", "abs")


def count_ops(g: Grid, U, dt):
    """Floating-point operations of one CFL dt plus one SSP-RK2 step of U, by
    kind (add/sub, mul, div, sqrt, compare, abs), as the oracle evaluates them
    (ghost cells included).  Runs on one thread."""
    U = _as_state(g, U)
    out = (ctypes.c_int64 * 6)()
    lib().oracle_count_ops(*g._args(), float(dt), _dptr(U), out)
    return dict(zip(OP_KINDS, list(out)))


def ops_per_zone_update(ndim, U_of_n, n_small, n_large, bc=None, dt=1e-4):
    """Operations per zone-update without the ghost-layer overhead: counts on
    an n_small^d and an n_large^d grid, with ops(n) = a n^d + b n^(d-1) solved
    for a per kind (the ghost-cell and extra-face work grows with n^(d-1))."""
    out = {}
    res = []
    for n in (n_small, n_large):
        g = Grid((n,) * ndim, bc=bc or (PERIODIC, PERIODIC))
        res.append(count_ops(g, U_of_n(n), dt))
    a, b = float(n_small), float(n_large)
    for k in OP_KINDS:
        c1, c2 = res[0][k] / a ** (ndim - 1), res[1][k] / b ** (ndim - 1)
        out[k] = (c2 - c1) / (b - a)
    return out


def threads():
    """OpenMP threads the oracle's loops use."""
    return lib().oracle_threads()


def set_threads(n):
    """Use n OpenMP threads from now on (the results are the same for any n)."""
    lib().oracle_set_threads(int(n))


def minmod(a, b):
    return lib().oracle_minmod(float(a), float(b))


def hll(WL, WR, gamma=1.4):
    """HLL flux for face states (rho, un, ut..., p) -> (mass, mom_n, mom_t..., energy)."""
    WL = np.ascontiguousarray(WL, dtype=np.float64)
    WR = np.ascontiguousarray(WR, dtype=np.float64)
    nt = WL.size - 3
    F = np.empty(nt + 3)
    lib().oracle_hll(nt, float(gamma), _dptr(WL), _dptr(WR), _dptr(F))
    return F


def weno5z(v):
    """WENO5-Z value at the right face of the middle cell of five cell values."""
    v = np.ascontiguousarray(v, dtype=np.float64)
    assert v.size == 5
    return lib().oracle_weno5z(_dptr(v))


def weno5z_indicators(v):
    """The three smoothness indicators beta_k of five cell values."""
    v = np.ascontiguousarray(v, dtype=np.float64)
    assert v.size == 5
    b = np.empty(3)
    lib().oracle_weno5z_indicators(_dptr(v), _dptr(b))
    return b


def primitives(U, gamma=1.4):
    """(rho, u_d..., p) of a conserved state array (NumPy, same formulas)."""
    nd = U.shape[0] - 2
    rho = U[0]
    q = U[1] * U[1]
    for d in range(1, nd):
        q = q + U[1 + d] * U[1 + d]
    ke = 0.5 * q / rho
    p = (gamma - 1.0) * (U[nd + 1] - ke)
    return [rho] + [U[1 + d] / rho for d in range(nd)] + [p]
