"""Python binding of libhard (include/hard.h): argument marshalling only.

Every function here has the name of the C entry point it calls and does
nothing but turn torch tensors, streams and grid descriptions into the plain
pointers and sizes of the C ABI.  All computation runs in the HIP kernels of
libhard.so; there is no fallback path: if the library is not built, or no
GPU is present, calls raise.

Tensors are torch tensors on the GPU (HIP under ROCm): state U of shape
(nvar, [nz, [ny,]] nx), float64 or float32, contiguous; dt buffers are
float64 device tensors; the workspace is a uint8 device tensor.
"""
import ctypes
import os

import torch  # loads the HIP runtime that libhard.so then shares

__all__ = [
    "HardError", "hard_grid_t", "make_grid", "lib",
    "hard_last_error", "hard_workspace_bytes", "hard_workspace_init", "hard_cfl_dt",
    "hard_hydro_step", "hard_hydro_step_noalloc", "hard_hydro_stage", "hard_run", "hard_status_read", "hard_conservation_sums",
    "hard_batch_plan_create", "hard_batch_plan_destroy", "hard_batch_offsets",
    "hard_batch_workspace_bytes", "hard_cfl_dt_batched", "hard_hydro_step_batched",
    "hard_run_batched", "batch_pack", "batch_unpack",
    "hard_adjoint_workspace_bytes", "hard_hydro_step_adjoint", "hard_hydro_step_adjoint_given_u1",
    "workspace",
    "hard_gmg_opts_t", "hard_gmg_levels", "hard_rad_diffuse_workspace_bytes", "hard_rad_diffuse",
    "hard_run_rhd",
    "PERIODIC", "OUTFLOW", "REFLECT", "F64", "F32", "FLD_EDDINGTON", "FLD_LEVERMORE",
]

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libhard.so")

PERIODIC, OUTFLOW, REFLECT = 0, 1, 2
F64, F32 = 0, 1
MUSCL_HLLC, WENO5Z_HLL = 0, 1  # face schemes (HARD_SCHEME_*)
OK, ERR_INVALID_ARG, ERR_UNSUPPORTED, ERR_WORKSPACE, ERR_NONPHYSICAL, ERR_HIP = range(6)
FLAG_DENSITY, FLAG_PRESSURE, FLAG_NONFINITE, FLAG_RADIATION = 1, 2, 4, 8
NOALLOC_SCRATCH_BYTES = 64 << 20  # HARD_NOALLOC_SCRATCH_BYTES
FLD_EDDINGTON, FLD_LEVERMORE = 0, 1  # flux limiters of the radiation diffusion (HARD_FLD_*)


class HardError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"libhard error {code}: {msg}")
        self.code = code


class hard_grid_t(ctypes.Structure):
    _fields_ = [
        ("ndim", ctypes.c_int32),
        ("dtype", ctypes.c_int32),
        ("n", ctypes.c_int64 * 3),
        ("dx", ctypes.c_double * 3),
        ("gamma", ctypes.c_double),
        ("bc", (ctypes.c_int32 * 2) * 3),
        ("scheme", ctypes.c_int32),
        ("rad", ctypes.c_int32),
        ("kappa", ctypes.c_double),
        ("mu", ctypes.c_double),
    ]


class hard_gmg_opts_t(ctypes.Structure):
    _fields_ = [
        ("limiter", ctypes.c_int32),
        ("ncycles", ctypes.c_int32),
        ("nu1", ctypes.c_int32),
        ("nu2", ctypes.c_int32),
        ("ncoarse", ctypes.c_int32),
    ]


_lib = None
_vp = ctypes.c_void_p
_sz = ctypes.c_size_t
_gp = ctypes.POINTER(hard_grid_t)


def lib():
    """Load libhard.so (built in-tree by __graft_entry__.build())."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is not built; run __graft_entry__.build()")
        L = ctypes.CDLL(LIB_PATH)
        st = ctypes.c_int32
        L.hard_last_error.restype = ctypes.c_char_p
        L.hard_last_error.argtypes = []
        sig = {
            "hard_workspace_bytes": [_gp, ctypes.POINTER(_sz)],
            "hard_workspace_init": [_vp, _sz, _vp],
            "hard_cfl_dt": [_gp, _vp, ctypes.c_double, _vp, ctypes.POINTER(ctypes.c_double), _vp,
                            _sz, _vp],
            "hard_hydro_step": [_gp, _vp, _vp, ctypes.c_double, _vp, _vp, _sz, _vp],
            "hard_hydro_step_noalloc": [_gp, _vp, _vp, ctypes.c_double, _vp, _vp, _vp],
            "hard_hydro_stage": [_gp, ctypes.c_int32, _vp, _vp, _vp, _vp, ctypes.c_double, _vp,
                                 _vp, _sz, _vp],
            "hard_run": [_gp, _vp, ctypes.c_double, ctypes.c_double, ctypes.c_int64,
                         ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int64), _vp, _sz,
                         _vp],
            "hard_status_read": [_vp, _sz, ctypes.POINTER(ctypes.c_uint32), _vp],
            "hard_conservation_sums": [_gp, _vp, _vp, _vp, _sz, _vp],
            "hard_batch_plan_create": [_gp, ctypes.c_int32, ctypes.c_char_p, ctypes.POINTER(_vp)],
            "hard_batch_plan_destroy": [_vp],
            "hard_batch_offsets": [_vp, ctypes.POINTER(ctypes.c_int64)],
            "hard_batch_workspace_bytes": [_vp, ctypes.POINTER(_sz)],
            "hard_cfl_dt_batched": [_vp, _vp, ctypes.c_double, _vp, _vp, _sz, _vp],
            "hard_hydro_step_batched": [_vp, _vp, _vp, ctypes.c_double, ctypes.c_int32, _vp, _sz,
                                        _vp],
            "hard_run_batched": [_vp, _vp, ctypes.c_double, ctypes.c_double, ctypes.c_int64, _vp,
                                 ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int64),
                                 _vp, _sz, _vp],
            "hard_adjoint_workspace_bytes": [_gp, ctypes.POINTER(_sz)],
            "hard_hydro_step_adjoint": [_gp, _vp, _vp, _vp, _vp, _sz, _vp],
            "hard_hydro_step_adjoint_given_u1": [_gp, _vp, _vp, _vp, _vp, _vp, _sz, _vp],
            "hard_gmg_levels": [_gp, ctypes.c_int32, ctypes.POINTER(ctypes.c_int64),
                                ctypes.POINTER(ctypes.c_int32)],
            "hard_rad_diffuse_workspace_bytes": [_gp, ctypes.POINTER(_sz)],
            "hard_rad_diffuse": [_gp, _vp, _vp, ctypes.POINTER(hard_gmg_opts_t), _vp, _vp, _sz,
                                 _vp],
            "hard_run_rhd": [_gp, _vp, ctypes.c_double, ctypes.c_double, ctypes.c_int64,
                             ctypes.POINTER(hard_gmg_opts_t), ctypes.POINTER(ctypes.c_double),
                             ctypes.POINTER(ctypes.c_int64), _vp, _sz, _vp, _sz, _vp],
        }
        for name, args in sig.items():
            f = getattr(L, name)
            f.argtypes = args
            f.restype = st
        _lib = L
    return _lib


def hard_last_error():
    return lib().hard_last_error().decode()


def _check(code):
    if code != OK:
        raise HardError(code, hard_last_error())


def make_grid(n, dx=None, gamma=1.4, bc=(OUTFLOW, OUTFLOW), dtype=torch.float64,
              scheme=0, rad=None):
    """hard_grid_t for n = (nx[, ny[, nz]]); bc is (lo, hi) per axis, flattened
    (a single pair applies to every axis); dx defaults to 1/n (unit box);
    scheme is MUSCL_HLLC (default) or WENO5Z_HLL; rad = (kappa, mu) adds the
    radiation energy density as the last field."""
    n = tuple(int(v) for v in n)
    nd = len(n)
    if dx is None:
        dx = tuple(1.0 / v for v in n)
    bc = tuple(int(v) for v in bc)
    if len(bc) == 2:
        bc = bc * nd
    g = hard_grid_t()
    g.ndim = nd
    g.dtype = F64 if dtype in (torch.float64, "f64", F64) else F32
    for d in range(3):
        g.n[d] = n[d] if d < nd else 1
        g.dx[d] = float(dx[d]) if d < nd else 1.0
        g.bc[d][0] = bc[2 * d] if d < nd else 0
        g.bc[d][1] = bc[2 * d + 1] if d < nd else 0
    g.gamma = float(gamma)
    g.scheme = int(scheme)
    if rad is not None:
        g.rad = 1
        g.kappa, g.mu = float(rad[0]), float(rad[1])
    else:
        g.rad, g.kappa, g.mu = 0, 0.0, 1.0
    return g


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _stream(stream):
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def _grid(g):
    return ctypes.byref(g)


def hard_workspace_bytes(g):
    b = _sz(0)
    _check(lib().hard_workspace_bytes(_grid(g), ctypes.byref(b)))
    return b.value


def workspace(nbytes, device="cuda"):
    """Zeroed uint8 device buffer (torch's allocator aligns to >= 256 bytes)."""
    w = torch.zeros(int(nbytes), dtype=torch.uint8, device=device)
    assert w.data_ptr() % 256 == 0
    return w


def hard_workspace_init(work, stream=None):
    _check(lib().hard_workspace_init(_ptr(work), work.numel(), _stream(stream)))


def hard_cfl_dt(g, U, cfl, dt_dev, work, want_host=False, stream=None):
    """Writes dt into dt_dev (float64 device tensor, 1 element); returns the
    host value if want_host (synchronises)."""
    host = ctypes.c_double(0.0)
    _check(lib().hard_cfl_dt(_grid(g), _ptr(U), float(cfl), _ptr(dt_dev),
                             ctypes.byref(host) if want_host else None, _ptr(work), work.numel(),
                             _stream(stream)))
    return host.value if want_host else None


def hard_hydro_step(g, U, dt_dev, work, cfl=0.4, next_dt_dev=None, stream=None):
    _check(lib().hard_hydro_step(_grid(g), _ptr(U), _ptr(dt_dev), float(cfl), _ptr(next_dt_dev),
                                 _ptr(work), work.numel(), _stream(stream)))


def hard_hydro_step_noalloc(g, U, dt_dev, cfl=0.4, next_dt_dev=None, flags_dev=None,
                            stream=None):
    """hard_hydro_step without a workspace argument (the library's static
    device scratch; grids up to NOALLOC_SCRATCH_BYTES of workspace)."""
    _check(lib().hard_hydro_step_noalloc(_grid(g), _ptr(U), _ptr(dt_dev), float(cfl),
                                         _ptr(next_dt_dev), _ptr(flags_dev), _stream(stream)))


def hard_hydro_stage(g, stage, src, un, dst, dt_dev, work, cfl=0.4, next_dt_dev=None,
                     stream=None):
    _check(lib().hard_hydro_stage(_grid(g), int(stage), _ptr(src), _ptr(un), _ptr(dst),
                                  _ptr(dt_dev), float(cfl), _ptr(next_dt_dev), _ptr(work),
                                  work.numel(), _stream(stream)))


def hard_run(g, U, cfl, t_end, work, max_steps=10_000_000, stream=None):
    """Run to t_end in place; returns (t, steps)."""
    t = ctypes.c_double(0.0)
    s = ctypes.c_int64(0)
    _check(lib().hard_run(_grid(g), _ptr(U), float(cfl), float(t_end), int(max_steps),
                          ctypes.byref(t), ctypes.byref(s), _ptr(work), work.numel(),
                          _stream(stream)))
    return t.value, s.value


def hard_status_read(work, stream=None, raise_on_flags=False):
    f = ctypes.c_uint32(0)
    code = lib().hard_status_read(_ptr(work), work.numel(), ctypes.byref(f), _stream(stream))
    if code != OK and (code != ERR_NONPHYSICAL or raise_on_flags):
        _check(code)
    return f.value


def hard_conservation_sums(g, U, sums_dev, work, stream=None):
    _check(lib().hard_conservation_sums(_grid(g), _ptr(U), _ptr(sums_dev), _ptr(work),
                                        work.numel(), _stream(stream)))


# ---- batched -------------------------------------------------------------
def hard_batch_plan_create(grids, tune_cache=None):
    arr = (hard_grid_t * len(grids))(*grids)
    plan = ctypes.c_void_p(None)
    _check(lib().hard_batch_plan_create(arr, len(grids),
                                        tune_cache.encode() if tune_cache else None,
                                        ctypes.byref(plan)))
    return plan


def hard_batch_plan_destroy(plan):
    _check(lib().hard_batch_plan_destroy(plan))


def hard_batch_offsets(plan, nprob):
    off = (ctypes.c_int64 * (nprob + 1))()
    _check(lib().hard_batch_offsets(plan, off))
    return list(off)


def hard_batch_workspace_bytes(plan):
    b = _sz(0)
    _check(lib().hard_batch_workspace_bytes(plan, ctypes.byref(b)))
    return b.value


def hard_cfl_dt_batched(plan, U, cfl, dt_dev, work, stream=None):
    _check(lib().hard_cfl_dt_batched(plan, _ptr(U), float(cfl), _ptr(dt_dev), _ptr(work),
                                     work.numel(), _stream(stream)))


def hard_hydro_step_batched(plan, U, dt_dev, work, cfl=0.4, update_dt=True, stream=None):
    _check(lib().hard_hydro_step_batched(plan, _ptr(U), _ptr(dt_dev), float(cfl),
                                         1 if update_dt else 0, _ptr(work), work.numel(),
                                         _stream(stream)))


def hard_run_batched(plan, nprob, U, cfl, t_end, dt_dev, work, max_steps=10_000_000,
                     stream=None):
    """Run every problem to t_end; returns (t list, steps list)."""
    t = (ctypes.c_double * nprob)()
    s = (ctypes.c_int64 * nprob)()
    _check(lib().hard_run_batched(plan, _ptr(U), float(cfl), float(t_end), int(max_steps),
                                  _ptr(dt_dev), t, s, _ptr(work), work.numel(), _stream(stream)))
    return list(t), list(s)


def batch_pack(states, offsets, dtype=torch.float64, device="cuda"):
    """Copy per-problem state arrays into one packed device buffer at the
    plan's element offsets."""
    total = int(offsets[-1])
    U = torch.zeros(total, dtype=dtype, device=device)
    for p, a in enumerate(states):
        t = torch.as_tensor(a).reshape(-1)
        U[offsets[p]:offsets[p] + t.numel()] = t.to(device=device, dtype=dtype)
    return U


def batch_unpack(U, offsets, shapes):
    """Views of the packed buffer as per-problem state arrays."""
    out = []
    for p, shp in enumerate(shapes):
        n = 1
        for v in shp:
            n *= int(v)
        out.append(U[offsets[p]:offsets[p] + n].view(*shp))
    return out


# ---- adjoint ---------------------------------------------------------------
def hard_adjoint_workspace_bytes(g):
    b = _sz(0)
    _check(lib().hard_adjoint_workspace_bytes(_grid(g), ctypes.byref(b)))
    return b.value


def hard_hydro_step_adjoint(g, U_n, dt_dev, lam, work, stream=None):
    _check(lib().hard_hydro_step_adjoint(_grid(g), _ptr(U_n), _ptr(dt_dev), _ptr(lam), _ptr(work),
                                         work.numel(), _stream(stream)))


def hard_hydro_step_adjoint_given_u1(g, U_n, U_1, dt_dev, lam, work, stream=None):
    _check(lib().hard_hydro_step_adjoint_given_u1(_grid(g), _ptr(U_n), _ptr(U_1), _ptr(dt_dev),
                                                  _ptr(lam), _ptr(work), work.numel(),
                                                  _stream(stream)))


def hard_gmg_levels(g):
    """Multigrid level sizes [(nx, ny, nz), ...], finest first (host only)."""
    out = (ctypes.c_int64 * (3 * 64))()
    nl = ctypes.c_int32(0)
    _check(lib().hard_gmg_levels(_grid(g), 64, out, ctypes.byref(nl)))
    return [tuple(out[3 * l + d] for d in range(3)) for l in range(min(nl.value, 64))]


def hard_rad_diffuse_workspace_bytes(g):
    b = _sz(0)
    _check(lib().hard_rad_diffuse_workspace_bytes(_grid(g), ctypes.byref(b)))
    return b.value


def hard_rad_diffuse(g, U, dt_dev, work, limiter=FLD_LEVERMORE, ncycles=4, nu1=2, nu2=2,
                     ncoarse=8, resid_dev=None, stream=None):
    """One implicit diffusion step of E_r in U (in place) by ncycles V(nu1, nu2)
    cycles; resid_dev (float64 device tensor of ncycles + 1, or None) receives
    the finest-level residual norms."""
    o = hard_gmg_opts_t(int(limiter), int(ncycles), int(nu1), int(nu2), int(ncoarse))
    _check(lib().hard_rad_diffuse(_grid(g), _ptr(U), _ptr(dt_dev), ctypes.byref(o),
                                  _ptr(resid_dev), _ptr(work), work.numel(), _stream(stream)))


def hard_run_rhd(g, U, cfl, t_end, work, fld_work, limiter=FLD_LEVERMORE, ncycles=4, nu1=2, nu2=2,
                 ncoarse=8, max_steps=10_000_000, stream=None):
    """Run to t_end in place with the diffusion in every step; returns (t, steps)."""
    o = hard_gmg_opts_t(int(limiter), int(ncycles), int(nu1), int(nu2), int(ncoarse))
    t = ctypes.c_double(0.0)
    n = ctypes.c_int64(0)
    _check(lib().hard_run_rhd(_grid(g), _ptr(U), float(cfl), float(t_end), int(max_steps),
                              ctypes.byref(o), ctypes.byref(t), ctypes.byref(n), _ptr(work),
                              work.numel(), _ptr(fld_work), fld_work.numel(), _stream(stream)))
    return t.value, n.value
