"""C ABI of libhard, checked on the host (no GPU needed): every function
declared in include/hard.h is exported, and invalid arguments are rejected
before anything is enqueued."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

H = pytest.importorskip("paper_2509_08971_amd")


def declared_functions():
    src = open(os.path.join(ROOT, "include", "hard.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(hard_[a-z0-9_]+)\s*\(", src)))


def test_every_declared_function_is_exported():
    names = declared_functions()
    assert "hard_hydro_step" in names and "hard_hydro_step_adjoint" in names
    L = H.lib()
    for n in names:
        assert hasattr(L, n), n


def test_library_is_gfx950_hip_code():
    out = open(H.LIB_PATH, "rb").read()
    assert b"gfx950" in out


def grid(**kw):
    g = H.make_grid((32, 16, 8), bc=(H.PERIODIC, H.PERIODIC))
    for k, v in kw.items():
        setattr(g, k, v)
    return g


FAKE = 1 << 40  # never dereferenced: every call below fails validation first


def call_step(g, U=FAKE, dt=FAKE, cfl=0.4, nxt=None, work=FAKE, nbytes=None):
    L = H.lib()
    if nbytes is None:
        nbytes = 1 << 40
    return L.hard_hydro_step(ctypes.byref(g) if g is not None else None, U, dt, cfl, nxt, work,
                             nbytes, None)


@pytest.mark.parametrize("mut", [
    dict(ndim=0), dict(ndim=4), dict(dtype=7), dict(gamma=1.0), dict(gamma=float("nan")),
])
def test_invalid_grid_scalar(mut):
    g = grid(**mut)
    assert call_step(g, work=None) == H.ERR_INVALID_ARG
    assert H.hard_last_error()


def test_invalid_grid_fields():
    g = grid()
    g.n[0] = 1
    assert call_step(g) == H.ERR_INVALID_ARG
    g = H.make_grid((32, 16))
    g.n[2] = 4
    assert call_step(g) == H.ERR_INVALID_ARG
    g = grid()
    g.dx[1] = 0.0
    assert call_step(g) == H.ERR_INVALID_ARG
    g = grid()
    g.dx[2] = float("inf")
    assert call_step(g) == H.ERR_INVALID_ARG
    g = grid()
    g.bc[1][0] = 5
    assert call_step(g) == H.ERR_INVALID_ARG
    g = grid()
    g.bc[0][0] = H.OUTFLOW  # periodic on one side only
    assert call_step(g) == H.ERR_INVALID_ARG
    assert call_step(None) == H.ERR_INVALID_ARG


def test_invalid_pointers_and_sizes():
    g = grid()
    assert call_step(g, U=None) == H.ERR_INVALID_ARG
    assert call_step(g, U=FAKE + 4) == H.ERR_INVALID_ARG  # misaligned double
    assert call_step(g, dt=None) == H.ERR_INVALID_ARG
    assert call_step(g, nxt=FAKE, cfl=0.0) == H.ERR_INVALID_ARG
    assert call_step(g, nxt=FAKE, cfl=1.5) == H.ERR_INVALID_ARG
    assert call_step(g, work=None) == H.ERR_INVALID_ARG
    assert call_step(g, work=FAKE + 8) == H.ERR_INVALID_ARG
    need = H.hard_workspace_bytes(g)
    assert call_step(g, nbytes=need - 1) == H.ERR_WORKSPACE


def test_workspace_size_formula():
    g = H.make_grid((256, 256, 256), bc=(H.REFLECT, H.REFLECT))
    b = H.hard_workspace_bytes(g)
    state = 5 * 256 ** 3 * 8
    assert state <= b <= state + 256 * 1024
    g32 = H.make_grid((64, 64), dtype="f32")
    assert H.hard_workspace_bytes(g32) >= 4 * 64 * 64 * 4


def test_cfl_and_run_argument_checks():
    L = H.lib()
    g = grid()
    host = ctypes.c_double()
    assert L.hard_cfl_dt(ctypes.byref(g), FAKE, 0.0, FAKE, ctypes.byref(host), FAKE, 1 << 40,
                         None) == H.ERR_INVALID_ARG
    t = ctypes.c_double()
    s = ctypes.c_int64()
    assert L.hard_run(ctypes.byref(g), FAKE, 0.4, -1.0, 10, ctypes.byref(t), ctypes.byref(s), FAKE,
                      1 << 40, None) == H.ERR_INVALID_ARG
    assert L.hard_run(ctypes.byref(g), FAKE, 0.4, 1.0, 0, ctypes.byref(t), ctypes.byref(s), FAKE,
                      1 << 40, None) == H.ERR_INVALID_ARG


def test_adjoint_is_fp64_only():
    g = H.make_grid((16, 16), dtype="f32")
    L = H.lib()
    b = ctypes.c_size_t()
    assert L.hard_adjoint_workspace_bytes(ctypes.byref(g), ctypes.byref(b)) == H.ERR_UNSUPPORTED
    g = H.make_grid((16, 16))
    assert L.hard_adjoint_workspace_bytes(ctypes.byref(g), ctypes.byref(b)) == H.OK
    assert b.value >= 3 * 4 * 16 * 16 * 8


def test_batched_plan_rejects_mixed_dtypes():
    grids = [H.make_grid((64,)), H.make_grid((32, 32), dtype="f32")]
    arr = (H.hard_grid_t * 2)(*grids)
    plan = ctypes.c_void_p()
    assert H.lib().hard_batch_plan_create(arr, 2, None, ctypes.byref(plan)) == H.ERR_INVALID_ARG
    assert not plan.value


def test_scheme_checks():
    """The face scheme is validated; WENO5-Z needs three cells per axis, its
    pipeline arrays are part of the workspace, and the batched and adjoint
    calls reject it."""
    L = H.lib()
    assert call_step(grid(scheme=2), work=None) == H.ERR_INVALID_ARG
    g = H.make_grid((2, 16), scheme=H.WENO5Z_HLL)
    assert call_step(g, work=None) == H.ERR_INVALID_ARG
    n = 64
    gm = H.make_grid((n, n, n))
    gw = H.make_grid((n, n, n), scheme=H.WENO5Z_HLL)
    extra = H.hard_workspace_bytes(gw) - H.hard_workspace_bytes(gm)
    # W and the x and y face arrays (the z faces of a 3D grid stay in registers)
    assert extra >= 5 * 8 * (n ** 3 + 2 * n * n * (n + 1))
    b = ctypes.c_size_t()
    assert L.hard_adjoint_workspace_bytes(ctypes.byref(gw), ctypes.byref(b)) == H.ERR_UNSUPPORTED
    arr = (H.hard_grid_t * 1)(H.make_grid((64,), scheme=H.WENO5Z_HLL))
    plan = ctypes.c_void_p()
    assert L.hard_batch_plan_create(arr, 1, None, ctypes.byref(plan)) == H.ERR_UNSUPPORTED
    assert not plan.value


def test_radiation_checks():
    """Radiation parameters are validated; the field is counted in the
    workspace; stages, batched and adjoint calls reject it."""
    L = H.lib()
    assert call_step(grid(rad=2), work=None) == H.ERR_INVALID_ARG
    g = H.make_grid((16, 16), rad=(-1.0, 0.6))
    assert call_step(g, work=None) == H.ERR_INVALID_ARG
    g = H.make_grid((16, 16), rad=(0.4, 0.0))
    assert call_step(g, work=None) == H.ERR_INVALID_ARG
    g = H.make_grid((16, 16), rad=(0.4, 0.6), scheme=H.WENO5Z_HLL)
    assert call_step(g, work=None) == H.ERR_UNSUPPORTED
    n = 64
    g0 = H.make_grid((n, n, n))
    g1 = H.make_grid((n, n, n), rad=(0.4, 0.6))
    assert H.hard_workspace_bytes(g1) - H.hard_workspace_bytes(g0) >= n ** 3 * 8
    assert L.hard_hydro_stage(ctypes.byref(g1), 1, FAKE, None, FAKE + 256, FAKE, 0.4, None, FAKE,
                              1 << 40, None) == H.ERR_UNSUPPORTED
    b = ctypes.c_size_t()
    assert L.hard_adjoint_workspace_bytes(ctypes.byref(g1), ctypes.byref(b)) == H.ERR_UNSUPPORTED
    arr = (H.hard_grid_t * 1)(H.make_grid((64,), rad=(0.4, 0.6)))
    plan = ctypes.c_void_p()
    assert L.hard_batch_plan_create(arr, 1, None, ctypes.byref(plan)) == H.ERR_UNSUPPORTED


def call_diffuse(g, U=FAKE, dt=FAKE, opts=None, resid=None, work=FAKE, nbytes=1 << 40):
    L = H.lib()
    if opts is None:
        opts = H.hard_gmg_opts_t(H.FLD_LEVERMORE, 4, 2, 2, 8)
    return L.hard_rad_diffuse(ctypes.byref(g), U, dt, ctypes.byref(opts) if opts != 0 else None,
                              resid, work, nbytes, None)


def test_diffusion_checks():
    """The implicit diffusion call needs the radiation field, kappa > 0 and
    even periodic axes; its options and workspace are validated."""
    rad = (0.4, 0.6)
    assert call_diffuse(H.make_grid((16, 16))) == H.ERR_INVALID_ARG
    assert call_diffuse(H.make_grid((16, 16), rad=(0.0, 0.6))) == H.ERR_INVALID_ARG
    gf = H.make_grid((16, 16), rad=rad, dtype="f32")
    assert call_diffuse(gf, U=FAKE + 4, nbytes=H.hard_rad_diffuse_workspace_bytes(gf) - 1) == \
        H.ERR_WORKSPACE  # float states are accepted (4-byte aligned U)
    assert call_diffuse(H.make_grid((15, 16), bc=(0, 0, 1, 1), rad=rad)) == H.ERR_UNSUPPORTED
    g = H.make_grid((15, 16), bc=(1, 2, 1, 1), rad=rad)  # odd walls are fine
    assert H.hard_rad_diffuse_workspace_bytes(g) > 0
    g = H.make_grid((16, 16), rad=rad)
    assert call_diffuse(g, U=None) == H.ERR_INVALID_ARG
    assert call_diffuse(g, dt=None) == H.ERR_INVALID_ARG
    assert call_diffuse(g, opts=0) == H.ERR_INVALID_ARG
    for o in [(2, 4, 2, 2, 8), (1, -1, 2, 2, 8), (1, 1001, 2, 2, 8), (1, 4, -1, 2, 8),
              (1, 4, 2, 65, 8), (1, 4, 2, 2, 0), (1, 4, 2, 2, 1025)]:
        assert call_diffuse(g, opts=H.hard_gmg_opts_t(*o)) == H.ERR_INVALID_ARG, o
    need = H.hard_rad_diffuse_workspace_bytes(g)
    assert call_diffuse(g, nbytes=need - 1) == H.ERR_WORKSPACE
    assert call_diffuse(g, work=FAKE + 8) == H.ERR_INVALID_ARG  # not 256-byte aligned
    # level arrays: b and D on the finest level, x, b and D on the coarser ones
    g3 = H.make_grid((64, 64, 64), bc=(0, 0), rad=rad)
    b3 = H.hard_rad_diffuse_workspace_bytes(g3)
    assert 2 * 64 ** 3 * 8 + 3 * 32 ** 3 * 8 < b3 < 3.5 * 64 ** 3 * 8


@pytest.mark.parametrize("n, bc", [
    ((32, 32), (0, 0, 1, 1)), ((48, 40, 24), (0, 0, 1, 1, 2, 2)), ((6,), (0, 0)), ((6,), (1, 1)),
    ((12, 4), (1, 1, 1, 1)), ((256, 256, 256), (2, 2)), ((100, 36), (0, 0, 0, 0)),
    ((2, 2, 2), (0, 0)),
])
def test_multigrid_levels_match_the_oracle(n, bc):
    import oracle
    from oracle import fld
    want = fld.gmg_levels(oracle.Grid(n, bc=bc, rad=(0.4, 0.6)))
    got = H.hard_gmg_levels(H.make_grid(n, bc=bc, rad=(0.4, 0.6)))
    assert got == want


def test_run_rhd_checks():
    """hard_run_rhd validates the grid (radiation field needed), both
    workspaces and the multigrid options before anything is enqueued."""
    L = H.lib()
    t = ctypes.c_double()
    n = ctypes.c_int64()
    opts = H.hard_gmg_opts_t(H.FLD_LEVERMORE, 2, 2, 2, 8)

    def call(g, o=opts, work_bytes=1 << 40, fld_bytes=1 << 40, fld=FAKE):
        return L.hard_run_rhd(ctypes.byref(g), FAKE, 0.4, 1.0, 10, ctypes.byref(o) if o else None,
                              ctypes.byref(t), ctypes.byref(n), FAKE, work_bytes, fld, fld_bytes,
                              None)

    assert call(H.make_grid((16, 16))) == H.ERR_INVALID_ARG  # no radiation field
    g = H.make_grid((16, 16), rad=(0.4, 0.6))
    assert call(g, o=None) == H.ERR_INVALID_ARG
    assert call(g, fld_bytes=H.hard_rad_diffuse_workspace_bytes(g) - 1) == H.ERR_WORKSPACE
    assert call(g, work_bytes=H.hard_workspace_bytes(g) - 1) == H.ERR_WORKSPACE
    assert call(g, fld=None) == H.ERR_INVALID_ARG
    assert call(H.make_grid((15, 16), bc=(0, 0, 1, 1), rad=(0.4, 0.6))) == H.ERR_UNSUPPORTED


def test_cell_count_limit():
    """Grids of 2^31 cells or more are refused before any work: the kernels
    index cells and level arrays with 32-bit arithmetic below that bound."""
    for call in (H.hard_workspace_bytes, H.hard_rad_diffuse_workspace_bytes):
        with pytest.raises(H.HardError) as e:
            call(H.make_grid((2048, 1024, 1024), rad=(0.4, 0.6)))
        assert e.value.code == H.ERR_INVALID_ARG
    assert H.hard_workspace_bytes(H.make_grid((2048, 1024, 1023))) > 0


def test_noalloc_refuses_grids_beyond_its_scratch():
    """hard_hydro_step_noalloc checks the grid and the size of the workspace
    it would need against its static scratch before touching the device."""
    L = H.lib()
    g = H.make_grid((256, 256, 256), bc=(H.PERIODIC, H.PERIODIC))
    assert L.hard_hydro_step_noalloc(ctypes.byref(g), FAKE, FAKE, 0.4, None, None, None) \
        == H.ERR_WORKSPACE
    assert "scratch" in H.hard_last_error()
    assert H.hard_workspace_bytes(g) > H.NOALLOC_SCRATCH_BYTES
    assert L.hard_hydro_step_noalloc(ctypes.byref(grid(ndim=0)), FAKE, FAKE, 0.4, None, None,
                                     None) == H.ERR_INVALID_ARG
    assert L.hard_hydro_step_noalloc(ctypes.byref(H.make_grid((16, 16))), FAKE, FAKE, 0.4, None,
                                     FAKE + 2, None) == H.ERR_INVALID_ARG  # misaligned flags_dev
