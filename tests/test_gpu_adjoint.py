"""Adjoint of the Heun step (dt held fixed) and the checkpointed rollout.

* One step: <Adjoint(lam), v> equals <lam, Tangent(v)> where the tangent is
  the oracle's forward-mode dual derivative of the same step (relative
  1e-10).  The GPU adjoint and the oracle tangent are independent
  implementations (reverse mode on the GPU, forward mode on the CPU).
* Rollout, config-4 recipe (2D periodic, log-normal rho, p = 1, solenoidal u;
  loss J = dx^2/2 sum (rho_N - rho_T)^2, target from rho (1 + 0.01 g')):
  <grad J, v> against the oracle's dual directional derivative (each side
  with its own CFL step list), and against central differences of the GPU
  forward map (remainders shrink with h; minmod kinks make them O(h)), and
  on samples that the oracle's branch signature shows to cross no kink,
  where the remainder is O(h^2).
"""
import numpy as np
import pytest

import oracle
import workloads

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
H = pytest.importorskip("paper_2509_08971_amd")
AG = pytest.importorskip("paper_2509_08971_amd.autograd")

P, O, R = 0, 1, 2
DEV = "cuda"


def log(*a):
    print(*a, flush=True)


def smooth_state(n, seed):
    rng = np.random.default_rng(seed)
    shape = tuple(reversed(n))
    gf = lambda: workloads.gaussian_random_field(shape, rng, spectral_index=-3.0)
    vel = [0.3 * gf() for _ in n]
    return workloads.conserved_from_primitive(np.exp(0.2 * gf()), vel, 1.0 + 0.2 * gf()), rng


# (600,) and (70, 52) hold tiles away from every edge (256-cell rows, 16 x 16
# tiles), which compute no far-end face, beside edge tiles that do
@pytest.mark.parametrize("n,bc", [((64,), (O, O)), ((48,), (R, R)), ((40, 32), (P, P, R, R)),
                                  ((32, 24), (O, O, P, P)), ((16, 12, 10), (P, P, R, R, O, O)),
                                  ((600,), (R, O)), ((70, 52), (R, O, O, R))])
def test_one_step_adjoint_dot_product(n, bc):
    log("adjoint dot product", n, bc)
    U0, rng = smooth_state(n, 3)
    og = oracle.Grid(n, bc=bc)
    dt, _ = oracle.cfl_dt(og, U0, 0.4)
    g = H.make_grid(n, bc=bc)
    U = torch.from_numpy(U0).to(DEV)
    dtd = torch.full((1,), dt, dtype=torch.float64, device=DEV)
    aw = H.workspace(H.hard_adjoint_workspace_bytes(g))
    for trial in range(3):
        lam = rng.standard_normal(U0.shape)
        v = rng.standard_normal(U0.shape) * np.abs(U0).mean(axis=tuple(range(1, U0.ndim)),
                                                           keepdims=True)
        lt = torch.from_numpy(lam.copy()).to(DEV)
        H.hard_hydro_step_adjoint(g, U, dtd, lt, aw)
        lhs = float((lt.cpu().numpy() * v).sum())
        _, dU, _ = oracle.steps_tangent(og, U0, v, [dt])
        rhs = float((lam * dU).sum())
        scale = np.abs(lt.cpu().numpy() * v).sum()
        assert abs(lhs - rhs) <= 1e-10 * scale, (trial, lhs, rhs)


@pytest.mark.parametrize("n,bc", [((40, 32), (P, P, R, R)), ((16, 12, 10), (P, P, R, R, O, O)),
                                  ((64,), (O, O))])
def test_adjoint_given_stage_state_equals_recomputed(n, bc):
    """hard_hydro_step_adjoint_given_u1 with the stage-1 state from
    hard_hydro_stage gives the same bits as hard_hydro_step_adjoint, which
    recomputes that stage itself."""
    U0, rng = smooth_state(n, 8)
    g = H.make_grid(n, bc=bc)
    U = torch.from_numpy(U0).to(DEV)
    dt = torch.zeros(1, dtype=torch.float64, device=DEV)
    work = H.workspace(H.hard_workspace_bytes(g))
    H.hard_cfl_dt(g, U, 0.4, dt, work)
    U1 = torch.empty_like(U)
    H.hard_hydro_stage(g, 1, U, None, U1, dt, work)
    aw = H.workspace(H.hard_adjoint_workspace_bytes(g))
    lam = torch.from_numpy(rng.standard_normal(U0.shape)).to(DEV)
    a, b = lam.clone(), lam.clone()
    H.hard_hydro_step_adjoint(g, U, dt, a, aw)
    H.hard_hydro_step_adjoint_given_u1(g, U, U1, dt, b, aw)
    torch.cuda.synchronize()
    assert torch.equal(a, b)


def c4_state(n, seed=4):
    return workloads.turbulent_box(n, ndim=2, seed=seed)


def c4_target_state(n, seed=4, seed2=5):
    return workloads.turbulent_box(n, ndim=2, seed=seed, rho_perturb=(0.01, seed2))


def gpu_grad(n, nsteps, every):
    """(J, grad J wrt U0) on the GPU through HydroRollout."""
    g = H.make_grid((n, n), bc=(P, P))
    U0 = torch.from_numpy(c4_state(n)).to(DEV)
    UT0 = torch.from_numpy(c4_target_state(n)).to(DEV)
    dts, _ = AG.recorded_dts(U0, g, nsteps)
    rhoT = AG.run_fixed(UT0, g, dts)[0]
    X = U0.clone().requires_grad_(True)
    UN = AG.rollout(X, g, nsteps, 0.4, every)
    dx2 = (1.0 / n) ** 2
    J = 0.5 * dx2 * ((UN[0] - rhoT) ** 2).sum()
    J.backward()
    return J.item(), X.grad.cpu().numpy(), g, dts


def oracle_dir_deriv(n, nsteps, V):
    """Oracle J and D_V J with the oracle's own recorded CFL steps."""
    og = oracle.Grid((n, n), bc=(P, P))
    U0 = c4_state(n)
    UT0 = c4_target_state(n)
    _, _, _, _, dts = oracle.run(og, U0, 0.4, 1e9, max_steps=nsteps, record_dts=True)
    rhoT = oracle.steps(og, UT0, dts)[0][0]
    out = []
    for v in V:
        UN, dUN, _ = oracle.steps_tangent(og, U0, v, dts)
        out.append((1.0 / n) ** 2 * float(((UN[0] - rhoT) * dUN[0]).sum()))
    return out


def test_rollout_gradient_vs_oracle_dual_64():
    """64x64, 200 steps, checkpoints every 20, eight random directions."""
    n, nsteps = 64, 200
    J, grad, g, _ = gpu_grad(n, nsteps, 20)
    rng = np.random.default_rng(9)
    U0 = c4_state(n)
    V = [rng.standard_normal(U0.shape) * np.abs(U0).mean(axis=(1, 2), keepdims=True)
         for _ in range(8)]
    ref = oracle_dir_deriv(n, nsteps, V)
    for k, v in enumerate(V):
        got = float((grad * v).sum())
        scale = float(np.abs(grad * v).sum())
        log(f"  dir {k}: gpu {got:.12e} oracle {ref[k]:.12e}")
        assert abs(got - ref[k]) <= 1e-10 * scale + 1e-14 * abs(ref[k]), (k, got, ref[k])


def test_rollout_gradient_vs_oracle_dual_512_full():
    """The config-4 workload at full size: 512x512, 200 steps, checkpoints
    every 20, eight random directions, each against the oracle's dual-number
    directional derivative (one evaluation carrying the eight derivative
    components) with the oracle's own CFL step list."""
    n, nsteps = 512, 200
    J, grad, g, _ = gpu_grad(n, nsteps, 20)
    rng = np.random.default_rng(12)
    U0 = c4_state(n)
    V = [rng.standard_normal(U0.shape) * np.abs(U0).mean(axis=(1, 2), keepdims=True)
         for _ in range(8)]
    og = oracle.Grid((n, n), bc=(P, P))
    _, _, _, _, dts = oracle.run(og, U0, 0.4, 1e9, max_steps=nsteps, record_dts=True)
    rhoT = oracle.steps(og, c4_target_state(n), dts)[0][0]
    UN, dUN, st = oracle.steps_tangent_multi(og, U0, V, dts)
    assert st == 0
    for k, v in enumerate(V):
        ref = (1.0 / n) ** 2 * float(((UN[0] - rhoT) * dUN[k][0]).sum())
        got = float((grad * v).sum())
        scale = float(np.abs(grad * v).sum())
        log(f"  dir {k}: gpu {got:.12e} oracle {ref:.12e}")
        assert abs(got - ref) <= 1e-10 * scale, (k, got, ref)


def test_rollout_gradient_vs_oracle_dual_512_short():
    """The 512x512 config-4 grid at full size, 20 steps (checkpoints every 5),
    one direction."""
    n, nsteps = 512, 20
    J, grad, g, _ = gpu_grad(n, nsteps, 5)
    rng = np.random.default_rng(10)
    U0 = c4_state(n)
    v = rng.standard_normal(U0.shape) * np.abs(U0).mean(axis=(1, 2), keepdims=True)
    ref = oracle_dir_deriv(n, nsteps, [v])[0]
    got = float((grad * v).sum())
    scale = float(np.abs(grad * v).sum())
    assert abs(got - ref) <= 1e-10 * scale, (got, ref)


def test_rollout_gradient_vs_finite_differences_64():
    """Central differences of J along smooth density perturbations at fixed
    velocity and pressure.  The loss is piecewise smooth: minmod switches
    between its arguments wherever two one-sided differences have equal
    magnitude, and such switches are dense in smooth fields, so a finite h
    crosses a number of kinks proportional to h and the remainder falls like
    h (not h^2).  The oracle's own central differences against its own dual
    derivative show the same remainders; the gate is that the remainder
    shrinks with h and is small at h = 1e-6."""
    n, nsteps = 64, 200
    J, grad, g, dts = gpu_grad(n, nsteps, 20)
    U0 = c4_state(n)
    rho, ux, uy, p = oracle.primitives(U0)
    rng = np.random.default_rng(11)
    UT0 = torch.from_numpy(c4_target_state(n)).to(DEV)
    rhoT = AG.run_fixed(UT0, g, dts)[0]

    def Jof(Uh):
        UN = AG.run_fixed(torch.from_numpy(Uh).to(DEV), g, dts)
        return 0.5 * (1.0 / n) ** 2 * float(((UN[0] - rhoT) ** 2).sum())

    for k in range(2):
        w = workloads.gaussian_random_field((n, n), rng, spectral_index=-3.0)
        # d/dh of U(rho (1 + h w), u, p)
        rw = rho * w
        dU = np.stack([rw, rw * ux, rw * uy, 0.5 * rw * (ux * ux + uy * uy)])
        pred = float((grad * dU).sum())
        errs = []
        for h in (1e-4, 1e-5, 1e-6):
            Up = workloads.conserved_from_primitive(rho * (1 + h * w), [ux, uy], p)
            Um = workloads.conserved_from_primitive(rho * (1 - h * w), [ux, uy], p)
            fd = (Jof(Up) - Jof(Um)) / (2.0 * h)
            errs.append(abs(fd - pred) / abs(pred))
        log(f"  direction {k}: relative FD remainders {errs}")
        assert errs[-1] < 1e-5
        assert errs[-1] < 0.2 * errs[0]


def test_rollout_gradient_fd_kink_free_samples_64():
    """Central differences of J on the GPU forward map against the GPU
    gradient, on samples that cross no branch point of the method.

    Smooth 64x64 periodic state with non-uniform pressure, 20 steps
    (checkpoints every 5), loss on rho against the run from 1.001 U0.
    Samples: 48 single entries of U0 (random field and cell, size the mean
    |U| of the field), steps h1 = 1e-4 and h2 = h1/4.  The oracle's branch
    signature (every comparison of the method, in order) of U0 +- h v is
    compared with that of U0: a sample whose signature changes crosses a
    limiter or Riemann-solver kink and is left out.  On the others the
    central-difference remainder is O(h^2): r(h2) <= r(h1)/8 + f(h2) (a
    factor 16 in exact arithmetic), where f(h) = 4 eps dx^2 sum|rho_N -
    rho_T| |rho_N| / (h |<g, v>|) bounds the rounding of the difference
    quotient (a worst case; the measured rounding is far smaller).  At least
    three samples must show the factor directly (r(h1) / r(h2) >= 8)."""
    n, nsteps, every = 64, 20, 5
    rng = np.random.default_rng(3)
    shape = (n, n)
    gf = lambda: workloads.gaussian_random_field(shape, rng, spectral_index=-3.0)
    vel = [0.3 * gf() for _ in range(2)]
    U0 = workloads.conserved_from_primitive(np.exp(0.2 * gf()), vel, 1.0 + 0.2 * gf())
    g = H.make_grid(shape, bc=(P, P))
    og = oracle.Grid(shape, bc=(P, P))
    Ud = torch.from_numpy(U0).to(DEV)
    dts, _ = AG.recorded_dts(Ud, g, nsteps)
    dth = dts.cpu().numpy()
    rhoT = AG.run_fixed(Ud * 1.001, g, dts)[0]
    X = Ud.clone().requires_grad_(True)
    UN = AG.rollout(X, g, nsteps, 0.4, every)
    dx2 = (1.0 / n) ** 2
    J = 0.5 * dx2 * ((UN[0] - rhoT) ** 2).sum()
    J.backward()
    grad = X.grad.cpu().numpy()
    UNd = UN.detach()
    bound = dx2 * float(((UNd[0] - rhoT).abs() * UNd[0].abs()).sum())

    def Jof(Uh):
        UNh = AG.run_fixed(torch.from_numpy(Uh).to(DEV), g, dts)
        return 0.5 * dx2 * float(((UNh[0] - rhoT) ** 2).sum())

    s0 = oracle.branch_signature(og, U0, dth)
    h1, h2 = 1e-4, 2.5e-5
    eps = np.finfo(np.float64).eps
    pick = np.random.default_rng(7)
    kink_free = quadratic = 0
    for k in range(48):
        f = int(pick.integers(0, 4))
        i, j = (int(a) for a in pick.integers(0, n, 2))
        v = np.zeros_like(U0)
        v[f, i, j] = np.abs(U0[f]).mean()
        if any(oracle.branch_signature(og, U0 + sg * h * v, dth) != s0
               for h in (h1, h2) for sg in (1.0, -1.0)):
            continue
        kink_free += 1
        pred = float(grad[f, i, j] * v[f, i, j])
        r = [abs((Jof(U0 + h * v) - Jof(U0 - h * v)) / (2.0 * h) - pred) / abs(pred)
             for h in (h1, h2)]
        floor = [4.0 * eps * bound / (h * abs(pred)) for h in (h1, h2)]
        log(f"  sample {k} (field {f}, cell {i},{j}): remainders {r[0]:.2e} {r[1]:.2e}, "
            f"rounding floor {floor[0]:.1e} {floor[1]:.1e}")
        assert r[1] <= r[0] / 8.0 + floor[1], (k, r, floor)
        quadratic += r[0] >= 8.0 * r[1]
    log(f"  {kink_free} kink-free samples of 48, {quadratic} with r(h1)/r(h2) >= 8")
    assert kink_free >= 6 and quadratic >= 3
