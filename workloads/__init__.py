"""Seeded synthetic initial states shared by the tests, the benchmark and smoke.

This module holds no step arithmetic: it only builds initial conserved states
(rho, m_d, E) on [0,1]^d from primitive data, using the ideal-gas relation
E = p/(gamma-1) + rho |u|^2 / 2 once, at t = 0.  All arrays are NumPy float64,
layout U[nvar][nz][ny][nx] (x fastest), nvar = ndim + 2.

Workloads (the paper publishes no data; every input here is synthetic):
  * two_state / random_two_state: 1D Riemann problems with a jump at x = 0.5
    (the paper's Sod tube, section 3.1, is the instance
    (1, 0, 1) | (0.125, 0, 0.1));
  * blast_3d: point-energy blast (a Sedov-type problem, named in the paper's
    abstract and section 1);
  * turbulent_box: log-normal density from a Gaussian random field with a
    k^-2 shell spectrum, uniform pressure, solenoidal velocity at a given rms
    Mach number;
  * acoustic_1d: a right-moving linear sound wave (section 3.5, the acoustic
    relations P_A = c_s^2 rho_A, u_A = c_s rho_A / rho_0);
  * batch_problems: thousands of uneven 1D and 2D two-state problems.
"""
import os

import numpy as np
import scipy.fft as sfft

_WORKERS = int(os.environ.get("OMP_NUM_THREADS", "0")) or -1

GAMMA = 1.4


def conserved_from_primitive(rho, vel, p, gamma=GAMMA):
    """Stack (rho, rho*u_d..., p/(gamma-1) + rho|u|^2/2) into U."""
    rho = np.asarray(rho, dtype=np.float64)
    vel = [np.asarray(v, dtype=np.float64) for v in vel]
    p = np.asarray(p, dtype=np.float64)
    U = np.empty((len(vel) + 2,) + rho.shape)
    U[0] = rho
    q = np.zeros(rho.shape)
    for d, v in enumerate(vel):
        np.multiply(rho, v, out=U[1 + d])
        q += v * v
    np.multiply(0.5 * rho, q, out=U[-1])
    U[-1] += p / (gamma - 1.0)
    return U


def cell_centres(n):
    return (np.arange(n) + 0.5) / n


def two_state(n, left, right, gamma=GAMMA, ndim=1, x0=0.5):
    """Planar jump at x = x0 (a cell is 'left' when its centre is below x0).

    left/right = (rho, u, p); u is the x velocity.  ndim = 2 gives an n x n
    grid with the same jump along x.
    """
    x = cell_centres(n)
    lm = x < x0
    rho1 = np.where(lm, left[0], right[0])
    u1 = np.where(lm, left[1], right[1])
    p1 = np.where(lm, left[2], right[2])
    if ndim == 1:
        return conserved_from_primitive(rho1, [u1], p1, gamma)
    shape = (n, n)
    b = lambda a: np.broadcast_to(a[None, :], shape)
    return conserved_from_primitive(b(rho1), [b(u1), np.zeros(shape)], b(p1), gamma)


def sod(n=1024, gamma=GAMMA):
    """Sod tube, paper section 3.1: (1, 0, 1) for x <= 0.5, (0.125, 0, 0.1) above."""
    return two_state(n, (1.0, 0.0, 1.0), (0.125, 0.0, 0.1), gamma)


def random_two_state_params(seed):
    """(rho_L, p_L, rho_R, p_R) uniform in [0.1, 1], drawn in that order."""
    rng = np.random.default_rng(seed)
    rL, pL, rR, pR = rng.uniform(0.1, 1.0, 4)
    return float(rL), float(pL), float(rR), float(pR)


def random_two_state(n=1024, seed=0, gamma=GAMMA):
    rL, pL, rR, pR = random_two_state_params(seed)
    return two_state(n, (rL, 0.0, pL), (rR, 0.0, pR), gamma)


def blast_hot_mask(n):
    """Cells whose centre lies within 2 dx of the domain centre (1/2,1/2,1/2)."""
    c = cell_centres(n) - 0.5
    dx = 1.0 / n
    r2 = c[:, None, None] ** 2 + c[None, :, None] ** 2 + c[None, None, :] ** 2
    return r2 <= (2.0 * dx) ** 2


def blast_3d(n=256, gamma=GAMMA, rho0=1.0, p0=1e-5, E0=1.0):
    """Point-energy blast: E0 spread uniformly over the hot cells."""
    hot = blast_hot_mask(n)
    count = int(hot.sum())
    dx = 1.0 / n
    shape = (n, n, n)
    U = np.empty((5,) + shape)
    U[0] = rho0
    U[1:4] = 0.0
    U[4] = p0 / (gamma - 1.0)
    U[4][hot] += E0 / (count * dx ** 3)
    return U


def gaussian_random_field(shape, rng, spectral_index=-2.0):
    """Zero-mean unit-variance periodic GRF with shell spectrum E(k) ~ k^index.

    Per-mode power P(k) ~ |k|^(index - (d - 1)) so that the shell-integrated
    spectrum has the requested slope; the k = 0 mode and the Nyquist planes
    are removed.
    """
    d = len(shape)
    white = rng.standard_normal(shape)
    wk = sfft.rfftn(white, workers=_WORKERS)
    k2 = np.zeros(wk.shape)
    for a, n in enumerate(shape):
        if a == d - 1:
            k = np.fft.rfftfreq(n, 1.0 / n)
        else:
            k = np.fft.fftfreq(n, 1.0 / n)
        sh = [1] * d
        sh[a] = k.size
        k2 = k2 + (k.reshape(sh)) ** 2
    kk = np.sqrt(k2)
    amp = np.zeros_like(kk)
    nz = kk > 0
    # drop the Nyquist planes (their derivative sign is ambiguous for real fields)
    for a, n in enumerate(shape):
        if n % 2 == 0:
            idx = [slice(None)] * d
            idx[a] = n // 2
            nz[tuple(idx)] = False
    amp[nz] = kk[nz] ** (0.5 * (spectral_index - (d - 1)))
    field = sfft.irfftn(wk * amp, s=shape, axes=tuple(range(d)), workers=_WORKERS)
    field -= field.mean()
    field /= field.std()
    return field


def solenoidal_velocity(shape, rng, spectral_index=-2.0):
    """d independent GRFs projected to zero divergence in Fourier space."""
    d = len(shape)
    comps = [sfft.rfftn(gaussian_random_field(shape, rng, spectral_index), workers=_WORKERS)
             for _ in range(d)]
    ks = []
    for a, n in enumerate(shape):
        k = np.fft.rfftfreq(n, 1.0 / n) if a == d - 1 else np.fft.fftfreq(n, 1.0 / n)
        sh = [1] * d
        sh[a] = k.size
        ks.append(k.reshape(sh))
    k2 = sum(k * k for k in ks)
    k2 = np.where(k2 == 0, 1.0, k2)
    kdotu = sum(ks[a] * comps[a] for a in range(d))
    out = []
    for a in range(d):
        ua = sfft.irfftn(comps[a] - ks[a] * kdotu / k2, s=shape, axes=tuple(range(d)),
                         workers=_WORKERS)
        ua -= ua.mean()
        out.append(ua)
    return out


def turbulent_box(n, ndim=3, seed=2, gamma=GAMMA, sigma_rho=0.3, mach=0.5, p0=1.0,
                  rho_perturb=None):
    """Log-normal density (mean 1, std sigma_rho), p = p0, solenoidal u.

    The array axes are (z, y, x) for ndim = 3 and (y, x) for ndim = 2; the
    velocity list is returned in the order (u_x, u_y[, u_z]).  rms |u| is
    mach * sqrt(gamma p0 / 1).  If rho_perturb = (eps, seed2), rho is
    multiplied by (1 + eps g') for an independent unit GRF g' (same p and u).
    """
    rng = np.random.default_rng(seed)
    shape = (n,) * ndim
    s = np.sqrt(np.log(1.0 + sigma_rho ** 2))
    g = gaussian_random_field(shape, rng)
    rho = np.exp(s * g - 0.5 * s * s)
    vel_axes = solenoidal_velocity(shape, rng)  # components along array axes
    vel = list(reversed(vel_axes))  # array axes (z, y, x) -> (u_x, u_y, u_z)
    rms = np.sqrt(np.mean(sum(v * v for v in vel)))
    target = mach * np.sqrt(gamma * p0 / 1.0)
    vel = [v * (target / rms) for v in vel]
    if rho_perturb is not None:
        eps, seed2 = rho_perturb
        g2 = gaussian_random_field(shape, np.random.default_rng(seed2))
        rho = rho * (1.0 + eps * g2)
    p = np.full(shape, p0)
    return conserved_from_primitive(rho, vel, p, gamma)


def acoustic_1d(n, amplitude=1e-6, gamma=GAMMA, t=0.0):
    """Right-moving sound wave, rho0 = 1, p0 = 1/gamma (c_s = 1), k = 2 pi.

    Cell averages of the sine are exact: <sin(k(x - t))> over [a, b] is
    (cos(k(a - t)) - cos(k(b - t))) / (k (b - a)).
    """
    rho0, p0 = 1.0, 1.0 / gamma
    cs = np.sqrt(gamma * p0 / rho0)
    k = 2.0 * np.pi
    a = np.arange(n) / n
    b = (np.arange(n) + 1) / n
    s = (np.cos(k * (a - cs * t)) - np.cos(k * (b - cs * t))) / (k * (b - a))
    rho = rho0 + amplitude * s
    u = cs * amplitude * s / rho0
    p = p0 + cs * cs * amplitude * s
    return rho, u, p


def acoustic_state(n, amplitude=1e-6, gamma=GAMMA):
    rho, u, p = acoustic_1d(n, amplitude, gamma)
    return conserved_from_primitive(rho, [u], p, gamma)


def batch_problem_specs(nprob=4096, n1d=3072, seed=0):
    """Per-problem (ndim, n, (rho_L, p_L, rho_R, p_R)).

    Problem i draws from default_rng([seed, i]): first its size (1D: nx in
    [64, 4096]; 2D: side in [32, 256]), then the four states in [0.1, 1].
    """
    specs = []
    for i in range(nprob):
        rng = np.random.default_rng([seed, i])
        if i < n1d:
            ndim, n = 1, int(rng.integers(64, 4097))
        else:
            ndim, n = 2, int(rng.integers(32, 257))
        rL, pL, rR, pR = (float(v) for v in rng.uniform(0.1, 1.0, 4))
        specs.append((ndim, n, (rL, pL, rR, pR)))
    return specs


def batch_problem_state(spec, gamma=GAMMA):
    ndim, n, (rL, pL, rR, pR) = spec
    return two_state(n, (rL, 0.0, pL), (rR, 0.0, pR), gamma, ndim=ndim)


def turbulent_box_torch(n, ndim=3, seed=2, gamma=GAMMA, sigma_rho=0.3, mach=0.5, p0=1.0,
                        device="cuda", dtype=None):
    """The turbulent_box recipe evaluated with torch on a device (for large
    benchmark inputs: 512^3 in seconds).  Same steps as turbulent_box; the
    random numbers come from torch's generator seeded with `seed`, so the
    field is a different draw of the same distribution."""
    import torch

    g_ = torch.Generator(device=device)
    g_.manual_seed(seed)
    shape = (n,) * ndim
    dims = tuple(range(ndim))

    def kgrid():
        ks = []
        for a in range(ndim):
            if a == ndim - 1:
                k = torch.fft.rfftfreq(n, 1.0 / n, device=device, dtype=torch.float64)
            else:
                k = torch.fft.fftfreq(n, 1.0 / n, device=device, dtype=torch.float64)
            sh = [1] * ndim
            sh[a] = k.numel()
            ks.append(k.reshape(sh))
        return ks

    ks = kgrid()
    k2 = sum(k * k for k in ks)
    nyq = torch.zeros_like(k2, dtype=torch.bool)
    for a in range(ndim):
        nyq = nyq | (ks[a].abs() == n // 2)
    amp = torch.where((k2 > 0) & ~nyq, k2.clamp_min(1e-300) ** (0.25 * (-2.0 - (ndim - 1))),
                      torch.zeros_like(k2))

    def grf():
        white = torch.randn(shape, generator=g_, device=device, dtype=torch.float64)
        f = torch.fft.irfftn(torch.fft.rfftn(white, dim=dims) * amp, s=shape, dim=dims)
        f = f - f.mean()
        return f / f.std(unbiased=False)

    s_ = float(np.sqrt(np.log(1.0 + sigma_rho ** 2)))
    rho = torch.exp(s_ * grf() - 0.5 * s_ * s_)
    comps = [torch.fft.rfftn(grf(), dim=dims) for _ in range(ndim)]
    k2s = torch.where(k2 == 0, torch.ones_like(k2), k2)
    kdotu = sum(ks[a] * comps[a] for a in range(ndim))
    vel_axes = []
    for a in range(ndim):
        u = torch.fft.irfftn(comps[a] - ks[a] * kdotu / k2s, s=shape, dim=dims)
        vel_axes.append(u - u.mean())
    del comps, kdotu
    vel = list(reversed(vel_axes))
    rms = torch.sqrt(sum(v * v for v in vel).mean())
    scale = mach * np.sqrt(gamma * p0) / rms
    vel = [v * scale for v in vel]
    U = torch.empty((ndim + 2,) + shape, device=device, dtype=torch.float64)
    U[0] = rho
    q = torch.zeros(shape, device=device, dtype=torch.float64)
    for d, v in enumerate(vel):
        U[1 + d] = rho * v
        q += v * v
    U[-1] = 0.5 * rho * q + p0 / (gamma - 1.0)
    return U if dtype is None else U.to(dtype)
