"""Seeded synthetic initial conditions for the benchmark and test cases.

This module only produces *inputs*: a case description (a plain dict) and the
primitive variables W = (rho, u, v, w, p) at the interior cells, as a float64
array of shape (5, nz, ny, nx). It holds none of the solver's arithmetic (no
conversion to conservative variables, no fluxes), so that the HIP path and the
CPU oracle can both consume exactly the same arrays.

Case keys: ``n`` (interior extents x, y, z; 1 = inactive axis), ``nh`` (halo
width), ``lo``/``hi`` (box), ``gamma``, ``mu``, ``prandtl``, ``cfl``, ``bc``
(x-, x+, y-, y+, z-, z+; 0 periodic, 1 zero gradient) and ``flags``
(1 inviscid, 2 viscous, 4 heat, 8 WENO5-Z instead of WENO5-JS).
"""
from __future__ import annotations

import math

import numpy as np

PERIODIC = 0
ZERO_GRADIENT = 1
REFLECT = 2  # slip wall: mirrored halo, normal momentum negated
INVISCID, VISCOUS, HEAT = 1, 2, 4
WENOZ = 8
ROE = 16  # flux splitting in characteristic space with Roe eigenvalues (the ROE setup)
WENO3 = 32
RUSANOV = 64
RK2 = 128
RUSANOV_NN = 256
SAFE_RECON = 512  # first-order states at faces whose reconstructed rho or p is not positive
NN_PARAMS = 2305  # Rusanov-NN weights: W1 (32x4), b1, W2 (32x32), b2, W3 (32x32), b3, W4 (1x32), b4
ALL_PHYSICS = INVISCID | VISCOUS | HEAT


def make_case(n, lo=(0.0, 0.0, 0.0), hi=(1.0, 1.0, 1.0), gamma=1.4, mu=0.0, prandtl=0.72,
              cfl=0.5, bc=(PERIODIC,) * 6, flags=INVISCID, nh=3):
    return {"n": tuple(int(x) for x in n), "nh": int(nh), "lo": tuple(map(float, lo)),
            "hi": tuple(map(float, hi)), "gamma": float(gamma), "mu": float(mu),
            "prandtl": float(prandtl), "cfl": float(cfl), "bc": tuple(int(b) for b in bc),
            "flags": int(flags)}


def cell_centres(case, axis):
    n = case["n"][axis]
    lo, hi = case["lo"][axis], case["hi"][axis]
    dx = (hi - lo) / n
    return lo + (np.arange(n) + 0.5) * dx


def _mesh(case):
    x = cell_centres(case, 0)
    y = cell_centres(case, 1)
    z = cell_centres(case, 2)
    Z, Y, X = np.meshgrid(z, y, x, indexing="ij")
    return X, Y, Z


def _stack(rho, u, v, w, p, shape):
    out = np.empty((5,) + shape)
    for k, f in enumerate((rho, u, v, w, p)):
        out[k] = f
    return out


# ----------------------------------------------------------------------------
def sod(n=200, nh=3):
    """Sod's shock tube (§5.1.2): x in [0,1], diaphragm at 0.5, (rho,u,p) =
    (1,0,1) | (0.125,0,0.1), zero-gradient ends, inviscid, CFL 0.5, t_end 0.2."""
    case = make_case((n, 1, 1), bc=(ZERO_GRADIENT,) * 6, flags=INVISCID, cfl=0.5, nh=nh)
    X, _, _ = _mesh(case)
    left = X <= 0.5
    rho = np.where(left, 1.0, 0.125)
    p = np.where(left, 1.0, 0.1)
    zero = np.zeros_like(X)
    case["t_end"] = 0.2
    return case, _stack(rho, zero, zero, zero, p, X.shape)


def lax(n=100, nh=3):
    """Lax's shock tube (§5.1.2 runs it to t = 0.14 on N = 100 cells of [0,1]
    and leaves the states to its reference): (rho, u, p) = (0.445, 0.698,
    3.528) | (0.5, 0, 0.571), diaphragm at 0.5, zero-gradient ends, inviscid,
    CFL 0.5."""
    case = make_case((n, 1, 1), bc=(ZERO_GRADIENT,) * 6, flags=INVISCID, cfl=0.5, nh=nh)
    X, _, _ = _mesh(case)
    left = X <= 0.5
    rho = np.where(left, 0.445, 0.5)
    u = np.where(left, 0.698, 0.0)
    p = np.where(left, 3.528, 0.571)
    zero = np.zeros_like(X)
    case["t_end"] = 0.14
    return case, _stack(rho, u, zero, zero, p, X.shape)


def implosion(n=128, nh=3, flags=INVISCID | WENO3 | RK2):
    """The implosion of §7.4 as printed: (rho, u, v, p) = (0.14, 0, 0, 0.125)
    where x + y <= 0.15 and (1, 0, 0, 1) elsewhere on [0,1]^2, reflecting walls
    on all four sides, inviscid; the paper's ground truth runs WENO3-JS, TVD-RK2
    and HLLC at 128^2 with a fixed dt = 2.5e-4."""
    case = make_case((n, n, 1), bc=(REFLECT,) * 4 + (PERIODIC,) * 2, flags=flags, nh=nh)
    X, Y, _ = _mesh(case)
    inner = X + Y <= 0.15
    rho = np.where(inner, 0.14, 1.0)
    p = np.where(inner, 0.125, 1.0)
    zero = np.zeros_like(X)
    case["dt"] = 2.5e-4
    return case, _stack(rho, zero, zero, zero, p, X.shape)


def nn_weights(seed=0, alpha0=1.0, scale=1.0):
    """Seeded Rusanov-NN weights (§7.4 network: 4 inputs, three hidden ReLU
    layers of 32, exp output): He-normal hidden layers with zero biases, the
    output layer scaled by `scale` (times 1/sqrt(32)) with bias ln(alpha0), so
    that scale = 0 gives alpha = alpha0 everywhere."""
    rng = np.random.default_rng(seed)
    parts = []
    for fan_in, fan_out in ((4, 32), (32, 32), (32, 32)):
        parts.append(rng.normal(0.0, np.sqrt(2.0 / fan_in), (fan_out, fan_in)).ravel())
        parts.append(np.zeros(fan_out))
    parts.append(scale * rng.normal(0.0, np.sqrt(1.0 / 32.0), 32))
    parts.append(np.array([np.log(alpha0)]))
    th = np.concatenate(parts)
    assert th.size == NN_PARAMS
    return th


def entropy_wave(n, nh=3):
    """Density wave advected at u = p = 1 on periodic [0,1] (§5.1.1, Eq. SinusDensity):
    cell averages of rho = 1.5 + sin(2 pi x)."""
    case = make_case((n, 1, 1), bc=(PERIODIC,) * 6, flags=INVISCID, nh=nh)
    dx = 1.0 / n
    xl = np.arange(n) * dx
    xr = xl + dx
    rho = 1.5 - (np.cos(2 * np.pi * xr) - np.cos(2 * np.pi * xl)) / (2 * np.pi * dx)
    rho = rho.reshape(1, 1, n)
    one = np.ones_like(rho)
    zero = np.zeros_like(rho)
    return case, _stack(rho, one, zero, zero, one, rho.shape)


def taylor_green(n, ma=0.1, re=1600.0, prandtl=0.72, gamma=1.4, cfl=0.5, nh=3, shape=None):
    """Compressible Taylor-Green vortex on the periodic cube [0, 2 pi)^3 (§6):
    rho = 1, u = sin x cos y cos z, v = -cos x sin y cos z, w = 0,
    p = 1/(gamma Ma^2) + (cos 2x + cos 2y)(cos 2z + 2)/16, mu = 1/Re."""
    ext = tuple(shape) if shape is not None else (n, n, n)
    case = make_case(ext, lo=(0.0,) * 3, hi=(2 * np.pi,) * 3, gamma=gamma, mu=1.0 / re,
                     prandtl=prandtl, cfl=cfl, bc=(PERIODIC,) * 6, flags=ALL_PHYSICS, nh=nh)
    X, Y, Z = _mesh(case)
    rho = np.ones_like(X)
    u = np.sin(X) * np.cos(Y) * np.cos(Z)
    v = -np.cos(X) * np.sin(Y) * np.cos(Z)
    w = np.zeros_like(X)
    p = 1.0 / (gamma * ma * ma) + (np.cos(2 * X) + np.cos(2 * Y)) * (np.cos(2 * Z) + 2.0) / 16.0
    return case, _stack(rho, u, v, w, p, X.shape)


def taylor_green_noisy(n, sigma=1e-3, seed=4, **kw):
    """Taylor-Green vortex with seeded Gaussian noise of standard deviation sigma
    on u, v, w (the differentiation case)."""
    case, W = taylor_green(n, **kw)
    rng = np.random.default_rng(seed)
    W[1:4] += sigma * rng.standard_normal(W[1:4].shape)
    return case, W


def isotropic_turbulence(n, seed=2203, k0=4.0, mach_t=0.3, re_lambda=100.0, gamma=1.4,
                         prandtl=0.72, cfl=0.5, nh=3):
    """Decaying compressible isotropic turbulence on the periodic cube [0, 2 pi)^3
    (§5.1.4): solenoidal random-phase velocity with energy spectrum
    E(k) ~ k^4 exp(-2 k^2 / k0^2), rms velocity u' = 1 per component, rho = 1,
    uniform p = rho c^2 / gamma with c = sqrt(3) u' / Mt, and mu = rho u' lambda_g / Re_lambda
    with the Taylor microscale lambda_g = u' / <(du/dx)^2>^(1/2) measured on the field.
    Returns (case, W); case["stats"] holds the realised u', lambda_g, Mt and Re_lambda."""
    rng = np.random.default_rng(seed)
    kfull = np.fft.fftfreq(n, d=1.0 / n)   # integer wavenumbers on the z and y axes
    khalf = np.fft.rfftfreq(n, d=1.0 / n)  # x is the last (real-FFT) axis
    KZ, KY, KX = np.meshgrid(kfull, kfull, khalf, indexing="ij")
    k2 = KX ** 2 + KY ** 2 + KZ ** 2
    kmag = np.sqrt(k2)
    k2s = np.where(k2 == 0, 1.0, k2)
    # white Gaussian noise per component -> Hermitian-consistent spectra
    uh = [np.fft.rfftn(rng.standard_normal((n, n, n))) for _ in range(3)]
    # solenoidal projection: u_hat <- u_hat - k (k . u_hat)/|k|^2
    kdotu = KX * uh[0] + KY * uh[1] + KZ * uh[2]
    uh = [uh[0] - KX * kdotu / k2s, uh[1] - KY * kdotu / k2s, uh[2] - KZ * kdotu / k2s]
    # shell amplitude so that the shell-integrated energy follows E(k)
    E = kmag ** 4 * np.exp(-2.0 * k2 / (k0 * k0))
    amp = np.where(k2 == 0, 0.0, np.sqrt(E / (4.0 * np.pi * k2s)))
    uh = [a * amp for a in uh]
    vel = [np.fft.irfftn(a, s=(n, n, n), axes=(0, 1, 2)) for a in uh]
    urms = math.sqrt(sum(float(np.mean(f * f)) for f in vel) / 3.0)
    vel = [f / urms for f in vel]
    uh = [a / urms for a in uh]
    uprime = 1.0
    # Taylor microscale from the spectral derivative du/dx
    dudx = np.fft.irfftn(1j * KX * uh[0], s=(n, n, n), axes=(0, 1, 2))
    lam = uprime / math.sqrt(float(np.mean(dudx * dudx)))
    rho0 = 1.0
    c = math.sqrt(3.0) * uprime / mach_t
    p0 = rho0 * c * c / gamma
    mu = rho0 * uprime * lam / re_lambda
    case = make_case((n, n, n), lo=(0.0,) * 3, hi=(2 * np.pi,) * 3, gamma=gamma, mu=mu,
                     prandtl=prandtl, cfl=cfl, bc=(PERIODIC,) * 6, flags=ALL_PHYSICS, nh=nh)
    shape = (n, n, n)
    W = _stack(np.full(shape, rho0), vel[0], vel[1], vel[2], np.full(shape, p0), shape)
    case["stats"] = {"u_prime": uprime, "lambda_g": lam, "mach_t": math.sqrt(3.0) * uprime / c,
                     "re_lambda": rho0 * uprime * lam / mu, "mu": mu, "p0": p0}
    return case, W


def kelvin_helmholtz(n, seed=0, amplitude=0.01, gamma=1.4, cfl=0.5, nh=3):
    """2D Kelvin-Helmholtz shear layer on periodic [0,1]^2: rho = 2 and u = +0.5 for
    |y - 1/2| < 1/4, rho = 1 and u = -0.5 elsewhere, p = 2.5,
    v = amplitude * sin(4 pi (x + phi)) with a seeded phase phi in [0, 1). Inviscid."""
    rng = np.random.default_rng(seed)
    phi = float(rng.random())
    case = make_case((n, n, 1), gamma=gamma, cfl=cfl, bc=(PERIODIC,) * 6, flags=INVISCID, nh=nh)
    X, Y, _ = _mesh(case)
    inside = np.abs(Y - 0.5) < 0.25
    rho = np.where(inside, 2.0, 1.0)
    u = np.where(inside, 0.5, -0.5)
    v = amplitude * np.sin(4 * np.pi * (X + phi))
    w = np.zeros_like(X)
    p = np.full_like(X, 2.5)
    return case, _stack(rho, u, v, w, p, X.shape)


def random_smooth(shape, seed=0, gamma=1.4, mu=0.01, flags=ALL_PHYSICS, bc=(PERIODIC,) * 6,
                  nh=3, amplitude=0.2, lo=(0.0, 0.0, 0.0), hi=(1.0, 1.0, 1.0)):
    """Random smooth positive state (a few low Fourier modes per variable), for
    parity tests on ragged, non-cubic grids."""
    rng = np.random.default_rng(seed)
    case = make_case(shape, lo=lo, hi=hi, gamma=gamma, mu=mu, bc=bc, flags=flags, nh=nh)
    X, Y, Z = _mesh(case)
    L = [case["hi"][d] - case["lo"][d] for d in range(3)]

    def field(base, amp):
        f = np.full(X.shape, base, dtype=np.float64)
        for _ in range(4):
            kk = rng.integers(0, 3, size=3)
            ph = rng.random(3) * 2 * np.pi
            f += amp * rng.uniform(-1, 1) * (np.sin(2 * np.pi * kk[0] * X / L[0] + ph[0])
                                             * np.cos(2 * np.pi * kk[1] * Y / L[1] + ph[1])
                                             * np.cos(2 * np.pi * kk[2] * Z / L[2] + ph[2]))
        return f

    rho = field(1.0, amplitude)
    u = field(0.0, 0.5)
    v = field(0.0, 0.5)
    w = field(0.0, 0.5)
    p = field(1.0, amplitude)
    return case, _stack(rho, u, v, w, p, X.shape)


def random_shocky(shape, seed=0, gamma=1.4, flags=INVISCID, bc=(ZERO_GRADIENT,) * 6, nh=3):
    """Piecewise-constant random blocks (discontinuities in every variable), for
    parity tests that exercise every HLLC branch and the WENO weights away from
    their smooth limit."""
    rng = np.random.default_rng(seed)
    case = make_case(shape, gamma=gamma, bc=bc, flags=flags, nh=nh)
    nx, ny, nz = shape
    sh = (nz, ny, nx)
    out = np.empty((5,) + sh)
    for v, (lo, hi) in enumerate(((0.2, 2.0), (-2.5, 2.5), (-2.5, 2.5), (-2.5, 2.5), (0.1, 3.0))):
        blocks = rng.uniform(lo, hi, size=(max(1, nz // 4 + 1), max(1, ny // 4 + 1), max(1, nx // 4 + 1)))
        zi = np.minimum(np.arange(nz) // 4, blocks.shape[0] - 1)
        yi = np.minimum(np.arange(ny) // 4, blocks.shape[1] - 1)
        xi = np.minimum(np.arange(nx) // 4, blocks.shape[2] - 1)
        out[v] = blocks[np.ix_(zi, yi, xi)]
    return case, out
