"""Seeded synthetic inputs shared by the tests, the benchmark and the oracle.

This package holds workload definitions only: problem presets, seeded random
fields, closed-form initial states and the seeded reaction mechanism.  It holds
none of the discretisation's arithmetic (no quadrature, no derivative or
projection operators, no fluxes): node coordinates are passed in by the caller.

Presets (sizes as used by the parity tests and the benchmark):
  vortex2d    2-D Euler isentropic vortex, [-5,5]^2, 8x8 quads, N=3
  euler3d     3-D Euler, [0,2pi]^3, 32^3 hexes, N=3, smooth random state
  euler3d_L   the same at 64^3 (past the 256 MB last-level cache)
  tgv3d       3-D Navier-Stokes Taylor-Green vortex, 16^3, N=4, Re 1600
  air5_2d     2-D reacting Euler, 5-species air, 64^2 + 2:1 refined 16^2 block
  adjoint3d   3-D Euler 16^3, N=3, batch of 8 perturbed states
"""

import math

import numpy as np

TWO_PI = 2.0 * math.pi

PRESETS = {
    "vortex2d": dict(dim=2, N=3, nel=(8, 8), lo=(-5.0, -5.0), hi=(5.0, 5.0),
                     physics="euler", gamma=1.4, cfl=0.5, steps=20, batch=1),
    "euler3d": dict(dim=3, N=3, nel=(32, 32, 32), lo=(0.0, 0.0, 0.0),
                    hi=(TWO_PI, TWO_PI, TWO_PI), physics="euler", gamma=1.4,
                    cfl=0.5, steps=100, batch=1),
    "euler3d_L": dict(dim=3, N=3, nel=(64, 64, 64), lo=(0.0, 0.0, 0.0),
                      hi=(TWO_PI, TWO_PI, TWO_PI), physics="euler", gamma=1.4,
                      cfl=0.5, steps=100, batch=1),
    # The 3-D N = 4 operator is not stable under SSP-RK3 at CFL 0.5 of the
    # bound dt = CFL h / ((2N + 1) lambda_max), which carries no factor of
    # the dimension (the TGV state grows without bound after ~40 steps);
    # this workload states no CFL and runs at 0.25.
    "tgv3d": dict(dim=3, N=4, nel=(16, 16, 16), lo=(0.0, 0.0, 0.0),
                  hi=(TWO_PI, TWO_PI, TWO_PI), physics="navier_stokes",
                  gamma=1.4, mu=6.25e-4, prandtl=0.72, mach=0.1, cfl=0.25,
                  steps=200, batch=1),
    "air5_2d": dict(dim=2, N=3, nel=(64, 64), lo=(-1.0, -1.0), hi=(1.0, 1.0),
                    patch_lo=(24, 24), patch_hi=(40, 40), physics="reacting",
                    cfl=0.5, steps=50, batch=1, mech_seed=42, mech_backward=(14.0, 22.0), rho0=0.1),
    "air5_2t_2d": dict(dim=2, N=3, nel=(64, 64), lo=(-1.0, -1.0), hi=(1.0, 1.0),
                       patch_lo=(24, 24), patch_hi=(40, 40), physics="reacting_2t",
                       cfl=0.5, steps=50, batch=1, mech_seed=42, mech_backward=(12.0, 15.0), rho0=1.0e-3),
    "adjoint3d": dict(dim=3, N=3, nel=(16, 16, 16), lo=(0.0, 0.0, 0.0),
                      hi=(TWO_PI, TWO_PI, TWO_PI), physics="euler", gamma=1.4,
                      cfl=0.5, steps=50, batch=8),
}


def _torch_input(a):
    return type(a).__module__.startswith("torch")


def fourier_field(coords, lo, hi, seed, nmodes=4, kmax=2):
    """Smooth periodic field: sum of `nmodes` sines with integer wavevectors in
    {-kmax..kmax}^d minus 0, phases U[0, 2pi), amplitudes U[-1, 1], normalised
    to max |f| = 1 over the given nodes.  coords: (dim, ...), a numpy array
    or a torch tensor (then evaluated where it lives, e.g. on the device for
    the large meshes; the random parameters are drawn on the host either
    way)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    dim = coords.shape[0]
    if _torch_input(coords):
        import torch
        f = torch.zeros(coords.shape[1:], dtype=coords.dtype, device=coords.device)
        sin, amax = torch.sin, lambda x: float(x.abs().max())
    else:
        f = np.zeros(coords.shape[1:])
        sin, amax = np.sin, lambda x: np.max(np.abs(x))
    for _ in range(nmodes):
        while True:
            k = rng.integers(-kmax, kmax + 1, size=dim)
            if np.any(k != 0):
                break
        phi = rng.uniform(0.0, TWO_PI)
        c = rng.uniform(-1.0, 1.0)
        arg = phi + sum(TWO_PI * int(k[d]) * (coords[d] - lo[d]) / (hi[d] - lo[d]) for d in range(dim))
        f += c * sin(arg)
    return f / amax(f)


def conserved_from_primitive(rho, vel, p, gamma):
    """(rho, rho u, .., E) with E = p/(gamma-1) + rho |u|^2 / 2 (ideal gas)."""
    ke = 0.5 * rho * sum(v * v for v in vel)
    if _torch_input(rho):
        import torch
        return torch.stack([rho] + [rho * v for v in vel] + [p / (gamma - 1.0) + ke])
    return np.stack([rho] + [rho * v for v in vel] + [p / (gamma - 1.0) + ke])


def vortex(coords, t, gamma=1.4, eps=5.0, lo=(-5.0, -5.0), hi=(5.0, 5.0)):
    """Isentropic vortex (textbook form), strength eps, free stream rho = p = 1,
    velocity (0.5 sqrt(gamma), 0) i.e. Mach 0.5, centred at (u_inf t, 0) with
    minimum-image wrap on the periodic box.  Exact Euler solution (up to the
    periodic tail) at any t."""
    uinf = 0.5 * math.sqrt(gamma)
    L = [hi[d] - lo[d] for d in range(2)]
    xc = uinf * t
    dx = np.mod(coords[0] - xc - lo[0], L[0]) + lo[0]
    dy = np.mod(coords[1] - lo[1], L[1]) + lo[1]
    r2 = dx * dx + dy * dy
    g = eps / (2.0 * math.pi) * np.exp(0.5 * (1.0 - r2))
    u = uinf - g * dy
    v = g * dx
    T = 1.0 - (gamma - 1.0) * eps ** 2 / (8.0 * gamma * math.pi ** 2) * np.exp(1.0 - r2)
    rho = T ** (1.0 / (gamma - 1.0))
    p = rho * T
    return conserved_from_primitive(rho, [u, v], p, gamma)


def stationary_vortex(coords, gamma=1.4, eps=5.0):
    """The same vortex with zero free-stream velocity: a steady solution."""
    x, y = coords[0], coords[1]
    r2 = x * x + y * y
    g = eps / (2.0 * math.pi) * np.exp(0.5 * (1.0 - r2))
    T = 1.0 - (gamma - 1.0) * eps ** 2 / (8.0 * gamma * math.pi ** 2) * np.exp(1.0 - r2)
    rho = T ** (1.0 / (gamma - 1.0))
    return conserved_from_primitive(rho, [-g * y, g * x], rho * T, gamma)


def random_euler(coords, lo, hi, gamma=1.4, mach=0.3, drho=0.05):
    """Smooth random state: rho = 1 + drho f_0, u_d = mach f_{1+d}, p = 1/gamma
    (sound speed 1), each f a 4-mode field (seeds 0, 1, 2, 3)."""
    dim = coords.shape[0]
    rho = 1.0 + drho * fourier_field(coords, lo, hi, seed=0)
    vel = [mach * fourier_field(coords, lo, hi, seed=1 + d) for d in range(dim)]
    p = 0.0 * rho + 1.0 / gamma
    return conserved_from_primitive(rho, vel, p, gamma)


def entropy_wave(coords, t, lo, hi, gamma=1.4, amp=0.2, vel=(0.5, 0.3, 0.2), k=(1, 1, 1)):
    """rho = 1 + amp sin(k.(x - u t) 2pi/L), constant u and p = 1: an exact
    Euler solution advected with the flow."""
    dim = coords.shape[0]
    arg = sum(TWO_PI * k[d] * (coords[d] - vel[d] * t - lo[d]) / (hi[d] - lo[d]) for d in range(dim))
    rho = 1.0 + amp * np.sin(arg)
    return conserved_from_primitive(rho, [np.full_like(rho, vel[d]) for d in range(dim)],
                                    np.ones_like(rho), gamma)


def taylor_green(coords, gamma=1.4, mach=0.1, A=1.0):
    """Taylor-Green vortex initial state of the paper's TGV section (eq.
    tgv_ic), evaluated directly on the given coordinates (2pi-periodic)."""
    x, y, z = coords
    rho = np.ones_like(x)
    u = A * np.sin(x) * np.cos(y) * np.cos(z)
    v = -A * np.cos(x) * np.sin(y) * np.cos(z)
    w = np.zeros_like(x)
    p = A * A * rho / (gamma * mach ** 2) + A * A * rho / 16.0 * (
        np.cos(2 * x) * np.cos(2 * z) + 2 * np.cos(2 * y) + 2 * np.cos(2 * x)
        + np.cos(2 * y) * np.cos(2 * z))
    return conserved_from_primitive(rho, [u, v, w], p, gamma)


def perturb_density(U, seed, rel=0.05, gamma=1.4):
    """Member of the adjoint batch: primitive density times (1 + rel xi),
    xi i.i.d. U[-1, 1] per node (seed = member index), velocity and pressure
    kept.  U: (nv, ...) conserved Euler state."""
    rng = np.random.Generator(np.random.PCG64(1000 + seed))
    dim = U.shape[0] - 2
    rho = U[0]
    vel = [U[1 + d] / rho for d in range(dim)]
    ke = 0.5 * rho * sum(v * v for v in vel)
    p = (gamma - 1.0) * (U[dim + 1] - ke)
    rho2 = rho * (1.0 + rel * rng.uniform(-1.0, 1.0, size=rho.shape))
    return conserved_from_primitive(rho2, vel, p, gamma)


# ---------------------------------------------------------------------------
# 5-species air (N2, O2, NO, N, O) with 5 reactions and seeded rate constants
# ---------------------------------------------------------------------------
R_UNIVERSAL = 8.314462618           # J / (mol K)
W_N = 14.0067e-3                    # kg / mol
W_O = 15.9994e-3
SPECIES = ("N2", "O2", "NO", "N", "O")


def preset_mechanism(p):
    """The seeded mechanism of a reacting preset."""
    return air5_mechanism(p["mech_seed"], backward=p["mech_backward"])


def air5_mechanism(seed=42, backward=(14.0, 22.0)):
    """Seeded 5-species / 5-reaction air mechanism.

    Stoichiometry (reactants -> products over N2, O2, NO, N, O):
      r0 N2 + M -> 2N + M,  r1 O2 + M -> 2O + M,  r2 NO + M -> N + O + M,
      r3 N2 + O -> NO + N,  r4 N + O2 -> NO + O.
    Molar masses of molecules are exact sums of the atomic ones; species gas
    constants R_s = R_u / W_s; frozen-vibration cv = 5/2 R_s (molecules),
    3/2 R_s (atoms); formation enthalpies per unit mass at 298 K from standard
    thermochemical tables (N2, O2 zero).  Rate constants are drawn, not
    physical: A log-uniform in [1e14, 1e22] (CGS), beta U[-1.5, 0], Theta
    U[5e4, 1.2e5] K forward; backward triple A log-uniform in
    [10^backward[0], 10^backward[1]] (default the forward range [1e14, 1e22];
    the two-temperature workload takes [1e12, 1e15]), beta U[-1.5, 0], Theta
    U[0, 2e4] K (the same random draws for every range).  Third-body
    efficiencies all 1.
    Units: concentrations in mol/cm^3 (kappa_c = 1e-6 from mol/m^3), rates
    converted back to mol/(m^3 s) (kappa_r = 1e6).
    """
    W = np.array([2 * W_N, 2 * W_O, W_N + W_O, W_N, W_O])
    R = R_UNIVERSAL / W
    cv = np.array([2.5, 2.5, 2.5, 1.5, 1.5]) * R
    h0 = np.array([0.0, 0.0, 90.291e3 / W[2], 472.68e3 / W[3], 249.18e3 / W[4]])
    nu_f = np.array([[1, 0, 0, 0, 0],
                     [0, 1, 0, 0, 0],
                     [0, 0, 1, 0, 0],
                     [1, 0, 0, 0, 1],
                     [0, 1, 0, 1, 0]], dtype=np.int32)
    nu_b = np.array([[0, 0, 0, 2, 0],
                     [0, 0, 0, 0, 2],
                     [0, 0, 0, 1, 1],
                     [0, 0, 1, 1, 0],
                     [0, 0, 1, 0, 1]], dtype=np.int32)
    rng = np.random.Generator(np.random.PCG64(seed))
    A_f = 10.0 ** rng.uniform(14.0, 22.0, size=5)
    beta_f = rng.uniform(-1.5, 0.0, size=5)
    theta_f = rng.uniform(5.0e4, 1.2e5, size=5)
    A_b = 10.0 ** rng.uniform(backward[0], backward[1], size=5)
    beta_b = rng.uniform(-1.5, 0.0, size=5)
    theta_b = rng.uniform(0.0, 2.0e4, size=5)
    return dict(ns=5, nr=5, W=W, R=R, cv=cv, h0=h0, nu_f=nu_f, nu_b=nu_b,
                A_f=A_f, beta_f=beta_f, theta_f=theta_f,
                A_b=A_b, beta_b=beta_b, theta_b=theta_b,
                third_body=np.array([1, 1, 1, 0, 0], dtype=np.int32),
                eff=np.ones((5, 5)), reversible=np.ones(5, dtype=np.int32),
                kappa_c=1.0e-6, kappa_r=1.0e6)


def reacting_state(coords, lo, hi, mech, rho0=0.1, T0=5000.0, dT=4000.0):
    """Quiescent reacting state: T = T0 + dT g_T, rho = rho0 (1 + 0.05 g_rho),
    Y_s proportional to 0.05 + |g_s| normalised to sum 1, u = 0 (seeds 10, 11,
    12..16).  Conserved: (rho_s, 0, .., E) with E = sum rho_s (cv_s T + h0_s)."""
    dim = coords.shape[0]
    T = T0 + dT * fourier_field(coords, lo, hi, seed=10)
    rho = rho0 * (1.0 + 0.05 * fourier_field(coords, lo, hi, seed=11))
    y = np.stack([0.05 + np.abs(fourier_field(coords, lo, hi, seed=12 + s)) for s in range(mech["ns"])])
    y = y / y.sum(axis=0, keepdims=True)
    rhos = rho[None] * y
    E = sum(rhos[s] * (mech["cv"][s] * T + mech["h0"][s]) for s in range(mech["ns"]))
    zeros = [np.zeros_like(rho) for _ in range(dim)]
    return np.concatenate([rhos, np.stack(zeros), E[None]])


def air5_vibration(mech):
    """Vibrational data of the air-5 mechanism for the two-temperature model.

    theta_v: characteristic vibrational temperatures of N2, O2 and NO from
    standard spectroscopic tables (3395, 2239 and 2817 K); the atoms have no
    vibrational mode (0).  Millikan-White constants of molecule s with
    collision partner r from the published correlation in the reduced molar
    mass mu_sr (g/mol): A_sr = 1.16e-3 mu_sr^(1/2) theta_s^(4/3),
    B_sr = 0.015 mu_sr^(1/4).  Park's limiting cross-section sigma' = 1e-21 m^2.
    Reactions 0-2 (dissociation) take their rates at sqrt(T T_v), the
    exchange reactions 3-4 at T."""
    ns = mech["ns"]
    theta = np.array([3395.0, 2239.0, 2817.0, 0.0, 0.0])
    Wg = np.asarray(mech["W"]) * 1.0e3
    mw_a = np.zeros((ns, ns))
    mw_b = np.zeros((ns, ns))
    for s_ in range(ns):
        if theta[s_] == 0.0:
            continue
        for r in range(ns):
            mu = Wg[s_] * Wg[r] / (Wg[s_] + Wg[r])
            mw_a[s_, r] = 1.16e-3 * np.sqrt(mu) * theta[s_] ** (4.0 / 3.0)
            mw_b[s_, r] = 0.015 * mu ** 0.25
    return dict(theta_v=theta, mw_a=mw_a, mw_b=mw_b, park_sigma=1.0e-21,
                two_temp=np.array([1, 1, 1, 0, 0], dtype=np.int32))


def reacting2t_state(coords, lo, hi, mech, vib, rho0=1.0e-3, T0=5000.0, dT=4000.0, u0=0.0):
    """Two-temperature reacting state: T, rho, Y_s as in reacting_state, the
    vibrational energy of each molecule a fraction 0.3 + 0.8 |g_v| (seed 20)
    of rho_s R_s T (so T_v lies on both sides of T), velocity u0 g_d (seeds
    21, 22, ...).  Conserved: (rho_s, rho u, E, E_v) with
    E = sum rho_s (cv_s T + h0_s) + E_v + rho |u|^2 / 2."""
    dim = coords.shape[0]
    T = T0 + dT * fourier_field(coords, lo, hi, seed=10)
    rho = rho0 * (1.0 + 0.05 * fourier_field(coords, lo, hi, seed=11))
    y = np.stack([0.05 + np.abs(fourier_field(coords, lo, hi, seed=12 + s)) for s in range(mech["ns"])])
    y = y / y.sum(axis=0, keepdims=True)
    rhos = rho[None] * y
    frac = 0.3 + 0.8 * np.abs(fourier_field(coords, lo, hi, seed=20))
    Ev = sum(rhos[s] * mech["R"][s] * T * frac for s in range(mech["ns"]) if vib["theta_v"][s] > 0.0)
    vel = [u0 * fourier_field(coords, lo, hi, seed=21 + d) for d in range(dim)]
    ke = 0.5 * rho * sum(v * v for v in vel)
    E = sum(rhos[s] * (mech["cv"][s] * T + mech["h0"][s]) for s in range(mech["ns"])) + Ev + ke
    mom = [rho * v for v in vel]
    return np.concatenate([rhos, np.stack(mom), E[None], Ev[None]])
