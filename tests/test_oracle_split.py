"""Pins of the oracle's split-form volume integral (eq. vol_split) and of the
Ranocha two-point flux against what the mathematics fixes: the logarithmic
mean against its series in extended precision, symmetry and consistency of
the two-point flux with the physical flux, Tadmor's entropy-conservation
condition (which the energy row as printed in the paper fails), free stream,
discrete conservation, discrete entropy conservation with the entropy-
conservative interface flux, entropy dissipation with the Rusanov flux, and
convergence on the isentropic vortex."""

import numpy as np
import pytest
import torch

import dginputs as di
from oracle.dgsem import Operator
from oracle.mesh import cartesian_mesh
from oracle.physics import Euler
from oracle.split import SplitOperator, log_mean, ranocha_flux
from oracle.timestep import integrals, tensor_weights, ssprk33_step, dt_cfl

G = 1.4


def random_states(n, seed):
    rng = np.random.default_rng(seed)
    rho = rng.uniform(0.5, 2.0, n)
    vel = [rng.uniform(-1.0, 1.0, n) for _ in range(3)]
    p = rng.uniform(0.5, 2.0, n)
    return torch.tensor(di.conserved_from_primitive(rho, vel, p, G))[None]   # (1, 5, n)


def entropy_vars(U):
    """w = d eta / dU for eta = -rho s / (gamma - 1), s = ln(p rho^-gamma)."""
    rho, m, E = U[:, 0], U[:, 1:-1], U[:, -1]
    u = m / rho[:, None]
    p = (G - 1) * (E - 0.5 * (m * u).sum(1))
    s = torch.log(p) - G * torch.log(rho)
    w0 = (G - s) / (G - 1) - 0.5 * rho * (u * u).sum(1) / p
    return torch.cat([w0[:, None], rho[:, None] * u / p[:, None], -(rho / p)[:, None]], 1)


# --- logarithmic mean ---------------------------------------------------------

def test_log_mean_against_extended_precision_series():
    rng = np.random.default_rng(3)
    a = rng.uniform(0.1, 10.0, 2000)
    for rel in (1e-14, 1e-10, 1e-6, 1e-3, 3e-2):
        b = a * (1.0 + rel * rng.uniform(-1, 1, a.size))
        la, lb = a.astype(np.longdouble), b.astype(np.longdouble)
        u = ((la - lb) / (la + lb)) ** 2
        series = (la + lb) / (2 * (1 + u / 3 + u ** 2 / 5 + u ** 3 / 7 + u ** 4 / 9 + u ** 5 / 11))
        got = log_mean(torch.tensor(a), torch.tensor(b)).numpy()
        assert np.max(np.abs(got - series) / series) < 4e-16, rel
    # far apart: the closed form, limit and symmetry
    assert abs(float(log_mean(torch.tensor(1.0, dtype=torch.float64), torch.tensor(np.e, dtype=torch.float64))) - (np.e - 1)) < 1e-15
    x = torch.tensor([0.3, 2.0, 7.5], dtype=torch.float64)
    assert torch.equal(log_mean(x, x), x)
    y = torch.tensor([4.0, 0.1, 7.6], dtype=torch.float64)
    assert torch.allclose(log_mean(x, y), log_mean(y, x), rtol=1e-15, atol=0)


# --- two-point flux -------------------------------------------------------------

@pytest.mark.parametrize("l", [0, 1, 2])
def test_ranocha_flux_symmetric_and_consistent(l):
    UL, UR = random_states(500, 1), random_states(500, 2)
    assert torch.allclose(ranocha_flux(UL, UR, l, G), ranocha_flux(UR, UL, l, G), rtol=1e-14, atol=1e-14)
    ph = Euler(3)
    F = ph.flux(UL, l, ph.prims(UL))
    assert torch.allclose(ranocha_flux(UL, UL, l, G), F, rtol=1e-14, atol=1e-14)


@pytest.mark.parametrize("l", [0, 1, 2])
def test_tadmor_entropy_conservation_condition(l):
    """(w_R - w_L) . F#_l = psi_R - psi_L with psi = rho u_l: the defining
    property of an entropy-conservative two-point flux."""
    UL, UR = random_states(2000, 10 + l), random_states(2000, 20 + l)
    lhs = ((entropy_vars(UR) - entropy_vars(UL)) * ranocha_flux(UL, UR, l, G)).sum(1)
    rhs = UR[:, 1 + l] - UL[:, 1 + l]
    assert float(((lhs - rhs).abs() / (rhs.abs() + 1)).max()) < 1e-13


def test_energy_row_as_printed_fails_tadmor():
    """The reading's evidence: the printed energy row (1/2 in the first term,
    squared arithmetic means, {{p u}}) violates the condition by O(1)."""
    UL, UR = random_states(200, 5), random_states(200, 6)
    F = ranocha_flux(UL, UR, 0, G).clone()
    rL, rR = UL[:, 0], UR[:, 0]
    uL, uR = UL[:, 1:4] / rL[:, None], UR[:, 1:4] / rR[:, None]
    pL = (G - 1) * (UL[:, 4] - 0.5 * rL * (uL * uL).sum(1))
    pR = (G - 1) * (UR[:, 4] - 0.5 * rR * (uR * uR).sum(1))
    ua = 0.5 * (uL + uR)
    F[:, 4] = F[:, 0] * (1 / (2 * (G - 1) * log_mean(rL / pL, rR / pR)) + 0.5 * (ua * ua).sum(1)) \
        + 0.5 * (pL * uL[:, 0] + pR * uR[:, 0])
    lhs = ((entropy_vars(UR) - entropy_vars(UL)) * F).sum(1)
    rhs = UR[:, 1] - UL[:, 1]
    assert float(((lhs - rhs).abs() / (rhs.abs() + 1)).max()) > 1e-2


# --- the semi-discretisation -------------------------------------------------------

def split_op(dim, N, nel, lo, hi, surface="rusanov", patch=None):
    m = cartesian_mesh(dim, N, nel, lo, hi, *(patch or (None, None)))
    return SplitOperator(m, Euler(dim), surface=surface)


def random_state(op, seed):
    rng = np.random.default_rng(seed)
    shape = (op.mesh.E,) + (op.n,) * op.dim
    rho = rng.uniform(0.5, 1.5, shape)
    vel = [rng.uniform(-0.5, 0.5, shape) for _ in range(op.dim)]
    p = rng.uniform(0.5, 1.5, shape)
    return torch.tensor(di.conserved_from_primitive(rho, vel, p, G))[None]


def jw(op):
    Wt = tensor_weights(op)
    return op.J.reshape((-1,) + (1,) * op.dim) * Wt


@pytest.mark.parametrize("case", ["2d", "3d", "mortar"])
def test_free_stream_and_conservation(case):
    if case == "2d":
        op = split_op(2, 3, (4, 3), (0, 0), (1.0, 1.3))
    elif case == "3d":
        op = split_op(3, 2, (3, 2, 3), (0, 0, 0), (1.0, 0.8, 1.2))
    else:
        op = split_op(2, 3, (8, 8), (0, 0), (1.0, 1.0), patch=((2, 2), (5, 6)))
    U = random_state(op, 4)
    c = U.mean(dim=tuple(range(2, U.dim())), keepdim=True).expand_as(U).clone()
    assert float(op.rhs(c).abs().max()) < 1e-12
    dU = op.rhs(U)
    I = integrals(op, dU, with_ke=False)[:, :-1]
    red = tuple(range(2, 3 + op.dim))
    scale = (jw(op) * dU.abs()).sum(dim=red).numpy()
    assert np.abs(I / scale).max() < 1e-13


@pytest.mark.parametrize("dim,N", [(2, 2), (2, 4), (3, 3)])
def test_entropy_conserved_with_ec_interfaces_and_dissipated_with_rusanov(dim, N):
    """sum J w_i w(U_i) . L(U)_i is zero (to rounding) when the interfaces use
    the two-point flux itself, and negative with the Rusanov flux."""
    nel = (4, 3) if dim == 2 else (3, 2, 2)
    lo, hi = (0.0,) * dim, (1.0, 1.2, 0.9)[:dim]
    op_ec = split_op(dim, N, nel, lo, hi, surface="ec")
    op_rs = split_op(dim, N, nel, lo, hi, surface="rusanov")
    U = random_state(op_ec, 11 + N)
    W = entropy_vars(U.reshape(1, dim + 2, -1)).reshape(U.shape)
    wts = jw(op_ec)
    def production(op):
        dU = op.rhs(U)
        return float((wts * (W * dU).sum(1)).sum()), float((wts * (W * dU).abs().sum(1)).sum())
    p_ec, s_ec = production(op_ec)
    p_rs, s_rs = production(op_rs)
    assert abs(p_ec) < 1e-13 * s_ec
    assert p_rs < -1e-6 * s_rs


def test_split_differs_from_standard_but_converges_with_it():
    """On a smooth, resolved periodic state the two volume forms approximate
    the same divergence to O(h^N): at N = 3 their nodal difference is nonzero
    and falls by 2^3 per halving of h (a wrong D index, a missing factor 2 or a
    non-symmetric two-point flux makes it O(1) instead)."""
    diffs = []
    for nel in (8, 16, 32):
        m = cartesian_mesh(2, 3, (nel, nel), (0, 0), (1, 1))
        x, y = m.coords()
        rho = 1 + 0.2 * np.sin(2 * np.pi * x) * np.cos(2 * np.pi * y)
        u = 0.3 + 0.1 * np.cos(2 * np.pi * y)
        v = -0.2 + 0.1 * np.sin(2 * np.pi * (x + y))
        p = 1 + 0.1 * np.cos(2 * np.pi * x)
        U = torch.tensor(di.conserved_from_primitive(rho, [u, v], p, G))[None]
        a = SplitOperator(m, Euler(2)).rhs(U)
        b = Operator(m, Euler(2)).rhs(U)
        diffs.append(float((a - b).abs().max()))
    assert diffs[0] > 1e-4
    rates = [diffs[i] / diffs[i + 1] for i in range(2)]
    assert rates[0] > 2 ** 2.5 and rates[1] > 2 ** 2.8, (diffs, rates)


def test_vortex_convergence():
    errs = []
    for nel in (8, 16):
        m = cartesian_mesh(2, 3, (nel, nel), (-5, -5), (5, 5))
        op = SplitOperator(m, Euler(2))
        U = torch.tensor(di.vortex(m.coords(), 0.0))[None]
        T = 0.5
        dt = dt_cfl(op, U, 0.5)
        nsteps = int(np.ceil(T / dt))
        dt = T / nsteps
        for _ in range(nsteps):
            U = ssprk33_step(op, U, dt)
        ex = torch.tensor(di.vortex(m.coords(), T))[None]
        errs.append(float((U[:, 0] - ex[:, 0]).abs().max()))
    order = np.log2(errs[0] / errs[1])
    assert 3.0 < order < 5.5, (errs, order)


def test_split_navier_stokes_free_stream_conservation_and_viscous_part():
    """Split form with the BR1 viscous terms: a uniform state is steady, the
    right-hand side of a rough state conserves mass, momentum and energy, and
    the viscous part is the standard operator's (the split form changes only
    the inviscid volume term)."""
    from oracle.split import SplitOperator
    from oracle.timestep import integrals
    visc = dict(mu=2e-2, prandtl=0.72, gamma=1.4)
    mesh = cartesian_mesh(3, 3, (3, 4, 3), (0, 0, 0), (1.0, 1.2, 0.9))
    ns = SplitOperator(mesh, Euler(3), viscous=visc)
    eu = SplitOperator(mesh, Euler(3))
    std = Operator(mesh, Euler(3), viscous=visc)
    c = torch.zeros((1, 5, mesh.E) + (4,) * 3, dtype=torch.float64)
    c[:, 0], c[:, 1], c[:, 2], c[:, 3] = 1.1, 0.33, -0.22, 0.11
    c[:, 4] = 0.9 / 0.4 + 0.5 * (0.33 ** 2 + 0.22 ** 2 + 0.11 ** 2) / 1.1
    assert float(ns.rhs(c).abs().max()) < 1e-12
    rng = np.random.default_rng(4)
    shape = (1, mesh.E) + (4,) * 3
    rho = rng.uniform(0.5, 1.5, shape)
    vel = [rng.uniform(-0.5, 0.5, shape) for _ in range(3)]
    p = rng.uniform(0.5, 1.5, shape)
    U = torch.tensor(np.stack([di.conserved_from_primitive(rho[0], [v[0] for v in vel], p[0], 1.4)]))
    dU = ns.rhs(U)
    I = np.asarray(integrals(ns, dU, with_ke=False))[0, :5]
    S = np.asarray(integrals(ns, dU.abs(), with_ke=False))[0, :5]
    assert float((np.abs(I) / S).max()) < 1e-13
    assert float((dU - eu.rhs(U) - std.rhs_viscous(U)).abs().max()) <= 1e-13 * float(dU.abs().max())


def test_split_navier_stokes_tgv_dissipation_rate():
    """Taylor-Green initial state (continuous across elements, so the
    Rusanov jumps vanish): the split form's inviscid volume term preserves
    kinetic energy up to the pressure work, which vanishes for this
    divergence-free field, so dE_k/dt of the whole right-hand side is the
    viscous -3/4 mu (rho = 1; measured to 3e-12 on 8^3, N = 4), and the
    inviscid part alone to round-off."""
    from oracle.split import SplitOperator
    from oracle.timestep import tensor_weights
    P = di.PRESETS["tgv3d"]
    mesh = cartesian_mesh(3, 4, (8, 8, 8), P["lo"], P["hi"])
    op = SplitOperator(mesh, Euler(3), viscous=dict(mu=P["mu"], prandtl=P["prandtl"], gamma=1.4))
    U = torch.tensor(di.taylor_green(mesh.coords(), mach=P["mach"]))[None]
    dU = op.rhs(U)
    vel = U[:, 1:4] / U[:, 0:1]
    ke_rate = (vel * dU[:, 1:4]).sum(1) - 0.5 * (vel * vel).sum(1) * dU[:, 0]
    w = tensor_weights(op) * op.J.reshape((-1,) + (1,) * 3)
    rate = float((w[None] * ke_rate).sum()) / (2 * np.pi) ** 3
    assert abs(rate / (-0.75 * P["mu"]) - 1.0) < 1e-8, rate
    # the inviscid split part alone: kinetic energy preserved to round-off
    dE = SplitOperator(mesh, Euler(3)).rhs(U)
    ke_e = (vel * dE[:, 1:4]).sum(1) - 0.5 * (vel * vel).sum(1) * dE[:, 0]
    assert abs(float((w[None] * ke_e).sum()) / (2 * np.pi) ** 3) < 1e-12 * P["mu"]
