"""Pins of the oracle's curvilinear operator and boundary fluxes against what
the mathematics fixes: reduction to the Cartesian operator at zero warp,
free-stream preservation (the discrete GCL) and conservation on warped
periodic meshes, the Jacobian against the analytic determinant of the warp
(spectral convergence and the preserved area), vortex convergence on a warped
mesh, slip walls (no mass or energy through them; a flow tangent to straight
walls is steady) and supersonic inflow/outflow (a uniform supersonic stream is
steady through curved boundaries).  The split form on curvilinear elements:
the two-point flux along a vector against the Cartesian one and its
linearity, reduction to the Cartesian split operator at zero warp, free
stream, conservation and entropy conservation (EC interfaces) on warped
meshes -- the last two failing when the pair's metrics are not averaged --
and vortex convergence.  BR1 viscous terms with per-node metrics: reduction to
the Cartesian Navier-Stokes operator at zero warp, free stream and
conservation on warped meshes (both volume forms), the lifted gradient
integrating to zero on a periodic mesh (and not with the face terms' sign
flipped), convergence of the viscous term to its exact value for a
manufactured state at the Cartesian operator's rate, and the Taylor-Green
dissipation rate -3/4 mu approached on a warped box."""

import math

import numpy as np
import pytest
import torch

import dginputs as di
from oracle.curvilinear import CurvMesh, CurvOperator
from oracle.dgsem import Operator
from oracle.mesh import cartesian_mesh
from oracle.physics import Euler
from oracle.timestep import ssprk33_step

G = 1.4


def weights(m):
    w = m.w
    Wt = w
    for _ in range(m.dim - 1):
        Wt = Wt.unsqueeze(0) * w.reshape((-1,) + (1,) * Wt.dim())
    return m.J * Wt[None]


def rand_state(m, seed):
    rng = np.random.default_rng(seed)
    shape = m.X.shape[1:]
    rho = rng.uniform(0.5, 1.5, shape)
    vel = [rng.uniform(-0.5, 0.5, shape) for _ in range(m.dim)]
    p = rng.uniform(0.5, 1.5, shape)
    return torch.tensor(di.conserved_from_primitive(rho, vel, p, G))[None]


def uniform(m, rho, vel, p):
    U = torch.zeros((1, m.dim + 2) + tuple(m.X.shape[1:]), dtype=torch.float64)
    U[:, 0] = rho
    for d in range(m.dim):
        U[:, 1 + d] = rho * vel[d]
    U[:, -1] = p / (G - 1) + 0.5 * rho * sum(v * v for v in vel)
    return U


def flux_scale(m, U):
    ph = Euler(m.dim)
    P = ph.prims(U)
    F = max(float(ph.flux(U, l, P).abs().max()) for l in range(m.dim))
    Ja = max(float(m.Ja[l].abs().max()) for l in range(m.dim))
    return F * Ja * float(m.D.abs().sum(1).max()) / float(m.J.abs().min())


@pytest.mark.parametrize("dim", [2, 3])
def test_zero_warp_equals_cartesian_operator(dim):
    nel, lo, hi = ((4, 3), (0, 0), (1.0, 1.3)) if dim == 2 else ((3, 2, 3), (0, 0, 0), (1.0, 0.8, 1.2))
    m = CurvMesh(dim, 3, nel, lo, hi, 0.0)
    U = rand_state(m, 1)
    a = CurvOperator(m).rhs(U)
    b = Operator(cartesian_mesh(dim, 3, nel, lo, hi), Euler(dim)).rhs(U)
    assert float((a - b).abs().max()) < 1e-13 * float(b.abs().max())


@pytest.mark.parametrize("dim,N", [(2, 2), (2, 4), (3, 2), (3, 3)])
def test_free_stream_and_conservation_on_warped_mesh(dim, N):
    nel = (4, 3) if dim == 2 else (3, 3, 2)
    lo, hi = (0.0,) * dim, (1.0, 1.2, 0.9)[:dim]
    m = CurvMesh(dim, N, nel, lo, hi, 0.04)
    assert float(m.J.min()) > 0
    op = CurvOperator(m)
    c = uniform(m, 1.1, (0.3, -0.2, 0.1)[:dim], 0.9)
    assert float(op.rhs(c).abs().max()) < 1e-13 * flux_scale(m, c)
    U = rand_state(m, 2)
    dU = op.rhs(U)
    wJ = weights(m)
    red = tuple(range(1, 1 + dim))
    I = torch.stack([(wJ * dU[0, v]).sum(dim=(0,) + red) for v in range(dim + 2)])
    S = torch.stack([(wJ * dU[0, v].abs()).sum(dim=(0,) + red) for v in range(dim + 2)])
    assert float((I.abs() / S).max()) < 1e-13


def test_jacobian_against_the_analytic_determinant():
    """2-D warp: det = 1 - 4 pi^2 A^2 cos(2 pi s_x) cos(2 pi s_y) in physical
    units; the reference Jacobian is that times (h_x/2)(h_y/2).  The
    polynomial J converges spectrally and the area is preserved."""
    A, lo, hi, nel = 0.05, (0.0, 0.0), (1.0, 1.0), (4, 4)
    errs = []
    for N in (3, 6):
        m = CurvMesh(2, N, nel, lo, hi, A)
        Xc = torch.tensor(m.base.coords())
        exact = (1 - 4 * math.pi ** 2 * A ** 2 * torch.cos(2 * math.pi * Xc[0]) * torch.cos(2 * math.pi * Xc[1]))
        exact = exact * (0.25 / 2) ** 2
        errs.append(float(((m.J - exact) / exact).abs().max()))
        area = float(weights(m).sum())
        assert abs(area - 1.0) < (1e-3 if N == 3 else 1e-7)
    assert errs[1] < errs[0] / 50 and errs[1] < 1e-5, errs


def test_vortex_convergence_on_warped_mesh():
    errs = []
    for nel in (8, 16):
        m = CurvMesh(2, 3, (nel, nel), (-5, -5), (5, 5), 0.02)
        op = CurvOperator(m)
        U = torch.tensor(di.vortex(m.coords(), 0.0))[None]
        T = 0.5
        h = 10.0 / nel
        dt = 0.5 * h / (7 * op.lam_max(U))
        nsteps = int(np.ceil(T / dt))
        dt = T / nsteps
        for _ in range(nsteps):
            U = ssprk33_step(op, U, dt)
        ex = torch.tensor(di.vortex(m.coords(), T))[None]
        errs.append(float((U[:, 0] - ex[:, 0]).abs().max()))
    order = math.log2(errs[0] / errs[1])
    assert 2.8 < order < 5.5, (errs, order)


def test_slip_walls_conserve_mass_and_energy():
    for dim in (2, 3):
        nel = (4, 3) if dim == 2 else (3, 2, 2)
        m = CurvMesh(dim, 3, nel, (0.0,) * dim, (1.0, 1.2, 0.9)[:dim], 0.03, bc=("wall",) * (2 * dim))
        op = CurvOperator(m)
        U = rand_state(m, 3)
        dU = op.rhs(U)
        wJ = weights(m)
        red = tuple(range(0, 1 + dim))
        for v in (0, dim + 1):
            assert abs(float((wJ * dU[0, v]).sum())) < 1e-13 * float((wJ * dU[0, v].abs()).sum())
        mom = abs(float((wJ * dU[0, 1]).sum())) / float((wJ * dU[0, 1].abs()).sum())
        assert mom > 1e-6          # walls push: momentum is not conserved


def test_flow_tangent_to_straight_walls_is_steady():
    m = CurvMesh(2, 3, (4, 3), (0.0, 0.0), (1.0, 1.0), 0.0, bc=("periodic", "periodic", "wall", "wall"))
    c = uniform(m, 1.2, (0.7, 0.0), 1.1)
    assert float(CurvOperator(m).rhs(c).abs().max()) < 1e-13 * flux_scale(m, c)


@pytest.mark.parametrize("dim", [2, 3])
def test_uniform_supersonic_stream_through_curved_boundaries(dim):
    nel = (4, 3) if dim == 2 else (3, 2, 2)
    bc = ("inflow", "outflow") + ("periodic", "periodic") * (dim - 1)
    m = CurvMesh(dim, 3, nel, (0.0,) * dim, (1.0, 1.0, 1.0)[:dim], 0.03, bc=bc)
    vel = (2.5, 0.3, -0.2)[:dim]                # Mach > 2 along x
    c = uniform(m, 1.0, vel, 1.0 / G)
    op = CurvOperator(m, bc_state=c[0, :, 0].reshape(dim + 2, -1)[:, 0].numpy())
    assert float(op.rhs(c).abs().max()) < 1e-13 * flux_scale(m, c)


@pytest.mark.parametrize("dim", [2, 3])
def test_free_stream_far_from_the_origin(dim):
    """The same warped box translated to 1000: free stream is still preserved
    to rounding relative to the element size.  (Metric terms formed from
    absolute coordinates lose the digits of |x| / h, about 1e-11 of the flux
    scale here.)"""
    nel = (4, 3) if dim == 2 else (3, 3, 2)
    N = 4
    size = (1.0, 1.2, 0.9)[:dim]
    for off in (0.0, 1000.0):
        lo = tuple(off for _ in range(dim))
        hi = tuple(off + s for s in size)
        m = CurvMesh(dim, N, nel, lo, hi, 0.04)
        op = CurvOperator(m)
        c = uniform(m, 1.1, (0.3, -0.2, 0.1)[:dim], 0.9)
        res = float(op.rhs(c).abs().max()) / flux_scale(m, c)
        assert res < 2e-14, (off, res)


# --- split form on curvilinear elements -------------------------------------------

def _entropy_vars(U):
    """d eta / dU for eta = -rho s / (gamma - 1), s = ln(p rho^-gamma)."""
    rho, m, E = U[:, 0], U[:, 1:-1], U[:, -1]
    u = m / rho[:, None]
    p = (G - 1) * (E - 0.5 * (m * u).sum(1))
    s = torch.log(p) - G * torch.log(rho)
    w0 = (G - s) / (G - 1) - 0.5 * rho * (u * u).sum(1) / p
    return torch.cat([w0[:, None], rho[:, None] * u / p[:, None], -(rho / p)[:, None]], 1)


def test_ranocha_flux_along_a_vector_reduces_and_is_linear():
    """F#(U_L, U_R) . n: n = e_l gives the Cartesian flux along l bit for bit,
    and the flux is linear in n."""
    from oracle.split import ranocha_flux, ranocha_flux_n
    rng = np.random.default_rng(5)
    def states(seed):
        r = np.random.default_rng(seed)
        return torch.tensor(di.conserved_from_primitive(r.uniform(0.5, 2, 50), [r.uniform(-1, 1, 50) for _ in range(3)],
                                                        r.uniform(0.5, 2, 50), G))[None]
    UL, UR = states(1), states(2)
    for l in range(3):
        e = [torch.full((50,), 1.0 if d == l else 0.0, dtype=torch.float64) for d in range(3)]
        assert torch.equal(ranocha_flux_n(UL, UR, e, G), ranocha_flux(UL, UR, l, G))
    n1 = [torch.tensor(rng.normal(size=50)) for _ in range(3)]
    n2 = [torch.tensor(rng.normal(size=50)) for _ in range(3)]
    a, b = 0.7, -1.3
    lhs = ranocha_flux_n(UL, UR, [a * x + b * y for x, y in zip(n1, n2)], G)
    rhs = a * ranocha_flux_n(UL, UR, n1, G) + b * ranocha_flux_n(UL, UR, n2, G)
    assert float((lhs - rhs).abs().max()) < 1e-13 * float(rhs.abs().max())


@pytest.mark.parametrize("dim", [2, 3])
def test_split_zero_warp_equals_cartesian_split_operator(dim):
    from oracle.split import SplitOperator
    nel, lo, hi = ((4, 3), (0, 0), (1.0, 1.3)) if dim == 2 else ((3, 2, 3), (0, 0, 0), (1.0, 0.8, 1.2))
    m = CurvMesh(dim, 3, nel, lo, hi, 0.0)
    U = rand_state(m, 1)
    a = CurvOperator(m, volume="split").rhs(U)
    b = SplitOperator(cartesian_mesh(dim, 3, nel, lo, hi), Euler(dim)).rhs(U)
    assert float((a - b).abs().max()) < 1e-13 * float(b.abs().max())


def _split_volume_one_sided(op, U, side):
    """The split volume term with the metrics of node i only (side 0) or of
    node m only (side 1) instead of their average: planted mistakes."""
    from oracle.dgsem import node_axis
    from oracle.split import ranocha_flux_n
    m, dim = op.mesh, op.dim
    out = torch.zeros_like(U)
    for l in range(dim):
        ax = node_axis(dim, l)
        X = U.movedim(ax, -1)
        n = X.shape[-1]
        XL = X.unsqueeze(-1).expand(*X.shape, n)
        XR = X.unsqueeze(-2).expand(*X.shape[:-1], n, n)
        Ja = m.Ja[l].movedim(ax - 1, -1)
        Jav = [(Ja[d].unsqueeze(-1) if side == 0 else Ja[d].unsqueeze(-2)).expand(*Ja[d].shape, n)
               for d in range(dim)]
        F = ranocha_flux_n(XL, XR, Jav, G)
        out = out - 2.0 * torch.einsum("...im,im->...i", F, m.D).movedim(-1, ax)
    return out


@pytest.mark.parametrize("dim,N", [(2, 2), (2, 4), (3, 2), (3, 3)])
def test_split_free_stream_conservation_and_entropy_on_warped_mesh(dim, N):
    """Warped periodic mesh: a constant state stays constant (discrete GCL);
    sum J w dU/dt = 0 (the two-point flux with averaged metrics is
    symmetric in its nodes); with the two-point flux at the interfaces the
    entropy production sum J w w(U) . dU/dt is zero to rounding, and negative
    with the Rusanov flux.  The metrics of one node only keep the free stream
    but break conservation and entropy conservation."""
    nel = (4, 3) if dim == 2 else (3, 3, 2)
    lo, hi = (0.0,) * dim, (1.0, 1.2, 0.9)[:dim]
    m = CurvMesh(dim, N, nel, lo, hi, 0.04)
    op = CurvOperator(m, volume="split")
    op_ec = CurvOperator(m, volume="split", surface="ec")
    c = uniform(m, 1.1, (0.3, -0.2, 0.1)[:dim], 0.9)
    assert float(op.rhs(c).abs().max()) < 1e-13 * flux_scale(m, c)
    U = rand_state(m, 2 + N)
    wJ = weights(m)
    red = tuple(range(1, 1 + dim))

    def cons(dU):
        I = torch.stack([(wJ * dU[0, v]).sum(dim=(0,) + red) for v in range(dim + 2)])
        S = torch.stack([(wJ * dU[0, v].abs()).sum(dim=(0,) + red) for v in range(dim + 2)])
        return float((I.abs() / S).max())

    W = _entropy_vars(U.reshape(1, dim + 2, -1)).reshape(U.shape)

    def production(dU):
        return float((wJ * (W * dU).sum(1)[0]).sum()), float((wJ * (W * dU).abs().sum(1)[0]).sum())

    assert cons(op.rhs(U)) < 1e-13
    p_ec, s_ec = production(op_ec.rhs(U))
    assert abs(p_ec) < 1e-13 * s_ec
    p_rs, s_rs = production(op.rhs(U))
    assert p_rs < -1e-6 * s_rs
    # planted: metrics of one node of each pair (3-D only: the 2-D warp keeps
    # each Ja^l constant along its own lines, where the average is exact)
    for side in ((0, 1) if dim == 3 else ()):
        bad = op_ec.rhs(U) - op_ec.split_volume(U) / m.J[None, None] + _split_volume_one_sided(op_ec, U, side) / m.J[None, None]
        p_bad, s_bad = production(bad)
        assert cons(bad) > 1e-8 or abs(p_bad) > 1e-8 * s_bad


def test_split_vortex_convergence_on_warped_mesh():
    """The isentropic vortex advected to T = 0.5 on a warped periodic mesh
    with the split form: the density error converges at the standard form's
    rate (8^2 -> 16^2, N = 3)."""
    errs = []
    for nel in (8, 16):
        m = CurvMesh(2, 3, (nel, nel), (-5, -5), (5, 5), 0.02)
        op = CurvOperator(m, volume="split")
        U = torch.tensor(di.vortex(m.coords(), 0.0))[None]
        T = 0.5
        h = 10.0 / nel
        dt = 0.5 * h / (7 * op.lam_max(U))
        nsteps = int(np.ceil(T / dt))
        dt = T / nsteps
        for _ in range(nsteps):
            U = ssprk33_step(op, U, dt)
        ex = torch.tensor(di.vortex(m.coords(), T))[None]
        errs.append(float((U[:, 0] - ex[:, 0]).abs().max()))
    order = math.log2(errs[0] / errs[1])
    assert 2.8 < order < 5.5, (errs, order)


# --- BR1 viscous terms on curvilinear elements ------------------------------------

VIS = dict(mu=0.05, prandtl=0.72, gamma=G)


@pytest.mark.parametrize("dim", [2, 3])
def test_viscous_zero_warp_equals_cartesian_navier_stokes(dim):
    nel, lo, hi = ((4, 3), (0, 0), (1.0, 1.3)) if dim == 2 else ((3, 2, 3), (0, 0, 0), (1.0, 0.8, 1.2))
    m = CurvMesh(dim, 3, nel, lo, hi, 0.0)
    U = rand_state(m, 1)
    a = CurvOperator(m, viscous=VIS).rhs(U)
    b = Operator(cartesian_mesh(dim, 3, nel, lo, hi), Euler(dim), viscous=VIS).rhs(U)
    assert float((a - b).abs().max()) < 1e-13 * float(b.abs().max())


@pytest.mark.parametrize("dim,N", [(2, 2), (2, 4), (3, 2), (3, 3)])
def test_viscous_free_stream_and_conservation_on_warped_mesh(dim, N):
    nel = (4, 3) if dim == 2 else (3, 3, 2)
    lo, hi = (0.0,) * dim, (1.0, 1.2, 0.9)[:dim]
    m = CurvMesh(dim, N, nel, lo, hi, 0.04)
    for volume in ("standard", "split"):
        op = CurvOperator(m, viscous=VIS, volume=volume)
        c = uniform(m, 1.1, (0.3, -0.2, 0.1)[:dim], 0.9)
        assert float(op.rhs(c).abs().max()) < 1e-13 * flux_scale(m, c)
        U = rand_state(m, 2 + N)
        dU = op.rhs_viscous(U)
        wJ = weights(m)
        red = tuple(range(1, 1 + dim))
        I = torch.stack([(wJ * dU[0, v]).sum(dim=(0,) + red) for v in range(dim + 2)])
        S = torch.stack([(wJ * dU[0, v].abs()).sum(dim=(0,) + red) for v in range(1, dim + 2)])
        assert float(I[0].abs()) == 0.0   # no mass row
        assert float((I[1:].abs() / S).max()) < 1e-13


def _manufactured(X):
    """A smooth periodic state on the unit box and its exact viscous term
    div F_v(U, grad W) (by automatic differentiation in physical space)."""
    tp = 2 * math.pi
    x = X[0].reshape(-1).clone().requires_grad_(True)
    y = X[1].reshape(-1).clone().requires_grad_(True)
    rho = 1 + 0.1 * torch.sin(tp * x) * torch.cos(tp * y)
    u = 0.3 * torch.sin(tp * y) + 0.1 * torch.cos(tp * x)
    v = 0.2 * torch.cos(tp * x) * torch.sin(tp * y)
    p = 1 + 0.1 * torch.cos(tp * (x + y))
    T = p / rho

    def grad(f):
        return torch.autograd.grad(f.sum(), (x, y), create_graph=True)

    ux, uy = grad(u)
    vx, vy = grad(v)
    Tx, Ty = grad(T)
    mu = VIS["mu"]
    k = G * mu / (VIS["prandtl"] * (G - 1))
    div = ux + vy
    txx, tyy, txy = mu * (2 * ux - 2 / 3 * div), mu * (2 * vy - 2 / 3 * div), mu * (uy + vx)
    Fx = [txx, txy, u * txx + v * txy + k * Tx]
    Fy = [txy, tyy, u * txy + v * tyy + k * Ty]
    ex = torch.stack([torch.zeros_like(x)] + [grad(Fx[i])[0] + grad(Fy[i])[1] for i in range(3)])
    U = di.conserved_from_primitive(rho.detach().numpy(), [u.detach().numpy(), v.detach().numpy()],
                                    p.detach().numpy(), G)
    shape = X.shape[1:]
    return torch.tensor(U).reshape((1, 4) + shape), ex.detach().reshape((1, 4) + shape)


class _LiftSignFlipped(CurvOperator):
    """A planted mistake: the gradient's face terms with the wrong sign."""

    def br1_gradient(self, W):
        m = self.mesh
        S = super().br1_gradient(W)
        # the D-sweep part alone, recomputed, and the face part subtracted twice
        from oracle.dgsem import dsweep as _dsweep
        out = []
        for q in range(W.shape[1]):
            row = []
            for d in range(self.dim):
                vol = sum(_dsweep(m.Ja[l][d][None, None] * W[:, q:q + 1], m.D, self.dim, l)
                          for l in range(self.dim))[:, 0] / m.J[None]
                row.append(2 * vol - S[q][d])
            out.append(row)
        return out


def _l2_rates(cls, A, N):
    errs = []
    for nel in (4, 8, 16):
        m = CurvMesh(2, N, (nel, nel), (0, 0), (1, 1), A)
        U, ex = _manufactured(m.X)
        err = cls(m, viscous=VIS).rhs_viscous(U) - ex
        wJ = weights(m)
        errs.append(float(torch.sqrt((wJ[None, None] * err ** 2).sum() / wJ.sum())))
    return [math.log2(errs[i] / errs[i + 1]) for i in range(2)], errs


@pytest.mark.parametrize("N", [3, 4])
def test_viscous_term_converges_on_warped_mesh(N):
    """The BR1 viscous term of a smooth periodic state against its exact value
    (L2 over the box, 4^2 -> 8^2 -> 16^2): on the warped mesh the rate of the
    finest pair is near the Cartesian operator's (2.9 at N = 3, 2.8 at
    N = 4)."""
    rates, errs = _l2_rates(CurvOperator, 0.04, N)
    rates0, _ = _l2_rates(CurvOperator, 0.0, N)
    assert rates[-1] > 2.5 and abs(rates[-1] - rates0[-1]) < 0.4, (rates, rates0, errs)


@pytest.mark.parametrize("dim,N", [(2, 3), (3, 2)])
def test_br1_gradient_integrates_to_zero(dim, N):
    """With a single-valued face trace W^ the lifted gradient of any W -- here
    discontinuous across every face -- integrates to the sum over faces of
    W^ n, which cancels on a periodic mesh: sum J w S = 0 (SBP property and
    the discrete GCL).  The face terms with the wrong sign leave
    sum (2 W - W^) n instead."""
    nel = (4, 3) if dim == 2 else (3, 3, 2)
    m = CurvMesh(dim, N, nel, (0.0,) * dim, (1.0, 1.2, 0.9)[:dim], 0.04)
    rng = np.random.default_rng(7)
    W = torch.tensor(rng.uniform(0.5, 1.5, (1, dim + 2) + tuple(m.X.shape[1:])))
    wJ = weights(m)

    def totals(cls):
        S = cls(m, viscous=VIS).br1_gradient(W)
        I = torch.tensor([[float((wJ * S[q][d][0]).sum()) for d in range(dim)] for q in range(dim + 2)])
        A = torch.tensor([[float((wJ * S[q][d][0].abs()).sum()) for d in range(dim)] for q in range(dim + 2)])
        return float((I.abs() / A).max())

    assert totals(CurvOperator) < 1e-13
    assert totals(_LiftSignFlipped) > 1e-3


def test_taylor_green_dissipation_rate_on_warped_box():
    """The Taylor-Green initial state on the [0, 2 pi]^3 box warped by 0.03,
    N = 4: the kinetic-energy rate of the right-hand side converges to the
    exact -3/4 mu (the viscous dissipation of the initial field; the
    inviscid part, both volume forms, is zero to round-off since the state
    is continuous and divergence-free): relative deviation 8.8e-6 on 4^3 and
    7.6e-8 on 8^3 as measured."""
    P = di.PRESETS["tgv3d"]
    vis = dict(mu=P["mu"], prandtl=P["prandtl"], gamma=G)
    devs = []
    for nel in (4, 8):
        m = CurvMesh(3, 4, (nel,) * 3, P["lo"], P["hi"], 0.03)
        U = torch.tensor(di.taylor_green(m.coords(), mach=P["mach"]))[None]
        wJ = weights(m)
        vel = U[:, 1:4] / U[:, 0:1]

        def rate(dU):
            ke = (vel * dU[:, 1:4]).sum(1) - 0.5 * (vel * vel).sum(1) * dU[:, 0]
            return float((wJ[None] * ke).sum()) / (2 * math.pi) ** 3

        for volume in ("standard", "split"):
            assert abs(rate(CurvOperator(m, volume=volume).rhs(U))) < 1e-11 * P["mu"]
        devs.append(abs(rate(CurvOperator(m, viscous=vis).rhs(U)) / (-0.75 * P["mu"]) - 1.0))
    assert devs[1] < 1e-6 and devs[0] > 30 * devs[1], devs
