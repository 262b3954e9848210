"""Entropy-conservative split-form volume integral for the Euler equations on
affine Cartesian elements (eq. vol_split; the appendix paragraph on the
inviscid volume flux in entropy-conservative split form, eq.
split_form_3D) -- test infrastructure, as the rest of the oracle.

At node i of an element, direction l contributes
    -(2 / J) sum_m D_im  Ja^l F#_l(U_i, U_m),
the sum running over the nodes m of the line through i along l (for an
affine element Ja^l = (2J/h_l) e_l at both partner nodes, so their average is
that same vector).  The surface term is the strong-form lift of eq. surf_int
unchanged: (F* - F(U_i)) at face nodes, with F the physical flux.

Two-point flux: the kinetic-energy-preserving, entropy-conservative flux of
Ranocha that the paper names and cites, in its published form
    f_rho = {{rho}}_ln {{u_l}},
    f_m_d = f_rho {{u_d}} + {{p}} delta_dl,
    f_E   = f_rho (1 / ((gamma - 1) {{rho/p}}_ln) + u_L . u_R / 2)
            + (p_L u_R,l + p_R u_L,l) / 2,
with {{a}} the arithmetic and {{a}}_ln = (a_L - a_R) / (ln a_L - ln a_R) the
logarithmic mean.  Reading: the energy row as printed in the paper (a factor
1/2 in the first term, the arithmetic means squared instead of u_L . u_R,
{{p u}} instead of the crossed product) does not satisfy Tadmor's
entropy-conservation condition the paper relies on; the published row does
(pinned in the tests by that identity).
"""

import torch

from .dgsem import Operator, node_axis


def log_mean(a, b):
    """{{a}}_ln = (a - b) / (ln a - ln b), with its limit a at a = b.  Written
    as (a - b) / log1p((a - b) / b): for nearby arguments a - b is exact and
    log1p keeps the relative accuracy that ln a - ln b would lose."""
    d = a - b
    out = d / torch.log1p(d / b)
    return torch.where(d == 0, a, out)


def euler_prims(U, gamma):
    """rho, velocity components, p of a conserved state (B, nv, ...)."""
    dim = U.shape[1] - 2
    rho = U[:, 0]
    u = [U[:, 1 + d] / rho for d in range(dim)]
    ke = 0.5 * sum(U[:, 1 + d] * u[d] for d in range(dim))
    p = (gamma - 1.0) * (U[:, dim + 1] - ke)
    return rho, u, p


def ranocha_flux(UL, UR, l, gamma):
    """F#_l(U_L, U_R) along Cartesian direction l, stacked over variables."""
    dim = UL.shape[1] - 2
    rL, uL, pL = euler_prims(UL, gamma)
    rR, uR, pR = euler_prims(UR, gamma)
    rho_ln = log_mean(rL, rR)
    b_ln = log_mean(rL / pL, rR / pR)
    ua = [0.5 * (uL[d] + uR[d]) for d in range(dim)]
    pa = 0.5 * (pL + pR)
    f_rho = rho_ln * ua[l]
    rows = [f_rho]
    for d in range(dim):
        rows.append(f_rho * ua[d] + (pa if d == l else 0.0))
    uu = sum(uL[d] * uR[d] for d in range(dim))
    rows.append(f_rho * (1.0 / ((gamma - 1.0) * b_ln) + 0.5 * uu) + 0.5 * (pL * uR[l] + pR * uL[l]))
    return torch.stack(rows, dim=1)


def ranocha_flux_n(UL, UR, nvec, gamma):
    """F#(U_L, U_R) . n for a direction field n (dim tensors broadcasting
    against the states' node axes): the flux above is linear in the
    direction, f_rho = {{rho}}_ln {{u}} . n, f_m_d = f_rho {{u_d}} + {{p}} n_d,
    f_E = f_rho (1 / ((gamma - 1) {{rho/p}}_ln) + u_L . u_R / 2)
          + (p_L u_R . n + p_R u_L . n) / 2;
    n = e_l gives ranocha_flux along l."""
    dim = UL.shape[1] - 2
    rL, uL, pL = euler_prims(UL, gamma)
    rR, uR, pR = euler_prims(UR, gamma)
    rho_ln = log_mean(rL, rR)
    b_ln = log_mean(rL / pL, rR / pR)
    ua = [0.5 * (uL[d] + uR[d]) for d in range(dim)]
    pa = 0.5 * (pL + pR)
    f_rho = rho_ln * sum(ua[d] * nvec[d] for d in range(dim))
    rows = [f_rho]
    for d in range(dim):
        rows.append(f_rho * ua[d] + pa * nvec[d])
    uu = sum(uL[d] * uR[d] for d in range(dim))
    uRn = sum(uR[d] * nvec[d] for d in range(dim))
    uLn = sum(uL[d] * nvec[d] for d in range(dim))
    rows.append(f_rho * (1.0 / ((gamma - 1.0) * b_ln) + 0.5 * uu) + 0.5 * (pL * uRn + pR * uLn))
    return torch.stack(rows, dim=1)


def split_volume(op, U):
    """-(2/J) sum_l sum_m D_im Ja^l F#_l(U_i, U_m) for every node."""
    dim, gamma = op.dim, op.phys.gamma
    J = op.per_elem(op.J)
    out = torch.zeros_like(U)
    for l in range(dim):
        ax = node_axis(dim, l)
        X = U.movedim(ax, -1)                      # (..., n) along l
        n = X.shape[-1]
        XL = X.unsqueeze(-1).expand(*X.shape, n)   # U_i at [..., i, m]
        XR = X.unsqueeze(-2).expand(*X.shape[:-1], n, n)  # U_m at [..., i, m]
        F = ranocha_flux(XL, XR, l, gamma)        # (B, nv, ..., i, m)
        s = torch.einsum("...im,im->...i", F, op.D)
        Ja = op.per_elem(op.Ja[l])
        out = out - 2.0 * (Ja * s.movedim(-1, ax)) / J
    return out


class SplitOperator(Operator):
    """L(U) with the split-form volume integral and the strong-form surface
    lift; surface="rusanov" (the solver's interface flux) or "ec" (the
    two-point flux itself at the interfaces, for the entropy-conservation
    check).  Euler physics, conforming or 2:1 mortar meshes; with viscous=
    (mu, prandtl, gamma) the BR1 viscous terms of the standard operator are
    added unchanged (Navier-Stokes, the paper's Taylor-Green setting)."""

    def __init__(self, mesh, phys, surface="rusanov", viscous=None):
        super().__init__(mesh, phys, viscous=viscous)
        if surface not in ("rusanov", "ec"):
            raise ValueError(surface)
        self.surface = surface

    def rusanov(self, UL, UR, PL, PR, l, nmag):
        if self.surface == "rusanov":
            return super().rusanov(UL, UR, PL, PR, l, nmag)
        return nmag.unsqueeze(1) * ranocha_flux(UL, UR, l, self.phys.gamma)

    def volume_term(self, U, F, form):
        if form != "strong":
            raise ValueError("the split form is a strong-form operator")
        return split_volume(self, U)
