"""Pointwise physics: conserved -> primitive recovery with positivity checks,
physical fluxes, viscous flux, reacting-mixture closure.

* Euler / Navier-Stokes: state (rho, rho u, rho v[, rho w], E); inviscid fluxes
  of the Governing Equations section (eq. CNSe and the flux vectors under it);
  ideal-gas closure p = (gamma-1)(E - |m|^2/(2 rho)).
* Viscous flux (Parabolic Terms, eq. tau; Governing Equations): Newtonian
  stress with the Stokes hypothesis, Fourier heat flux q = -k grad T with
  k = gamma mu / (Pr (gamma-1)), non-dimensional R = 1 so T = p / rho; the
  energy row is u.tau - q.
* Reacting Euler (Thermochemical non-equilibrium subsection): state
  (rho_1..rho_Ns, m, E); flux columns rho_s u_n, momentum, (E+p) u_n.  Reading
  taken (single temperature, vibration frozen): translational-rotational energy
  calorically perfect per species, E = sum rho_s cv_s T + |m|^2/(2 rho) +
  sum rho_s h0_s, p = T sum rho_s R_s, frozen sound speed
  a^2 = gamma_f p / rho with gamma_f = 1 + sum rho_s R_s / sum rho_s cv_s.

Non-physical states (rho <= 0, p <= 0, T <= 0) raise NonPhysical.
"""

import torch


class NonPhysical(ArithmeticError):
    pass


class Euler:
    """Compressible Euler (and the inviscid part of Navier-Stokes)."""

    def __init__(self, dim, gamma=1.4, check=True):
        self.dim = dim
        self.gamma = gamma
        self.nv = dim + 2
        self.check = check

    def prims(self, U):
        """U: (B, nv, ...) -> dict(rho, u[list], p, a)."""
        g = self.gamma
        rho = U[:, 0]
        m = [U[:, 1 + d] for d in range(self.dim)]
        E = U[:, self.dim + 1]
        u = [m[d] / rho for d in range(self.dim)]
        ke = 0.5 * sum(m[d] * u[d] for d in range(self.dim))
        p = (g - 1.0) * (E - ke)
        if self.check:
            if bool((rho <= 0).any()) or bool((p <= 0).any()):
                raise NonPhysical("rho <= 0 or p <= 0")
        a = torch.sqrt(g * p / rho)
        return dict(rho=rho, u=u, p=p, a=a, E=E, m=m)

    def flux(self, U, l, P):
        """Physical flux in Cartesian direction l, stacked over variables."""
        u_l = P["u"][l]
        rows = [P["m"][l]]
        for d in range(self.dim):
            rows.append(P["m"][d] * u_l + (P["p"] if d == l else 0.0))
        rows.append((P["E"] + P["p"]) * u_l)
        return torch.stack(rows, dim=1)

    def speed(self, P, l):
        """|u_l| + a (unit normal along e_l)."""
        u = P["u"][l]
        return torch.where(u >= 0, u, -u) + P["a"]


class ReactingEuler:
    """Multi-species Euler with one temperature (reading above)."""

    def __init__(self, dim, mech, check=True):
        self.dim = dim
        self.mech = mech
        self.ns = mech["ns"]
        self.nv = self.ns + dim + 1
        self.check = check

    def temperature(self, rhos, ke, E):
        mech = self.mech
        cvsum = sum(rhos[s] * mech["cv"][s] for s in range(self.ns))
        h0sum = sum(rhos[s] * mech["h0"][s] for s in range(self.ns))
        return (E - ke - h0sum) / cvsum

    def prims(self, U):
        mech = self.mech
        ns = self.ns
        rhos = [U[:, s] for s in range(ns)]
        rho = sum(rhos)
        m = [U[:, ns + d] for d in range(self.dim)]
        E = U[:, ns + self.dim]
        u = [m[d] / rho for d in range(self.dim)]
        ke = 0.5 * sum(m[d] * u[d] for d in range(self.dim))
        T = self.temperature(rhos, ke, E)
        Rmix = sum(rhos[s] * mech["R"][s] for s in range(ns))
        cvmix = sum(rhos[s] * mech["cv"][s] for s in range(ns))
        p = T * Rmix
        if self.check:
            if bool((rho <= 0).any()) or bool((T <= 0).any()) or bool((p <= 0).any()):
                raise NonPhysical("rho <= 0, T <= 0 or p <= 0")
        gam = 1.0 + Rmix / cvmix
        a = torch.sqrt(gam * p / rho)
        return dict(rho=rho, rhos=rhos, u=u, p=p, a=a, E=E, m=m, T=T)

    def flux(self, U, l, P):
        u_l = P["u"][l]
        rows = [P["rhos"][s] * u_l for s in range(self.ns)]
        for d in range(self.dim):
            rows.append(P["m"][d] * u_l + (P["p"] if d == l else 0.0))
        rows.append((P["E"] + P["p"]) * u_l)
        return torch.stack(rows, dim=1)

    def speed(self, P, l):
        u = P["u"][l]
        return torch.where(u >= 0, u, -u) + P["a"]


def viscous_flux(dim, P, S, l, mu, gamma, prandtl):
    """Viscous flux in Cartesian direction l (rows 0, tau_l., u.tau_l. - q_l).

    S[q][d] is d W_q / d x_d for W = (rho, u, v[, w], T).
    """
    k = gamma * mu / (prandtl * (gamma - 1.0))
    du = [[S[1 + i][j] for j in range(dim)] for i in range(dim)]  # du_i/dx_j
    div = sum(du[i][i] for i in range(dim))
    tau_l = []
    for d in range(dim):
        t = mu * (du[l][d] + du[d][l])
        if d == l:
            t = t - (2.0 / 3.0) * mu * div
        tau_l.append(t)
    zero = torch.zeros_like(P["rho"])
    energy = sum(P["u"][d] * tau_l[d] for d in range(dim)) + k * S[dim + 1][l]
    return torch.stack([zero] + tau_l + [energy], dim=1)
