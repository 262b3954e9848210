"""Two-temperature thermochemical non-equilibrium (Thermochemical
non-equilibrium section; Kernel Architecture for Source Terms) -- test
infrastructure, as the rest of the oracle.

State U = (rho_1..rho_Ns, rho u_1..rho u_dim, E, E_v).  Closure (the paper's
energy decomposition with calorically perfect translation-rotation):
    E = sum_s rho_s (cv_s T + h0_s) + E_v + |m|^2 / (2 rho),   p = T sum_s rho_s R_s,
    E_v = sum_{s mol} rho_s e_v,s(T_v),   e_v,s(T) = R_s theta_s / (exp(theta_s / T) - 1)
(harmonic oscillator; species with theta_s = 0 have no vibrational mode).
The flux is that of the one-temperature model plus the column E_v u_l; the
sound speed is the frozen one, a^2 = (1 + sum rho_s R_s / sum rho_s cv_s) p / rho.

Source (eq. src_vector): wdot_s in the species rows (eqs. src_reaction_rate,
src_omega with each reaction's rates at its controlling temperature:
T_a = sqrt(T T_v) for the reactions flagged as dissociation, T otherwise;
forward and backward rates at the same T_a), zero in momentum and E, and
    Q_T-v + sum_{s mol} wdot_s e_v,s(T_v)
in the E_v row, with the Landau-Teller term (eq. src_landau_teller)
    Q_T-v = sum_{s mol} rho_s (e_v,s(T) - e_v,s(T_v)) / tau_s,
    tau_s = tau_MW,s + tau_P,s,
    tau_MW,s = sum_r x_r / sum_r (x_r / tau_sr),
    tau_sr = exp(A_sr (T^(-1/3) - B_sr) - 18.42) / (p / 101325)   [s]
(Millikan-White correlation, molar fractions x_r),
    tau_P,s = 1 / (sigma_v cbar_s n),  sigma_v = sigma' (50000 / T)^2,
    cbar_s = sqrt(8 R_u T / (pi W_s)),  n = p / (k_B T)
(Park's high-temperature limiting correction).

Implicit substep (eq. source_residual): Newton on
    R(Y*) = Y* - Y^n - h S_Y(Y*),  Y = (rho_1..rho_Ns, E_v),
momentum and E fixed, T and T_v recovered at every evaluation (Newton and
its globalisation: see implicit_substep).

T_v is recovered from E_v by bisection on a logarithmic bracket (e_v is
increasing in T_v), which needs no starting guess and ends at rounding.
"""

import math

import torch

from .chem import gauss_jordan
from .physics import NonPhysical

R_UNIVERSAL = 8.31446261815324      # J/(mol K)
K_BOLTZMANN = 1.380649e-23          # J/K
P_ATM = 101325.0                    # Pa


def e_vib(theta, R, T):
    """Harmonic-oscillator vibrational energy per unit mass at T."""
    if theta == 0.0:
        return torch.zeros_like(T)
    return R * theta / torch.expm1(theta / T)


def vib_energy(mech, vib, rhos, Tv):
    return sum(rhos[s] * e_vib(vib["theta_v"][s], mech["R"][s], Tv) for s in range(mech["ns"]))


def t_vib(mech, vib, rhos, Ev, lo=1.0, hi=1.0e6, iters=110):
    """T_v with vib_energy(T_v) = E_v, by bisection in ln T_v."""
    a = torch.full_like(Ev, math.log(lo))
    b = torch.full_like(Ev, math.log(hi))
    for _ in range(iters):
        mid = 0.5 * (a + b)
        f = vib_energy(mech, vib, rhos, torch.exp(mid)) - Ev
        a = torch.where(f < 0, mid, a)
        b = torch.where(f < 0, b, mid)
    return torch.exp(0.5 * (a + b))


class ReactingEuler2T:
    """Multi-species Euler with translational-rotational T and vibrational T_v."""

    def __init__(self, dim, mech, vib, check=True):
        self.dim = dim
        self.mech = mech
        self.vib = vib
        self.ns = mech["ns"]
        self.nv = self.ns + dim + 2
        self.check = check

    def split(self, U):
        ns, dim = self.ns, self.dim
        rhos = [U[:, s] for s in range(ns)]
        m = [U[:, ns + d] for d in range(dim)]
        return rhos, m, U[:, ns + dim], U[:, ns + dim + 1]

    def temperature(self, rhos, ke, E, Ev):
        mech = self.mech
        cvsum = sum(rhos[s] * mech["cv"][s] for s in range(self.ns))
        h0sum = sum(rhos[s] * mech["h0"][s] for s in range(self.ns))
        return (E - Ev - ke - h0sum) / cvsum

    def prims(self, U):
        mech = self.mech
        rhos, m, E, Ev = self.split(U)
        rho = sum(rhos)
        u = [m[d] / rho for d in range(self.dim)]
        ke = 0.5 * sum(m[d] * u[d] for d in range(self.dim))
        T = self.temperature(rhos, ke, E, Ev)
        Rmix = sum(rhos[s] * mech["R"][s] for s in range(self.ns))
        cvmix = sum(rhos[s] * mech["cv"][s] for s in range(self.ns))
        p = T * Rmix
        if self.check:
            if bool((rho <= 0).any()) or bool((T <= 0).any()) or bool((p <= 0).any()):
                raise NonPhysical("rho <= 0, T <= 0 or p <= 0")
        a = torch.sqrt((1.0 + Rmix / cvmix) * p / rho)
        return dict(rho=rho, rhos=rhos, u=u, p=p, a=a, E=E, Ev=Ev, m=m, T=T)

    def flux(self, U, l, P):
        u_l = P["u"][l]
        rows = [P["rhos"][s] * u_l for s in range(self.ns)]
        for d in range(self.dim):
            rows.append(P["m"][d] * u_l + (P["p"] if d == l else 0.0))
        rows.append((P["E"] + P["p"]) * u_l)
        rows.append(P["Ev"] * u_l)
        return torch.stack(rows, dim=1)

    def speed(self, P, l):
        u = P["u"][l]
        return torch.where(u >= 0, u, -u) + P["a"]


def wdot_2t(mech, vib, rhos, T, Tv):
    """Species production rates with each reaction's rates at its
    controlling temperature (sqrt(T T_v) where flagged, else T)."""
    ns, nr = mech["ns"], mech["nr"]
    X = [mech["kappa_c"] * rhos[s] / mech["W"][s] for s in range(ns)]
    out = [torch.zeros_like(T) for _ in range(ns)]
    Ta_diss = torch.sqrt(T * Tv)
    for r in range(nr):
        Ta = Ta_diss if vib["two_temp"][r] else T
        fwd = mech["A_f"][r] * Ta ** mech["beta_f"][r] * torch.exp(-mech["theta_f"][r] / Ta)
        for s in range(ns):
            for _ in range(int(mech["nu_f"][r][s])):
                fwd = fwd * X[s]
        bwd = torch.zeros_like(T)
        if mech["reversible"][r]:
            bwd = mech["A_b"][r] * Ta ** mech["beta_b"][r] * torch.exp(-mech["theta_b"][r] / Ta)
            for s in range(ns):
                for _ in range(int(mech["nu_b"][r][s])):
                    bwd = bwd * X[s]
        M = sum(mech["eff"][r][s] * X[s] for s in range(ns)) if mech["third_body"][r] else 1.0
        Rr = M * (fwd - bwd)
        for s in range(ns):
            dnu = int(mech["nu_b"][r][s]) - int(mech["nu_f"][r][s])
            if dnu != 0:
                out[s] = out[s] + mech["kappa_r"] * mech["W"][s] * dnu * Rr
    return out


def tau_vt(mech, vib, rhos, T, p):
    """Relaxation time tau_s of every species (0 where theta_s = 0)."""
    ns = mech["ns"]
    moles = [rhos[r] / mech["W"][r] for r in range(ns)]
    ntot = sum(moles)
    x = [moles[r] / ntot for r in range(ns)]
    patm = p / P_ATM
    n = p / (K_BOLTZMANN * T)
    sigma = vib["park_sigma"] * (50000.0 / T) ** 2
    out = []
    for s in range(ns):
        if vib["theta_v"][s] == 0.0:
            out.append(torch.zeros_like(T))
            continue
        inv = sum(x[r] / (torch.exp(vib["mw_a"][s][r] * (T ** (-1.0 / 3.0) - vib["mw_b"][s][r]) - 18.42) / patm)
                  for r in range(ns))
        tau_mw = 1.0 / inv                              # sum_r x_r = 1
        cbar = torch.sqrt(8.0 * R_UNIVERSAL * T / (math.pi * mech["W"][s]))
        out.append(tau_mw + 1.0 / (sigma * cbar * n))
    return out


def q_vt(mech, vib, rhos, T, Tv, p):
    """Landau-Teller term Q_T-v."""
    tau = tau_vt(mech, vib, rhos, T, p)
    q = torch.zeros_like(T)
    for s in range(mech["ns"]):
        th = vib["theta_v"][s]
        if th == 0.0:
            continue
        R = mech["R"][s]
        q = q + rhos[s] * (e_vib(th, R, T) - e_vib(th, R, Tv)) / tau[s]
    return q


def source_terms(mech, vib, rhos, T, Tv):
    """(wdot_s list, S_Ev) at given densities and temperatures."""
    p = T * sum(rhos[s] * mech["R"][s] for s in range(mech["ns"]))
    w = wdot_2t(mech, vib, rhos, T, Tv)
    sev = q_vt(mech, vib, rhos, T, Tv, p)
    for s in range(mech["ns"]):
        th = vib["theta_v"][s]
        if th != 0.0:
            sev = sev + w[s] * e_vib(th, mech["R"][s], Tv)
    return w, sev


def source(phys, U):
    """S(U) (eq. src_vector) for the two-temperature state."""
    mech, vib = phys.mech, phys.vib
    rhos, m, E, Ev = phys.split(U)
    rho = sum(rhos)
    ke = 0.5 * sum(mm * mm for mm in m) / rho
    T = phys.temperature(rhos, ke, E, Ev)
    if bool((T <= 0).any()) or bool((Ev < 0).any()):
        raise NonPhysical("T <= 0 or E_v < 0")
    Tv = t_vib(mech, vib, rhos, Ev)
    w, sev = source_terms(mech, vib, rhos, T, Tv)
    S = torch.zeros_like(U)
    for s in range(phys.ns):
        S[:, s] = w[s]
    S[:, -1] = sev
    return S


def implicit_substep(phys, U, h, max_iter=25, tol=1e-13, max_halvings=30):
    """One backward-Euler substep of length h on Y = (rho_s, E_v) at fixed
    momentum and E.  Returns (U_new, stats).

    Newton with the one-sided difference Jacobian and Gauss-Jordan (as the
    paper describes), globalised (reading; the exponential temperature
    dependence of the rates makes plain Newton steps cycle at some stiff
    nodes): the step length alpha is first halved while the clipped update
    would move T outside [T/2, 2T], then halved further until the scaled
    residual norm max_k |R_k| / scale_k decreases by the factor
    (1 - 1e-4 alpha) (at most max_halvings halvings each).  The residual of
    the accepted update is the next iteration's residual.  Converged when the
    undamped Newton step satisfies max_k |dY_k| / scale_k <= tol (it is then
    applied in full); scale = rho for the species and the thermal energy
    E - |m|^2/(2 rho) - sum rho_s h0_s for E_v.  rho_s and E_v are clipped at
    0 after every update (counted)."""
    mech, vib, ns = phys.mech, phys.vib, phys.ns
    nY = ns + 1
    shape = U.shape
    rhos, m, E, Ev = phys.split(U)
    Yn = torch.stack([r.reshape(-1) for r in rhos] + [Ev.reshape(-1)])
    Ef = E.reshape(-1)
    rho = Yn[:ns].sum(dim=0)
    ke = 0.5 * sum(mm.reshape(-1) ** 2 for mm in m) / rho
    h0sum = sum(Yn[s] * mech["h0"][s] for s in range(ns))
    scale = torch.cat([rho[None].expand(ns, -1), (Ef - ke - h0sum).abs()[None]])

    def temp(Y, kea, Ea):
        return phys.temperature([Y[s] for s in range(ns)], kea, Ea, Y[ns])

    def residual(Y, Yna, kea, Ea):
        T = temp(Y, kea, Ea)
        if bool((T <= 0).any()):
            raise NonPhysical("T <= 0 inside the implicit substep")
        Tv = t_vib(mech, vib, [Y[s] for s in range(ns)], Y[ns])
        w, sev = source_terms(mech, vib, [Y[s] for s in range(ns)], T, Tv)
        return Y - Yna - h * torch.stack(w + [sev]), T

    P = Yn.shape[1]
    Y = Yn.clone()
    R, T = residual(Y, Yn, ke, Ef)
    active = torch.ones(P, dtype=torch.bool)
    iters = torch.zeros(P, dtype=torch.int64)
    clips = 0
    for _ in range(max_iter):
        if not bool(active.any()):
            break
        idx = active.nonzero().squeeze(1)
        Ya, Yna, kea, Ea, sca = Y[:, idx], Yn[:, idx], ke[idx], Ef[idx], scale[:, idx]
        R0, T0 = R[:, idx], T[idx]
        Jm = torch.zeros(len(idx), nY, nY, dtype=torch.float64)
        for k in range(nY):
            eps = torch.maximum(1e-7 * Ya[k].abs(), torch.full_like(Ya[k], 1e-12))
            Yp = Ya.clone()
            Yp[k] = Yp[k] + eps
            Rk, _ = residual(Yp, Yna, kea, Ea)
            Jm[:, :, k] = ((Rk - R0) / eps).T
        dY = gauss_jordan(Jm, -R0.T).T
        done = (dY.abs() / sca).max(dim=0).values <= tol
        alpha = torch.ones(len(idx), dtype=torch.float64)
        for _ in range(max_halvings):
            Tt = temp(torch.clamp(Ya + alpha * dY, min=0.0), kea, Ea)
            bad = ~done & ((Tt < 0.5 * T0) | (Tt > 2.0 * T0))
            if not bool(bad.any()):
                break
            alpha = torch.where(bad, 0.5 * alpha, alpha)
        n0 = (R0.abs() / sca).max(dim=0).values
        for _ in range(max_halvings + 1):
            used = alpha
            Yt = torch.clamp(Ya + used * dY, min=0.0)
            Rt, Tt = residual(Yt, Yna, kea, Ea)
            bad = ~done & ((Rt.abs() / sca).max(dim=0).values > (1.0 - 1e-4 * used) * n0)
            if not bool(bad.any()):
                break
            alpha = torch.where(bad, 0.5 * alpha, alpha)
        clips += int((Ya + used * dY < 0).sum())
        Y[:, idx] = Yt
        R[:, idx] = Rt
        T[idx] = Tt
        iters[idx] += 1
        active[idx[done]] = False
    out = U.clone()
    for s in range(ns):
        out[:, s] = Y[s].reshape(shape[0], *shape[2:])
    out[:, -1] = Y[ns].reshape(shape[0], *shape[2:])
    return out, dict(iters=iters, unconverged=int(active.sum()), clips=clips)
