"""Finite-rate chemistry source and its implicit substep (Kernel Architecture
for Source Terms; finite-rate appendix).

Per node, with concentrations [X_s] = kappa_c rho_s / W_s:
  k_f,r = A_r T^beta_r exp(-Theta_r / T)           (modified Arrhenius; one T)
  k_b,r = same form with the backward triple         (reading of the curve-fit
                                                      equilibrium constant:
                                                      K_c = k_f / k_b)
  R_r   = [M]_r (k_f prod [X]^nu' - k_b prod [X]^nu'')   (eq. src_reaction_rate;
          [M]_r = sum_s eff_rs [X_s] for third-body reactions, else 1)
  wdot_s = kappa_r W_s sum_r (nu''_sr - nu'_sr) R_r      (eq. src_omega)
The source vector (eq. src_vector) has wdot_s in the species rows and zero in
momentum and total energy (single temperature: no E_v row).

Implicit substep (eq. source_residual): Newton on
  R(Y*) = Y* - Y^n - h S_Y(Y*),  Y = (rho_1..rho_Ns), momentum and E fixed,
T recovered from the closure at every evaluation.  Jacobian column k by a
one-sided difference with eps_k = max(1e-7 |Y_k|, 1e-12) (the paper's rule);
linear update by Gauss-Jordan elimination.  Readings where the paper is silent:
start at Y* = Y^n; partial pivoting; the step is halved while the clipped
update would move T outside [T/2, 2T]; after each update clip rho_s >= 0 (and
count the clips); converged when a full (undamped) step has max_k |dY_k| <=
tol rho.

Globalisation (reading): where h |dS/dY| is very large (dense gas, fast
backward rates) Newton from Y^n can be drawn to a spurious corner -- a species
driven to zero with a residual of order h |S| -- instead of the root.  A node
not converged after max_iter iterations restarts from Y^n and follows the
root along the substep length: the same Newton iteration solves the residual
with h_j = h 2^-j for j = levels, .., 1, 0, each level starting from the
previous level's result.  For small h_j the root is next to Y^n, and halving
factors keep every level's start within reach of its root; the last level is
the residual of the requested h.  Non-convergence is flagged only if that last
level does not converge.
"""

import math

import numpy as np
import torch

from .physics import NonPhysical


def temperature(mech, rhos, ke, E):
    ns = mech["ns"]
    cv = sum(rhos[s] * mech["cv"][s] for s in range(ns))
    h0 = sum(rhos[s] * mech["h0"][s] for s in range(ns))
    return (E - ke - h0) / cv


def wdot(mech, rhos, T):
    """Species production rates (list over s) at temperature T."""
    ns, nr = mech["ns"], mech["nr"]
    X = [mech["kappa_c"] * rhos[s] / mech["W"][s] for s in range(ns)]
    out = [torch.zeros_like(T) for _ in range(ns)]
    for r in range(nr):
        kf = mech["A_f"][r] * T ** mech["beta_f"][r] * torch.exp(-mech["theta_f"][r] / T)
        fwd = kf
        for s in range(ns):
            for _ in range(int(mech["nu_f"][r][s])):
                fwd = fwd * X[s]
        if mech["reversible"][r]:
            kb = mech["A_b"][r] * T ** mech["beta_b"][r] * torch.exp(-mech["theta_b"][r] / T)
            bwd = kb
            for s in range(ns):
                for _ in range(int(mech["nu_b"][r][s])):
                    bwd = bwd * X[s]
        else:
            bwd = torch.zeros_like(T)
        if mech["third_body"][r]:
            M = sum(mech["eff"][r][s] * X[s] for s in range(ns))
        else:
            M = 1.0
        Rr = M * (fwd - bwd)
        for s in range(ns):
            dnu = int(mech["nu_b"][r][s]) - int(mech["nu_f"][r][s])
            if dnu != 0:
                out[s] = out[s] + mech["kappa_r"] * mech["W"][s] * dnu * Rr
    return out


def split_state(mech, dim, U):
    ns = mech["ns"]
    rhos = [U[:, s] for s in range(ns)]
    m = [U[:, ns + d] for d in range(dim)]
    E = U[:, ns + dim]
    return rhos, m, E


def source(mech, dim, U):
    """S(U) for the reacting Euler state (species rows only non-zero)."""
    rhos, m, E = split_state(mech, dim, U)
    rho = sum(rhos)
    ke = 0.5 * sum(mm * mm for mm in m) / rho
    T = temperature(mech, rhos, ke, E)
    if bool((T <= 0).any()):
        raise NonPhysical("T <= 0")
    w = wdot(mech, rhos, T)
    S = torch.zeros_like(U)
    for s in range(mech["ns"]):
        S[:, s] = w[s]
    return S


def _residual(mech, Y, Yn, h, ke, E):
    """R(Y) = Y - Y^n - h S_Y(Y) for node-batched Y (ns, P)."""
    rhos = [Y[s] for s in range(Y.shape[0])]
    T = temperature(mech, rhos, ke, E)
    w = wdot(mech, rhos, T)
    return torch.stack([Y[s] - Yn[s] - h * w[s] for s in range(Y.shape[0])]), T


def gauss_jordan(A, b):
    """Solve A x = b for a batch of small systems, A: (P, n, n), b: (P, n).
    Gauss-Jordan elimination with partial pivoting (row swaps)."""
    A = A.clone()
    b = b.clone()
    P, n, _ = A.shape
    ar = torch.arange(P)
    for k in range(n):
        piv = k + torch.argmax(A[:, k:, k].abs(), dim=1)
        # swap rows k and piv
        rowk = A[ar, k].clone()
        A[ar, k] = A[ar, piv]
        A[ar, piv] = rowk
        bk = b[ar, k].clone()
        b[ar, k] = b[ar, piv]
        b[ar, piv] = bk
        pivval = A[:, k, k].clone()
        A[:, k] = A[:, k] / pivval[:, None]
        b[:, k] = b[:, k] / pivval
        for i in range(n):
            if i == k:
                continue
            f = A[:, i, k].clone()
            A[:, i] = A[:, i] - f[:, None] * A[:, k]
            b[:, i] = b[:, i] - f * b[:, k]
    return b


def _newton(mech, Y, Yn, h, ke, E, rho, max_iter, tol, max_halvings, stats):
    """The Newton iteration on the residual of step length h for the nodes
    (columns) of Y, from Y; returns (Y, converged mask, iterations)."""
    ns = Y.shape[0]
    Y = Y.clone()
    P = Y.shape[1]
    active = torch.ones(P, dtype=torch.bool)
    conv = torch.zeros(P, dtype=torch.bool)
    iters = torch.zeros(P, dtype=torch.int64)
    for it in range(max_iter):
        if not bool(active.any()):
            break
        idx = active.nonzero().squeeze(1)
        Ya, Yna, kea, Ea = Y[:, idx], Yn[:, idx], ke[idx], E[idx]
        R0, T0 = _residual(mech, Ya, Yna, h, kea, Ea)
        if bool((T0 <= 0).any()):
            raise NonPhysical("T <= 0 inside the implicit substep")
        Jm = torch.zeros(len(idx), ns, ns, dtype=torch.float64)
        for k in range(ns):
            eps = torch.maximum(1e-7 * Ya[k].abs(), torch.full_like(Ya[k], 1e-12))
            Yp = Ya.clone()
            Yp[k] = Yp[k] + eps
            Rk, _ = _residual(mech, Yp, Yna, h, kea, Ea)
            Jm[:, :, k] = ((Rk - R0) / eps).T
        dY = gauss_jordan(Jm, -R0.T).T
        # temperature trust region: halve the step until the clipped update
        # keeps T within a factor 2 of the current iterate's T
        alpha = torch.ones(len(idx), dtype=torch.float64)
        for _ in range(max_halvings):
            Ytry = torch.clamp(Ya + alpha * dY, min=0.0)
            Tt = temperature(mech, [Ytry[s] for s in range(ns)], kea, Ea)
            bad = (Tt < 0.5 * T0) | (Tt > 2.0 * T0)
            if not bool(bad.any()):
                break
            alpha = torch.where(bad, 0.5 * alpha, alpha)
        full = alpha == 1.0
        dY = alpha * dY
        Ynew = Ya + dY
        neg = Ynew < 0
        stats["clips"] += int(neg.sum())
        Ynew = torch.where(neg, torch.zeros_like(Ynew), Ynew)
        Y[:, idx] = Ynew
        iters[idx] += 1
        done = full & (dY.abs().max(dim=0).values <= tol * rho[idx])
        active[idx[done]] = False
        conv[idx[done]] = True
    return Y, conv, iters


def implicit_substep(mech, dim, U, h, max_iter=25, tol=1e-13, max_halvings=30, levels=40):
    """One backward-Euler substep of length h on the species densities.

    Returns (U_new, stats) with stats = dict(iters, unconverged, clips,
    continued): iters counts every Newton iteration of a node (all levels),
    continued the nodes that took the continuation in h.  Momentum and total
    energy are copied unchanged.
    """
    ns = mech["ns"]
    shape = U.shape
    # flatten nodes: (ns, P)
    rhos, m, E = split_state(mech, dim, U)
    Yn = torch.stack([r.reshape(-1) for r in rhos])
    mflat = [mm.reshape(-1) for mm in m]
    Ef = E.reshape(-1)
    rho = Yn.sum(dim=0)
    ke = 0.5 * sum(mm * mm for mm in mflat) / rho
    stats = {"clips": 0}
    Y, conv, iters = _newton(mech, Yn, Yn, h, ke, Ef, rho, max_iter, tol, max_halvings, stats)
    cont = (~conv).nonzero().squeeze(1)
    if len(cont) > 0:
        Yc, Ync, kec, Ec, rhoc = Yn[:, cont].clone(), Yn[:, cont], ke[cont], Ef[cont], rho[cont]
        cc = torch.zeros(len(cont), dtype=torch.bool)
        for j in range(levels, -1, -1):
            Yc, cc, ic = _newton(mech, Yc, Ync, h * 2.0 ** (-j), kec, Ec, rhoc, max_iter, tol, max_halvings, stats)
            iters[cont] += ic
        Y[:, cont] = Yc
        conv[cont] = cc
    out = U.clone()
    for s in range(ns):
        out[:, s] = Y[s].reshape(shape[0], *shape[2:])
    return out, dict(iters=iters, unconverged=int((~conv).sum()), clips=stats["clips"], continued=len(cont))
