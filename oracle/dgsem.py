"""The DGSEM semi-discrete operator L(U) on affine Cartesian elements.

Follows the paper's hyperbolic pipeline (Kernel Architecture for Hyperbolic
Terms) and parabolic pipeline (Kernel Architecture for Parabolic Terms):

* volume term, strong form (eq. vol_weak):
      R_i = -(1/J) sum_l sum_m D_im Ft^l_m,   Ft^l = Ja^l . F;
  the weak form with Dhat = -W^{-1} D^T W and an F*-only surface term is
  provided for the strong == weak check (the paper states they coincide on
  GLL nodes);
* interface flux: local Lax-Friedrichs (Rusanov) with the unnormalised
  contravariant normal Ja^l (Surface Fluxes paragraph).  Reading taken:
      F* = 1/2 (F_L + F_R).n - 1/2 lam (U_R - U_L),
      lam = max(|u_L.n| + a_L |n|, |u_R.n| + a_R |n|),
  with L the element on the -xi_l side; both elements use the same value
  (+ for L, - for R);
* surface integral and Jacobian rescale (eq. surf_int), with w the 1-D end
  weight normal to the face (reading: tangential weights cancel):
      dU_i = R_i - 1/(J w_end) sum_{f ni i} (F*_f - Ft^{l_f}_i) (n_ref)_f;
* 2:1 mortars (Surface Fluxes paragraph): coarse trace interpolated onto each
  mortar, Riemann flux with the fine face normal, fine side lifts it directly,
  coarse side lifts sum_k Pr_k (2 F*_k) (factor 2 = coarse/mortar face ratio);
* BR1 viscous terms (Parabolic Terms, eqs. br1_avg, tau, br1_flux, and the
  BR1 paragraphs of the strong-form appendix): gradient of W = (rho, u, v, w,
  T) with the central trace W^ = (W^- + W^+)/2, viscous flux from each side's
  own lifted gradient, central interface flux {{F_v}}, added with a + sign
  since div F_v sits on the right-hand side.

Layout: U has shape (B, nv, E, n, .., n) with node axes (k, j, i).
"""

import numpy as np
import torch

from .refelem import gll, mortar_matrices
from .physics import viscous_flux


def node_axis(dim, l):
    """Tensor axis of reference direction l in a (B, nv, E, k, j, i) array."""
    return 3 + (dim - 1 - l)


def dsweep(F, D, dim, l):
    """out[.., i, ..] = sum_m D[i, m] F[.., m, ..] along direction l."""
    ax = node_axis(dim, l)
    return torch.matmul(F.movedim(ax, -1), D.T).movedim(-1, ax)


def trace(X, dim, l, end):
    """Face trace of every element at index `end` along direction l."""
    return X.select(node_axis(dim, l), end)


class Operator:
    """L(U) for one mesh and one physics, float64 throughout."""

    def __init__(self, mesh, phys, viscous=None):
        self.mesh = mesh
        self.phys = phys
        self.dim = mesh.dim
        self.N = mesh.N
        self.n = mesh.N + 1
        xi, w, D = gll(mesh.N)
        self.xi = xi
        self.w = torch.tensor(w, dtype=torch.float64)
        self.D = torch.tensor(D, dtype=torch.float64)
        self.Dhat = torch.tensor(-np.diag(1.0 / w) @ D.T @ np.diag(w), dtype=torch.float64)
        E = mesh.E
        self.J = torch.tensor(mesh.jac(), dtype=torch.float64)
        self.h = torch.tensor(mesh.h, dtype=torch.float64)
        # |Ja^l| = 2 J / h_l per element
        self.Ja = [2.0 * self.J / self.h[:, l] for l in range(self.dim)]
        self.bshape = (1, 1, E) + (1,) * self.dim
        self.viscous = viscous  # dict(mu, prandtl, gamma) or None
        self.conf = [(torch.as_tensor(L), torch.as_tensor(R)) for (L, R) in mesh.conf]
        if mesh.mortars:
            Pf, Pr = mortar_matrices(mesh.N)
            self.Pf = [torch.tensor(P, dtype=torch.float64) for P in Pf]
            self.Pr = [torch.tensor(P, dtype=torch.float64) for P in Pr]
            groups = {}
            for rec in mesh.mortars:
                groups.setdefault((rec["l"], rec["side"]), []).append(rec)
            self.mortar_groups = []
            for (l, side), recs in sorted(groups.items()):
                c = torch.tensor([r["coarse"] for r in recs])
                f0 = torch.tensor([r["fine"][0] for r in recs])
                f1 = torch.tensor([r["fine"][1] for r in recs])
                self.mortar_groups.append((l, side, c, (f0, f1)))
            if viscous is not None:
                raise NotImplementedError("BR1 on non-conforming meshes is out of scope")

    # -- helpers ----------------------------------------------------------
    def per_elem(self, v):
        return v.reshape(self.bshape)

    def lift_into(self, shape, elems, val, l, end, like):
        """Zero tensor of `shape` with val/w_end placed at face `end` (dir l)
        of elements `elems`.  val: (B, nv, nf, rest...)."""
        ax = node_axis(self.dim, l)
        e = torch.zeros(self.n, dtype=torch.float64)
        e[end] = 1.0 / self.w[end]
        eshape = [1] * (3 + self.dim)
        eshape[ax] = self.n
        contrib = val.unsqueeze(ax) * e.reshape(eshape)
        out = torch.zeros(shape, dtype=torch.float64)
        return out.index_add(2, elems, contrib)

    def rusanov(self, UL, UR, PL, PR, l, nmag):
        """F*(U_L, U_R; n = nmag e_l), unnormalised normal (reading above)."""
        ph = self.phys
        FL = ph.flux(UL, l, PL)
        FR = ph.flux(UR, l, PR)
        cL = ph.speed(PL, l)
        cR = ph.speed(PR, l)
        lam = torch.where(cL >= cR, cL, cR)
        return 0.5 * nmag.unsqueeze(1) * (FL + FR) - 0.5 * (nmag * lam).unsqueeze(1) * (UR - UL)

    # -- inviscid part -----------------------------------------------------
    def rhs_inviscid(self, U, form="strong"):
        ph, dim, N = self.phys, self.dim, self.N
        P = ph.prims(U)
        F = [self.per_elem(self.Ja[l]) * ph.flux(U, l, P) for l in range(dim)]   # contravariant fluxes
        dU = self.volume_term(U, F, form)
        strong = 1.0 if form == "strong" else 0.0
        shape = U.shape
        # conforming interfaces
        for l in range(dim):
            L, R = self.conf[l]
            if len(L) == 0:
                continue
            UL = trace(U, dim, l, N)[:, :, L]
            UR = trace(U, dim, l, 0)[:, :, R]
            PL = ph.prims(UL)
            PR = ph.prims(UR)
            nmag = self.Ja[l][L].reshape((1, -1) + (1,) * (dim - 1))
            Fs = self.rusanov(UL, UR, PL, PR, l, nmag)
            FtL = trace(F[l], dim, l, N)[:, :, L]
            FtR = trace(F[l], dim, l, 0)[:, :, R]
            JL = self.J[L].reshape((1, 1, -1) + (1,) * (dim - 1))
            JR = self.J[R].reshape((1, 1, -1) + (1,) * (dim - 1))
            # L: upper face along l, outward reference normal +e_l
            dU = dU - self.lift_into(shape, L, (Fs - strong * FtL) / JL, l, N, U)
            # R: lower face along l, outward reference normal -e_l
            dU = dU + self.lift_into(shape, R, (Fs - strong * FtR) / JR, l, 0, U)
        # 2:1 mortars
        if self.mesh.mortars:
            dU = dU + self.mortar_terms(U, F, strong)
        return dU

    def volume_term(self, U, F, form):
        """-(1/J) sum_l D Ft^l (eq. vol_weak), or its weak-form counterpart."""
        J = self.per_elem(self.J)
        dU = torch.zeros_like(U)
        Dop = self.D if form == "strong" else self.Dhat
        for l in range(self.dim):
            dU = dU - dsweep(F[l], Dop, self.dim, l) / J
        return dU

    def mortar_terms(self, U, F, strong):
        """Contributions of all 2:1 non-conforming faces (2-D)."""
        ph, dim, N = self.phys, self.dim, self.N
        shape = U.shape
        out = torch.zeros(shape, dtype=torch.float64)
        for (l, side, c, fine) in self.mortar_groups:
            cend = N if side == 1 else 0      # coarse face index along l
            fend = 0 if side == 1 else N      # fine face index along l
            Uc = trace(U, dim, l, cend)[:, :, c]          # (B, nv, nm, n)
            Fc = trace(F[l], dim, l, cend)[:, :, c]
            Jc = self.J[c].reshape(1, 1, -1, 1)
            Fstar_c = torch.zeros_like(Uc)
            for k in range(2):
                fk = fine[k]
                Uf = trace(U, dim, l, fend)[:, :, fk]
                Ff = trace(F[l], dim, l, fend)[:, :, fk]
                Jf = self.J[fk].reshape(1, 1, -1, 1)
                Uck = torch.einsum("ij,bvej->bvei", self.Pf[k], Uc)
                Pck = ph.prims(Uck)
                Pfk = ph.prims(Uf)
                nmag = self.Ja[l][fk].reshape(1, -1, 1)
                if side == 1:   # coarse on the -l side of the face
                    Fs = self.rusanov(Uck, Uf, Pck, Pfk, l, nmag)
                else:
                    Fs = self.rusanov(Uf, Uck, Pfk, Pck, l, nmag)
                # fine element lifts the mortar flux directly
                if side == 1:   # fine is R (its lower face)
                    out = out + self.lift_into(shape, fk, (Fs - strong * Ff) / Jf, l, fend, U)
                else:           # fine is L (its upper face)
                    out = out - self.lift_into(shape, fk, (Fs - strong * Ff) / Jf, l, fend, U)
                Fstar_c = Fstar_c + torch.einsum("ij,bvej->bvei", self.Pr[k], 2.0 * Fs)
            if side == 1:       # coarse is L (upper face)
                out = out - self.lift_into(shape, c, (Fstar_c - strong * Fc) / Jc, l, cend, U)
            else:
                out = out + self.lift_into(shape, c, (Fstar_c - strong * Fc) / Jc, l, cend, U)
        return out

    # -- viscous part (BR1) --------------------------------------------------
    def br1_gradient(self, W):
        """S[q][d] = d W_q / d x_d by the BR1 strong-form lifted gradient.

        W: (B, nq, E, nodes).  Cartesian affine map: only reference direction d
        contributes to the x_d derivative (Ja^l parallel to e_l).
        """
        dim, N = self.dim, self.N
        shape = W.shape
        J = self.per_elem(self.J)
        Sd = []
        for l in range(dim):
            G = dsweep(W, self.D, dim, l)
            L, R = self.conf[l]
            WL = trace(W, dim, l, N)[:, :, L]
            WR = trace(W, dim, l, 0)[:, :, R]
            What = 0.5 * (WL + WR)
            G = G + self.lift_into(shape, L, What - WL, l, N, W)
            G = G - self.lift_into(shape, R, What - WR, l, 0, W)
            Sd.append(self.per_elem(self.Ja[l]) / J * G)
        return [[Sd[d][:, q] for d in range(dim)] for q in range(shape[1])]

    def rhs_viscous(self, U):
        vis = self.viscous
        ph, dim, N = self.phys, self.dim, self.N
        P = ph.prims(U)
        T = P["p"] / P["rho"]       # R = 1
        W = torch.stack([P["rho"]] + P["u"] + [T], dim=1)
        S = self.br1_gradient(W)
        J = self.per_elem(self.J)
        shape = U.shape
        dU = torch.zeros_like(U)
        for l in range(dim):
            Fv = self.per_elem(self.Ja[l]) * viscous_flux(dim, P, S, l, vis["mu"], vis["gamma"], vis["prandtl"])
            dU = dU + dsweep(Fv, self.D, dim, l) / J
            L, R = self.conf[l]
            FL = trace(Fv, dim, l, N)[:, :, L]
            FR = trace(Fv, dim, l, 0)[:, :, R]
            Fs = 0.5 * (FL + FR)
            JL = self.J[L].reshape((1, 1, -1) + (1,) * (dim - 1))
            JR = self.J[R].reshape((1, 1, -1) + (1,) * (dim - 1))
            dU = dU + self.lift_into(shape, L, (Fs - FL) / JL, l, N, U)
            dU = dU - self.lift_into(shape, R, (Fs - FR) / JR, l, 0, U)
        return dU

    # -- public ----------------------------------------------------------------
    def rhs(self, U, form="strong"):
        dU = self.rhs_inviscid(U, form)
        if self.viscous is not None:
            dU = dU + self.rhs_viscous(U)
        return dU

    def lam_max(self, U):
        """max over nodes of |u| + a (C-R6 reading of lambda_max)."""
        P = self.phys.prims(U)
        un = torch.sqrt(sum(P["u"][d] ** 2 for d in range(self.dim)))
        return float((un + P["a"]).max())


def to_logical(U, dim, n):
    """(B, nv, E, Np) flat node layout -> (B, nv, E, n, .., n) view."""
    return U.reshape(U.shape[:3] + (n,) * dim)


def to_flat(U):
    return U.reshape(U.shape[:3] + (-1,))
