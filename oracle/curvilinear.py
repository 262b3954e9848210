"""Curvilinear elements with per-node metrics and boundary fluxes for the
Euler equations (Kernel Architecture for Hyperbolic Terms: the element map
x = X(xi), its Jacobian J, the contravariant vectors Ja^l satisfying the
discrete GCL, contravariant fluxes Ja^l . F; boundary fluxes dispatched per
type) -- test infrastructure, as the rest of the oracle.

Mesh: the periodic Cartesian box of `cartesian_mesh` (its element order and
face pairs) with every node moved by the warp
    2-D:  x~ = x + A L_x sin(2 pi s_y),   y~ = y + A L_y sin(2 pi s_x),
    3-D:  x~_d = x_d + A L_d sin(2 pi s_{d+1}) sin(2 pi s_{d+2})  (indices mod 3),
with s_d = (x_d - lo_d) / L_d: smooth, and translation-compatible across the
box so that periodic faces still match.  The geometry of an element is the
degree-N interpolant of its node coordinates.

Metrics at each node, from the collocation derivative D applied to the node
coordinates X_d (so they are exact for the interpolant):
    2-D:  Ja^1 = ( dy/dxi_2, -dx/dxi_2),  Ja^2 = (-dy/dxi_1, dx/dxi_1);
    3-D:  conservative curl form (Kopriva's metric identities):
          (Ja^i)_n = -[curl_xi (X_l grad_xi X_m)]_i,  (n, m, l) cyclic,
          the product X_l grad X_m formed node by node before the curl;
    J = det(dX_d / dxi_m) node by node.
Both forms give sum_l d/dxi_l (Ja^l) = 0 exactly in the collocation
algebra (D's applied along different directions commute), so a constant state
stays constant.

Operator (strong form, eq. vol_weak and eq. surf_int with per-node metrics):
    J dU_i = -sum_l sum_m D_im Ft^l_m - (1/w_end) sum_faces s (F* - Ft^l(U_i)),
with Ft^l = Ja^l . F (Cartesian fluxes F_d), s = +1 on the +xi_l face and -1
on the -xi_l face, and F* the Rusanov flux for the unnormalised normal n =
Ja^l at the face node (each side uses its own node's Ja^l):
    F* = (F(U_L) + F(U_R)) . n / 2 - lam |n| (U_R - U_L) / 2,
    lam = max(|v_L . n^| + a_L, |v_R . n^| + a_R),  L on the -xi_l side.
Split form (volume="split", eq. vol_split on curvilinear elements): the
volume term becomes
    J dU_i = -sum_l sum_m 2 D_im F#(U_i, U_m) . {{Ja^l}}_im - (lift as above),
with Ranocha's two-point flux contracted with the average of the two nodes'
contravariant vectors, {{Ja^l}}_im = (Ja^l_i + Ja^l_m) / 2 (the form whose
conservation and entropy conservation rest on the discrete GCL above); the
surface term is unchanged (F* - Ft^l(U_i) at face nodes).  surface="ec" puts
the two-point flux itself at the interfaces, F#(U_L, U_R) . n with each side's
own n, for the entropy check.
BR1 viscous terms (viscous=dict(mu, prandtl, gamma); periodic meshes): the
gradient of W = (rho, u, v, w, T) by the strong-form operator of the
hyperbolic pipeline applied to the flux W e_d (reading of Parabolic Terms,
step 1: same structure as the hyperbolic surface pipeline, then rescaled by
1/J),
    J S_d = sum_l [ sum_m D_im (Ja^l_d W)_m + (+-1/w_end)(W^ - W_i) Ja^l_d,i ],
W^ = (W^- + W^+)/2 on the face (eq. br1_avg); the contravariant viscous
fluxes Fv~^l = Ja^l . F_v(U, S) (eq. tau, q = -k grad T), their strong-form
divergence and the central interface flux {{Fv~^l}} (eq. br1_flux), the
average of the two sides' own contravariant fluxes at the shared face node
(the two Ja^l agree there to rounding), added with a + sign.
Boundary faces (box sides that are not periodic), per type:
    wall     slip wall: ghost state with the normal velocity reversed,
             U_g = (rho, m - 2 (m . n^) n^, E), in the Rusanov flux (its mass
             and energy fluxes vanish, its momentum flux is normal);
    inflow   supersonic inflow: F* = F(U_bc) . n for a prescribed state;
    outflow  supersonic outflow: F* = F(U_i) . n (no correction).
"""

import math

import numpy as np
import torch

from .dgsem import dsweep, node_axis, trace
from .mesh import cartesian_mesh
from .physics import Euler, viscous_flux
from .refelem import gll
from .split import ranocha_flux_n as split_ranocha_n


def warp(X, lo, hi, A):
    """Warped copy of Cartesian coordinates X (dim, ...)."""
    dim = X.shape[0]
    L = [hi[d] - lo[d] for d in range(dim)]
    s = [(X[d] - lo[d]) / L[d] for d in range(dim)]
    out = np.empty_like(X)
    if dim == 2:
        out[0] = X[0] + A * L[0] * np.sin(2 * math.pi * s[1])
        out[1] = X[1] + A * L[1] * np.sin(2 * math.pi * s[0])
    else:
        for d in range(3):
            out[d] = X[d] + A * L[d] * np.sin(2 * math.pi * s[(d + 1) % 3]) * np.sin(2 * math.pi * s[(d + 2) % 3])
    return out


class CurvMesh:
    def __init__(self, dim, N, nel, lo, hi, A, bc=None):
        self.base = cartesian_mesh(dim, N, nel, lo, hi)
        self.dim, self.N, self.n = dim, N, N + 1
        self.lo, self.hi, self.nel, self.A = tuple(lo), tuple(hi), tuple(nel), A
        self.bc = tuple(bc) if bc is not None else ("periodic",) * (2 * dim)
        for l in range(dim):
            if (self.bc[2 * l] == "periodic") != (self.bc[2 * l + 1] == "periodic"):
                raise ValueError("a periodic direction needs both sides periodic")
        _, w, D = gll(N)
        self.D = torch.tensor(D)
        self.w = torch.tensor(w)
        X = warp(self.base.coords(), lo, hi, A)
        self.X = torch.tensor(X)                                        # (dim, E, n..n)
        # The metric terms are taken from coordinates relative to each
        # element's first node: D annihilates constants, and the curl of a
        # constant times a gradient vanishes (the tensor-product derivatives
        # of different directions commute), so the terms are unchanged in
        # exact arithmetic, while their rounding is relative to the element's
        # size instead of its distance from the origin.
        Xl = self.X - self.X.reshape(dim, self.base.E, -1)[:, :, :1].reshape((dim, self.base.E) + (1,) * dim)
        # dX[d][m] = d X_d / d xi_m at every node
        dX = [[dsweep(Xl[d][None, None], self.D, dim, m)[0, 0] for m in range(dim)] for d in range(dim)]
        if dim == 2:
            self.Ja = [torch.stack([dX[1][1], -dX[0][1]]), torch.stack([-dX[1][0], dX[0][0]])]
            self.J = dX[0][0] * dX[1][1] - dX[0][1] * dX[1][0]
        else:
            def dxi(f, m):
                return dsweep(f[None, None], self.D, 3, m)[0, 0]
            Ja = [[None] * 3 for _ in range(3)]
            for nn in range(3):
                mm, ll = (nn + 1) % 3, (nn + 2) % 3
                V = [Xl[ll] * dX[mm][k] for k in range(3)]             # X_l grad X_m
                for i in range(3):
                    curl_i = dxi(V[(i + 2) % 3], (i + 1) % 3) - dxi(V[(i + 1) % 3], (i + 2) % 3)
                    Ja[i][nn] = -curl_i
            self.Ja = [torch.stack(Ja[i]) for i in range(3)]
            M = [[dX[d][m] for m in range(3)] for d in range(3)]
            self.J = (M[0][0] * (M[1][1] * M[2][2] - M[1][2] * M[2][1])
                      - M[0][1] * (M[1][0] * M[2][2] - M[1][2] * M[2][0])
                      + M[0][2] * (M[1][0] * M[2][1] - M[1][1] * M[2][0]))
        # face pairs per direction, split into interior and boundary (the
        # wrap-around pairs of a non-periodic direction)
        cells = self._cell_index()
        self.pairs, self.bfaces = [], []
        for l in range(dim):
            Lr, Rr = self.base.conf[l]
            Lr, Rr = np.asarray(Lr), np.asarray(Rr)
            wrap = (cells[Lr, l] == nel[l] - 1) & (cells[Rr, l] == 0)
            if self.bc[2 * l] == "periodic":
                self.pairs.append((Lr, Rr))
                self.bfaces.append(None)
            else:
                self.pairs.append((Lr[~wrap], Rr[~wrap]))
                # (elements on the lo side of the box, elements on the hi side)
                self.bfaces.append((Rr[wrap], Lr[wrap]))

    def _cell_index(self):
        h0 = [(self.hi[d] - self.lo[d]) / self.nel[d] for d in range(self.dim)]
        c = np.rint((self.base.corner - np.array(self.lo)) / np.array(h0)).astype(np.int64)
        return c

    def coords(self):
        return self.X.numpy()

    def hmin(self):
        return self.base.hmin()


class CurvOperator:
    """L(U) for the Euler equations on a CurvMesh (strong form); bc_state is
    the prescribed conserved state of inflow sides."""

    def __init__(self, mesh, gamma=1.4, bc_state=None, volume="standard", surface="rusanov", viscous=None):
        if volume not in ("standard", "split") or surface not in ("rusanov", "ec"):
            raise ValueError((volume, surface))
        if viscous is not None and any(b != "periodic" for b in mesh.bc):
            raise ValueError("viscous terms on curvilinear meshes: periodic sides only")
        self.mesh = mesh
        self.phys = Euler(mesh.dim, gamma)
        self.dim, self.N, self.n = mesh.dim, mesh.N, mesh.n
        self.bc_state = None if bc_state is None else torch.tensor(bc_state, dtype=torch.float64)
        self.volume, self.surface = volume, surface
        self.viscous = viscous  # dict(mu, prandtl, gamma) or None

    def br1_gradient(self, W):
        """S[q][d] = d W_q / d x_d (W: (B, nq, E, nodes)), the strong-form
        lifted gradient with per-node metrics."""
        m, dim, N = self.mesh, self.dim, self.N
        winv = 1.0 / float(m.w[0])
        Sd = []
        for d in range(dim):
            G = torch.zeros_like(W)
            for l in range(dim):
                ax = node_axis(dim, l)
                Jd = m.Ja[l][d][None, None]
                G = G + dsweep(Jd * W, m.D, dim, l)
                Lr, Rr = (torch.as_tensor(a) for a in m.pairs[l])
                WL = trace(W[:, :, Lr], dim, l, N)
                WR = trace(W[:, :, Rr], dim, l, 0)
                What = 0.5 * (WL + WR)
                nL = trace(Jd[:, :, Lr], dim, l, N)
                nR = trace(Jd[:, :, Rr], dim, l, 0)
                G[:, :, Lr] = _add_face(G[:, :, Lr], winv * (What - WL) * nL, dim, ax, N)
                G[:, :, Rr] = _add_face(G[:, :, Rr], -winv * (What - WR) * nR, dim, ax, 0)
            Sd.append(G / m.J[None, None])
        return [[Sd[d][:, q] for d in range(dim)] for q in range(W.shape[1])]

    def rhs_viscous(self, U):
        """(1/J) [sum_l D Fv~^l + lift of ({{Fv~^l}} - Fv~^l)] with Fv~^l = Ja^l . F_v."""
        m, ph, dim, N, vis = self.mesh, self.phys, self.dim, self.N, self.viscous
        P = ph.prims(U)
        W = torch.stack([P["rho"]] + P["u"] + [P["p"] / P["rho"]], dim=1)
        S = self.br1_gradient(W)
        Fv = [viscous_flux(dim, P, S, d, vis["mu"], vis["gamma"], vis["prandtl"]) for d in range(dim)]
        winv = 1.0 / float(m.w[0])
        dU = torch.zeros_like(U)
        for l in range(dim):
            ax = node_axis(dim, l)
            Ft = self._ft(Fv, m.Ja[l])
            dU = dU + dsweep(Ft, m.D, dim, l)
            Lr, Rr = (torch.as_tensor(a) for a in m.pairs[l])
            FL = trace(Ft[:, :, Lr], dim, l, N)
            FR = trace(Ft[:, :, Rr], dim, l, 0)
            Fs = 0.5 * (FL + FR)
            dU[:, :, Lr] = _add_face(dU[:, :, Lr], winv * (Fs - FL), dim, ax, N)
            dU[:, :, Rr] = _add_face(dU[:, :, Rr], -winv * (Fs - FR), dim, ax, 0)
        return dU / m.J[None, None]

    def split_volume(self, U):
        """-sum_l sum_m 2 D_im F#(U_i, U_m) . (Ja^l_i + Ja^l_m) / 2 (times J)."""
        m, dim = self.mesh, self.dim
        out = torch.zeros_like(U)
        for l in range(dim):
            ax = node_axis(dim, l)
            X = U.movedim(ax, -1)                                   # (B, nv, E, .., n) along l
            n = X.shape[-1]
            XL = X.unsqueeze(-1).expand(*X.shape, n)                # U_i at [.., i, m]
            XR = X.unsqueeze(-2).expand(*X.shape[:-1], n, n)        # U_m at [.., i, m]
            Ja = m.Ja[l].movedim(ax - 1, -1)                         # (dim, E, .., n)
            Jav = [0.5 * (Ja[d].unsqueeze(-1) + Ja[d].unsqueeze(-2)) for d in range(dim)]
            F = split_ranocha_n(XL, XR, Jav, self.phys.gamma)        # (B, nv, E, .., i, m)
            s = torch.einsum("...im,im->...i", F, m.D)
            out = out - 2.0 * s.movedim(-1, ax)
        return out

    def _ft(self, F, Ja):
        """Ja . F: F list over d of (B, nv, ...), Ja (dim, ...) -> (B, nv, ...)."""
        return sum(Ja[d][None, None] * F[d] for d in range(self.dim))

    def _rusanov(self, UL, UR, n):
        """F* . n for states (B, nv, ...) and unnormalised normal n (dim, ...)."""
        if self.surface == "ec":
            return split_ranocha_n(UL, UR, [n[d][None] for d in range(self.dim)], self.phys.gamma)
        ph = self.phys
        PL, PR = ph.prims(UL), ph.prims(UR)
        FL = [ph.flux(UL, d, PL) for d in range(self.dim)]
        FR = [ph.flux(UR, d, PR) for d in range(self.dim)]
        nmag = torch.sqrt(sum(n[d] * n[d] for d in range(self.dim)))
        vnL = sum(PL["u"][d] * n[d] for d in range(self.dim)) / nmag
        vnR = sum(PR["u"][d] * n[d] for d in range(self.dim)) / nmag
        lam = torch.maximum(vnL.abs() + PL["a"], vnR.abs() + PR["a"])
        return 0.5 * (self._ft(FL, n) + self._ft(FR, n)) - 0.5 * (lam * nmag)[:, None] * (UR - UL)

    def _boundary_flux(self, kind, Ui, n, own_is_left):
        ph = self.phys
        if kind == "outflow":
            P = ph.prims(Ui)
            return self._ft([ph.flux(Ui, d, P) for d in range(self.dim)], n)
        if kind == "inflow":
            Ub = self.bc_state.reshape((1, -1) + (1,) * (Ui.dim() - 2)).expand_as(Ui).clone()
            P = ph.prims(Ub)
            return self._ft([ph.flux(Ub, d, P) for d in range(self.dim)], n)
        if kind == "wall":
            nmag = torch.sqrt(sum(n[d] * n[d] for d in range(self.dim)))
            nh = [n[d] / nmag for d in range(self.dim)]
            mn = sum(Ui[:, 1 + d] * nh[d] for d in range(self.dim))
            Ug = Ui.clone()
            for d in range(self.dim):
                Ug[:, 1 + d] = Ui[:, 1 + d] - 2.0 * mn * nh[d]
            return self._rusanov(Ui, Ug, n) if own_is_left else self._rusanov(Ug, Ui, n)
        raise ValueError(kind)

    def rhs(self, U):
        m, ph, dim = self.mesh, self.phys, self.dim
        P = ph.prims(U)
        F = [ph.flux(U, d, P) for d in range(dim)]
        Ft = [self._ft(F, m.Ja[l]) for l in range(dim)]
        if self.volume == "split":
            dU = self.split_volume(U)
        else:
            dU = torch.zeros_like(U)
            for l in range(dim):
                dU = dU - dsweep(Ft[l], m.D, dim, l)
        winv = 1.0 / float(m.w[0])
        for l in range(dim):
            ax = node_axis(dim, l)
            Lr, Rr = m.pairs[l]
            Lr, Rr = torch.as_tensor(Lr), torch.as_tensor(Rr)
            if len(Lr):
                UL = trace(U[:, :, Lr], dim, l, m.N)
                UR = trace(U[:, :, Rr], dim, l, 0)
                nL = trace(m.Ja[l][:, Lr][None], dim, l, m.N)[0]
                nR = trace(m.Ja[l][:, Rr][None], dim, l, 0)[0]
                FsL = self._rusanov(UL, UR, nL)
                FsR = self._rusanov(UL, UR, nR)
                FoL = trace(Ft[l][:, :, Lr], dim, l, m.N)
                FoR = trace(Ft[l][:, :, Rr], dim, l, 0)
                dU[:, :, Lr] = _add_face(dU[:, :, Lr], -winv * (FsL - FoL), dim, ax, m.N)
                dU[:, :, Rr] = _add_face(dU[:, :, Rr], winv * (FsR - FoR), dim, ax, 0)
            if m.bfaces[l] is not None:
                lo_el, hi_el = (torch.as_tensor(a) for a in m.bfaces[l])
                # -xi_l faces of the elements on the lo side of the box
                Ui = trace(U[:, :, lo_el], dim, l, 0)
                n = trace(m.Ja[l][:, lo_el][None], dim, l, 0)[0]
                Fs = self._boundary_flux(m.bc[2 * l], Ui, n, own_is_left=False)
                Fo = trace(Ft[l][:, :, lo_el], dim, l, 0)
                dU[:, :, lo_el] = _add_face(dU[:, :, lo_el], winv * (Fs - Fo), dim, ax, 0)
                # +xi_l faces of the elements on the hi side
                Ui = trace(U[:, :, hi_el], dim, l, m.N)
                n = trace(m.Ja[l][:, hi_el][None], dim, l, m.N)[0]
                Fs = self._boundary_flux(m.bc[2 * l + 1], Ui, n, own_is_left=True)
                Fo = trace(Ft[l][:, :, hi_el], dim, l, m.N)
                dU[:, :, hi_el] = _add_face(dU[:, :, hi_el], -winv * (Fs - Fo), dim, ax, m.N)
        dU = dU / m.J[None, None]
        if self.viscous is not None:
            dU = dU + self.rhs_viscous(U)
        return dU

    def lam_max(self, U):
        P = self.phys.prims(U)
        return float((torch.sqrt(sum(u * u for u in P["u"])) + P["a"]).max())


def _add_face(X, val, dim, ax, end):
    """X (B, nv, E', n..n) with val added on the face slice index `end` of
    node axis `ax` (val: (B, nv, E', n..n without that axis))."""
    X = X.clone()
    idx = [slice(None)] * X.dim()
    idx[ax] = end
    X[tuple(idx)] = X[tuple(idx)] + val
    return X
