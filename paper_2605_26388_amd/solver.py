"""Thin Python binding over libdg: argument marshalling only.

Tensors are torch device tensors in the library's layout [B][nv][E][Np]
(structure of arrays, node index i fastest); every call passes raw device
pointers and torch's current HIP stream to the C ABI of include/dg.h.
"""

import ctypes

import numpy as np
import torch

from . import _abi
from ._abi import check

PHYSICS = {"euler": _abi.DG_EULER, "navier_stokes": _abi.DG_NAVIER_STOKES, "reacting": _abi.DG_REACTING_EULER,
           "reacting_2t": _abi.DG_REACTING_2T}
PRECISION = {"f64": _abi.DG_F64, "f32": _abi.DG_F32}
VOLUME = {"standard": _abi.DG_VOLUME_STANDARD, "split": _abi.DG_VOLUME_SPLIT}
BC = {"periodic": _abi.DG_BC_PERIODIC, "wall": _abi.DG_BC_WALL, "inflow": _abi.DG_BC_INFLOW,
      "outflow": _abi.DG_BC_OUTFLOW}


def mechanism_struct(mech):
    """dg_mechanism from a mechanism dict (see dginputs.air5_mechanism)."""
    m = _abi.Mechanism()
    ns, nr = int(mech["ns"]), int(mech["nr"])
    m.nspecies, m.nreactions = ns, nr
    for s in range(ns):
        m.W[s], m.R[s], m.cv[s], m.h0[s] = (float(mech[k][s]) for k in ("W", "R", "cv", "h0"))
    for r in range(nr):
        for s in range(ns):
            m.nu_f[r][s] = int(mech["nu_f"][r][s])
            m.nu_b[r][s] = int(mech["nu_b"][r][s])
            m.eff[r][s] = float(mech["eff"][r][s])
        for k in ("A_f", "beta_f", "theta_f", "A_b", "beta_b", "theta_b"):
            getattr(m, k)[r] = float(mech[k][r])
        m.third_body[r] = int(mech["third_body"][r])
        m.reversible[r] = int(mech["reversible"][r])
    m.kappa_c = float(mech["kappa_c"])
    m.kappa_r = float(mech["kappa_r"])
    return m


def vibration_struct(vib):
    """dg_vibration from a vibrational-data dict (see dginputs.air5_vibration)."""
    v = _abi.Vibration()
    for s, th in enumerate(vib["theta_v"]):
        v.theta_v[s] = float(th)
    for s, row in enumerate(vib["mw_a"]):
        for r, a in enumerate(row):
            v.mw_a[s][r] = float(a)
            v.mw_b[s][r] = float(vib["mw_b"][s][r])
    v.park_sigma = float(vib["park_sigma"])
    for r, f in enumerate(vib["two_temp"]):
        v.two_temp[r] = int(f)
    return v


def _stream(device):
    return ctypes.c_void_p(torch.cuda.current_stream(device).cuda_stream)


class Solver:
    """One libdg context: a mesh, a physics, a precision and a batch size."""

    def __init__(self, dim, degree, nel, lo, hi, physics="euler", precision="f64", batch=1,
                 patch_lo=None, patch_hi=None, gamma=1.4, mu=0.0, prandtl=0.72, mech=None,
                 newton_max_iter=25, newton_tol=1e-13, device=0, volume="standard", rho_floor=0.0, p_floor=0.0,
                 vib=None, warp=0.0, bc=None, bc_state=None):
        self.lib = _abi.load()
        d = _abi.Desc()
        d.dim, d.degree = int(dim), int(degree)
        d.physics = PHYSICS[physics]
        d.precision = PRECISION[precision]
        d.batch = int(batch)
        for l in range(3):
            d.nel[l] = int(nel[l]) if l < dim else 1
            d.lo[l] = float(lo[l]) if l < dim else 0.0
            d.hi[l] = float(hi[l]) if l < dim else 1.0
        if patch_lo is not None:
            for l in range(2):
                d.patch_lo[l], d.patch_hi[l] = int(patch_lo[l]), int(patch_hi[l])
        d.gamma, d.mu, d.prandtl = float(gamma), float(mu), float(prandtl)
        self._mech = mechanism_struct(mech) if mech is not None else None
        d.mech = ctypes.pointer(self._mech) if self._mech is not None else None
        d.newton_max_iter, d.newton_tol = int(newton_max_iter), float(newton_tol)
        d.device = int(device)
        d.volume = VOLUME[volume]
        d.rho_floor, d.p_floor = float(rho_floor), float(p_floor)
        self._vib = vibration_struct(vib) if vib is not None else None
        d.vib = ctypes.pointer(self._vib) if self._vib is not None else None
        d.warp = float(warp)
        for q, kind in enumerate(bc or ()):
            d.bc[q] = BC[kind] if isinstance(kind, str) else int(kind)
        for q, val in enumerate(bc_state if bc_state is not None else ()):
            d.bc_state[q] = float(val)
        self.device = torch.device("cuda", int(device))
        self.dim, self.N, self.batch = int(dim), int(degree), int(batch)
        self.physics, self.precision, self.volume = physics, precision, volume
        self.dtype = torch.float64 if precision == "f64" else torch.float32
        ctx = ctypes.c_void_p()
        check(self.lib.dg_create(ctypes.byref(d), ctypes.byref(ctx)), "dg_create")
        self._ctx = ctx
        E, Np, nv = ctypes.c_int64(), ctypes.c_int32(), ctypes.c_int32()
        check(self.lib.dg_sizes(ctx, ctypes.byref(E), ctypes.byref(Np), ctypes.byref(nv)), "dg_sizes")
        self.E, self.Np, self.nv = E.value, Np.value, nv.value
        self.shape = (self.batch, self.nv, self.E, self.Np)
        self._numel = self.batch * self.nv * self.E * self.Np

    # -- helpers ---------------------------------------------------------------
    def close(self):
        if getattr(self, "_ctx", None):
            self.lib.dg_destroy(self._ctx)
            self._ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def empty(self):
        return torch.empty(self.shape, dtype=self.dtype, device=self.device)

    def _ptr(self, t, name):
        if t is None:
            return None
        if not isinstance(t, torch.Tensor) or t.device != self.device:
            raise ValueError(f"{name}: expected a tensor on {self.device}")
        if t.dtype != self.dtype or not t.is_contiguous() or t.numel() != self._numel:
            raise ValueError(f"{name}: expected a contiguous {self.dtype} tensor of shape {self.shape}")
        return ctypes.c_void_p(t.data_ptr())

    # -- the C ABI -------------------------------------------------------------
    def node_coords(self):
        xyz = torch.empty((self.dim, self.E, self.Np), dtype=torch.float64, device=self.device)
        check(self.lib.dg_node_coords(self._ctx, ctypes.c_void_p(xyz.data_ptr()), _stream(self.device)),
              "dg_node_coords")
        return xyz

    def rhs(self, U, out=None):
        out = self.empty() if out is None else out
        check(self.lib.dg_rhs(self._ctx, self._ptr(U, "U"), self._ptr(out, "dUdt"), _stream(self.device)), "dg_rhs")
        return out

    def rk_stage(self, U0, Uk, out, a, b, c_dt):
        check(self.lib.dg_rk_stage(self._ctx, self._ptr(U0, "U0") if a != 0.0 else None, self._ptr(Uk, "Uk"),
                                   self._ptr(out, "Uout"), float(a), float(b), float(c_dt), _stream(self.device)),
              "dg_rk_stage")
        return out

    def rk_stage_dual(self, U0, Uk, out, a, b, c_dt, V, out2, a2, b2, c2_dt):
        check(self.lib.dg_rk_stage_dual(self._ctx, self._ptr(U0, "U0") if a != 0.0 else None, self._ptr(Uk, "Uk"),
                                        self._ptr(out, "Uout"), float(a), float(b), float(c_dt),
                                        self._ptr(V, "V") if a2 != 0.0 else None, self._ptr(out2, "Wout"),
                                        float(a2), float(b2), float(c2_dt), _stream(self.device)),
              "dg_rk_stage_dual")
        return out, out2

    def ssprk54_step(self, U, dt, tmp1=None, tmp2=None, tmp3=None):
        """One SSPRK54 step in place on U (three scratch states; tmp3 holds
        U^(4) afterwards)."""
        t1 = self.empty() if tmp1 is None else tmp1
        t2 = self.empty() if tmp2 is None else tmp2
        t3 = self.empty() if tmp3 is None else tmp3
        check(self.lib.dg_ssprk54_step(self._ctx, self._ptr(U, "U"), float(dt), self._ptr(t1, "t1"),
                                       self._ptr(t2, "t2"), self._ptr(t3, "t3"), _stream(self.device)),
              "dg_ssprk54_step")
        return U

    def source_chem(self, U, out, h, mode):
        check(self.lib.dg_source_chem(self._ctx, self._ptr(U, "U"), self._ptr(out, "out"), float(h), int(mode),
                                      _stream(self.device)), "dg_source_chem")
        return out

    def rhs_adjoint(self, U, lam_L, out=None):
        out = self.empty() if out is None else out
        check(self.lib.dg_rhs_adjoint(self._ctx, self._ptr(U, "U"), self._ptr(lam_L, "lam_L"),
                                      self._ptr(out, "lam_U"), _stream(self.device)), "dg_rhs_adjoint")
        return out

    LAM0_ACCUMULATE, LAM0_FOLD, LAM0_INIT = 0, 1, 2

    def rk_stage_adjoint(self, Uk, lam_out, lam_k, lam_0, a, b, c_dt, lam0_mode=0):
        check(self.lib.dg_rk_stage_adjoint(self._ctx, self._ptr(Uk, "Uk"), self._ptr(lam_out, "lam_out"),
                                           self._ptr(lam_k, "lam_k"), self._ptr(lam_0, "lam_0"), float(a),
                                           float(b), float(c_dt), int(lam0_mode), _stream(self.device)),
              "dg_rk_stage_adjoint")
        return lam_k

    def ssprk3_step_adjoint(self, states, dt, lam, lam_prev, acc, mu2, mu1):
        """Reverse sweep of one SSP-RK3 step with stored stage states
        (U^n, U1, U2): lam_prev = (dU^{n+1}/dU^n)^T lam.  Three library calls;
        acc, mu2 and mu1 are scratch states."""
        Un, U1, U2 = states
        self.rk_stage_adjoint(U2, lam, mu2, acc, 1.0 / 3.0, 2.0 / 3.0, 2.0 / 3.0 * dt, self.LAM0_INIT)
        self.rk_stage_adjoint(U1, mu2, mu1, acc, 0.75, 0.25, 0.25 * dt, self.LAM0_ACCUMULATE)
        self.rk_stage_adjoint(Un, mu1, lam_prev, acc, 0.0, 1.0, dt, self.LAM0_FOLD)
        return lam_prev

    def dt_cfl(self, U, cfl):
        dt = ctypes.c_double()
        check(self.lib.dg_dt_cfl(self._ctx, self._ptr(U, "U"), float(cfl), ctypes.byref(dt), _stream(self.device)),
              "dg_dt_cfl")
        return dt.value

    def integrals(self, U):
        out = (ctypes.c_double * (self.batch * (self.nv + 1)))()
        check(self.lib.dg_integrals(self._ctx, self._ptr(U, "U"), out, _stream(self.device)), "dg_integrals")
        return np.array(out[:]).reshape(self.batch, self.nv + 1)

    def integrals_noalloc(self, U, out):
        """dg_integrals_noalloc: integrals into the device tensor `out`
        (float64, [batch, nv + 1]) on the current stream, no host copy."""
        if out.dtype != torch.float64 or out.device != self.device or not out.is_contiguous() \
                or out.numel() != self.batch * (self.nv + 1):
            raise ValueError("out must be a contiguous float64 device tensor of batch * (nv + 1) values")
        check(self.lib.dg_integrals_noalloc(self._ctx, self._ptr(U, "U"), ctypes.c_void_p(out.data_ptr()),
                                            _stream(self.device)), "dg_integrals_noalloc")
        return out

    def status(self, reset=False):
        c = _abi.Counters()
        check(self.lib.dg_status_read(self._ctx, ctypes.byref(c), int(bool(reset)), _stream(self.device)),
              "dg_status_read")
        return dict(nonphysical=c.nonphysical, newton_unconverged=c.newton_unconverged,
                    species_clips=c.species_clips, newton_iters_max=c.newton_iters_max, first_bad=c.first_bad,
                    floored=c.floored)

    # -- composite drivers (sequences of library calls) ------------------------
    def ssprk3_step(self, U, dt, tmp1=None, tmp2=None):
        """One Shu-Osher SSP-RK3 step, in place on U (two scratch states, which
        hold the stage states U1 and U2 afterwards)."""
        t1 = self.empty() if tmp1 is None else tmp1
        t2 = self.empty() if tmp2 is None else tmp2
        self.rk_stage(None, U, t1, 0.0, 1.0, dt)
        self.rk_stage(U, t1, t2, 0.75, 0.25, 0.25 * dt)
        self.rk_stage(U, t2, U, 1.0 / 3.0, 2.0 / 3.0, 2.0 / 3.0 * dt)
        return U

    def strang_step(self, U, dt, tmp1=None, tmp2=None, tmp3=None, transport="ssprk3"):
        """S_{dt/2} o T_dt o S_{dt/2}: implicit source half steps around one
        transport step (eq. strang_split), in place on U.  transport is
        "ssprk3" (three Shu-Osher stages; scratch tmp1, tmp2) or "ssprk54"
        (the paper's five-stage method; scratch tmp1, tmp2, tmp3)."""
        self.source_chem(U, U, 0.5 * dt, 1)
        if transport == "ssprk54":
            self.ssprk54_step(U, dt, tmp1, tmp2, tmp3)
        elif transport == "ssprk3":
            self.ssprk3_step(U, dt, tmp1, tmp2)
        else:
            raise ValueError(f"unknown transport step {transport!r}")
        self.source_chem(U, U, 0.5 * dt, 1)
        return U
