/*
 * dg.h -- C ABI of the MI355X DGSEM right-hand-side library (libdg.so).
 *
 * The library evaluates the semi-discrete operator dU/dt = L(U) of a nodal
 * discontinuous Galerkin spectral element method (tensor-product
 * Gauss-Lobatto-Legendre collocation) on periodic Cartesian meshes and on
 * warped (curvilinear) meshes with boundary fluxes, fuses it into the
 * Shu-Osher Runge-Kutta stage (also SSPRK54 with a per-stage positivity
 * floor), supplies the finite-rate chemistry source (one or two temperatures)
 * and its implicit substep, and the discrete adjoint of L and of the stage.
 * The operations follow the paper (MARUT, arXiv 2605.26388):
 *   - the semi-discrete system and the SSP-RK stage: SSP-RK Time
 *     Discretization appendix;
 *   - the volume integral and surface lift: eqs. vol_weak and surf_int of the
 *     Kernel Architecture for Hyperbolic Terms section, with the Rusanov flux
 *     of its Surface Fluxes paragraph and 2:1 mortars; the entropy-conservative
 *     split form eq. vol_split with Ranocha's flux; curvilinear metrics and
 *     boundary fluxes of the same section;
 *   - BR1 viscous terms: eqs. br1_avg, tau and br1_flux (Parabolic Terms);
 *   - the source and its implicit substep: eqs. src_reaction_rate, src_omega,
 *     strang_split and source_residual (Source Terms), with the two-temperature
 *     terms of eq. src_landau_teller (Thermochemical non-equilibrium).
 *
 * Conventions shared by every call
 *   Layout.  Every state-like buffer (U, dUdt, adjoint variables) is
 *     structure-of-arrays  X[b][v][e][k][j][i]  (i fastest): batch member b,
 *     conserved variable v, element e, node (k, j, i).  Element order: coarse
 *     cells lexicographically (x fastest); a 2:1-refined cell contributes its
 *     four children (0,0), (1,0), (0,1), (1,1) in place.  dtype is the
 *     context's precision: double (DG_F64) or float (DG_F32).
 *   Variables.  Euler / Navier-Stokes: (rho, rho u, rho v[, rho w], E).
 *     Reacting Euler (2-D): (rho_1..rho_Ns, rho u, rho v, E), and E_v last
 *     with two temperatures.
 *   Ownership.  State buffers are device memory owned by the caller; the
 *     library neither frees nor retains them past the call.  The context owns
 *     its tables, constants, scratch and status counters, so a context serves
 *     one stream at a time; calls that overlap on one context race.
 *   Streams.  `stream` is a hipStream_t passed as void* (NULL = default
 *     stream).  Compute calls are asynchronous on that stream; calls marked
 *     "synchronises" wait for the stream before returning.
 *   Errors.  Argument errors (null pointers, unsupported dim/degree/physics,
 *     forbidden aliasing) are returned synchronously before any launch as
 *     DG_ERR_ARG or DG_ERR_UNSUPPORTED; a failed launch returns DG_ERR_HIP.
 *     Device-side numerical faults (non-physical state, Newton failure,
 *     species clipping) and positivity-floor activity never abort a launch:
 *     they are sticky counters read by dg_status_read.  dg_last_error() describes the last failure of the
 *     calling thread.
 */
#ifndef DG_H
#define DG_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define DG_MAX_SPECIES 8
#define DG_MAX_REACTIONS 8

enum dg_status {
  DG_OK = 0,
  DG_ERR_ARG = 1,
  DG_ERR_UNSUPPORTED = 2,
  DG_ERR_HIP = 3,
  DG_ERR_OOM = 4,
  DG_ERR_NONPHYSICAL = 5,
  DG_ERR_NEWTON = 6
};

/* DG_REACTING_EULER: one temperature, vibration frozen.
 * DG_REACTING_2T: translational-rotational T and vibrational T_v (Thermochemical
 *   non-equilibrium section): the state gains E_v (last variable). */
enum dg_physics { DG_EULER = 0, DG_NAVIER_STOKES = 1, DG_REACTING_EULER = 2, DG_REACTING_2T = 3 };
/* DG_F64: state in double, every step in double.
 * DG_F32 (the FP32 form): state buffers in float.  Primitive recovery and its
 *   positivity checks, the physical and interface fluxes, the face corrections,
 *   the chemistry source and the reductions stay in double; the volume sweep
 *   operand (the element's fluxes less those of its first node), the
 *   accumulation of dU/dt and the stage combination are float.  The split form
 *   keeps its sweep, accumulation and stage combination in double in both. */
enum dg_precision { DG_F64 = 0, DG_F32 = 1 };

/* Volume integral of the inviscid flux.
 * DG_VOLUME_STANDARD: strong form of eq. vol_weak, sum_m D_im F_l(U_m).
 * DG_VOLUME_SPLIT: entropy-conservative split form (eq. vol_split, the
 *   appendix on the inviscid volume flux): 2 sum_m D_im F#_l(U_i, U_m) with
 *   Ranocha's kinetic-energy-preserving, entropy-conservative two-point flux
 *   in its published form (the energy row as printed in the paper is not
 *   entropy conservative), logarithmic means of rho and rho/p.  Euler and
 *   Navier-Stokes physics (with the BR1 viscous terms unchanged, the paper's
 *   Taylor-Green setting) on Cartesian meshes; the interface flux stays
 *   Rusanov; no adjoint. */
enum dg_volume { DG_VOLUME_STANDARD = 0, DG_VOLUME_SPLIT = 1 };

/* Box-side boundary types.  DG_BC_WALL: slip wall, the Rusanov flux against
 * the mirrored state (rho, m - 2 (m.n) n, E) (no mass or energy through it).
 * DG_BC_INFLOW: supersonic inflow, the exact flux of dg_desc.bc_state.
 * DG_BC_OUTFLOW: supersonic outflow, the exact flux of the interior state. */
enum dg_bc { DG_BC_PERIODIC = 0, DG_BC_WALL = 1, DG_BC_INFLOW = 2, DG_BC_OUTFLOW = 3 };

/* Reaction mechanism (Source Terms section; finite-rate appendix).
 * Species data per unit mass (SI); rate constants k = A T^beta exp(-Theta/T)
 * in the units implied by kappa_c: concentrations [X_s] = kappa_c rho_s/W_s,
 * molar rates converted back by kappa_r.  nu_f / nu_b are the reactant /
 * product stoichiometric coefficients; third_body[r] != 0 multiplies the
 * net rate by [M] = sum_s eff[r][s] [X_s]; reversible[r] == 0 drops the
 * backward rate.  The struct is copied by dg_create. */
typedef struct dg_mechanism {
  int32_t nspecies, nreactions;
  double W[DG_MAX_SPECIES];   /* molar mass, kg/mol */
  double R[DG_MAX_SPECIES];   /* specific gas constant, J/(kg K) */
  double cv[DG_MAX_SPECIES];  /* translational-rotational cv, J/(kg K) */
  double h0[DG_MAX_SPECIES];  /* formation enthalpy, J/kg */
  int32_t nu_f[DG_MAX_REACTIONS][DG_MAX_SPECIES];
  int32_t nu_b[DG_MAX_REACTIONS][DG_MAX_SPECIES];
  double A_f[DG_MAX_REACTIONS], beta_f[DG_MAX_REACTIONS], theta_f[DG_MAX_REACTIONS];
  double A_b[DG_MAX_REACTIONS], beta_b[DG_MAX_REACTIONS], theta_b[DG_MAX_REACTIONS];
  int32_t third_body[DG_MAX_REACTIONS];
  int32_t reversible[DG_MAX_REACTIONS];
  double eff[DG_MAX_REACTIONS][DG_MAX_SPECIES];
  double kappa_c, kappa_r;
} dg_mechanism;

/* Vibrational data of the two-temperature model (Thermochemical
 * non-equilibrium section; eq. src_landau_teller).  Harmonic oscillator
 * e_v,s(T) = R_s theta_v[s] / (exp(theta_v[s]/T) - 1); theta_v = 0 marks a
 * species without a vibrational mode.  Relaxation time of molecule s:
 * tau_s = tau_MW + tau_P with the Millikan-White mixture time
 * 1 / tau_MW = (p / 1 atm) sum_r x_r exp(-(mw_a[s][r] (T^(-1/3) - mw_b[s][r]) - 18.42))
 * (x_r molar fractions) and Park's correction tau_P = 1 / (sigma_v cbar_s n),
 * sigma_v = park_sigma (50000 K / T)^2, cbar_s = sqrt(8 R_u T / (pi W_s)),
 * n = p / (k_B T).  two_temp[r] != 0: reaction r takes its forward and
 * backward rates at T_a = sqrt(T T_v) (dissociation), else at T.  The
 * struct is copied by dg_create. */
typedef struct dg_vibration {
  double theta_v[DG_MAX_SPECIES];                 /* K */
  double mw_a[DG_MAX_SPECIES][DG_MAX_SPECIES];    /* K^(1/3) */
  double mw_b[DG_MAX_SPECIES][DG_MAX_SPECIES];
  double park_sigma;                              /* m^2 */
  int32_t two_temp[DG_MAX_REACTIONS];
} dg_vibration;

/* Problem description.  Periodic box [lo, hi] with nel cells per direction;
 * 2-D only: the coarse block [patch_lo, patch_hi) is refined once (2:1),
 * coupled through mortars (empty when patch_lo == patch_hi).
 * Supported: dim 2 or 3; degree 1..7 (Euler), 2..4 (Navier-Stokes, 3-D),
 * 3 (reacting, 2-D, up to DG_MAX_SPECIES species); batch >= 1.
 * Navier-Stokes uses constant mu, non-dimensional R = 1 (T = p/rho) and
 * k = gamma mu / (Pr (gamma - 1)).  Reacting Euler reads mech (copied); the
 * two-temperature physics also reads vib (copied). */
typedef struct dg_desc {
  int32_t dim, degree, physics, precision, batch;
  int32_t nel[3];
  double lo[3], hi[3];
  int32_t patch_lo[2], patch_hi[2];
  double gamma, mu, prandtl;
  const dg_mechanism* mech;
  int32_t newton_max_iter; /* implicit source substep, default 25 if <= 0 */
  double newton_tol;       /* stop when max |dY| <= tol * rho, default 1e-13 */
  int32_t device;          /* HIP device ordinal the context lives on */
  int32_t volume;          /* dg_volume; 0 (standard) when zero-initialised */
  /* Per-stage positivity floor (the paper's rho >= rho_min, p >= p_min after
   * every stage): applied node by node to the stage output of dg_rk_stage and
   * to the first output of dg_rk_stage_dual, never to dg_rhs.  rho is
   * clipped to rho_floor with the momentum unchanged, then E is raised to
   * p_floor/(gamma-1) + |m|^2/(2 rho) where it lies below.  0 for both turns
   * it off; Euler and Navier-Stokes physics only. */
  double rho_floor, p_floor;
  const dg_vibration* vib; /* DG_REACTING_2T only; NULL otherwise */
  /* Curvilinear elements and boundary fluxes (Kernel Architecture for
   * Hyperbolic Terms: element map x = X(xi), per-node J and Ja^l with the
   * discrete GCL; boundary fluxes per type).  warp != 0 moves every node of
   * the box by the smooth map
   *   2-D: x~ = x + warp L_x sin(2 pi s_y),  y~ = y + warp L_y sin(2 pi s_x),
   *   3-D: x~_d = x_d + warp L_d sin(2 pi s_{d+1}) sin(2 pi s_{d+2}),
   * s_d = (x_d - lo_d)/L_d; the element geometry is the degree-N interpolant
   * of its nodes, metrics come from it (cross-product form in 2-D, conservative
   * curl form in 3-D).  bc[2l] / bc[2l+1] is the type of the lo / hi side of
   * direction l (dg_bc; both periodic or neither); bc_state is the conserved
   * state of inflow sides.  Curvilinear meshes (warp != 0 or a non-periodic
   * side): Euler physics, both volume integrals (the split form pairs the
   * two-point flux with the average of the two nodes' Ja^l), FP64 or FP32
   * state (the FP32 form computes in double), no refined patch, no adjoint;
   * the mesh must not fold (J > 0 at every node). */
  double warp;
  int32_t bc[6];
  double bc_state[5];
} dg_desc;

/* Sticky device-side counters (dg_status_read). */
typedef struct dg_counters {
  int32_t nonphysical;       /* nodes seen with rho <= 0, p <= 0 or T <= 0 */
  int32_t newton_unconverged;/* nodes whose implicit substep hit max_iter */
  int32_t species_clips;     /* species densities clipped at 0 in Newton */
  int32_t newton_iters_max;  /* largest iteration count of any node */
  int64_t first_bad;         /* flat (b*E + e)*Np + node of the first
                                non-physical node seen, -1 if none */
  int32_t floored;           /* stage outputs changed by the positivity floor */
} dg_counters;

typedef struct dg_ctx dg_ctx;

/* Build a context: mesh tables, reference-element constants, mortar
 * operators and mechanism on the device.  Synchronous; allocates.
 * Size limit: the kernels address one batch member's state (nvars * E * Np
 * values of the context precision) with 32-bit byte offsets, so that block
 * must stay below 4 GiB (3-D, N = 3, FP64: at most 1,677,721 elements per
 * member); larger meshes are rejected with DG_ERR_UNSUPPORTED, as are
 * element counts beyond the int32 range. */
int dg_create(const dg_desc* desc, dg_ctx** out);
int dg_destroy(dg_ctx* ctx);

/* Sizes of the context: elements, nodes per element, conserved variables. */
int dg_sizes(const dg_ctx* ctx, int64_t* nelem, int32_t* nodes_per_elem, int32_t* nvars);

/* Node coordinates as double, layout xyz[d][e][node] (device, caller-owned,
 * dim * E * Np doubles).  Asynchronous. */
int dg_node_coords(const dg_ctx* ctx, double* xyz, void* stream);

/* dUdt = L(U)  (SSP-RK appendix: the semi-discrete operator).  Volume
 * integral (vol_weak), Rusanov interface flux, 2:1 mortars, surface lift
 * and Jacobian scaling (surf_int); for Navier-Stokes also the BR1 viscous
 * terms.  U and dUdt: [B][nv][E][Np]; dUdt must not alias U. */
int dg_rhs(dg_ctx* ctx, const void* U, void* dUdt, void* stream);

/* Uout = a U0 + b Uk + c_dt L(Uk)  (Shu-Osher stage, SSP-RK appendix),
 * fused with the evaluation of L.  Uout must not alias Uk (neighbour reads);
 * Uout == U0 is allowed.  U0 is not read when a == 0. */
int dg_rk_stage(dg_ctx* ctx, const void* U0, const void* Uk, void* Uout,
                double a, double b, double c_dt, void* stream);

/* Two Shu-Osher combinations of one evaluation of L(U_k), for methods whose
 * later stage reuses L of an earlier one (SSP-RK appendix; SSPRK54 needs
 * L(U^(3)) in stages 4 and 5):
 *   Uout = a U0 + b Uk + c_dt L(Uk)    (positivity floor applied, if set)
 *   Wout = a2 V + b2 Uk + c2_dt L(Uk)  (no floor: a partial sum, not a stage)
 * Same layout and stream semantics as dg_rk_stage.  U0 may equal Uout and V
 * may equal Wout (in place); Uk must not alias either output, the outputs
 * must not overlap each other, and U0 (V) is not read when a (a2) is 0. */
int dg_rk_stage_dual(dg_ctx* ctx, const void* U0, const void* Uk, void* Uout, double a, double b, double c_dt,
                     const void* V, void* Wout, double a2, double b2, double c2_dt, void* stream);

/* One step of the five-stage, fourth-order SSP Runge-Kutta method of Spiteri
 * and Ruuth (SSP coefficient 1.508; SSP-RK appendix, Shu-Osher form with the
 * method's published coefficients), in place on U: U <- U^(5).  Five fused
 * stage launches; the fourth is the dual form (it also forms the part of
 * U^(5) that needs L(U^(3))).  t1, t2, t3 are caller-owned scratch states of
 * the state's size, distinct from U and from each other; afterwards t3 holds
 * U^(4).  The positivity floor, if set, applies to U^(1), ..., U^(5). */
int dg_ssprk54_step(dg_ctx* ctx, void* U, double dt, void* t1, void* t2, void* t3, void* stream);

/* Chemistry source (reacting Euler only; arithmetic in double always).
 * mode 0: out += S(U), S from eqs. src_reaction_rate / src_omega (species
 *         rows only; momentum and energy carry no source).  out may be U.
 * mode 1: out = U with the species densities advanced by one backward-Euler
 *         substep of length h (eq. source_residual): Newton with one-sided
 *         finite-difference Jacobian and Gauss-Jordan elimination per node;
 *         momentum and energy copied unchanged.  out may be U. */
int dg_source_chem(dg_ctx* ctx, const void* U, void* out, double h, int32_t mode, void* stream);

/* Discrete adjoint of L (Euler physics, conforming meshes):
 * lam_U = (dL/dU)^T lam_L evaluated at U, in gather form (no atomics).
 * Subgradient convention at kinks: d max(x,y) -> x when x >= y, d|x| -> +1
 * when x >= 0.  Supported degrees 1..4.  lam_U must not alias U or lam_L. */
int dg_rhs_adjoint(dg_ctx* ctx, const void* U, const void* lam_L, void* lam_U, void* stream);

/* Adjoint of the fused stage Uout = a U0 + b Uk + c_dt L(Uk) at Uk
 * (Euler physics, conforming meshes; same conventions as dg_rhs_adjoint):
 *   lam_k = b lam_out + c_dt (dL/dU(Uk))^T lam_out     (+ lam_0 for DG_LAM0_FOLD)
 * and, depending on lam0_mode,
 *   DG_LAM0_ACCUMULATE: lam_0 = lam_0 + a lam_out,
 *   DG_LAM0_INIT:       lam_0 = a lam_out (lam_0 not read),
 *   DG_LAM0_FOLD:       lam_0 is only read (folded into lam_k).
 * lam_0 may be NULL (then it is neither read nor written).  This is what the
 * reverse sweep of one Shu-Osher step needs: INIT for the last stage,
 * ACCUMULATE for the middle one, FOLD for the first.  lam_k must not alias
 * Uk, lam_out or lam_0; lam_0 must not alias lam_out or Uk. */
enum { DG_LAM0_ACCUMULATE = 0, DG_LAM0_FOLD = 1, DG_LAM0_INIT = 2 };
int dg_rk_stage_adjoint(dg_ctx* ctx, const void* Uk, const void* lam_out, void* lam_k,
                        void* lam_0, double a, double b, double c_dt, int32_t lam0_mode,
                        void* stream);

/* Largest stable time step from the CFL bounds (SSP-RK appendix):
 * dt = cfl * h_min / ((2N+1) max(|u| + a)), and for Navier-Stokes
 * min with cfl * h_min^2 / ((2N+1)^2 max(mu/rho, mu/(Pr rho))).  Reduction
 * in double over all batch members.  Synchronises. */
int dg_dt_cfl(dg_ctx* ctx, const void* U, double cfl, double* dt, void* stream);

/* Integrals in double: out[b*(nv+1) + v] = sum_e J_e sum_i w_i U_v,i and
 * out[b*(nv+1) + nv] = sum_e J_e sum_i w_i |m_i|^2/(2 rho_i) (kinetic
 * energy; total density for reacting flow).  Deterministic two-level tree.
 * out is host memory of B*(nv+1) doubles.  Synchronises. */
int dg_integrals(dg_ctx* ctx, const void* U, double* out, void* stream);

/* Allocation-free variant of dg_integrals, for callers that cannot allocate
 * device memory during the call (code under HIP graph capture, tight serving
 * loops, harnesses that forbid hipMalloc): the same kernels and the same sums
 * in the same order, with the partial sums kept in one fixed device array per
 * GPU (2 MiB, held until the process ends) instead of the context's scratch.
 * out is DEVICE memory of B*(nv+1) doubles, caller-owned, written
 * asynchronously on `stream` (the call neither copies to the host nor
 * synchronises) in the layout of dg_integrals.  Calls no allocating routine.
 * Every call on one GPU shares the fixed array: calls that overlap on one GPU
 * (from any context, stream or thread) race.  Returns DG_ERR_UNSUPPORTED when
 * batch * (nvars + 1) exceeds 512, DG_ERR_ARG for null pointers. */
int dg_integrals_noalloc(dg_ctx* ctx, const void* U, double* out, void* stream);

/* Read (and optionally reset) the sticky counters.  Synchronises. */
int dg_status_read(dg_ctx* ctx, dg_counters* out, int32_t reset, void* stream);

const char* dg_strerror(int code);
const char* dg_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* DG_H */
