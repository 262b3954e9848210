// Finite-rate chemistry source (eqs. src_reaction_rate, src_omega) and its
// implicit backward-Euler substep (eq. source_residual), one lane per node,
// double precision throughout (also for float state buffers).
//
// Per node:  [X_s] = kappa_c rho_s / W_s,
//            k = A T^beta exp(-Theta/T) = A exp(beta ln T - Theta/T),
//            R_r = [M]_r (k_f prod [X]^nu' - k_b prod [X]^nu''),
//            wdot_s = kappa_r W_s sum_r (nu''_sr - nu'_sr) R_r,
// with T from the one-temperature closure at fixed momentum and energy.
//
// Implicit substep (Newton on Y* - Y^n - h wdot(Y*) = 0, Y = rho_s):
//   Jacobian column k by a one-sided difference with
//   eps_k = max(1e-7 |Y_k|, 1e-12); Gauss-Jordan elimination with partial
//   pivoting in registers; the step is halved while the clipped update would
//   move T outside [T/2, 2T] (temperature trust region, at most 30 halvings);
//   species are clipped at 0 after the update (counted); converged when a
//   full (undamped) step has max |dY| <= tol rho.  A node not converged after
//   max_iter iterations restarts from Y^n and follows the root along the
//   substep length: the same iteration on the residual of h 2^-j for
//   j = CONT_LEVELS, .., 1, 0, each level from the previous level's result
//   (where h |dS/dY| is huge, Newton from Y^n can otherwise be drawn to a
//   spurious corner with a species at zero); it counts as unconverged only if
//   the last level does not converge.  The state of a node never leaves
//   registers between evaluations; global traffic is one read and one write
//   of the state.  The substep runs in two passes: the first makes every
//   node's Newton iteration at h and hands the nodes that need the
//   continuation (a node index and its iteration count) to the second, which
//   runs each of them on a group of 32 lanes (k_source_cont below).
#include <algorithm>

#include "dg_device.hpp"

namespace dg {

// levels of the continuation in the substep length (h 2^-40 .. h)
constexpr int CONT_LEVELS = 40;

template <int NS, int NR>
struct Chem {
  const dg_mechanism* m;

  // temperature at species densities Y, fixed kinetic energy ke and energy E
  __device__ __forceinline__ double temperature(const double (&Y)[NS], double ke, double E) const {
    double cv = 0.0, h0 = 0.0;
#pragma unroll
    for (int s = 0; s < NS; ++s) {
      cv = fma(Y[s], m->cv[s], cv);
      h0 = fma(Y[s], m->h0[s], h0);
    }
    return (E - ke - h0) / cv;
  }

  __device__ __forceinline__ void wdot(const double (&Y)[NS], double T, double (&w)[NS]) const {
    double X[NS];
#pragma unroll
    for (int s = 0; s < NS; ++s) {
      X[s] = m->kappa_c * Y[s] / m->W[s];
      w[s] = 0.0;
    }
    const double lnT = log(T);
    const double Ti = 1.0 / T;
#pragma unroll
    for (int r = 0; r < NR; ++r) {
      double fwd = m->A_f[r] * exp(fma(m->beta_f[r], lnT, -m->theta_f[r] * Ti));
      double bwd = 0.0;
      for (int s = 0; s < NS; ++s)
        for (int q = 0; q < m->nu_f[r][s]; ++q) fwd *= X[s];
      if (m->reversible[r]) {
        bwd = m->A_b[r] * exp(fma(m->beta_b[r], lnT, -m->theta_b[r] * Ti));
        for (int s = 0; s < NS; ++s)
          for (int q = 0; q < m->nu_b[r][s]; ++q) bwd *= X[s];
      }
      double M = 1.0;
      if (m->third_body[r]) {
        M = 0.0;
#pragma unroll
        for (int s = 0; s < NS; ++s) M = fma(m->eff[r][s], X[s], M);
      }
      const double Rr = M * (fwd - bwd);
#pragma unroll
      for (int s = 0; s < NS; ++s) {
        const int dnu = m->nu_b[r][s] - m->nu_f[r][s];
        if (dnu != 0) w[s] = fma(m->kappa_r * m->W[s] * dnu, Rr, w[s]);
      }
    }
  }

  // net rate of reaction r alone, M_r (k_f prod X^nu' - k_b prod X^nu''), with
  // wdot's arithmetic term for term (wdot adds kappa_r W_s dnu_rs times it to
  // each species in the order r = 0, 1, ...)
  __device__ __forceinline__ double rate(int r, const double (&Y)[NS], double T) const {
    double X[NS];
#pragma unroll
    for (int s = 0; s < NS; ++s) X[s] = m->kappa_c * Y[s] / m->W[s];
    const double lnT = log(T);
    const double Ti = 1.0 / T;
    double fwd = m->A_f[r] * exp(fma(m->beta_f[r], lnT, -m->theta_f[r] * Ti));
    double bwd = 0.0;
    for (int s = 0; s < NS; ++s)
      for (int q = 0; q < m->nu_f[r][s]; ++q) fwd *= X[s];
    if (m->reversible[r]) {
      bwd = m->A_b[r] * exp(fma(m->beta_b[r], lnT, -m->theta_b[r] * Ti));
      for (int s = 0; s < NS; ++s)
        for (int q = 0; q < m->nu_b[r][s]; ++q) bwd *= X[s];
    }
    double M = 1.0;
    if (m->third_body[r]) {
      M = 0.0;
#pragma unroll
      for (int s = 0; s < NS; ++s) M = fma(m->eff[r][s], X[s], M);
    }
    return M * (fwd - bwd);
  }

  // R(Y) = Y - Yn - h wdot(Y, T(Y)); returns T(Y)
  __device__ __forceinline__ double residual(const double (&Y)[NS], const double (&Yn)[NS], double h, double ke,
                                             double E, double (&R)[NS]) const {
    const double T = temperature(Y, ke, E);
    double w[NS];
    wdot(Y, T, w);
#pragma unroll
    for (int s = 0; s < NS; ++s) R[s] = (Y[s] - Yn[s]) - h * w[s];
    return T;
  }
};

// Solve A x = b (n = NS) by Gauss-Jordan with partial pivoting; row swaps are
// done with selects so the matrix stays in registers.
template <int NS>
__device__ __forceinline__ void gauss_jordan(double (&A)[NS][NS], double (&b)[NS], double (&x)[NS]) {
#pragma unroll
  for (int k = 0; k < NS; ++k) {
    int p = k;
    double best = fabs(A[k][k]);
#pragma unroll
    for (int i = k + 1; i < NS; ++i) {
      const double a = fabs(A[i][k]);
      if (a > best) {
        best = a;
        p = i;
      }
    }
#pragma unroll
    for (int i = k + 1; i < NS; ++i) {
      const bool sw = (i == p);
#pragma unroll
      for (int j = 0; j < NS; ++j) {
        const double t = A[k][j];
        A[k][j] = sw ? A[i][j] : A[k][j];
        A[i][j] = sw ? t : A[i][j];
      }
      const double t = b[k];
      b[k] = sw ? b[i] : b[k];
      b[i] = sw ? t : b[i];
    }
    const double piv = A[k][k];
#pragma unroll
    for (int j = 0; j < NS; ++j) A[k][j] = A[k][j] / piv;
    b[k] = b[k] / piv;
#pragma unroll
    for (int i = 0; i < NS; ++i) {
      if (i == k) continue;
      const double f = A[i][k];
#pragma unroll
      for (int j = 0; j < NS; ++j) A[i][j] = A[i][j] - f * A[k][j];
      b[i] = b[i] - f * b[k];
    }
  }
#pragma unroll
  for (int i = 0; i < NS; ++i) x[i] = b[i];
}

// A node whose implicit substep takes the continuation in h, handed from the
// first pass to the second: its flat node index and the iterations spent.
struct DeferredNode {
  unsigned t;
  int it;
};

template <typename T, int NS, int NR, int DIM>
__global__ void __launch_bounds__(256)
k_source(const T* U, T* out, const dg_mechanism* mech, size_t plane, int B, double h, int mode, int max_iter,
         double tol, int* counters, unsigned long long* first_bad, DeferredNode* defer, int* defer_count) {
  constexpr int NV = NS + DIM + 1;
  const Chem<NS, NR> chem{mech};
  const size_t total = plane * B;
  for (size_t t = blockIdx.x * (size_t)blockDim.x + threadIdx.x; t < total; t += (size_t)gridDim.x * blockDim.x) {
    const size_t b = t / plane;
    const size_t r = t - b * plane;
    const size_t base = b * NV * plane + r;
    double Yn[NS], mom[DIM];
    double rho = 0.0;
#pragma unroll
    for (int s = 0; s < NS; ++s) {
      Yn[s] = static_cast<double>(U[base + s * plane]);
      rho += Yn[s];
    }
    double m2 = 0.0;
#pragma unroll
    for (int d = 0; d < DIM; ++d) {
      mom[d] = static_cast<double>(U[base + (NS + d) * plane]);
      m2 += mom[d] * mom[d];
    }
    const double E = static_cast<double>(U[base + (NS + DIM) * plane]);
    const double ke = 0.5 * m2 / rho;
    if (mode == 0) {
      const double Tn = chem.temperature(Yn, ke, E);
      if (!(Tn > 0.0)) report_nonphysical(counters, first_bad, t);
      double w[NS];
      chem.wdot(Yn, Tn, w);
#pragma unroll
      for (int s = 0; s < NS; ++s) {
        const double o = static_cast<double>(out[base + s * plane]);
        out[base + s * plane] = static_cast<T>(o + w[s]);
      }
      continue;
    }
    // ---- implicit substep ----------------------------------------------------
    double Y[NS];
#pragma unroll
    for (int s = 0; s < NS; ++s) Y[s] = Yn[s];
    int it = 0, clips = 0;
    bool nonphys = false;
    // Newton on the residual of step length hh from the current Y; returns
    // whether a full step met the tolerance within max_iter iterations
    auto newton = [&](double hh) -> bool {
      for (int k_it = 0; k_it < max_iter; ++k_it) {
        double R0[NS];
        const double T0 = chem.residual(Y, Yn, hh, ke, E, R0);
        if (!(T0 > 0.0)) {
          nonphys = true;
          return false;
        }
        ++it;
        double J[NS][NS];
#pragma unroll
        for (int k = 0; k < NS; ++k) {
          const double eps = fmax(1e-7 * fabs(Y[k]), 1e-12);
          double Yp[NS], Rk[NS];
#pragma unroll
          for (int s = 0; s < NS; ++s) Yp[s] = Y[s];
          Yp[k] = Yp[k] + eps;
          chem.residual(Yp, Yn, hh, ke, E, Rk);
#pragma unroll
          for (int s = 0; s < NS; ++s) J[s][k] = (Rk[s] - R0[s]) / eps;
        }
        double rhs[NS], dY[NS];
#pragma unroll
        for (int s = 0; s < NS; ++s) rhs[s] = -R0[s];
        gauss_jordan<NS>(J, rhs, dY);
        double alpha = 1.0;
        for (int hv = 0; hv < 30; ++hv) {
          double Yt[NS];
#pragma unroll
          for (int s = 0; s < NS; ++s) Yt[s] = fmax(Y[s] + alpha * dY[s], 0.0);
          const double Tt = chem.temperature(Yt, ke, E);
          if (!(Tt < 0.5 * T0) && !(Tt > 2.0 * T0)) break;
          alpha *= 0.5;
        }
        double dmax = 0.0;
#pragma unroll
        for (int s = 0; s < NS; ++s) {
          dY[s] = alpha * dY[s];
          double y = Y[s] + dY[s];
          if (y < 0.0) {
            ++clips;
            y = 0.0;
          }
          Y[s] = y;
          dmax = fmax(dmax, fabs(dY[s]));
        }
        if (alpha == 1.0 && dmax <= tol * rho) return true;
      }
      return false;
    };
    bool converged = newton(h);
    if (!converged && !nonphys && defer) {
      // the continuation runs in the second pass, on a group of lanes: hand
      // the node over with its iteration count (its species are written there)
      defer[atomicAdd(defer_count, 1)] = DeferredNode{static_cast<unsigned>(t), it};
      if (clips) atomicAdd(&counters[CNT_CLIPS], clips);
      if (out != U) {
#pragma unroll
        for (int d = 0; d < DIM; ++d) out[base + (NS + d) * plane] = static_cast<T>(mom[d]);
        out[base + (NS + DIM) * plane] = static_cast<T>(E);
      }
      continue;
    }
    if (!converged && !nonphys) {
#pragma unroll
      for (int s = 0; s < NS; ++s) Y[s] = Yn[s];
      for (int j = CONT_LEVELS; j >= 0 && !nonphys; --j) converged = newton(ldexp(h, -j));
    }
    if (nonphys) report_nonphysical(counters, first_bad, t);
    if (!converged) atomicAdd(&counters[CNT_NEWTON], 1);
    if (clips) atomicAdd(&counters[CNT_CLIPS], clips);
    atomicMax(&counters[CNT_ITERS], it);
#pragma unroll
    for (int s = 0; s < NS; ++s) out[base + s * plane] = static_cast<T>(Y[s]);
    if (out != U) {
#pragma unroll
      for (int d = 0; d < DIM; ++d) out[base + (NS + d) * plane] = static_cast<T>(mom[d]);
      out[base + (NS + DIM) * plane] = static_cast<T>(E);
    }
  }
}

// ---------------------------------------------------------------------------
// Second pass of the implicit substep: the continuation in h of the nodes the
// first pass handed over, one node per group of G = 32 lanes.  In each Newton
// iteration the six residual evaluations (the base point, the point displaced
// along Y_k for each k) run side by side, each spread over NR lanes, one per
// reaction: lane p NR + r evaluates reaction r's two Arrhenius rates at point
// p (p = NS the base point; lanes past NS NR + NR - 1 repeat the base point),
// the point's NR rates are gathered by lane shuffles and summed into the
// species rates in the order r = 0, 1, .. of the one-lane evaluation.  Every
// lane of the group then forms the same difference Jacobian and solves the
// same system, so the iterates are those of the one-lane iteration bit for
// bit, while an iteration takes about one reaction's latency (two
// exponentials) instead of six evaluations of NR reactions each.  The few nodes that need the
// continuation (a few per cent at the surveyed stiffness, up to 40 levels of
// Newton solves) otherwise keep their whole wave waiting.
// ---------------------------------------------------------------------------
template <typename T, int NS, int NR, int DIM>
__global__ void __launch_bounds__(256)
k_source_cont(const T* U, T* out, const dg_mechanism* mech, size_t plane, double h, int max_iter, double tol,
              int* counters, unsigned long long* first_bad, const DeferredNode* defer, const int* defer_count) {
  constexpr int G = 32, NV = NS + DIM + 1;
  static_assert((NS + 1) * NR <= G, "one lane per reaction of each Jacobian column and of the base point");
  const Chem<NS, NR> chem{mech};
  const int lane = threadIdx.x & (G - 1);
  const int pt = lane / NR < NS ? lane / NR : NS;  // this lane's point: displaced along Y_pt, or the base point
  const int rl = lane - (lane / NR) * NR;          // and its reaction
  const int pbase = pt * NR;                       // lane of reaction 0 of the point
  const int count = *defer_count;
  const int groups = (int)(((size_t)gridDim.x * blockDim.x) / G);
  for (int g = (int)((blockIdx.x * (size_t)blockDim.x + threadIdx.x) / G); g < count; g += groups) {
    const DeferredNode dn = defer[g];
    const size_t t = dn.t;
    const size_t b = t / plane;
    const size_t r = t - b * plane;
    const size_t base = b * NV * plane + r;
    double Yn[NS];
    double rho = 0.0;
#pragma unroll
    for (int s = 0; s < NS; ++s) {
      Yn[s] = static_cast<double>(U[base + s * plane]);
      rho += Yn[s];
    }
    double m2 = 0.0;
#pragma unroll
    for (int d = 0; d < DIM; ++d) {
      const double md = static_cast<double>(U[base + (NS + d) * plane]);
      m2 += md * md;
    }
    const double E = static_cast<double>(U[base + (NS + DIM) * plane]);
    const double ke = 0.5 * m2 / rho;
    double Y[NS];
#pragma unroll
    for (int s = 0; s < NS; ++s) Y[s] = Yn[s];
    int it = dn.it, clips = 0;
    bool nonphys = false;
    auto newton = [&](double hh) -> bool {
      for (int k_it = 0; k_it < max_iter; ++k_it) {
        // this lane's point: Y displaced along Y_pt (pt < NS), else Y
        double Yp[NS], eps = 1.0;
#pragma unroll
        for (int s = 0; s < NS; ++s) {
          Yp[s] = Y[s];
          if (s == pt) {
            eps = fmax(1e-7 * fabs(Y[s]), 1e-12);
            Yp[s] = Yp[s] + eps;
          }
        }
        // the point's residual: reaction rl's rate here, the point's NR rates
        // gathered and summed as in the one-lane residual
        const double Tl = chem.temperature(Yp, ke, E);
        const double Rr = chem.rate(rl, Yp, Tl);
        double w[NS];
#pragma unroll
        for (int s = 0; s < NS; ++s) w[s] = 0.0;
#pragma unroll
        for (int r = 0; r < NR; ++r) {
          const double Rq = __shfl(Rr, pbase + r, G);
#pragma unroll
          for (int s = 0; s < NS; ++s) {
            const int dnu = mech->nu_b[r][s] - mech->nu_f[r][s];
            if (dnu != 0) w[s] = fma(mech->kappa_r * mech->W[s] * dnu, Rq, w[s]);
          }
        }
        double Rl[NS];
#pragma unroll
        for (int s = 0; s < NS; ++s) Rl[s] = (Yp[s] - Yn[s]) - hh * w[s];
        double R0[NS];
#pragma unroll
        for (int s = 0; s < NS; ++s) R0[s] = __shfl(Rl[s], NS * NR, G);
        const double T0 = __shfl(Tl, NS * NR, G);
        if (!(T0 > 0.0)) {
          nonphys = true;
          return false;
        }
        ++it;
        double J[NS][NS];
#pragma unroll
        for (int k = 0; k < NS; ++k) {
          const double ek = __shfl(eps, k * NR, G);
#pragma unroll
          for (int s = 0; s < NS; ++s) J[s][k] = (__shfl(Rl[s], k * NR, G) - R0[s]) / ek;
        }
        double rhs[NS], dY[NS];
#pragma unroll
        for (int s = 0; s < NS; ++s) rhs[s] = -R0[s];
        gauss_jordan<NS>(J, rhs, dY);
        double alpha = 1.0;
        for (int hv = 0; hv < 30; ++hv) {
          double Yt[NS];
#pragma unroll
          for (int s = 0; s < NS; ++s) Yt[s] = fmax(Y[s] + alpha * dY[s], 0.0);
          const double Tt = chem.temperature(Yt, ke, E);
          if (!(Tt < 0.5 * T0) && !(Tt > 2.0 * T0)) break;
          alpha *= 0.5;
        }
        double dmax = 0.0;
#pragma unroll
        for (int s = 0; s < NS; ++s) {
          dY[s] = alpha * dY[s];
          double y = Y[s] + dY[s];
          if (y < 0.0) {
            ++clips;
            y = 0.0;
          }
          Y[s] = y;
          dmax = fmax(dmax, fabs(dY[s]));
        }
        if (alpha == 1.0 && dmax <= tol * rho) return true;
      }
      return false;
    };
    bool converged = false;
    for (int j = CONT_LEVELS; j >= 0 && !nonphys; --j) converged = newton(ldexp(h, -j));
    if (lane == 0) {
      if (nonphys) report_nonphysical(counters, first_bad, t);
      if (!converged) atomicAdd(&counters[CNT_NEWTON], 1);
      if (clips) atomicAdd(&counters[CNT_CLIPS], clips);
      atomicMax(&counters[CNT_ITERS], it);
#pragma unroll
      for (int s = 0; s < NS; ++s) out[base + s * plane] = static_cast<T>(Y[s]);
    }
  }
}

__global__ void k_zero_count(int* p) {
  if (threadIdx.x == 0) *p = 0;
}

// ---------------------------------------------------------------------------
// Two temperatures (Thermochemical non-equilibrium section; eqs.
// src_reaction_rate, src_omega, src_landau_teller, source_residual).  State
// (rho_s, m, E, E_v).  Per node:
//   T   from E - E_v - |m|^2/(2 rho) - sum rho_s h0_s = T sum rho_s cv_s;
//   T_v from E_v = sum_mol rho_s e_v,s(T_v), e_v,s = R_s theta_s / (exp(theta_s/T) - 1),
//       by Newton in ln T_v from the inverse of a single mode with the
//       mixture's mean theta (exact when the thetas agree; a few steps);
//   rates of reaction r at T_a = sqrt(T T_v) when flagged (dissociation),
//       else at T;
//   Q_T-v = sum_mol rho_s (e_v,s(T) - e_v,s(T_v)) / tau_s with the
//       Millikan-White mixture time plus Park's correction;
//   S_Ev = Q_T-v + sum_mol wdot_s e_v,s(T_v).
// Implicit substep on Y = (rho_s, E_v): Newton with the one-sided difference
// Jacobian and Gauss-Jordan, globalised as follows: the step length alpha is
// halved while the clipped update would move T outside [T/2, 2T], then
// further until the scaled residual max_k |R_k|/scale_k falls by
// (1 - 1e-4 alpha) (at most 30 halvings each); the accepted update's residual
// is the next iteration's; converged when the undamped step satisfies
// max_k |dY_k|/scale_k <= tol (then applied in full); scale = rho for the
// species and E - |m|^2/(2 rho) - sum rho_s h0_s for E_v; rho_s and E_v are
// clipped at 0 (counted).
// ---------------------------------------------------------------------------
constexpr double kRUniversal = 8.31446261815324;  // J/(mol K)
constexpr double kBoltzmann = 1.380649e-23;       // J/K
constexpr double kAtm = 101325.0;                 // Pa
constexpr double kPi = 3.14159265358979323846;

template <int NS, int NR>
struct Chem2T {
  const dg_mechanism* m;
  const dg_vibration* v;

  __device__ __forceinline__ double temperature(const double (&Y)[NS + 1], double ke, double E) const {
    double cv = 0.0, h0 = 0.0;
#pragma unroll
    for (int s = 0; s < NS; ++s) {
      cv = fma(Y[s], m->cv[s], cv);
      h0 = fma(Y[s], m->h0[s], h0);
    }
    return (E - Y[NS] - ke - h0) / cv;
  }

  __device__ __forceinline__ double ev(int s, double T) const {
    const double th = v->theta_v[s];
    return th > 0.0 ? m->R[s] * th / expm1(th / T) : 0.0;
  }

  // T_v with sum_mol rho_s e_v,s(T_v) = Ev (1 K for Ev <= 0, 1e6 K without molecules)
  __device__ __forceinline__ double t_vib(const double (&Y)[NS + 1]) const {
    const double Ev = Y[NS];
    if (!(Ev > 0.0)) return 1.0;
    double A = 0.0, B = 0.0;
#pragma unroll
    for (int s = 0; s < NS; ++s) {
      const double th = v->theta_v[s];
      if (th > 0.0) {
        const double a = Y[s] * m->R[s];
        A = fma(a, th, A);
        B += a;
      }
    }
    if (!(B > 0.0)) return 1.0e6;
    double T = (A / B) / log1p(A / Ev);
    for (int it = 0; it < 40; ++it) {
      double f = -Ev, fp = 0.0;
#pragma unroll
      for (int s = 0; s < NS; ++s) {
        const double th = v->theta_v[s];
        if (th > 0.0) {
          const double x = th / T;
          const double em = expm1(x);
          const double a = Y[s] * m->R[s];
          f = fma(a, th / em, f);
          fp = fma(a * x * x, (em + 1.0) / (em * em), fp);  // d/dT of rho_s e_v,s
        }
      }
      const double dl = f / (T * fp);  // Newton step in ln T
      T *= exp(-dl);
      if (fabs(dl) <= 1e-12) break;
    }
    return T;
  }

  __device__ __forceinline__ void wdot(const double (&Y)[NS + 1], double T, double Tv, double (&w)[NS]) const {
    double X[NS];
#pragma unroll
    for (int s = 0; s < NS; ++s) {
      X[s] = m->kappa_c * Y[s] / m->W[s];
      w[s] = 0.0;
    }
    const double lnT = log(T);
    const double Ti = 1.0 / T;
    const double Ta = sqrt(T * Tv);
    const double lnTa = log(Ta);
    const double Tai = 1.0 / Ta;
#pragma unroll
    for (int r = 0; r < NR; ++r) {
      const bool two = v->two_temp[r] != 0;
      const double lt = two ? lnTa : lnT;
      const double ti = two ? Tai : Ti;
      double fwd = m->A_f[r] * exp(fma(m->beta_f[r], lt, -m->theta_f[r] * ti));
      double bwd = 0.0;
      for (int s = 0; s < NS; ++s)
        for (int q = 0; q < m->nu_f[r][s]; ++q) fwd *= X[s];
      if (m->reversible[r]) {
        bwd = m->A_b[r] * exp(fma(m->beta_b[r], lt, -m->theta_b[r] * ti));
        for (int s = 0; s < NS; ++s)
          for (int q = 0; q < m->nu_b[r][s]; ++q) bwd *= X[s];
      }
      double M = 1.0;
      if (m->third_body[r]) {
        M = 0.0;
#pragma unroll
        for (int s = 0; s < NS; ++s) M = fma(m->eff[r][s], X[s], M);
      }
      const double Rr = M * (fwd - bwd);
#pragma unroll
      for (int s = 0; s < NS; ++s) {
        const int dnu = m->nu_b[r][s] - m->nu_f[r][s];
        if (dnu != 0) w[s] = fma(m->kappa_r * m->W[s] * dnu, Rr, w[s]);
      }
    }
  }

  // Landau-Teller term at densities Y, temperatures T, T_v
  __device__ __forceinline__ double q_vt(const double (&Y)[NS + 1], double T, double Tv) const {
    double moles[NS], ntot = 0.0, Rm = 0.0;
#pragma unroll
    for (int s = 0; s < NS; ++s) {
      moles[s] = Y[s] / m->W[s];
      ntot += moles[s];
      Rm = fma(Y[s], m->R[s], Rm);
    }
    const double p = T * Rm;
    const double patm = p / kAtm;
    const double n = p / (kBoltzmann * T);
    const double sig = v->park_sigma * (50000.0 / T) * (50000.0 / T);
    const double Tm13 = exp(-log(T) / 3.0);
    double q = 0.0;
#pragma unroll
    for (int s = 0; s < NS; ++s) {
      if (!(v->theta_v[s] > 0.0)) continue;
      double inv = 0.0;
#pragma unroll
      for (int r = 0; r < NS; ++r)
        inv = fma(moles[r] / ntot, exp(-(v->mw_a[s][r] * (Tm13 - v->mw_b[s][r]) - 18.42)), inv);
      const double tau_mw = 1.0 / (patm * inv);
      const double cbar = sqrt(8.0 * kRUniversal * T / (kPi * m->W[s]));
      const double tau = tau_mw + 1.0 / (sig * cbar * n);
      q += Y[s] * (ev(s, T) - ev(s, Tv)) / tau;
    }
    return q;
  }

  // S_Y = (wdot_s, Q_T-v + sum_mol wdot_s e_v,s(T_v)) at Y with temperature T
  __device__ __forceinline__ void source(const double (&Y)[NS + 1], double T, double (&S)[NS + 1]) const {
    const double Tv = t_vib(Y);
    double w[NS];
    wdot(Y, T, Tv, w);
    double sev = q_vt(Y, T, Tv);
#pragma unroll
    for (int s = 0; s < NS; ++s) {
      S[s] = w[s];
      if (v->theta_v[s] > 0.0) sev = fma(w[s], ev(s, Tv), sev);
    }
    S[NS] = sev;
  }

  // R(Y) = Y - Yn - h S_Y(Y); returns T(Y)
  __device__ __forceinline__ double residual(const double (&Y)[NS + 1], const double (&Yn)[NS + 1], double h,
                                             double ke, double E, double (&R)[NS + 1]) const {
    const double T = temperature(Y, ke, E);
    double S[NS + 1];
    source(Y, T, S);
#pragma unroll
    for (int k = 0; k <= NS; ++k) R[k] = (Y[k] - Yn[k]) - h * S[k];
    return T;
  }
};

template <typename T, int NS, int NR, int DIM>
__global__ void __launch_bounds__(256)
k_source2t(const T* U, T* out, const dg_mechanism* mech, const dg_vibration* vib, size_t plane, int B, double h,
           int mode, int max_iter, double tol, int* counters, unsigned long long* first_bad) {
  constexpr int NV = NS + DIM + 2;
  constexpr int NY = NS + 1;
  const Chem2T<NS, NR> chem{mech, vib};
  const size_t total = plane * B;
  for (size_t t = blockIdx.x * (size_t)blockDim.x + threadIdx.x; t < total; t += (size_t)gridDim.x * blockDim.x) {
    const size_t b = t / plane;
    const size_t r = t - b * plane;
    const size_t base = b * NV * plane + r;
    double Yn[NY], mom[DIM];
    double rho = 0.0, h0 = 0.0;
#pragma unroll
    for (int s = 0; s < NS; ++s) {
      Yn[s] = static_cast<double>(U[base + s * plane]);
      rho += Yn[s];
      h0 = fma(Yn[s], mech->h0[s], h0);
    }
    Yn[NS] = static_cast<double>(U[base + (NS + DIM + 1) * plane]);
    double m2 = 0.0;
#pragma unroll
    for (int d = 0; d < DIM; ++d) {
      mom[d] = static_cast<double>(U[base + (NS + d) * plane]);
      m2 += mom[d] * mom[d];
    }
    const double E = static_cast<double>(U[base + (NS + DIM) * plane]);
    const double ke = 0.5 * m2 / rho;
    if (mode == 0) {
      const double Tn = chem.temperature(Yn, ke, E);
      if (!(Tn > 0.0) || !(Yn[NS] >= 0.0)) report_nonphysical(counters, first_bad, t);
      double S[NY];
      chem.source(Yn, Tn, S);
#pragma unroll
      for (int s = 0; s < NS; ++s) {
        const double o = static_cast<double>(out[base + s * plane]);
        out[base + s * plane] = static_cast<T>(o + S[s]);
      }
      const size_t iv = base + (NS + DIM + 1) * plane;
      out[iv] = static_cast<T>(static_cast<double>(out[iv]) + S[NS]);
      continue;
    }
    // ---- implicit substep ----------------------------------------------------
    double scale[NY];
#pragma unroll
    for (int s = 0; s < NS; ++s) scale[s] = rho;
    scale[NS] = fabs(E - ke - h0);
    double Y[NY], R0[NY];
#pragma unroll
    for (int k = 0; k < NY; ++k) Y[k] = Yn[k];
    double T0 = chem.residual(Y, Yn, h, ke, E, R0);
    bool converged = false, bad_state = false;
    int it = 0, clips = 0;
    for (; it < max_iter; ++it) {
      if (!(T0 > 0.0)) {
        bad_state = true;
        break;
      }
      double J[NY][NY];
#pragma unroll
      for (int k = 0; k < NY; ++k) {
        const double eps = fmax(1e-7 * fabs(Y[k]), 1e-12);
        double Yp[NY], Rk[NY];
#pragma unroll
        for (int q = 0; q < NY; ++q) Yp[q] = Y[q];
        Yp[k] = Yp[k] + eps;
        chem.residual(Yp, Yn, h, ke, E, Rk);
#pragma unroll
        for (int q = 0; q < NY; ++q) J[q][k] = (Rk[q] - R0[q]) / eps;
      }
      double rhs[NY], dY[NY];
#pragma unroll
      for (int k = 0; k < NY; ++k) rhs[k] = -R0[k];
      gauss_jordan<NY>(J, rhs, dY);
      double dn = 0.0, n0 = 0.0;
#pragma unroll
      for (int k = 0; k < NY; ++k) {
        dn = fmax(dn, fabs(dY[k]) / scale[k]);
        n0 = fmax(n0, fabs(R0[k]) / scale[k]);
      }
      const bool done = dn <= tol;
      double alpha = 1.0;
      if (!done) {
        for (int hv = 0; hv < 30; ++hv) {
          double Yt[NY];
#pragma unroll
          for (int k = 0; k < NY; ++k) Yt[k] = fmax(Y[k] + alpha * dY[k], 0.0);
          const double Tt = chem.temperature(Yt, ke, E);
          if (!(Tt < 0.5 * T0) && !(Tt > 2.0 * T0)) break;
          alpha *= 0.5;
        }
      }
      double Yt[NY], Rt[NY], Tt = T0, used = alpha;
      for (int hv = 0; hv <= 30; ++hv) {
        used = alpha;
#pragma unroll
        for (int k = 0; k < NY; ++k) Yt[k] = fmax(Y[k] + used * dY[k], 0.0);
        Tt = chem.residual(Yt, Yn, h, ke, E, Rt);
        if (done) break;
        double nt = 0.0;
#pragma unroll
        for (int k = 0; k < NY; ++k) nt = fmax(nt, fabs(Rt[k]) / scale[k]);
        if (!(nt > (1.0 - 1e-4 * used) * n0)) break;
        alpha *= 0.5;
      }
#pragma unroll
      for (int k = 0; k < NY; ++k) {
        if (Y[k] + used * dY[k] < 0.0) ++clips;
        Y[k] = Yt[k];
        R0[k] = Rt[k];
      }
      T0 = Tt;
      if (done) {
        converged = true;
        ++it;
        break;
      }
    }
    if (bad_state) report_nonphysical(counters, first_bad, t);
    if (!converged) atomicAdd(&counters[CNT_NEWTON], 1);
    if (clips) atomicAdd(&counters[CNT_CLIPS], clips);
    atomicMax(&counters[CNT_ITERS], it);
#pragma unroll
    for (int s = 0; s < NS; ++s) out[base + s * plane] = static_cast<T>(Y[s]);
    out[base + (NS + DIM + 1) * plane] = static_cast<T>(Y[NS]);
    if (out != U) {
#pragma unroll
      for (int d = 0; d < DIM; ++d) out[base + (NS + d) * plane] = static_cast<T>(mom[d]);
      out[base + (NS + DIM) * plane] = static_cast<T>(E);
    }
  }
}

hipError_t launch_source(const Ctx& c, const void* U, void* out, double h, int mode, hipStream_t s) {
  if (c.dim != 2 || c.mech.nspecies != 5 || c.mech.nreactions != 5) return hipErrorNotSupported;
  const size_t plane = (size_t)c.E * c.Np;
  const size_t total = plane * c.B;
  const int blocks = (int)std::min<size_t>((total + 255) / 256, 65535);
  const dg_mechanism* m = static_cast<const dg_mechanism*>(c.d_mech);
  if (c.desc.physics == DG_REACTING_2T) {
    const dg_vibration* v = static_cast<const dg_vibration*>(c.d_vib);
    if (c.desc.precision == DG_F32)
      hipLaunchKernelGGL((k_source2t<float, 5, 5, 2>), dim3(blocks), dim3(256), 0, s, static_cast<const float*>(U),
                         static_cast<float*>(out), m, v, plane, c.B, h, mode, c.desc.newton_max_iter,
                         c.desc.newton_tol, c.d_counters, c.d_first_bad);
    else
      hipLaunchKernelGGL((k_source2t<double, 5, 5, 2>), dim3(blocks), dim3(256), 0, s, static_cast<const double*>(U),
                         static_cast<double*>(out), m, v, plane, c.B, h, mode, c.desc.newton_max_iter,
                         c.desc.newton_tol, c.d_counters, c.d_first_bad);
    return hipGetLastError();
  }
  // mode 1 in two passes: the first runs every node's Newton iteration at h
  // and hands the nodes that need the continuation to the second
  const bool two_pass = mode == 1 && c.d_defer && total < ((size_t)1 << 31);
  DeferredNode* defer = two_pass ? static_cast<DeferredNode*>(c.d_defer) : nullptr;
  if (two_pass) {
    hipLaunchKernelGGL(k_zero_count, dim3(1), dim3(64), 0, s, c.d_defer_count);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  // the second pass: 8 nodes per 256-lane block, grid-stride beyond 1024 blocks
  const int cont_blocks = (int)std::min<size_t>((total + 7) / 8, 1024);
  if (c.desc.precision == DG_F32) {
    hipLaunchKernelGGL((k_source<float, 5, 5, 2>), dim3(blocks), dim3(256), 0, s, static_cast<const float*>(U),
                       static_cast<float*>(out), m, plane, c.B, h, mode, c.desc.newton_max_iter, c.desc.newton_tol,
                       c.d_counters, c.d_first_bad, defer, c.d_defer_count);
    if (two_pass)
      hipLaunchKernelGGL((k_source_cont<float, 5, 5, 2>), dim3(cont_blocks), dim3(256), 0, s,
                         static_cast<const float*>(U), static_cast<float*>(out), m, plane, h,
                         c.desc.newton_max_iter, c.desc.newton_tol, c.d_counters, c.d_first_bad, defer,
                         c.d_defer_count);
  } else {
    hipLaunchKernelGGL((k_source<double, 5, 5, 2>), dim3(blocks), dim3(256), 0, s, static_cast<const double*>(U),
                       static_cast<double*>(out), m, plane, c.B, h, mode, c.desc.newton_max_iter, c.desc.newton_tol,
                       c.d_counters, c.d_first_bad, defer, c.d_defer_count);
    if (two_pass)
      hipLaunchKernelGGL((k_source_cont<double, 5, 5, 2>), dim3(cont_blocks), dim3(256), 0, s,
                         static_cast<const double*>(U), static_cast<double*>(out), m, plane, h,
                         c.desc.newton_max_iter, c.desc.newton_tol, c.d_counters, c.d_first_bad, defer,
                         c.d_defer_count);
  }
  return hipGetLastError();
}

}  // namespace dg
