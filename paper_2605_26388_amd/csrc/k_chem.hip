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
//   species are clipped at 0 after the update (counted); stop when
//   max |dY| <= tol rho or after max_iter iterations (then counted as
//   unconverged).  The state of a node never leaves registers between
//   evaluations; global traffic is one read and one write of the state.
#include <algorithm>

#include "dg_device.hpp"

namespace dg {

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

template <typename T, int NS, int NR, int DIM>
__global__ void __launch_bounds__(256)
k_source(const T* U, T* out, const dg_mechanism* mech, size_t plane, int B, double h, int mode, int max_iter,
         double tol, int* counters, unsigned long long* first_bad) {
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
    bool converged = false;
    int it = 0, clips = 0;
    for (; it < max_iter; ++it) {
      double R0[NS];
      const double T0 = chem.residual(Y, Yn, h, ke, E, R0);
      if (!(T0 > 0.0)) {
        report_nonphysical(counters, first_bad, t);
        break;
      }
      double J[NS][NS];
#pragma unroll
      for (int k = 0; k < NS; ++k) {
        const double eps = fmax(1e-7 * fabs(Y[k]), 1e-12);
        double Yp[NS], Rk[NS];
#pragma unroll
        for (int s = 0; s < NS; ++s) Yp[s] = Y[s];
        Yp[k] = Yp[k] + eps;
        chem.residual(Yp, Yn, h, ke, E, Rk);
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
      if (dmax <= tol * rho) {
        converged = true;
        ++it;
        break;
      }
    }
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

hipError_t launch_source(const Ctx& c, const void* U, void* out, double h, int mode, hipStream_t s) {
  if (c.dim != 2 || c.mech.nspecies != 5 || c.mech.nreactions != 5) return hipErrorNotSupported;
  const size_t plane = (size_t)c.E * c.Np;
  const size_t total = plane * c.B;
  const int blocks = (int)std::min<size_t>((total + 255) / 256, 65535);
  const dg_mechanism* m = static_cast<const dg_mechanism*>(c.d_mech);
  if (c.desc.precision == DG_F32)
    hipLaunchKernelGGL((k_source<float, 5, 5, 2>), dim3(blocks), dim3(256), 0, s, static_cast<const float*>(U),
                       static_cast<float*>(out), m, plane, c.B, h, mode, c.desc.newton_max_iter, c.desc.newton_tol,
                       c.d_counters, c.d_first_bad);
  else
    hipLaunchKernelGGL((k_source<double, 5, 5, 2>), dim3(blocks), dim3(256), 0, s, static_cast<const double*>(U),
                       static_cast<double*>(out), m, plane, c.B, h, mode, c.desc.newton_max_iter, c.desc.newton_tol,
                       c.d_counters, c.d_first_bad);
  return hipGetLastError();
}

}  // namespace dg
