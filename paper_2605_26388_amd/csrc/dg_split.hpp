// Interface wave speed and the entropy-conservative split-form volume sum
// (eq. vol_split with Ranocha's two-point flux), shared by the inviscid stage
// kernel and the Navier-Stokes pass that adds the BR1 viscous terms to it.
#pragma once

#include "dg_device.hpp"

namespace dg {

// Speed of sound for the Rusanov dissipation coefficient.  The FP32 form
// takes the single-precision hardware square root (about one unit in the
// last place of a float): the coefficient only scales the jump term, so its
// relative error of about 1e-7 stays far below the form's stated accuracy.
template <class PHYS, bool F32>
__device__ __forceinline__ double wave_sound(const Thermo& t) {
  if constexpr (F32) {
    return static_cast<double>(__builtin_amdgcn_sqrtf(static_cast<float>(t.k * t.p * t.ri)));
  } else {
    // The FP64 form: the hardware reciprocal square root refined by one
    // coupled Goldschmidt step, relative error about 1.5 e^2 for an estimate
    // error e of about 2^-23, i.e. near 1e-14 -- the coefficient only scales
    // the jump term, and both elements of a face evaluate it on the same
    // operands, so they still agree to the bit.
    const double x = t.k * t.p * t.ri;
    const double y = __builtin_amdgcn_rsq(x);
    const double g = x * y, h = 0.5 * y;
    return fma(g, fma(-g, h, 0.5), g);
  }
}

// Logarithmic mean {{x}}_ln = (x - y) / (ln x - ln y) of positive x, y and its
// reciprocal.  With f = (x - y)/(x + y) and u = f^2, ln(x/y) = 2 atanh f =
// 2 f P(u), P(u) = sum_k u^k / (2k + 1), hence {{x}}_ln = (x + y) / (2 P(u)) =
// (x + y) Q(u) / 2 with Q = 1/P = 1 - u/3 - 4u^2/45 - 44u^3/945 - ... (the
// coefficients of the reciprocal power series, exact rationals below): no
// cancellation as x -> y, the limit x at x = y comes out exactly, and no
// division.  For u < SERIES_U_MAX = 1e-3 (x/y within about 1.065) the series
// through u^4 leave a relative truncation below 1e-16 (P: u^5 / 11; Q: its
// next coefficient 10196/467775 times u^5); smooth states stay far below (the
// 32^3 benchmark state: u <= 4e-5 for every pair of every line).  The fast
// form uses the series for every pair and raises `far` where u >=
// SERIES_U_MAX; the exact form takes the closed form there, with ln x and ln y
// read from LDS.  Branches inside the unrolled sweep would make it spill
// registers, so a lane that raised `far` redoes its whole volume sum in the
// exact form (a path smooth states never take; the logarithms are only
// computed when some lane of the block needs them).
constexpr double SERIES_U_MAX = 1e-3;

__device__ __forceinline__ double atanh_ratio_series(double u) {  // P(u)
  double P = 1.0 / 9.0;
  P = fma(P, u, 1.0 / 7.0);
  P = fma(P, u, 1.0 / 5.0);
  P = fma(P, u, 1.0 / 3.0);
  return fma(P, u, 1.0);
}

__device__ __forceinline__ double inv_atanh_ratio_series(double u) {  // Q(u) = 1 / P(u)
  double Q = -428.0 / 14175.0;
  Q = fma(Q, u, -44.0 / 945.0);
  Q = fma(Q, u, -4.0 / 45.0);
  Q = fma(Q, u, -1.0 / 3.0);
  return fma(Q, u, 1.0);
}

// Both means take the halves hx = x/2, hy = y/2 (the block stages halved
// rho and beta): (x - y)/(x + y) = (hx - hy)/(hx + hy), so
//   {{x}}_ln = (hx + hy) Q(u),   1 / {{x}}_ln = P(u) / (hx + hy),
// and the closed forms are 2 (hx - hy) / (ln x - ln y) and its reciprocal.
template <bool EXACT>
__device__ __forceinline__ double log_mean(double hx, double hy, const double* lnx, const double* lny, bool& far) {
  const double hs = hx + hy, hd = hx - hy;
  const double f = hd * frcp(hs);
  const double u = f * f;
  double r = hs * inv_atanh_ratio_series(u);
  if constexpr (EXACT) {
    if (u >= SERIES_U_MAX) r = 2.0 * hd / (*lnx - *lny);
  } else {
    far |= u >= SERIES_U_MAX;
  }
  return r;
}

template <bool EXACT>
__device__ __forceinline__ double inv_log_mean(double hx, double hy, const double* lnx, const double* lny, bool& far) {
  const double hs = hx + hy, hd = hx - hy;
  const double rs = frcp(hs);
  const double f = hd * rs;
  const double u = f * f;
  double r = atanh_ratio_series(u) * rs;
  if constexpr (EXACT) {
    if (u >= SERIES_U_MAX) r = (*lnx - *lny) / (2.0 * hd);
  } else {
    far |= u >= SERIES_U_MAX;
  }
  return r;
}

// Own-node values a lane keeps in registers for its two-point fluxes.
template <int DIM>
struct SplitNode {
  double hr;        // rho / 2
  double v[DIM];    // velocity
  double hv[DIM];   // velocity / 2
  double p, hp;     // pressure and its half
  double hb;        // rho / (2 p)
};

// Ranocha's entropy-conservative, kinetic-energy-preserving two-point flux
// along direction l between node i (registers) and node m (LDS):
//   f_rho = {{rho}}_ln {{v_l}},  f_v_d = f_rho {{v_d}} + {{p}} delta_dl,
//   f_E = f_rho (1 / ((gamma - 1) {{beta}}_ln) + v_i . v_m / 2)
//         + (p_i v_m,l + p_m v_i,l) / 2,   beta = rho / p.
// With halved velocities in LDS the arithmetic means are single additions,
// v_i . v_m / 2 = v_i . (v_m / 2) and (p_i v_m,l + p_m v_i,l)/2 =
// p_i (v_m,l / 2) + p_m (v_i,l / 2).  LDS rows: Q[0] = rho/2, Q[1..DIM] =
// v/2, Q[DIM+1] = p, Q[DIM+2] = beta/2, Q[DIM+3] = ln rho, Q[DIM+4] = ln beta
// (the last two filled only when the exact form runs).
template <int DIM, int l, bool EXACT, int W>
__device__ __forceinline__ void ranocha_flux(const SplitNode<DIM>& a, const double (*Q)[W], int i, int m,
                                             double gm1i, bool& far, double (&F)[DIM + 2]) {
  const double hrm = Q[0][m], pm = Q[DIM + 1][m], hbm = Q[DIM + 2][m];
  double hvm[DIM];
#pragma unroll
  for (int d = 0; d < DIM; ++d) hvm[d] = Q[1 + d][m];
  const double rho_ln = log_mean<EXACT>(a.hr, hrm, &Q[DIM + 3][i], &Q[DIM + 3][m], far);
  const double ib_ln = inv_log_mean<EXACT>(a.hb, hbm, &Q[DIM + 4][i], &Q[DIM + 4][m], far);
  double va[DIM];
  double hvv = a.v[0] * hvm[0];
#pragma unroll
  for (int d = 0; d < DIM; ++d) {
    va[d] = a.hv[d] + hvm[d];
    if (d > 0) hvv = fma(a.v[d], hvm[d], hvv);
  }
  const double fr = rho_ln * va[l];
  F[0] = fr;
#pragma unroll
  for (int d = 0; d < DIM; ++d) F[1 + d] = d == l ? fma(fr, va[d], fma(0.5, pm, a.hp)) : fr * va[d];
  F[DIM + 1] = fma(fr, fma(ib_ln, gm1i, hvv), fma(a.p, hvm[l], pm * a.hv[l]));
}

// One term of the split sum: s += D_im F#_l(U_i, U_m) for the k-th partner
// m = i + k (mod n) of the lane's line along l.
template <int DIM, int N, int l, bool EXACT, int W>
__device__ __forceinline__ void split_term(int k, int tid, int il, int base, int st, const SplitNode<DIM>& a,
                                           const double (*Q)[W], const double* sD, double gm1i, bool& far,
                                           double (&s)[DIM + 2]) {
  constexpr int n = N + 1;
  const int m = il + k < n ? il + k : il + k - n;
  double F[DIM + 2];
  ranocha_flux<DIM, l, EXACT>(a, Q, tid, base + m * st, gm1i, far, F);
  const double dim = sD[il * n + m];
#pragma unroll
  for (int v = 0; v < DIM + 2; ++v) s[v] = fma(dim, F[v], s[v]);
}

// Split-form volume sum of one lane, directions l..DIM-1:
// acc -= 2 (2/h_l) sum_{m != i} D_im F#_l(U_i, U_m) over the lane's line along
// l.  The partner index runs i+1, ..., i+N modulo n, so every lane makes the
// same N flux evaluations per direction (the m = i term is added elsewhere).
// This serves the exact form, and the fast form where a line spans waves
// (split_sweep_pairs below halves the evaluations otherwise).  The fast form
// is fully unrolled; the exact form keeps its partner loop rolled (it only
// runs for lanes with widely separated partner states).
template <int DIM, int N, int l, bool EXACT, int W>
__device__ __forceinline__ void split_sweep(int tid, const int (&ii)[3], const int (&stride)[3],
                                            const SplitNode<DIM>& a, const double (*Q)[W], const double* sD,
                                            const double (&g)[DIM], double gm1i, bool& far,
                                            double (&acc)[DIM + 2]) {
  if constexpr (l < DIM) {
    constexpr int NV = DIM + 2;
    const int il = ii[l];
    const int st = stride[l];
    const int base = tid - il * st;
    double s[NV];
#pragma unroll
    for (int v = 0; v < NV; ++v) s[v] = 0.0;
    if constexpr (EXACT) {
#pragma unroll 1
      for (int k = 1; k <= N; ++k)
        split_term<DIM, N, l, true>(k, tid, il, base, st, a, Q, sD, gm1i, far, s);
    } else {
#pragma unroll
      for (int k = 1; k <= N; ++k)
        split_term<DIM, N, l, false>(k, tid, il, base, st, a, Q, sD, gm1i, far, s);
    }
    const double c = -2.0 * g[l];
#pragma unroll
    for (int v = 0; v < NV; ++v) acc[v] = fma(c, s[v], acc[v]);
    split_sweep<DIM, N, l + 1, EXACT>(tid, ii, stride, a, Q, sD, g, gm1i, far, acc);
  }
}

// Fast split sum with every unordered pair of a line evaluated once (the
// two-point flux is symmetric): for k = 1 .. (n-1)/2 the lane evaluates
// F#_l(U_i, U_{i+k}) and hands it to the lane of node i+k, which adds
// D_{i+k,i} times it; for even n the opposite partner i + n/2 is evaluated by
// both of its lanes.  A lane thus makes floor(n/2) flux evaluations per
// direction instead of n - 1 (two instead of three at N = 3).  A pair's
// far flag travels with its flux, so both lanes of a far pair redo their sums
// in the exact form.  The hand-over is a lane shuffle, so a whole line must
// lie in one wave (one-wave workgroups).
template <int DIM, int N, int l, int W>
__device__ __forceinline__ void split_sweep_pairs(int tid, const int (&ii)[3], const int (&stride)[3],
                                                  const SplitNode<DIM>& a, const double (*Q)[W], const double* sD,
                                                  const double (&g)[DIM], double gm1i, bool& far,
                                                  double (&acc)[DIM + 2]) {
  if constexpr (l < DIM) {
    constexpr int NV = DIM + 2, n = N + 1, K1 = (n - 1) / 2;
    const int il = ii[l];
    const int st = stride[l];
    const int base = tid - il * st;
    const int lbase = (tid & 63) - il * st;  // wave lane of the line's node 0
    double s[NV];
#pragma unroll
    for (int v = 0; v < NV; ++v) s[v] = 0.0;
#pragma unroll
    for (int k = 1; k <= K1; ++k) {
      const int m = il + k < n ? il + k : il + k - n;   // partner evaluated here
      const int j = il - k >= 0 ? il - k : il - k + n;  // partner whose flux arrives
      double F[NV];
      bool fp = false;
      ranocha_flux<DIM, l, false>(a, Q, tid, base + m * st, gm1i, fp, F);
      const double dm = sD[il * n + m];
      const double dj = sD[il * n + j];
      const int src = lbase + j * st;
      const int fr = __shfl(fp ? 1 : 0, src);
#pragma unroll
      for (int v = 0; v < NV; ++v) {
        const double Fr = __shfl(F[v], src);
        s[v] = fma(dm, F[v], s[v]);
        s[v] = fma(dj, Fr, s[v]);
      }
      far = far || fp || fr != 0;
    }
    if constexpr (n % 2 == 0) {
      const int m = il + n / 2 < n ? il + n / 2 : il - n / 2;
      double F[NV];
      ranocha_flux<DIM, l, false>(a, Q, tid, base + m * st, gm1i, far, F);
      const double dm = sD[il * n + m];
#pragma unroll
      for (int v = 0; v < NV; ++v) s[v] = fma(dm, F[v], s[v]);
    }
    const double c = -2.0 * g[l];
#pragma unroll
    for (int v = 0; v < NV; ++v) acc[v] = fma(c, s[v], acc[v]);
    split_sweep_pairs<DIM, N, l + 1>(tid, ii, stride, a, Q, sD, g, gm1i, far, acc);
  }
}

// The same two-point flux contracted with a direction vector nv (curvilinear
// elements: nv = Ja^l_i + Ja^l_m, twice the pair's averaged contravariant
// vector; the flux is linear in the direction):
//   f_rho = {{rho}}_ln {{v}} . nv,  f_v_d = f_rho {{v_d}} + {{p}} nv_d,
//   f_E = f_rho (1 / ((gamma - 1) {{beta}}_ln) + v_i . v_m / 2)
//         + (p_i v_m . nv + p_m v_i . nv) / 2.
template <int DIM, bool EXACT, int W>
__device__ __forceinline__ void ranocha_flux_n(const SplitNode<DIM>& a, const double (*Q)[W], int i, int m,
                                               const double (&nv)[DIM], double gm1i, bool& far,
                                               double (&F)[DIM + 2]) {
  const double hrm = Q[0][m], pm = Q[DIM + 1][m], hbm = Q[DIM + 2][m];
  double hvm[DIM];
#pragma unroll
  for (int d = 0; d < DIM; ++d) hvm[d] = Q[1 + d][m];
  const double rho_ln = log_mean<EXACT>(a.hr, hrm, &Q[DIM + 3][i], &Q[DIM + 3][m], far);
  const double ib_ln = inv_log_mean<EXACT>(a.hb, hbm, &Q[DIM + 4][i], &Q[DIM + 4][m], far);
  double va[DIM];
  double hvv = a.v[0] * hvm[0];
  double van = 0.0, hvmn = 0.0, hvin = 0.0;
#pragma unroll
  for (int d = 0; d < DIM; ++d) {
    va[d] = a.hv[d] + hvm[d];
    if (d > 0) hvv = fma(a.v[d], hvm[d], hvv);
    van = fma(va[d], nv[d], van);
    hvmn = fma(hvm[d], nv[d], hvmn);
    hvin = fma(a.hv[d], nv[d], hvin);
  }
  const double pa = fma(0.5, pm, a.hp);
  const double fr = rho_ln * van;
  F[0] = fr;
#pragma unroll
  for (int d = 0; d < DIM; ++d) F[1 + d] = fma(fr, va[d], pa * nv[d]);
  F[DIM + 1] = fma(fr, fma(ib_ln, gm1i, hvv), fma(a.p, hvmn, pm * hvin));
}

// Split-form volume sum of one lane on curvilinear elements, directions
// l..DIM-1: acc -= sum_{m != i} D_im F#(U_i, U_m) . (Ja^l_i + Ja^l_m), i.e.
// -2 sum_m D_im F# . {{Ja^l}}_im, over the lane's line along l (partners i+1,
// ..., i+N modulo n; the m = i term is added with the faces).  Ja[l][d] holds
// the lane's own contravariant vectors, J rows the LDS copies of all nodes'.
template <int DIM, int N, int l, bool EXACT, int W>
__device__ __forceinline__ void split_sweep_curv(int tid, const int (&ii)[3], const int (&stride)[3],
                                                 const SplitNode<DIM>& a, const double (*Q)[W],
                                                 const double (*Jm)[W], const double (&Ja)[DIM][DIM],
                                                 const double* sD, double gm1i, bool& far, double (&acc)[DIM + 2]) {
  if constexpr (l < DIM) {
    constexpr int NV = DIM + 2, n = N + 1;
    const int il = ii[l];
    const int st = stride[l];
    const int base = tid - il * st;
    double s[NV];
#pragma unroll
    for (int v = 0; v < NV; ++v) s[v] = 0.0;
    auto term = [&](int k) {
      const int mi = il + k < n ? il + k : il + k - n;
      const int m = base + mi * st;
      double nv[DIM];
#pragma unroll
      for (int d = 0; d < DIM; ++d) nv[d] = Ja[l][d] + Jm[l * DIM + d][m];
      double F[NV];
      ranocha_flux_n<DIM, EXACT>(a, Q, tid, m, nv, gm1i, far, F);
      const double dim = sD[il * n + mi];
#pragma unroll
      for (int v = 0; v < NV; ++v) s[v] = fma(dim, F[v], s[v]);
    };
    if constexpr (EXACT) {  // rare path: partner loop kept rolled
#pragma unroll 1
      for (int k = 1; k <= N; ++k) term(k);
    } else {
#pragma unroll
      for (int k = 1; k <= N; ++k) term(k);
    }
#pragma unroll
    for (int v = 0; v < NV; ++v) acc[v] -= s[v];
    split_sweep_curv<DIM, N, l + 1, EXACT>(tid, ii, stride, a, Q, Jm, Ja, sD, gm1i, far, acc);
  }
}

// The pairwise form of split_sweep_curv for lines inside one wave: each
// unordered pair's flux F# . (Ja^l_i + Ja^l_m) is evaluated once (flux and
// metric sum are both symmetric in the pair) and handed to the partner lane
// by a shuffle, as in split_sweep_pairs.
template <int DIM, int N, int l, int W>
__device__ __forceinline__ void split_sweep_pairs_curv(int tid, const int (&ii)[3], const int (&stride)[3],
                                                       const SplitNode<DIM>& a, const double (*Q)[W],
                                                       const double (*Jm)[W], const double (&Ja)[DIM][DIM],
                                                       const double* sD, double gm1i, bool& far,
                                                       double (&acc)[DIM + 2]) {
  if constexpr (l < DIM) {
    constexpr int NV = DIM + 2, n = N + 1, K1 = (n - 1) / 2;
    const int il = ii[l];
    const int st = stride[l];
    const int base = tid - il * st;
    const int lbase = (tid & 63) - il * st;  // wave lane of the line's node 0
    double s[NV];
#pragma unroll
    for (int v = 0; v < NV; ++v) s[v] = 0.0;
    auto flux = [&](int m, bool& fl, double (&F)[NV]) {
      double nv[DIM];
#pragma unroll
      for (int d = 0; d < DIM; ++d) nv[d] = Ja[l][d] + Jm[l * DIM + d][m];
      ranocha_flux_n<DIM, false>(a, Q, tid, m, nv, gm1i, fl, F);
    };
#pragma unroll
    for (int k = 1; k <= K1; ++k) {
      const int m = il + k < n ? il + k : il + k - n;   // partner evaluated here
      const int j = il - k >= 0 ? il - k : il - k + n;  // partner whose flux arrives
      double F[NV];
      bool fp = false;
      flux(base + m * st, fp, F);
      const double dm = sD[il * n + m];
      const double dj = sD[il * n + j];
      const int src = lbase + j * st;
      const int fr = __shfl(fp ? 1 : 0, src);
#pragma unroll
      for (int v = 0; v < NV; ++v) {
        const double Fr = __shfl(F[v], src);
        s[v] = fma(dm, F[v], s[v]);
        s[v] = fma(dj, Fr, s[v]);
      }
      far = far || fp || fr != 0;
    }
    if constexpr (n % 2 == 0) {
      const int m = il + n / 2 < n ? il + n / 2 : il - n / 2;
      double F[NV];
      flux(base + m * st, far, F);
      const double dm = sD[il * n + m];
#pragma unroll
      for (int v = 0; v < NV; ++v) s[v] = fma(dm, F[v], s[v]);
    }
#pragma unroll
    for (int v = 0; v < NV; ++v) acc[v] -= s[v];
    split_sweep_pairs_curv<DIM, N, l + 1>(tid, ii, stride, a, Q, Jm, Ja, sD, gm1i, far, acc);
  }
}

}  // namespace dg
