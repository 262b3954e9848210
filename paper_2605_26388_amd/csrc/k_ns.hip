// Compressible Navier-Stokes stage with BR1 viscous terms (Kernel
// Architecture for Parabolic Terms: eqs. br1_avg, tau, br1_flux; the BR1
// paragraphs of the strong-form appendix), 3-D affine Cartesian elements.
//
// Two passes per evaluation of L, each finishing before the next:
//   pass 1 (k_br1_face): per element, the lifted gradient S = grad W of the
//     primitive variables W = (rho, u, v, w, T) (only u, v, w, T enter the
//     viscous flux), with the central trace W^ = (W^- + W^+)/2 on every face;
//     then the viscous flux normal to each face, F_v^l(U, S), at the element's
//     own face nodes is written to a face buffer [B][E][2*DIM][n^2][4]
//     (momentum and energy components; the mass component is zero).
//   pass 2 (k_ns_stage): recomputes S at all nodes (again with the neighbour
//     traces), forms the combined flux G^l = F_inv^l - F_v^l, takes its
//     strong-form divergence with the LGL derivative matrix, adds the surface
//     lift of the Rusanov inviscid flux and of the central viscous flux
//     {{F_v}} = (F_v^- + F_v^+)/2 built from the face buffer (both sides read
//     the same two buffer values, so the interface flux is single-valued), and
//     applies the Shu-Osher stage update.
// Closure: non-dimensional R = 1 so T = p / rho; Newtonian stress with the
// Stokes hypothesis; q = -k grad T with k = gamma mu / (Pr (gamma - 1)).
// LDS operands stay in double for both state precisions.
//
// Split form (SPLIT, eq. vol_split with the BR1 terms added, the paper's
// Taylor-Green setting): pass 2 stages only -F_v^l for the D-sweep and the
// primitives of the two-point flux, the inviscid volume term is the split sum
// -2 (2/h_l) sum_m D_im F#_l(U_i, U_m) of the inviscid stage kernel (its m = i
// term added on the face lanes with the own physical flux), and the surfaces
// are unchanged.
//
// Curvilinear elements (CURV; periodic warped meshes): per-node metrics 1/J
// and Ja^l.  The gradient is the strong-form
// operator with the metrics inside the sweep, J S_d = sum_l [sum_m D_im (Ja^l_d
// W)_m + (+-1/w_end) (W^ - W_i) Ja^l_d,i], staged direction by direction
// (twelve products Ja^l_d W_q per node); the face buffer holds the
// contravariant viscous flux Ja^l . F_v of the own face node; pass 2 stages
// G^l = Ja^l . (F_inv - F_v), takes the Rusanov flux along the own node's
// Ja^l (as the curvilinear Euler stage) and the central viscous flux of the
// two buffered contravariant fluxes, and scales by 1/J; with the split form
// it stages -Ja^l . F_v for the sweep and every node's Ja^l for the split sum
// of the curvilinear Euler stage (two-point flux contracted with Ja^l_i +
// Ja^l_m), whose m = i term -2 D_ii Ja^l . F_inv is added on the face lanes.
#include <type_traits>

#include "dg_device.hpp"
#include "dg_split.hpp"

namespace dg {

constexpr int NS_DIM = 3;

// face-node index of node (i, j, k) on a face normal to direction l
template <int n>
__device__ __forceinline__ int face_node(const int (&ii)[3], int l) {
  return l == 0 ? ii[1] + n * ii[2] : (l == 1 ? ii[0] + n * ii[2] : ii[0] + n * ii[1]);
}

// W = (u, v, w, T) from the conserved state (rho is not needed by F_v)
__device__ __forceinline__ void prim_w(const double (&U)[5], double gm1, double (&W)[4]) {
  const double ri = frcp(U[0]);
  double m2 = 0.0;
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    W[d] = U[1 + d] * ri;
    m2 = fma(U[1 + d], U[1 + d], m2);
  }
  const double p = gm1 * fma(-0.5 * m2, ri, U[4]);
  W[3] = p * ri;
}

// Viscous flux along direction l (momentum and energy rows) from the
// velocity, the gradient S[d][q] = d W_q / d x_d and mu, k.
__device__ __forceinline__ void visc_flux(const double (&W)[4], const double (&S)[3][4], int l, double mu, double kc,
                                          double (&Fv)[4]) {
  const double div = S[0][0] + S[1][1] + S[2][2];
  double e = kc * S[l][3];
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    double t = mu * (S[d][l] + S[l][d]);
    if (d == l) t = fma(-2.0 / 3.0 * mu, div, t);
    Fv[d] = t;
    e = fma(W[d], t, e);
  }
  Fv[3] = e;
}

template <int N, typename T, int PASS, bool SPLIT = false, bool CURV = false>
__global__ void __launch_bounds__((Shape<3, N>::BS))
k_ns(StageParams sp, MeshView mv, PhysConst pc, T* face, const double* met) {
  using S = Shape<3, N>;
  constexpr int n = S::n, NP = S::NP, NF = S::NF, EPB = S::EPB, NV = 5;
  using PHYS = EulerPhys<3>;
  constexpr bool SPL = SPLIT && PASS == 2;

  __shared__ double sW[CURV ? 12 : 4][EPB * NP];  // W (curvilinear: Ja^l_d W_q of one direction l)
  __shared__ double sF[PASS == 2 ? 3 : 1][NV][PASS == 2 ? EPB * NP : 1];
  __shared__ double sD[n * n];
  __shared__ double sQ[SPL ? 8 : 1][SPL ? EPB * NP : 1];  // split form: rho/2, v/2, p, rho/(2p), ln rho, ln(rho/p)
  __shared__ double sJ[SPL && CURV ? 9 : 1][SPL && CURV ? EPB * NP : 1];  // curvilinear split: Ja^l_d, row 3l + d
  __shared__ int sFar;

  const int tid = threadIdx.x;
  // the lane's entry of D, written to LDS only before the first barrier
  static_assert(n * n <= S::BS, "one D entry per lane");
  const double dval = tid < n * n ? mv.K->D[tid] : 0.0;

  const int E = mv.E;
  const int nEB = (E + EPB - 1) / EPB;
  const int blk = xcd_remap(blockIdx.x, gridDim.x);
  const int b = blk / nEB;
  const int eb = blk - b * nEB;
  const int el = tid / NP;
  const int node = tid - el * NP;
  const int e = eb * EPB + el;
  const bool active = (tid < S::NT) && (e < E);
  const int ec = active ? e : 0;
  int ii[3];
  ii[0] = node % n;
  ii[1] = (node / n) % n;
  ii[2] = node / (n * n);
  const int stride[3] = {1, n, n * n};

  // Element tables before any store or atomic (scalar loads, no mid-kernel
  // waits): neighbours, scales 2/h, 1/w_end.
  const int* nb = mv.nbr + (size_t)ec * 6;
  int nbl[6];
#pragma unroll
  for (int q = 0; q < 6; ++q) nbl[q] = nb[q];
  double g[3];
#pragma unroll
  for (int l = 0; l < 3; ++l) g[l] = mv.geo[(size_t)ec * 4 + l];
  const double winv = mv.K->wend_inv;

  const size_t plane = (size_t)E * NP;
  const size_t pbytes = plane * sizeof(T);
  const T* Ub = static_cast<const T*>(sp.Uk) + (size_t)b * NV * plane;
  rsrc_t rU[NV];
#pragma unroll
  for (int v = 0; v < NV; ++v) rU[v] = make_rsrc(Ub + v * plane, pbytes);
  const unsigned off = (unsigned)(ec * NP + node);
  double u[NV];
#pragma unroll
  for (int v = 0; v < NV; ++v) u[v] = Buf<T>::load(rU[v], off);

  int side[3], nbe[3];
  double un[3][NV];
#pragma unroll
  for (int l = 0; l < 3; ++l) {
    side[l] = (ii[l] == 0) ? 0 : ((ii[l] == N) ? 1 : -1);
    nbe[l] = (active && side[l] >= 0) ? nbl[2 * l + side[l]] : -1;
    if (nbe[l] >= 0) {
      const unsigned noff = (unsigned)(nbe[l] * NP + node + (side[l] ? -N : N) * stride[l]);
#pragma unroll
      for (int v = 0; v < NV; ++v) un[l][v] = Buf<T>::load(rU[v], noff);
    }
  }
  const bool use_u0 = (PASS == 2) && (sp.mode != 0) && (sp.a != 0.0);

  const double gm1 = pc.gamma - 1.0;
  const double mu = pc.mu;
  const double kc = pc.gamma * pc.mu / (pc.prandtl * gm1);
  // curvilinear: the node's 1/J and Ja^l_d (shared by all batch members)
  double jinv = 0.0, Ja[3][3] = {};
  if constexpr (CURV) {
    const size_t at = (size_t)ec * NP + node;
    jinv = met[plane + at];
#pragma unroll
    for (int l = 0; l < 3; ++l)
#pragma unroll
      for (int d = 0; d < 3; ++d) Ja[l][d] = met[(2 + l * 3 + d) * plane + at];
  }
  double W[4];
  prim_w(u, gm1, W);
  if (tid < n * n) sD[tid] = dval;
  if (!CURV && tid < S::NT) {
#pragma unroll
    for (int q = 0; q < 4; ++q) sW[q][tid] = W[q];
  }
  __syncthreads();

  // ---- lifted gradient S[l][q] = dW_q / dx_l --------------------------------
  double Sg[3][4];
#pragma unroll
  for (int l = 0; l < 3; ++l)
#pragma unroll
    for (int q = 0; q < 4; ++q) Sg[l][q] = 0.0;
  if constexpr (CURV) {
    // J S_d = sum_l [D (Ja^l_d W) + lift_l((W^ - W) Ja^l_d)], one direction at a time
#pragma unroll
    for (int l = 0; l < 3; ++l) {
      if (tid < S::NT) {
#pragma unroll
        for (int d = 0; d < 3; ++d)
#pragma unroll
          for (int q = 0; q < 4; ++q) sW[d * 4 + q][tid] = Ja[l][d] * W[q];
      }
      __syncthreads();
      if (tid < S::NT) {
        const int il = ii[l], st = stride[l];
        const int base = tid - il * st;
        double dr[n];
#pragma unroll
        for (int m = 0; m < n; ++m) dr[m] = sD[il * n + m];
#pragma unroll
        for (int d = 0; d < 3; ++d)
#pragma unroll
          for (int q = 0; q < 4; ++q) {
            double s = 0.0;
#pragma unroll
            for (int m = 0; m < n; ++m) s = fma(dr[m], sW[d * 4 + q][base + m * st], s);
            Sg[d][q] += s;
          }
        if (nbe[l] >= 0) {
          double Wn[4];
          prim_w(un[l], gm1, Wn);
          const double c = (side[l] ? 0.5 : -0.5) * winv;
#pragma unroll
          for (int d = 0; d < 3; ++d) {
            const double cd = c * Ja[l][d];
#pragma unroll
            for (int q = 0; q < 4; ++q) Sg[d][q] = fma(cd, Wn[q] - W[q], Sg[d][q]);
          }
        }
      }
      __syncthreads();  // the next direction overwrites the staged products
    }
#pragma unroll
    for (int d = 0; d < 3; ++d)
#pragma unroll
      for (int q = 0; q < 4; ++q) Sg[d][q] *= jinv;
  } else if (tid < S::NT) {
#pragma unroll
    for (int l = 0; l < 3; ++l) {
      const int il = ii[l], st = stride[l];
      const int base = tid - il * st;
      double dr[n];
#pragma unroll
      for (int m = 0; m < n; ++m) dr[m] = sD[il * n + m];
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        double s = 0.0;
#pragma unroll
        for (int m = 0; m < n; ++m) s = fma(dr[m], sW[q][base + m * st], s);
        Sg[l][q] = s;
      }
      if (nbe[l] >= 0) {
        // W^ - W_own = (W_nbr - W_own)/2; + on the upper face, - on the lower
        double Wn[4];
        prim_w(un[l], gm1, Wn);
        const double c = (side[l] ? 0.5 : -0.5) * winv;
#pragma unroll
        for (int q = 0; q < 4; ++q) Sg[l][q] = fma(c, Wn[q] - W[q], Sg[l][q]);
      }
#pragma unroll
      for (int q = 0; q < 4; ++q) Sg[l][q] *= g[l];
    }
  }

  if constexpr (PASS == 1) {
    // normal viscous flux at the element's own face nodes -> face buffer
    if (active) {
      double Fa[CURV ? 3 : 1][4];  // curvilinear: F_v along every physical direction
      if constexpr (CURV) {
#pragma unroll
        for (int d = 0; d < 3; ++d) visc_flux(W, Sg, d, mu, kc, Fa[d]);
      }
#pragma unroll
      for (int l = 0; l < 3; ++l) {
        if (side[l] < 0) continue;
        double Fv[4];
        if constexpr (CURV) {
#pragma unroll
          for (int c = 0; c < 4; ++c) Fv[c] = Ja[l][0] * Fa[0][c] + Ja[l][1] * Fa[1][c] + Ja[l][2] * Fa[2][c];
        } else {
          visc_flux(W, Sg, l, mu, kc, Fv);
        }
        const int f = 2 * l + side[l];
        T* dst = face + ((((size_t)b * E + e) * 6 + f) * NF + face_node<n>(ii, l)) * 4;
#pragma unroll
        for (int q = 0; q < 4; ++q) dst[q] = static_cast<T>(Fv[q]);
      }
    }
    return;
  } else {
    // ---- combined flux G^l = F_inv^l - F_v^l in LDS -------------------------
    Thermo th;
    const bool ok = PHYS::thermo(u, th, pc);
    if (active && !ok)
      report_nonphysical(mv.counters, mv.first_bad, ((unsigned long long)b * E + e) * NP + node);
    double vel[3];
#pragma unroll
    for (int d = 0; d < 3; ++d) vel[d] = u[1 + d] * th.ri;
    SplitNode<3> own;
    if (CURV && tid < S::NT) {
      double Fa[3][4];
#pragma unroll
      for (int d = 0; d < 3; ++d) visc_flux(W, Sg, d, mu, kc, Fa[d]);
#pragma unroll
      for (int l = 0; l < 3; ++l) {
        double F[NV];
        if constexpr (SPL) {  // only -Ja^l . F_v goes through the D sweep; Ja^l for the partners
          sF[l][0][tid] = 0.0;
#pragma unroll
          for (int q = 0; q < 4; ++q)
            sF[l][1 + q][tid] = -(Ja[l][0] * Fa[0][q] + Ja[l][1] * Fa[1][q] + Ja[l][2] * Fa[2][q]);
#pragma unroll
          for (int d = 0; d < 3; ++d) sJ[3 * l + d][tid] = Ja[l][d];
        } else {
          normal_flux<3>(u, vel, th.p, Ja[l], F);
          sF[l][0][tid] = F[0];
#pragma unroll
          for (int q = 0; q < 4; ++q)
            sF[l][1 + q][tid] = F[1 + q] - (Ja[l][0] * Fa[0][q] + Ja[l][1] * Fa[1][q] + Ja[l][2] * Fa[2][q]);
        }
      }
    } else if (tid < S::NT) {
#pragma unroll
      for (int l = 0; l < 3; ++l) {
        double F[NV], Fv[4];
        visc_flux(W, Sg, l, mu, kc, Fv);
        if constexpr (SPL) {
          sF[l][0][tid] = 0.0;
#pragma unroll
          for (int q = 0; q < 4; ++q) sF[l][1 + q][tid] = -Fv[q];
        } else {
          PHYS::flux(u, vel[l], th.p, l, F);
          sF[l][0][tid] = F[0];
#pragma unroll
          for (int q = 0; q < 4; ++q) sF[l][1 + q][tid] = F[1 + q] - Fv[q];
        }
      }
    }
    if constexpr (SPL) {
      own.hr = 0.5 * u[0];
#pragma unroll
      for (int d = 0; d < 3; ++d) {
        own.v[d] = vel[d];
        own.hv[d] = 0.5 * vel[d];
      }
      own.p = th.p;
      own.hp = 0.5 * th.p;
      own.hb = 0.5 * (u[0] * frcp(th.p));
      if (tid < S::NT) {
        sQ[0][tid] = own.hr;
#pragma unroll
        for (int d = 0; d < 3; ++d) sQ[1 + d][tid] = own.hv[d];
        sQ[4][tid] = own.p;
        sQ[5][tid] = own.hb;
      }
      if (tid == 0) sFar = 0;
    }
    __syncthreads();
    double acc[NV];
#pragma unroll
    for (int v = 0; v < NV; ++v) acc[v] = 0.0;
    if constexpr (SPL) {
      // inviscid volume term: the split sum (the exact log means for the
      // lanes with a far pair, as in the inviscid stage kernel)
      const double gm1i = 1.0 / gm1;
      bool far = false;
      if (tid < S::NT) {
        if constexpr (CURV)
          split_sweep_curv<3, N, 0, false>(tid, ii, stride, own, sQ, sJ, Ja, sD, gm1i, far, acc);
        else if constexpr (S::BS == 64)
          split_sweep_pairs<3, N, 0>(tid, ii, stride, own, sQ, sD, g, gm1i, far, acc);
        else
          split_sweep<3, N, 0, false>(tid, ii, stride, own, sQ, sD, g, gm1i, far, acc);
      }
      if (far) sFar = 1;
      __syncthreads();
      if (sFar) {
        if (tid < S::NT) {
          sQ[6][tid] = log(u[0]);
          sQ[7][tid] = log(2.0 * own.hb);
        }
        __syncthreads();
        if (far) {
#pragma unroll
          for (int v = 0; v < NV; ++v) acc[v] = 0.0;
          if constexpr (CURV)
            split_sweep_curv<3, N, 0, true>(tid, ii, stride, own, sQ, sJ, Ja, sD, gm1i, far, acc);
          else
            split_sweep<3, N, 0, true>(tid, ii, stride, own, sQ, sD, g, gm1i, far, acc);
        }
      }
    }
    if (tid < S::NT) {
#pragma unroll
      for (int l = 0; l < 3; ++l) {
        const int il = ii[l], st = stride[l];
        const int base = tid - il * st;
        double dr[n];
#pragma unroll
        for (int m = 0; m < n; ++m) dr[m] = CURV ? -sD[il * n + m] : sD[il * n + m] * (-g[l]);
#pragma unroll
        for (int v = 0; v < NV; ++v) {
          double s = 0.0;
#pragma unroll
          for (int m = 0; m < n; ++m) s = fma(dr[m], sF[l][v][base + m * st], s);
          acc[v] += s;
        }
      }
    }
    // ---- surface terms ----------------------------------------------------------
    bool on_face = side[0] >= 0 || side[1] >= 0 || side[2] >= 0;
    if (active && on_face) {
      const double aown = sound<PHYS>(th);
#pragma unroll
      for (int l = 0; l < 3; ++l) {
        if (side[l] < 0) continue;
        // the two buffered viscous face fluxes of this face, loaded only here
        // and U0 only for the output: held from the start, with the neighbour
        // states, they kept pass 2 at 3 waves per SIMD instead of 4 (measured
        // 3-9 % slower)
        double fvo_l[4], fvn_l[4];
        {
          const int q = face_node<n>(ii, l);
          const size_t own = ((((size_t)b * E + ec) * 6 + 2 * l + side[l]) * NF + q) * 4;
          const size_t oth = nbe[l] >= 0 ? ((((size_t)b * E + nbe[l]) * 6 + 2 * l + 1 - side[l]) * NF + q) * 4 : own;
#pragma unroll
          for (int c = 0; c < 4; ++c) {
            fvo_l[c] = static_cast<double>(face[own + c]);
            fvn_l[c] = static_cast<double>(face[oth + c]);
          }
        }
        // Rusanov as a difference to the own flux, 2 (F* - F_own) =
        // (F_nb - F_own) - s lam (U_nb - U_own), s = +1 on the +xi_l face;
        // the central viscous flux likewise, 2 ({{F_v}} - F_v,own) = F_v,nb - F_v,own.
        double Fo[NV], Fn[NV], Dv[NV];
        Thermo tn;
        PHYS::thermo(un[l], tn, pc);
        double hs;
        if constexpr (CURV) {  // Rusanov along the own node's Ja^l (|Ja^l| times the unit-normal flux)
          double vnv[3];
#pragma unroll
          for (int d = 0; d < 3; ++d) vnv[d] = un[l][1 + d] * tn.ri;
          normal_flux<3>(u, vel, th.p, Ja[l], Fo);
          normal_flux<3>(un[l], vnv, tn.p, Ja[l], Fn);
          double nrm2 = 0.0, vo = 0.0, vg = 0.0;
#pragma unroll
          for (int d = 0; d < 3; ++d) {
            nrm2 = fma(Ja[l][d], Ja[l][d], nrm2);
            vo = fma(vel[d], Ja[l][d], vo);
            vg = fma(vnv[d], Ja[l][d], vg);
          }
          const double nmag = fsqrt(nrm2);
          const double nmi = frcp(nmag);
          const double co = fabs(vo) * nmi + aown;
          const double cn = fabs(vg) * nmi + sound<PHYS>(tn);
          const double lam = co >= cn ? co : cn;
          hs = (side[l] ? lam : -lam) * nmag;
        } else {
          PHYS::flux(u, vel[l], th.p, l, Fo);
          const double vn = un[l][1 + l] * tn.ri;
          PHYS::flux(un[l], vn, tn.p, l, Fn);
          const double co = fabs(vel[l]) + aown;
          const double cn = fabs(vn) + sound<PHYS>(tn);
          const double lam = co >= cn ? co : cn;
          hs = side[l] ? lam : -lam;
        }
#pragma unroll
        for (int v = 0; v < NV; ++v) Dv[v] = fma(-hs, un[l][v] - u[v], Fn[v] - Fo[v]);
        const double sc = (side[l] ? -1.0 : 1.0) * (CURV ? 1.0 : g[l]) * (0.5 * winv);
        acc[0] = fma(sc, Dv[0], acc[0]);
#pragma unroll
        for (int c = 0; c < 4; ++c) acc[1 + c] = fma(sc, Dv[1 + c] - (fvn_l[c] - fvo_l[c]), acc[1 + c]);
        if constexpr (SPL) {
          // the split sum's m = i term, 2 D_ii F_l(U_i)
          const double cd = -2.0 * (CURV ? 1.0 : g[l]) * sD[ii[l] * (n + 1)];
#pragma unroll
          for (int v = 0; v < NV; ++v) acc[v] = fma(cd, Fo[v], acc[v]);
        }
      }
    }
    if constexpr (CURV) {
#pragma unroll
      for (int v = 0; v < NV; ++v) acc[v] *= jinv;
    }
    if (active) {
      T* outb = static_cast<T*>(sp.out) + (size_t)b * NV * plane;
      double u0[NV];
      if (use_u0) {
        const T* U0b = static_cast<const T*>(sp.U0) + (size_t)b * NV * plane;
#pragma unroll
        for (int v = 0; v < NV; ++v) u0[v] = Buf<T>::load(make_rsrc(U0b + v * plane, pbytes), off);
      }
      double r[NV];
#pragma unroll
      for (int v = 0; v < NV; ++v) {
        r[v] = acc[v];
        if (sp.mode != 0) {
          r[v] = fma(sp.c, acc[v], sp.b * u[v]);
          if (use_u0) r[v] = fma(sp.a, u0[v], r[v]);
        }
      }
      if (sp.mode != 0 && (sp.rho_min > 0.0 || sp.p_min > 0.0))
        positivity_floor(r, sp.rho_min, sp.p_min, 1.0 / gm1, mv.counters);
#pragma unroll
      for (int v = 0; v < NV; ++v) Buf<T>::store(make_rsrc(outb + v * plane, pbytes), off, r[v]);
      if (sp.mode == 2) {  // second combination of the same L(Uk), no floor
        T* out2 = static_cast<T*>(sp.out2) + (size_t)b * NV * plane;
        const T* Vb = static_cast<const T*>(sp.a2 != 0.0 ? sp.V : sp.Uk) + (size_t)b * NV * plane;
#pragma unroll
        for (int v = 0; v < NV; ++v) {
          double w = fma(sp.c2, acc[v], sp.b2 * u[v]);
          if (sp.a2 != 0.0) w = fma(sp.a2, Buf<T>::load(make_rsrc(Vb + v * plane, pbytes), off), w);
          Buf<T>::store(make_rsrc(out2 + v * plane, pbytes), off, w);
        }
      }
    }
  }
}

template <int N, typename T>
static hipError_t ns_go(const Ctx& c, const StageParams& sp, hipStream_t s) {
  using SH = Shape<3, N>;
  const int nEB = (c.E + SH::EPB - 1) / SH::EPB;
  const int nblk = nEB * c.B;
  T* face = static_cast<T*>(c.d_face);
  const MeshView mv = mesh_view(c);
  if (c.curv) {
    hipLaunchKernelGGL((k_ns<N, T, 1, false, true>), dim3(nblk), dim3(SH::BS), 0, s, sp, mv, c.pc, face, c.d_met);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    if (c.desc.volume == DG_VOLUME_SPLIT)
      hipLaunchKernelGGL((k_ns<N, T, 2, true, true>), dim3(nblk), dim3(SH::BS), 0, s, sp, mv, c.pc, face, c.d_met);
    else
      hipLaunchKernelGGL((k_ns<N, T, 2, false, true>), dim3(nblk), dim3(SH::BS), 0, s, sp, mv, c.pc, face, c.d_met);
    return hipGetLastError();
  }
  hipLaunchKernelGGL((k_ns<N, T, 1>), dim3(nblk), dim3(SH::BS), 0, s, sp, mv, c.pc, face, nullptr);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  if (c.desc.volume == DG_VOLUME_SPLIT)
    hipLaunchKernelGGL((k_ns<N, T, 2, true>), dim3(nblk), dim3(SH::BS), 0, s, sp, mv, c.pc, face, nullptr);
  else
    hipLaunchKernelGGL((k_ns<N, T, 2>), dim3(nblk), dim3(SH::BS), 0, s, sp, mv, c.pc, face, nullptr);
  return hipGetLastError();
}

template <typename T>
static hipError_t ns_t(const Ctx& c, const StageParams& sp, hipStream_t s) {
  switch (c.N) {
    case 2: return ns_go<2, T>(c, sp, s);
    case 3: return ns_go<3, T>(c, sp, s);
    case 4: return ns_go<4, T>(c, sp, s);
  }
  return hipErrorNotSupported;
}

hipError_t launch_ns(const Ctx& c, const StageParams& sp, hipStream_t s) {
  return c.desc.precision == DG_F32 ? ns_t<float>(c, sp, s) : ns_t<double>(c, sp, s);
}

}  // namespace dg
