// Fused DGSEM stage for the Euler equations on curvilinear elements with
// boundary fluxes (Kernel Architecture for Hyperbolic Terms: element map
// x = X(xi), per-node Jacobian J and contravariant vectors Ja^l satisfying the
// discrete GCL, contravariant fluxes Ja^l . F; boundary fluxes per type).
//
// One lane per node, EPB elements per workgroup, as the Cartesian stage:
//   1. load U_k, the node's 1/J and Ja^l (metric planes, coalesced);
//   2. volume integral: contravariant fluxes Ft^l = Ja^l . F (written as
//      rho v_n, m v_n + p n, (E + p) v_n with n = Ja^l) staged through LDS and
//      swept with D, -sum_l sum_m D_im Ft^l_m;
//   3. faces: a lane on the +-xi_l face takes the normal n = Ja^l of its own
//      node and applies the Rusanov flux as a difference to its own
//      contravariant flux,
//         2 (F* - Ft_own) = (Ft_nb - Ft_own) - s lam |n| (U_nb - U_own),
//         lam = max(|v_own . n^| + a_own, |v_nb . n^| + a_nb),
//      s = +1 on the +xi_l face, -1 on the -xi_l face, with U_nb the
//      neighbour's matching node or, on a box side, the boundary state: the
//      mirrored state (rho, m - 2 (m . n^) n^, E) for a slip wall; a
//      supersonic inflow takes F* = n . F(U_bc) and a supersonic outflow
//      F* = Ft_own (no correction);
//   4. dU = (volume + lift) / J, or the stage combination (positivity floor
//      and dual output as the Cartesian stage).
// Split form (SPLIT, eq. vol_split on curvilinear elements): step 2 stages
// the primitives of the two-point flux and every node's Ja^l in LDS instead,
// and the volume term is -sum_l sum_{m != i} D_im F#(U_i, U_m) . (Ja^l_i +
// Ja^l_m), Ranocha's flux contracted with twice the pair's averaged
// contravariant vector (the log means by the series of the Cartesian split
// kernel, with the same exact redo for widely separated pairs); its m = i term
// -2 D_ii Ft^l(U_i) is added on the face lanes, whose own flux Ft^l is then
// evaluated in registers; the surface term is unchanged.
// FP32 form (T = float): the state is read and written in float; all
// arithmetic, the metrics and the LDS tiles stay in double.
#include <type_traits>

#include "dg_device.hpp"
#include "dg_split.hpp"

namespace dg {

struct CurvArgs {
  const double* met;  // [2 + dim*dim][E*Np]: J, 1/J, Ja^l_d at plane 2 + l*dim + d
  double ub[5];       // conserved inflow state
};

// NT: the stage's streams (state arrays and metrics) together exceed the
// Infinity Cache: U0 and the outputs, which no other workgroup of the stage
// reads, then carry the non-temporal hint so that they do not displace the
// metrics and U_k's neighbour faces
template <int DIM, int N, bool SPLIT, typename T, bool NT = false>
__global__ void __launch_bounds__((Shape<DIM, N>::BS)) __attribute__((amdgpu_waves_per_eu(3)))
k_stage_curv(StageParams sp, MeshView mv, PhysConst pc, CurvArgs ca) {
  using S = Shape<DIM, N>;
  using PHYS = EulerPhys<DIM>;
  constexpr int n = S::n, NP = S::NP, EPB = S::EPB, NV = DIM + 2;
  constexpr bool UNIFORM_ELEM = (NP % 64) == 0;
  constexpr int W = EPB * NP;

  __shared__ double sF[SPLIT ? 1 : DIM][SPLIT ? 1 : NV][SPLIT ? 1 : W];
  __shared__ double sQ[SPLIT ? DIM + 5 : 1][SPLIT ? W : 1];    // rho/2, v/2, p, rho/(2p), ln rho, ln(rho/p)
  __shared__ double sJ[SPLIT ? DIM * DIM : 1][SPLIT ? W : 1];  // Ja^l_d of every node, row l*DIM + d
  __shared__ int sFar;  // some lane of the block needs the exact log means
  __shared__ double sD[n * n];

  const int tid = threadIdx.x;
  static_assert(n * n <= S::BS, "one D entry per lane");
  const double dval = tid < n * n ? mv.K->D[tid] : 0.0;
  // 3-D, N = 3 (one element per wave): the standard volume sweep runs on the
  // FP64 matrix core as in the Cartesian stage kernel, whose header describes
  // the lane layout; A operand -D[i][k] on lane i + 4b + 16k
  constexpr bool MMA = (DIM == 3 && N == 3 && !SPLIT);
  const double dA = MMA ? -mv.K->D[(tid & 3) * n + (tid >> 4)] : 0.0;

  const int E = mv.E;
  const int nEB = (E + EPB - 1) / EPB;
  const int blk = xcd_remap(blockIdx.x, gridDim.x);
  const int b = blk / nEB;
  const int eb = blk - b * nEB;
  const int el = tid / NP;
  const int node = tid - el * NP;
  const int e = eb * EPB + el;
  const bool active = (tid < S::NT) && (e < E);
  int ec = active ? e : 0;  // clamped for address arithmetic only
  if constexpr (UNIFORM_ELEM) ec = wave_uniform(ec);

  const int* nb = mv.nbr + (size_t)ec * 2 * DIM;
  int nbl[2 * DIM];
#pragma unroll
  for (int q = 0; q < 2 * DIM; ++q) nbl[q] = nb[q];
  const double hwinv = 0.5 * mv.K->wend_inv;

  int ii[3];
  ii[0] = node % n;
  ii[1] = (node / n) % n;
  ii[2] = node / (n * n);
  const int stride[3] = {1, n, n * n};

  const size_t plane = (size_t)E * NP;
  const size_t abytes = (size_t)NV * plane * sizeof(T);
  const unsigned pstride = (unsigned)(plane * sizeof(T));
  const rsrc_t rU = make_rsrc(static_cast<const T*>(sp.Uk) + (size_t)b * NV * plane, abytes);
  const unsigned off = (unsigned)(ec * NP + node);

  double u[NV];
#pragma unroll
  for (int v = 0; v < NV; ++v) u[v] = Buf<T>::load(rU, off, v * pstride);
  // metrics of the own node (shared by all batch members)
  const size_t at = (size_t)ec * NP + node;
  const double jinv = ca.met[plane + at];
  double Ja[DIM][DIM];
#pragma unroll
  for (int l = 0; l < DIM; ++l)
#pragma unroll
    for (int d = 0; d < DIM; ++d) Ja[l][d] = ca.met[(2 + l * DIM + d) * plane + at];

  const bool use_u0 = (sp.mode != 0) && (sp.a != 0.0);
  constexpr int CP = NT ? CPOL_NT : 0;  // policy of U0 and the outputs

  Thermo th;
  const bool ok = PHYS::thermo(u, th, pc);
  if (active && !ok)
    report_nonphysical(mv.counters, mv.first_bad, ((unsigned long long)b * E + e) * NP + node);
  double vel[DIM];
#pragma unroll
  for (int d = 0; d < DIM; ++d) vel[d] = u[1 + d] * th.ri;

  // ---- contravariant fluxes (split form: primitives and metrics) in LDS ------
  if (tid < n * n) sD[tid] = dval;
  SplitNode<DIM> own;
  if constexpr (SPLIT) {
    own.hr = 0.5 * u[0];
#pragma unroll
    for (int d = 0; d < DIM; ++d) {
      own.v[d] = vel[d];
      own.hv[d] = 0.5 * vel[d];
    }
    own.p = th.p;
    own.hp = 0.5 * th.p;
    own.hb = 0.5 * (u[0] * frcp(th.p));
    if (tid < S::NT) {
      sQ[0][tid] = own.hr;
#pragma unroll
      for (int d = 0; d < DIM; ++d) sQ[1 + d][tid] = own.hv[d];
      sQ[DIM + 1][tid] = own.p;
      sQ[DIM + 2][tid] = own.hb;
#pragma unroll
      for (int l = 0; l < DIM; ++l)
#pragma unroll
        for (int d = 0; d < DIM; ++d) sJ[l * DIM + d][tid] = Ja[l][d];
    }
    if (tid == 0) sFar = 0;
  } else if (tid < S::NT) {
#pragma unroll
    for (int l = 0; l < DIM; ++l) {
      double F[NV];
      normal_flux<DIM>(u, vel, th.p, Ja[l], F);
#pragma unroll
      for (int v = 0; v < NV; ++v) sF[l][v][tid] = F[v];
    }
  }
  __syncthreads();

  // ---- volume integral: -sum_l sum_m D_im Ft^l_m ----------------------------
  double acc[NV];
#pragma unroll
  for (int v = 0; v < NV; ++v) acc[v] = 0.0;
  if constexpr (SPLIT) {
    const double gm1i = 1.0 / (pc.gamma - 1.0);
    bool far = false;
    if (tid < S::NT) {
      if constexpr (S::BS == 64)  // lines inside one wave: each pair once, handed over by a shuffle
        split_sweep_pairs_curv<DIM, N, 0>(tid, ii, stride, own, sQ, sJ, Ja, sD, gm1i, far, acc);
      else
        split_sweep_curv<DIM, N, 0, false>(tid, ii, stride, own, sQ, sJ, Ja, sD, gm1i, far, acc);
    }
    if (far) sFar = 1;
    __syncthreads();
    if (sFar) {  // block-uniform: some pair is too far apart for the series
      if (tid < S::NT) {
        sQ[DIM + 3][tid] = log(u[0]);
        sQ[DIM + 4][tid] = log(2.0 * own.hb);
      }
      __syncthreads();
      if (far) {  // only the lanes that flagged a far pair redo their sum
#pragma unroll
        for (int v = 0; v < NV; ++v) acc[v] = 0.0;
        split_sweep_curv<DIM, N, 0, true>(tid, ii, stride, own, sQ, sJ, Ja, sD, gm1i, far, acc);
      }
    }
  } else if constexpr (MMA) {
    // z: the lane's own flux is the B operand; x (y): the flux of the node
    // whose lane bits 0-1 (2-3) and 4-5 are swapped, the result fetched back
    // from that lane (both swaps are their own inverse)
    const int tx = (tid >> 4) | (tid & 12) | ((tid & 3) << 4);
    const int ty = (tid & 3) | ((tid >> 4) << 2) | (((tid >> 2) & 3) << 4);
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      acc[v] = __builtin_amdgcn_mfma_f64_4x4x4f64(dA, sF[2][v][tid], acc[v], 0, 0, 0);
      acc[v] += lane_fetch(tx, __builtin_amdgcn_mfma_f64_4x4x4f64(dA, sF[0][v][tx], 0.0, 0, 0, 0));
      acc[v] += lane_fetch(ty, __builtin_amdgcn_mfma_f64_4x4x4f64(dA, sF[1][v][ty], 0.0, 0, 0, 0));
    }
  } else if (tid < S::NT) {
#pragma unroll
    for (int l = 0; l < DIM; ++l) {
      const int il = ii[l];
      const int st = stride[l];
      const int base = tid - il * st;
      double drow[n];
#pragma unroll
      for (int m = 0; m < n; ++m) drow[m] = sD[il * n + m];
#pragma unroll
      for (int v = 0; v < NV; ++v) {
        double s = 0.0;
#pragma unroll
        for (int m = 0; m < n; ++m) s = fma(drow[m], sF[l][v][base + m * st], s);
        acc[v] -= s;
      }
    }
  }

  // Neighbour's matching node on conforming faces (lanes on a face only),
  // loaded after the volume sweep and U0 only for the output: held from the
  // start they would stay live in registers through the sweep.
  int side[DIM];
  double un[DIM][NV];
#pragma unroll
  for (int l = 0; l < DIM; ++l) {
    side[l] = (ii[l] == 0) ? 0 : ((ii[l] == N) ? 1 : -1);
    const int ne = side[l] >= 0 ? nbl[2 * l + side[l]] : -1;
    if (ne >= 0) {
      const int shift = side[l] == 1 ? -N : N;
      const unsigned noff = (unsigned)(ne * NP + node + shift * stride[l]);
#pragma unroll
      for (int v = 0; v < NV; ++v) un[l][v] = Buf<T>::load(rU, noff, v * pstride);
    } else {
#pragma unroll
      for (int v = 0; v < NV; ++v) un[l][v] = u[v];
    }
  }

  // ---- surface lift ----------------------------------------------------------
  const double aown = sound<PHYS>(th);
#pragma unroll
  for (int l = 0; l < DIM; ++l) {
    if (side[l] < 0) continue;  // lanes not on a face in direction l
    const int code = nbl[2 * l + side[l]];
    double Fo[NV];
    if constexpr (SPLIT) {
      normal_flux<DIM>(u, vel, th.p, Ja[l], Fo);
      // the split sum's m = i term, -2 D_ii Ft^l(U_i) (D_ii = 0 off the faces)
      const double cd = -2.0 * sD[ii[l] * (n + 1)];
#pragma unroll
      for (int v = 0; v < NV; ++v) acc[v] = fma(cd, Fo[v], acc[v]);
    } else {
#pragma unroll
      for (int v = 0; v < NV; ++v) Fo[v] = sF[l][v][tid < S::NT ? tid : 0];
    }
    if (code == -(1 + DG_BC_OUTFLOW)) continue;  // F* = own flux
    double nrm2 = 0.0;
#pragma unroll
    for (int d = 0; d < DIM; ++d) nrm2 = fma(Ja[l][d], Ja[l][d], nrm2);
    const double nmag = fsqrt(nrm2);
    const double nmi = frcp(nmag);
    double Dv[NV];
    if (code == -(1 + DG_BC_INFLOW)) {
      double ub[NV];
#pragma unroll
      for (int v = 0; v < NV; ++v) ub[v] = ca.ub[v];
      Thermo tb;
      PHYS::thermo(ub, tb, pc);
      double vb[DIM], Fb[NV];
#pragma unroll
      for (int d = 0; d < DIM; ++d) vb[d] = ub[1 + d] * tb.ri;
      normal_flux<DIM>(ub, vb, tb.p, Ja[l], Fb);
#pragma unroll
      for (int v = 0; v < NV; ++v) Dv[v] = 2.0 * (Fb[v] - Fo[v]);
    } else {
      double ug[NV];
      if (code >= 0) {
#pragma unroll
        for (int v = 0; v < NV; ++v) ug[v] = un[l][v];
      } else {  // slip wall: mirrored state
        double mn = 0.0;
#pragma unroll
        for (int d = 0; d < DIM; ++d) mn = fma(u[1 + d], Ja[l][d], mn);
        mn *= nmi;
        ug[0] = u[0];
#pragma unroll
        for (int d = 0; d < DIM; ++d) ug[1 + d] = fma(-2.0 * mn, Ja[l][d] * nmi, u[1 + d]);
        ug[DIM + 1] = u[DIM + 1];
      }
      Thermo tn;
      PHYS::thermo(ug, tn, pc);
      double vn[DIM], Fn[NV];
#pragma unroll
      for (int d = 0; d < DIM; ++d) vn[d] = ug[1 + d] * tn.ri;
      normal_flux<DIM>(ug, vn, tn.p, Ja[l], Fn);
      double vo = 0.0, vg = 0.0;
#pragma unroll
      for (int d = 0; d < DIM; ++d) {
        vo = fma(vel[d], Ja[l][d], vo);
        vg = fma(vn[d], Ja[l][d], vg);
      }
      const double co = fabs(vo) * nmi + aown;
      const double cg = fabs(vg) * nmi + sound<PHYS>(tn);
      const double lam = co >= cg ? co : cg;
      const double hs = (side[l] == 1 ? lam : -lam) * nmag;
#pragma unroll
      for (int v = 0; v < NV; ++v) Dv[v] = fma(-hs, ug[v] - u[v], Fn[v] - Fo[v]);
    }
    const double sc = side[l] == 1 ? -hwinv : hwinv;
#pragma unroll
    for (int v = 0; v < NV; ++v) acc[v] = fma(sc, Dv[v], acc[v]);
  }

  // ---- output ----------------------------------------------------------------
  if (active) {
#pragma unroll
    for (int v = 0; v < NV; ++v) acc[v] *= jinv;
    const rsrc_t ro = make_rsrc(static_cast<T*>(sp.out) + (size_t)b * NV * plane, abytes);
    if (sp.mode == 0) {
#pragma unroll
      for (int v = 0; v < NV; ++v) Buf<T>::template store<CP>(ro, off, acc[v], v * pstride);
    } else {
      double u0[NV];
      if (use_u0) {
        const rsrc_t r0 = make_rsrc(static_cast<const T*>(sp.U0) + (size_t)b * NV * plane, abytes);
#pragma unroll
        for (int v = 0; v < NV; ++v) u0[v] = Buf<T>::template load<CP>(r0, off, v * pstride);
      }
      double r[NV];
#pragma unroll
      for (int v = 0; v < NV; ++v) {
        r[v] = fma(sp.c, acc[v], sp.b * u[v]);
        if (use_u0) r[v] = fma(sp.a, u0[v], r[v]);
      }
      if (sp.rho_min > 0.0 || sp.p_min > 0.0)
        positivity_floor(r, sp.rho_min, sp.p_min, 1.0 / (pc.gamma - 1.0), mv.counters);
#pragma unroll
      for (int v = 0; v < NV; ++v) Buf<T>::template store<CP>(ro, off, r[v], v * pstride);
      if (sp.mode == 2) {  // second combination of the same L(Uk), no floor
        const rsrc_t r2 = make_rsrc(static_cast<T*>(sp.out2) + (size_t)b * NV * plane, abytes);
        const bool use_v = sp.a2 != 0.0;
        const rsrc_t rv = make_rsrc(static_cast<const T*>(use_v ? sp.V : sp.Uk) + (size_t)b * NV * plane, abytes);
#pragma unroll
        for (int v = 0; v < NV; ++v) {
          double w = fma(sp.c2, acc[v], sp.b2 * u[v]);
          if (use_v) w = fma(sp.a2, Buf<T>::template load<CP>(rv, off, v * pstride), w);
          Buf<T>::template store<CP>(r2, off, w, v * pstride);
        }
      }
    }
  }
}

template <int DIM, int N, typename T>
static void go_curv_t(const Ctx& c, const StageParams& sp, const CurvArgs& ca, hipStream_t s) {
  using SH = Shape<DIM, N>;
  const int nEB = (c.E + SH::EPB - 1) / SH::EPB;
  // bytes the stage streams: U_k, the output, U0 and the dual stage's second
  // output and V, plus the 1/J and Ja^l planes of the metrics
  const size_t state = (size_t)c.B * (DIM + 2) * c.E * SH::NP * sizeof(T);
  const int arrays = 2 + (sp.mode != 0 && sp.a != 0.0 ? 1 : 0) + (sp.mode == 2 ? 1 + (sp.a2 != 0.0 ? 1 : 0) : 0);
  const size_t metrics = (size_t)(1 + DIM * DIM) * c.E * SH::NP * sizeof(double);
  const bool nt = DIM == 3 && N == 3 && state * arrays + metrics > ((size_t)256 << 20);  // the Infinity Cache
  if (c.desc.volume == DG_VOLUME_SPLIT) {
    if (nt)
      hipLaunchKernelGGL((k_stage_curv<DIM, N, true, T, (DIM == 3 && N == 3)>), dim3(nEB * c.B), dim3(SH::BS), 0, s,
                         sp, mesh_view(c), c.pc, ca);
    else
      hipLaunchKernelGGL((k_stage_curv<DIM, N, true, T>), dim3(nEB * c.B), dim3(SH::BS), 0, s, sp, mesh_view(c),
                         c.pc, ca);
  } else {
    if (nt)
      hipLaunchKernelGGL((k_stage_curv<DIM, N, false, T, (DIM == 3 && N == 3)>), dim3(nEB * c.B), dim3(SH::BS), 0,
                         s, sp, mesh_view(c), c.pc, ca);
    else
      hipLaunchKernelGGL((k_stage_curv<DIM, N, false, T>), dim3(nEB * c.B), dim3(SH::BS), 0, s, sp, mesh_view(c),
                         c.pc, ca);
  }
}

template <int DIM, int N>
static hipError_t go_curv(const Ctx& c, const StageParams& sp, const CurvArgs& ca, hipStream_t s) {
  if (c.desc.precision == DG_F32)
    go_curv_t<DIM, N, float>(c, sp, ca, s);
  else
    go_curv_t<DIM, N, double>(c, sp, ca, s);
  return hipGetLastError();
}

template <int DIM>
static hipError_t curv_n(const Ctx& c, const StageParams& sp, const CurvArgs& ca, hipStream_t s) {
  switch (c.N) {
    case 1: return go_curv<DIM, 1>(c, sp, ca, s);
    case 2: return go_curv<DIM, 2>(c, sp, ca, s);
    case 3: return go_curv<DIM, 3>(c, sp, ca, s);
    case 4: return go_curv<DIM, 4>(c, sp, ca, s);
    case 5: return go_curv<DIM, 5>(c, sp, ca, s);
    case 6: return go_curv<DIM, 6>(c, sp, ca, s);
    case 7: return go_curv<DIM, 7>(c, sp, ca, s);
  }
  return hipErrorInvalidValue;
}

hipError_t launch_curv(const Ctx& c, const StageParams& sp, hipStream_t s) {
  if (c.desc.physics != DG_EULER) return hipErrorInvalidValue;
  CurvArgs ca;
  ca.met = c.d_met;
  for (int v = 0; v < 5; ++v) ca.ub[v] = c.desc.bc_state[v];
  return c.dim == 2 ? curv_n<2>(c, sp, ca, s) : curv_n<3>(c, sp, ca, s);
}

}  // namespace dg
