// Discrete adjoint of the fused Euler stage, gather form (no atomics).
//
// With L_i = -sum_l g_l sum_m D_im F_l(U_m) + sum_{f ni i} s_f (F*_f - F_l(U_i)),
// g_l = 2/h_l, s_f = -g_l/w_end on an upper face and +g_l/w_end on a lower
// face, the transpose applied to lambda at node m of element e is
//   sum_l A_l(U_m)^T nu_l,  nu_l = -g_l sum_i D_im lambda_i - sum_{f ni m} s_f lambda_m
//   + sum_{f ni m} (dF*_f / dU_m)^T s_f (lambda_m - lambda_m'),
// where A_l = dF_l/dU, and m' is the matching node of the face neighbour
// (which receives the same interface flux with the opposite sign), so every
// element only gathers U and lambda of its neighbours' face nodes.  For the
// Rusanov flux F* = (F_L + F_R)/2 - Lam (U_R - U_L)/2, Lam = max(c_L, c_R),
// c = |u_l| + a, the own-side derivative is
//   A/2 +- Lam/2 I - (U_R - U_L) (x) dLam/dU_own / 2     (+ for the left side),
// with the subgradient conventions d max(x,y) -> x when x >= y and
// d|x| -> sign(x), sign(0) = +1.
//
// Stage adjoint of U_out = a U0 + b U_k + c L(U_k):
//   lam_k = b lam_out + c (dL/dU)^T lam_out  (+ lam_0 when mode == 1),
//   mode 0: lam_0 += a lam_out;  mode 2: lam_0 = a lam_out;  mode 1: lam_0
//   is only read.
#include <type_traits>

#include "dg_device.hpp"

namespace dg {

struct AdjParams {
  const void* U;
  const void* lam_out;
  void* lam_k;
  void* lam_0;
  double a, b, c;
  int mode;  // 0: lam_0 += a lam; 1: lam_k += lam_0; 2: lam_0 = a lam; 3: no lam_0
};

// g += A_l(U)^T nu for the Euler flux along l (u velocity, p pressure)
template <int DIM>
__device__ __forceinline__ void flux_vjp(const double (&U)[DIM + 2], const double (&vel)[DIM], double p, double ri,
                                         int l, double gamma, const double (&nu)[DIM + 2], double (&g)[DIM + 2]) {
  constexpr int NV = DIM + 2;
  const double g1 = gamma - 1.0;
  double q2 = 0.0, nm_u = 0.0;
#pragma unroll
  for (int d = 0; d < DIM; ++d) {
    q2 = fma(vel[d], vel[d], q2);
    nm_u = fma(nu[1 + d], vel[d], nm_u);
  }
  const double ul = vel[l];
  const double H = (U[NV - 1] + p) * ri;
  const double hq = 0.5 * g1 * q2;
  // rho
  double gr = fma(nu[1 + l], hq, nu[NV - 1] * (hq - H) * ul);
  gr = fma(-nm_u, ul, gr);
  g[0] += gr;
  // momentum
#pragma unroll
  for (int d = 0; d < DIM; ++d) {
    double t = nu[1 + d] * ul - nu[1 + l] * g1 * vel[d] - nu[NV - 1] * g1 * vel[d] * ul;
    if (d == l) t += nu[0] + nm_u + nu[NV - 1] * H;
    g[1 + d] += t;
  }
  // energy
  g[NV - 1] += fma(nu[1 + l], g1, nu[NV - 1] * gamma * ul);
}

template <int DIM, int N, typename T>
__global__ void __launch_bounds__((Shape<DIM, N>::BS))
k_adjoint(AdjParams ap, MeshView mv, PhysConst pc) {
  using S = Shape<DIM, N>;
  using PHYS = EulerPhys<DIM>;
  constexpr int n = S::n, NP = S::NP, EPB = S::EPB, NV = PHYS::NV;

  __shared__ T sL[NV][EPB * NP];
  __shared__ T sDt[n * n];

  const int tid = threadIdx.x;
  // the lane's entry of D^T, written to LDS only before the first barrier
  static_assert(n * n <= S::BS, "one D entry per lane");
  const T dtval = tid < n * n ? static_cast<T>(mv.K->Dt[tid]) : T(0);

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
  // element tables first (scalar loads for a wave-uniform element, never
  // waited on in the middle of the computation)
  const int* nb = mv.nbr + (size_t)ec * 2 * DIM;
  int nbl[2 * DIM];
#pragma unroll
  for (int q = 0; q < 2 * DIM; ++q) nbl[q] = nb[q];
  double g[DIM];
#pragma unroll
  for (int l = 0; l < DIM; ++l) g[l] = mv.geo[(size_t)ec * 4 + l];
  const double winv = mv.K->wend_inv;
  int ii[3];
  ii[0] = node % n;
  ii[1] = (node / n) % n;
  ii[2] = node / (n * n);
  const int stride[3] = {1, n, n * n};

  const size_t plane = (size_t)E * NP;
  const size_t pbytes = plane * sizeof(T);
  const size_t bo = (size_t)b * NV * plane;
  rsrc_t rU[NV], rL[NV];
#pragma unroll
  for (int v = 0; v < NV; ++v) {
    rU[v] = make_rsrc(static_cast<const T*>(ap.U) + bo + v * plane, pbytes);
    rL[v] = make_rsrc(static_cast<const T*>(ap.lam_out) + bo + v * plane, pbytes);
  }
  const unsigned off = (unsigned)(ec * NP + node);
  double u[NV], lam[NV];
#pragma unroll
  for (int v = 0; v < NV; ++v) {
    u[v] = Buf<T>::load(rU[v], off);
    lam[v] = Buf<T>::load(rL[v], off);
  }
  int side[DIM], nbe[DIM];
#pragma unroll
  for (int l = 0; l < DIM; ++l) {
    side[l] = (ii[l] == 0) ? 0 : ((ii[l] == N) ? 1 : -1);
    nbe[l] = (active && side[l] >= 0) ? nbl[2 * l + side[l]] : -1;
  }
  T* lam0b = ap.lam_0 ? static_cast<T*>(ap.lam_0) + bo : nullptr;

  Thermo th;
  PHYS::thermo(u, th, pc);
  double vel[DIM];
#pragma unroll
  for (int d = 0; d < DIM; ++d) vel[d] = u[1 + d] * th.ri;

  if (tid < n * n) sDt[tid] = dtval;
  if (tid < S::NT) {
#pragma unroll
    for (int v = 0; v < NV; ++v) sL[v][tid] = static_cast<T>(lam[v]);
  }
  __syncthreads();

  const double gamma = pc.gamma;
  double aown = 0.0;
  bool on_face = false;
#pragma unroll
  for (int l = 0; l < DIM; ++l) on_face |= side[l] >= 0;
  if (on_face) aown = sound<PHYS>(th);

  double gout[NV];
#pragma unroll
  for (int v = 0; v < NV; ++v) gout[v] = 0.0;
  if (tid < S::NT) {
#pragma unroll
    for (int l = 0; l < DIM; ++l) {
      // the neighbour's state and adjoint for this direction only (all three
      // held from the start took 3 waves per SIMD instead of 4 in FP32, and
      // the FP32 reverse sweep 10 % longer)
      double unl[NV], lnl[NV];
      if (nbe[l] >= 0) {
        const unsigned noff = (unsigned)(nbe[l] * NP + node + (side[l] ? -N : N) * stride[l]);
#pragma unroll
        for (int v = 0; v < NV; ++v) {
          unl[v] = Buf<T>::load(rU[v], noff);
          lnl[v] = Buf<T>::load(rL[v], noff);
        }
      }
      const int il = ii[l], st = stride[l];
      const int base = tid - il * st;
      T drow[n];
#pragma unroll
      for (int m = 0; m < n; ++m) drow[m] = sDt[il * n + m] * static_cast<T>(-g[l]);
      double nu[NV];
#pragma unroll
      for (int v = 0; v < NV; ++v) {
        T s = 0;
#pragma unroll
        for (int m = 0; m < n; ++m) s = fma(drow[m], sL[v][base + m * st], s);
        nu[v] = static_cast<double>(s);
      }
      if (side[l] >= 0) {
        const double sc = (side[l] ? -g[l] : g[l]) * winv;   // s_f
        const bool ownL = side[l] == 1;
        // neighbour thermodynamics (same sequence as the forward stage)
        Thermo tn;
        PHYS::thermo(unl, tn, pc);
        const double vn = unl[1 + l] * tn.ri;
        const double co = fabs(vel[l]) + aown;
        const double cn = fabs(vn) + sound<PHYS>(tn);
        const double lamx = co >= cn ? co : cn;
        // own branch of the max: left wins ties
        const bool sel = ownL ? (co >= cn) : (cn < co);
        double mu[NV], dU = 0.0;
#pragma unroll
        for (int v = 0; v < NV; ++v) {
          mu[v] = sc * (lam[v] - lnl[v]);
          // (U_R - U_L) . mu
          const double jump = ownL ? (unl[v] - u[v]) : (u[v] - unl[v]);
          dU = fma(jump, mu[v], dU);
        }
        // own-flux lift term and half of the flux Jacobian of F*
#pragma unroll
        for (int v = 0; v < NV; ++v) nu[v] = fma(0.5, mu[v], fma(-sc, lam[v], nu[v]));
        // +- Lam/2 mu
        const double hl = (ownL ? 0.5 : -0.5) * lamx;
#pragma unroll
        for (int v = 0; v < NV; ++v) gout[v] = fma(hl, mu[v], gout[v]);
        // -(dU/2) dc_own/dU_own on the selected branch
        if (sel) {
          const double ri = th.ri;
          const double ul = vel[l];
          const double sg = ul >= 0.0 ? 1.0 : -1.0;
          const double f = -0.5 * dU;
          const double ca = 0.5 * gamma * ri / aown;           // d a / d p
          const double g1 = gamma - 1.0;
          double q2 = 0.0;
#pragma unroll
          for (int d = 0; d < DIM; ++d) q2 = fma(vel[d], vel[d], q2);
          // da/dU = ca * dp/dU - (a / (2 rho)) e_rho,  dp/dU = g1 (q2/2, -u, 1)
          gout[0] += f * (-sg * ul * ri + ca * g1 * 0.5 * q2 - 0.5 * aown * ri);
#pragma unroll
          for (int d = 0; d < DIM; ++d) gout[1 + d] += f * ((d == l ? sg * ri : 0.0) - ca * g1 * vel[d]);
          gout[NV - 1] += f * ca * g1;
        }
      }
      flux_vjp<DIM>(u, vel, th.p, th.ri, l, gamma, nu, gout);
    }
  }

  if (active) {
    double l0[NV];  // lambda_0 in, loaded only here
#pragma unroll
    for (int v = 0; v < NV; ++v) l0[v] = 0.0;
    if (ap.mode == 0 || ap.mode == 1) {
#pragma unroll
      for (int v = 0; v < NV; ++v) l0[v] = Buf<T>::load(make_rsrc(lam0b + v * plane, pbytes), off);
    }
    T* lkb = static_cast<T*>(ap.lam_k) + bo;
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      double r = fma(ap.c, gout[v], ap.b * lam[v]);
      if (ap.mode == 1) r += l0[v];
      Buf<T>::store(make_rsrc(lkb + v * plane, pbytes), off, r);
    }
    if (ap.mode == 0 || ap.mode == 2) {
#pragma unroll
      for (int v = 0; v < NV; ++v) {
        const double r = ap.mode == 0 ? fma(ap.a, lam[v], l0[v]) : ap.a * lam[v];
        Buf<T>::store(make_rsrc(lam0b + v * plane, pbytes), off, r);
      }
    }
  }
}

// ---------------------------------------------------------------------------
// The same adjoint for 3-D, N = 3 (64 nodes: one element per single-wave
// workgroup) with every global read issued at entry, as the forward stage of
// this shape: own U_k and lambda_out into registers, the neighbour face nodes
// of U_k and lambda_out of all three directions into LDS by buffer-to-LDS
// loads (FP64: lane L fetches dword L & 1 of face slot L >> 1; FP32: lanes <
// 32 fetch slot L; slots 0-15 the -xi_l face, 16-31 the +xi_l face,
// tangential index a + 4 b), so that a wave waits for memory once instead of
// once per direction.  lambda_0 goes to LDS at entry as well in FP32; in FP64
// it is loaded for the output (its 2.5 KB of LDS would cap the workgroups per
// CU below the 4 waves per SIMD the registers allow; measured 1.5 % slower).
// Same arithmetic per term as k_adjoint (FP32 reverse step 13 % faster than
// k_adjoint at the adjoint workload, FP64 5 %).
// ---------------------------------------------------------------------------
// NT: the step's streams exceed the Infinity Cache; lambda_0 and lambda_k,
// which no other workgroup reads, carry the non-temporal hint
template <typename T, bool NT = false>
__global__ void __launch_bounds__(64) k_adjoint_n3(AdjParams ap, MeshView mv, PhysConst pc) {
  using PHYS = EulerPhys<3>;
  constexpr int DIM = 3, N = 3, n = 4, NP = 64, NV = 5;
  constexpr bool F32 = std::is_same<T, float>::value;
  constexpr int WPV = F32 ? 32 : 64;  // dwords of face data per direction and variable
  __shared__ T sL[NV][NP];
  __shared__ T sDt[n * n];
  __shared__ __attribute__((aligned(16))) unsigned sNU[DIM][NV][WPV];
  __shared__ __attribute__((aligned(16))) unsigned sNL[DIM][NV][WPV];
  __shared__ __attribute__((aligned(16))) unsigned sL0[F32 ? NV : 1][F32 ? NP : 1];  // FP32 lambda_0

  const int tid = threadIdx.x;
  const T dtval = tid < n * n ? static_cast<T>(mv.K->Dt[tid]) : T(0);
  const int E = mv.E;
  const int blk = xcd_remap(blockIdx.x, gridDim.x);
  const int b = blk / E;
  const int ec = wave_uniform(blk - b * E);
  const int* nb = mv.nbr + (size_t)ec * 2 * DIM;
  int nbl[2 * DIM];
#pragma unroll
  for (int q = 0; q < 2 * DIM; ++q) nbl[q] = nb[q];
  double g[DIM];
#pragma unroll
  for (int l = 0; l < DIM; ++l) g[l] = mv.geo[(size_t)ec * 4 + l];
  const double winv = mv.K->wend_inv;
  const int ii[3] = {tid & 3, (tid >> 2) & 3, tid >> 4};
  const int stride[3] = {1, 4, 16};

  const size_t plane = (size_t)E * NP;
  const size_t abytes = (size_t)NV * plane * sizeof(T);
  const unsigned pstride = (unsigned)(plane * sizeof(T));
  const size_t bo = (size_t)b * NV * plane;
  const rsrc_t rU = make_rsrc(static_cast<const T*>(ap.U) + bo, abytes);
  const rsrc_t rL = make_rsrc(static_cast<const T*>(ap.lam_out) + bo, abytes);
  const unsigned off = (unsigned)(ec * NP + tid);

  double u[NV], lam[NV];
#pragma unroll
  for (int v = 0; v < NV; ++v) {
    u[v] = Buf<T>::load(rU, off, v * pstride);
    lam[v] = Buf<T>::load(rL, off, v * pstride);
  }
  {  // neighbour face nodes of U_k and lambda_out into LDS
    const int slot = F32 ? tid : tid >> 1, half = F32 ? 0 : tid & 1;
    const bool upper = (slot & 16) != 0;
    const int ta = slot & 3, tb = (slot >> 2) & 3;
    if (!F32 || tid < 32) {
#pragma unroll
      for (int l = 0; l < DIM; ++l) {
        const int o1 = l == 0 ? 1 : 0, o2 = l == 2 ? 1 : 2;
        const int lo = nbl[2 * l], hi = nbl[2 * l + 1];
        const int ne = upper ? hi : lo;
        const int node = (upper ? 0 : N) * stride[l] + ta * stride[o1] + tb * stride[o2];
        const unsigned voff = (unsigned)(ne * NP + node) * (unsigned)sizeof(T) + 4u * (unsigned)half;
#pragma unroll
        for (int v = 0; v < NV; ++v) {
          __builtin_amdgcn_raw_ptr_buffer_load_lds(rU, DG_LDS_PTR(&sNU[l][v][0]), 4, voff, v * pstride, 0, 0);
          __builtin_amdgcn_raw_ptr_buffer_load_lds(rL, DG_LDS_PTR(&sNL[l][v][0]), 4, voff, v * pstride, 0, 0);
        }
      }
    }
  }
  const bool read_l0 = ap.mode == 0 || ap.mode == 1;
  if constexpr (F32) {  // lambda_0 into LDS, one load per variable
    if (read_l0) {
      const rsrc_t r0 = make_rsrc(static_cast<const T*>(ap.lam_0) + bo, abytes);
#pragma unroll
      for (int v = 0; v < NV; ++v)
        __builtin_amdgcn_raw_ptr_buffer_load_lds(r0, DG_LDS_PTR(&sL0[v][0]), 4, off * 4u, v * pstride, 0, NT ? CPOL_NT : 0);
    }
  }

  Thermo th;
  PHYS::thermo(u, th, pc);
  double vel[DIM];
#pragma unroll
  for (int d = 0; d < DIM; ++d) vel[d] = u[1 + d] * th.ri;
  if (tid < n * n) sDt[tid] = dtval;
#pragma unroll
  for (int v = 0; v < NV; ++v) sL[v][tid] = static_cast<T>(lam[v]);
  wave_lds_fence();

  const double gamma = pc.gamma;
  const double aown = sound<PHYS>(th);
  double gout[NV];
#pragma unroll
  for (int v = 0; v < NV; ++v) gout[v] = 0.0;
  // the neighbour face nodes of U_k and lambda_out (and FP32 lambda_0) arrive
  // in LDS by buffer-to-LDS loads
  wait_vmem_all();
#pragma unroll
  for (int l = 0; l < DIM; ++l) {
    const int il = ii[l], st = stride[l];
    const int base = tid - il * st;
    T drow[n];
#pragma unroll
    for (int m = 0; m < n; ++m) drow[m] = sDt[il * n + m] * static_cast<T>(-g[l]);
    double nu[NV];
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      T s = 0;
#pragma unroll
      for (int m = 0; m < n; ++m) s = fma(drow[m], sL[v][base + m * st], s);
      nu[v] = static_cast<double>(s);
    }
    const int side = (il == 0) ? 0 : ((il == N) ? 1 : -1);
    if (side >= 0) {
      const int o1 = l == 0 ? 1 : 0, o2 = l == 2 ? 1 : 2;
      const int slot = side * 16 + ii[o1] + 4 * ii[o2];
      double unl[NV], lnl[NV];
#pragma unroll
      for (int v = 0; v < NV; ++v) {
        if constexpr (F32) {
          unl[v] = static_cast<double>(__builtin_bit_cast(float, sNU[l][v][slot]));
          lnl[v] = static_cast<double>(__builtin_bit_cast(float, sNL[l][v][slot]));
        } else {
          unl[v] = *reinterpret_cast<const double*>(&sNU[l][v][2 * slot]);
          lnl[v] = *reinterpret_cast<const double*>(&sNL[l][v][2 * slot]);
        }
      }
      const double sc = (side ? -g[l] : g[l]) * winv;  // s_f
      const bool ownL = side == 1;
      Thermo tn;
      PHYS::thermo(unl, tn, pc);
      const double vn = unl[1 + l] * tn.ri;
      const double co = fabs(vel[l]) + aown;
      const double cn = fabs(vn) + sound<PHYS>(tn);
      const double lamx = co >= cn ? co : cn;
      const bool sel = ownL ? (co >= cn) : (cn < co);
      double mu[NV], dU = 0.0;
#pragma unroll
      for (int v = 0; v < NV; ++v) {
        mu[v] = sc * (lam[v] - lnl[v]);
        const double jump = ownL ? (unl[v] - u[v]) : (u[v] - unl[v]);
        dU = fma(jump, mu[v], dU);
      }
#pragma unroll
      for (int v = 0; v < NV; ++v) nu[v] = fma(0.5, mu[v], fma(-sc, lam[v], nu[v]));
      const double hl = (ownL ? 0.5 : -0.5) * lamx;
#pragma unroll
      for (int v = 0; v < NV; ++v) gout[v] = fma(hl, mu[v], gout[v]);
      if (sel) {
        const double ri = th.ri;
        const double ul = vel[l];
        const double sg = ul >= 0.0 ? 1.0 : -1.0;
        const double f = -0.5 * dU;
        const double ca = 0.5 * gamma * ri / aown;
        const double g1 = gamma - 1.0;
        double q2 = 0.0;
#pragma unroll
        for (int d = 0; d < DIM; ++d) q2 = fma(vel[d], vel[d], q2);
        gout[0] += f * (-sg * ul * ri + ca * g1 * 0.5 * q2 - 0.5 * aown * ri);
#pragma unroll
        for (int d = 0; d < DIM; ++d) gout[1 + d] += f * ((d == l ? sg * ri : 0.0) - ca * g1 * vel[d]);
        gout[NV - 1] += f * ca * g1;
      }
    }
    flux_vjp<DIM>(u, vel, th.p, th.ri, l, gamma, nu, gout);
  }

  double l0[NV];
#pragma unroll
  for (int v = 0; v < NV; ++v) {
    if (!read_l0) l0[v] = 0.0;
    else if constexpr (F32) l0[v] = static_cast<double>(__builtin_bit_cast(float, sL0[v][tid]));
    else l0[v] = Buf<T>::template load<NT ? CPOL_NT : 0>(make_rsrc(static_cast<const T*>(ap.lam_0) + bo, abytes), off, v * pstride);
  }
  const rsrc_t rk = make_rsrc(static_cast<T*>(ap.lam_k) + bo, abytes);
#pragma unroll
  for (int v = 0; v < NV; ++v) {
    double r = fma(ap.c, gout[v], ap.b * lam[v]);
    if (ap.mode == 1) r += l0[v];
    Buf<T>::template store<NT ? CPOL_NT : 0>(rk, off, r, v * pstride);
  }
  if (ap.mode == 0 || ap.mode == 2) {
    const rsrc_t r0 = make_rsrc(static_cast<T*>(ap.lam_0) + bo, abytes);
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      const double r = ap.mode == 0 ? fma(ap.a, lam[v], l0[v]) : ap.a * lam[v];
      Buf<T>::template store<NT ? CPOL_NT : 0>(r0, off, r, v * pstride);
    }
  }
}

template <int DIM, int N, typename T>
static hipError_t adj_go(const Ctx& c, const AdjParams& ap, hipStream_t s) {
  using SH = Shape<DIM, N>;
  const int nEB = (c.E + SH::EPB - 1) / SH::EPB;
  if constexpr (DIM == 3 && N == 3) {
    // U_k, lambda_out, lambda_k and lambda_0 (read and written)
    const size_t state = (size_t)c.B * 5 * c.E * 64 * sizeof(T);
    if (state * 5 > ((size_t)256 << 20))  // the Infinity Cache
      hipLaunchKernelGGL((k_adjoint_n3<T, true>), dim3(c.E * c.B), dim3(64), 0, s, ap, mesh_view(c), c.pc);
    else
      hipLaunchKernelGGL((k_adjoint_n3<T>), dim3(c.E * c.B), dim3(64), 0, s, ap, mesh_view(c), c.pc);
    return hipGetLastError();
  }
  hipLaunchKernelGGL((k_adjoint<DIM, N, T>), dim3(nEB * c.B), dim3(SH::BS), 0, s, ap, mesh_view(c), c.pc);
  return hipGetLastError();
}

template <int DIM, typename T>
static hipError_t adj_n(const Ctx& c, const AdjParams& ap, hipStream_t s) {
  switch (c.N) {
    case 1: return adj_go<DIM, 1, T>(c, ap, s);
    case 2: return adj_go<DIM, 2, T>(c, ap, s);
    case 3: return adj_go<DIM, 3, T>(c, ap, s);
    case 4: return adj_go<DIM, 4, T>(c, ap, s);
  }
  return hipErrorNotSupported;
}

hipError_t launch_adjoint(const Ctx& c, const void* U, const void* lam_out, void* lam_k, void* lam_0, double a,
                          double b, double cdt, int mode, hipStream_t s) {
  AdjParams ap;
  ap.U = U;
  ap.lam_out = lam_out;
  ap.lam_k = lam_k;
  ap.lam_0 = lam_0;
  ap.a = a;
  ap.b = b;
  ap.c = cdt;
  ap.mode = lam_0 ? mode : 3;
  if (c.desc.precision == DG_F32) return c.dim == 2 ? adj_n<2, float>(c, ap, s) : adj_n<3, float>(c, ap, s);
  return c.dim == 2 ? adj_n<2, double>(c, ap, s) : adj_n<3, double>(c, ap, s);
}

}  // namespace dg
