// Fused DGSEM right-hand side and Shu-Osher stage for the inviscid physics
// (Euler, reacting Euler) on affine Cartesian elements.
//
// One lane per solution node, EPB elements per workgroup.  Per element:
//   1. load U_k (coalesced: the block's elements are contiguous in every
//      variable plane), recover primitives in double and flag non-physical
//      nodes;
//   2. volume integral (eq. vol_weak): contravariant fluxes (2/h_l) F_l are
//      staged through LDS and each lane sums its three lines with the GLL
//      derivative matrix;
//   3. surface lift and Jacobian rescale (eq. surf_int): lanes on a face read
//      the neighbour's matching node straight from U_k (no trace buffer, no
//      atomics) and evaluate the Rusanov flux with the element on the -xi_l
//      side as left state, so both elements of a face get the same bits; 2:1
//      mortar faces take the flux from the mortar kernel's rows instead;
//   4. write dU/dt, or the stage a U0 + b U_k + c dU/dt (with the positivity
//      floor, if set), and in the dual form also a2 V + b2 U_k + c2 dU/dt.
//
// Split form (eq. vol_split): instead of fluxes the block stages primitives
// (rho, v, p, rho/p and the logarithms of rho and rho/p) in LDS, and each lane sums 2 D_im F#_l(U_i, U_m) over
// the other nodes m of its line with Ranocha's two-point flux (published
// form: log means of rho and rho/p, arithmetic means of v and p, the crossed
// pressure-velocity product in the energy row).  The m = i term, D_ii F_l(U_i),
// is nonzero only at the line's end nodes (GLL: D_ii = 0 inside), so it is
// added in the face step, which computes F_l(U_i) there anyway.  Where a line
// lies in one wave, each unordered pair is evaluated by one of its two lanes
// and handed to the other by a lane shuffle.  Faces, lift and output are
// those of the standard form.
//
// FP32 form: states and the LDS flux operand are float, the D-sweep is a
// float FMA chain, and dU/dt and the stage combination accumulate in float.
// Primitive recovery, flux evaluation and the face corrections (F* - F) stay
// in double; before rounding to float the volume flux has the flux of the
// element's first node subtracted, which leaves sum_m D_im F_m unchanged (D
// annihilates constants) but keeps the rounding error relative to the
// variation inside the element.
#include <type_traits>

#include "dg_device.hpp"
#include "dg_split.hpp"

namespace dg {

template <typename T> __device__ __forceinline__ T dmat_entry(const RefConsts* K, int q);
template <> __device__ __forceinline__ double dmat_entry<double>(const RefConsts* K, int q) { return K->D[q]; }
template <> __device__ __forceinline__ float dmat_entry<float>(const RefConsts* K, int q) { return K->Df[q]; }

// register budget: four waves per SIMD; the reacting physics (eight
// variables, mortar faces, 77,824-node workloads) takes three, which it needs
// to keep its face state in registers, and so does the split form, whose
// unrolled two-point fluxes would spill at four
template <class PHYS, bool SPLIT>
struct StageWaves {
  static constexpr int value = (PHYS::NV > 5 || SPLIT) ? 3 : 4;
};

template <int DIM, int N, class PHYS, typename T, bool MORTAR, bool SPLIT>
__global__ void __launch_bounds__((Shape<DIM, N>::BS)) __attribute__((amdgpu_waves_per_eu(StageWaves<PHYS, SPLIT>::value)))
k_stage(StageParams sp, MeshView mv, PhysConst pc) {
  using S = Shape<DIM, N>;
  constexpr int n = S::n, NP = S::NP, EPB = S::EPB, NV = PHYS::NV, MOM = PHYS::MOM;
  constexpr bool F32 = std::is_same<T, float>::value;
  // an element fills whole waves: its index and tables are wave-uniform
  constexpr bool UNIFORM_ELEM = (NP % 64) == 0;
  constexpr bool MASK_FACES = !F32 && !MORTAR;

  // D in the sweep's precision: the split form sums in double
  using DT = typename std::conditional<SPLIT, double, T>::type;
  static_assert(!SPLIT || std::is_same<PHYS, EulerPhys<DIM>>::value, "split form: Euler physics");

  __shared__ T sF[SPLIT ? 1 : DIM][SPLIT ? 1 : NV][SPLIT ? 1 : EPB * NP];
  __shared__ double sQ[SPLIT ? DIM + 5 : 1][SPLIT ? EPB * NP : 1];  // rho, v, p, rho/p, their logs
  __shared__ int sFar;  // split form: some lane of the block needs the exact log means
  __shared__ DT sD[n * n];
  // One element per workgroup: D scaled by -2/h_l for each direction, so the
  // volume sweep accumulates straight into dU/dt (no per-direction rescale).
  constexpr bool DSCALED = (EPB == 1) && !SPLIT;
  __shared__ T sDg[DSCALED ? DIM : 1][DSCALED ? n * n : 1];
  __shared__ double sRef[(F32 && !SPLIT) ? EPB : 1][DIM][NV];

  const int tid = threadIdx.x;
  // the lane's entry of D, stored to LDS only just before the first barrier
  // (no wait on this load ahead of the state loads)
  static_assert(n * n <= S::BS, "one D entry per lane");
  const DT dval = (!DSCALED && tid < n * n) ? dmat_entry<DT>(mv.K, tid) : DT(0);
  const double dsc = (DSCALED && tid < n * n) ? mv.K->D[tid] : 0.0;

  const int E = mv.E;
  const int nEB = (E + EPB - 1) / EPB;
  const int blk = xcd_remap(blockIdx.x, gridDim.x);
  const int b = blk / nEB;
  const int eb = zfast_block<EPB>(blk - b * nEB, mv);
  const int el = tid / NP;
  const int node = tid - el * NP;
  int e = eb * EPB + el;
  const bool active = (tid < S::NT) && (e < E);
  int ec = active ? e : 0;  // clamped for address arithmetic only
  if constexpr (UNIFORM_ELEM) ec = wave_uniform(ec);

  // Per-element tables first, before any store or atomic: with a
  // wave-uniform element they become scalar loads, and none of them is
  // waited on in the middle of the computation.
  const int* nb = mv.nbr + (size_t)ec * 2 * DIM;
  int nbl[2 * DIM];
#pragma unroll
  for (int q = 0; q < 2 * DIM; ++q) nbl[q] = nb[q];
  double g[DIM];
#pragma unroll
  for (int l = 0; l < DIM; ++l) g[l] = mv.geo[(size_t)ec * 4 + l];
  const double hwinv = 0.5 * mv.K->wend_inv;

  int ii[3];
  ii[0] = node % n;
  ii[1] = (node / n) % n;
  ii[2] = node / (n * n);
  const int stride[3] = {1, n, n * n};

  // One buffer descriptor per state array (this batch member); variable
  // planes are reached through a scalar byte offset.
  const size_t plane = (size_t)E * NP;
  const size_t abytes = (size_t)NV * plane * sizeof(T);
  const unsigned pstride = (unsigned)(plane * sizeof(T));
  const rsrc_t rU = make_rsrc(static_cast<const T*>(sp.Uk) + (size_t)b * NV * plane, abytes);
  const unsigned off = (unsigned)(ec * NP + node);

  double u[NV];
#pragma unroll
  for (int v = 0; v < NV; ++v) u[v] = Buf<T>::load(rU, off, v * pstride);

  // Neighbour's matching node for each direction.  A lane that is not on a
  // face in direction l uses its own node: the interface flux of a state
  // with itself is its physical flux, so that direction's correction below
  // is exactly zero and no lane has to branch.  The FP64 form on conforming
  // meshes instead masks such lanes out of that direction's loads and face
  // arithmetic: idle lanes draw less power, which at the board power limit
  // the device sustains under this kernel is worth more than the uniform
  // control flow (measured; the FP32 form measures the other way, and the
  // mortar form would spill registers).
  int side[DIM], nbe[DIM];
  double un[DIM][NV];
  auto load_neighbours = [&]() {
#pragma unroll
  for (int l = 0; l < DIM; ++l) {
    side[l] = (ii[l] == 0) ? 0 : ((ii[l] == N) ? 1 : -1);
    const int lo = nbl[2 * l], hi = nbl[2 * l + 1];
    nbe[l] = side[l] == 0 ? lo : (side[l] == 1 ? hi : ec);
    const bool conf = !MORTAR || nbe[l] >= 0;
    const int ne = conf ? nbe[l] : ec;
    const int shift = side[l] == 1 ? -N : (side[l] == 0 ? N : 0);
    const unsigned noff = (unsigned)(ne * NP + node + shift * stride[l]);
    if (!MASK_FACES || side[l] >= 0) {  // masked lanes never read un[l]
#pragma unroll
      for (int v = 0; v < NV; ++v) un[l][v] = Buf<T>::load(rU, noff, v * pstride);
    }
  }
  };
  // The neighbour states are loaded after the volume sweep and U0 only for
  // the output: held from the start they would stay live in registers
  // through the sweep (measured: 4 waves per SIMD instead of 5, and slower).
  const bool use_u0 = (sp.mode != 0) && (sp.a != 0.0);

  Thermo th;
  const bool ok = PHYS::thermo(u, th, pc);
  if (active && !ok)
    report_nonphysical(mv.counters, mv.first_bad, ((unsigned long long)b * E + e) * NP + node);
  double vel[DIM];
#pragma unroll
  for (int d = 0; d < DIM; ++d) vel[d] = u[MOM + d] * th.ri;

  // ---- stage physical fluxes (split form: primitives) in LDS -------------
  if (!DSCALED && tid < n * n) sD[tid] = dval;
  if constexpr (DSCALED) {
    if (tid < n * n) {
#pragma unroll
      for (int l = 0; l < DIM; ++l) sDg[l][tid] = static_cast<T>(-g[l] * dsc);
    }
  }
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
    }
    if (tid == 0) sFar = 0;
  } else if constexpr (F32) {
    if (tid < S::NT && node == 0) {
#pragma unroll
      for (int l = 0; l < DIM; ++l) {
        double F[NV];
        PHYS::flux(u, vel[l], th.p, l, F);
#pragma unroll
        for (int v = 0; v < NV; ++v) sRef[el][l][v] = F[v];
      }
    }
    __syncthreads();
  }
  if (!SPLIT && tid < S::NT) {
#pragma unroll
    for (int l = 0; l < DIM; ++l) {
      double F[NV];
      PHYS::flux(u, vel[l], th.p, l, F);
#pragma unroll
      for (int v = 0; v < NV; ++v) {
        if constexpr (F32) sF[l][v][tid] = static_cast<float>(F[v] - sRef[el][l][v]);
        else sF[l][v][tid] = F[v];
      }
    }
  }
  __syncthreads();

  // ---- volume integral: -sum_l (2/h_l) sum_m D_im F_l,m ----------------
  // accumulator of dU/dt: float in the FP32 form (its stage output is rounded
  // to float anyway; half the registers and no conversions), else double
  using AT = typename std::conditional<SPLIT, double, T>::type;
  AT acc[NV];
#pragma unroll
  for (int v = 0; v < NV; ++v) acc[v] = AT(0);
  if constexpr (SPLIT) {
    const double gm1i = 1.0 / (pc.gamma - 1.0);
    bool far = false;
    if (tid < S::NT) {
      if constexpr (S::BS == 64)
        split_sweep_pairs<DIM, N, 0>(tid, ii, stride, own, sQ, sD, g, gm1i, far, acc);
      else
        split_sweep<DIM, N, 0, false>(tid, ii, stride, own, sQ, sD, g, gm1i, far, acc);
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
        split_sweep<DIM, N, 0, true>(tid, ii, stride, own, sQ, sD, g, gm1i, far, acc);
      }
    }
  } else if (tid < S::NT) {
#pragma unroll
    for (int l = 0; l < DIM; ++l) {
      const int il = ii[l];
      const int st = stride[l];
      const int base = tid - il * st;
      T drow[n];
#pragma unroll
      for (int m = 0; m < n; ++m) drow[m] = DSCALED ? sDg[DSCALED ? l : 0][il * n + m] : sD[il * n + m];
#pragma unroll
      for (int v = 0; v < NV; ++v) {
        if constexpr (DSCALED) {
#pragma unroll
          for (int m = 0; m < n; ++m) acc[v] = fma(AT(drow[m]), AT(sF[l][v][base + m * st]), acc[v]);
        } else {
          T s = 0;
#pragma unroll
          for (int m = 0; m < n; ++m) s = fma(drow[m], sF[l][v][base + m * st], s);
          acc[v] = fma(AT(-g[l]), static_cast<AT>(s), acc[v]);
        }
      }
    }
  }

  load_neighbours();

  // ---- surface lift (eq. surf_int) ----------------------------------------
  const double aown = wave_sound<PHYS, F32>(th);
#pragma unroll
  for (int l = 0; l < DIM; ++l) {
    if (MASK_FACES && side[l] < 0) continue;  // masked lane: no face in direction l
    // own physical flux: the FP64 form reads it back from the volume stage
    double Fo[NV];
    if constexpr (F32 || SPLIT) {
      PHYS::flux(u, vel[l], th.p, l, Fo);
    } else {
#pragma unroll
      for (int v = 0; v < NV; ++v) Fo[v] = sF[l][v][tid < S::NT ? tid : 0];
    }
    // Rusanov flux F* with the element on the -xi_l side as left state,
    // applied as the difference 2 (F* - F_own) = (F_nb - F_own) - s lam (U_nb - U_own),
    // s = +1 on the +xi_l face and -1 on the -xi_l face.
    Thermo tn;
    PHYS::thermo(un[l], tn, pc);
    const double vn = un[l][MOM + l] * tn.ri;
    double Fn[NV], Dv[NV];
    PHYS::flux(un[l], vn, tn.p, l, Fn);
    const double co = fabs(vel[l]) + aown;
    const double cn = fabs(vn) + wave_sound<PHYS, F32>(tn);
    const double lam = fmax(co, cn);
    const double sgn = side[l] == 1 ? 1.0 : -1.0;  // +1 on the +xi_l face
    const double hs = sgn * lam;
#pragma unroll
    for (int v = 0; v < NV; ++v) Dv[v] = fma(-hs, un[l][v] - u[v], Fn[v] - Fo[v]);
    if constexpr (MORTAR) {
      if (side[l] >= 0 && nbe[l] < 0) {  // 2:1 face: flux from the mortar kernel
        const int row = -nbe[l] - 1;
        const int t = (DIM == 2) ? ii[1 - l] : 0;
        const double* src = mv.mortar_flux + (((size_t)b * mv.nrows + row) * S::NF + t) * NV;
#pragma unroll
        for (int v = 0; v < NV; ++v) Dv[v] = 2.0 * (src[v] - Fo[v]);
      }
    }
    const double sc = -sgn * (g[l] * hwinv);
#pragma unroll
    for (int v = 0; v < NV; ++v) acc[v] = fma(AT(sc), AT(Dv[v]), acc[v]);
    if constexpr (SPLIT) {
      // the split sum's m = i term, 2 D_ii F_l(U_i)
      const double cd = -2.0 * g[l] * static_cast<double>(sD[ii[l] * (n + 1)]);
#pragma unroll
      for (int v = 0; v < NV; ++v) acc[v] = fma(cd, Fo[v], acc[v]);
    }
  }

  // ---- output ----------------------------------------------------------------
  if (active) {
    const rsrc_t ro = make_rsrc(static_cast<T*>(sp.out) + (size_t)b * NV * plane, abytes);
    if (sp.mode == 0) {
#pragma unroll
      for (int v = 0; v < NV; ++v) Buf<T>::store(ro, off, acc[v], v * pstride);
    } else {
      double u0[NV];
      if (use_u0) {
        const rsrc_t r0 = make_rsrc(static_cast<const T*>(sp.U0) + (size_t)b * NV * plane, abytes);
#pragma unroll
        for (int v = 0; v < NV; ++v) u0[v] = Buf<T>::load(r0, off, v * pstride);
      }
      AT r[NV];
#pragma unroll
      for (int v = 0; v < NV; ++v) {
        r[v] = fma(AT(sp.c), acc[v], AT(sp.b) * AT(u[v]));
        if (use_u0) r[v] = fma(AT(sp.a), AT(u0[v]), r[v]);
      }
      if constexpr (std::is_same<PHYS, EulerPhys<DIM>>::value) {
        if (sp.rho_min > 0.0 || sp.p_min > 0.0) {  // the floor itself in double
          double rd[NV];
#pragma unroll
          for (int v = 0; v < NV; ++v) rd[v] = r[v];
          positivity_floor(rd, sp.rho_min, sp.p_min, 1.0 / (pc.gamma - 1.0), mv.counters);
#pragma unroll
          for (int v = 0; v < NV; ++v) r[v] = AT(rd[v]);
        }
      }
#pragma unroll
      for (int v = 0; v < NV; ++v) Buf<T>::store(ro, off, r[v], v * pstride);
      if (sp.mode == 2) {  // second combination of the same L(Uk), no floor
        const rsrc_t r2 = make_rsrc(static_cast<T*>(sp.out2) + (size_t)b * NV * plane, abytes);
        const bool use_v = sp.a2 != 0.0;
        const rsrc_t rv = make_rsrc(static_cast<const T*>(use_v ? sp.V : sp.Uk) + (size_t)b * NV * plane, abytes);
#pragma unroll
        for (int v = 0; v < NV; ++v) {
          AT w = fma(AT(sp.c2), acc[v], AT(sp.b2) * AT(u[v]));
          if (use_v) w = fma(AT(sp.a2), AT(Buf<T>::load(rv, off, v * pstride)), w);
          Buf<T>::store(r2, off, w, v * pstride);
        }
      }
    }
  }
}

// ---------------------------------------------------------------------------
// The headline shape -- 3-D, N = 3 (64 nodes: one element per single-wave
// workgroup), conforming faces, FP64 and the FP32 form -- with every global
// read of the stage issued at the start, so that a wave waits for memory once
// instead of three times (own state, then neighbour face nodes, then U0):
//   * U_k of the element's own nodes into registers (coalesced);
//   * the neighbour face nodes of all three directions straight into LDS by
//     buffer-to-LDS loads (no registers held): per direction and variable
//     one 4-byte load per lane -- in FP64 lane L fetches dword L & 1 of face
//     slot L >> 1, in FP32 lane L < 32 fetches slot L (slots 0-15 the -xi_l
//     face, 16-31 the +xi_l face, tangential index a + 4 b in the two other
//     directions);
//   * U0, when the stage reads it, into LDS by buffer-to-LDS loads as well
//     (FP64: two 4-byte loads per lane and variable, FP32: one), read only
//     by the output.
// The directions are then processed one after the other, each followed by
// the interface correction of the lanes on its faces (own flux still in
// registers).  In FP64 the derivative sweeps run on the matrix core: the
// 4-block 4x4x4 MFMA multiplies, in block b, A[i][k] held by lane
// i + 4b + 16k with B[k][n] held by lane n + 4b + 16k and accumulates into
// C[i][n] held by lane n + 4b + 16i, i.e. it contracts over lane bits 4-5 and
// returns the result in those bits.  The node index is x + 4y + 16z on the
// lane, so
//   * along z the lane's own flux is the B operand, the scaled D entry
//     D[i][k] of lane i + 4b + 16k the A operand, the lane's own accumulator
//     the C operand: no data movement at all;
//   * along x (y) lane L takes as B operand the flux of node T(L) (S(L)),
//     T swapping lane bits 0-1 with 4-5 (S: 2-3 with 4-5), so that the
//     contraction index sits in bits 4-5; lane L then holds the result of
//     node T(L) (S(L)).  T and S are their own inverses, so both moves are a
//     fetch from lane T(L) (S(L)) by a lane permute (ds_bpermute, two 32-bit
//     moves per double): the operand before the product, the result after.
// Per direction that is 5 matrix instructions and 5 KB of permute traffic
// per wave instead of 20 FMAs and 14.5 KB of LDS traffic (a staged flux swept
// with D read from LDS), and no LDS tile for the flux: with U0 in LDS
// instead of ten registers the FP64 kernel holds 74 VGPRs and runs 6 waves
// per SIMD (86 VGPRs and 5 waves with U0 in registers and a staged flux).
// Being one wave, the workgroup needs no barrier: LDS accesses of a wave
// complete in order, and a wave-level fence keeps the compiler from
// reordering them.  The LDS data of the buffer-to-LDS loads is read only
// after an explicit wait for all of the wave's loads (wait_vmem_all).
//
// FP32 form: the state, U0, the output and the neighbour face nodes in LDS
// are float, fluxes and face corrections double.  In every direction it
// stages the flux as the float difference from the element's first-node
// flux (D annihilates constants, so the sum is unchanged and the rounding
// error is relative to the variation inside the element) and sweeps it in
// float from LDS into a float accumulator.  It is bound by vector
// instruction issue at cache-resident sizes, and the FP64 matrix instruction
// occupies the SIMD about as long as the FMAs it replaces: a double matrix
// path measured slower there (and, needing more registers, one wave per
// SIMD fewer, also past the Infinity Cache).
//
// The interface correction of a lane on the s face of direction l
// (s = +1 on the +xi_l face, -1 on the -xi_l face) is the Rusanov
// difference 2 (F* - F_own) = (F_nb - F_own) - s lam (U_nb - U_own) times
// -s (2/h_l) / (2 w_end); with c = (2/h_l) / (2 w_end) it is
//     c lam (U_nb - U_own) - s c (F_nb - F_own).
// ---------------------------------------------------------------------------
// double value of lane 0 (wave-uniform)
__device__ __forceinline__ double lane0(double x) {
  const u32x2 w = __builtin_bit_cast(u32x2, x);
  u32x2 r;
  r.x = __builtin_amdgcn_readfirstlane(w.x);
  r.y = __builtin_amdgcn_readfirstlane(w.y);
  return __builtin_bit_cast(double, r);
}

// U0: whether the stage reads U0 (a != 0 in a Shu-Osher stage); without it
// the FP64 kernel needs 3.8 KB of LDS and 72 VGPRs and runs 7 waves per SIMD
// instead of 6.  PV: a dual stage (mode 2) that reads V, with U0: V is loaded
// into registers at entry with the other reads instead of at the output.
template <typename T, bool NT, bool U0, bool PV>
__global__ void __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu((!std::is_same<T, float>::value && !U0) ? 7 : 4)))
k_stage_n3(StageParams sp, MeshView mv, PhysConst pc) {
  using PHYS = EulerPhys<3>;
  constexpr int DIM = 3, N = 3, n = 4, NP = 64, NV = 5;
  constexpr bool F32 = std::is_same<T, float>::value;
  constexpr int CP = NT ? CPOL_NT : 0;  // policy of the streams no other workgroup reads: U0 and the output
  constexpr int WPV = F32 ? 32 : 64;  // dwords of face data per direction and variable
  __shared__ T sF[F32 ? NV : 1][F32 ? NP : 1];  // FP32: the staged flux of the float sweeps
  __shared__ float sDg[F32 ? DIM : 1][F32 ? n * n : 1];  // FP32: D scaled by -2/h_l
  __shared__ __attribute__((aligned(16))) unsigned sNb[DIM][NV][WPV];
  __shared__ __attribute__((aligned(16))) T sU0[U0 ? NV : 1][U0 ? NP : 1];

  const int tid = threadIdx.x;
  // matrix-core A operand: D[i][k] on lane i + 4b + 16k
  // D[tid] for the FP32 form's tables of scaled rows (lanes < 16)
  const double dsc = (F32 && tid < n * n) ? mv.K->D[tid] : 0.0;
  const double dA = F32 ? 0.0 : mv.K->D[(tid & 3) * n + (tid >> 4)];
  const int E = mv.E;
  const int blk = xcd_remap(blockIdx.x, gridDim.x);
  const int b = blk / E;
  const int e = zfast_block<1>(blk - b * E, mv);
  const int ec = wave_uniform(e);
  const int* nb = mv.nbr + (size_t)ec * 2 * DIM;
  int nbl[2 * DIM];
#pragma unroll
  for (int q = 0; q < 2 * DIM; ++q) nbl[q] = nb[q];
  double g[DIM];
#pragma unroll
  for (int l = 0; l < DIM; ++l) g[l] = mv.geo[(size_t)ec * 4 + l];
  const double hwinv = 0.5 * mv.K->wend_inv;
  const int ii[3] = {tid & 3, (tid >> 2) & 3, tid >> 4};
  const int stride[3] = {1, 4, 16};

  const size_t plane = (size_t)E * NP;
  const size_t abytes = (size_t)NV * plane * sizeof(T);
  const unsigned pstride = (unsigned)(plane * sizeof(T));
  const rsrc_t rU = make_rsrc(static_cast<const T*>(sp.Uk) + (size_t)b * NV * plane, abytes);
  const unsigned off = (unsigned)(ec * NP + tid);

  // own state into registers
  double u[NV];
#pragma unroll
  for (int v = 0; v < NV; ++v) u[v] = Buf<T>::load(rU, off, v * pstride);
  // neighbour face nodes into LDS
  {
    const int slot = F32 ? tid : tid >> 1, half = F32 ? 0 : tid & 1;
    const bool upper = (slot & 16) != 0;  // slot on the +xi_l face
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
        for (int v = 0; v < NV; ++v)
          __builtin_amdgcn_raw_ptr_buffer_load_lds(rU, DG_LDS_PTR(&sNb[l][v][0]), 4, voff, v * pstride, 0, 0);
      }
    }
  }
  constexpr bool use_u0 = U0;  // the host launches this instantiation iff mode != 0 and a != 0
  double vr[PV ? NV : 1];       // PV: V of the dual stage, in registers from the start
  if constexpr (PV) {
    const rsrc_t rv = make_rsrc(static_cast<const T*>(sp.V) + (size_t)b * NV * plane, abytes);
#pragma unroll
    for (int v = 0; v < NV; ++v) vr[v] = Buf<T>::template load<CP>(rv, off, v * pstride);
  }
  if constexpr (use_u0) {  // U0 into LDS, one 4-byte load per lane and dword
    const rsrc_t r0 = make_rsrc(static_cast<const T*>(sp.U0) + (size_t)b * NV * plane, abytes);
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      if constexpr (F32) {
        __builtin_amdgcn_raw_ptr_buffer_load_lds(r0, DG_LDS_PTR(&sU0[v][0]), 4, off * 4u, v * pstride, 0, CP);
      } else {
        // lane L fetches dword L of the element's 512-byte plane, then dword 64 + L
        const unsigned o = (unsigned)(ec * NP) * 8u + 4u * (unsigned)tid;
        __builtin_amdgcn_raw_ptr_buffer_load_lds(r0, DG_LDS_PTR(&sU0[v][0]), 4, o, v * pstride, 0, CP);
        __builtin_amdgcn_raw_ptr_buffer_load_lds(r0, DG_LDS_PTR(&sU0[v][32]), 4, o + 256u, v * pstride, 0, CP);
      }
    }
  }

  Thermo th;
  const bool ok = PHYS::thermo(u, th, pc);
  if (!ok) report_nonphysical(mv.counters, mv.first_bad, ((unsigned long long)b * E + e) * NP + tid);
  double vel[DIM];
#pragma unroll
  for (int d = 0; d < DIM; ++d) vel[d] = u[1 + d] * th.ri;
  const double aown = wave_sound<PHYS, F32>(th);
  if constexpr (F32) {
    if (tid < n * n) {
#pragma unroll
      for (int l = 0; l < DIM; ++l) sDg[l][tid] = static_cast<float>(-g[l] * dsc);
    }
  }
  // nodes whose flux this lane holds as B operand along x and y
  const int tx = (tid >> 4) | (tid & 12) | ((tid & 3) << 4);
  const int ty = (tid & 3) | ((tid >> 4) << 2) | (((tid >> 2) & 3) << 4);
  // byte offset of this lane's slot in sNb[l][v] for each direction l, one
  // byte per direction (meaningful on the lanes of an l face, whose face
  // side is the low bit of their index along l):
  //   x: slot 16 (i & 1) + j + 4 k,  y: 16 (j & 1) + i + 4 k,  z: 16 (k & 1) + i + 4 j
  const unsigned sx = ((tid & 1) << 4) | (tid >> 2);
  const unsigned sy = (((tid >> 2) & 1) << 4) | (tid & 3) | ((tid >> 4) << 2);
  const unsigned sz = (((tid >> 4) & 1) << 4) | (tid & 15);
  constexpr unsigned SB = F32 ? 2 : 3;  // log2 of the bytes of one slot
  const unsigned fslots = (sx << SB) | ((sy << SB) << 8) | ((sz << SB) << 16);

  T acc[NV];
#pragma unroll
  for (int v = 0; v < NV; ++v) acc[v] = T(0);
#pragma unroll
  for (int l = 0; l < DIM; ++l) {
    const int il = ii[l];
    double F[NV];
    PHYS::flux(u, vel[l], th.p, l, F);
    if constexpr (F32) {
      // float sweep of the staged flux difference from LDS
#pragma unroll
      for (int v = 0; v < NV; ++v) sF[v][tid] = static_cast<float>(F[v] - lane0(F[v]));
      wave_lds_fence();
      const int st = stride[l], base = tid - il * st;
      float drow[n];
#pragma unroll
      for (int m = 0; m < n; ++m) drow[m] = sDg[l][il * n + m];
#pragma unroll
      for (int v = 0; v < NV; ++v)
#pragma unroll
        for (int m = 0; m < n; ++m) acc[v] = fma(drow[m], sF[v][base + m * st], acc[v]);
      // interface correction on the l faces: 2 (F* - F_own) = (F_nb - F_own) - s lam (U_nb - U_own),
      // added times -s (2/h_l) / (2 w_end); the neighbour face nodes (and U0)
      // arrive in LDS by buffer-to-LDS loads
      if (l == 0) wait_vmem_all();
      const int side = (il == 0) ? 0 : ((il == N) ? 1 : -1);
      if (side >= 0) {
        const int o1 = l == 0 ? 1 : 0, o2 = l == 2 ? 1 : 2;
        const int slot = side * 16 + ii[o1] + 4 * ii[o2];
        double un[NV];
#pragma unroll
        for (int v = 0; v < NV; ++v) un[v] = static_cast<double>(__builtin_bit_cast(float, sNb[l][v][slot]));
        Thermo tn;
        PHYS::thermo(un, tn, pc);
        const double vn = un[1 + l] * tn.ri;
        double Fn[NV];
        PHYS::flux(un, vn, tn.p, l, Fn);
        const double lam = fmax(fabs(vel[l]) + aown, fabs(vn) + wave_sound<PHYS, F32>(tn));
        const double sgn = side == 1 ? 1.0 : -1.0;
        const double hs = sgn * lam;
        const double sc = -sgn * (g[l] * hwinv);
#pragma unroll
        for (int v = 0; v < NV; ++v) {
          const double dv = fma(-hs, un[v] - u[v], Fn[v] - F[v]);
          acc[v] = fma(static_cast<float>(sc), static_cast<float>(dv), acc[v]);
        }
      }
      wave_lds_fence();  // the next direction overwrites sF
    } else {
      const double al = -g[l] * dA;  // D scaled by -2/h_l
      if (l < 2) {
        const int src = l == 0 ? tx : ty;
#pragma unroll
        for (int v = 0; v < NV; ++v)
          acc[v] += lane_fetch(src, __builtin_amdgcn_mfma_f64_4x4x4f64(al, lane_fetch(src, F[v]), 0.0, 0, 0, 0));
      } else {
#pragma unroll
        for (int v = 0; v < NV; ++v) acc[v] = __builtin_amdgcn_mfma_f64_4x4x4f64(al, F[v], acc[v], 0, 0, 0);
      }
      // interface correction on the l faces; the neighbour face nodes (and
      // U0) arrive in LDS by buffer-to-LDS loads
      if (l == 0) wait_vmem_all();
      if (il == 0 || il == N) {
        const unsigned so = (fslots >> (8 * l)) & 0xffu;
        double un[NV];
#pragma unroll
        for (int v = 0; v < NV; ++v)
          un[v] = *reinterpret_cast<const double*>(reinterpret_cast<const char*>(&sNb[l][v][0]) + so);
        Thermo tn;
        PHYS::thermo(un, tn, pc);
        const double vn = un[1 + l] * tn.ri;
        double Fn[NV];
        PHYS::flux(un, vn, tn.p, l, Fn);
        const double lam = fmax(fabs(vel[l]) + aown, fabs(vn) + wave_sound<PHYS, F32>(tn));
        const double c = g[l] * hwinv;
        const double cl = c * lam;
        const double cs = (il == N) ? -c : c;
#pragma unroll
        for (int v = 0; v < NV; ++v) acc[v] = fma(cs, Fn[v] - F[v], fma(cl, un[v] - u[v], acc[v]));
      }
    }
  }

  // ---- output ----------------------------------------------------------------
  const rsrc_t ro = make_rsrc(static_cast<T*>(sp.out) + (size_t)b * NV * plane, abytes);
  if (sp.mode == 0) {
#pragma unroll
    for (int v = 0; v < NV; ++v) Buf<T>::template store<CP>(ro, off, acc[v], v * pstride);
    return;
  }
  T r[NV];
#pragma unroll
  for (int v = 0; v < NV; ++v) {
    r[v] = fma(T(sp.c), acc[v], T(sp.b) * T(u[v]));
    if constexpr (use_u0) r[v] = fma(T(sp.a), sU0[v][tid], r[v]);
  }
  if (sp.rho_min > 0.0 || sp.p_min > 0.0) {  // the floor itself in double
    if constexpr (F32) {
      double rd[NV];
#pragma unroll
      for (int v = 0; v < NV; ++v) rd[v] = r[v];
      positivity_floor(rd, sp.rho_min, sp.p_min, 1.0 / (pc.gamma - 1.0), mv.counters);
#pragma unroll
      for (int v = 0; v < NV; ++v) r[v] = T(rd[v]);
    } else {
      positivity_floor(r, sp.rho_min, sp.p_min, 1.0 / (pc.gamma - 1.0), mv.counters);
    }
  }
#pragma unroll
  for (int v = 0; v < NV; ++v) Buf<T>::template store<CP>(ro, off, r[v], v * pstride);
  if (sp.mode == 2) {  // second combination of the same L(Uk), no floor
    const rsrc_t r2 = make_rsrc(static_cast<T*>(sp.out2) + (size_t)b * NV * plane, abytes);
    const bool use_v = sp.a2 != 0.0;
    const rsrc_t rv = make_rsrc(static_cast<const T*>(use_v ? sp.V : sp.Uk) + (size_t)b * NV * plane, abytes);
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      T w = fma(T(sp.c2), acc[v], T(sp.b2) * T(u[v]));
      if constexpr (PV) w = fma(T(sp.a2), T(vr[v]), w);
      else if (use_v) w = fma(T(sp.a2), T(Buf<T>::load(rv, off, v * pstride)), w);
      Buf<T>::store(r2, off, w, v * pstride);
    }
  }
}

// ---------------------------------------------------------------------------
// 2:1 mortar fluxes (2-D): one workgroup per non-conforming face and batch
// member.  Lane (k, q) interpolates the coarse trace onto node q of mortar k,
// evaluates the Rusanov flux against fine element k (unit normal: fine and
// coarse lifts both use their own 2/h), and writes the fine row; the coarse
// row is the L2 projection sum_k Pr_k F*_k (the coarse/mortar length ratio 2
// cancels against the ratio of the contravariant normals).
// ---------------------------------------------------------------------------
template <int N, class PHYS, typename T>
__global__ void __launch_bounds__(64)
k_mortar(const MortarRec* recs, const T* U, MeshView mv, PhysConst pc) {
  constexpr int n = N + 1, NP = n * n, NV = PHYS::NV;
  __shared__ double sFs[2][n][NV];
  const MortarRec r = recs[blockIdx.x];
  const int b = blockIdx.y;
  const int tid = threadIdx.x;
  const int E = mv.E;
  const size_t plane = (size_t)E * NP;
  const size_t bofs = (size_t)b * NV * plane;
  const int l = r.l;
  auto nodeidx = [&](int along, int tang) { return l == 0 ? along + n * tang : tang + n * along; };
  const int cend = r.side ? N : 0;
  const int fend = r.side ? 0 : N;
  if (tid < 2 * n) {
    const int k = tid / n, q = tid - (tid / n) * n;
    double uc[NV], uf[NV];
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      double s = 0.0;
#pragma unroll
      for (int j = 0; j < n; ++j)
        s = fma(mv.K->Pf[k][q * n + j], ld(U + bofs + v * plane + (size_t)r.coarse * NP + nodeidx(cend, j)), s);
      uc[v] = s;
      uf[v] = ld(U + bofs + v * plane + (size_t)r.fine[k] * NP + nodeidx(fend, q));
    }
    Thermo tc, tf;
    PHYS::thermo(uc, tc, pc);
    PHYS::thermo(uf, tf, pc);
    double Fs[NV];
    if (r.side == 1) rusanov<PHYS>(uc, tc, uf, tf, l, Fs);   // coarse on the -xi_l side
    else rusanov<PHYS>(uf, tf, uc, tc, l, Fs);
    double* dst = const_cast<double*>(mv.mortar_flux) + (((size_t)b * mv.nrows + r.row_f[k]) * n + q) * NV;
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      dst[v] = Fs[v];
      sFs[k][q][v] = Fs[v];
    }
  }
  __syncthreads();
  if (tid < n) {
    const int i = tid;
    double* dst = const_cast<double*>(mv.mortar_flux) + (((size_t)b * mv.nrows + r.row_c) * n + i) * NV;
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      double s = 0.0;
#pragma unroll
      for (int k = 0; k < 2; ++k)
#pragma unroll
        for (int q = 0; q < n; ++q) s = fma(mv.K->Pr[k][i * n + q], sFs[k][q][v], s);
      dst[v] = s;
    }
  }
}

// ---------------------------------------------------------------------------
// dispatch
// ---------------------------------------------------------------------------
// the Infinity Cache (MALL) of the device: 256 MiB
constexpr size_t NT_STATE_BYTES = (size_t)256 << 20;

template <int DIM, int N, class PHYS, typename T, bool MORTAR, bool SPLIT>
static hipError_t go(const Ctx& c, const StageParams& sp, hipStream_t s) {
  using SH = Shape<DIM, N>;
  const int nEB = (c.E + SH::EPB - 1) / SH::EPB;
  const int nblk = nEB * c.B;
  if constexpr (DIM == 3 && N == 3 && std::is_same<PHYS, EulerPhys<3>>::value && !MORTAR && !SPLIT) {
    // states larger than the Infinity Cache are not read back from it by the
    // next stage: there the non-temporal hint keeps U0 and the output from
    // displacing the neighbour faces in L2 (at cache-resident sizes it would
    // send the output past the cache the next stage reads it from)
    const size_t state_bytes = (size_t)c.B * 5 * c.E * 64 * sizeof(T);
    const bool u0 = sp.mode != 0 && sp.a != 0.0;
    // arrays the stage streams: U_k, the output, U0; the dual stage also a
    // second output and V
    const int arrays = 2 + (u0 ? 1 : 0) + (sp.mode == 2 ? 1 + (sp.a2 != 0.0 ? 1 : 0) : 0);
    const bool nt = state_bytes * (sp.mode == 2 ? arrays : 1) > NT_STATE_BYTES;
    const bool pv = u0 && sp.mode == 2 && sp.a2 != 0.0;
    const MeshView mvw = mesh_view(c);
    if (nt && pv) hipLaunchKernelGGL((k_stage_n3<T, true, true, true>), dim3(nblk), dim3(64), 0, s, sp, mvw, c.pc);
    else if (nt && u0) hipLaunchKernelGGL((k_stage_n3<T, true, true, false>), dim3(nblk), dim3(64), 0, s, sp, mvw, c.pc);
    else if (nt) hipLaunchKernelGGL((k_stage_n3<T, true, false, false>), dim3(nblk), dim3(64), 0, s, sp, mvw, c.pc);
    else if (pv) hipLaunchKernelGGL((k_stage_n3<T, false, true, true>), dim3(nblk), dim3(64), 0, s, sp, mvw, c.pc);
    else if (u0) hipLaunchKernelGGL((k_stage_n3<T, false, true, false>), dim3(nblk), dim3(64), 0, s, sp, mvw, c.pc);
    else hipLaunchKernelGGL((k_stage_n3<T, false, false, false>), dim3(nblk), dim3(64), 0, s, sp, mvw, c.pc);
    return hipGetLastError();
  }
  hipLaunchKernelGGL((k_stage<DIM, N, PHYS, T, MORTAR, SPLIT>), dim3(nblk), dim3(SH::BS), 0, s, sp, mesh_view(c),
                     c.pc);
  return hipGetLastError();
}

template <int DIM, class PHYS, typename T, bool MORTAR, bool SPLIT>
static hipError_t go_n(const Ctx& c, const StageParams& sp, hipStream_t s) {
  switch (c.N) {
    case 1: return go<DIM, 1, PHYS, T, MORTAR, SPLIT>(c, sp, s);
    case 2: return go<DIM, 2, PHYS, T, MORTAR, SPLIT>(c, sp, s);
    case 3: return go<DIM, 3, PHYS, T, MORTAR, SPLIT>(c, sp, s);
    case 4: return go<DIM, 4, PHYS, T, MORTAR, SPLIT>(c, sp, s);
    case 5: return go<DIM, 5, PHYS, T, MORTAR, SPLIT>(c, sp, s);
    case 6: return go<DIM, 6, PHYS, T, MORTAR, SPLIT>(c, sp, s);
    case 7: return go<DIM, 7, PHYS, T, MORTAR, SPLIT>(c, sp, s);
  }
  return hipErrorInvalidValue;
}

template <typename T>
static hipError_t stage_t(const Ctx& c, const StageParams& sp, hipStream_t s) {
  if (c.desc.physics == DG_REACTING_EULER) {
    if (c.dim == 2 && c.N == 3 && c.mech.nspecies == 5) return go<2, 3, ReactPhys<2, 5>, T, true, false>(c, sp, s);
    return hipErrorInvalidValue;
  }
  if (c.desc.physics == DG_REACTING_2T) {
    if (c.dim == 2 && c.N == 3 && c.mech.nspecies == 5)
      return go<2, 3, ReactPhys<2, 5, true>, T, true, false>(c, sp, s);
    return hipErrorInvalidValue;
  }
  if (c.desc.volume == DG_VOLUME_SPLIT) {
    if (c.dim == 2) return go_n<2, EulerPhys<2>, T, true, true>(c, sp, s);
    return go_n<3, EulerPhys<3>, T, false, true>(c, sp, s);
  }
  if (c.dim == 2) return go_n<2, EulerPhys<2>, T, true, false>(c, sp, s);
  return go_n<3, EulerPhys<3>, T, false, false>(c, sp, s);
}

hipError_t launch_stage(const Ctx& c, const StageParams& sp, hipStream_t s) {
  return c.desc.precision == DG_F32 ? stage_t<float>(c, sp, s) : stage_t<double>(c, sp, s);
}

template <typename T>
static hipError_t mortar_t(const Ctx& c, const void* U, hipStream_t s) {
  const T* Ut = static_cast<const T*>(U);
  dim3 grid(c.nmortar, c.B);
  if (is_reacting(c.desc.physics)) {
    if (c.N != 3) return hipErrorInvalidValue;
    if (c.desc.physics == DG_REACTING_2T)
      hipLaunchKernelGGL((k_mortar<3, ReactPhys<2, 5, true>, T>), grid, dim3(64), 0, s, c.d_mortars, Ut, mesh_view(c),
                         c.pc);
    else
      hipLaunchKernelGGL((k_mortar<3, ReactPhys<2, 5>, T>), grid, dim3(64), 0, s, c.d_mortars, Ut, mesh_view(c), c.pc);
    return hipGetLastError();
  }
  switch (c.N) {
#define DG_MORTAR_CASE(NN)                                                                                      \
  case NN:                                                                                                      \
    hipLaunchKernelGGL((k_mortar<NN, EulerPhys<2>, T>), grid, dim3(64), 0, s, c.d_mortars, Ut, mesh_view(c), c.pc); \
    return hipGetLastError();
    DG_MORTAR_CASE(1)
    DG_MORTAR_CASE(2)
    DG_MORTAR_CASE(3)
    DG_MORTAR_CASE(4)
    DG_MORTAR_CASE(5)
    DG_MORTAR_CASE(6)
    DG_MORTAR_CASE(7)
#undef DG_MORTAR_CASE
  }
  return hipErrorInvalidValue;
}

hipError_t launch_mortar(const Ctx& c, const void* U, hipStream_t s) {
  if (c.nmortar == 0) return hipSuccess;
  return c.desc.precision == DG_F32 ? mortar_t<float>(c, U, s) : mortar_t<double>(c, U, s);
}

}  // namespace dg
