// Device-side building blocks shared by the DGSEM kernels: compile-time
// element shapes, the XCD-aware block remap, the pointwise physics (primitive
// recovery with positivity flags, physical fluxes, wave speeds) and the
// sticky status reporting.
//
// Arithmetic note: the library is compiled with floating-point contraction
// off, so the same inline function evaluated on the same operands gives the
// same bits at every call site.  Both elements sharing a face evaluate the
// interface flux with the same function on the same (L, R) operands, which is
// what makes the discrete conservation exact up to the summation order.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "dg_internal.hpp"

namespace dg {

constexpr int ipow(int b, int e) { return e == 0 ? 1 : b * ipow(b, e - 1); }

template <int DIM, int N>
struct Shape {
  static constexpr int n = N + 1;
  static constexpr int NP = ipow(n, DIM);       // nodes per element
  static constexpr int NF = ipow(n, DIM - 1);   // nodes per face
  // elements per workgroup: one wave's worth of lanes, at least one element
  // (small workgroups keep the barrier local to one element's wave)
  static constexpr int EPB = NP >= 64 ? 1 : 64 / NP;
  static constexpr int NT = EPB * NP;
  static constexpr int BS = ((NT + 63) / 64) * 64;
};

// Blocks are dispatched round-robin over the 8 XCDs (block w goes to XCD
// w % 8).  Remap so that each XCD walks one contiguous range of element
// blocks: face neighbours then tend to sit in the same XCD's L2.
__device__ __forceinline__ int xcd_remap(int w, int nblocks) {
  const int q = nblocks / 8, r = nblocks % 8;
  const int xcd = w % 8, slot = w / 8;
  return (xcd < r) ? xcd * (q + 1) + slot : r * (q + 1) + (xcd - r) * q + slot;
}

// Order of the element blocks inside each XCD's range.  In lexicographic
// order the z-neighbour of an element is a whole plane (nx*ny elements) away
// in time, beyond what the XCD's L2 keeps while the other streams of the
// stage pass through it; taking groups of dz whole z-planes with z fastest
// (then x, then y) brings the z-neighbour to the adjacent block and the x- and
// y-neighbours to within dz and dz*nx blocks.  On wide meshes dz*nx is itself
// too far (the y-neighbour's lines are evicted before they are used again):
// there the group's columns are cut into tiles of tx = 2^zf_txs, each tile
// taken whole (z fastest, then x inside the tile, then y) before the next, so
// that the y-neighbour is dz*tx blocks away and only the x-neighbours across
// a tile edge are far.  Only for one element per block (the block index is
// the element index); a bijection of [0, E) when dz divides nz and the tiles
// divide nx, which the host ensures.  The Cartesian stage kernel uses it
// (measured at 32^3: 16 % fewer bytes fetched, 1 % faster); the curvilinear,
// Navier-Stokes and adjoint kernels, which stream more arrays per element,
// measured 1-2 % slower with it and keep the plain order.
template <int EPB>
__device__ __forceinline__ int zfast_block(int eb, const MeshView& mv) {
  if constexpr (EPB != 1) {
    return eb;
  } else {
    if (mv.zf_plane == 0) return eb;
    const unsigned dz = 1u << mv.zf_shift;
    const unsigned G = dz * (unsigned)mv.zf_plane;
    if (mv.zf_txs == 0) {
      const unsigned g = (unsigned)eb / G, t = (unsigned)eb - g * G;
      return (int)(g * G + (t & (dz - 1)) * (unsigned)mv.zf_plane + (t >> mv.zf_shift));
    }
    // block ordinal = ((g * nh + h) * ny + y) * tx * dz + xl * dz + zl
    const unsigned Gs = G >> mv.zf_nhs;  // one tile of one group
    const unsigned sg = (unsigned)eb / Gs, t = (unsigned)eb - sg * Gs;
    const unsigned g = sg >> mv.zf_nhs, h = sg & ((1u << mv.zf_nhs) - 1u);
    const unsigned zl = t & (dz - 1), xl = (t >> mv.zf_shift) & ((1u << mv.zf_txs) - 1u);
    const unsigned y = t >> (mv.zf_shift + mv.zf_txs);
    return (int)(g * G + zl * (unsigned)mv.zf_plane + y * (unsigned)mv.zf_nx + (h << mv.zf_txs) + xl);
  }
}

__device__ __forceinline__ void report_nonphysical(int* counters, unsigned long long* first_bad,
                                                   unsigned long long flat) {
  atomicAdd(&counters[CNT_NONPHYSICAL], 1);
  atomicMin(first_bad, flat);
}

template <typename T>
__device__ __forceinline__ double ld(const T* p) { return static_cast<double>(*p); }

// Raw buffer access to one variable plane: the base address and extent live
// in scalar registers, each lane supplies a 32-bit element offset (no 64-bit
// address arithmetic per lane; reads past the extent return 0).  A plane must
// be smaller than 4 GiB, which the library checks at context creation.
typedef __amdgpu_buffer_rsrc_t rsrc_t;
typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));

__device__ __forceinline__ rsrc_t make_rsrc(const void* base, size_t bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), (short)0, (int)(unsigned)bytes, 0x00020000);
}

// Element index i within the descriptor's range; the optional soff is a
// uniform byte offset (e.g. of a variable plane) added in a scalar register.
template <typename T> struct Buf;
// CPOL: the instruction's cache-policy bits (0: default; CPOL_NT: the
// non-temporal hint, for streams that no other workgroup reads again soon).
constexpr int CPOL_NT = 2;
template <> struct Buf<double> {
  template <int CPOL = 0>
  static __device__ __forceinline__ double load(rsrc_t r, unsigned i, unsigned soff = 0) {
    return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, i * 8u, soff, CPOL));
  }
  template <int CPOL = 0>
  static __device__ __forceinline__ void store(rsrc_t r, unsigned i, double x, unsigned soff = 0) {
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2, x), r, i * 8u, soff, CPOL);
  }
};
template <> struct Buf<float> {
  template <int CPOL = 0>
  static __device__ __forceinline__ double load(rsrc_t r, unsigned i, unsigned soff = 0) {
    return static_cast<double>(
        __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, i * 4u, soff, CPOL)));
  }
  template <int CPOL = 0>
  static __device__ __forceinline__ void store(rsrc_t r, unsigned i, double x, unsigned soff = 0) {
    __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, static_cast<float>(x)), r, i * 4u, soff,
                                          CPOL);
  }
};

// n . F(U) for the Euler flux: (rho v_n, m v_n + p n, (E + p) v_n), v_n = v . n
template <int DIM>
__device__ __forceinline__ void normal_flux(const double (&U)[DIM + 2], const double (&vel)[DIM], double p,
                                            const double (&n)[DIM], double (&F)[DIM + 2]) {
  double vn = 0.0;
#pragma unroll
  for (int d = 0; d < DIM; ++d) vn = fma(vel[d], n[d], vn);
  F[0] = U[0] * vn;
#pragma unroll
  for (int d = 0; d < DIM; ++d) F[1 + d] = fma(U[1 + d], vn, p * n[d]);
  F[DIM + 1] = (U[DIM + 1] + p) * vn;
}

// Single-wave workgroups: LDS accesses of a wave complete in order, so a
// wave-level fence (no barrier) orders one lane's LDS writes before another
// lane's reads and keeps the compiler from moving them across.
__device__ __forceinline__ void wave_lds_fence() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// The value x of lane src (a lane index of the wave), for a double: two
// 32-bit lane permutes (ds_bpermute, on the LDS crossbar; no LDS memory).
__device__ __forceinline__ double lane_fetch(int src, double x) {
  const unsigned lo = (unsigned)__builtin_bit_cast(unsigned long long, x);
  const unsigned hi = (unsigned)(__builtin_bit_cast(unsigned long long, x) >> 32);
  const unsigned rlo = (unsigned)__builtin_amdgcn_ds_bpermute(src * 4, (int)lo);
  const unsigned rhi = (unsigned)__builtin_amdgcn_ds_bpermute(src * 4, (int)hi);
  return __builtin_bit_cast(double, ((unsigned long long)rhi << 32) | rlo);
}

// Wait until every vector-memory load of the wave has completed.  Data that
// buffer-to-LDS loads write is read with plain LDS loads; the compiler's own
// wait before such a read has been found to count only part of the
// outstanding buffer-to-LDS loads when more than a few are in flight, so the
// kernels that use them wait for all loads explicitly before their first
// read of that data.
__device__ __forceinline__ void wait_vmem_all() { asm volatile("s_waitcnt vmcnt(0)" ::: "memory"); }

// an LDS address for the buffer-to-LDS load builtin
#define DG_LDS_PTR(p) ((__attribute__((address_space(3))) void*)(p))

// Make a value the compiler cannot prove uniform a scalar (only valid when it
// is uniform across the wave).
__device__ __forceinline__ int wave_uniform(int x) { return __builtin_amdgcn_readfirstlane(x); }

// Reciprocal and square root for the hot loops, from the hardware estimates
// (relative error about 2^-24) refined in FMA chains: the reciprocal by one
// Newton-Raphson step (at most 11 units in the last place, measured over 2^20
// operands in [1e-3, 1e3]); the square root by one step of the coupled
// Goldschmidt iteration (Markstein's formulation) and one residual
// correction (at most 0.5 units in the last place on the same operands).
// Plain sequences of fma: every call site rounds identically.
__device__ __forceinline__ double frcp(double x) {
  const double r = __builtin_amdgcn_rcp(x);
  return fma(r, fma(-x, r, 1.0), r);
}

__device__ __forceinline__ double fsqrt(double x) {
  const double y = __builtin_amdgcn_rsq(x);
  double g = x * y;
  double h = 0.5 * y;
  const double r = fma(-g, h, 0.5);
  g = fma(g, r, g);
  h = fma(h, r, h);
  const double d = fma(-g, g, x);
  return fma(d, h, g);
}

// Positivity floor of an ideal-gas stage output r = (rho, m, E): rho is
// clipped to rho_min with the momentum kept, then E is raised to
// p_min/(gamma-1) + |m|^2/(2 rho) where it lies below, i.e. to pressure p_min.
// Returns whether it changed anything.  Nodes it acts on are counted per wave
// (one atomic per wave) in counters[CNT_FLOORED].
template <int NV>
__device__ __forceinline__ void positivity_floor(double (&r)[NV], double rho_min, double p_min, double gm1i,
                                                 int* counters) {
  bool acted = false;
  if (r[0] < rho_min) {
    r[0] = rho_min;
    acted = true;
  }
  double m2 = 0.0;
#pragma unroll
  for (int d = 1; d < NV - 1; ++d) m2 = fma(r[d], r[d], m2);
  const double emin = fma(0.5 * m2, frcp(r[0]), p_min * gm1i);
  if (r[NV - 1] < emin) {
    r[NV - 1] = emin;
    acted = true;
  }
  const unsigned long long mask = __ballot(acted);
  if (acted && (int)__lane_id() == __ffsll(mask) - 1) atomicAdd(&counters[CNT_FLOORED], (int)__popcll(mask));
}

// ---------------------------------------------------------------------------
// Pointwise physics.  Thermo holds what a flux or a wave speed needs beyond U:
// 1/rho, the pressure and the factor k with a^2 = k p / rho.
// ---------------------------------------------------------------------------
struct Thermo {
  double ri;  // 1 / rho
  double p;   // pressure
  double k;   // a^2 = k p ri
};

// Euler / inviscid Navier-Stokes: U = (rho, m_1..m_DIM, E), ideal gas.
template <int DIM>
struct EulerPhys {
  static constexpr int NV = DIM + 2;
  static constexpr int MOM = 1;  // index of the first momentum component
  static constexpr int NDIM = DIM;
  // Returns false for rho <= 0 or p <= 0 (values still computed).
  __device__ static __forceinline__ bool thermo(const double (&U)[NV], Thermo& t, const PhysConst& c) {
    t.ri = frcp(U[0]);
    double m2 = 0.0;
#pragma unroll
    for (int d = 0; d < DIM; ++d) m2 = fma(U[1 + d], U[1 + d], m2);
    t.p = (c.gamma - 1.0) * fma(-0.5 * m2, t.ri, U[DIM + 1]);
    t.k = c.gamma;
    return (U[0] > 0.0) && (t.p > 0.0);
  }
  // physical flux along Cartesian direction l, given u_l and p
  __device__ static __forceinline__ void flux(const double (&U)[NV], double ul, double p, int l, double (&F)[NV]) {
    F[0] = U[1 + l];
#pragma unroll
    for (int d = 0; d < DIM; ++d) F[1 + d] = U[1 + d] * ul;
    F[1 + l] += p;
    F[DIM + 1] = (U[DIM + 1] + p) * ul;
  }
};

// Reacting Euler, one temperature: U = (rho_1..rho_NS, m, E).
//   E = sum rho_s cv_s T + |m|^2/(2 rho) + sum rho_s h0_s,  p = T sum rho_s R_s,
//   frozen sound speed a^2 = (1 + sum rho_s R_s / sum rho_s cv_s) p / rho.
// Two temperatures (TWO_T): U = (rho_1..rho_NS, m, E, E_v), the vibrational
// energy E_v taken out of E before T is recovered and advected as E_v u_l.
template <int DIM, int NS, bool TWO_T = false>
struct ReactPhys {
  // (rho_1..rho_NS, m_1..m_DIM, E) and, with two temperatures, E_v last
  static constexpr int NV = NS + DIM + 1 + (TWO_T ? 1 : 0);
  static constexpr int MOM = NS;
  static constexpr int NDIM = DIM;
  __device__ static __forceinline__ bool thermo(const double (&U)[NV], Thermo& t, const PhysConst& c) {
    double rho = 0.0, cv = 0.0, h0 = 0.0, Rm = 0.0;
#pragma unroll
    for (int s = 0; s < NS; ++s) {
      rho += U[s];
      cv = fma(U[s], c.cv[s], cv);
      h0 = fma(U[s], c.h0[s], h0);
      Rm = fma(U[s], c.R[s], Rm);
    }
    t.ri = frcp(rho);
    double m2 = 0.0;
#pragma unroll
    for (int d = 0; d < DIM; ++d) m2 = fma(U[NS + d], U[NS + d], m2);
    const double cvi = frcp(cv);
    // translational-rotational energy: the vibrational energy E_v is its own variable
    const double e_tr = TWO_T ? U[NS + DIM] - U[NS + DIM + 1] : U[NS + DIM];
    const double T = (fma(-0.5 * m2, t.ri, e_tr) - h0) * cvi;
    t.p = T * Rm;
    t.k = fma(Rm, cvi, 1.0);
    return (rho > 0.0) && (T > 0.0) && (t.p > 0.0);
  }
  __device__ static __forceinline__ void flux(const double (&U)[NV], double ul, double p, int l, double (&F)[NV]) {
#pragma unroll
    for (int s = 0; s < NS; ++s) F[s] = U[s] * ul;
#pragma unroll
    for (int d = 0; d < DIM; ++d) F[NS + d] = U[NS + d] * ul;
    F[NS + l] += p;
    F[NS + DIM] = (U[NS + DIM] + p) * ul;
    if constexpr (TWO_T) F[NS + DIM + 1] = U[NS + DIM + 1] * ul;
  }
};

template <class PHYS>
__device__ __forceinline__ double velocity(const double (&U)[PHYS::NV], const Thermo& t, int d) {
  return U[PHYS::MOM + d] * t.ri;
}

template <class PHYS>
__device__ __forceinline__ double sound(const Thermo& t) {
  return fsqrt(t.k * t.p * t.ri);
}

// Rusanov (local Lax-Friedrichs) flux for the unit normal e_l between the
// state on the -xi_l side (L) and the +xi_l side (R):
//   F* = (F_l(UL) + F_l(UR))/2 - lam (UR - UL)/2,
//   lam = max(|uL_l| + aL, |uR_l| + aR).
// The caller scales by |Ja^l|: with an axis-aligned normal the flux and the
// dissipation both scale linearly, so the unnormalised-normal flux of the
// surface integral is |Ja^l| times this value.
template <class PHYS>
__device__ __forceinline__ void rusanov(const double (&UL)[PHYS::NV], const Thermo& tL, const double (&UR)[PHYS::NV],
                                        const Thermo& tR, int l, double (&Fs)[PHYS::NV]) {
  double FL[PHYS::NV], FR[PHYS::NV];
  const double uL = velocity<PHYS>(UL, tL, l), uR = velocity<PHYS>(UR, tR, l);
  PHYS::flux(UL, uL, tL.p, l, FL);
  PHYS::flux(UR, uR, tR.p, l, FR);
  const double cL = fabs(uL) + sound<PHYS>(tL);
  const double cR = fabs(uR) + sound<PHYS>(tR);
  const double hl = 0.5 * ((cL >= cR) ? cL : cR);
#pragma unroll
  for (int v = 0; v < PHYS::NV; ++v) Fs[v] = fma(-hl, UR[v] - UL[v], 0.5 * (FL[v] + FR[v]));
}

}  // namespace dg
