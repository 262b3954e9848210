// Internal declarations of libdg: the context, the per-launch argument
// blocks and the kernel launchers (one translation unit per kernel family).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>
#include <vector>

#include "dg.h"

namespace dg {

constexpr int MAXN1 = 8;  // highest supported N + 1

enum CounterIdx { CNT_NONPHYSICAL = 0, CNT_NEWTON = 1, CNT_CLIPS = 2, CNT_ITERS = 3, CNT_FLOORED = 4, CNT_N = 5 };

// Reference-element and mortar constants, resident in device memory.
struct RefConsts {
  double D[MAXN1 * MAXN1];          // D[i*n + m]: d l_m / dxi at xi_i
  double Dt[MAXN1 * MAXN1];         // transpose, D[m*n + i]
  float Df[MAXN1 * MAXN1];          // D rounded to float (FP32 form)
  double w[MAXN1];                  // GLL weights
  double xi[MAXN1];                 // GLL nodes
  double wend_inv;                  // 1 / w_0 (= 1 / w_N)
  double Pf[2][MAXN1 * MAXN1];      // coarse face -> mortar k  [i*n + j]
  double Pr[2][MAXN1 * MAXN1];      // mortar k -> coarse face  [i*n + j]
};

// Pointwise physics constants passed by value with every launch.
struct PhysConst {
  double gamma, mu, prandtl;
  double cv[DG_MAX_SPECIES], h0[DG_MAX_SPECIES], R[DG_MAX_SPECIES];
};

// Everything a stage/RHS launch reads besides the state buffers.
struct MeshView {
  int E;
  int B;
  const int* nbr;             // [E][2*dim]: >= 0 conforming neighbour, < 0: -(row+1)
  const double* geo;          // [E][4]: 2/h_x, 2/h_y, 2/h_z, J
  const RefConsts* K;
  const double* mortar_flux;  // [B][rows][NF][nv], unit-normal interface flux
  int nrows;
  int* counters;
  unsigned long long* first_bad;
  // 3-D Cartesian meshes (lexicographic element order, x fastest): element
  // blocks are taken in groups of 2^zf_shift whole z-planes of zf_plane
  // elements each, z fastest inside a group; zf_plane = 0 keeps the order.
  // zf_txs > 0: the group's x range (zf_nx columns) is cut into 2^zf_nhs
  // tiles of 2^zf_txs columns, taken one after the other
  int zf_shift = 0, zf_plane = 0;
  int zf_txs = 0, zf_nhs = 0, zf_nx = 0;
};

// One 2:1 non-conforming face (2-D): coarse element, direction, side of the
// coarse element the face lies on (1: its +l face), the two fine elements in
// order of increasing tangential coordinate, and the flux rows of the coarse
// face and of the two fine faces.
struct MortarRec {
  int coarse, l, side;
  int fine[2];
  int row_c, row_f[2];
};

struct StageParams {
  const void* U0;
  const void* Uk;
  void* out;
  double a, b, c;
  int mode;  // 0: out = L(Uk);  1: out = a U0 + b Uk + c L(Uk);  2: also out2
  // mode 2: out2 = a2 V + b2 Uk + c2 L(Uk), without the floor
  const void* V = nullptr;
  void* out2 = nullptr;
  double a2 = 0.0, b2 = 0.0, c2 = 0.0;
  // positivity floor on out (modes 1 and 2); off when both are 0
  double rho_min = 0.0, p_min = 0.0;
};

struct Ctx {
  dg_desc desc;
  dg_mechanism mech;
  dg_vibration vib;              // two-temperature physics only (zeroed otherwise)
  int dim, N, n, Np, nv, E, B;
  int device;
  double hmin;
  PhysConst pc;
  // device buffers
  int* d_nbr = nullptr;
  double* d_geo = nullptr;
  double* d_corner = nullptr;
  RefConsts* d_K = nullptr;
  RefConsts h_K;
  int* d_counters = nullptr;
  unsigned long long* d_first_bad = nullptr;
  MortarRec* d_mortars = nullptr;
  int nmortar = 0;
  int nrows = 0;
  double* d_mortar_flux = nullptr;
  double* d_red = nullptr;       // reduction partials
  size_t red_cap = 0;            // doubles
  double* d_red_out = nullptr;   // final reduction results
  void* d_face = nullptr;        // BR1 face buffer
  // implicit chemistry substep: nodes handed from the first pass to the
  // continuation pass ([B*E*Np] records) and their count
  void* d_defer = nullptr;
  int* d_defer_count = nullptr;
  void* d_mech = nullptr;        // mechanism copy on device
  void* d_vib = nullptr;         // vibrational data on device (two-temperature)
  // curvilinear meshes: metric planes [2 + dim*dim][E*Np] (J, 1/J, Ja^l_d at
  // plane 2 + l*dim + d) and the warped node coordinates [dim][E*Np]
  bool curv = false;
  double* d_met = nullptr;
  double* d_xyz = nullptr;
  std::vector<double> h_corner;  // host copy [E][3] lower corners (coords)
  std::vector<double> h_geo;     // host copy [E][4]
};

MeshView mesh_view(const Ctx& c);

inline bool is_reacting(int physics) { return physics == DG_REACTING_EULER || physics == DG_REACTING_2T; }

// ---- launchers (return hipError_t of the launch) ---------------------------
hipError_t launch_stage(const Ctx& c, const StageParams& sp, hipStream_t s);
hipError_t launch_mortar(const Ctx& c, const void* U, hipStream_t s);
hipError_t launch_coords(const Ctx& c, const double* corner, double* xyz, hipStream_t s);
hipError_t launch_integrals(const Ctx& c, const void* U, double* d_out, hipStream_t s);
// allocation-free integrals: partials in a fixed per-GPU device array of
// NOALLOC_SCRATCH_DOUBLES doubles whose address is looked up once per device
constexpr size_t NOALLOC_SCRATCH_DOUBLES = (size_t)1 << 18;  // 2 MiB
hipError_t noalloc_scratch_init(int device);                  // with `device` current
size_t noalloc_integrals_need(const Ctx& c);                   // doubles of scratch one call uses
hipError_t launch_integrals_noalloc(const Ctx& c, const void* U, double* d_out, hipStream_t s);
hipError_t launch_lam_max(const Ctx& c, const void* U, double* d_out, hipStream_t s);
hipError_t launch_source(const Ctx& c, const void* U, void* out, double h, int mode, hipStream_t s);
hipError_t launch_ns(const Ctx& c, const StageParams& sp, hipStream_t s);
hipError_t launch_curv(const Ctx& c, const StageParams& sp, hipStream_t s);
hipError_t launch_adjoint(const Ctx& c, const void* U, const void* lam_out, void* lam_k, void* lam_0,
                          double a, double b, double cdt, int accumulate, hipStream_t s);

}  // namespace dg
