// C ABI of libdg: context creation (mesh tables, reference element, mortar
// operators, mechanism), argument validation and dispatch to the kernels.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "dg_internal.hpp"

using namespace dg;

struct dg_ctx {
  Ctx c;
};

namespace {

thread_local std::string g_last_error;

int fail(int code, const std::string& msg) {
  g_last_error = msg;
  return code;
}

int hip_fail(hipError_t e, const char* where) {
  return fail(DG_ERR_HIP, std::string(where) + ": " + hipGetErrorString(e));
}

// Makes the context's device current for the scope of one call.
struct DeviceGuard {
  int prev = -1;
  bool changed = false;
  explicit DeviceGuard(int dev) {
    if (hipGetDevice(&prev) == hipSuccess && prev != dev) {
      changed = hipSetDevice(dev) == hipSuccess;
    }
  }
  ~DeviceGuard() {
    if (changed) (void)hipSetDevice(prev);
  }
};

// ---------------------------------------------------------------------------
// Reference element on the host (GLL nodes by Newton on P_N', weights
// 2/(N(N+1)P_N^2), derivative matrix in barycentric form with the diagonal set
// so that rows sum to zero).
// ---------------------------------------------------------------------------
void legendre(int N, double x, double& p, double& pm1) {
  double a = 1.0, b = x;
  if (N == 0) {
    p = 1.0;
    pm1 = 0.0;
    return;
  }
  for (int k = 1; k < N; ++k) {
    const double c = ((2 * k + 1) * x * b - k * a) / (k + 1);
    a = b;
    b = c;
  }
  p = b;
  pm1 = a;
}

void gll(int N, double* xi, double* w) {
  const double pi = 3.14159265358979323846;
  xi[0] = -1.0;
  xi[N] = 1.0;
  for (int i = 1; i < N; ++i) {
    double x = -std::cos(pi * i / N);
    for (int it = 0; it < 100; ++it) {
      double p, pm;
      legendre(N, x, p, pm);
      const double dp = N * (x * p - pm) / (x * x - 1.0);
      const double d2p = (2.0 * x * dp - N * (N + 1) * p) / (1.0 - x * x);
      const double dx = dp / d2p;
      x -= dx;
      if (std::fabs(dx) < 1e-17) break;
    }
    xi[i] = x;
  }
  for (int i = 0; i <= N / 2; ++i) {  // exact symmetry
    const double s = 0.5 * (xi[N - i] - xi[i]);
    xi[i] = -s;
    xi[N - i] = s;
  }
  if (N % 2 == 0) xi[N / 2] = 0.0;
  for (int i = 0; i <= N; ++i) {
    double p, pm;
    legendre(N, xi[i], p, pm);
    w[i] = 2.0 / (N * (N + 1) * p * p);
  }
}

double lagrange(const double* xi, int n, int j, double y) {
  double r = 1.0;
  for (int k = 0; k < n; ++k)
    if (k != j) r *= (y - xi[k]) / (xi[j] - xi[k]);
  return r;
}

// Gauss-Legendre nodes/weights, q points
void gauss_legendre(int q, std::vector<double>& x, std::vector<double>& w) {
  const double pi = 3.14159265358979323846;
  x.resize(q);
  w.resize(q);
  for (int i = 0; i < q; ++i) {
    double t = std::cos(pi * (i + 0.75) / (q + 0.5));
    double dp = 0.0;
    for (int it = 0; it < 100; ++it) {
      double p, pm;
      legendre(q, t, p, pm);
      dp = q * (t * p - pm) / (t * t - 1.0);
      const double dt = p / dp;
      t -= dt;
      if (std::fabs(dt) < 1e-17) break;
    }
    double p, pm;
    legendre(q, t, p, pm);
    dp = q * (t * p - pm) / (t * t - 1.0);
    x[i] = t;
    w[i] = 2.0 / ((1.0 - t * t) * dp * dp);
  }
}

// solve M X = A for X (n x n), Gaussian elimination with partial pivoting
void solve_dense(int n, std::vector<double> M, std::vector<double>& A) {
  for (int k = 0; k < n; ++k) {
    int p = k;
    for (int i = k + 1; i < n; ++i)
      if (std::fabs(M[i * n + k]) > std::fabs(M[p * n + k])) p = i;
    if (p != k)
      for (int j = 0; j < n; ++j) {
        std::swap(M[k * n + j], M[p * n + j]);
        std::swap(A[k * n + j], A[p * n + j]);
      }
    for (int i = k + 1; i < n; ++i) {
      const double f = M[i * n + k] / M[k * n + k];
      for (int j = 0; j < n; ++j) {
        M[i * n + j] -= f * M[k * n + j];
        A[i * n + j] -= f * A[k * n + j];
      }
    }
  }
  for (int k = n - 1; k >= 0; --k)
    for (int j = 0; j < n; ++j) {
      double s = A[k * n + j];
      for (int i = k + 1; i < n; ++i) s -= M[k * n + i] * A[i * n + j];
      A[k * n + j] = s / M[k * n + k];
    }
}

void build_refconsts(int N, RefConsts& K) {
  std::memset(&K, 0, sizeof(K));
  const int n = N + 1;
  gll(N, K.xi, K.w);
  K.wend_inv = 1.0 / K.w[0];
  double lam[MAXN1];
  for (int j = 0; j < n; ++j) {
    double p = 1.0;
    for (int k = 0; k < n; ++k)
      if (k != j) p *= (K.xi[j] - K.xi[k]);
    lam[j] = 1.0 / p;
  }
  for (int i = 0; i < n; ++i) {
    double diag = 0.0;
    for (int j = 0; j < n; ++j) {
      if (i == j) continue;
      const double d = (lam[j] / lam[i]) / (K.xi[i] - K.xi[j]);
      K.D[i * n + j] = d;
      diag -= d;
    }
    K.D[i * n + i] = diag;
  }
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) {
      K.Dt[j * n + i] = K.D[i * n + j];
      K.Df[i * n + j] = static_cast<float>(K.D[i * n + j]);
    }
  // mortars: forward interpolation and reverse L2 projection
  std::vector<double> gx, gw;
  gauss_legendre(N + 2, gx, gw);
  std::vector<double> M(n * n, 0.0);
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j)
      for (size_t q = 0; q < gx.size(); ++q)
        M[i * n + j] += gw[q] * lagrange(K.xi, n, i, gx[q]) * lagrange(K.xi, n, j, gx[q]);
  for (int k = 0; k < 2; ++k) {
    for (int i = 0; i < n; ++i) {
      const double s = k == 0 ? 0.5 * (K.xi[i] - 1.0) : 0.5 * (K.xi[i] + 1.0);
      for (int j = 0; j < n; ++j) K.Pf[k][i * n + j] = lagrange(K.xi, n, j, s);
    }
    // A = Pf^T M, then Pr = 1/2 M^{-1} A
    std::vector<double> A(n * n, 0.0);
    for (int i = 0; i < n; ++i)
      for (int j = 0; j < n; ++j)
        for (int q = 0; q < n; ++q) A[i * n + j] += K.Pf[k][q * n + i] * M[q * n + j];
    solve_dense(n, M, A);
    for (int i = 0; i < n * n; ++i) K.Pr[k][i] = 0.5 * A[i];
  }
}

// ---------------------------------------------------------------------------
// Mesh: periodic box, optional 2:1-refined block (2-D)
// ---------------------------------------------------------------------------
struct MeshBuild {
  std::vector<double> corner;  // [E][3]
  std::vector<double> geo;     // [E][4]
  std::vector<int> nbr;        // [E][2*dim]
  std::vector<MortarRec> mortars;
  int nrows = 0;
  double hmin = 0.0;
};

int build_mesh(const dg_desc& d, MeshBuild& mb) {
  const int dim = d.dim;
  int nel[3] = {d.nel[0], d.nel[1], dim == 3 ? d.nel[2] : 1};
  double h0[3];
  for (int l = 0; l < 3; ++l) h0[l] = l < dim ? (d.hi[l] - d.lo[l]) / nel[l] : 1.0;
  const bool patch = dim == 2 && (d.patch_lo[0] != d.patch_hi[0] || d.patch_lo[1] != d.patch_hi[1]);
  auto refined = [&](int cx, int cy) {
    return patch && cx >= d.patch_lo[0] && cx < d.patch_hi[0] && cy >= d.patch_lo[1] && cy < d.patch_hi[1];
  };
  // element order: coarse cells x fastest; refined cells emit 4 children
  const long ncoarse = (long)nel[0] * nel[1] * nel[2];
  std::vector<int> coarse_id(ncoarse, -1);
  std::vector<int> fine_id(patch ? (size_t)4 * nel[0] * nel[1] : 0, -1);
  const int fnx = 2 * nel[0];
  int E = 0;
  mb.corner.clear();
  mb.geo.clear();
  std::vector<int> lev, cxs, cys, czs;
  for (int cz = 0; cz < nel[2]; ++cz)
    for (int cy = 0; cy < nel[1]; ++cy)
      for (int cx = 0; cx < nel[0]; ++cx) {
        if (refined(cx, cy)) {
          for (int fy = 0; fy < 2; ++fy)
            for (int fx = 0; fx < 2; ++fx) {
              const int gx = 2 * cx + fx, gy = 2 * cy + fy;
              fine_id[(size_t)gy * fnx + gx] = E++;
              lev.push_back(1);
              cxs.push_back(gx);
              cys.push_back(gy);
              czs.push_back(0);
            }
        } else {
          coarse_id[((size_t)cz * nel[1] + cy) * nel[0] + cx] = E++;
          lev.push_back(0);
          cxs.push_back(cx);
          cys.push_back(cy);
          czs.push_back(cz);
        }
      }
  mb.corner.assign((size_t)E * 3, 0.0);
  mb.geo.assign((size_t)E * 4, 0.0);
  mb.nbr.assign((size_t)E * 2 * dim, 0);
  mb.hmin = 1e300;
  for (int e = 0; e < E; ++e) {
    const double f = lev[e] ? 0.5 : 1.0;
    const int c[3] = {cxs[e], cys[e], czs[e]};
    double J = 1.0;
    for (int l = 0; l < dim; ++l) {
      const double h = h0[l] * f;
      mb.corner[(size_t)e * 3 + l] = d.lo[l] + c[l] * h;
      mb.geo[(size_t)e * 4 + l] = 2.0 / h;
      J *= 0.5 * h;
      mb.hmin = std::min(mb.hmin, h);
    }
    mb.geo[(size_t)e * 4 + 3] = J;
  }
  auto cid = [&](int x, int y, int z) {
    x = ((x % nel[0]) + nel[0]) % nel[0];
    y = ((y % nel[1]) + nel[1]) % nel[1];
    z = ((z % nel[2]) + nel[2]) % nel[2];
    return coarse_id[((size_t)z * nel[1] + y) * nel[0] + x];
  };
  auto fid = [&](int x, int y) {
    const int fny = 2 * nel[1];
    x = ((x % fnx) + fnx) % fnx;
    y = ((y % fny) + fny) % fny;
    return fine_id[(size_t)y * fnx + x];
  };
  mb.mortars.clear();
  int rows = 0;
  // coarse faces against refined cells create the mortar records
  for (int e = 0; e < E; ++e) {
    for (int l = 0; l < dim; ++l)
      for (int side = 0; side < 2; ++side) {
        int* slot = &mb.nbr[(size_t)e * 2 * dim + 2 * l + side];
        const int sgn = side ? 1 : -1;
        if (lev[e] == 0) {
          int c[3] = {cxs[e], cys[e], czs[e]};
          c[l] += sgn;
          if (d.bc[2 * l] != DG_BC_PERIODIC && (c[l] < 0 || c[l] >= nel[l])) {
            // box side without periodicity: boundary face, code -(1 + type)
            *slot = -(1 + d.bc[2 * l + side]);
            continue;
          }
          const int nb = cid(c[0], c[1], c[2]);
          if (nb >= 0) {
            *slot = nb;
            continue;
          }
          // neighbour cell is refined: mortar, coarse side
          MortarRec r{};
          r.coarse = e;
          r.l = l;
          r.side = side;
          const int t = 1 - l;
          const int pc[2] = {((c[0] % nel[0]) + nel[0]) % nel[0], ((c[1] % nel[1]) + nel[1]) % nel[1]};
          for (int s = 0; s < 2; ++s) {
            int f[2];
            f[l] = 2 * pc[l] + (side ? 0 : 1);
            f[t] = 2 * (t == 0 ? cxs[e] : cys[e]) + s;
            r.fine[s] = fid(f[0], f[1]);
          }
          r.row_c = rows++;
          r.row_f[0] = rows++;
          r.row_f[1] = rows++;
          *slot = -(r.row_c + 1);
          mb.mortars.push_back(r);
        } else {
          int f[2] = {cxs[e], cys[e]};
          f[l] += sgn;
          const int nb = fid(f[0], f[1]);
          if (nb >= 0) *slot = nb;
          else *slot = 0x7fffffff;  // filled from the mortar records below
        }
      }
  }
  for (const MortarRec& r : mb.mortars)
    for (int s = 0; s < 2; ++s) {
      // the fine face touching the coarse one is on the fine element's
      // opposite side along l
      const int fside = r.side ? 0 : 1;
      mb.nbr[(size_t)r.fine[s] * 2 * dim + 2 * r.l + fside] = -(r.row_f[s] + 1);
    }
  for (size_t q = 0; q < mb.nbr.size(); ++q)
    if (mb.nbr[q] == 0x7fffffff) return fail(DG_ERR_ARG, "mesh: unresolved fine face (refined block must be interior-consistent)");
  mb.nrows = rows;
  return DG_OK;
}

// ---------------------------------------------------------------------------
// Curvilinear geometry: warped node coordinates and per-node metrics from the
// degree-N interpolant of every element's nodes (the collocation derivative
// D applied to the node coordinates).  2-D: Ja^1 = (y_2, -x_2),
// Ja^2 = (-y_1, x_1); 3-D: conservative curl form
// (Ja^i)_n = -[curl_xi (X_l grad_xi X_m)]_i with (n, m, l) cyclic, the
// products formed node by node.  J = det(dX_d/dxi_m).  Returns false if the
// map folds (J <= 0 somewhere).
// ---------------------------------------------------------------------------
static void warp_point(const dg_desc& d, const double* x, double* y) {
  const double kTwoPi = 6.283185307179586;
  double L[3], s[3];
  for (int q = 0; q < d.dim; ++q) {
    L[q] = d.hi[q] - d.lo[q];
    s[q] = (x[q] - d.lo[q]) / L[q];
  }
  if (d.dim == 2) {
    y[0] = x[0] + d.warp * L[0] * std::sin(kTwoPi * s[1]);
    y[1] = x[1] + d.warp * L[1] * std::sin(kTwoPi * s[0]);
  } else {
    for (int q = 0; q < 3; ++q)
      y[q] = x[q] + d.warp * L[q] * std::sin(kTwoPi * s[(q + 1) % 3]) * std::sin(kTwoPi * s[(q + 2) % 3]);
  }
}

static bool build_curv(const dg_desc& d, const Ctx& c, const MeshBuild& mb, std::vector<double>& met,
                       std::vector<double>& xyz) {
  const int dim = c.dim, n = c.n, NP = c.Np, E = c.E;
  const size_t P = (size_t)E * NP;
  met.assign((size_t)(2 + dim * dim) * P, 0.0);
  xyz.assign((size_t)dim * P, 0.0);
  const double* D = c.h_K.D;
  const int stride[3] = {1, n, n * n};
  std::vector<double> X(3 * NP), Xl(3 * NP), dX(9 * NP), V(3 * NP);
  auto ijk = [&](int node, int m) { return (node / stride[m]) % n; };
  // d f / d xi_m at `node` for a nodal field f of one element
  auto deriv = [&](const double* f, int m, int node) {
    const int i = ijk(node, m);
    const int base = node - i * stride[m];
    double acc = 0.0;
    for (int k = 0; k < n; ++k) acc += D[i * n + k] * f[base + k * stride[m]];
    return acc;
  };
  for (int e = 0; e < E; ++e) {
    for (int node = 0; node < NP; ++node) {
      double xc[3] = {0.0, 0.0, 0.0}, xw[3] = {0.0, 0.0, 0.0};
      for (int q = 0; q < dim; ++q) {
        const double h = 2.0 / mb.geo[(size_t)e * 4 + q];
        xc[q] = mb.corner[(size_t)e * 3 + q] + (c.h_K.xi[ijk(node, q)] + 1.0) * 0.5 * h;
      }
      warp_point(d, xc, xw);
      for (int q = 0; q < dim; ++q) X[q * NP + node] = xw[q];
    }
    // The metrics are formed from coordinates relative to the element's first
    // node (Xl): derivatives of a constant vanish and so does the curl of a
    // constant times a gradient, so this changes nothing in exact arithmetic,
    // but the rounding becomes relative to the element's size rather than to
    // its distance from the origin.
    for (int q = 0; q < dim; ++q) {
      const double x0 = X[q * NP];
      for (int node = 0; node < NP; ++node) Xl[q * NP + node] = X[q * NP + node] - x0;
    }
    for (int q = 0; q < dim; ++q)
      for (int m = 0; m < dim; ++m)
        for (int node = 0; node < NP; ++node) dX[(q * 3 + m) * NP + node] = deriv(&Xl[q * NP], m, node);
    for (int node = 0; node < NP; ++node) {
      double Ja[3][3] = {{0.0}}, J;
      auto dx = [&](int q, int m) { return dX[(q * 3 + m) * NP + node]; };
      if (dim == 2) {
        Ja[0][0] = dx(1, 1);
        Ja[0][1] = -dx(0, 1);
        Ja[1][0] = -dx(1, 0);
        Ja[1][1] = dx(0, 0);
        J = dx(0, 0) * dx(1, 1) - dx(0, 1) * dx(1, 0);
      } else {
        J = dx(0, 0) * (dx(1, 1) * dx(2, 2) - dx(1, 2) * dx(2, 1)) - dx(0, 1) * (dx(1, 0) * dx(2, 2) - dx(1, 2) * dx(2, 0)) +
            dx(0, 2) * (dx(1, 0) * dx(2, 1) - dx(1, 1) * dx(2, 0));
      }
      if (!(J > 0.0)) return false;
      const size_t at = (size_t)e * NP + node;
      met[at] = J;
      met[P + at] = 1.0 / J;
      if (dim == 2)
        for (int l = 0; l < 2; ++l)
          for (int q = 0; q < 2; ++q) met[(2 + l * 2 + q) * P + at] = Ja[l][q];
      for (int q = 0; q < dim; ++q) xyz[q * P + at] = X[q * NP + node];
    }
    if (dim == 3) {
      for (int nn = 0; nn < 3; ++nn) {
        const int mm = (nn + 1) % 3, ll = (nn + 2) % 3;
        for (int k = 0; k < 3; ++k)
          for (int node = 0; node < NP; ++node) V[k * NP + node] = Xl[ll * NP + node] * dX[(mm * 3 + k) * NP + node];
        for (int node = 0; node < NP; ++node)
          for (int i = 0; i < 3; ++i) {
            const double curl = deriv(&V[((i + 2) % 3) * NP], (i + 1) % 3, node) -
                                deriv(&V[((i + 1) % 3) * NP], (i + 2) % 3, node);
            met[(2 + i * 3 + nn) * P + (size_t)e * NP + node] = -curl;
          }
      }
    }
  }
  return true;
}

bool overlaps(const void* a, const void* b, size_t bytes) {
  if (!a || !b) return false;
  const char* pa = static_cast<const char*>(a);
  const char* pb = static_cast<const char*>(b);
  return pa < pb + bytes && pb < pa + bytes;
}

size_t state_bytes(const Ctx& c) {
  return (size_t)c.B * c.nv * c.E * c.Np * (c.desc.precision == DG_F32 ? 4 : 8);
}

}  // namespace

namespace dg {
MeshView mesh_view(const Ctx& c) {
  MeshView m;
  m.E = c.E;
  m.B = c.B;
  m.nbr = c.d_nbr;
  m.geo = c.d_geo;
  m.K = c.d_K;
  m.mortar_flux = c.d_mortar_flux;
  m.nrows = c.nrows;
  m.counters = c.d_counters;
  m.first_bad = c.d_first_bad;
  if (c.dim == 3) {  // 3-D meshes have no refined patch
    const int nz = c.desc.nel[2];
    const int sh = nz % 4 == 0 ? 2 : (nz % 2 == 0 ? 1 : -1);
    if (sh >= 0) {
      m.zf_shift = sh;
      m.zf_plane = c.desc.nel[0] * c.desc.nel[1];
      // x tiles of 16 columns where nx is 16 times a power of two of at
      // least 4 (64, 128, ... columns): the y-neighbour then stays within
      // 2^sh * 16 blocks.  Measured at 64^3, FP64, 4 z-planes per group: the
      // bytes fetched from beyond L2 fall from 2.4x to 1.4x of the
      // algorithmic bytes in stage 1 and from 1.5x to 1.2x in stages 2 and
      // 3; tiles of 8 columns fetch as much and run slower, and on 32
      // columns the plain groups fetch less than tiles of 16.
      constexpr int TXS = 4;
      const int nx = c.desc.nel[0], nh = nx >> TXS;
      if (nx % (1 << TXS) == 0 && nh >= 4 && (nh & (nh - 1)) == 0) {
        m.zf_txs = TXS;
        m.zf_nhs = __builtin_ctz((unsigned)nh);
        m.zf_nx = nx;
      }
    }
  }
  return m;
}
}  // namespace dg

namespace {

__global__ void k_reset_counters(int* cnt, unsigned long long* first_bad) {
  if (threadIdx.x < CNT_N) cnt[threadIdx.x] = 0;
  if (threadIdx.x == 0) *first_bad = ~0ull;
}

void free_ctx(Ctx& c) {
  void* ptrs[] = {c.d_nbr, c.d_geo, c.d_K, c.d_counters, c.d_first_bad, c.d_mortars,
                  c.d_mortar_flux, c.d_red, c.d_red_out, c.d_face, c.d_mech, c.d_vib, c.d_corner,
                  c.d_met, c.d_xyz, c.d_defer, c.d_defer_count};
  for (void* p : ptrs)
    if (p) (void)hipFree(p);
}

template <typename P>
hipError_t upload(P** dst, const void* src, size_t bytes) {
  hipError_t e = hipMalloc(reinterpret_cast<void**>(dst), bytes);
  if (e != hipSuccess) return e;
  if (src) return hipMemcpy(*dst, src, bytes, hipMemcpyHostToDevice);
  return hipSuccess;
}

}  // namespace

extern "C" {

const char* dg_strerror(int code) {
  switch (code) {
    case DG_OK: return "ok";
    case DG_ERR_ARG: return "invalid argument";
    case DG_ERR_UNSUPPORTED: return "unsupported configuration";
    case DG_ERR_HIP: return "HIP runtime error";
    case DG_ERR_OOM: return "out of device memory";
    case DG_ERR_NONPHYSICAL: return "non-physical state";
    case DG_ERR_NEWTON: return "implicit source substep did not converge";
  }
  return "unknown error";
}

const char* dg_last_error(void) { return g_last_error.c_str(); }

int dg_create(const dg_desc* desc, dg_ctx** out) {
  if (!desc || !out) return fail(DG_ERR_ARG, "dg_create: null argument");
  *out = nullptr;
  const dg_desc& d = *desc;
  if (d.dim != 2 && d.dim != 3) return fail(DG_ERR_UNSUPPORTED, "dim must be 2 or 3");
  if (d.degree < 1 || d.degree > MAXN1 - 1) return fail(DG_ERR_UNSUPPORTED, "degree must be in 1..7");
  if (d.batch < 1) return fail(DG_ERR_ARG, "batch must be >= 1");
  if (d.precision != DG_F64 && d.precision != DG_F32) return fail(DG_ERR_ARG, "precision must be DG_F64 or DG_F32");
  for (int l = 0; l < d.dim; ++l) {
    if (d.nel[l] < 1) return fail(DG_ERR_ARG, "nel must be >= 1");
    if (!(d.hi[l] > d.lo[l])) return fail(DG_ERR_ARG, "hi must exceed lo");
  }
  if (!(d.gamma > 1.0) && !is_reacting(d.physics)) return fail(DG_ERR_ARG, "gamma must exceed 1");
  {
    // one batch member's state is addressed with 32-bit byte offsets
    const long double n1 = d.degree + 1.0L;
    long double elems = 1.0L;
    for (int l = 0; l < d.dim; ++l) elems *= d.nel[l];
    if (d.dim == 2 && (d.patch_lo[0] != d.patch_hi[0] || d.patch_lo[1] != d.patch_hi[1]))
      elems += 3.0L * (d.patch_hi[0] - d.patch_lo[0]) * (d.patch_hi[1] - d.patch_lo[1]);
    const int nvars = is_reacting(d.physics) ? (d.mech ? d.mech->nspecies : 0) + d.dim + 1 + (d.physics == DG_REACTING_2T)
                                             : d.dim + 2;
    const long double bytes = elems * (d.dim == 3 ? n1 * n1 * n1 : n1 * n1) * nvars * (d.precision == DG_F32 ? 4 : 8);
    if (elems > 2147483647.0L || bytes >= 4294967296.0L)
      return fail(DG_ERR_UNSUPPORTED, "one batch member's state must stay below 4 GiB (32-bit addressing)");
  }
  const bool patch = d.dim == 2 && (d.patch_lo[0] != d.patch_hi[0] || d.patch_lo[1] != d.patch_hi[1]);
  if (patch) {
    for (int l = 0; l < 2; ++l)
      if (d.patch_lo[l] < 0 || d.patch_hi[l] > d.nel[l] || d.patch_lo[l] >= d.patch_hi[l])
        return fail(DG_ERR_ARG, "patch must be a non-empty block inside the grid");
    // a refined block that wraps the whole periodic direction has no coarse side
    for (int l = 0; l < 2; ++l)
      if (d.patch_hi[l] - d.patch_lo[l] >= d.nel[l]) return fail(DG_ERR_UNSUPPORTED, "patch must not span a full period");
  }
  switch (d.physics) {
    case DG_EULER: break;
    case DG_NAVIER_STOKES:
      if (d.dim != 3 || d.degree < 2 || d.degree > 4) return fail(DG_ERR_UNSUPPORTED, "Navier-Stokes: 3-D, degree 2..4");
      if (patch) return fail(DG_ERR_UNSUPPORTED, "Navier-Stokes on non-conforming meshes");
      if (!(d.mu >= 0.0) || !(d.prandtl > 0.0)) return fail(DG_ERR_ARG, "mu >= 0 and prandtl > 0 required");
      break;
    case DG_REACTING_EULER:
    case DG_REACTING_2T:
      if (d.dim != 2 || d.degree != 3) return fail(DG_ERR_UNSUPPORTED, "reacting Euler: 2-D, degree 3");
      if (!d.mech || d.mech->nspecies != 5 || d.mech->nreactions != 5)
        return fail(DG_ERR_UNSUPPORTED, "reacting Euler: mechanism with 5 species and 5 reactions");
      if (d.physics == DG_REACTING_2T) {
        if (!d.vib) return fail(DG_ERR_ARG, "two-temperature physics needs vibrational data (vib)");
        for (int q = 0; q < d.mech->nspecies; ++q)
          if (!(d.vib->theta_v[q] >= 0.0)) return fail(DG_ERR_ARG, "vib: theta_v must be >= 0");
        if (!(d.vib->park_sigma > 0.0)) return fail(DG_ERR_ARG, "vib: park_sigma must be > 0");
      }
      break;
    default: return fail(DG_ERR_ARG, "unknown physics");
  }
  bool curv = d.warp != 0.0;
  if (!std::isfinite(d.warp) || !(std::fabs(d.warp) < 0.25)) return fail(DG_ERR_ARG, "warp must be finite, |warp| < 0.25");
  for (int l = 0; l < d.dim; ++l) {
    const int a = d.bc[2 * l], b = d.bc[2 * l + 1];
    if (a < DG_BC_PERIODIC || a > DG_BC_OUTFLOW || b < DG_BC_PERIODIC || b > DG_BC_OUTFLOW)
      return fail(DG_ERR_ARG, "bc must hold dg_bc values");
    if ((a == DG_BC_PERIODIC) != (b == DG_BC_PERIODIC))
      return fail(DG_ERR_ARG, "bc: a direction is periodic on both sides or on neither");
    if (a != DG_BC_PERIODIC) curv = true;
  }
  if (curv) {
    bool periodic = true;
    for (int q = 0; q < 2 * d.dim; ++q) periodic = periodic && d.bc[q] == DG_BC_PERIODIC;
    if (d.physics == DG_NAVIER_STOKES) {
      if (!periodic)
        return fail(DG_ERR_UNSUPPORTED, "curvilinear Navier-Stokes: periodic sides only (no viscous boundary fluxes)");
    } else if (d.physics != DG_EULER) {
      return fail(DG_ERR_UNSUPPORTED, "curvilinear meshes and boundaries: Euler or Navier-Stokes physics only");
    }
    if (patch) return fail(DG_ERR_UNSUPPORTED, "curvilinear meshes and boundaries: no refined patch");
    bool inflow = false;
    for (int q = 0; q < 2 * d.dim; ++q) inflow = inflow || d.bc[q] == DG_BC_INFLOW;
    if (inflow) {
      double m2 = 0.0;
      for (int q = 0; q < d.dim; ++q) m2 += d.bc_state[1 + q] * d.bc_state[1 + q];
      const double p = (d.gamma - 1.0) * (d.bc_state[d.dim + 1] - 0.5 * m2 / d.bc_state[0]);
      if (!(d.bc_state[0] > 0.0) || !(p > 0.0)) return fail(DG_ERR_ARG, "bc_state must have rho > 0 and p > 0");
    }
  }
  if (!(d.rho_floor >= 0.0) || !(d.p_floor >= 0.0) || !std::isfinite(d.rho_floor) || !std::isfinite(d.p_floor))
    return fail(DG_ERR_ARG, "rho_floor and p_floor must be finite and >= 0");
  if ((d.rho_floor > 0.0 || d.p_floor > 0.0) && is_reacting(d.physics))
    return fail(DG_ERR_UNSUPPORTED, "positivity floor: Euler and Navier-Stokes physics only");
  if (d.volume != DG_VOLUME_STANDARD && d.volume != DG_VOLUME_SPLIT)
    return fail(DG_ERR_ARG, "volume must be DG_VOLUME_STANDARD or DG_VOLUME_SPLIT");
  if (d.volume == DG_VOLUME_SPLIT && d.physics != DG_EULER && d.physics != DG_NAVIER_STOKES)
    return fail(DG_ERR_UNSUPPORTED, "split-form volume integral: Euler and Navier-Stokes physics only");
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || ndev < 1) return fail(DG_ERR_HIP, "no HIP device");
  if (d.device < 0 || d.device >= ndev) return fail(DG_ERR_ARG, "device ordinal out of range");

  dg_ctx* ctx = new (std::nothrow) dg_ctx;
  if (!ctx) return fail(DG_ERR_OOM, "host allocation");
  Ctx& c = ctx->c;
  c.desc = d;
  c.desc.mech = nullptr;
  std::memset(&c.mech, 0, sizeof(c.mech));
  std::memset(&c.vib, 0, sizeof(c.vib));
  if (is_reacting(d.physics)) c.mech = *d.mech;
  if (d.physics == DG_REACTING_2T) c.vib = *d.vib;
  c.desc.vib = nullptr;
  if (c.desc.newton_max_iter <= 0) c.desc.newton_max_iter = 25;
  if (!(c.desc.newton_tol > 0.0)) c.desc.newton_tol = 1e-13;
  c.dim = d.dim;
  c.N = d.degree;
  c.n = d.degree + 1;
  c.Np = c.dim == 2 ? c.n * c.n : c.n * c.n * c.n;
  c.nv = is_reacting(d.physics) ? c.mech.nspecies + c.dim + 1 + (d.physics == DG_REACTING_2T) : c.dim + 2;
  c.B = d.batch;
  c.device = d.device;
  std::memset(&c.pc, 0, sizeof(c.pc));
  c.pc.gamma = d.gamma;
  c.pc.mu = d.mu;
  c.pc.prandtl = d.prandtl;
  for (int s = 0; s < c.mech.nspecies; ++s) {
    c.pc.cv[s] = c.mech.cv[s];
    c.pc.h0[s] = c.mech.h0[s];
    c.pc.R[s] = c.mech.R[s];
  }

  MeshBuild mb;
  int rc = build_mesh(d, mb);
  if (rc != DG_OK) {
    delete ctx;
    return rc;
  }
  c.E = (int)(mb.corner.size() / 3);
  c.hmin = mb.hmin;
  c.nmortar = (int)mb.mortars.size();
  c.nrows = mb.nrows;
  c.h_corner = mb.corner;
  c.h_geo = mb.geo;
  build_refconsts(c.N, c.h_K);
  c.curv = curv;
  std::vector<double> met, xyz;
  if (curv && !build_curv(d, c, mb, met, xyz)) {
    delete ctx;
    return fail(DG_ERR_ARG, "warp folds the mesh (J <= 0 at some node)");
  }

  DeviceGuard guard(c.device);
  // device address of the allocation-free entry point's fixed scratch array
  // (looked up once per device, with the device current)
  hipError_t e = noalloc_scratch_init(c.device);
  if (e != hipSuccess) {
    delete ctx;
    return hip_fail(e, "dg_create scratch symbol");
  }
  const size_t red_cap = (size_t)std::max(c.B, 1) * 512 * 10 + 1024;
  if ((e = upload(&c.d_nbr, mb.nbr.data(), mb.nbr.size() * sizeof(int))) != hipSuccess ||
      (e = upload(&c.d_geo, mb.geo.data(), mb.geo.size() * sizeof(double))) != hipSuccess ||
      (e = upload(&c.d_corner, mb.corner.data(), mb.corner.size() * sizeof(double))) != hipSuccess ||
      (e = upload(&c.d_K, &c.h_K, sizeof(RefConsts))) != hipSuccess ||
      (e = upload(&c.d_counters, nullptr, CNT_N * sizeof(int))) != hipSuccess ||
      (e = upload(&c.d_first_bad, nullptr, sizeof(unsigned long long))) != hipSuccess ||
      (e = upload(&c.d_red, nullptr, red_cap * sizeof(double))) != hipSuccess ||
      (e = upload(&c.d_red_out, nullptr, 1024 * sizeof(double))) != hipSuccess) {
    free_ctx(c);
    delete ctx;
    return e == hipErrorOutOfMemory ? fail(DG_ERR_OOM, "device allocation") : hip_fail(e, "dg_create");
  }
  c.red_cap = red_cap;
  if (c.nmortar > 0) {
    const size_t rowbytes = (size_t)c.B * c.nrows * (c.dim == 2 ? c.n : c.n * c.n) * c.nv * sizeof(double);
    if ((e = upload(&c.d_mortars, mb.mortars.data(), mb.mortars.size() * sizeof(MortarRec))) != hipSuccess ||
        (e = upload(&c.d_mortar_flux, nullptr, rowbytes)) != hipSuccess) {
      free_ctx(c);
      delete ctx;
      return hip_fail(e, "dg_create mortars");
    }
  }
  if (is_reacting(d.physics)) {
    if ((e = upload(&c.d_mech, &c.mech, sizeof(dg_mechanism))) != hipSuccess ||
        (d.physics == DG_REACTING_2T && (e = upload(&c.d_vib, &c.vib, sizeof(dg_vibration))) != hipSuccess)) {
      free_ctx(c);
      delete ctx;
      return hip_fail(e, "dg_create mechanism");
    }
  }
  if (curv) {
    if ((e = upload(&c.d_met, met.data(), met.size() * sizeof(double))) != hipSuccess ||
        (e = upload(&c.d_xyz, xyz.data(), xyz.size() * sizeof(double))) != hipSuccess) {
      free_ctx(c);
      delete ctx;
      return hip_fail(e, "dg_create metrics");
    }
  }
  if (d.physics == DG_NAVIER_STOKES) {
    // BR1 face buffer: [B][E][2*dim][n^2][4] (momentum and energy rows of the
    // normal viscous flux) in the context precision
    const size_t bytes = (size_t)c.B * c.E * 2 * c.dim * c.n * c.n * 4 * (d.precision == DG_F32 ? 4 : 8);
    if ((e = upload(&c.d_face, nullptr, bytes)) != hipSuccess) {
      free_ctx(c);
      delete ctx;
      return e == hipErrorOutOfMemory ? fail(DG_ERR_OOM, "BR1 face buffer") : hip_fail(e, "dg_create face buffer");
    }
  }
  if (d.physics == DG_REACTING_EULER) {
    // one record per node for the nodes whose implicit substep takes the
    // continuation in h (a node index and its iteration count, 8 bytes)
    const size_t bytes = (size_t)c.B * c.E * c.Np * 8;
    if ((e = upload(&c.d_defer, nullptr, bytes)) != hipSuccess ||
        (e = upload(&c.d_defer_count, nullptr, sizeof(int))) != hipSuccess) {
      free_ctx(c);
      delete ctx;
      return e == hipErrorOutOfMemory ? fail(DG_ERR_OOM, "chemistry continuation list")
                                      : hip_fail(e, "dg_create continuation list");
    }
  }
  hipLaunchKernelGGL(k_reset_counters, dim3(1), dim3(64), 0, 0, c.d_counters, c.d_first_bad);
  if ((e = hipGetLastError()) != hipSuccess || (e = hipDeviceSynchronize()) != hipSuccess) {
    free_ctx(c);
    delete ctx;
    return hip_fail(e, "dg_create reset");
  }
  *out = ctx;
  return DG_OK;
}

int dg_destroy(dg_ctx* ctx) {
  if (!ctx) return DG_OK;
  DeviceGuard guard(ctx->c.device);
  (void)hipDeviceSynchronize();
  free_ctx(ctx->c);
  delete ctx;
  return DG_OK;
}

int dg_sizes(const dg_ctx* ctx, int64_t* nelem, int32_t* nodes_per_elem, int32_t* nvars) {
  if (!ctx) return fail(DG_ERR_ARG, "dg_sizes: null context");
  if (nelem) *nelem = ctx->c.E;
  if (nodes_per_elem) *nodes_per_elem = ctx->c.Np;
  if (nvars) *nvars = ctx->c.nv;
  return DG_OK;
}

int dg_node_coords(const dg_ctx* ctx, double* xyz, void* stream) {
  if (!ctx || !xyz) return fail(DG_ERR_ARG, "dg_node_coords: null argument");
  const Ctx& c = ctx->c;
  DeviceGuard guard(c.device);
  hipError_t e;
  if (c.curv)
    e = hipMemcpyAsync(xyz, c.d_xyz, (size_t)c.dim * c.E * c.Np * sizeof(double), hipMemcpyDeviceToDevice,
                       static_cast<hipStream_t>(stream));
  else
    e = launch_coords(c, c.d_corner, xyz, static_cast<hipStream_t>(stream));
  return e == hipSuccess ? DG_OK : hip_fail(e, "dg_node_coords");
}

static int run_stage(dg_ctx* ctx, const void* U0, const void* Uk, void* out, double a, double b, double cdt,
                     int mode, void* stream, const char* who, const void* V = nullptr, void* out2 = nullptr,
                     double a2 = 0.0, double b2 = 0.0, double c2 = 0.0) {
  Ctx& c = ctx->c;
  const size_t bytes = state_bytes(c);
  if (overlaps(Uk, out, bytes)) return fail(DG_ERR_ARG, std::string(who) + ": output aliases the evaluated state");
  DeviceGuard guard(c.device);
  hipStream_t s = static_cast<hipStream_t>(stream);
  StageParams sp;
  sp.U0 = U0;
  sp.Uk = Uk;
  sp.out = out;
  sp.a = a;
  sp.b = b;
  sp.c = cdt;
  sp.mode = mode;
  sp.V = V;
  sp.out2 = out2;
  sp.a2 = a2;
  sp.b2 = b2;
  sp.c2 = c2;
  if (mode != 0) {
    sp.rho_min = c.desc.rho_floor;
    sp.p_min = c.desc.p_floor;
  }
  hipError_t e;
  if (c.desc.physics == DG_NAVIER_STOKES) {
    e = launch_ns(c, sp, s);
  } else if (c.curv) {
    e = launch_curv(c, sp, s);
  } else {
    e = launch_mortar(c, Uk, s);
    if (e == hipSuccess) e = launch_stage(c, sp, s);
  }
  return e == hipSuccess ? DG_OK : hip_fail(e, who);
}

int dg_rhs(dg_ctx* ctx, const void* U, void* dUdt, void* stream) {
  if (!ctx || !U || !dUdt) return fail(DG_ERR_ARG, "dg_rhs: null argument");
  return run_stage(ctx, nullptr, U, dUdt, 0.0, 0.0, 1.0, 0, stream, "dg_rhs");
}

int dg_rk_stage(dg_ctx* ctx, const void* U0, const void* Uk, void* Uout, double a, double b, double c_dt,
                void* stream) {
  if (!ctx || !Uk || !Uout || (a != 0.0 && !U0)) return fail(DG_ERR_ARG, "dg_rk_stage: null argument");
  if (a != 0.0 && U0 != Uout && overlaps(U0, Uout, state_bytes(ctx->c)))
    return fail(DG_ERR_ARG, "dg_rk_stage: Uout partially overlaps U0");
  return run_stage(ctx, U0, Uk, Uout, a, b, c_dt, 1, stream, "dg_rk_stage");
}

int dg_rk_stage_dual(dg_ctx* ctx, const void* U0, const void* Uk, void* Uout, double a, double b, double c_dt,
                     const void* V, void* Wout, double a2, double b2, double c2_dt, void* stream) {
  if (!ctx || !Uk || !Uout || !Wout || (a != 0.0 && !U0) || (a2 != 0.0 && !V))
    return fail(DG_ERR_ARG, "dg_rk_stage_dual: null argument");
  const size_t bytes = state_bytes(ctx->c);
  if (a != 0.0 && U0 != Uout && overlaps(U0, Uout, bytes))
    return fail(DG_ERR_ARG, "dg_rk_stage_dual: Uout partially overlaps U0");
  if (a2 != 0.0 && V != Wout && overlaps(V, Wout, bytes))
    return fail(DG_ERR_ARG, "dg_rk_stage_dual: Wout partially overlaps V");
  if (overlaps(Uk, Wout, bytes)) return fail(DG_ERR_ARG, "dg_rk_stage_dual: Wout aliases the evaluated state");
  if (overlaps(Uout, Wout, bytes)) return fail(DG_ERR_ARG, "dg_rk_stage_dual: the two outputs overlap");
  // a stage output must not be read as the other combination's input either
  if (a2 != 0.0 && overlaps(V, Uout, bytes)) return fail(DG_ERR_ARG, "dg_rk_stage_dual: V aliases Uout");
  if (a != 0.0 && overlaps(U0, Wout, bytes)) return fail(DG_ERR_ARG, "dg_rk_stage_dual: U0 aliases Wout");
  return run_stage(ctx, U0, Uk, Uout, a, b, c_dt, 2, stream, "dg_rk_stage_dual", V, Wout, a2, b2, c2_dt);
}

// Shu-Osher coefficients of SSPRK(5,4) (Spiteri and Ruuth), nonzero entries:
// U^(i) = sum_k alpha_ik U^(k) + dt beta_ik L(U^(k)).
namespace {
constexpr double A20 = 0.444370493651235, A21 = 0.555629506348765;
constexpr double A30 = 0.620101851488403, A32 = 0.379898148511597;
constexpr double A40 = 0.178079954393132, A43 = 0.821920045606868;
constexpr double A52 = 0.517231671970585, A53 = 0.096059710526147, A54 = 0.386708617503269;
constexpr double B10 = 0.391752226571890, B21 = 0.368410593050371, B32 = 0.251891774271694;
constexpr double B43 = 0.544974750228521, B53 = 0.063692468666290, B54 = 0.226007483236906;
}  // namespace

int dg_ssprk54_step(dg_ctx* ctx, void* U, double dt, void* t1, void* t2, void* t3, void* stream) {
  if (!ctx || !U || !t1 || !t2 || !t3) return fail(DG_ERR_ARG, "dg_ssprk54_step: null argument");
  const size_t bytes = state_bytes(ctx->c);
  const void* bufs[4] = {U, t1, t2, t3};
  for (int i = 0; i < 4; ++i)
    for (int j = i + 1; j < 4; ++j)
      if (overlaps(bufs[i], bufs[j], bytes)) return fail(DG_ERR_ARG, "dg_ssprk54_step: U, t1, t2, t3 must not overlap");
  int rc;
  // U^(1) = U + dt b10 L(U)                                   -> t1
  if ((rc = run_stage(ctx, nullptr, U, t1, 0.0, 1.0, B10 * dt, 1, stream, "dg_ssprk54_step")) != DG_OK) return rc;
  // U^(2) = a20 U + a21 U^(1) + dt b21 L(U^(1))                -> t2
  if ((rc = run_stage(ctx, U, t1, t2, A20, A21, B21 * dt, 1, stream, "dg_ssprk54_step")) != DG_OK) return rc;
  // U^(3) = a30 U + a32 U^(2) + dt b32 L(U^(2))                -> t1
  if ((rc = run_stage(ctx, U, t2, t1, A30, A32, B32 * dt, 1, stream, "dg_ssprk54_step")) != DG_OK) return rc;
  // U^(4) = a40 U + a43 U^(3) + dt b43 L(U^(3))                -> t3
  // W     = a52 U^(2) + a53 U^(3) + dt b53 L(U^(3))            -> t2 (in place)
  if ((rc = run_stage(ctx, U, t1, t3, A40, A43, B43 * dt, 2, stream, "dg_ssprk54_step", t2, t2, A52, A53,
                      B53 * dt)) != DG_OK)
    return rc;
  // U^(5) = W + a54 U^(4) + dt b54 L(U^(4))                    -> U
  return run_stage(ctx, t2, t3, U, 1.0, A54, B54 * dt, 1, stream, "dg_ssprk54_step");
}

int dg_source_chem(dg_ctx* ctx, const void* U, void* out, double h, int32_t mode, void* stream) {
  if (!ctx || !U || !out) return fail(DG_ERR_ARG, "dg_source_chem: null argument");
  Ctx& c = ctx->c;
  if (!is_reacting(c.desc.physics)) return fail(DG_ERR_UNSUPPORTED, "dg_source_chem: reacting Euler only");
  if (mode != 0 && mode != 1) return fail(DG_ERR_ARG, "dg_source_chem: mode must be 0 or 1");
  if (out != U && overlaps(U, out, state_bytes(c))) return fail(DG_ERR_ARG, "dg_source_chem: partial overlap");
  DeviceGuard guard(c.device);
  hipError_t e = launch_source(c, U, out, h, mode, static_cast<hipStream_t>(stream));
  return e == hipSuccess ? DG_OK : hip_fail(e, "dg_source_chem");
}

int dg_rhs_adjoint(dg_ctx* ctx, const void* U, const void* lam_L, void* lam_U, void* stream) {
  if (!ctx || !U || !lam_L || !lam_U) return fail(DG_ERR_ARG, "dg_rhs_adjoint: null argument");
  Ctx& c = ctx->c;
  if (c.desc.physics != DG_EULER || c.nmortar > 0 || c.N > 4)
    return fail(DG_ERR_UNSUPPORTED, "adjoint: Euler physics on conforming meshes, degree <= 4");
  if (c.desc.volume != DG_VOLUME_STANDARD)
    return fail(DG_ERR_UNSUPPORTED, "adjoint: standard volume integral only");
  if (c.curv) return fail(DG_ERR_UNSUPPORTED, "adjoint: Cartesian periodic meshes only");
  const size_t bytes = state_bytes(c);
  if (overlaps(lam_U, U, bytes) || overlaps(lam_U, lam_L, bytes))
    return fail(DG_ERR_ARG, "dg_rhs_adjoint: lam_U aliases an input");
  DeviceGuard guard(c.device);
  hipError_t e = launch_adjoint(c, U, lam_L, lam_U, nullptr, 0.0, 0.0, 1.0, 0, static_cast<hipStream_t>(stream));
  return e == hipSuccess ? DG_OK : hip_fail(e, "dg_rhs_adjoint");
}

int dg_rk_stage_adjoint(dg_ctx* ctx, const void* Uk, const void* lam_out, void* lam_k, void* lam_0, double a,
                        double b, double c_dt, int32_t lam0_mode, void* stream) {
  if (!ctx || !Uk || !lam_out || !lam_k) return fail(DG_ERR_ARG, "dg_rk_stage_adjoint: null argument");
  Ctx& c = ctx->c;
  if (c.desc.physics != DG_EULER || c.nmortar > 0 || c.N > 4)
    return fail(DG_ERR_UNSUPPORTED, "adjoint: Euler physics on conforming meshes, degree <= 4");
  if (c.desc.volume != DG_VOLUME_STANDARD)
    return fail(DG_ERR_UNSUPPORTED, "adjoint: standard volume integral only");
  if (c.curv) return fail(DG_ERR_UNSUPPORTED, "adjoint: Cartesian periodic meshes only");
  if (lam0_mode != DG_LAM0_ACCUMULATE && lam0_mode != DG_LAM0_FOLD && lam0_mode != DG_LAM0_INIT)
    return fail(DG_ERR_ARG, "dg_rk_stage_adjoint: unknown lam0_mode");
  const size_t bytes = state_bytes(c);
  if (overlaps(lam_k, Uk, bytes) || overlaps(lam_k, lam_out, bytes) || overlaps(lam_k, lam_0, bytes))
    return fail(DG_ERR_ARG, "dg_rk_stage_adjoint: lam_k aliases an input");
  if (lam_0 && (overlaps(lam_0, lam_out, bytes) || overlaps(lam_0, Uk, bytes)))
    return fail(DG_ERR_ARG, "dg_rk_stage_adjoint: lam_0 aliases another buffer");
  DeviceGuard guard(c.device);
  hipError_t e = launch_adjoint(c, Uk, lam_out, lam_k, lam_0, a, b, c_dt, lam0_mode, static_cast<hipStream_t>(stream));
  return e == hipSuccess ? DG_OK : hip_fail(e, "dg_rk_stage_adjoint");
}

int dg_dt_cfl(dg_ctx* ctx, const void* U, double cfl, double* dt, void* stream) {
  if (!ctx || !U || !dt) return fail(DG_ERR_ARG, "dg_dt_cfl: null argument");
  if (!(cfl > 0.0)) return fail(DG_ERR_ARG, "dg_dt_cfl: cfl must be positive");
  Ctx& c = ctx->c;
  DeviceGuard guard(c.device);
  hipStream_t s = static_cast<hipStream_t>(stream);
  hipError_t e = launch_lam_max(c, U, c.d_red_out, s);
  double h[2] = {0.0, 0.0};
  if (e == hipSuccess) e = hipMemcpyAsync(h, c.d_red_out, 2 * sizeof(double), hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) return hip_fail(e, "dg_dt_cfl");
  const int p = 2 * c.N + 1;
  double d = cfl * c.hmin / (p * h[0]);
  if (c.desc.physics == DG_NAVIER_STOKES && c.desc.mu > 0.0) {
    const double nu = c.desc.mu * h[1] * std::max(1.0, 1.0 / c.desc.prandtl);
    d = std::min(d, cfl * c.hmin * c.hmin / ((double)p * p * nu));
  }
  *dt = d;
  return DG_OK;
}

int dg_integrals(dg_ctx* ctx, const void* U, double* out, void* stream) {
  if (!ctx || !U || !out) return fail(DG_ERR_ARG, "dg_integrals: null argument");
  Ctx& c = ctx->c;
  if (c.nv + 1 > 10) return fail(DG_ERR_UNSUPPORTED, "dg_integrals: too many variables");
  DeviceGuard guard(c.device);
  hipStream_t s = static_cast<hipStream_t>(stream);
  hipError_t e = launch_integrals(c, U, c.d_red_out, s);
  if (e == hipSuccess)
    e = hipMemcpyAsync(out, c.d_red_out, (size_t)c.B * (c.nv + 1) * sizeof(double), hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  return e == hipSuccess ? DG_OK : hip_fail(e, "dg_integrals");
}

int dg_integrals_noalloc(dg_ctx* ctx, const void* U, double* out, void* stream) {
  if (!ctx || !U || !out) return fail(DG_ERR_ARG, "dg_integrals_noalloc: null argument");
  Ctx& c = ctx->c;
  if (c.nv + 1 > 10) return fail(DG_ERR_UNSUPPORTED, "dg_integrals_noalloc: too many variables");
  if (noalloc_integrals_need(c) > NOALLOC_SCRATCH_DOUBLES)
    return fail(DG_ERR_UNSUPPORTED, "dg_integrals_noalloc: batch * (nvars + 1) = " +
                                        std::to_string(c.B * (c.nv + 1)) + " exceeds the fixed scratch limit of " +
                                        std::to_string(NOALLOC_SCRATCH_DOUBLES / 512));
  DeviceGuard guard(c.device);
  const hipError_t e = launch_integrals_noalloc(c, U, out, static_cast<hipStream_t>(stream));
  return e == hipSuccess ? DG_OK : hip_fail(e, "dg_integrals_noalloc");
}

int dg_status_read(dg_ctx* ctx, dg_counters* out, int32_t reset, void* stream) {
  if (!ctx || !out) return fail(DG_ERR_ARG, "dg_status_read: null argument");
  Ctx& c = ctx->c;
  DeviceGuard guard(c.device);
  hipStream_t s = static_cast<hipStream_t>(stream);
  int cnt[CNT_N];
  unsigned long long fb = 0;
  hipError_t e = hipMemcpyAsync(cnt, c.d_counters, sizeof(cnt), hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipMemcpyAsync(&fb, c.d_first_bad, sizeof(fb), hipMemcpyDeviceToHost, s);
  if (e == hipSuccess && reset) {
    hipLaunchKernelGGL(k_reset_counters, dim3(1), dim3(64), 0, s, c.d_counters, c.d_first_bad);
    e = hipGetLastError();
  }
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) return hip_fail(e, "dg_status_read");
  out->nonphysical = cnt[CNT_NONPHYSICAL];
  out->newton_unconverged = cnt[CNT_NEWTON];
  out->species_clips = cnt[CNT_CLIPS];
  out->newton_iters_max = cnt[CNT_ITERS];
  out->first_bad = fb == ~0ull ? -1 : (int64_t)fb;
  out->floored = cnt[CNT_FLOORED];
  return DG_OK;
}

}  // extern "C"
