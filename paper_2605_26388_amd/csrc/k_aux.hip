// Auxiliary kernels: node coordinates, FP64 integrals (conservation sums and
// kinetic energy) and the wave-speed maxima for the CFL bounds.
//
// Reductions are deterministic: every block writes its partial in a fixed
// order (wave shuffles, then LDS across waves), and a second single-block pass
// adds the partials in index order.  No atomics.
#include <mutex>

#include "dg_device.hpp"

namespace dg {

constexpr int RED_BS = 256;
constexpr int RED_BLOCKS = 512;   // partial blocks per batch member
constexpr int RED_MAXQ = 10;      // quantities per reduction (nv + 1 <= 10)

__global__ void k_coords(int dim, int n, int E, const double* corner, const double* geo,
                         const RefConsts* K, double* xyz) {
  const int Np = dim == 2 ? n * n : n * n * n;
  const size_t total = (size_t)E * Np;
  for (size_t t = blockIdx.x * (size_t)blockDim.x + threadIdx.x; t < total;
       t += (size_t)gridDim.x * blockDim.x) {
    const int e = (int)(t / Np);
    const int node = (int)(t - (size_t)e * Np);
    const int ii[3] = {node % n, (node / n) % n, node / (n * n)};
    for (int d = 0; d < dim; ++d)
      xyz[(size_t)d * total + t] = corner[(size_t)e * 3 + d] + (K->xi[ii[d]] + 1.0) / geo[(size_t)e * 4 + d];
  }
}

hipError_t launch_coords(const Ctx& c, const double* corner, double* xyz, hipStream_t s) {
  const size_t total = (size_t)c.E * c.Np;
  const int blocks = (int)((total + 255) / 256 < 65536 ? (total + 255) / 256 : 65536);
  hipLaunchKernelGGL(k_coords, dim3(blocks), dim3(256), 0, s, c.dim, c.n, c.E, corner, c.d_geo, c.d_K, xyz);
  return hipGetLastError();
}

// block-wide sum of NQ doubles (fixed order); result valid in thread 0
template <int NQ>
__device__ void block_sum(double (&x)[NQ], double (*sh)[NQ]) {
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
#pragma unroll
  for (int q = 0; q < NQ; ++q)
    for (int o = 32; o > 0; o >>= 1) x[q] += __shfl_down(x[q], o, 64);
  if (lane == 0)
#pragma unroll
    for (int q = 0; q < NQ; ++q) sh[wid][q] = x[q];
  __syncthreads();
  if (threadIdx.x == 0) {
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
      double s = 0.0;
      for (int w = 0; w < RED_BS / 64; ++w) s += sh[w][q];
      x[q] = s;
    }
  }
}

// Partial sums of J_e w_i U_v,i (v < nv) and of J_e w_i |m|^2/(2 rho).
// Grid (RED_BLOCKS, B); block j covers a contiguous node range.
template <typename T>
__global__ void __launch_bounds__(RED_BS)
k_integrals(const T* U, int dim, int n, int E, int nv, int nspec, const double* geo, const double* jnode,
            const RefConsts* K, double* partial) {
  __shared__ double sh[RED_BS / 64][RED_MAXQ];
  const int b = blockIdx.y;
  const int Np = dim == 2 ? n * n : n * n * n;
  const size_t total = (size_t)E * Np;
  const size_t plane = total;
  const T* Ub = U + (size_t)b * nv * plane;
  const size_t chunk = (total + gridDim.x - 1) / gridDim.x;
  const size_t t0 = blockIdx.x * chunk;
  const size_t t1 = t0 + chunk < total ? t0 + chunk : total;
  double x[RED_MAXQ];
  for (int q = 0; q < RED_MAXQ; ++q) x[q] = 0.0;
  for (size_t t = t0 + threadIdx.x; t < t1; t += RED_BS) {
    const int e = (int)(t / Np);
    const int node = (int)(t - (size_t)e * Np);
    // Jacobian per element (affine) or per node (curvilinear)
    double wt = (jnode ? jnode[t] : geo[(size_t)e * 4 + 3]) * K->w[node % n] * K->w[(node / n) % n];
    if (dim == 3) wt *= K->w[node / (n * n)];
    double rho = 0.0, m2 = 0.0;
    for (int v = 0; v < nv; ++v) {
      const double val = static_cast<double>(Ub[(size_t)v * plane + t]);
      x[v] += wt * val;
      if (v < nspec) rho += val;
      else if (v < nspec + dim) m2 += val * val;
    }
    x[nv] += wt * 0.5 * m2 / rho;
  }
  block_sum<RED_MAXQ>(x, sh);
  if (threadIdx.x == 0)
    for (int q = 0; q <= nv; ++q) partial[((size_t)b * gridDim.x + blockIdx.x) * (nv + 1) + q] = x[q];
}

__global__ void __launch_bounds__(RED_BS)
k_final_sum(const double* partial, int nparts, int nq, double* out) {
  __shared__ double sh[RED_BS / 64][RED_MAXQ];
  const int b = blockIdx.x;
  double x[RED_MAXQ];
  for (int q = 0; q < RED_MAXQ; ++q) x[q] = 0.0;
  for (int j = threadIdx.x; j < nparts; j += RED_BS)
    for (int q = 0; q < nq; ++q) x[q] += partial[((size_t)b * nparts + j) * nq + q];
  block_sum<RED_MAXQ>(x, sh);
  if (threadIdx.x == 0)
    for (int q = 0; q < nq; ++q) out[(size_t)b * nq + q] = x[q];
}

// Both passes of the integrals with the partials in `partial` (B x
// RED_BLOCKS x (nv + 1) doubles, every one written before it is read).
static hipError_t integrals_into(const Ctx& c, const void* U, double* partial, double* d_out, hipStream_t s) {
  const int nspec = is_reacting(c.desc.physics) ? c.mech.nspecies : 1;
  dim3 grid(RED_BLOCKS, c.B);
  if (c.desc.precision == DG_F32)
    hipLaunchKernelGGL((k_integrals<float>), grid, dim3(RED_BS), 0, s, static_cast<const float*>(U), c.dim, c.n,
                       c.E, c.nv, nspec, c.d_geo, c.curv ? c.d_met : nullptr, c.d_K, partial);
  else
    hipLaunchKernelGGL((k_integrals<double>), grid, dim3(RED_BS), 0, s, static_cast<const double*>(U), c.dim, c.n,
                       c.E, c.nv, nspec, c.d_geo, c.curv ? c.d_met : nullptr, c.d_K, partial);
  hipError_t err = hipGetLastError();
  if (err != hipSuccess) return err;
  hipLaunchKernelGGL(k_final_sum, dim3(c.B), dim3(RED_BS), 0, s, partial, RED_BLOCKS, c.nv + 1, d_out);
  return hipGetLastError();
}

hipError_t launch_integrals(const Ctx& c, const void* U, double* d_out, hipStream_t s) {
  return integrals_into(c, U, c.d_red, d_out, s);
}

// ---------------------------------------------------------------------------
// Allocation-free integrals.  The partials live in one fixed device array per
// GPU (file scope, zero-initialised at load, held until the process ends)
// instead of the context's scratch.  In host code `scratch` only names the
// symbol; its device address is looked up once per device, with that device
// current, and only that address is ever handed to a kernel.  Every call on a
// GPU shares the array: calls that overlap on one GPU (two streams, two
// threads) race.  Nothing in it needs clearing: the first pass writes every
// partial the second pass reads.
// ---------------------------------------------------------------------------
static __device__ __align__(256) double scratch[NOALLOC_SCRATCH_DOUBLES];

namespace {
constexpr int NOALLOC_MAX_DEVICES = 64;
std::mutex g_scratch_mu;
double* g_scratch_ptr[NOALLOC_MAX_DEVICES] = {};
}  // namespace

hipError_t noalloc_scratch_init(int device) {
  if (device < 0 || device >= NOALLOC_MAX_DEVICES) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (g_scratch_ptr[device]) return hipSuccess;
  void* p = nullptr;
  const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
  if (e != hipSuccess) return e;
  g_scratch_ptr[device] = static_cast<double*>(p);
  return hipSuccess;
}

size_t noalloc_integrals_need(const Ctx& c) { return (size_t)c.B * RED_BLOCKS * (size_t)(c.nv + 1); }

hipError_t launch_integrals_noalloc(const Ctx& c, const void* U, double* d_out, hipStream_t s) {
  double* p = nullptr;
  {
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (c.device >= 0 && c.device < NOALLOC_MAX_DEVICES) p = g_scratch_ptr[c.device];
  }
  if (!p) return hipErrorNotInitialized;
  return integrals_into(c, U, p, d_out, s);
}

// Maxima of |u| + a and of 1/rho over all nodes and batch members.
template <typename T, class PHYS>
__global__ void __launch_bounds__(RED_BS)
k_lam_max(const T* U, int E, int Np, int B, PhysConst pc, double* partial) {
  constexpr int NV = PHYS::NV;
  __shared__ double sh[RED_BS / 64][2];
  const size_t plane = (size_t)E * Np;
  const size_t total = plane * B;
  double lam = 0.0, rinv = 0.0;
  for (size_t t = blockIdx.x * (size_t)RED_BS + threadIdx.x; t < total; t += (size_t)gridDim.x * RED_BS) {
    const size_t b = t / plane;
    const size_t r = t - b * plane;
    double u[NV];
    for (int v = 0; v < NV; ++v) u[v] = static_cast<double>(U[(b * NV + v) * plane + r]);
    Thermo th;
    PHYS::thermo(u, th, pc);
    double u2 = 0.0;
    for (int d = 0; d < PHYS::NDIM; ++d) {
      const double vd = u[PHYS::MOM + d] * th.ri;
      u2 += vd * vd;
    }
    const double c = sqrt(u2) + sqrt(th.k * th.p * th.ri);
    lam = c > lam ? c : lam;
    rinv = th.ri > rinv ? th.ri : rinv;
  }
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  for (int o = 32; o > 0; o >>= 1) {
    const double a = __shfl_down(lam, o, 64), r2 = __shfl_down(rinv, o, 64);
    lam = a > lam ? a : lam;
    rinv = r2 > rinv ? r2 : rinv;
  }
  if (lane == 0) {
    sh[wid][0] = lam;
    sh[wid][1] = rinv;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int w = 1; w < RED_BS / 64; ++w) {
      lam = sh[w][0] > lam ? sh[w][0] : lam;
      rinv = sh[w][1] > rinv ? sh[w][1] : rinv;
    }
    partial[blockIdx.x * 2 + 0] = lam;
    partial[blockIdx.x * 2 + 1] = rinv;
  }
}

__global__ void __launch_bounds__(RED_BS) k_final_max(const double* partial, int nparts, double* out) {
  __shared__ double sh[RED_BS / 64][2];
  double a = 0.0, r = 0.0;
  for (int j = threadIdx.x; j < nparts; j += RED_BS) {
    a = partial[2 * j] > a ? partial[2 * j] : a;
    r = partial[2 * j + 1] > r ? partial[2 * j + 1] : r;
  }
  for (int o = 32; o > 0; o >>= 1) {
    const double x = __shfl_down(a, o, 64), y = __shfl_down(r, o, 64);
    a = x > a ? x : a;
    r = y > r ? y : r;
  }
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  if (lane == 0) {
    sh[wid][0] = a;
    sh[wid][1] = r;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int w = 1; w < RED_BS / 64; ++w) {
      a = sh[w][0] > a ? sh[w][0] : a;
      r = sh[w][1] > r ? sh[w][1] : r;
    }
    out[0] = a;
    out[1] = r;
  }
}

template <typename T>
static hipError_t lam_t(const Ctx& c, const void* U, double* d_out, hipStream_t s) {
  const T* Ut = static_cast<const T*>(U);
  const int nb = RED_BLOCKS;
  if (c.desc.physics == DG_REACTING_EULER)
    hipLaunchKernelGGL((k_lam_max<T, ReactPhys<2, 5>>), dim3(nb), dim3(RED_BS), 0, s, Ut, c.E, c.Np, c.B, c.pc, c.d_red);
  else if (c.desc.physics == DG_REACTING_2T)
    hipLaunchKernelGGL((k_lam_max<T, ReactPhys<2, 5, true>>), dim3(nb), dim3(RED_BS), 0, s, Ut, c.E, c.Np, c.B, c.pc,
                       c.d_red);
  else if (c.dim == 2)
    hipLaunchKernelGGL((k_lam_max<T, EulerPhys<2>>), dim3(nb), dim3(RED_BS), 0, s, Ut, c.E, c.Np, c.B, c.pc, c.d_red);
  else
    hipLaunchKernelGGL((k_lam_max<T, EulerPhys<3>>), dim3(nb), dim3(RED_BS), 0, s, Ut, c.E, c.Np, c.B, c.pc, c.d_red);
  hipError_t err = hipGetLastError();
  if (err != hipSuccess) return err;
  hipLaunchKernelGGL(k_final_max, dim3(1), dim3(RED_BS), 0, s, c.d_red, nb, d_out);
  return hipGetLastError();
}

hipError_t launch_lam_max(const Ctx& c, const void* U, double* d_out, hipStream_t s) {
  return c.desc.precision == DG_F32 ? lam_t<float>(c, U, d_out, s) : lam_t<double>(c, U, d_out, s);
}

}  // namespace dg
