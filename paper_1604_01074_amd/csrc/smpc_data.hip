// Float64 kernels outside the APG iteration, for gfx950:
//
//   k_cost_uhat_e, k_cost_beta   the cost update of App. A for new demands and
//                                pumping costs (Alg. 2, step 2), per node
//   k_root_beta                  the root's linear term for a new previous
//                                input q
//   k_obj_primal, k_obj_dual,    the primal objective f(z) + g(t), the dual
//   k_obj_reduce                 objective D(y) = f*(-H'y) + g*(y) of
//                                eq. optim:prob and the duality gap of
//                                Sec. IV-E, reduced in a fixed order
//   k_scale_dual, k_narrow       element-wise helpers
//
// The objective kernels take their partial sums from a caller-provided
// buffer: a per-tree allocation (smpc_tree_objective) or the file-scope
// `scratch` array (smpc_tree_objective_noalloc).
//
// One workgroup of 128 threads per node (grid-stride): thread j handles input
// component j and state component j (nx, nu <= 128).  Node arrays are in the
// library's internal (chain-major) order.
#include <mutex>

#include "smpc_internal.h"

namespace smpc {

namespace {

constexpr int kDB = 128;  // threads per workgroup (two wave64)

// Sum over the 64 lanes of a wave, every lane receives it.
__device__ __forceinline__ double wsum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

__device__ __forceinline__ double wmax(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_xor(v, off, 64));
  return v;
}

// Sum of K values over the workgroup (wave 0 + wave 1, in that order); every
// thread receives the K sums.  `red` holds 2 K doubles of LDS.
template <int K>
__device__ __forceinline__ void block_sum(double (&v)[K], double* red) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int k = 0; k < K; ++k) v[k] = wsum(v[k]);
  __syncthreads();
  if (lane == 0)
#pragma unroll
    for (int k = 0; k < K; ++k) red[wave * K + k] = v[k];
  __syncthreads();
#pragma unroll
  for (int k = 0; k < K; ++k) v[k] = red[k] + red[K + k];
}

__device__ __forceinline__ double block_max(double v, double* red) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  v = wmax(v);
  __syncthreads();
  if (lane == 0) red[wave] = v;
  __syncthreads();
  return fmax(red[0], red[1]);
}

// ---------------------------------------------------------------------------
// App. A: uhat_n = Mu d_n (the minimum-norm solution of E u + Ed d_n = 0) and
// e_n = B uhat_n + Gd d_n.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kDB) void k_cost_uhat_e(CostSysDev s, CostTreeDev t) {
  extern __shared__ double sm[];
  double* sd = sm;          // nd
  double* su = sm + s.nd;   // nu
  const int tid = threadIdx.x;
  const int nx = s.nx, nu = s.nu, nd = s.nd;
  for (int n = blockIdx.x; n < t.M; n += gridDim.x) {
    for (int k = tid; k < nd; k += kDB) sd[k] = t.d[(size_t)t.perm[n] * nd + k];
    __syncthreads();
    if (tid < nu) {
      double acc = 0.0;
      for (int k = 0; k < nd; ++k) acc += s.Mu[(size_t)tid * nd + k] * sd[k];
      su[tid] = acc;
      t.uhat[(size_t)n * nu + tid] = acc;
      if (t.uhat32) t.uhat32[(size_t)n * nu + tid] = (float)acc;
    }
    __syncthreads();
    if (tid < nx) {
      double acc = 0.0;
      for (int q = s.b_rp[tid]; q < s.b_rp[tid + 1]; ++q) acc += s.b_v[q] * su[s.b_ci[q]];
      for (int k = 0; k < nd; ++k) acc += s.Gd[(size_t)tid * nd + k] * sd[k];
      t.e[(size_t)n * nx + tid] = acc;
      if (t.e32) t.e32[(size_t)n * nx + tid] = (float)acc;
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// App. A, the linear term of v_n after the smoothing cost is expanded and
// regrouped per node, here in input space (its v-space form is L' beta_n):
//   beta_n = pi_n W_alpha (alpha1 + alpha2_{s(n)})
//            + 2 Wu (pibar_n uhat_n - pi_n uhat_{a(n)} - sum_c pi_c uhat_c),
//   pibar_n = pi_n + sum_c pi_c.
// For the root the term of the previous input q is left out
// (beta_root0); k_root_beta adds it for each solve.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kDB) void k_cost_beta(CostSysDev s, CostTreeDev t) {
  extern __shared__ double sm[];
  double* smix = sm;  // nu
  const int tid = threadIdx.x;
  const int nu = s.nu;
  for (int n = blockIdx.x; n < t.M; n += gridDim.x) {
    const int c0 = t.child_rp[n], c1 = t.child_rp[n + 1];
    const int a = t.parent[n];
    const double pin = t.pi[n];
    if (tid < nu) {
      double pib = pin;
      for (int k = c0; k < c1; ++k) pib += t.pi[t.child_ci[k]];
      double m = pib * t.uhat[(size_t)n * nu + tid];
      if (a >= 0) m -= pin * t.uhat[(size_t)a * nu + tid];
      for (int k = c0; k < c1; ++k) {
        const int c = t.child_ci[k];
        m -= t.pi[c] * t.uhat[(size_t)c * nu + tid];
      }
      smix[tid] = m;
    }
    __syncthreads();
    if (tid < nu) {
      double acc = 0.0;
      for (int k = 0; k < nu; ++k) acc += s.Wu[(size_t)tid * nu + k] * smix[k];
      const double lin = s.W_alpha * (s.alpha1[tid] + t.alpha2[(size_t)t.stage[n] * nu + tid]);
      const double b = pin * lin + 2.0 * acc;
      t.beta[(size_t)n * nu + tid] = b;
      if (t.beta32) t.beta32[(size_t)n * nu + tid] = (float)b;
      if (n == t.root) t.beta_root0[tid] = b;
    }
    __syncthreads();
  }
}

// beta_root = beta_root0 - 2 pi_root Wu q (the smoothing cost of the first
// input against the input applied before the horizon).
__global__ __launch_bounds__(kDB) void k_root_beta(CostSysDev s, CostTreeDev t) {
  const int tid = threadIdx.x;
  const int nu = s.nu;
  if (tid >= nu) return;
  double acc = 0.0;
  for (int k = 0; k < nu; ++k) acc += s.Wu[(size_t)tid * nu + k] * t.q[k];
  const double b = t.beta_root0[tid] - 2.0 * t.pi[t.root] * acc;
  t.beta[(size_t)t.root * nu + tid] = b;
  if (t.beta32) t.beta32[(size_t)t.root * nu + tid] = (float)b;
}

// ---------------------------------------------------------------------------
// Objectives (Sec. IV-A, IV-E).  Per node n, with u_{a(root)} = q:
//   stage_n = pi_n [W_alpha (alpha1 + alpha2_{s(n)})' u_n + du' Wu du],
//             du = u_n - u_{a(n)}                    (the smooth part of f)
//   soft(v) = cS_n dist(v_sigma | x >= xs) + cd dist(v_zeta | [xmin, xmax])
// Primal pass at (z^nu, t^nu): stage(u), soft(t), soft(x); t is recovered
// from the dual update y^{nu+1} = w + lambda S (Hz - t) with
// w = y^nu + c (y^nu - y^{nu-1}), all scaled by S per (node, block).
// Dual pass at z = z(y) for the unscaled y = S y^{nu+1}: stage(u), <y, Hz>,
// the support function of the sets of g,
//   sum xs' y_sigma + sum max(xmax y_zeta, xmin y_zeta)
//   + sum max(umax y_psi, umin y_psi),
// and the violation of dom g* (y_sigma <= 0, ||y_sigma|| <= cS_n,
// ||y_zeta|| <= cd).
// ---------------------------------------------------------------------------
__device__ __forceinline__ double stage_term(const CostSysDev& s, const CostTreeDev& t, const double* z, int n,
                                             double* sdu, double* red) {
  const int tid = threadIdx.x;
  const int nx = s.nx, nu = s.nu, W = nx + nu;
  const int a = t.parent[n];
  double lin = 0.0;
  if (tid < nu) {
    const double u = z[(size_t)n * W + nx + tid];
    const double ua = a >= 0 ? z[(size_t)a * W + nx + tid] : t.q[tid];
    sdu[tid] = u - ua;
    lin = s.W_alpha * (s.alpha1[tid] + t.alpha2[(size_t)t.stage[n] * nu + tid]) * u;
  }
  __syncthreads();
  double quad = 0.0;
  if (tid < nu) {
    double acc = 0.0;
    for (int k = 0; k < nu; ++k) acc += s.Wu[(size_t)tid * nu + k] * sdu[k];
    quad = sdu[tid] * acc;
  }
  double v[1] = {lin + quad};
  block_sum<1>(v, red);
  return t.pi[n] * v[0];
}

__device__ __forceinline__ double safety_weight(const CostSysDev& s, const CostTreeDev& t, int n) {
  return s.safety_by_prob ? s.W_x * t.pi[n] : s.W_x;
}

__global__ __launch_bounds__(kDB) void k_obj_primal(CostSysDev s, CostTreeDev t, ObjDev o, double* part) {
  __shared__ double sdu[128];
  __shared__ double red[2 * 4];
  const int tid = threadIdx.x;
  const int nx = s.nx, nu = s.nu, D = 2 * nx + nu, W = nx + nu;
  double acc[3] = {0.0, 0.0, 0.0};
  for (int n = blockIdx.x; n < t.M; n += gridDim.x) {
    const double st = stage_term(s, t, o.z, n, sdu, red);
    // squared distances of t_sigma, t_zeta, x (half-space), x (box)
    double q[4] = {0.0, 0.0, 0.0, 0.0};
    if (tid < nx) {
      const double x = o.z[(size_t)n * W + tid];
      const double lo = s.xmin[tid], hi = s.xmax[tid], xs = s.xs[tid];
      double tb[2];
#pragma unroll
      for (int b = 0; b < 2; ++b) {
        const size_t k = (size_t)n * D + (size_t)b * nx + tid;
        const double w = o.yc[k] + o.c * (o.yc[k] - o.yp[k]);
        tb[b] = x - (o.yn[k] - w) / (o.lam * o.scale[(size_t)n * 3 + b]);
      }
      const double ds = tb[0] < xs ? xs - tb[0] : 0.0;
      const double dz = tb[1] < lo ? lo - tb[1] : (tb[1] > hi ? tb[1] - hi : 0.0);
      const double xsd = x < xs ? xs - x : 0.0;
      const double xzd = x < lo ? lo - x : (x > hi ? x - hi : 0.0);
      q[0] = ds * ds;
      q[1] = dz * dz;
      q[2] = xsd * xsd;
      q[3] = xzd * xzd;
    }
    block_sum<4>(q, red);
    const double cs = safety_weight(s, t, n), cd = s.gamma_d;
    acc[0] += st;
    acc[1] += cs * sqrt(q[0]) + cd * sqrt(q[1]);
    acc[2] += cs * sqrt(q[2]) + cd * sqrt(q[3]);
    __syncthreads();
  }
  if (tid == 0) {
    part[(size_t)blockIdx.x * kObjSlots + 0] = acc[0];
    part[(size_t)blockIdx.x * kObjSlots + 1] = acc[1];
    part[(size_t)blockIdx.x * kObjSlots + 2] = acc[2];
  }
}

__global__ __launch_bounds__(kDB) void k_obj_dual(CostSysDev s, CostTreeDev t, ObjDev o, double* part) {
  __shared__ double sdu[128];
  __shared__ double red[2 * 4];
  const int tid = threadIdx.x;
  const int nx = s.nx, nu = s.nu, D = 2 * nx + nu, W = nx + nu;
  double acc[3] = {0.0, 0.0, 0.0};
  double viol = -HUGE_VAL;
  for (int n = blockIdx.x; n < t.M; n += gridDim.x) {
    const double st = stage_term(s, t, o.z, n, sdu, red);
    const double s0 = o.scale[(size_t)n * 3 + 0], s1 = o.scale[(size_t)n * 3 + 1], s2 = o.scale[(size_t)n * 3 + 2];
    // <y, Hz>, support, ||y_sigma||^2, ||y_zeta||^2
    double q[4] = {0.0, 0.0, 0.0, 0.0};
    double vmax = -HUGE_VAL;
    if (tid < nx) {
      const double x = o.z[(size_t)n * W + tid];
      const double ys = s0 * o.yn[(size_t)n * D + tid];
      const double yz = s1 * o.yn[(size_t)n * D + nx + tid];
      q[0] += (ys + yz) * x;
      q[1] += ys * s.xs[tid] + fmax(yz * s.xmax[tid], yz * s.xmin[tid]);
      q[2] = ys * ys;
      q[3] = yz * yz;
      vmax = ys;
    }
    if (tid < nu) {
      const double u = o.z[(size_t)n * W + nx + tid];
      const double yu = s2 * o.yn[(size_t)n * D + 2 * nx + tid];
      q[0] += yu * u;
      q[1] += fmax(yu * s.umax[tid], yu * s.umin[tid]);
    }
    block_sum<4>(q, red);
    vmax = block_max(vmax, red);
    acc[0] += st;
    acc[1] += q[0];
    acc[2] += q[1];
    viol = fmax(viol, fmax(vmax, fmax(sqrt(q[2]) - safety_weight(s, t, n), sqrt(q[3]) - s.gamma_d)));
    __syncthreads();
  }
  if (tid == 0) {
    part[(size_t)blockIdx.x * kObjSlots + 3] = acc[0];
    part[(size_t)blockIdx.x * kObjSlots + 4] = acc[1];
    part[(size_t)blockIdx.x * kObjSlots + 5] = acc[2];
    part[(size_t)blockIdx.x * kObjSlots + 6] = viol;
  }
}

// out[k] = sum over workgroups of slot k (slot 6: max), workgroup order fixed.
__global__ __launch_bounds__(64) void k_obj_reduce(const double* part, int blocks, int first, int last, double* out) {
  const int lane = threadIdx.x;
  for (int k = first; k <= last; ++k) {
    double v = k == 6 ? -HUGE_VAL : 0.0;
    for (int b = lane; b < blocks; b += 64) {
      const double p = part[(size_t)b * kObjSlots + k];
      v = k == 6 ? fmax(v, p) : v + p;
    }
    v = k == 6 ? wmax(v) : wsum(v);
    if (lane == 0) out[k] = v;
  }
}

__global__ void k_scale_dual(const double* __restrict__ src, double* __restrict__ dst, const double* __restrict__ scale,
                             int M, int nx, int nu) {
  const int D = 2 * nx + nu;
  const size_t n_all = (size_t)M * D;
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n_all; i += (size_t)gridDim.x * blockDim.x) {
    const size_t n = i / D;
    const int k = (int)(i - n * D);
    const int b = k < nx ? 0 : (k < 2 * nx ? 1 : 2);
    dst[i] = scale[n * 3 + b] * src[i];
  }
}

__global__ void k_narrow(const double* __restrict__ src, float* __restrict__ dst, size_t n) {
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
    dst[i] = (float)src[i];
}

int grid_for(size_t n, int block) {
  const size_t g = (n + block - 1) / block;
  return (int)(g < 4096 ? (g > 0 ? g : 1) : 4096);
}

// Device scratch of the no-allocation objective entry point: the partial
// sums of up to kObjMaxBlocks workgroups and the kObjSlots results.  Each GPU
// holds its own copy for the life of the process; every call on a GPU
// shares it.
static __device__ __align__(256) double scratch[kObjSlots * (kObjMaxBlocks + 1)];

}  // namespace

// The device address of `scratch` on the current device, looked up once per
// device (the array's name in host code is not a device address).
hipError_t objective_scratch(double** ptr) {
  static std::mutex mu;
  static double* addr[64] = {nullptr};
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= 64) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> g(mu);
  if (!addr[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    addr[dev] = static_cast<double*>(p);
  }
  *ptr = addr[dev];
  return hipSuccess;
}

hipError_t launch_cost_update(const CostSysDev& s, const CostTreeDev& t, hipStream_t st) {
  const int grid = t.M < 8192 ? t.M : 8192;
  hipLaunchKernelGGL(k_cost_uhat_e, dim3(grid), dim3(kDB), sizeof(double) * (s.nd + s.nu), st, s, t);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_cost_beta, dim3(grid), dim3(kDB), sizeof(double) * s.nu, st, s, t);
  return hipGetLastError();
}

hipError_t launch_root_beta(const CostSysDev& s, const CostTreeDev& t, hipStream_t st) {
  hipLaunchKernelGGL(k_root_beta, dim3(1), dim3(kDB), 0, st, s, t);
  return hipGetLastError();
}

hipError_t launch_objective(const CostSysDev& s, const CostTreeDev& t, const ObjDev& o, bool dual, double* part,
                            int blocks, double* out, hipStream_t st) {
  if (blocks < 1 || blocks > kObjMaxBlocks) return hipErrorInvalidValue;
  if (dual)
    hipLaunchKernelGGL(k_obj_dual, dim3(blocks), dim3(kDB), 0, st, s, t, o, part);
  else
    hipLaunchKernelGGL(k_obj_primal, dim3(blocks), dim3(kDB), 0, st, s, t, o, part);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_obj_reduce, dim3(1), dim3(64), 0, st, part, blocks, dual ? 3 : 0, dual ? 6 : 2, out);
  return hipGetLastError();
}

hipError_t launch_scale_dual(const double* src, double* dst, const double* scale, int M, int nx, int nu,
                             hipStream_t st) {
  const size_t n = (size_t)M * (2 * nx + nu);
  hipLaunchKernelGGL(k_scale_dual, dim3(grid_for(n, 256)), dim3(256), 0, st, src, dst, scale, M, nx, nu);
  return hipGetLastError();
}

hipError_t launch_narrow(const double* src, float* dst, size_t n, hipStream_t st) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_narrow, dim3(grid_for(n, 256)), dim3(256), 0, st, src, dst, n);
  return hipGetLastError();
}

}  // namespace smpc
