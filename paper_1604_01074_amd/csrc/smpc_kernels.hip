// HIP kernels of the APG iteration for scenario-tree SMPC on gfx950.
//
// One iteration of eq. apg-iteration is, per level of the chain tree,
//   k_backward  (leaf chains first):  extrapolation + backward sweep of the
//                solve step (Alg. 1, first loop) over every chain of the level;
//   k_forward   (root chain first):   forward rollout of the solve step (Alg. 1,
//                second loop) fused with the prox of App. C and the dual update;
//   k_iter_end  (one workgroup per tree): float64 residual reduction, stop
//                test, iteration counter.
//
// A chain is a maximal path of single-child nodes.  One workgroup walks one
// chain, so the sequential stage dependence inside a chain never leaves the
// workgroup; only the (few) branching levels need a kernel boundary.
//
// The solve step is computed in input space rather than in the reduced
// variables v of App. A: with P = L (L' Wu L)^{-1} L' (independent of the
// choice of L), the backward sweep is
//   Q_n   = xi_n + A' sum_c Q_c                      (nx)
//   rho_n = beta_n + psi~_n + B' Q_n + sum_c rho_c    (nu)
//   du_n  = -P rho_n / (2 pi_n)                       (nu)
// and the forward rollout is
//   ut_n = ut_{a(n)} + du_n,  u_n = ut_n + uhat_n,  x_n = A x_{a(n)} + B ut_n + e_n
// which is Alg. 1 multiplied through by L (du_n = L dv_n, ut_n = L v_n).
// B and A are applied in sparse (CSR) form, P is staged in LDS.
#include "smpc_internal.h"

namespace smpc {

namespace {

template <typename T>
__device__ __forceinline__ T wave_sum(T v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// max that lets a NaN through (a NaN residual must not be hidden)
__device__ __forceinline__ double nanmax(double a, double b) {
  if (a != a || b != b) return __longlong_as_double(0x7ff8000000000000LL);
  return a > b ? a : b;
}

__device__ __forceinline__ double wave_nanmax(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v = nanmax(v, __shfl_xor(v, off, 64));
  return v;
}

template <typename T>
__device__ __forceinline__ T clampv(T a, T lo, T hi) {
  return a < lo ? lo : (a > hi ? hi : a);
}

// Dynamic LDS: 32 float64 reduction slots, then T-typed arrays.
constexpr int kRedDoubles = 32;

}  // namespace

size_t lds_bytes_backward(int nx, int nu, size_t elem) {
  // P, Q (2 x nx), rho (2 x nu), psi (nu), partial sums (4 x nu)
  return kRedDoubles * sizeof(double) + elem * ((size_t)nu * nu + 2 * nx + 7 * (size_t)nu);
}

size_t lds_bytes_forward(int nx, int nu, size_t elem) {
  // x (2 x nx), ut (2 x nu), u (nu)
  return kRedDoubles * sizeof(double) + elem * (2 * (size_t)nx + 3 * (size_t)nu);
}

// ---------------------------------------------------------------------------
// backward sweep of one chain
// ---------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(kBlock) void k_backward(SysDev<T> sys, const TreeDev<T>* __restrict__ trees,
                                                     const WorkItem* __restrict__ items,
                                                     const double* __restrict__ ctab, int mode) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const int tid = threadIdx.x;
  const WorkItem wi = items[blockIdx.x];
  const TreeDev<T>& td = trees[wi.tree];
  const TreeState* st = td.st;
  if (st->done) return;
  const int it = st->iter;
  const ChainDesc ch = td.chains[wi.chain];
  const int nx = sys.nx, nu = sys.nu, D = sys.D;

  T c = T(0), in_scale = T(1);
  if (mode == kModeAPG) c = (T)ctab[it];
  if (mode == kModePower) in_scale = (T)st->in_scale;
  const bool affine = (mode != kModePower);
  const bool scaled = (td.scale != nullptr) && (mode != kModeSolve);
  const T* __restrict__ ycur = td.y[it % 3];
  const T* __restrict__ yprv = td.y[(it + 2) % 3];

  T* sm = reinterpret_cast<T*>(smem_raw + kRedDoubles * sizeof(double));
  T* sP = sm;
  T* sQa = sP + (size_t)nu * nu;
  T* sQb = sQa + nx;
  T* sRa = sQb + nx;
  T* sRb = sRa + nu;
  T* sPsi = sRb + nu;
  T* sPart = sPsi + nu;

  for (int i = tid; i < nu * nu; i += kBlock) sP[i] = sys.P[i];
  // cost-to-go terms handed up by the child chains of the bottom node
  for (int i = tid; i < nx; i += kBlock) {
    T acc = T(0);
    for (int cc = 0; cc < ch.child_count; ++cc) acc += td.ctopQ[(size_t)(ch.child_begin + cc) * nx + i];
    sQa[i] = acc;
  }
  for (int j = tid; j < nu; j += kBlock) {
    T acc = T(0);
    for (int cc = 0; cc < ch.child_count; ++cc) acc += td.ctopR[(size_t)(ch.child_begin + cc) * nu + j];
    sRa[j] = acc;
  }
  __syncthreads();

  T* Qc = sQa;  // child term (A' applied below)
  T* Qn = sQb;
  T* Rc = sRa;
  T* Rn = sRb;
  const int NR = nu <= 64 ? 64 : (nu <= 128 ? 128 : 256);
  const int splits = kBlock / NR;
  const int mj = tid % NR;
  const int mh = tid / NR;
  const int kc = (nu + splits - 1) / splits;
  const int k0 = mh * kc;
  const int k1 = min(nu, k0 + kc);

  for (int k = ch.len - 1; k >= 0; --k) {
    const int n = ch.first + k;
    const T* yn = ycur + (size_t)n * D;
    const T* ypn = yprv + (size_t)n * D;
    T s0 = T(1), s1 = T(1), s2 = T(1);
    if (scaled) {
      s0 = td.scale[(size_t)n * 3 + 0];
      s1 = td.scale[(size_t)n * 3 + 1];
      s2 = td.scale[(size_t)n * 3 + 2];
    }
    // Q_n = S(w_sigma + w_zeta) + A' Q_c
    for (int i = tid; i < nx; i += kBlock) {
      T wa = yn[i], wb = yn[nx + i];
      if (mode == kModeAPG) {
        wa += c * (wa - ypn[i]);
        wb += c * (wb - ypn[nx + i]);
      } else if (mode == kModePower) {
        wa *= in_scale;
        wb *= in_scale;
      }
      T q = s0 * wa + s1 * wb;
      if (sys.a_identity) {
        q += Qc[i];
      } else {
        for (int r = sys.at_rp[i]; r < sys.at_rp[i + 1]; ++r) q += sys.at_v[r] * Qc[sys.at_ci[r]];
      }
      Qn[i] = q;
    }
    for (int j = tid; j < nu; j += kBlock) {
      T w = yn[2 * nx + j];
      if (mode == kModeAPG) w += c * (w - ypn[2 * nx + j]);
      else if (mode == kModePower) w *= in_scale;
      sPsi[j] = s2 * w;
    }
    __syncthreads();
    // rho_n = beta_n + psi_n + B' Q_n + sum_c rho_c
    for (int j = tid; j < nu; j += kBlock) {
      T r = sPsi[j] + Rc[j];
      if (affine) r += td.beta[(size_t)n * nu + j];
      for (int q = sys.bt_rp[j]; q < sys.bt_rp[j + 1]; ++q) r += sys.bt_v[q] * Qn[sys.bt_ci[q]];
      Rn[j] = r;
    }
    __syncthreads();
    // du_n = -P rho_n / (2 pi_n): rows split over NR lanes, K split in `splits`
    if (mj < nu) {
      T acc = T(0);
      for (int kk = k0; kk < k1; ++kk) acc += sP[(size_t)kk * nu + mj] * Rn[kk];
      sPart[mh * nu + mj] = acc;
    }
    __syncthreads();
    const T scl = T(-0.5) / td.pi[n];
    for (int j = tid; j < nu; j += kBlock) {
      T acc = T(0);
      for (int h = 0; h < splits; ++h) acc += sPart[h * nu + j];
      td.du[(size_t)n * nu + j] = scl * acc;
    }
    T* t = Qc; Qc = Qn; Qn = t;
    t = Rc; Rc = Rn; Rn = t;
  }
  // top node of the chain: hand Q and rho to the parent chain
  for (int i = tid; i < nx; i += kBlock) td.ctopQ[(size_t)wi.chain * nx + i] = Qc[i];
  for (int j = tid; j < nu; j += kBlock) td.ctopR[(size_t)wi.chain * nu + j] = Rc[j];
}

// ---------------------------------------------------------------------------
// forward rollout of one chain, fused with prox and dual update
// ---------------------------------------------------------------------------
template <typename T, int PT>
__global__ __launch_bounds__(kBlock) void k_forward(SysDev<T> sys, const TreeDev<T>* __restrict__ trees,
                                                    const WorkItem* __restrict__ items,
                                                    const double* __restrict__ ctab, int mode) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  double* sRed = reinterpret_cast<double*>(smem_raw);
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const WorkItem wi = items[blockIdx.x];
  const TreeDev<T>& td = trees[wi.tree];
  const TreeState* st = td.st;
  if (st->done) return;
  const int it = st->iter;
  const ChainDesc ch = td.chains[wi.chain];
  const int nx = sys.nx, nu = sys.nu, D = sys.D;
  const bool affine = (mode != kModePower);
  const bool scaled = (td.scale != nullptr) && (mode != kModeSolve);
  const bool check = (mode != kModeAPG) || ((it + 1) % st->check_every == 0) || (it + 1 >= st->max_iter);

  T c = T(0), in_scale = T(1), lam = T(1), ilam = T(1);
  if (mode == kModeAPG) {
    c = (T)ctab[it];
    lam = (T)st->lambda;
    ilam = T(1) / lam;
  }
  if (mode == kModePower) in_scale = (T)st->in_scale;
  const T* __restrict__ ycur = td.y[it % 3];
  const T* __restrict__ yprv = td.y[(it + 2) % 3];
  T* __restrict__ ynew = td.y[(it + 1) % 3];

  T* sm = reinterpret_cast<T*>(smem_raw + kRedDoubles * sizeof(double));
  T* sXa = sm;
  T* sXb = sXa + nx;
  T* sUa = sXb + nx;  // ut (u - uhat) of the parent / current node
  T* sUb = sUa + nu;
  T* sUf = sUb + nu;  // u of the current node

  if (ch.parent < 0) {
    for (int i = tid; i < nx; i += kBlock) sXa[i] = affine ? td.p[i] : T(0);
    for (int j = tid; j < nu; j += kBlock) sUa[j] = T(0);
  } else {
    for (int i = tid; i < nx; i += kBlock) sXa[i] = td.cbotX[(size_t)ch.parent * nx + i];
    for (int j = tid; j < nu; j += kBlock) sUa[j] = td.cbotU[(size_t)ch.parent * nu + j];
  }
  __syncthreads();

  T* Xa = sXa;
  T* Xn = sXb;
  T* Ua = sUa;
  T* Un = sUb;
  const T xi_cS = (T)(sys.W_x);
  const T gam_d = (T)(sys.gamma_d);

  double st0 = 0.0, st1 = 0.0, st2 = 0.0;  // residual / |Hz| / |t| maxima, or power sums

  for (int k = 0; k < ch.len; ++k) {
    const int n = ch.first + k;
    // ut_n = ut_a + du_n,  u_n = ut_n + uhat_n
    for (int j = tid; j < nu; j += kBlock) {
      const T ut = Ua[j] + td.du[(size_t)n * nu + j];
      Un[j] = ut;
      sUf[j] = affine ? ut + td.uhat[(size_t)n * nu + j] : ut;
    }
    __syncthreads();
    // x_n = A x_a + B ut_n + e_n
    for (int i = tid; i < nx; i += kBlock) {
      T x;
      if (sys.a_identity) {
        x = Xa[i];
      } else {
        x = T(0);
        for (int r = sys.a_rp[i]; r < sys.a_rp[i + 1]; ++r) x += sys.a_v[r] * Xa[sys.a_ci[r]];
      }
      for (int r = sys.b_rp[i]; r < sys.b_rp[i + 1]; ++r) x += sys.b_v[r] * Un[sys.b_ci[r]];
      if (affine) x += td.e[(size_t)n * nx + i];
      Xn[i] = x;
    }
    __syncthreads();

    if (mode == kModeSolve || (mode == kModeAPG && check)) {
      const size_t zo = (size_t)n * (nx + nu);
      for (int i = tid; i < nx; i += kBlock) td.z[zo + i] = Xn[i];
      for (int j = tid; j < nu; j += kBlock) td.z[zo + nx + j] = sUf[j];
    }

    if (mode == kModeAPG) {
      T s0 = T(1), s1 = T(1), s2 = T(1);
      if (scaled) {
        s0 = td.scale[(size_t)n * 3 + 0];
        s1 = td.scale[(size_t)n * 3 + 1];
        s2 = td.scale[(size_t)n * 3 + 2];
      }
      const T* yn = ycur + (size_t)n * D;
      const T* ypn = yprv + (size_t)n * D;
      T r_w[PT], r_hz[PT], r_a[PT], r_p[PT], r_s[PT];
      int r_b[PT];
      T dsq0 = T(0), dsq1 = T(0);
#pragma unroll
      for (int r = 0; r < PT; ++r) {
        const int idx = tid + r * kBlock;
        r_b[r] = 3;
        if (idx < D) {
          int b, comp;
          if (idx < nx) { b = 0; comp = idx; }
          else if (idx < 2 * nx) { b = 1; comp = idx - nx; }
          else { b = 2; comp = idx - 2 * nx; }
          const T s = b == 0 ? s0 : (b == 1 ? s1 : s2);
          T y = yn[idx];
          const T w = y + c * (y - ypn[idx]);
          const T hzv = b < 2 ? Xn[comp] : sUf[comp];
          const T a = (w * ilam + s * hzv) / s;  // prox argument in unscaled units
          T pa;
          if (b == 0) pa = a > sys.xs[comp] ? a : sys.xs[comp];
          else if (b == 1) pa = clampv(a, sys.xmin[comp], sys.xmax[comp]);
          else pa = clampv(a, sys.umin[comp], sys.umax[comp]);
          const T dd = a - pa;
          if (b == 0) dsq0 += dd * dd;
          else if (b == 1) dsq1 += dd * dd;
          r_b[r] = b; r_w[r] = w; r_hz[r] = hzv; r_a[r] = a; r_p[r] = pa; r_s[r] = s;
        }
      }
      // two block sums (fixed order -> deterministic)
      dsq0 = wave_sum(dsq0);
      dsq1 = wave_sum(dsq1);
      if (lane == 0) {
        sRed[wave * 2 + 0] = (double)dsq0;
        sRed[wave * 2 + 1] = (double)dsq1;
      }
      __syncthreads();
      const T del0 = (T)sqrt(sRed[0] + sRed[2] + sRed[4] + sRed[6]);
      const T del1 = (T)sqrt(sRed[1] + sRed[3] + sRed[5] + sRed[7]);
      const T cS = sys.safety_by_prob ? xi_cS * td.pi[n] : xi_cS;
#pragma unroll
      for (int r = 0; r < PT; ++r) {
        const int idx = tid + r * kBlock;
        if (idx < D) {
          const int b = r_b[r];
          const T s = r_s[r], a = r_a[r], pa = r_p[r];
          T tun;
          if (b < 2) {
            const T del = b == 0 ? del0 : del1;
            const T cb = b == 0 ? cS : gam_d;
            const T tau = cb * ilam / (s * s);
            tun = del <= tau ? pa : a - (tau / del) * (a - pa);
          } else {
            tun = pa;
          }
          const T hzv = r_hz[r];
          ynew[(size_t)n * D + idx] = r_w[r] + lam * (s * hzv - s * tun);
          st0 = nanmax(st0, fabs((double)hzv - (double)tun));
          st1 = nanmax(st1, fabs((double)hzv));
          st2 = nanmax(st2, fabs((double)tun));
        }
      }
    } else if (mode == kModePower) {
      T s0 = T(1), s1 = T(1), s2 = T(1);
      if (scaled) {
        s0 = td.scale[(size_t)n * 3 + 0];
        s1 = td.scale[(size_t)n * 3 + 1];
        s2 = td.scale[(size_t)n * 3 + 2];
      }
      const T* yn = ycur + (size_t)n * D;
#pragma unroll
      for (int r = 0; r < PT; ++r) {
        const int idx = tid + r * kBlock;
        if (idx < D) {
          int b, comp;
          if (idx < nx) { b = 0; comp = idx; }
          else if (idx < 2 * nx) { b = 1; comp = idx - nx; }
          else { b = 2; comp = idx - 2 * nx; }
          const T s = b == 0 ? s0 : (b == 1 ? s1 : s2);
          const T hzv = b < 2 ? Xn[comp] : sUf[comp];
          const T g = -s * hzv;
          const T w = in_scale * yn[idx];
          ynew[(size_t)n * D + idx] = g;
          st0 += (double)g * (double)g;
          st1 += (double)w * (double)g;
        }
      }
    }
    if (mode != kModeAPG) __syncthreads();  // sUf / Xn reuse in the next node
    T* t = Xa; Xa = Xn; Xn = t;
    t = Ua; Ua = Un; Un = t;
  }
  // bottom node of the chain: hand x and ut to the child chains
  if (ch.child_count > 0) {
    for (int i = tid; i < nx; i += kBlock) td.cbotX[(size_t)wi.chain * nx + i] = Xa[i];
    for (int j = tid; j < nu; j += kBlock) td.cbotU[(size_t)wi.chain * nu + j] = Ua[j];
  }
  // chain partials
  if (mode == kModeAPG) {
    st0 = wave_nanmax(st0);
    st1 = wave_nanmax(st1);
    st2 = wave_nanmax(st2);
  } else if (mode == kModePower) {
    st0 = wave_sum(st0);
    st1 = wave_sum(st1);
  }
  __syncthreads();
  if (lane == 0) {
    sRed[8 + wave * 3 + 0] = st0;
    sRed[8 + wave * 3 + 1] = st1;
    sRed[8 + wave * 3 + 2] = st2;
  }
  __syncthreads();
  if (tid == 0) {
    double* out = td.cstat + (size_t)wi.chain * kStat;
    if (mode == kModeAPG) {
      double a0 = sRed[8], a1 = sRed[9], a2 = sRed[10];
      for (int w = 1; w < kBlock / 64; ++w) {
        a0 = nanmax(a0, sRed[8 + 3 * w]);
        a1 = nanmax(a1, sRed[9 + 3 * w]);
        a2 = nanmax(a2, sRed[10 + 3 * w]);
      }
      out[0] = a0; out[1] = a1; out[2] = a2; out[3] = 0.0;
    } else if (mode == kModePower) {
      double a0 = sRed[8], a1 = sRed[9];
      for (int w = 1; w < kBlock / 64; ++w) {
        a0 += sRed[8 + 3 * w];
        a1 += sRed[9 + 3 * w];
      }
      out[0] = a0; out[1] = a1; out[2] = 0.0; out[3] = 0.0;
    }
  }
}

// ---------------------------------------------------------------------------
// per-tree end of iteration
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(64) void k_iter_end(const IterRef* __restrict__ refs, int mode) {
  const IterRef r = refs[blockIdx.x];
  TreeState* st = r.st;
  const int lane = threadIdx.x;
  const int done0 = st->done;
  if (done0) {
    if (lane == 0) r.done_out[r.slot] = 1;
    return;
  }
  const int it = st->iter;
  if (mode == kModeAPG) {
    const bool check = ((it + 1) % st->check_every == 0) || (it + 1 >= st->max_iter);
    int done = 0;
    if (check) {
      double rm = 0.0, hm = 0.0;
      for (int c = lane; c < r.n_chains; c += 64) {
        rm = nanmax(rm, r.cstat[(size_t)c * kStat + 0]);
        hm = nanmax(hm, r.cstat[(size_t)c * kStat + 1]);
        hm = nanmax(hm, r.cstat[(size_t)c * kStat + 2]);
      }
      rm = wave_nanmax(rm);
      hm = wave_nanmax(hm);
      if (lane == 0) {
        st->r_p = rm;
        st->hzt = hm;
        const bool finite = (rm == rm) && (hm == hm) && rm < 1e300 && hm < 1e300;
        if (!finite) {
          done = 1;
          st->status = -9;
        } else if (st->tol > 0.0 && rm <= st->tol * (1.0 + hm)) {
          done = 1;
          st->status = 0;
        } else if (it + 1 >= st->max_iter) {
          done = 1;
          st->status = 1;
        }
        if (done) {
          st->done = 1;
          st->iters_done = it + 1;
        }
      }
    }
    if (lane == 0) {
      st->iter = it + 1;
      r.done_out[r.slot] = done;
    }
  } else if (mode == kModePower) {
    double gg = 0.0, wg = 0.0;
    for (int c = lane; c < r.n_chains; c += 64) {
      gg += r.cstat[(size_t)c * kStat + 0];
      wg += r.cstat[(size_t)c * kStat + 1];
    }
    gg = wave_sum(gg);
    wg = wave_sum(wg);
    if (lane == 0) {
      st->lmax_est = wg;
      st->in_scale = gg > 0.0 ? 1.0 / sqrt(gg) : 0.0;
      st->iter = it + 1;
      r.done_out[r.slot] = 0;
    }
  }
}

template <typename T>
__global__ void k_narrow(const double* __restrict__ src, T* __restrict__ dst, size_t n) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) dst[i] = (T)src[i];
}

template <typename T>
__global__ void k_widen(const T* __restrict__ src, double* __restrict__ dst, size_t n) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) dst[i] = (double)src[i];
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
template <typename T>
hipError_t launch_backward(const SysDev<T>& sys, const TreeDev<T>* trees, const WorkItem* items, int n_items,
                           const double* ctab, int mode, hipStream_t s) {
  if (n_items <= 0) return hipSuccess;
  const size_t lds = lds_bytes_backward(sys.nx, sys.nu, sizeof(T));
  static bool attr_set = false;
  if (!attr_set) {
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(&k_backward<T>),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
    if (e != hipSuccess) return e;
    attr_set = true;
  }
  hipLaunchKernelGGL(k_backward<T>, dim3(n_items), dim3(kBlock), lds, s, sys, trees, items, ctab, mode);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_forward(const SysDev<T>& sys, const TreeDev<T>* trees, const WorkItem* items, int n_items,
                          const double* ctab, int mode, hipStream_t s) {
  if (n_items <= 0) return hipSuccess;
  const size_t lds = lds_bytes_forward(sys.nx, sys.nu, sizeof(T));
  const int maxdim = sys.D;
  if (maxdim <= kBlock) {
    hipLaunchKernelGGL((k_forward<T, 1>), dim3(n_items), dim3(kBlock), lds, s, sys, trees, items, ctab, mode);
  } else if (maxdim <= 2 * kBlock) {
    hipLaunchKernelGGL((k_forward<T, 2>), dim3(n_items), dim3(kBlock), lds, s, sys, trees, items, ctab, mode);
  } else {
    hipLaunchKernelGGL((k_forward<T, 4>), dim3(n_items), dim3(kBlock), lds, s, sys, trees, items, ctab, mode);
  }
  return hipGetLastError();
}

hipError_t launch_iter_end_refs(const void* refs, int n_trees, int mode, hipStream_t s) {
  if (n_trees <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_iter_end, dim3(n_trees), dim3(64), 0, s, reinterpret_cast<const IterRef*>(refs), mode);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_convert_dual(const double* src, T* dst, size_t n, hipStream_t s) {
  if (n == 0) return hipSuccess;
  const unsigned blocks = (unsigned)((n + 255) / 256);
  hipLaunchKernelGGL(k_narrow<T>, dim3(blocks), dim3(256), 0, s, src, dst, n);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_widen(const T* src, double* dst, size_t n, hipStream_t s) {
  if (n == 0) return hipSuccess;
  const unsigned blocks = (unsigned)((n + 255) / 256);
  hipLaunchKernelGGL(k_widen<T>, dim3(blocks), dim3(256), 0, s, src, dst, n);
  return hipGetLastError();
}

template hipError_t launch_backward<double>(const SysDev<double>&, const TreeDev<double>*, const WorkItem*, int,
                                            const double*, int, hipStream_t);
template hipError_t launch_backward<float>(const SysDev<float>&, const TreeDev<float>*, const WorkItem*, int,
                                           const double*, int, hipStream_t);
template hipError_t launch_forward<double>(const SysDev<double>&, const TreeDev<double>*, const WorkItem*, int,
                                           const double*, int, hipStream_t);
template hipError_t launch_forward<float>(const SysDev<float>&, const TreeDev<float>*, const WorkItem*, int,
                                          const double*, int, hipStream_t);
template hipError_t launch_convert_dual<float>(const double*, float*, size_t, hipStream_t);
template hipError_t launch_widen<float>(const float*, double*, size_t, hipStream_t);

}  // namespace smpc
