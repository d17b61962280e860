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
// B and A are applied in sparse (CSR) form; P is held in registers.
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

// Nodes of one chain processed together (24 in float32, 12 in float64, which
// keeps a chunk's staging within LDS at several workgroups per CU).  Within a
// chunk the work is: wide loads, short per-component scans for the
// recursions, then wide compute.
template <typename T>
struct Chunk {
  static constexpr int value = sizeof(T) == 4 ? 24 : 12;
};

}  // namespace

int p_stride(int nu) { return nu <= 64 ? 64 : 128; }

size_t lds_bytes_backward(int nx, int nu, size_t elem) {
  // per chunk node: w (D), beta (nu), xi/Q (nx), r/rho (row padded to the P
  // stride), -1/(2 pi), 3 scales; two carries
  const size_t ch = elem == 4 ? Chunk<float>::value : Chunk<double>::value;
  const size_t D = 2 * (size_t)nx + nu;
  return kRedDoubles * sizeof(double) + elem * (ch * (D + nu + nx + p_stride(nu) + 4) + nx + nu);
}

size_t lds_bytes_forward(int nx, int nu, size_t elem) {
  // per chunk node: w (D), du/ut, uhat (nu each), e/x (nx), pi, 3 scales;
  // two carries
  const size_t ch = elem == 4 ? Chunk<float>::value : Chunk<double>::value;
  const size_t D = 2 * (size_t)nx + nu;
  return kRedDoubles * sizeof(double) + elem * (ch * (D + 2 * nu + nx + 4) + nx + nu);
}

// Loads per thread and array issued in one staging batch, before any LDS
// store (halved in float64 to leave registers for the P slice).
template <typename T>
struct Stage {
  static constexpr int Y = sizeof(T) == 4 ? 12 : 6;
  static constexpr int U = sizeof(T) == 4 ? 6 : 3;
  static constexpr int X = sizeof(T) == 4 ? 4 : 2;
};

namespace {

// ---------------------------------------------------------------------------
// backward sweep of one chain
//
// Per chunk (bottom-up): load xi_n = S(w_sigma + w_zeta) and
// r_n = beta_n + S w_psi of all its nodes at once; run the recursions
// Q_n = xi_n + A' Q_below and rho_n = r_n + B' Q_n + rho_below as per-component
// scans (one thread per component when A = I); then du_n = -P rho_n / (2 pi_n)
// for all nodes of the chunk with P held in registers: thread (j, h) keeps
// P[j][h*KH .. h*KH + KH) and the S k-parts of a row sit in adjacent lanes,
// so the partial sums combine with lane shuffles.
// ---------------------------------------------------------------------------
template <typename T, int S, int KH>
__global__ __launch_bounds__(kBlock, 2) void k_backward(SysDev<T> sys, const TreeDev<T>* __restrict__ trees,
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

  constexpr int kChunk = Chunk<T>::value;
  constexpr int kStageY = Stage<T>::Y, kStageU = Stage<T>::U;
  constexpr int KP = S * KH;  // padded P stride and rho row stride
  T* sW = reinterpret_cast<T*>(smem_raw + kRedDoubles * sizeof(double));  // kChunk x D
  T* sB = sW + (size_t)kChunk * D;                                        // kChunk x nu
  T* sQ = sB + (size_t)kChunk * nu;                                       // kChunk x nx
  T* sR = sQ + (size_t)kChunk * nx;  // kChunk x KP, entries nu..KP-1 stay zero
  T* sI = sR + (size_t)kChunk * KP;  // kChunk
  T* sS = sI + kChunk;               // kChunk x 3
  T* sQc = sS + 3 * kChunk;
  T* sRc = sQc + nx;

  // P slice of this thread (P is stored zero-padded to KP x KP)
  const int pj = tid / S;
  const int ph = tid % S;
  T preg[KH];
#pragma unroll
  for (int kk = 0; kk < KH; ++kk) preg[kk] = sys.P[(size_t)(ph * KH + kk) * KP + pj];
  for (int e = tid; e < kChunk * (KP - nu); e += kBlock) {
    const int cc = e / (KP - nu);
    sR[cc * KP + nu + (e - cc * (KP - nu))] = T(0);
  }
  // this thread's sparse row of B' (a flow touches few tanks), kept in
  // registers; unused slots have weight 0 and index 0
  constexpr int kNnz = 4;
  int bt_c[kNnz];
  T bt_w[kNnz];
  int bt_n = 0, bt_q0 = 0, bt_q1 = 0;
  if (tid < nu) {
    bt_q0 = sys.bt_rp[tid];
    bt_q1 = sys.bt_rp[tid + 1];
    bt_n = bt_q1 - bt_q0;
  }
#pragma unroll
  for (int q = 0; q < kNnz; ++q) {
    bt_c[q] = q < bt_n ? sys.bt_ci[bt_q0 + q] : 0;
    bt_w[q] = q < bt_n ? sys.bt_v[bt_q0 + q] : T(0);
  }

  // cost-to-go terms handed up by the child chains of the bottom node
  for (int i = tid; i < nx; i += kBlock) {
    T acc = T(0);
    for (int cc = 0; cc < ch.child_count; ++cc) acc += td.ctopQ[(size_t)(ch.child_begin + cc) * nx + i];
    sQc[i] = acc;
  }
  for (int j = tid; j < nu; j += kBlock) {
    T acc = T(0);
    for (int cc = 0; cc < ch.child_count; ++cc) acc += td.ctopR[(size_t)(ch.child_begin + cc) * nu + j];
    sRc[j] = acc;
  }

  const int W = nx + nu;
  for (int top = ch.len; top > 0; top -= kChunk) {
    const int k0 = top > kChunk ? top - kChunk : 0;
    const int C = top - k0;
    const int nb = ch.first + k0;  // internal index of the chunk's first node
    // stage the chunk: its nodes are consecutive, so y, y_prev and beta are
    // contiguous ranges; every batch issues all its loads before any store
    {
      const int ny = C * D;
      const int nbt = affine ? C * nu : 0;
      const size_t oy = (size_t)nb * D, ob = (size_t)nb * nu;
      for (int b = 0; b * kStageY * kBlock < ny || b * kStageU * kBlock < nbt; ++b) {
        T ry[kStageY], rp[kStageY], rb[kStageU];
        T rs = T(1), rpi = T(1);
#pragma unroll
        for (int u = 0; u < kStageY; ++u) {
          const int e = (b * kStageY + u) * kBlock + tid;
          ry[u] = e < ny ? ycur[oy + e] : T(0);
          rp[u] = (mode == kModeAPG && e < ny) ? yprv[oy + e] : T(0);
        }
#pragma unroll
        for (int u = 0; u < kStageU; ++u) {
          const int e = (b * kStageU + u) * kBlock + tid;
          rb[u] = e < nbt ? td.beta[ob + e] : T(0);
        }
        if (b == 0) {
          if (tid < 3 * C && scaled) rs = td.scale[(size_t)nb * 3 + tid];
          if (tid < C) rpi = td.pi[nb + tid];
        }
#pragma unroll
        for (int u = 0; u < kStageY; ++u) {
          const int e = (b * kStageY + u) * kBlock + tid;
          if (e < ny) {
            const T y = ry[u];
            sW[e] = mode == kModeAPG ? y + c * (y - rp[u]) : (mode == kModePower ? in_scale * y : y);
          }
        }
#pragma unroll
        for (int u = 0; u < kStageU; ++u) {
          const int e = (b * kStageU + u) * kBlock + tid;
          if (e < nbt) sB[e] = rb[u];
        }
        if (b == 0) {
          if (tid < 3 * C) sS[tid] = rs;
          if (tid < C) sI[tid] = T(-0.5) / rpi;
        }
      }
    }
    __syncthreads();
    // xi = S(w_sigma + w_zeta) and r = beta + S w_psi from LDS
    for (int e = tid; e < C * nx; e += kBlock) {
      const int cc = e / nx;
      const int i = e - cc * nx;
      sQ[e] = sS[3 * cc] * sW[cc * D + i] + sS[3 * cc + 1] * sW[cc * D + nx + i];
    }
    for (int e = tid; e < C * nu; e += kBlock) {
      const int cc = e / nu;
      const int j = e - cc * nu;
      sR[cc * KP + j] = (affine ? sB[e] : T(0)) + sS[3 * cc + 2] * sW[cc * D + 2 * nx + j];
    }
    __syncthreads();
    // Q recursion, bottom node of the chunk first
    if (sys.a_identity) {
      for (int i = tid; i < nx; i += kBlock) {
        T q = sQc[i];
        for (int cc = C - 1; cc >= 0; --cc) {
          q += sQ[cc * nx + i];
          sQ[cc * nx + i] = q;
        }
        sQc[i] = q;
      }
    } else {
      for (int cc = C - 1; cc >= 0; --cc) {
        for (int i = tid; i < nx; i += kBlock) {
          T q = sQ[cc * nx + i];
          for (int r = sys.at_rp[i]; r < sys.at_rp[i + 1]; ++r) q += sys.at_v[r] * sQc[sys.at_ci[r]];
          sQ[cc * nx + i] = q;
        }
        __syncthreads();
        for (int i = tid; i < nx; i += kBlock) sQc[i] = sQ[cc * nx + i];
        __syncthreads();
      }
    }
    __syncthreads();
    // rho recursion (one thread per input component; nu <= kBlock)
    if (tid < nu) {
      const int j = tid;
      T r = sRc[j];
      for (int cc = C - 1; cc >= 0; --cc) {
        T g = sR[cc * KP + j];
        if (bt_n <= kNnz) {
#pragma unroll
          for (int q = 0; q < kNnz; ++q) g += bt_w[q] * sQ[cc * nx + bt_c[q]];
        } else {
          for (int q = bt_q0; q < bt_q1; ++q) g += sys.bt_v[q] * sQ[cc * nx + sys.bt_ci[q]];
        }
        r += g;
        sR[cc * KP + j] = r;
      }
      sRc[j] = r;
    }
    __syncthreads();
    // du = -P rho / (2 pi) for the chunk
    T acc[kChunk];
#pragma unroll
    for (int cc = 0; cc < kChunk; ++cc) acc[cc] = T(0);
    // branch-free: padded entries of P and rho are zero, rows cc >= C are
    // computed from stale finite values and not stored
#pragma unroll
    for (int kk = 0; kk < KH; ++kk) {
      const T pv = preg[kk];
      const int k = ph * KH + kk;
#pragma unroll
      for (int cc = 0; cc < kChunk; ++cc) acc[cc] += pv * sR[cc * KP + k];
    }
#pragma unroll
    for (int cc = 0; cc < kChunk; ++cc) {
      T v = acc[cc];
      if (S >= 2) v += __shfl_xor(v, 1, 64);
      if (S >= 4) v += __shfl_xor(v, 2, 64);
      acc[cc] = v;
    }
    if (ph == 0 && pj < nu) {
#pragma unroll
      for (int cc = 0; cc < kChunk; ++cc)
        if (cc < C) td.du[(size_t)(nb + cc) * nu + pj] = acc[cc] * sI[cc];
    }
    __syncthreads();
  }
  // top node of the chain: hand Q and rho to the parent chain
  for (int i = tid; i < nx; i += kBlock) td.ctopQ[(size_t)wi.chain * nx + i] = sQc[i];
  for (int j = tid; j < nu; j += kBlock) td.ctopR[(size_t)wi.chain * nu + j] = sRc[j];
}

// ---------------------------------------------------------------------------
// forward rollout of one chain, fused with prox and dual update
//
// Per chunk (top-down): stage the dual point w, du, uhat and e of all its
// nodes in LDS with one round of wide loads, run the recursions
// ut_n = ut_above + du_n and x_n = A x_above + B ut_n + e_n as per-component
// scans, then the prox (App. C) and the dual update for every entry of the
// chunk: each (node, sigma|zeta) block is handled by one wave with its
// Euclidean norm reduced by lane shuffles, the psi entries are spread over all
// threads.  NXL = ceil(nx / 64) entries per lane of a distance block.
// ---------------------------------------------------------------------------
template <typename T, int NXL>
__global__ __launch_bounds__(kBlock) void k_forward(SysDev<T> sys, const TreeDev<T>* __restrict__ trees,
                                                    const WorkItem* __restrict__ items,
                                                    const double* __restrict__ ctab, int mode) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  constexpr int kChunk = Chunk<T>::value;
  constexpr int kStageY = Stage<T>::Y, kStageU = Stage<T>::U, kStageX = Stage<T>::X;
  constexpr int kWaves = kBlock / 64;
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
  const bool write_z = (mode == kModeSolve) || (mode == kModeAPG && check);

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

  T* sW = reinterpret_cast<T*>(smem_raw + kRedDoubles * sizeof(double));  // kChunk x D
  T* sU = sW + (size_t)kChunk * D;                                        // kChunk x nu
  T* sH = sU + (size_t)kChunk * nu;                                       // kChunk x nu (uhat)
  T* sX = sH + (size_t)kChunk * nu;                                       // kChunk x nx
  T* sPi = sX + (size_t)kChunk * nx;                                      // kChunk
  T* sS = sPi + kChunk;                                                   // kChunk x 3
  T* sUc = sS + 3 * kChunk;
  T* sXc = sUc + nu;

  if (ch.parent < 0) {
    for (int i = tid; i < nx; i += kBlock) sXc[i] = affine ? td.p[i] : T(0);
    for (int j = tid; j < nu; j += kBlock) sUc[j] = T(0);
  } else {
    for (int i = tid; i < nx; i += kBlock) sXc[i] = td.cbotX[(size_t)ch.parent * nx + i];
    for (int j = tid; j < nu; j += kBlock) sUc[j] = td.cbotU[(size_t)ch.parent * nu + j];
  }
  const T cSx = (T)sys.W_x;
  const T gam_d = (T)sys.gamma_d;
  double st0 = 0.0, st1 = 0.0, st2 = 0.0;  // residual / |Hz| / |t| maxima, or power sums
  const int W = nx + nu;
  const int L1 = D + 2 * nu + nx;  // staged values per node
  // this thread's sparse row of B (a tank is touched by few flows); unused
  // slots have weight 0 and index 0
  constexpr int kNnz = 8;
  int b_c[kNnz];
  T b_w[kNnz];
  int b_n = 0, b_r0 = 0, b_r1 = 0;
  if (tid < nx) {
    b_r0 = sys.b_rp[tid];
    b_r1 = sys.b_rp[tid + 1];
    b_n = b_r1 - b_r0;
  }
#pragma unroll
  for (int r = 0; r < kNnz; ++r) {
    b_c[r] = r < b_n ? sys.b_ci[b_r0 + r] : 0;
    b_w[r] = r < b_n ? sys.b_v[b_r0 + r] : T(0);
  }

  for (int k0 = 0; k0 < ch.len; k0 += kChunk) {
    const int C = ch.len - k0 < kChunk ? ch.len - k0 : kChunk;
    const int nb = ch.first + k0;
    // stage the chunk (consecutive nodes: contiguous ranges of y, y_prev,
    // du, uhat, e); every batch issues all its loads before any store
    {
      const int ny = mode == kModeSolve ? 0 : C * D;
      const int nuu = C * nu;
      const int nh = affine ? C * nu : 0;
      const int ne = affine ? C * nx : 0;
      const size_t oy = (size_t)nb * D, ou = (size_t)nb * nu, ox = (size_t)nb * nx;
      for (int b = 0; b * kStageY * kBlock < ny || b * kStageU * kBlock < nuu || b * kStageX * kBlock < C * nx;
           ++b) {
        T ry[kStageY], rp[kStageY], ru[kStageU], rh[kStageU], rx[kStageX];
        T rs = T(1), rpi = T(1);
#pragma unroll
        for (int u = 0; u < kStageY; ++u) {
          const int e = (b * kStageY + u) * kBlock + tid;
          ry[u] = e < ny ? ycur[oy + e] : T(0);
          rp[u] = (mode == kModeAPG && e < ny) ? yprv[oy + e] : T(0);
        }
#pragma unroll
        for (int u = 0; u < kStageU; ++u) {
          const int e = (b * kStageU + u) * kBlock + tid;
          ru[u] = e < nuu ? td.du[ou + e] : T(0);
          rh[u] = e < nh ? td.uhat[ou + e] : T(0);
        }
#pragma unroll
        for (int u = 0; u < kStageX; ++u) {
          const int e = (b * kStageX + u) * kBlock + tid;
          rx[u] = e < ne ? td.e[ox + e] : T(0);
        }
        if (b == 0) {
          if (tid < 3 * C && scaled) rs = td.scale[(size_t)nb * 3 + tid];
          if (tid < C) rpi = td.pi[nb + tid];
        }
#pragma unroll
        for (int u = 0; u < kStageY; ++u) {
          const int e = (b * kStageY + u) * kBlock + tid;
          if (e < ny) {
            const T y = ry[u];
            sW[e] = mode == kModeAPG ? y + c * (y - rp[u]) : in_scale * y;
          }
        }
#pragma unroll
        for (int u = 0; u < kStageU; ++u) {
          const int e = (b * kStageU + u) * kBlock + tid;
          if (e < nuu) {
            sU[e] = ru[u];
            sH[e] = rh[u];
          }
        }
#pragma unroll
        for (int u = 0; u < kStageX; ++u) {
          const int e = (b * kStageX + u) * kBlock + tid;
          if (e < C * nx) sX[e] = rx[u];
        }
        if (b == 0) {
          if (tid < 3 * C) sS[tid] = rs;
          if (tid < C) sPi[tid] = rpi;
        }
      }
    }
    __syncthreads();
    // ut recursion (top node of the chunk first)
    for (int j = tid; j < nu; j += kBlock) {
      T u = sUc[j];
      for (int cc = 0; cc < C; ++cc) {
        u += sU[cc * nu + j];
        sU[cc * nu + j] = u;
      }
      sUc[j] = u;
    }
    __syncthreads();
    // x recursion (one thread per state component; nx <= kBlock)
    if (sys.a_identity) {
      if (tid < nx) {
        const int i = tid;
        T x = sXc[i];
        for (int cc = 0; cc < C; ++cc) {
          T g = sX[cc * nx + i];
          if (b_n <= kNnz) {
#pragma unroll
            for (int r = 0; r < kNnz; ++r) g += b_w[r] * sU[cc * nu + b_c[r]];
          } else {
            for (int r = b_r0; r < b_r1; ++r) g += sys.b_v[r] * sU[cc * nu + sys.b_ci[r]];
          }
          x += g;
          sX[cc * nx + i] = x;
        }
        sXc[i] = x;
      }
    } else {
      for (int cc = 0; cc < C; ++cc) {
        for (int i = tid; i < nx; i += kBlock) {
          T x = sX[cc * nx + i];
          for (int r = sys.a_rp[i]; r < sys.a_rp[i + 1]; ++r) x += sys.a_v[r] * sXc[sys.a_ci[r]];
          for (int r = sys.b_rp[i]; r < sys.b_rp[i + 1]; ++r) x += sys.b_v[r] * sU[cc * nu + sys.b_ci[r]];
          sX[cc * nx + i] = x;
        }
        __syncthreads();
        for (int i = tid; i < nx; i += kBlock) sXc[i] = sX[cc * nx + i];
        __syncthreads();
      }
    }
    __syncthreads();

    // distance blocks: one wave per (node, block)
    for (int p = wave; p < 2 * C; p += kWaves) {  // wave-uniform loop
      const int cc = p >> 1;
      const int b = p & 1;
      const size_t n = (size_t)(nb + cc);
      const T s = sS[3 * cc + b];
      T a_[NXL], pa_[NXL], hz_[NXL];
      T dsq = T(0);
#pragma unroll
      for (int r = 0; r < NXL; ++r) {
        const int i = lane + 64 * r;
        a_[r] = pa_[r] = hz_[r] = T(0);
        if (i < nx) {
          const T hzv = sX[cc * nx + i];
          hz_[r] = hzv;
          if (write_z && b == 0) td.z[n * W + i] = hzv;
          if (mode == kModePower) {
            const T g = -s * hzv;
            ynew[n * D + b * nx + i] = g;
            st0 += (double)g * (double)g;
            st1 += (double)sW[cc * D + b * nx + i] * (double)g;
          } else if (mode == kModeAPG) {
            const T w = sW[cc * D + b * nx + i];
            const T a = (w * ilam + s * hzv) / s;
            const T pa = b == 0 ? (a > sys.xs[i] ? a : sys.xs[i]) : clampv(a, sys.xmin[i], sys.xmax[i]);
            const T dd = a - pa;
            dsq += dd * dd;
            a_[r] = a;
            pa_[r] = pa;
          }
        }
      }
      if (mode != kModeAPG) continue;
      dsq = wave_sum(dsq);
      const T del = sqrt(dsq);
      const T cb = b == 0 ? (sys.safety_by_prob ? cSx * sPi[cc] : cSx) : gam_d;
      const T tau = cb * ilam / (s * s);
#pragma unroll
      for (int r = 0; r < NXL; ++r) {
        const int i = lane + 64 * r;
        if (i < nx) {
          const T a = a_[r], pa = pa_[r];
          const T tun = del <= tau ? pa : a - (tau / del) * (a - pa);
          const T hzv = hz_[r];
          ynew[n * D + b * nx + i] = sW[cc * D + b * nx + i] + lam * (s * hzv - s * tun);
          st0 = nanmax(st0, fabs((double)hzv - (double)tun));
          st1 = nanmax(st1, fabs((double)hzv));
          st2 = nanmax(st2, fabs((double)tun));
        }
      }
    }
    // psi blocks: input box
    for (int e = tid; e < C * nu; e += kBlock) {
      const int cc = e / nu;
      const int j = e - cc * nu;
      const size_t n = (size_t)(nb + cc);
      const T u = sU[cc * nu + j] + sH[cc * nu + j];
      if (write_z) td.z[n * W + nx + j] = u;
      if (mode == kModeSolve) continue;
      const T s = sS[3 * cc + 2];
      const T w = sW[cc * D + 2 * nx + j];
      if (mode == kModePower) {
        const T g = -s * u;
        ynew[n * D + 2 * nx + j] = g;
        st0 += (double)g * (double)g;
        st1 += (double)w * (double)g;
        continue;
      }
      const T a = (w * ilam + s * u) / s;
      const T tun = clampv(a, sys.umin[j], sys.umax[j]);
      ynew[n * D + 2 * nx + j] = w + lam * (s * u - s * tun);
      st0 = nanmax(st0, fabs((double)u - (double)tun));
      st1 = nanmax(st1, fabs((double)u));
      st2 = nanmax(st2, fabs((double)tun));
    }
    __syncthreads();
  }
  // bottom node of the chain: hand x and ut to the child chains
  if (ch.child_count > 0) {
    for (int i = tid; i < nx; i += kBlock) td.cbotX[(size_t)wi.chain * nx + i] = sXc[i];
    for (int j = tid; j < nu; j += kBlock) td.cbotU[(size_t)wi.chain * nu + j] = sUc[j];
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
  if (lane == 0) {
    sRed[wave * 3 + 0] = st0;
    sRed[wave * 3 + 1] = st1;
    sRed[wave * 3 + 2] = st2;
  }
  __syncthreads();
  if (tid == 0) {
    double* out = td.cstat + (size_t)wi.chain * kStat;
    if (mode == kModeAPG) {
      double a0 = sRed[0], a1 = sRed[1], a2 = sRed[2];
      for (int w = 1; w < kBlock / 64; ++w) {
        a0 = nanmax(a0, sRed[3 * w]);
        a1 = nanmax(a1, sRed[3 * w + 1]);
        a2 = nanmax(a2, sRed[3 * w + 2]);
      }
      out[0] = a0; out[1] = a1; out[2] = a2; out[3] = 0.0;
    } else if (mode == kModePower) {
      double a0 = sRed[0], a1 = sRed[1];
      for (int w = 1; w < kBlock / 64; ++w) {
        a0 += sRed[3 * w];
        a1 += sRed[3 * w + 1];
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
// Dynamic LDS above 64 KiB needs an explicit per-kernel opt-in (gfx950 has
// 160 KiB per CU).
template <typename K>
hipError_t allow_lds(K kernel, size_t bytes) {
  if (bytes <= 64 * 1024) return hipSuccess;
  return hipFuncSetAttribute(reinterpret_cast<const void*>(kernel), hipFuncAttributeMaxDynamicSharedMemorySize,
                             (int)bytes);
}

}  // namespace

template <typename T>
hipError_t launch_backward(const SysDev<T>& sys, const TreeDev<T>* trees, const WorkItem* items, int n_items,
                           const double* ctab, int mode, hipStream_t s) {
  if (n_items <= 0) return hipSuccess;
  const size_t lds = lds_bytes_backward(sys.nx, sys.nu, sizeof(T));
  if (sys.nu <= 64) {
    hipError_t e = allow_lds(k_backward<T, 4, 16>, lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((k_backward<T, 4, 16>), dim3(n_items), dim3(kBlock), lds, s, sys, trees, items, ctab, mode);
  } else if (sys.nu <= 128) {
    hipError_t e = allow_lds(k_backward<T, 2, 64>, lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((k_backward<T, 2, 64>), dim3(n_items), dim3(kBlock), lds, s, sys, trees, items, ctab, mode);
  } else {
    return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <typename T>
hipError_t launch_forward(const SysDev<T>& sys, const TreeDev<T>* trees, const WorkItem* items, int n_items,
                          const double* ctab, int mode, hipStream_t s) {
  if (n_items <= 0) return hipSuccess;
  const size_t lds = lds_bytes_forward(sys.nx, sys.nu, sizeof(T));
  if (sys.nu > 128 || sys.nx > 128) return hipErrorInvalidValue;
  if (sys.nx <= 64) {
    hipError_t e = allow_lds(k_forward<T, 1>, lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((k_forward<T, 1>), dim3(n_items), dim3(kBlock), lds, s, sys, trees, items, ctab, mode);
  } else {
    hipError_t e = allow_lds(k_forward<T, 2>, lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((k_forward<T, 2>), dim3(n_items), dim3(kBlock), lds, s, sys, trees, items, ctab, mode);
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
