// HIP kernels of the APG iteration for scenario-tree SMPC on gfx950.
//
// One iteration of eq. apg-iteration is two kernels over the leaf chains of
// every tree of a launch (a chain is a maximal path of single-child nodes; a
// leaf chain ends at a leaf):
//
//   k_backward  extrapolation + the backward sweep of the solve step (Alg. 1,
//               first loop).  A workgroup sweeps its leaf chain, hands the
//               chain-top terms to the parent chain and counts itself done
//               there; the workgroup that completes the last child sweeps the
//               parent chain, and so on up to the root.  No workgroup waits.
//   k_forward   the forward rollout (Alg. 1, second loop) fused with the prox
//               of App. C and the dual update.  A workgroup first rebuilds the
//               states along the root path of its leaf chain (prefix sums of
//               the backward outputs) and applies the prox to the ancestor
//               nodes it is designated for (each inner node has exactly one
//               designated leaf chain), then rolls out its own chain.  The last
//               workgroup of a tree folds the float64 partials, applies the
//               stop test and advances the tree's iteration counter.
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
// B and A are applied in sparse form; P is held in registers.
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

// Values handed between workgroups of one launch (chain-top terms, reduction
// partials, counters) travel through agent-scope atomic loads and stores,
// which gfx950 keeps coherent across its XCDs without writing back or
// invalidating a whole L2 (what a device-scope fence does).
template <typename T>
__device__ __forceinline__ void st_agent(T* p, T v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

template <typename T>
__device__ __forceinline__ T ld_agent(const T* p) {
  return __hip_atomic_load(const_cast<T*>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Wait until this wave's memory operations have completed (stores
// acknowledged at the coherence point), so that a counter increment issued
// after the following barrier is seen only after them.
__device__ __forceinline__ void wait_mem() {
  __atomic_signal_fence(__ATOMIC_SEQ_CST);
  __builtin_amdgcn_s_waitcnt(0);
  __atomic_signal_fence(__ATOMIC_SEQ_CST);
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

// Loads per thread and array issued in one staging batch, before any LDS
// store (halved in float64 to leave registers for the P slice).
template <typename T>
struct Stage {
  static constexpr int Y = sizeof(T) == 4 ? 12 : 6;
  static constexpr int U = sizeof(T) == 4 ? 6 : 3;
  static constexpr int X = sizeof(T) == 4 ? 4 : 2;
};

// Sparse rows kept in registers: unused slots have weight 0 and index 0.
constexpr int kNnzBt = 4;  // B' rows: a flow touches few tanks
constexpr int kNnzB = 8;   // B rows: a tank is touched by few flows

template <typename T, int K>
struct RowCache {
  int c[K];
  T w[K];
  int n, q0, q1;
};

template <typename T, int K>
__device__ __forceinline__ void load_row(RowCache<T, K>& r, const int32_t* rp, const int32_t* ci, const T* v,
                                         int row, bool valid) {
  r.n = r.q0 = r.q1 = 0;
  if (valid) {
    r.q0 = rp[row];
    r.q1 = rp[row + 1];
    r.n = r.q1 - r.q0;
  }
#pragma unroll
  for (int q = 0; q < K; ++q) {
    r.c[q] = q < r.n ? ci[r.q0 + q] : 0;
    r.w[q] = q < r.n ? v[r.q0 + q] : T(0);
  }
}

// Per-workgroup view of one iteration of one tree.
template <typename T>
struct Iter {
  int it;
  T c, in_scale, lam, ilam;
  bool affine, scaled, write_z;
  const T* ycur;
  const T* yprv;
  T* ynew;
};

template <typename T>
__device__ __forceinline__ Iter<T> make_iter(const TreeDev<T>& td, const TreeState* st, const double* ctab,
                                             int mode) {
  Iter<T> x;
  x.it = st->iter;
  x.c = T(0);
  x.in_scale = T(1);
  x.lam = T(1);
  x.ilam = T(1);
  if (mode == kModeAPG) {
    x.c = (T)ctab[x.it];
    x.lam = (T)st->lambda;
    x.ilam = T(1) / x.lam;
  }
  if (mode == kModePower) x.in_scale = (T)st->in_scale;
  x.affine = mode != kModePower;
  x.scaled = (td.scale != nullptr) && (mode != kModeSolve);
  const bool check = (mode != kModeAPG) || ((x.it + 1) % st->check_every == 0) || (x.it + 1 >= st->max_iter);
  x.write_z = (mode == kModeSolve) || (mode == kModeAPG && check);
  x.ycur = td.y[x.it % 3];
  x.yprv = td.y[(x.it + 2) % 3];
  x.ynew = td.y[(x.it + 1) % 3];
  return x;
}

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

namespace {

// ---------------------------------------------------------------------------
// backward sweep of one chain
//
// Per chunk (bottom-up): stage w = y + c (y - y_prev) and beta of the chunk's
// nodes (consecutive in memory) with batched loads; form xi_n = S(w_sigma +
// w_zeta) and r_n = beta_n + S w_psi; run Q_n = xi_n + A' Q_below and
// rho_n = r_n + B' Q_n + rho_below as per-component scans (one thread per
// component when A = I); then du_n = -P rho_n / (2 pi_n) for the whole chunk
// with P held in registers: thread (j, h) keeps P[j][h*KH .. h*KH + KH), the
// S k-parts of a row sit in adjacent lanes and combine with lane shuffles.
// ---------------------------------------------------------------------------
template <typename T, int S, int KH>
__device__ void bwd_chain(const SysDev<T>& sys, const TreeDev<T>& td, const Iter<T>& x, int mode, int chain,
                          unsigned char* smem_raw, const T (&preg)[KH], const RowCache<T, kNnzBt>& bt) {
  constexpr int kChunk = Chunk<T>::value;
  constexpr int kStageY = Stage<T>::Y, kStageU = Stage<T>::U;
  constexpr int KP = S * KH;
  const int tid = threadIdx.x;
  const int nx = sys.nx, nu = sys.nu, D = sys.D;
  const ChainDesc ch = td.chains[chain];
  const int pj = tid / S;
  const int ph = tid % S;

  T* sW = reinterpret_cast<T*>(smem_raw + kRedDoubles * sizeof(double));  // kChunk x D
  T* sB = sW + (size_t)kChunk * D;                                        // kChunk x nu
  T* sQ = sB + (size_t)kChunk * nu;                                       // kChunk x nx
  T* sR = sQ + (size_t)kChunk * nx;  // kChunk x KP, entries nu..KP-1 stay zero
  T* sI = sR + (size_t)kChunk * KP;  // kChunk
  T* sS = sI + kChunk;               // kChunk x 3
  T* sQc = sS + 3 * kChunk;
  T* sRc = sQc + nx;

  // cost-to-go terms handed up by the child chains of the bottom node
  for (int i = tid; i < nx; i += kBlock) {
    T acc = T(0);
    for (int k = 0; k < ch.child_count; ++k) acc += ld_agent(&td.ctopQ[(size_t)(ch.child_begin + k) * nx + i]);
    sQc[i] = acc;
  }
  for (int j = tid; j < nu; j += kBlock) {
    T acc = T(0);
    for (int k = 0; k < ch.child_count; ++k) acc += ld_agent(&td.ctopR[(size_t)(ch.child_begin + k) * nu + j]);
    sRc[j] = acc;
  }
  for (int e = tid; e < kChunk * (KP - nu); e += kBlock) {
    const int cc = e / (KP - nu);
    sR[cc * KP + nu + (e - cc * (KP - nu))] = T(0);
  }

  for (int top = ch.len; top > 0; top -= kChunk) {
    const int k0 = top > kChunk ? top - kChunk : 0;
    const int C = top - k0;
    const int nb = ch.first + k0;  // internal index of the chunk's first node
    {
      const int ny = C * D;
      const int nbt = x.affine ? C * nu : 0;
      const size_t oy = (size_t)nb * D, ob = (size_t)nb * nu;
      for (int b = 0; b * kStageY * kBlock < ny || b * kStageU * kBlock < nbt; ++b) {
        T ry[kStageY], rp[kStageY], rb[kStageU];
        T rs = T(1), rpi = T(1);
#pragma unroll
        for (int u = 0; u < kStageY; ++u) {
          const int e = (b * kStageY + u) * kBlock + tid;
          ry[u] = e < ny ? x.ycur[oy + e] : T(0);
          rp[u] = (mode == kModeAPG && e < ny) ? x.yprv[oy + e] : T(0);
        }
#pragma unroll
        for (int u = 0; u < kStageU; ++u) {
          const int e = (b * kStageU + u) * kBlock + tid;
          rb[u] = e < nbt ? td.beta[ob + e] : T(0);
        }
        if (b == 0) {
          if (tid < 3 * C && x.scaled) rs = td.scale[(size_t)nb * 3 + tid];
          if (tid < C) rpi = td.pi[nb + tid];
        }
#pragma unroll
        for (int u = 0; u < kStageY; ++u) {
          const int e = (b * kStageY + u) * kBlock + tid;
          if (e < ny) {
            const T y = ry[u];
            sW[e] = mode == kModeAPG ? y + x.c * (y - rp[u]) : (mode == kModePower ? x.in_scale * y : y);
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
    // xi = S(w_sigma + w_zeta) and r = beta + S w_psi
    for (int e = tid; e < C * nx; e += kBlock) {
      const int cc = e / nx;
      const int i = e - cc * nx;
      sQ[e] = sS[3 * cc] * sW[cc * D + i] + sS[3 * cc + 1] * sW[cc * D + nx + i];
    }
    for (int e = tid; e < C * nu; e += kBlock) {
      const int cc = e / nu;
      const int j = e - cc * nu;
      sR[cc * KP + j] = (x.affine ? sB[e] : T(0)) + sS[3 * cc + 2] * sW[cc * D + 2 * nx + j];
    }
    __syncthreads();
    // Q recursion, bottom node of the chunk first
    if (sys.a_identity) {
      if (tid < nx) {
        T q = sQc[tid];
        for (int cc = C - 1; cc >= 0; --cc) {
          q += sQ[cc * nx + tid];
          sQ[cc * nx + tid] = q;
        }
        sQc[tid] = q;
      }
    } else {
      for (int cc = C - 1; cc >= 0; --cc) {
        if (tid < nx) {
          T q = sQ[cc * nx + tid];
          for (int r = sys.at_rp[tid]; r < sys.at_rp[tid + 1]; ++r) q += sys.at_v[r] * sQc[sys.at_ci[r]];
          sQ[cc * nx + tid] = q;
        }
        __syncthreads();
        if (tid < nx) sQc[tid] = sQ[cc * nx + tid];
        __syncthreads();
      }
    }
    __syncthreads();
    // rho recursion (one thread per input component)
    if (tid < nu) {
      T r = sRc[tid];
      for (int cc = C - 1; cc >= 0; --cc) {
        T g = sR[cc * KP + tid];
        if (bt.n <= kNnzBt) {
#pragma unroll
          for (int q = 0; q < kNnzBt; ++q) g += bt.w[q] * sQ[cc * nx + bt.c[q]];
        } else {
          for (int q = bt.q0; q < bt.q1; ++q) g += sys.bt_v[q] * sQ[cc * nx + sys.bt_ci[q]];
        }
        r += g;
        sR[cc * KP + tid] = r;
      }
      sRc[tid] = r;
    }
    __syncthreads();
    // du = -P rho / (2 pi): branch-free; padded entries of P and rho are zero,
    // rows cc >= C are computed from stale finite values and not stored
    T acc[kChunk];
#pragma unroll
    for (int cc = 0; cc < kChunk; ++cc) acc[cc] = T(0);
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
  for (int i = tid; i < nx; i += kBlock) st_agent(&td.ctopQ[(size_t)chain * nx + i], sQc[i]);
  for (int j = tid; j < nu; j += kBlock) st_agent(&td.ctopR[(size_t)chain * nu + j], sRc[j]);
}

template <typename T, int S, int KH>
__global__ __launch_bounds__(kBlock, 2) void k_backward(SysDev<T> sys, const TreeDev<T>* __restrict__ trees,
                                                        const WorkItem* __restrict__ items,
                                                        const double* __restrict__ ctab, int mode) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  __shared__ int s_last;
  constexpr int KP = S * KH;
  const int tid = threadIdx.x;
  const WorkItem wi = items[blockIdx.x];
  const TreeDev<T>& td = trees[wi.tree];
  const TreeState* st = td.st;
  if (st->done) return;
  const Iter<T> x = make_iter(td, st, ctab, mode);
  const int nu = sys.nu;

  // P slice of this thread (P is stored zero-padded to KP x KP)
  T preg[KH];
  {
    const int pj = tid / S;
    const int ph = tid % S;
#pragma unroll
    for (int kk = 0; kk < KH; ++kk) preg[kk] = sys.P[(size_t)(ph * KH + kk) * KP + pj];
  }
  RowCache<T, kNnzBt> bt;
  load_row(bt, sys.bt_rp, sys.bt_ci, sys.bt_v, tid, tid < nu);

  int chain = wi.chain;
  while (true) {
    bwd_chain<T, S, KH>(sys, td, x, mode, chain, smem_raw, preg, bt);
    const int parent = td.chains[chain].parent;
    if (parent < 0) break;  // the root chain is done: the sweep is complete
    // this chain's top terms are stored: count this child done at the parent
    wait_mem();
    __syncthreads();
    if (tid == 0) {
      const int pc = td.chains[parent].child_count;
      const int prev = __hip_atomic_fetch_add(&td.cnt[parent], 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      s_last = (prev == pc - 1);
      if (s_last) st_agent(&td.cnt[parent], 0);  // ready for the next iteration
    }
    __syncthreads();
    if (!s_last) break;  // a sibling is still running; it will sweep the parent
    chain = parent;
  }
}

// ---------------------------------------------------------------------------
// forward rollout and prox of consecutive nodes [first, first + len)
//
// The carries sXc / sUc hold the state x and input increment ut of the node
// above.  With do_prox the nodes' prox, dual update and primal output are
// computed; otherwise only the recursion runs (an ancestor another leaf chain
// owns).  Per chunk: stage w, du, uhat, e (consecutive nodes: contiguous
// ranges) with batched loads, run ut_n = ut_above + du_n and
// x_n = A x_above + B ut_n + e_n as per-component scans, then the prox: each
// (node, sigma|zeta) block is one wave with its Euclidean norm reduced by lane
// shuffles, the psi entries are spread over all threads.
// ---------------------------------------------------------------------------
template <typename T, int NXL>
__device__ void fwd_segment(const SysDev<T>& sys, const TreeDev<T>& td, const Iter<T>& x, int mode, int first,
                            int len, bool do_prox, unsigned char* smem_raw, const RowCache<T, kNnzB>& brow,
                            double& st0, double& st1, double& st2) {
  constexpr int kChunk = Chunk<T>::value;
  constexpr int kStageY = Stage<T>::Y, kStageU = Stage<T>::U, kStageX = Stage<T>::X;
  constexpr int kWaves = kBlock / 64;
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int nx = sys.nx, nu = sys.nu, D = sys.D;
  const int W = nx + nu;
  const T cSx = (T)sys.W_x;
  const T gam_d = (T)sys.gamma_d;
  const bool prox = do_prox && mode != kModeSolve;

  T* sW = reinterpret_cast<T*>(smem_raw + kRedDoubles * sizeof(double));  // kChunk x D
  T* sU = sW + (size_t)kChunk * D;                                        // kChunk x nu
  T* sH = sU + (size_t)kChunk * nu;                                       // kChunk x nu (uhat)
  T* sX = sH + (size_t)kChunk * nu;                                       // kChunk x nx
  T* sPi = sX + (size_t)kChunk * nx;                                      // kChunk
  T* sS = sPi + kChunk;                                                   // kChunk x 3
  T* sUc = sS + 3 * kChunk;
  T* sXc = sUc + nu;

  for (int k0 = 0; k0 < len; k0 += kChunk) {
    const int C = len - k0 < kChunk ? len - k0 : kChunk;
    const int nb = first + k0;
    {
      const int ny = prox ? C * D : 0;
      const int nuu = C * nu;
      const int nh = (x.affine && do_prox) ? C * nu : 0;
      const int ne = x.affine ? C * nx : 0;
      const size_t oy = (size_t)nb * D, ou = (size_t)nb * nu, ox = (size_t)nb * nx;
      for (int b = 0; b * kStageY * kBlock < ny || b * kStageU * kBlock < nuu || b * kStageX * kBlock < C * nx;
           ++b) {
        T ry[kStageY], rp[kStageY], ru[kStageU], rh[kStageU], rx[kStageX];
        T rs = T(1), rpi = T(1);
#pragma unroll
        for (int u = 0; u < kStageY; ++u) {
          const int e = (b * kStageY + u) * kBlock + tid;
          ry[u] = e < ny ? x.ycur[oy + e] : T(0);
          rp[u] = (mode == kModeAPG && e < ny) ? x.yprv[oy + e] : T(0);
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
        if (b == 0 && prox) {
          if (tid < 3 * C && x.scaled) rs = td.scale[(size_t)nb * 3 + tid];
          if (tid < C) rpi = td.pi[nb + tid];
        }
#pragma unroll
        for (int u = 0; u < kStageY; ++u) {
          const int e = (b * kStageY + u) * kBlock + tid;
          if (e < ny) {
            const T y = ry[u];
            sW[e] = mode == kModeAPG ? y + x.c * (y - rp[u]) : x.in_scale * y;
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
    if (tid < nu) {
      T u = sUc[tid];
      for (int cc = 0; cc < C; ++cc) {
        u += sU[cc * nu + tid];
        sU[cc * nu + tid] = u;
      }
      sUc[tid] = u;
    }
    __syncthreads();
    // x recursion
    if (sys.a_identity) {
      if (tid < nx) {
        T xv = sXc[tid];
        for (int cc = 0; cc < C; ++cc) {
          T g = sX[cc * nx + tid];
          if (brow.n <= kNnzB) {
#pragma unroll
            for (int r = 0; r < kNnzB; ++r) g += brow.w[r] * sU[cc * nu + brow.c[r]];
          } else {
            for (int r = brow.q0; r < brow.q1; ++r) g += sys.b_v[r] * sU[cc * nu + sys.b_ci[r]];
          }
          xv += g;
          sX[cc * nx + tid] = xv;
        }
        sXc[tid] = xv;
      }
    } else {
      for (int cc = 0; cc < C; ++cc) {
        if (tid < nx) {
          T xv = sX[cc * nx + tid];
          for (int r = sys.a_rp[tid]; r < sys.a_rp[tid + 1]; ++r) xv += sys.a_v[r] * sXc[sys.a_ci[r]];
          for (int r = sys.b_rp[tid]; r < sys.b_rp[tid + 1]; ++r) xv += sys.b_v[r] * sU[cc * nu + sys.b_ci[r]];
          sX[cc * nx + tid] = xv;
        }
        __syncthreads();
        if (tid < nx) sXc[tid] = sX[cc * nx + tid];
        __syncthreads();
      }
    }
    __syncthreads();

    if (do_prox) {
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
            if (x.write_z && b == 0) td.z[n * W + i] = hzv;
            if (mode == kModePower) {
              const T g = -s * hzv;
              x.ynew[n * D + b * nx + i] = g;
              st0 += (double)g * (double)g;
              st1 += (double)sW[cc * D + b * nx + i] * (double)g;
            } else if (mode == kModeAPG) {
              const T w = sW[cc * D + b * nx + i];
              const T a = (w * x.ilam + s * hzv) / s;
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
        const T tau = cb * x.ilam / (s * s);
#pragma unroll
        for (int r = 0; r < NXL; ++r) {
          const int i = lane + 64 * r;
          if (i < nx) {
            const T a = a_[r], pa = pa_[r];
            const T tun = del <= tau ? pa : a - (tau / del) * (a - pa);
            const T hzv = hz_[r];
            x.ynew[n * D + b * nx + i] = sW[cc * D + b * nx + i] + x.lam * (s * hzv - s * tun);
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
        if (x.write_z) td.z[n * W + nx + j] = u;
        if (mode == kModeSolve) continue;
        const T s = sS[3 * cc + 2];
        const T w = sW[cc * D + 2 * nx + j];
        if (mode == kModePower) {
          const T g = -s * u;
          x.ynew[n * D + 2 * nx + j] = g;
          st0 += (double)g * (double)g;
          st1 += (double)w * (double)g;
          continue;
        }
        const T a = (w * x.ilam + s * u) / s;
        const T tun = clampv(a, sys.umin[j], sys.umax[j]);
        x.ynew[n * D + 2 * nx + j] = w + x.lam * (s * u - s * tun);
        st0 = nanmax(st0, fabs((double)u - (double)tun));
        st1 = nanmax(st1, fabs((double)u));
        st2 = nanmax(st2, fabs((double)tun));
      }
    }
    __syncthreads();
  }
}

template <typename T, int NXL>
__global__ __launch_bounds__(kBlock, 2) void k_forward(SysDev<T> sys, const TreeDev<T>* __restrict__ trees,
                                                       const WorkItem* __restrict__ items,
                                                       const double* __restrict__ ctab, int mode,
                                                       int32_t* __restrict__ done_out) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  __shared__ int s_last;
  double* sRed = reinterpret_cast<double*>(smem_raw);
  constexpr int kChunk = Chunk<T>::value;
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const WorkItem wi = items[blockIdx.x];
  const TreeDev<T>& td = trees[wi.tree];
  TreeState* st = td.st;
  if (st->done) {
    if (tid == 0) done_out[wi.tree] = 1;
    return;
  }
  const Iter<T> x = make_iter(td, st, ctab, mode);
  const int nx = sys.nx, nu = sys.nu, D = sys.D;
  RowCache<T, kNnzB> brow;
  load_row(brow, sys.b_rp, sys.b_ci, sys.b_v, tid, tid < nx);

  T* sUc = reinterpret_cast<T*>(smem_raw + kRedDoubles * sizeof(double)) +
           (size_t)kChunk * (D + 2 * nu + nx + 4);
  T* sXc = sUc + nu;
  for (int i = tid; i < nx; i += kBlock) sXc[i] = x.affine ? td.p[i] : T(0);
  for (int j = tid; j < nu; j += kBlock) sUc[j] = T(0);
  __syncthreads();

  double st0 = 0.0, st1 = 0.0, st2 = 0.0;  // residual / |Hz| / |t| maxima, or power sums
  // the root path: ancestors of this leaf chain, root first
  const int p0 = td.path_off[wi.chain], p1 = td.path_off[wi.chain + 1];
  for (int q = p0; q < p1; ++q) {
    const int code = td.path[q];
    const bool own = code < 0;
    const ChainDesc ac = td.chains[own ? -1 - code : code];
    fwd_segment<T, NXL>(sys, td, x, mode, ac.first, ac.len, own, smem_raw, brow, st0, st1, st2);
  }
  const ChainDesc ch = td.chains[wi.chain];
  fwd_segment<T, NXL>(sys, td, x, mode, ch.first, ch.len, true, smem_raw, brow, st0, st1, st2);

  // partials of this leaf chain
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
    double a0 = sRed[0], a1 = sRed[1], a2 = sRed[2];
    for (int w = 1; w < kBlock / 64; ++w) {
      if (mode == kModeAPG) {
        a0 = nanmax(a0, sRed[3 * w]);
        a1 = nanmax(a1, sRed[3 * w + 1]);
        a2 = nanmax(a2, sRed[3 * w + 2]);
      } else {
        a0 += sRed[3 * w];
        a1 += sRed[3 * w + 1];
      }
    }
    st_agent(&out[0], a0);
    st_agent(&out[1], a1);
    st_agent(&out[2], a2);
    st_agent(&out[3], 0.0);
  }
  if (mode == kModeSolve) return;

  // the last leaf chain of the tree to finish ends the tree's iteration
  wait_mem();
  __syncthreads();
  if (tid == 0) {
    const int prev = __hip_atomic_fetch_add(&st->fwd_count, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    s_last = (prev == td.n_leaves - 1);
  }
  __syncthreads();
  if (!s_last || wave != 0) return;
  const int it = x.it;
  if (mode == kModeAPG) {
    const bool check = ((it + 1) % st->check_every == 0) || (it + 1 >= st->max_iter);
    int done = 0;
    if (check) {
      double rm = 0.0, hm = 0.0;
      for (int k = lane; k < td.n_leaves; k += 64) {
        const double* cs = td.cstat + (size_t)td.leaves[k] * kStat;
        rm = nanmax(rm, ld_agent(&cs[0]));
        hm = nanmax(hm, ld_agent(&cs[1]));
        hm = nanmax(hm, ld_agent(&cs[2]));
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
      st_agent(&st->fwd_count, 0);
      st->iter = it + 1;
      done_out[wi.tree] = done;
    }
  } else {  // power iteration: Rayleigh quotient and normalisation
    double gg = 0.0, wg = 0.0;
    for (int k = lane; k < td.n_leaves; k += 64) {
      const double* cs = td.cstat + (size_t)td.leaves[k] * kStat;
      gg += ld_agent(&cs[0]);
      wg += ld_agent(&cs[1]);
    }
    gg = wave_sum(gg);
    wg = wave_sum(wg);
    if (lane == 0) {
      st->lmax_est = wg;
      st->in_scale = gg > 0.0 ? 1.0 / sqrt(gg) : 0.0;
      st_agent(&st->fwd_count, 0);
      st->iter = it + 1;
      done_out[wi.tree] = 0;
    }
  }
}

template <typename T>
__global__ void k_widen(const T* __restrict__ src, double* __restrict__ dst, size_t n) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) dst[i] = (double)src[i];
}

// Dynamic LDS above 64 KiB needs an explicit per-kernel opt-in (gfx950 has
// 160 KiB per CU).
template <typename K>
hipError_t allow_lds(K kernel, size_t bytes) {
  if (bytes <= 64 * 1024) return hipSuccess;
  return hipFuncSetAttribute(reinterpret_cast<const void*>(kernel), hipFuncAttributeMaxDynamicSharedMemorySize,
                             (int)bytes);
}

}  // namespace

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
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
                          const double* ctab, int mode, int32_t* done_out, hipStream_t s) {
  if (n_items <= 0) return hipSuccess;
  const size_t lds = lds_bytes_forward(sys.nx, sys.nu, sizeof(T));
  if (sys.nu > 128 || sys.nx > 128) return hipErrorInvalidValue;
  if (sys.nx <= 64) {
    hipError_t e = allow_lds(k_forward<T, 1>, lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((k_forward<T, 1>), dim3(n_items), dim3(kBlock), lds, s, sys, trees, items, ctab, mode,
                       done_out);
  } else {
    hipError_t e = allow_lds(k_forward<T, 2>, lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((k_forward<T, 2>), dim3(n_items), dim3(kBlock), lds, s, sys, trees, items, ctab, mode,
                       done_out);
  }
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
                                           const double*, int, int32_t*, hipStream_t);
template hipError_t launch_forward<float>(const SysDev<float>&, const TreeDev<float>*, const WorkItem*, int,
                                          const double*, int, int32_t*, hipStream_t);
template hipError_t launch_widen<float>(const float*, double*, size_t, hipStream_t);

}  // namespace smpc
