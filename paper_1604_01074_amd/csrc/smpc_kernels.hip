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
// The library builds this file once (SMPC_KERNEL_PART undefined, every
// instantiation) or three times in parallel: part 1 holds the float64 kernels
// and the precision-conversion helpers, part 2 the float32 kernels, part 3
// the float32 solve steps on a float64 dual.
#include "smpc_internal.h"

#ifndef SMPC_KERNEL_PART
#define SMPC_KERNEL_PART 0
#endif

#include <algorithm>
#include <map>
#include <mutex>
#include <tuple>
#include <type_traits>

namespace smpc {

namespace {

// Pointers read from the tree and system tables are generic; accesses through
// them compile to FLAT instructions, whose completion the hardware counts
// with the LDS counter as well (a wait for LDS data would also wait for
// outstanding HBM loads).  Every device array lives in global memory, so the
// kernels access it through address-space-1 pointers.
// (The host compilation pass never runs these functions; there the alias is
// the plain type.)
#if defined(__HIP_DEVICE_COMPILE__)
template <typename T>
using G = __attribute__((address_space(1))) T;
#else
template <typename T>
using G = T;
#endif

template <typename T>
__device__ __forceinline__ G<T>* gp(T* p) {
  return (G<T>*)p;
}

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
  __hip_atomic_store(gp(p), v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

template <typename T>
__device__ __forceinline__ T ld_agent(const T* p) {
  return __hip_atomic_load(gp(const_cast<T*>(p)), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Wait until this wave's memory operations have completed (stores
// acknowledged at the coherence point), so that a counter increment issued
// after the following barrier is seen only after them.
__device__ __forceinline__ void wait_mem() {
  __atomic_signal_fence(__ATOMIC_SEQ_CST);
  __builtin_amdgcn_s_waitcnt(0);
  __atomic_signal_fence(__ATOMIC_SEQ_CST);
}


// ---------------------------------------------------------------------------
// Work layout.  A workgroup is four wave64s with fixed roles:
//
//   wave 0      state components i = lane + 64 r (r < NXL): Q in the backward
//               sweep, x and the sigma~ blocks in the forward rollout
//   wave 1      idle in the backward scans; x and the zeta~ blocks forward
//   waves 2, 3  input components j = threadIdx.x - 128: rho backward, ut, u
//               and the psi~ blocks forward
//
// A chain is processed in chunks of consecutive nodes.  Each thread keeps its
// component's values for every node of the chunk in registers, so the
// recursions along the chain are running sums in registers; LDS only carries
// what crosses components (Q for B'Q, ut for B ut, rho for the P product).
// ---------------------------------------------------------------------------

// Chunk lengths are template parameters (CH): nodes per backward chunk (the
// P product of a chunk is CH / 16 MFMA row tiles) and nodes per forward chunk
// (register arrays of this length per thread).  The launchers accept the
// lengths listed in chunk_supported; the host picks one per launch plan.

// 16x16x4 matrix-core products.  Operand layouts (both precisions): lane l
// holds A[l % 16][l / 16] and B[l / 16][l % 16]; the four accumulator values
// of lane l are D[row(l, r)][l % 16], r = 0..3.
template <typename T>
struct Mfma;

template <>
struct Mfma<double> {
  typedef double v4 __attribute__((ext_vector_type(4)));
  static __device__ __forceinline__ v4 op(double a, double b, v4 c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int row(int lane, int r) { return (lane >> 4) + 4 * r; }
};

template <>
struct Mfma<float> {
  typedef float v4 __attribute__((ext_vector_type(4)));
  static __device__ __forceinline__ v4 op(float a, float b, v4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int row(int lane, int r) { return 4 * (lane >> 4) + r; }
};

// Sparse rows kept in registers: unused slots have weight 0 and index 0;
// longer rows are read from the CSR arrays.
constexpr int kNnzBt = 4;  // B' rows: a flow touches few tanks
constexpr int kNnzB = 8;   // B rows: a tank is touched by few flows

// Nodes whose loads may be in flight together in the backward staging: the
// scheduler may not hoist later loads above each batch (with P in registers
// that would spill).
constexpr int kLoadBatch = 8;
// The longest chain whose P product runs on the VALU instead of the matrix
// cores (a 16-row MFMA tile costs the same for one row as for sixteen).
constexpr int kValuChain = 4;

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
    r.q0 = gp(rp)[row];
    r.q1 = gp(rp)[row + 1];
    r.n = r.q1 - r.q0;
  }
#pragma unroll
  for (int q = 0; q < K; ++q) {
    r.c[q] = q < r.n ? gp(ci)[r.q0 + q] : 0;
    r.w[q] = q < r.n ? gp(v)[r.q0 + q] : T(0);
  }
}

// DPP moves within rows of 16 lanes (gfx9 encodings).
constexpr int kDppQuadSwap1 = 0xB1;  // quad_perm [1, 0, 3, 2]
constexpr int kDppQuadSwap2 = 0x4E;  // quad_perm [2, 3, 0, 1]
constexpr int kDppRowMirror = 0x140;      // lane i of a row takes lane 15 - i
constexpr int kDppRowHalfMirror = 0x141;  // lane i of a half row takes lane 7 - i

template <int CTRL>
__device__ __forceinline__ float dpp_mov(float v) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, 0xF, 0xF, false));
}

template <int CTRL>
__device__ __forceinline__ double dpp_mov(double v) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)(b & 0xffffffffLL), CTRL, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), CTRL, 0xF, 0xF, false);
  return __longlong_as_double(((long long)hi << 32) | (long long)(unsigned)lo);
}

// v plus the value of the partner lane 16 (HALF: 32) lanes away, for v equal
// in all lanes of each row (HALF: each half wave): v_permlane16_swap hands
// each row of one copy the value of the partner row, so the two copies'
// sum holds the same two addends, in the same order, in every lane.
template <bool HALF>
__device__ __forceinline__ float add_partner(float v) {
  const unsigned u = __float_as_uint(v);
  if constexpr (HALF) {
    const auto p = __builtin_amdgcn_permlane32_swap(u, u, false, false);
    return __uint_as_float(p[0]) + __uint_as_float(p[1]);
  } else {
    const auto p = __builtin_amdgcn_permlane16_swap(u, u, false, false);
    return __uint_as_float(p[0]) + __uint_as_float(p[1]);
  }
}

template <bool HALF>
__device__ __forceinline__ double add_partner(double v) {
  const unsigned long long b = (unsigned long long)__double_as_longlong(v);
  const unsigned lo = (unsigned)b, hi = (unsigned)(b >> 32);
  auto join = [](unsigned h, unsigned l) {
    return __longlong_as_double((long long)(((unsigned long long)h << 32) | l));
  };
  if constexpr (HALF) {
    const auto pl = __builtin_amdgcn_permlane32_swap(lo, lo, false, false);
    const auto ph = __builtin_amdgcn_permlane32_swap(hi, hi, false, false);
    return join(ph[0], pl[0]) + join(ph[1], pl[1]);
  } else {
    const auto pl = __builtin_amdgcn_permlane16_swap(lo, lo, false, false);
    const auto ph = __builtin_amdgcn_permlane16_swap(hi, hi, false, false);
    return join(ph[0], pl[0]) + join(ph[1], pl[1]);
  }
}

// Sums over the 64 lanes of a wave of N values at once, each returned to
// every lane; every lane must be active.  Each step adds two copies of the
// same partial sum (xor partners within quads, mirrored quads within half
// rows, mirrored half rows within rows, then partner rows and halves), so
// every lane holds the same bits at every step.  The N sums are independent
// and each step is taken for all of them before the next, so that their
// latencies overlap.
template <typename T, int N>
__device__ __forceinline__ void wave_allsum(T (&v)[N]) {
#pragma unroll
  for (int i = 0; i < N; ++i) v[i] += dpp_mov<kDppQuadSwap1>(v[i]);
#pragma unroll
  for (int i = 0; i < N; ++i) v[i] += dpp_mov<kDppQuadSwap2>(v[i]);
#pragma unroll
  for (int i = 0; i < N; ++i) v[i] += dpp_mov<kDppRowHalfMirror>(v[i]);
#pragma unroll
  for (int i = 0; i < N; ++i) v[i] += dpp_mov<kDppRowMirror>(v[i]);
#pragma unroll
  for (int i = 0; i < N; ++i) v[i] = add_partner<false>(v[i]);
#pragma unroll
  for (int i = 0; i < N; ++i) v[i] = add_partner<true>(v[i]);
}

// 1/sqrt(v) for finite v > 0: the hardware estimate refined by Newton steps
// on y^-2 = v, each of which doubles the correct bits (two in float64, one in
// float32).  v = 0 gives a NaN; callers select around it.
__device__ __forceinline__ double rsqrt_refined(double v) {
  double y = __builtin_amdgcn_rsq(v);
#pragma unroll
  for (int s = 0; s < 2; ++s) {
    const double e = __builtin_fma(-v * y, y, 1.0);
    y = __builtin_fma(0.5 * y, e, y);
  }
  return y;
}

__device__ __forceinline__ float rsqrt_refined(float v) {
  const float y = __builtin_amdgcn_rsqf(v);
  const float e = __builtin_fmaf(-v * y, y, 1.0f);
  return __builtin_fmaf(0.5f * y, e, y);
}

// Per-workgroup view of one iteration of one tree.  T is the precision of
// the solve step, Y that of the dual iterates: the extrapolation, the prox
// and the dual update run in Y (Y = T, or float solve steps on a float64
// dual).
template <typename T, typename Y>
struct Iter {
  int it;
  Y c, lam, ilam;
  T in_scale;
  bool affine, scaled, write_z;
  const G<Y>* ycur;
  const G<Y>* yprv;
  G<Y>* ynew;
};

template <typename T, typename Y>
__device__ __forceinline__ Iter<T, Y> make_iter_at(const TreeDev<T, Y>& td, const G<TreeState>* st,
                                                   const double* ctab, int mode, int it) {
  Iter<T, Y> x;
  x.it = it;
  x.c = Y(0);
  x.in_scale = T(1);
  x.lam = Y(1);
  x.ilam = Y(1);
  if (mode == kModeAPG) {
    x.c = (Y)gp(ctab)[x.it];
    x.lam = (Y)st->lambda;
    x.ilam = Y(1) / x.lam;
  }
  if (mode == kModePower) x.in_scale = (T)st->in_scale;
  x.affine = mode != kModePower;
  x.scaled = mode != kModeSolve;  // an unscaled tree holds ones
  const bool check = (mode != kModeAPG) || ((x.it + 1) % st->check_every == 0) || (x.it + 1 >= st->max_iter);
  x.write_z = (mode == kModeSolve) || (mode == kModeAPG && check);
  x.ycur = gp(td.y[x.it % 3]);
  x.yprv = gp(td.y[(x.it + 2) % 3]);
  x.ynew = gp(td.y[(x.it + 1) % 3]);
  return x;
}

template <typename T, typename Y>
__device__ __forceinline__ Iter<T, Y> make_iter(const TreeDev<T, Y>& td, const G<TreeState>* st, const double* ctab,
                                                int mode) {
  return make_iter_at(td, st, ctab, mode, (int)st->iter);
}

// The arithmetic that forms the solve step's inputs from the dual iterates,
// fixed so that every code path gives the same bits: the extrapolation is
// one fused multiply-add, and the scaled dual point is rounded on its own
// (never fused into the sum that follows).
__device__ __forceinline__ double fmadd(double a, double b, double c) { return __builtin_fma(a, b, c); }
__device__ __forceinline__ float fmadd(float a, float b, float c) { return __builtin_fmaf(a, b, c); }

template <typename Y>
__device__ __forceinline__ Y extrapolate(Y y, Y y_prev, Y c) {
  return fmadd(c, y - y_prev, y);
}

template <typename T, typename Y>
__device__ __forceinline__ T scaled(T s, Y w) {
#pragma clang fp contract(off)
  return (T)((Y)s * w);
}

template <typename T, typename Y>
__device__ __forceinline__ T beta_plus_scaled(T beta, T s, Y w) {
#pragma clang fp contract(off)
  return beta + (T)((Y)s * w);
}

// The dual point the solve step is evaluated at: the extrapolated
// w = y + c (y - y_prev) (APG), the normalised power-iteration vector, or y.
template <typename T, typename Y, bool AG = false>
__device__ __forceinline__ Y wpoint(const Iter<T, Y>& x, int mode, uint32_t k) {
  // AG: y^nu was written in this launch by another workgroup (an inner node
  // of the fused iteration), so it is read at device scope
  const Y y = AG ? __hip_atomic_load(&x.ycur[k], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) : x.ycur[k];
  if (mode == kModeAPG) return extrapolate(y, x.yprv[k], x.c);
  if (mode == kModePower) return x.in_scale * y;
  return y;
}

}  // namespace

namespace {

// ---------------------------------------------------------------------------
// backward sweep of one chain
//
// Per chunk (bottom-up): wave 0 forms xi_n = S(w_sigma + w_zeta) for its
// state components and runs Q_n = xi_n + A' Q_below (a running sum when
// A = I) into LDS; waves 2-3 form r_n = beta_n + S w_psi; after a barrier
// they add B' Q_n and run rho_n = r_n + rho_below into LDS (transposed);
// after a second barrier all four waves compute du_n = -P rho_n / (2 pi_n) for
// the chunk as one GEMM on the matrix cores (P, symmetric, is the B operand
// held in registers: wave w owns columns [16 NT w, 16 NT (w + 1)) of every
// 4-row K step).
// ---------------------------------------------------------------------------
// stashed: the forward half of this launch has left the chain's xi, r and
// -1/(2 pi) in LDS (a leaf chain of at most CH nodes; see Stash), so the
// loads are skipped.  pcnt: the parent chain's count of swept children (null
// for the root chain) and pkids its number of children; the chain counts
// itself done there once its top terms are stored, before the last chunk's
// P product, and s_last tells (after a barrier) whether it was the last.
template <typename T, typename Y, int KP, int NXL, int CH, bool AG>
__device__ __forceinline__ void bwd_chain(const SysDev<T>& sys, const TreeDev<T, Y>& td, const Iter<T, Y>& x, int mode, int chain,
                          const ChainDesc ch, unsigned char* smem_raw, const T (&preg)[KP / 4 * (KP / 64)],
                          const RowCache<T, kNnzBt>& bt, int& par, bool stashed, int* pcnt, int pkids,
                          int& s_last) {
  constexpr int RS = CH + 1;  // row stride of the transposed rho (bank spread)
  constexpr int NT = KP / 64, KS = KP / 4, MT = CH / 16;
  constexpr int XS = 64 * NXL;  // row stride of the Q parts (>= nx, a constant)
  typedef typename Mfma<T>::v4 v4;
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int nx = sys.nx, nu = sys.nu, D = sys.D;
  const int j = tid - 128;
  const bool ju = wave >= 2 && j < nu;

  T* sQ = reinterpret_cast<T*>(smem_raw);  // 2 x CH x XS: Q parts of waves 0, 1
  T* sRt = sQ + 2 * CH * XS;               // KP x RS: sRt[j * RS + cc]; rows nu..KP-1 zero
  T* sI = sRt + (size_t)KP * RS;           // 2 x CH
  T* sQc = sI + 2 * CH;                    // 2 x nx: carries (general A)
  T* sTop = sQc + 2 * nx;                  // nx: wave 1's carry at the chain top

  // Q is linear in xi = S_sigma w_sigma + S_zeta w_zeta: wave 0 runs the
  // recursion on the sigma~ part plus the children's terms, wave 1 on the
  // zeta~ part; B' Q reads both.  Cost-to-go terms handed up by the child
  // chains: all loads of a batch are issued before the (ordered) sum.
  const int nch = ch.child_count;
  T qc[NXL], rc = T(0);
#pragma unroll
  for (int r = 0; r < NXL; ++r) qc[r] = T(0);
  if (wave == 0) {
#pragma unroll
    for (int r = 0; r < NXL; ++r) {
      const int i = lane + 64 * r;
      if (i < nx) {
        for (int k0 = 0; k0 < nch; k0 += 8) {
          T v[8];
#pragma unroll
          for (int k = 0; k < 8; ++k)
            v[k] = k0 + k < nch ? ld_agent(&td.ctopQ[(size_t)(ch.child_begin + k0 + k) * nx + i]) : T(0);
#pragma unroll
          for (int k = 0; k < 8; ++k)
            if (k0 + k < nch) qc[r] += v[k];
        }
      }
    }
  } else if (ju) {
    for (int k0 = 0; k0 < nch; k0 += 8) {
      T v[8];
#pragma unroll
      for (int k = 0; k < 8; ++k)
        v[k] = k0 + k < nch ? ld_agent(&td.ctopR[(size_t)(ch.child_begin + k0 + k) * nu + j]) : T(0);
#pragma unroll
      for (int k = 0; k < 8; ++k)
        if (k0 + k < nch) rc += v[k];
    }
  }

  for (int top = ch.len; top > 0; top -= CH) {
    const int k0 = top > CH ? top - CH : 0;
    const int C = top - k0;
    const int nb = ch.first + k0;  // internal index of the chunk's first node
    T* sIp = sI + par * CH;
    if (!stashed && tid < C) sIp[tid] = T(-0.5) / gp(td.pi)[nb + tid];
    if (wave < 2) {
      // this wave's part of xi_n (block b = wave); with A = I the Q recursion
      // runs along, bottom node first
      const int b = wave;
      T* sQw = sQ + wave * CH * XS;
      if (stashed) {
        // the raw xi parts are in place: with A = I the running sum over
        // them (the general-A recursion below reads them as they are), the
        // reads of a batch of nodes issued together
        if (sys.a_identity) {
#pragma unroll
          for (int r = 0; r < NXL; ++r) {
            const int i = lane + 64 * r;
            if (i < nx)
              for (int g = C - 1; g >= 0; g -= kLoadBatch) {
                T xi[kLoadBatch];
#pragma unroll
                for (int k = 0; k < kLoadBatch; ++k) xi[k] = sQw[(g - k >= 0 ? g - k : 0) * XS + i];
#pragma unroll
                for (int k = 0; k < kLoadBatch; ++k)
                  if (g - k >= 0) {
                    qc[r] += xi[k];
                    sQw[(g - k) * XS + i] = qc[r];
                  }
              }
          }
        }
      } else {
#pragma unroll
        for (int r = 0; r < NXL; ++r) {
          const int i = lane + 64 * r;
          const uint32_t ic = (uint32_t)(i < nx ? i : 0);
#pragma unroll
          for (int g = CH - kLoadBatch; g >= 0; g -= kLoadBatch) {
            if (g >= C) continue;  // wave-uniform: the batch lies past the chunk's end
            // every load of the batch first, unconditionally (nodes past the
            // chunk's end read its last node, lanes past nx component 0), so
            // that they are in flight together; then the recursion
            T xi[kLoadBatch];
#pragma unroll
            for (int k = kLoadBatch - 1; k >= 0; --k) {
              const uint32_t n = (uint32_t)(nb + (g + k < C ? g + k : C - 1));
              const T sb = x.scaled ? gp(td.scale)[n * 3 + b] : T(1);
              xi[k] = scaled<T, Y>(sb, wpoint<T, Y, AG>(x, mode, n * D + b * nx + ic));
            }
#pragma unroll
            for (int k = kLoadBatch - 1; k >= 0; --k) {
              const int cc = g + k;
              if (cc < C && i < nx) {
                if (sys.a_identity) {
                  qc[r] += xi[k];
                  sQw[cc * XS + i] = qc[r];
                } else {
                  sQw[cc * XS + i] = xi[k];
                }
              }
            }
            __builtin_amdgcn_sched_barrier(0);
          }
        }
      }
      if (!sys.a_identity) {
        // Q_n = xi_n + A' Q_below one node at a time; the carry is exchanged
        // through LDS within this wave
        T* cq = sQc + (size_t)wave * nx;
#pragma unroll
        for (int r = 0; r < NXL; ++r)
          if (lane + 64 * r < nx) cq[lane + 64 * r] = qc[r];
        for (int cc = C - 1; cc >= 0; --cc) {
          __builtin_amdgcn_wave_barrier();
          T q[NXL];
#pragma unroll
          for (int r = 0; r < NXL; ++r) {
            const int i = lane + 64 * r;
            q[r] = T(0);
            if (i < nx) {
              q[r] = sQw[cc * XS + i];
              for (int k = gp(sys.at_rp)[i]; k < gp(sys.at_rp)[i + 1]; ++k) q[r] += gp(sys.at_v)[k] * cq[gp(sys.at_ci)[k]];
            }
          }
          __builtin_amdgcn_wave_barrier();
#pragma unroll
          for (int r = 0; r < NXL; ++r) {
            const int i = lane + 64 * r;
            if (i < nx) {
              sQw[cc * XS + i] = q[r];
              cq[i] = q[r];
              qc[r] = q[r];
            }
          }
        }
      }
    }
    if (ju && !stashed) {
      // r_n = beta_n + S w_psi, parked in this thread's row of the rho tile;
      // loads batched as above
#pragma unroll
      for (int g = 0; g < CH; g += kLoadBatch) {
        if (g >= C) break;  // wave-uniform
        T rv[kLoadBatch];
#pragma unroll
        for (int k = 0; k < kLoadBatch; ++k) {
          const uint32_t n = (uint32_t)(nb + (g + k < C ? g + k : C - 1));
          const T s2 = x.scaled ? gp(td.scale)[n * 3 + 2] : T(1);
          rv[k] = beta_plus_scaled<T, Y>(x.affine ? gp(td.beta)[n * nu + j] : T(0), s2,
                                         wpoint<T, Y, AG>(x, mode, n * D + 2 * nx + j));
        }
#pragma unroll
        for (int k = 0; k < kLoadBatch; ++k)
          if (g + k < C) sRt[j * RS + g + k] = rv[k];
        __builtin_amdgcn_sched_barrier(0);
      }
    }
    if (k0 == 0 && wave == 1) {
      // the chain's top node: wave 1's part of Q for wave 0 to hand up
#pragma unroll
      for (int r = 0; r < NXL; ++r)
        if (lane + 64 * r < nx) sTop[lane + 64 * r] = qc[r];
    }
    __syncthreads();  // Q parts complete
    // the last chunk holds the chain's top node: Q (both parts) goes up to
    // the parent chain now, rho right after its recursion, so that both
    // stores drain while the sweep goes on
    if (k0 == 0 && wave == 0) {
#pragma unroll
      for (int r = 0; r < NXL; ++r)
        if (lane + 64 * r < nx)
          st_agent(&td.ctopQ[(size_t)chain * nx + lane + 64 * r], qc[r] + sTop[lane + 64 * r]);
    }
    if (ju) {
      // rho recursion, bottom node first: r_n + B' Q_n + rho_below.  The
      // terms r_n + B' Q_n of a group of nodes are formed first, in one
      // branch-free block (a group reaching past the chunk's top reads node
      // 0 again and discards it), so that their LDS reads overlap; then the
      // running sum.  A lane whose B' row exceeds the register cache sends
      // the wave through the CSR arrays.
      const T* sQz = sQ + CH * XS;
      if (!__any(bt.n > kNnzBt)) {
        constexpr int RG = (sizeof(T) == 8 && NXL > 1) ? 1 : 2;  // as registers allow beside P
        for (int hi = C; hi > 0; hi -= RG) {
          T g[RG];
#pragma unroll
          for (int k = 0; k < RG; ++k) {
            const int cs = hi - 1 - k >= 0 ? hi - 1 - k : 0;
            T v = sRt[j * RS + cs];
#pragma unroll
            for (int q = 0; q < kNnzBt; ++q) v += bt.w[q] * (sQ[cs * XS + bt.c[q]] + sQz[cs * XS + bt.c[q]]);
            g[k] = v;
          }
#pragma unroll
          for (int k = 0; k < RG; ++k)
            if (hi - 1 - k >= 0) {  // wave-uniform
              rc += g[k];
              sRt[j * RS + hi - 1 - k] = rc;
            }
        }
      } else {
        for (int cc = C - 1; cc >= 0; --cc) {
          T g = sRt[j * RS + cc];
          for (int q = bt.q0; q < bt.q1; ++q)
            g += gp(sys.bt_v)[q] * (sQ[cc * XS + gp(sys.bt_ci)[q]] + sQz[cc * XS + gp(sys.bt_ci)[q]]);
          rc += g;
          sRt[j * RS + cc] = rc;
        }
      }
      if (k0 == 0) st_agent(&td.ctopR[(size_t)chain * nu + j], rc);
    }
    __syncthreads();  // sRt complete
    // In the last chunk the chain counts itself done at the parent once the
    // top terms are stored: the count is issued partway through the P
    // product (the stores have drained meanwhile) and its answer read after
    // it, before the du stores (which would otherwise have to drain first).
    const bool counting = k0 == 0 && pcnt != nullptr;  // workgroup-uniform
    int prev = 0;
    auto count_issue = [&] {
      if (counting) {
        wait_mem();
        __syncthreads();
        if (tid == 0) prev = __hip_atomic_fetch_add(pcnt, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      }
    };
    auto count_answer = [&] {
      if (counting && tid == 0) {
        s_last = (prev == pkids - 1);
        if (s_last) __hip_atomic_store(pcnt, 0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);  // ready for the next iteration
      }
    };
    if (ch.len <= kValuChain) {
      // a short chain (one chunk for every chunk length, so the choice never
      // depends on the chunk length): du = -P rho / (2 pi) on the VALU from
      // the same register-resident P.  Lane l of wave w sums its K residue
      // class, k = 4 st + l / 16, for columns 16 (w NT + t) + l % 16, in four
      // partial sums (st mod 4) fed by batches of eight LDS reads; the four
      // 16-lane rows are then added, (l, l ^ 16) + (l ^ 32, l ^ 48).
      for (int cc = 0; cc < kValuChain; ++cc) {
        if (cc >= C) break;  // wave-uniform
        T res[NT];
#pragma unroll
        for (int t = 0; t < NT; ++t) {
          T ps[4] = {T(0), T(0), T(0), T(0)};
#pragma unroll
          for (int g = 0; g < KS; g += 8) {
            T rv[8];
#pragma unroll
            for (int k = 0; k < 8; ++k) rv[k] = sRt[(4 * (g + k) + (lane >> 4)) * RS + cc];
#pragma unroll
            for (int k = 0; k < 8; ++k) ps[k & 3] = fmadd(preg[(g + k) * NT + t], rv[k], ps[k & 3]);
            __builtin_amdgcn_sched_barrier(0);
          }
          T a = (ps[0] + ps[1]) + (ps[2] + ps[3]);
          a += __shfl_xor(a, 16);
          a += __shfl_xor(a, 32);
          res[t] = a;
          if (cc == 0 && t == 0) count_issue();
        }
        if (cc == 0) count_answer();
#pragma unroll
        for (int t = 0; t < NT; ++t) {
          const int jj = 16 * (wave * NT + t) + (lane & 15);
          if (lane < 16 && jj < nu) gp(td.du)[(uint32_t)(nb + cc) * (uint32_t)nu + jj] = res[t] * sIp[cc];
        }
      }
      par ^= 1;
      continue;
    }
    // du = -P rho / (2 pi) on the matrix cores, in as many 16-row tiles as
    // the chunk's rows need (rows at or past C of the last tile hold stale
    // values: they only reach output rows that are not stored).  The A
    // operands of a K step are read from LDS one step ahead of their use, so
    // that the read is in flight while the step before runs.
    const int ks_run = (nu + 3) >> 2;  // K steps that meet a row of P below nu
    auto product = [&](auto tiles) {
      constexpr int MR = decltype(tiles)::value;
      v4 acc[MR][NT];
#pragma unroll
      for (int m = 0; m < MR; ++m)
#pragma unroll
        for (int t = 0; t < NT; ++t) acc[m][t] = v4{T(0), T(0), T(0), T(0)};
      T an[MR];
#pragma unroll
      for (int m = 0; m < MR; ++m) an[m] = sRt[(lane >> 4) * RS + 16 * m + (lane & 15)];
#pragma unroll
      for (int st = 0; st < KS; ++st) {
        T a[MR];
#pragma unroll
        for (int m = 0; m < MR; ++m) a[m] = an[m];
        if (st + 1 < KS) {
#pragma unroll
          for (int m = 0; m < MR; ++m) an[m] = sRt[(4 * (st + 1) + (lane >> 4)) * RS + 16 * m + (lane & 15)];
        }
        // a step whose rows of P all lie at or past nu adds zeros and is
        // skipped (only in the second half: KP is the least of 64, 128 >= nu)
        if (st < KS / 2 || st < ks_run) {
#pragma unroll
          for (int t = 0; t < NT; ++t)
#pragma unroll
            for (int m = 0; m < MR; ++m) acc[m][t] = Mfma<T>::op(a[m], preg[st * NT + t], acc[m][t]);
        }
        if (st % 8 == 7) __builtin_amdgcn_sched_barrier(0);
        if (st == KS / 2) count_issue();
      }
      count_answer();
#pragma unroll
      for (int m = 0; m < MR; ++m)
#pragma unroll
        for (int t = 0; t < NT; ++t) {
          const int jj = 16 * (wave * NT + t) + (lane & 15);
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const int cc = 16 * m + Mfma<T>::row(lane, r);
            if (cc < C && jj < nu) gp(td.du)[(uint32_t)(nb + cc) * (uint32_t)nu + jj] = acc[m][t][r] * sIp[cc];
          }
        }
    };
    if (MT > 1 && C <= 16)
      product(std::integral_constant<int, 1>{});
    else
      product(std::integral_constant<int, MT>{});
    par ^= 1;
  }
}

// The register-resident P of this lane (P[4 st + lane / 16][16 (wave NT + t)
// + lane % 16]) and the B' row of an input thread; then, in LDS, the zero
// rows of the transposed rho tile (they meet the zero rows of P; nothing
// else writes them).
template <typename T, int KP>
__device__ __forceinline__ void bwd_load_regs(const SysDev<T>& sys, T (&preg)[KP / 4 * (KP / 64)],
                                              RowCache<T, kNnzBt>& bt) {
  constexpr int NT = KP / 64, KS = KP / 4;
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
#pragma unroll
  for (int st = 0; st < KS; ++st)
#pragma unroll
    for (int t = 0; t < NT; ++t)
      preg[st * NT + t] = gp(sys.P)[(size_t)(4 * st + (lane >> 4)) * KP + 16 * (wave * NT + t) + (lane & 15)];
  load_row(bt, sys.bt_rp, sys.bt_ci, sys.bt_v, tid - 128, wave >= 2 && tid - 128 < sys.nu);
}

template <typename T, int KP, int NXL, int CH>
__device__ __forceinline__ void bwd_zero_rows(const SysDev<T>& sys, unsigned char* smem_raw) {
  const int nu = sys.nu;
  T* sRt = reinterpret_cast<T*>(smem_raw) + 2 * CH * 64 * NXL;
  for (int e = threadIdx.x; e < (KP - nu) * (CH + 1); e += kBlock) sRt[(size_t)nu * (CH + 1) + e] = T(0);
}

// The backward sweep of one leaf chain, then of each ancestor chain whose
// children have all been swept (the workgroup that completes a parent's
// count sweeps it).  AGP: the ancestors' y^nu was written in this launch by
// other workgroups and is read at device scope.
template <typename T, typename Y, int KP, int NXL, int CH, bool AGP>
__device__ __forceinline__ void bwd_item(const SysDev<T>& sys, const TreeDev<T, Y>& td, const Iter<T, Y>& x, int mode,
                                         int leaf, const ChainDesc leaf_desc, unsigned char* smem_raw,
                                         const T (&preg)[KP / 4 * (KP / 64)], const RowCache<T, kNnzBt>& bt,
                                         int& par, int& s_last, bool leaf_stashed = false) {
  int chain = leaf;
  ChainDesc ch = leaf_desc;
  while (true) {
    // the parent's descriptor (its number of children decides the count) is
    // fetched while this chain is swept
    const int parent = ch.parent;
    ChainDesc pdesc = ch;
    if (parent >= 0) pdesc = gp(td.chains)[parent];
    int* pcnt = parent >= 0 ? gp(td.cnt) + parent : nullptr;
    if (AGP && chain != leaf)
      bwd_chain<T, Y, KP, NXL, CH, true>(sys, td, x, mode, chain, ch, smem_raw, preg, bt, par, false, pcnt,
                                         pdesc.child_count, s_last);
    else
      bwd_chain<T, Y, KP, NXL, CH, false>(sys, td, x, mode, chain, ch, smem_raw, preg, bt, par,
                                          leaf_stashed && chain == leaf, pcnt, pdesc.child_count, s_last);
    if (parent < 0) break;  // the root chain is done: the sweep is complete
    __syncthreads();        // the count's answer is published
    if (!s_last) break;     // a sibling is still running; it will sweep the parent
    chain = parent;
    ch = pdesc;
  }
}

// Persistent: workgroup b takes leaf chains b, b + gridDim.x, ... (longest
// first), so the register-resident P is loaded once per workgroup.
template <typename T, typename Y, int KP, int NXL, int CH, int MODE>
__global__ __launch_bounds__(kBlock, 2) void k_backward(SysDev<T> sys, const TreeDev<T, Y>* __restrict__ trees,
                                                        const WorkItem* __restrict__ items, int n_items,
                                                        const double* __restrict__ ctab, int mode_arg) {
  const int mode = MODE == kModeAny ? mode_arg : MODE;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  __shared__ int s_last;
  constexpr int NT = KP / 64, KS = KP / 4;
  T preg[KS * NT];
  RowCache<T, kNnzBt> bt;
  bwd_load_regs<T, KP>(sys, preg, bt);
  bwd_zero_rows<T, KP, NXL, CH>(sys, smem_raw);
  int par = 0;
  for (int item = blockIdx.x; item < n_items; item += gridDim.x) {
    const WorkItem wi = items[item];
    const TreeDev<T, Y>& td = trees[wi.tree];
    const G<TreeState>* st = gp(td.st);
    if (st->done) continue;
    const Iter<T, Y> x = make_iter(td, st, ctab, mode);
    bwd_item<T, Y, KP, NXL, CH, false>(sys, td, x, mode, wi.chain, gp(td.chains)[wi.chain], smem_raw, preg, bt, par,
                                       s_last);
  }
}

// ---------------------------------------------------------------------------
// forward rollout and prox of a list of nodes, each the child of the one
// before it
//
// `codes` lists internal node indices (-1 - node: this workgroup owns the
// node); nullptr means the owned nodes [first, first + len).  For owned nodes
// the prox, dual update and primal output are computed; the others only pass
// the recursion on (ancestors another leaf chain owns).  Per chunk: waves 2-3
// run ut_n = ut_above + du_n in registers, publish ut in LDS and finish the
// psi~ blocks; after one barrier waves 0 and 1 both run
// x_n = A x_above + B ut_n + e_n (a running sum when A = I) and apply the
// distance prox to the sigma~ (wave 0) and zeta~ (wave 1) blocks, each block
// norm one wave reduction.
// ---------------------------------------------------------------------------
struct Partials {
  double s0, s1, s2;  // residual / |Hz| / |t| maxima, or power-iteration sums
  bool nan;           // a NaN met on the way (fmax would drop it)
};

// The fused iteration's hand-over from the forward rollout to the backward
// sweep of the same leaf chain: for the chain's own nodes the forward half
// writes what the next sweep would load -- xi_n = S (w_sigma + w_zeta) per
// block (raw, before the running sum), r_n = beta_n + S w_psi and
// -1/(2 pi_n) -- straight into the backward layout in LDS, with w the next
// iteration's extrapolated point formed from y^{nu+1} just computed and y^nu
// already in registers (the same expressions, in the same order, as the
// sweep's loads would give).  q == nullptr: no hand-over.
template <typename T, typename Y>
struct Stash {
  T* q;    // Q parts: block b at q + b * bch * xs, node k of the chain at row k
  T* r;    // transposed rho tile: r[j * rs + k]
  T* inv;  // -1/(2 pi) of node k
  int xs, rs, bch;
  Y cn;    // the extrapolation coefficient of the next iteration
};

// Store of a dual entry: AG and an inner node (an ancestor chain's node,
// read later in the same fused launch by the workgroup that sweeps that
// chain) -> device scope; otherwise a plain store.
template <typename Y, bool AG>
__device__ __forceinline__ void put_dual(G<Y>* p, Y v, bool inner) {
  if (AG && inner)
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  else
    *p = v;
}

// An empty asm that takes v in a register: the computation of v stays
// before this point (an optimisation barrier, no instruction).
template <typename T>
__device__ __forceinline__ void pin(T& v) {
  asm volatile("" : "+v"(v));
}

// The prox work of a chunk's nodes is pinned node by node (each node its own
// scheduling region: an inline asm bounds one) or after the whole chunk (the
// nodes' independent work overlaps, at the cost of more live registers).
// Overlap only for short chunks with one state row per lane and T = Y: the
// other variants would spill or lose a wave per SIMD.
template <typename T, typename Y, int NXL, int CH>
constexpr bool pin_per_node() {
  return sizeof(T) < sizeof(Y) || NXL * CH > 4;
}

__device__ __forceinline__ void fold_max(Partials& p, double hz, double t) {
  const double r = hz - t;
  p.nan |= (r != r);
  p.s0 = fmax(p.s0, fabs(r));
  p.s1 = fmax(p.s1, fabs(hz));
  p.s2 = fmax(p.s2, fabs(t));
}

// The extrapolated dual point from explicit arrays (see wpoint).
template <typename T, typename Y>
__device__ __forceinline__ Y wpoint2(int mode, Y c, T in_scale, const G<Y>* __restrict__ yc,
                                     const G<Y>* __restrict__ yp, uint32_t k) {
  const Y y = yc[k];
  if (mode == kModeAPG) return extrapolate(y, yp[k], c);
  if (mode == kModePower) return in_scale * y;
  return y;
}

// Entry k of a leaf chain's forward sequence: the plen root-path codes, then
// the chain's own nodes from `first` (owned: -1 - node).
__device__ __forceinline__ int32_t node_code(const G<int32_t>* __restrict__ codes, int plen, int first, int k) {
  return k < plen ? codes[k] : -1 - (first + k - plen);
}

// Node code of chunk entry cc from the wave's code register (lane cc holds
// entry cc of the chunk; entries past the sequence repeat its last node).
__device__ __forceinline__ int32_t chunk_code(int32_t cl, int cc) { return __builtin_amdgcn_readlane(cl, cc); }

// Waves 2-3, one chunk: ut_n = ut_above + du_n, u = ut + uhat, the input box
// of the psi~ blocks and the dual update.  The arrays are distinct
// allocations (the three dual slots rotate), so the loads of later nodes may
// be issued before the stores of earlier ones.
template <typename T, typename Y, int UP, int CH, bool AG>
__device__ __forceinline__ void fwd_psi_chunk(int mode, const Iter<T, Y>& x, int32_t cl, int C, int npath, int j,
                                              int nx, int nu, int D,
                                              const G<T>* __restrict__ du, const G<T>* __restrict__ uhat,
                                              const G<Y>* __restrict__ yc, const G<Y>* __restrict__ yp,
                                              const G<T>* __restrict__ scale, const G<T>* __restrict__ beta,
                                              G<Y>* __restrict__ ynew, G<T>* __restrict__ z, T* sUp, T& utc, T ulo,
                                              T uhi, const Stash<T, Y>& sh, Partials& pt) {
  constexpr int US = UP;
  const int W = nx + nu;
  const bool stash = sh.q != nullptr;
  // all loads of the chunk first, unconditionally (entries past the chunk's
  // end read a valid node), so that they are in flight together; then the
  // recursion, the prox and the stores
  T duv[CH], uhv[CH], sv[CH], bv[CH];
  Y yv[CH], wv[CH];
#pragma unroll
  for (int cc = 0; cc < CH; ++cc) {
    const int32_t code = chunk_code(cl, cc);
    const uint32_t n = (uint32_t)(code < 0 ? -1 - code : code);
    const uint32_t k = n * D + 2 * nx + j;
    duv[cc] = du[n * nu + j];
    uhv[cc] = x.affine ? uhat[n * nu + j] : T(0);
    yv[cc] = mode != kModeSolve ? yc[k] : Y(0);
    wv[cc] = mode == kModeAPG ? yp[k] : Y(0);
    sv[cc] = x.scaled ? scale[n * 3 + 2] : T(1);
    bv[cc] = stash ? beta[n * nu + j] : T(0);
  }
  // the dual point (see wpoint2)
#pragma unroll
  for (int cc = 0; cc < CH; ++cc)
    wv[cc] = mode == kModeAPG ? extrapolate(yv[cc], wv[cc], x.c) : (mode == kModePower ? x.in_scale * yv[cc] : Y(0));
  if (mode == kModeAPG) {
    // the recursion, the prox and the dual update of every node, branch-free
    // (entries past the chunk's end and nodes owned elsewhere are computed,
    // never stored, and enter the maxima as zeros); only the stores branch.
    // The prox and the update run in the dual's precision Y.
    T uv[CH];
    Y val[CH];
#pragma unroll
    for (int cc = 0; cc < CH; ++cc) {
      const bool keep = (cc < C) & (chunk_code(cl, cc) < 0);  // wave-uniform, no branch
      if (cc < C) utc += duv[cc];
      sUp[cc * US + j] = utc;  // rows past the chunk's end are never read
      const T u = utc + uhv[cc];
      const T s = sv[cc];
      const Y w = wv[cc];
      const Y a = (Y)u + w * (x.ilam / (Y)s);  // (w / lambda + s u) / s
      const Y t = clampv(a, (Y)ulo, (Y)uhi);
      uv[cc] = u;
      val[cc] = w + x.lam * (Y)s * ((Y)u - t);
      fold_max(pt, keep ? (double)u : 0.0, keep ? (double)t : 0.0);
      if constexpr (pin_per_node<T, Y, 1, CH>()) {
        pin(val[cc]);
        // the next sweep's r_n = beta_n + S w_psi, node by node here where
        // the registers would not hold the chunk's inputs past the loop
        if (stash && cc >= npath && cc < C)  // wave-uniform: a node of this chain
          sh.r[j * sh.rs + (cc - npath)] = beta_plus_scaled<T, Y>(bv[cc], s, extrapolate(val[cc], yv[cc], sh.cn));
      }
    }
    if constexpr (!pin_per_node<T, Y, 1, CH>()) {
#pragma unroll
      for (int cc = 0; cc < CH; ++cc) pin(val[cc]);
    }
    // the chain's own nodes: the next sweep's r_n = beta_n + S w_psi, after
    // the loop so that it has no branch
    if (!pin_per_node<T, Y, 1, CH>() && stash) {
#pragma unroll
      for (int cc = 0; cc < CH; ++cc)
        if (cc >= npath && cc < C)  // wave-uniform: a node of this chain
          sh.r[j * sh.rs + (cc - npath)] = beta_plus_scaled<T, Y>(bv[cc], sv[cc], extrapolate(val[cc], yv[cc], sh.cn));
    }
    if (npath <= 0 && C == CH) {
      // wave-uniform: a full chunk of the chain's own nodes (all owned here,
      // none an ancestor): no per-node test before the stores
#pragma unroll
      for (int cc = 0; cc < CH; ++cc) {
        const uint32_t n = (uint32_t)(-1 - chunk_code(cl, cc));
        if (x.write_z) z[n * W + nx + j] = uv[cc];
        ynew[n * D + 2 * nx + j] = val[cc];
      }
      return;
    }
#pragma unroll
    for (int cc = 0; cc < CH; ++cc) {
      if (cc >= C) continue;  // wave-uniform
      const int32_t code = chunk_code(cl, cc);
      if (code >= 0) continue;  // wave-uniform: the node is owned elsewhere
      const uint32_t n = (uint32_t)(-1 - code);
      if (x.write_z) z[n * W + nx + j] = uv[cc];
      put_dual<Y, AG>(&ynew[n * D + 2 * nx + j], val[cc], cc < npath);
    }
    return;
  }
#pragma unroll
  for (int cc = 0; cc < CH; ++cc)
    if (cc < C) {
      const int32_t code = chunk_code(cl, cc);
      const bool own = code < 0;
      const uint32_t n = (uint32_t)(own ? -1 - code : code);
      utc += duv[cc];
      sUp[cc * US + j] = utc;
      if (own) {
        const T u = utc + uhv[cc];
        if (x.write_z) z[n * W + nx + j] = u;
        if (mode != kModeSolve) {
          const T s = sv[cc];
          const Y w = wv[cc];
          if (mode == kModePower) {
            const T g = -s * u;
            ynew[n * D + 2 * nx + j] = (Y)g;
            pt.s0 += (double)g * (double)g;
            pt.s1 += (double)w * (double)g;
          } else {
            const Y a = (Y)u + w * (x.ilam / (Y)s);  // (w / lambda + s u) / s
            const Y t = clampv(a, (Y)ulo, (Y)uhi);
            ynew[n * D + 2 * nx + j] = w + x.lam * (Y)s * ((Y)u - t);
            fold_max(pt, (double)u, (double)t);
          }
        }
      }
    }
}

// Waves 0 (b = 0, sigma~) and 1 (b = 1, zeta~), one chunk after ut is
// published.  Phase A runs x_n = A x_above + B ut_n + e_n for every node of
// the chunk (with A = I the B ut terms of all nodes are formed first; only
// the running sum is sequential).  Phase B applies the distance prox of
// block b to every node at once -- the block norms and inverse square roots
// of different nodes are independent, so they overlap; each node's
// (1 / lambda) / s and radius come from LDS (sFT, staged by waves 2 and 3) --
// and stores the dual update and primal output of the owned nodes.  Every
// value is computed by the same expression as node by node.
template <typename T, typename Y, int NXL, int UP, int CH, bool AG>
__device__ __forceinline__ void fwd_state_chunk(const SysDev<T>& sys, int mode, const Iter<T, Y>& x, int b, int32_t cl,
                                                int C, int npath,
                                                const T (&ev)[NXL][CH], const Y (&wv)[NXL][CH],
                                                const Y (&yv)[NXL][CH], T* stq, int sxs, Y cn,
                                                const RowCache<T, kNnzB> (&brow)[NXL], const T (&bnd)[NXL][2],
                                                const T* sSP, const Y* sFT, G<Y>* __restrict__ ynew,
                                                G<T>* __restrict__ z, const T* sUp, T* cx, T (&xc)[NXL],
                                                Partials& pt) {
  constexpr int US = UP;
  const int lane = threadIdx.x & 63;
  const int nx = sys.nx, nu = sys.nu, D = sys.D;
  const int W = nx + nu;
  // phase A: the state of every node of the chunk (lanes past nx hold 0)
  T xs[NXL][CH];
  if (sys.a_identity) {
#pragma unroll
    for (int r = 0; r < NXL; ++r) {
      const int i = lane + 64 * r;
      T g[CH];
      // a lane whose B row exceeds the register cache sends the whole wave
      // through the CSR arrays; otherwise every LDS read of the chunk is
      // issued before the products (one basic block, no per-lane branch)
      if (!__any(brow[r].n > kNnzB)) {
        T bu[CH][kNnzB];
#pragma unroll
        for (int cc = 0; cc < CH; ++cc)
#pragma unroll
          for (int q = 0; q < kNnzB; ++q) bu[cc][q] = sUp[cc * US + brow[r].c[q]];
#pragma unroll
        for (int cc = 0; cc < CH; ++cc) {
          g[cc] = ev[r][cc];
#pragma unroll
          for (int q = 0; q < kNnzB; ++q) g[cc] += brow[r].w[q] * bu[cc][q];
        }
      } else {
#pragma unroll
        for (int cc = 0; cc < CH; ++cc) {
          g[cc] = ev[r][cc];
          for (int q = brow[r].q0; q < brow[r].q1; ++q) g[cc] += gp(sys.b_v)[q] * sUp[cc * US + gp(sys.b_ci)[q]];
        }
      }
#pragma unroll
      for (int cc = 0; cc < CH; ++cc) {
        if (cc < C && i < nx) xc[r] += g[cc];
        xs[r][cc] = i < nx ? xc[r] : T(0);
      }
    }
  } else {
#pragma unroll
    for (int r = 0; r < NXL; ++r)
      if (lane + 64 * r < nx) cx[lane + 64 * r] = xc[r];
#pragma unroll
    for (int cc = 0; cc < CH; ++cc) {
      if (cc >= C) {  // wave-uniform
#pragma unroll
        for (int r = 0; r < NXL; ++r) xs[r][cc] = T(0);
        continue;
      }
      // one node at a time; the carry is exchanged through LDS within this
      // wave
      __builtin_amdgcn_wave_barrier();
      T xn[NXL];
#pragma unroll
      for (int r = 0; r < NXL; ++r) {
        const int i = lane + 64 * r;
        xn[r] = T(0);
        if (i < nx) {
          T g = ev[r][cc];
          for (int q = gp(sys.a_rp)[i]; q < gp(sys.a_rp)[i + 1]; ++q) g += gp(sys.a_v)[q] * cx[gp(sys.a_ci)[q]];
          for (int q = gp(sys.b_rp)[i]; q < gp(sys.b_rp)[i + 1]; ++q) g += gp(sys.b_v)[q] * sUp[cc * US + gp(sys.b_ci)[q]];
          xn[r] = g;
        }
      }
      __builtin_amdgcn_wave_barrier();
#pragma unroll
      for (int r = 0; r < NXL; ++r) {
        const int i = lane + 64 * r;
        if (i < nx) {
          cx[i] = xn[r];
          xc[r] = xn[r];
        }
        xs[r][cc] = xn[r];
      }
    }
  }
  if (mode == kModeSolve || mode == kModePower) {
#pragma unroll
    for (int cc = 0; cc < CH; ++cc) {
      if (cc >= C) continue;  // wave-uniform
      const int32_t code = chunk_code(cl, cc);
      if (code >= 0) continue;  // wave-uniform: the node is owned elsewhere
      const uint32_t n = (uint32_t)(-1 - code);
      if (x.write_z && b == 0) {
#pragma unroll
        for (int r = 0; r < NXL; ++r)
          if (lane + 64 * r < nx) z[n * W + lane + 64 * r] = xs[r][cc];
      }
      if (mode == kModeSolve) continue;
      const T s = sSP[4 * cc + b];
#pragma unroll
      for (int r = 0; r < NXL; ++r) {
        const int i = lane + 64 * r;
        if (i < nx) {
          const T g = -s * xs[r][cc];
          ynew[n * D + b * nx + i] = (Y)g;
          pt.s0 += (double)g * (double)g;
          pt.s1 += (double)wv[r][cc] * (double)g;
        }
      }
    }
    return;
  }
  // phase B (APG): the prox and the dual update of every node, branch-free
  // (nodes past the chunk's end and nodes owned elsewhere are computed too,
  // never stored, and enter the maxima as zeros, which leaves them
  // unchanged).  The loop has no branch, so the nodes' chains (block norm,
  // inverse square root, step) form one scheduling region and overlap;
  // pin() keeps the compiler from sinking this work into the per-node store
  // branches below, where it would run node by node.  The prox and the
  // update run in the dual's precision Y.
  // bit cc: entry k0 + cc exists and is owned by this chain (wave-uniform)
  const uint64_t live = __ballot(cl < 0) & ((1ull << C) - 1);
  // Nodes are taken in groups of G whose chains overlap (all of the chunk,
  // or one at a time where the registers would not hold more).
  constexpr int G = pin_per_node<T, Y, NXL, CH>() ? 1 : CH;
  Y val[NXL][CH];
#pragma unroll
  for (int g0 = 0; g0 < CH; g0 += G) {
    // the prox input a = (w / lambda + s Hz) / s, its projection pa on the
    // block's set and the squared distance, for every node of the group
    Y a[NXL][G], pa[NXL][G], dsq[G];
#pragma unroll
    for (int c = 0; c < G; ++c) {
      const int cc = g0 + c;
      const Y f = sFT[4 * cc + b];  // (1 / lambda) / s
      dsq[c] = Y(0);
#pragma unroll
      for (int r = 0; r < NXL; ++r) {
        a[r][c] = (Y)xs[r][cc] + wv[r][cc] * f;
        const Y lo = (Y)bnd[r][0], hi = (Y)bnd[r][1];
        pa[r][c] = b == 0 ? (a[r][c] > lo ? a[r][c] : lo) : clampv(a[r][c], lo, hi);
        const Y d = lane + 64 * r < nx ? a[r][c] - pa[r][c] : Y(0);
        dsq[c] += d * d;
      }
    }
    wave_allsum(dsq);
    // the distance against the radius tau: inside, the projection; outside,
    // the step of length tau towards it
#pragma unroll
    for (int c = 0; c < G; ++c) {
      const int cc = g0 + c;
      const bool keep = (live >> cc) & 1;
      const T s = sSP[4 * cc + b];
      const Y tau = sFT[4 * cc + 2 + b];  // c_b (1 / lambda) / s^2
      const bool inside = dsq[c] <= tau * tau;
      const Y k = tau * rsqrt_refined(dsq[c]);
#pragma unroll
      for (int r = 0; r < NXL; ++r) {
        const bool in = keep && lane + 64 * r < nx;
        const Y t = inside ? pa[r][c] : a[r][c] - k * (a[r][c] - pa[r][c]);
        val[r][cc] = wv[r][cc] + x.lam * (Y)s * ((Y)xs[r][cc] - t);
        fold_max(pt, in ? (double)xs[r][cc] : 0.0, in ? (double)t : 0.0);
        if constexpr (pin_per_node<T, Y, NXL, CH>()) pin(val[r][cc]);
      }
    }
  }
  if constexpr (!pin_per_node<T, Y, NXL, CH>()) {
#pragma unroll
    for (int cc = 0; cc < CH; ++cc)
#pragma unroll
      for (int r = 0; r < NXL; ++r) pin(val[r][cc]);
  }
  // (one state row per lane, and for float64 short chunks: the other
  // variants have no registers to spare for this path)
  if (npath <= 0 && C == CH && NXL == 1 && (sizeof(T) == 4 || CH <= 4)) {
    // wave-uniform: a full chunk of the chain's own nodes (all owned here,
    // none an ancestor), so one lane test covers every store
    const bool wz = x.write_z && b == 0;
#pragma unroll
    for (int r = 0; r < NXL; ++r) {
      const int i = lane + 64 * r;
      if (i < nx) {
        // the next sweep's xi_n part of block b
        if (stq != nullptr) {
#pragma unroll
          for (int cc = 0; cc < CH; ++cc)
            stq[(cc - npath) * sxs + i] = scaled<T, Y>(sSP[4 * cc + b], extrapolate(val[r][cc], yv[r][cc], cn));
        }
#pragma unroll
        for (int cc = 0; cc < CH; ++cc) {
          const uint32_t n = (uint32_t)(-1 - chunk_code(cl, cc));
          if (wz) z[n * W + i] = xs[r][cc];
          ynew[n * D + b * nx + i] = val[r][cc];
        }
      }
    }
    return;
  }
  // the chain's own nodes: the next sweep's xi_n part of block b
  if (stq != nullptr) {
#pragma unroll
    for (int cc = 0; cc < CH; ++cc) {
      if (cc < npath || cc >= C) continue;  // wave-uniform
      const T s = sSP[4 * cc + b];
#pragma unroll
      for (int r = 0; r < NXL; ++r)
        if (lane + 64 * r < nx)
          stq[(cc - npath) * sxs + lane + 64 * r] = scaled<T, Y>(s, extrapolate(val[r][cc], yv[r][cc], cn));
    }
  }
#pragma unroll
  for (int cc = 0; cc < CH; ++cc) {
    if (cc >= C) continue;  // wave-uniform
    const int32_t code = chunk_code(cl, cc);
    if (code >= 0) continue;  // wave-uniform: the node is owned elsewhere
    const uint32_t n = (uint32_t)(-1 - code);
#pragma unroll
    for (int r = 0; r < NXL; ++r) {
      const int i = lane + 64 * r;
      if (i < nx) {
        if (x.write_z && b == 0) z[n * W + i] = xs[r][cc];
        put_dual<Y, AG>(&ynew[n * D + b * nx + i], val[r][cc], cc < npath);
      }
    }
  }
}

// Waves 0 and 1: e and the dual iterates of the wave's block for the nodes of
// a chunk (entries past the sequence repeat its last node; lanes past nx read
// component 0).
template <typename T, typename Y, int NXL, int CH>
struct StateLoads {
  T e[NXL][CH];
  Y y[NXL][CH], yp[NXL][CH];
};

// Loaded one chunk ahead of their use when two sets fit in registers beside
// the rest of the rollout (at most 96 bytes per lane each).
template <typename T, typename Y, int NXL, int CH>
constexpr bool state_prefetch() {
  return NXL * CH * (sizeof(T) + 2 * sizeof(Y)) <= 96;
}

template <typename T, typename Y, int NXL, int CH>
__device__ __forceinline__ void load_state(const TreeDev<T, Y>& td, const Iter<T, Y>& x, int mode, int nx, int D,
                                           int b, int32_t cl, StateLoads<T, Y, NXL, CH>& L) {
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int r = 0; r < NXL; ++r) {
    const int i = lane + 64 * r;
    const uint32_t ic = (uint32_t)(i < nx ? i : 0);
#pragma unroll
    for (int cc = 0; cc < CH; ++cc) {
      const int32_t code = chunk_code(cl, cc);
      const uint32_t n = (uint32_t)(code < 0 ? -1 - code : code);
      const uint32_t k = n * D + b * nx + ic;
      L.e[r][cc] = x.affine ? gp(td.e)[n * nx + ic] : T(0);
      L.y[r][cc] = mode != kModeSolve ? x.ycur[k] : Y(0);
      L.yp[r][cc] = mode == kModeAPG ? x.yprv[k] : Y(0);
    }
    if (NXL > 1) __builtin_amdgcn_sched_barrier(0);  // one state row's loads in flight at a time
  }
}

template <typename T, typename Y, int NXL, int UP, int CH, bool AG>
__device__ __forceinline__ void fwd_nodes(const SysDev<T>& sys, const TreeDev<T, Y>& td, const Iter<T, Y>& x, int mode,
                          const G<int32_t>* codes, int plen, int first, int len, unsigned char* smem_raw,
                          const RowCache<T, kNnzB> (&brow)[NXL], T (&xc)[NXL], T& utc, const T (&bnd)[NXL][2],
                          const T (&ubnd)[2], const Stash<T, Y>& sh, int& par, Partials& pt) {
  constexpr bool PF = state_prefetch<T, Y, NXL, CH>();
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int nx = sys.nx, nu = sys.nu, D = sys.D;
  const int j = tid - 128;
  const bool ju = wave >= 2 && j < nu;
  T* sU = reinterpret_cast<T*>(smem_raw);  // 2 x CH x UP (UP >= nu, a constant)
  T* sSP = sU + 2 * CH * UP;               // 2 x CH x 4: the scales of the chunk's nodes
  T* sXc = sSP + 2 * 4 * CH;               // 2 x nx (general A: carries of waves 0, 1)
  Y* sFT = reinterpret_cast<Y*>(sXc + 2 * nx);  // 2 x CH x 4: (1/lambda)/s and radii of both blocks
  // every wave keeps the node codes of the current and the next chunk in
  // registers (lane k: entry k0 + k, resp. k0 + CH + k; entries past the
  // sequence repeat its last node) and loads the codes one chunk further
  // while the current chunk runs
  const int last = len - 1;
  int32_t cl = node_code(codes, plen, first, lane < last ? lane : last);
  int32_t cn = node_code(codes, plen, first, CH + lane < last ? CH + lane : last);
  StateLoads<T, Y, NXL, CH> LA, LB;
  if (PF && wave < 2) load_state<T, Y, NXL, CH>(td, x, mode, nx, D, wave, cl, LA);

  // one chunk: Lc holds (without prefetch: receives) its state loads, Ln
  // receives the next chunk's (the loop below alternates the two sets, so
  // that no register copy waits for loads in flight)
  auto chunk = [&](int k0, StateLoads<T, Y, NXL, CH>& Lc, StateLoads<T, Y, NXL, CH>& Ln) {
    const int C = len - k0 < CH ? len - k0 : CH;
    const int npath = plen - k0;  // entries cc < npath are ancestor (inner) nodes
    const int32_t cur = cl;
    const int32_t nxt = cn;
    if (k0 + 2 * CH < len) cn = node_code(codes, plen, first, k0 + 2 * CH + lane < last ? k0 + 2 * CH + lane : last);
    cl = nxt;
    const int b = wave;  // 0: sigma~, 1: zeta~
    // the dual point of the wave's block (see wpoint)
    Y wv[NXL][CH];
    auto dual_point = [&] {
#pragma unroll
      for (int r = 0; r < NXL; ++r)
#pragma unroll
        for (int cc = 0; cc < CH; ++cc) {
          const Y y = Lc.y[r][cc];
          wv[r][cc] = mode == kModeAPG ? extrapolate(y, Lc.yp[r][cc], x.c) : (mode == kModePower ? x.in_scale * y : Y(0));
        }
    };
    if (wave < 2) {
      if (!PF) {
        load_state<T, Y, NXL, CH>(td, x, mode, nx, D, b, cur, Lc);
      } else {
        // this chunk's loads (issued one chunk ago) are consumed before the
        // next chunk's are issued: the wait counter counts loads in issue
        // order, so a first use after the next issue would wait for those too
        dual_point();
#pragma unroll
        for (int r = 0; r < NXL; ++r)
#pragma unroll
          for (int cc = 0; cc < CH; ++cc) {
            pin(wv[r][cc]);
            pin(Lc.e[r][cc]);
          }
        __builtin_amdgcn_sched_barrier(0);
        if (k0 + CH < len) load_state<T, Y, NXL, CH>(td, x, mode, nx, D, b, nxt, Ln);
      }
    }
    T* sUp = sU + par * CH * UP;
    T* sSPp = sSP + par * 4 * CH;
    Y* sFTp = sFT + par * 4 * CH;
    // waves 2 (block 0) and 3 (block 1) stage the scale of their block for
    // the chunk's nodes (lane k: entry k0 + k), with (1 / lambda) / s and the
    // prox radius c_b (1 / lambda) / s^2 (c_0 = W_x, times pi_n when the
    // safety term is weighted by probability; c_1 = gamma_d), around their own
    // loads, so that waves 0 and 1 neither wait for them nor divide
    const bool spl = wave >= 2 && lane < C;
    const int sb = wave - 2;
    T sp = T(1), sp3 = T(1);
    if (spl) {
      const uint32_t n = (uint32_t)(cur < 0 ? -1 - cur : cur);
      if (x.scaled) sp = gp(td.scale)[n * 3 + sb];
      if (sb == 0) sp3 = gp(td.pi)[n];
    }
    if (ju)
      fwd_psi_chunk<T, Y, UP, CH, AG>(mode, x, cur, C, npath, j, nx, nu, D, gp(td.du), gp(td.uhat), x.ycur,
                                      x.yprv, gp(td.scale), gp(td.beta), x.ynew, gp(td.z), sUp, utc, ubnd[0],
                                      ubnd[1], sh, pt);
    if (spl) {
      sSPp[4 * lane + sb] = sp;
      if (mode == kModeAPG) {
        const Y ys = (Y)sp;
        const Y pi_n = sb == 0 && sys.safety_by_prob ? (Y)sp3 : Y(1);
        const Y cb = sb == 0 ? (Y)sys.W_x * pi_n : (Y)sys.gamma_d;
        sFTp[4 * lane + sb] = x.ilam / ys;
        sFTp[4 * lane + 2 + sb] = cb * x.ilam / (ys * ys);
      }
      if (sb == 0 && sh.q != nullptr && lane >= npath) sh.inv[lane - npath] = T(-0.5) / sp3;  // a node of this chain
    }
    __syncthreads();  // ut and the scales of the chunk published
    if (wave < 2) {
      if (!PF) dual_point();
      fwd_state_chunk<T, Y, NXL, UP, CH, AG>(sys, mode, x, b, cur, C, npath, Lc.e, wv, Lc.y,
                                             sh.q != nullptr ? sh.q + (size_t)b * sh.bch * sh.xs : nullptr, sh.xs,
                                             sh.cn, brow, bnd, sSPp, sFTp, x.ynew, gp(td.z), sUp,
                                             sXc + (size_t)wave * nx, xc, pt);
    }
    par ^= 1;
  };
  if constexpr (PF) {
    for (int k0 = 0; k0 < len; k0 += 2 * CH) {
      chunk(k0, LA, LB);
      if (k0 + CH < len) chunk(k0 + CH, LB, LA);
    }
  } else {
    for (int k0 = 0; k0 < len; k0 += CH) chunk(k0, LA, LA);
  }
}

// Two workgroups per CU, except with two state rows per lane and long
// chunks (more than 32 bytes of each per-node array per lane): those need
// more than 256 registers per lane.
template <typename Y, int NXL, int CH>
constexpr int fwd_min_blocks() {
  return (NXL > 1 && CH * sizeof(Y) > 32) ? 1 : 2;
}

// Per-thread system rows and bounds of the thread's role in the forward
// rollout.  They depend on the system only, so kernels load them first,
// while the work item, tree and tree state are still on their way.
template <typename T, int NXL>
struct FwdSys {
  RowCache<T, kNnzB> brow[NXL];
  T bnd[NXL][2];
  T ubnd[2];
};

template <typename T, int NXL>
__device__ __forceinline__ void fwd_sys_loads(const SysDev<T>& sys, FwdSys<T, NXL>& f) {
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int nx = sys.nx, nu = sys.nu;
  const int j = tid - 128;
#pragma unroll
  for (int r = 0; r < NXL; ++r) {
    const int i = lane + 64 * r;
    const bool vi = wave < 2 && i < nx;
    load_row(f.brow[r], sys.b_rp, sys.b_ci, sys.b_v, i, vi);
    f.bnd[r][0] = vi ? (wave == 0 ? gp(sys.xs)[i] : gp(sys.xmin)[i]) : T(0);
    f.bnd[r][1] = vi ? gp(sys.xmax)[i] : T(0);
  }
  f.ubnd[0] = (wave >= 2 && j < nu) ? gp(sys.umin)[j] : T(0);
  f.ubnd[1] = (wave >= 2 && j < nu) ? gp(sys.umax)[j] : T(0);
}

// The forward rollout and prox of one leaf chain (with its root path), its
// residual partials, and -- in the tree's last workgroup -- the end of the
// iteration (stop test, counters).  AG: the ancestors' dual entries this
// chain owns are stored at device scope (the fused iteration reads them in
// the same launch).
template <typename T, typename Y, int NXL, int UP, int CH, bool AG, typename AfterRollout>
__device__ __forceinline__ void fwd_item(const SysDev<T>& sys, const FwdSys<T, NXL>& fs, const TreeDev<T, Y>& td,
                                         const WorkItem wi, G<TreeState>* st, const Iter<T, Y>& x, int mode,
                                         unsigned char* smem_raw, int& s_last, int32_t* __restrict__ done_out,
                                         const Stash<T, Y>& sh, AfterRollout after_rollout) {
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int nx = sys.nx, nu = sys.nu;
  double* sRed = reinterpret_cast<double*>(smem_raw + lds_bytes_forward(nx, nu, sizeof(T), CH) - 32 * sizeof(double));

  // the carries of the thread's role: the root's parent state
  T xc[NXL];
#pragma unroll
  for (int r = 0; r < NXL; ++r) {
    const int i = lane + 64 * r;
    xc[r] = (wave < 2 && i < nx && x.affine) ? gp(td.p)[i] : T(0);
  }
  T utc = T(0);
  int par = 0;
  Partials pt{0.0, 0.0, 0.0, false};

  // the root path (ancestor nodes of this leaf chain, root first), then the
  // chain itself, as one sequence (the work item carries both ranges)
  fwd_nodes<T, Y, NXL, UP, CH, AG>(sys, td, x, mode, gp(td.path) + wi.p0, wi.plen, wi.first, wi.plen + wi.len,
                                   smem_raw, fs.brow, xc, utc, fs.bnd, fs.ubnd, sh, par, pt);

  after_rollout();  // the fused iteration issues the next sweep's register loads here
  // partials of this leaf chain
  const double qnan = __longlong_as_double(0x7ff8000000000000LL);
  double s0 = pt.nan ? qnan : pt.s0, s1 = pt.s1, s2 = pt.s2;
  if (mode == kModeAPG) {
    s0 = wave_nanmax(s0);
    s1 = wave_nanmax(s1);
    s2 = wave_nanmax(s2);
  } else if (mode == kModePower) {
    s0 = wave_sum(s0);
    s1 = wave_sum(s1);
  }
  if (lane == 0) {
    sRed[wave * 3 + 0] = s0;
    sRed[wave * 3 + 1] = s1;
    sRed[wave * 3 + 2] = s2;
  }
  __syncthreads();
  if (tid == 0) {
    double* out = gp(td.cstat) + (size_t)wi.chain * kStat;
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
    // every field of the tree's record the stop test reads, loaded together
    const int check_every = st->check_every, max_iter = st->max_iter, stall_limit = st->stall_limit;
    const int stall = st->stall;
    const double tol = st->tol, best_rp = st->best_rp;
    const bool check = ((it + 1) % check_every == 0) || (it + 1 >= max_iter);
    int done = 0;
    if (check) {
      // the leaves' partials, a batch of eight per lane at a time: every
      // chain index of the batch is loaded first, then every partial, so
      // that each round of loads is in flight together (the maxima do not
      // depend on the order)
      double rm = 0.0, hm = 0.0;
      for (int k0 = 0; k0 < td.n_leaves; k0 += 64 * 8) {
        int lf[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
          const int k = k0 + lane + 64 * u;
          lf[u] = k < td.n_leaves ? gp(td.leaves)[k] : -1;
        }
        double v[8][3];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
          const double* cs = td.cstat + (size_t)(lf[u] >= 0 ? lf[u] : 0) * kStat;
#pragma unroll
          for (int q = 0; q < 3; ++q) v[u][q] = lf[u] >= 0 ? ld_agent(&cs[q]) : 0.0;
        }
#pragma unroll
        for (int u = 0; u < 8; ++u) {
          rm = nanmax(rm, v[u][0]);
          hm = nanmax(hm, v[u][1]);
          hm = nanmax(hm, v[u][2]);
        }
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
        } else if (tol > 0.0 && rm <= tol * (1.0 + hm)) {
          done = 1;
          st->status = 0;
        } else if (it + 1 >= max_iter) {
          done = 1;
          st->status = 1;
        } else if (stall_limit > 0) {
          // no new minimum of r_p for stall_limit checks: the iteration has
          // reached the accuracy floor of its number format
          if (rm < 0.99 * best_rp) {
            st->best_rp = rm;
            st->stall = 0;
          } else {
            st->stall = stall + 1;
            if (stall + 1 >= stall_limit) {
              done = 1;
              st->status = 2;
            }
          }
        }
        if (done) {
          st->done = 1;
          st->iters_done = it + 1;
        }
      }
    }
    if (lane == 0) {
      __hip_atomic_store(&st->fwd_count, 0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      st->iter = it + 1;
      done_out[wi.tree] = done;
    }
  } else {  // power iteration: Rayleigh quotient and normalisation
    double gg = 0.0, wg = 0.0;
    for (int k = lane; k < td.n_leaves; k += 64) {
      const double* cs = td.cstat + (size_t)gp(td.leaves)[k] * kStat;
      gg += ld_agent(&cs[0]);
      wg += ld_agent(&cs[1]);
    }
    gg = wave_sum(gg);
    wg = wave_sum(wg);
    if (lane == 0) {
      st->lmax_est = wg;
      st->in_scale = gg > 0.0 ? 1.0 / sqrt(gg) : 0.0;
      __hip_atomic_store(&st->fwd_count, 0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      st->iter = it + 1;
      done_out[wi.tree] = 0;
    }
  }
}


template <typename T, typename Y, int NXL, int UP, int CH, int MODE>
__global__ __launch_bounds__(kBlock, (fwd_min_blocks<Y, NXL, CH>())) void k_forward(SysDev<T> sys, const TreeDev<T, Y>* __restrict__ trees,
                                                       const WorkItem* __restrict__ items,
                                                       const double* __restrict__ ctab, int mode_arg,
                                                       int32_t* __restrict__ done_out) {
  const int mode = MODE == kModeAny ? mode_arg : MODE;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  __shared__ int s_last;
  FwdSys<T, NXL> fs;
  fwd_sys_loads<T, NXL>(sys, fs);
  const WorkItem wi = items[blockIdx.x];
  const TreeDev<T, Y>& td = trees[wi.tree];
  G<TreeState>* st = gp(td.st);
  if (st->done) {
    if (threadIdx.x == 0) done_out[wi.tree] = 1;
    return;
  }
  const Iter<T, Y> x = make_iter(td, st, ctab, mode);
  const Stash<T, Y> none{nullptr, nullptr, nullptr, 0, 0, 0, Y(0)};
  fwd_item<T, Y, NXL, UP, CH, false>(sys, fs, td, wi, st, x, mode, smem_raw, s_last, done_out, none, [] {});
}

// One fused APG iteration: the forward rollout of iteration nu for a leaf
// chain, then the backward sweep of iteration nu + 1 for the same chain (its
// y^{nu+1} was written just before by this workgroup) and for each ancestor
// chain this workgroup completes.  The launch before the first fused one of
// a run is a backward launch.  A tree that stops at iteration nu has swept
// iteration nu + 1 for nothing; nothing reads it.
// The fused kernel holds the backward kernel's registers too: with two
// state rows per lane and 128-wide float64 P it runs one workgroup per CU.
template <typename T, typename Y, int KP, int NXL, int FCH>
constexpr int iter_min_blocks() {
  return (fwd_min_blocks<Y, NXL, FCH>() == 1 || (NXL > 1 && sizeof(T) == 8 && KP == 128)) ? 1 : 2;
}

// stash_arg: the LDS holds the backward layout and the forward's after it, so
// that a leaf chain of at most BCH nodes hands its sweep inputs over in LDS
// (Stash); otherwise the two halves share the LDS and the sweep loads them.
template <typename T, typename Y, int KP, int NXL, int BCH, int FCH>
__global__ __launch_bounds__(kBlock, (iter_min_blocks<T, Y, KP, NXL, FCH>())) void k_iter(
    SysDev<T> sys, const TreeDev<T, Y>* __restrict__ trees, const WorkItem* __restrict__ items,
    const double* __restrict__ ctab, int32_t* __restrict__ done_out, int stash_arg) {
  constexpr int NT = KP / 64, KS = KP / 4;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  __shared__ int s_last;
  FwdSys<T, NXL> fs;
  fwd_sys_loads<T, NXL>(sys, fs);
  const WorkItem wi = items[blockIdx.x];
  const TreeDev<T, Y>& td = trees[wi.tree];
  G<TreeState>* st = gp(td.st);
  if (st->done) {
    if (threadIdx.x == 0) done_out[wi.tree] = 1;
    return;
  }
  const Iter<T, Y> xf = make_iter(td, st, ctab, kModeAPG);
  // P and the B' row of the backward half are loaded while the forward half
  // folds its partials (few registers are live there)
  // (and the next iteration's record and this chain's descriptor)
  T preg[KS * NT];
  RowCache<T, kNnzBt> bt;
  Iter<T, Y> xb;
  ChainDesc leaf_desc;
  const bool stash = stash_arg != 0 && wi.len <= BCH;
  T* sQs = reinterpret_cast<T*>(smem_raw);
  T* sRs = sQs + 2 * BCH * 64 * NXL;
  const Stash<T, Y> sh{stash ? sQs : nullptr, sRs, sRs + (size_t)KP * (BCH + 1), 64 * NXL, BCH + 1, BCH,
                       (Y)gp(ctab)[xf.it + 1]};
  unsigned char* fwd_lds = stash_arg != 0 ? smem_raw + lds_stash_offset(sys.nx, sys.nu, sizeof(T), BCH) : smem_raw;
  fwd_item<T, Y, NXL, KP, FCH, true>(sys, fs, td, wi, st, xf, kModeAPG, fwd_lds, s_last, done_out, sh, [&] {
    bwd_load_regs<T, KP>(sys, preg, bt);
    xb = make_iter_at(td, st, ctab, kModeAPG, xf.it + 1);
    leaf_desc = gp(td.chains)[wi.chain];
  });
  __syncthreads();  // the LDS now holds the backward layout
  bwd_zero_rows<T, KP, NXL, BCH>(sys, smem_raw);
  int par = 0;
  bwd_item<T, Y, KP, NXL, BCH, true>(sys, td, xb, kModeAPG, wi.chain, leaf_desc, smem_raw, preg, bt, par, s_last,
                                     stash);
}

template <typename T>
__global__ void k_widen(const T* __restrict__ src, double* __restrict__ dst, size_t n) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) dst[i] = (double)src[i];
}

// One thread per dual entry of the next tree: the entry of its image node in
// the previous dual, times the block's factor.
template <typename Ts, typename Td>
__global__ void k_shift(const Ts* __restrict__ src, Td* __restrict__ dst0, Td* __restrict__ dst2,
                        const int32_t* __restrict__ src_node, const double* __restrict__ f, int M, int nx, int nu) {
  const int D = 2 * nx + nu;
  const size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (size_t)M * D) return;
  const int n = (int)(e / D);
  const int k = (int)(e - (size_t)n * D);
  const int b = k < nx ? 0 : (k < 2 * nx ? 1 : 2);
  const Td v = (Td)(gp(f)[(size_t)n * 3 + b] * (double)gp(src)[(size_t)gp(src_node)[n] * D + k]);
  gp(dst0)[e] = v;
  gp(dst2)[e] = v;
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
// Workgroups of `kernel` that fit on the device at once (cached per kernel
// and LDS size).
template <typename K>
int resident_blocks(K kernel, size_t lds) {
  static std::mutex mu;
  static std::map<std::tuple<const void*, size_t, int>, int> cache;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 0;
  const auto key = std::make_tuple(reinterpret_cast<const void*>(kernel), lds, dev);
  std::lock_guard<std::mutex> g(mu);
  auto it = cache.find(key);
  if (it != cache.end()) return it->second;
  int per_cu = 0, cus = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, reinterpret_cast<const void*>(kernel), kBlock, lds) !=
          hipSuccess ||
      hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
    return 0;
  const int n = std::max(1, per_cu) * std::max(1, cus);
  cache[key] = n;
  return n;
}

// The APG iteration has an instantiation per chunk length with the mode
// fixed; the power iteration and the solve step share one with the mode a
// run-time argument and the default chunk length (the chunk length never
// changes the result).
template <typename T, typename Y, int KP, int NXL, int CH, int MODE>
hipError_t launch_backward_ch(const SysDev<T>& sys, const TreeDev<T, Y>* trees, const WorkItem* items, int n_items,
                              const double* ctab, int mode, hipStream_t s) {
  const size_t lds = lds_bytes_backward(sys.nx, sys.nu, sizeof(T), CH);
  hipError_t e = allow_lds(k_backward<T, Y, KP, NXL, CH, MODE>, lds);
  if (e != hipSuccess) return e;
  const int res = resident_blocks(k_backward<T, Y, KP, NXL, CH, MODE>, lds);
  if (res <= 0) return hipErrorInvalidValue;
  const int grid = std::min(n_items, res);
  hipLaunchKernelGGL((k_backward<T, Y, KP, NXL, CH, MODE>), dim3(grid), dim3(kBlock), lds, s, sys, trees, items,
                     n_items, ctab, mode);
  return hipGetLastError();
}

// A float32 solve step on a float64 dual exists for the APG iteration only.
template <typename T, int KP, int NXL, typename Y>
hipError_t launch_backward_kp(const SysDev<T>& sys, const TreeDev<T, Y>* trees, const WorkItem* items, int n_items,
                              const double* ctab, int mode, int chunk, hipStream_t s) {
  if (mode != kModeAPG) {
    if constexpr (std::is_same<T, Y>::value)
      return launch_backward_ch<T, Y, KP, NXL, Chunks<T>::bwd[0], kModeAny>(sys, trees, items, n_items, ctab, mode,
                                                                            s);
    return hipErrorInvalidValue;
  }
  if (chunk == 16) return launch_backward_ch<T, Y, KP, NXL, 16, kModeAPG>(sys, trees, items, n_items, ctab, mode, s);
  if constexpr (chunk_listed(Chunks<T>::bwd, 32))
    if (chunk == 32)
      return launch_backward_ch<T, Y, KP, NXL, 32, kModeAPG>(sys, trees, items, n_items, ctab, mode, s);
  return hipErrorInvalidValue;
}

template <typename T, typename Y>
hipError_t launch_backward(const SysDev<T>& sys, const TreeDev<T, Y>* trees, const WorkItem* items, int n_items,
                           const double* ctab, int mode, int chunk, hipStream_t s) {
  if (n_items <= 0) return hipSuccess;
  if (sys.nx > 128 || sys.nu > 128 || !chunk_listed(Chunks<T>::bwd, chunk)) return hipErrorInvalidValue;
  const bool x1 = sys.nx <= 64;
  if (sys.nu <= 64)
    return x1 ? launch_backward_kp<T, 64, 1>(sys, trees, items, n_items, ctab, mode, chunk, s)
              : launch_backward_kp<T, 64, 2>(sys, trees, items, n_items, ctab, mode, chunk, s);
  return x1 ? launch_backward_kp<T, 128, 1>(sys, trees, items, n_items, ctab, mode, chunk, s)
            : launch_backward_kp<T, 128, 2>(sys, trees, items, n_items, ctab, mode, chunk, s);
}

template <typename T, typename Y, int NXL, int UP, int CH, int MODE>
hipError_t launch_forward_ch(const SysDev<T>& sys, const TreeDev<T, Y>* trees, const WorkItem* items, int n_items,
                             const double* ctab, int mode, int32_t* done_out, hipStream_t s) {
  const size_t lds = lds_bytes_forward(sys.nx, sys.nu, sizeof(T), CH);
  hipError_t e = allow_lds(k_forward<T, Y, NXL, UP, CH, MODE>, lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((k_forward<T, Y, NXL, UP, CH, MODE>), dim3(n_items), dim3(kBlock), lds, s, sys, trees, items,
                     ctab, mode, done_out);
  return hipGetLastError();
}

template <typename T, int NXL, int UP, typename Y>
hipError_t launch_forward_t(const SysDev<T>& sys, const TreeDev<T, Y>* trees, const WorkItem* items, int n_items,
                            const double* ctab, int mode, int chunk, int32_t* done_out, hipStream_t s) {
  if (mode != kModeAPG) {
    if constexpr (std::is_same<T, Y>::value)
      return launch_forward_ch<T, Y, NXL, UP, Chunks<T>::fwd[0], kModeAny>(sys, trees, items, n_items, ctab, mode,
                                                                           done_out, s);
    return hipErrorInvalidValue;
  }
  if (chunk == 8)
    return launch_forward_ch<T, Y, NXL, UP, 8, kModeAPG>(sys, trees, items, n_items, ctab, mode, done_out, s);
  if constexpr (chunk_listed(Chunks<T>::fwd, 16))
    if (chunk == 16)
      return launch_forward_ch<T, Y, NXL, UP, 16, kModeAPG>(sys, trees, items, n_items, ctab, mode, done_out, s);
  if constexpr (chunk_listed(Chunks<T>::fwd, 4))
    if (chunk == 4)
      return launch_forward_ch<T, Y, NXL, UP, 4, kModeAPG>(sys, trees, items, n_items, ctab, mode, done_out, s);
  return hipErrorInvalidValue;
}

template <typename T, typename Y>
hipError_t launch_forward(const SysDev<T>& sys, const TreeDev<T, Y>* trees, const WorkItem* items, int n_items,
                          const double* ctab, int mode, int chunk, int32_t* done_out, hipStream_t s) {
  if (n_items <= 0) return hipSuccess;
  if (sys.nu > 128 || sys.nx > 128 || !chunk_listed(Chunks<T>::fwd, chunk)) return hipErrorInvalidValue;
  const bool x1 = sys.nx <= 64, u1 = sys.nu <= 64;
  if (x1) return u1 ? launch_forward_t<T, 1, 64>(sys, trees, items, n_items, ctab, mode, chunk, done_out, s)
                    : launch_forward_t<T, 1, 128>(sys, trees, items, n_items, ctab, mode, chunk, done_out, s);
  return u1 ? launch_forward_t<T, 2, 64>(sys, trees, items, n_items, ctab, mode, chunk, done_out, s)
            : launch_forward_t<T, 2, 128>(sys, trees, items, n_items, ctab, mode, chunk, done_out, s);
}

template <typename T, typename Y, int KP, int NXL, int BCH, int FCH>
hipError_t launch_iter_ch(const SysDev<T>& sys, const TreeDev<T, Y>* trees, const WorkItem* items, int n_items,
                          const double* ctab, int32_t* done_out, hipStream_t s) {
  // the LDS hand-over (both layouts side by side) is used where it leaves
  // room for the workgroups per CU the kernel's registers allow (two with
  // float64 solve steps, three with float32 ones)
  const size_t lf = lds_bytes_forward(sys.nx, sys.nu, sizeof(T), FCH);
  const size_t lb = lds_bytes_backward(sys.nx, sys.nu, sizeof(T), BCH);
  const size_t both = lds_stash_offset(sys.nx, sys.nu, sizeof(T), BCH) + lf;
  const int per_cu = iter_min_blocks<T, Y, KP, NXL, FCH>() == 1 ? 1 : (sizeof(T) == 8 ? 2 : 3);
  const int stash = both <= (size_t)kLdsPerCu / per_cu ? 1 : 0;
  const size_t lds = stash ? both : std::max(lf, lb);
  hipError_t e = allow_lds(k_iter<T, Y, KP, NXL, BCH, FCH>, lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((k_iter<T, Y, KP, NXL, BCH, FCH>), dim3(n_items), dim3(kBlock), lds, s, sys, trees, items, ctab,
                     done_out, stash);
  return hipGetLastError();
}

template <typename T, int KP, int NXL, int BCH, typename Y>
hipError_t launch_iter_b(const SysDev<T>& sys, const TreeDev<T, Y>* trees, const WorkItem* items, int n_items,
                         const double* ctab, int fchunk, int32_t* done_out, hipStream_t s) {
  if (fchunk == 8) return launch_iter_ch<T, Y, KP, NXL, BCH, 8>(sys, trees, items, n_items, ctab, done_out, s);
  if constexpr (chunk_listed(Chunks<T>::fwd, 16))
    if (fchunk == 16) return launch_iter_ch<T, Y, KP, NXL, BCH, 16>(sys, trees, items, n_items, ctab, done_out, s);
  if constexpr (chunk_listed(Chunks<T>::fwd, 4))
    if (fchunk == 4) return launch_iter_ch<T, Y, KP, NXL, BCH, 4>(sys, trees, items, n_items, ctab, done_out, s);
  return hipErrorInvalidValue;
}

template <typename T, int KP, int NXL, typename Y>
hipError_t launch_iter_kp(const SysDev<T>& sys, const TreeDev<T, Y>* trees, const WorkItem* items, int n_items,
                          const double* ctab, int bchunk, int fchunk, int32_t* done_out, hipStream_t s) {
  if (bchunk == 16) return launch_iter_b<T, KP, NXL, 16>(sys, trees, items, n_items, ctab, fchunk, done_out, s);
  if constexpr (chunk_listed(Chunks<T>::bwd, 32))
    if (bchunk == 32) return launch_iter_b<T, KP, NXL, 32>(sys, trees, items, n_items, ctab, fchunk, done_out, s);
  return hipErrorInvalidValue;
}

template <typename T, typename Y>
hipError_t launch_iter(const SysDev<T>& sys, const TreeDev<T, Y>* trees, const WorkItem* items, int n_items,
                       const double* ctab, int bchunk, int fchunk, int32_t* done_out, hipStream_t s) {
  if (n_items <= 0) return hipSuccess;
  if (sys.nx > 128 || sys.nu > 128 || !chunk_listed(Chunks<T>::bwd, bchunk) || !chunk_listed(Chunks<T>::fwd, fchunk))
    return hipErrorInvalidValue;
  const bool x1 = sys.nx <= 64;
  if (sys.nu <= 64)
    return x1 ? launch_iter_kp<T, 64, 1>(sys, trees, items, n_items, ctab, bchunk, fchunk, done_out, s)
              : launch_iter_kp<T, 64, 2>(sys, trees, items, n_items, ctab, bchunk, fchunk, done_out, s);
  return x1 ? launch_iter_kp<T, 128, 1>(sys, trees, items, n_items, ctab, bchunk, fchunk, done_out, s)
            : launch_iter_kp<T, 128, 2>(sys, trees, items, n_items, ctab, bchunk, fchunk, done_out, s);
}

// Part 1: float64; part 2: float32; part 3: float32 solve steps on a float64
// dual (0: all of them).
#if SMPC_KERNEL_PART == 0 || SMPC_KERNEL_PART == 1
template hipError_t launch_iter<double, double>(const SysDev<double>&, const TreeDev<double, double>*,
                                                const WorkItem*, int, const double*, int, int, int32_t*, hipStream_t);
template hipError_t launch_backward<double, double>(const SysDev<double>&, const TreeDev<double, double>*,
                                                    const WorkItem*, int, const double*, int, int, hipStream_t);
template hipError_t launch_forward<double, double>(const SysDev<double>&, const TreeDev<double, double>*,
                                                   const WorkItem*, int, const double*, int, int, int32_t*,
                                                   hipStream_t);
#endif
#if SMPC_KERNEL_PART == 0 || SMPC_KERNEL_PART == 2
template hipError_t launch_iter<float, float>(const SysDev<float>&, const TreeDev<float, float>*, const WorkItem*,
                                              int, const double*, int, int, int32_t*, hipStream_t);
template hipError_t launch_backward<float, float>(const SysDev<float>&, const TreeDev<float, float>*,
                                                  const WorkItem*, int, const double*, int, int, hipStream_t);
template hipError_t launch_forward<float, float>(const SysDev<float>&, const TreeDev<float, float>*,
                                                 const WorkItem*, int, const double*, int, int, int32_t*,
                                                 hipStream_t);
#endif
#if SMPC_KERNEL_PART == 0 || SMPC_KERNEL_PART == 3
template hipError_t launch_iter<float, double>(const SysDev<float>&, const TreeDev<float, double>*, const WorkItem*,
                                               int, const double*, int, int, int32_t*, hipStream_t);
template hipError_t launch_backward<float, double>(const SysDev<float>&, const TreeDev<float, double>*,
                                                   const WorkItem*, int, const double*, int, int, hipStream_t);
template hipError_t launch_forward<float, double>(const SysDev<float>&, const TreeDev<float, double>*,
                                                  const WorkItem*, int, const double*, int, int, int32_t*,
                                                  hipStream_t);
#endif

template <typename T>
hipError_t launch_widen(const T* src, double* dst, size_t n, hipStream_t s) {
  if (n == 0) return hipSuccess;
  const unsigned blocks = (unsigned)((n + 255) / 256);
  hipLaunchKernelGGL(k_widen<T>, dim3(blocks), dim3(256), 0, s, src, dst, n);
  return hipGetLastError();
}

#if SMPC_KERNEL_PART == 0 || SMPC_KERNEL_PART == 1
template hipError_t launch_widen<float>(const float*, double*, size_t, hipStream_t);
#endif

template <typename Ts, typename Td>
hipError_t launch_shift(const Ts* src, Td* dst0, Td* dst2, const int32_t* src_node, const double* f, int M,
                        int nx, int nu, hipStream_t s) {
  const size_t n = (size_t)M * (2 * nx + nu);
  if (n == 0) return hipSuccess;
  const unsigned blocks = (unsigned)((n + 255) / 256);
  hipLaunchKernelGGL((k_shift<Ts, Td>), dim3(blocks), dim3(256), 0, s, src, dst0, dst2, src_node, f, M, nx, nu);
  return hipGetLastError();
}

#if SMPC_KERNEL_PART == 0 || SMPC_KERNEL_PART == 1
template hipError_t launch_shift<double, double>(const double*, double*, double*, const int32_t*, const double*,
                                                 int, int, int, hipStream_t);
template hipError_t launch_shift<double, float>(const double*, float*, float*, const int32_t*, const double*, int,
                                                int, int, hipStream_t);
template hipError_t launch_shift<float, double>(const float*, double*, double*, const int32_t*, const double*, int,
                                                int, int, hipStream_t);
template hipError_t launch_shift<float, float>(const float*, float*, float*, const int32_t*, const double*, int,
                                               int, int, hipStream_t);
#endif

}  // namespace smpc
