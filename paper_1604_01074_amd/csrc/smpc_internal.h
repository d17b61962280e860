// Internal data structures shared by the host library and the HIP kernels.
//
// Device layout (all node arrays in the library's internal "chain-major"
// order: the nodes of chain 0 top to bottom, then chain 1, ...; chains are
// numbered breadth-first so the child chains of a chain are consecutive):
//
//   y[3]    M x D      rotating dual iterates y^nu, y^{nu-1}, y^{nu+1}
//                      (D = 2 nx + nu; block order sigma~ | zeta~ | psi~)
//   beta    M x nu     linear cost of the input in u-space (see smpc_setup.cpp)
//   uhat    M x nu     particular solution of E u + Ed d = 0
//   e       M x nx     B uhat + Gd d
//   pi      M          node probability
//   scale   M x 3      optional dual scaling per (node, block)
//   du      M x nu     backward-pass output: input increment of the node
//   z       M x (nx+nu)  primal iterate (x_n, u_n), written on check steps
//   ctopQ/ctopR  per chain: state / input cost-to-go coefficients of the
//                chain's top node, read by the parent chain's bottom node
//   cstat   per leaf chain: 4 float64 reduction partials
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace smpc {

constexpr int kBlock = 256;      // threads per workgroup (4 wave64)
constexpr int kStat = 4;         // float64 partials per chain

enum Mode : int {
  kModeAPG = 0,     // one APG iteration (extrapolate, solve step, prox, update)
  kModeSolve = 1,   // solve step only at w = y[0]; writes z
  kModePower = 2,   // linear part of the dual gradient, for the power iteration
  kModeAny = -1,    // kernel template argument: the mode is a run-time argument
};

struct ChainDesc {
  int32_t first;        // internal index of the top node
  int32_t len;          // number of nodes
  int32_t parent;       // parent chain (-1 for the root chain)
  int32_t child_begin;  // first child chain
  int32_t child_count;  // number of child chains (0 for a leaf chain)
  int32_t height;       // 0 for leaf chains, 1 + max over children otherwise
};

struct WorkItem {
  int32_t tree;   // slot in the launch's tree table
  int32_t chain;  // chain id within that tree (a leaf chain)
  int32_t first;  // its first node (internal index) and length
  int32_t len;
  int32_t p0;     // its ancestor nodes: path[p0, p0 + plen)
  int32_t plen;
};

// Per-tree iteration state, resident on the device.  Written by the host
// before a solve and by k_iter_end between iterations.
struct TreeState {
  int32_t iter;         // index nu of the iteration being run
  int32_t done;         // 1 -> kernels skip this tree
  int32_t max_iter;     // stop after this many iterations
  int32_t check_every;  // residual test period
  int32_t status;       // 0 converged, 1 max_iter, 2 stalled, -9 diverged
  int32_t iters_done;   // iterations when the tree stopped
  int32_t fwd_count;    // leaf chains finished in the current forward kernel
  int32_t pad1;
  double tol;
  double lambda;
  double r_p;           // last ||Hz - t||_inf
  double hzt;           // last max(||Hz||_inf, ||t||_inf)
  double in_scale;      // power iteration: 1 / ||g_k||
  double lmax_est;      // power iteration: Rayleigh quotient
  double best_rp;       // smallest r_p seen at a check (stall detection)
  int32_t stall;        // checks since r_p last fell below 0.99 best_rp
  int32_t stall_limit;  // stop with status 2 after this many; 0 = never
};

template <typename T>
struct SysDev {
  int32_t nx, nu, D;
  int32_t a_identity;
  const T* P;            // p_stride(nu) x p_stride(nu), symmetric, zero-padded
  const int32_t* b_rp; const int32_t* b_ci; const T* b_v;     // B  (CSR)
  const int32_t* bt_rp; const int32_t* bt_ci; const T* bt_v;  // B' (CSR)
  const int32_t* a_rp; const int32_t* a_ci; const T* a_v;     // A  (CSR)
  const int32_t* at_rp; const int32_t* at_ci; const T* at_v;  // A' (CSR)
  const T* umin; const T* umax;
  const T* xmin; const T* xmax; const T* xs;
  double W_x, gamma_d;
  int32_t safety_by_prob;
  int32_t pad;
};

// T: precision of the solve step and the node data; Y: precision of the
// dual iterates (Y = T, or a float32 solve step on a float64 dual).
template <typename T, typename Y = T>
struct TreeDev {
  Y* y[3];
  const T* beta;
  const T* uhat;
  const T* e;
  const T* pi;
  const T* scale;   // nullptr -> no scaling
  const T* p;       // nx: state of the root's parent
  T* du;
  T* z;
  T* ctopQ;
  T* ctopR;
  double* cstat;
  const ChainDesc* chains;
  TreeState* st;
  int32_t* cnt;             // per chain: children whose backward sweep is done
  const int32_t* leaves;    // the tree's leaf chains (height 0)
  const int32_t* path_off;  // per chain: range of its ancestor nodes in `path`
  const int32_t* path;      // ancestor nodes (internal index), root first; < 0
                            // marks a node whose prox this leaf chain performs
                            // (-1 - node); every inner node has one such chain
  int32_t n_chains;
  int32_t n_leaves;
  int32_t M;
  int32_t pad;
};

// Chunk lengths (nodes per chunk) the kernels are instantiated for, per
// precision and kernel; the first entry is the default.  The chunk length
// only changes how many nodes are staged between barriers, never the order
// of the arithmetic, so every length gives bit-identical iterates.
template <typename T>
struct Chunks;
template <>
struct Chunks<float> {
  static constexpr int bwd[2] = {16, 32};
  static constexpr int fwd[2] = {8, 4};
};
template <>
struct Chunks<double> {
  static constexpr int bwd[2] = {16, 32};
  static constexpr int fwd[2] = {4, 8};
};
template <int N>
constexpr bool chunk_listed(const int (&a)[N], int v) {
  for (int i = 0; i < N; ++i)
    if (a[i] == v) return true;
  return false;
}

// Kernel launchers (smpc_kernels.hip).  `items` lists the leaf chains of all
// trees of the launch; `trees` is a device table.  One iteration is
// launch_backward then launch_forward (or, after one launch_backward, one
// launch_iter per iteration); `done_out[tree]` receives each tree's stop flag
// at the end of the forward rollout.  `chunk` must be listed in
// Chunks<T> (hipErrorInvalidValue otherwise).
// Instantiated for (T, Y) = (double, double), (float, float) and (float,
// double); the last one for the APG mode only.
template <typename T, typename Y>
hipError_t launch_backward(const SysDev<T>& sys, const TreeDev<T, Y>* trees, const WorkItem* items,
                           int n_items, const double* ctab, int mode, int chunk, hipStream_t s);
template <typename T, typename Y>
hipError_t launch_forward(const SysDev<T>& sys, const TreeDev<T, Y>* trees, const WorkItem* items,
                          int n_items, const double* ctab, int mode, int chunk, int32_t* done_out, hipStream_t s);
// One fused APG iteration (forward of iteration nu, then backward of
// iteration nu + 1); the launch before the first fused one of a run must be
// a launch_backward of the APG mode.
template <typename T, typename Y>
hipError_t launch_iter(const SysDev<T>& sys, const TreeDev<T, Y>* trees, const WorkItem* items, int n_items,
                       const double* ctab, int bchunk, int fchunk, int32_t* done_out, hipStream_t s);
template <typename T>
hipError_t launch_widen(const T* src, double* dst, size_t n, hipStream_t s);
// Warm-start shift: dst0 = dst2 = f * src gathered by node (per dual block
// factors f, M x 3, float64); src must not alias dst0 or dst2.
template <typename Ts, typename Td>
hipError_t launch_shift(const Ts* src, Td* dst0, Td* dst2, const int32_t* src_node, const double* f, int M,
                        int nx, int nu, hipStream_t s);

// ---------------------------------------------------------------------------
// Float64 node data and objective kernels (smpc_data.hip).
//
// System matrices of the cost update of App. A and of the objectives.
struct CostSysDev {
  int32_t nx, nu, nd;
  int32_t safety_by_prob;
  const double* Mu;      // nu x nd: uhat = Mu d (minimum-norm solution of E u + Ed d = 0)
  const double* Wu;      // nu x nu
  const double* Gd;      // nx x nd (dense)
  const int32_t* b_rp;   // B (CSR)
  const int32_t* b_ci;
  const double* b_v;
  const double* alpha1;  // nu
  const double* umin;
  const double* umax;
  const double* xmin;
  const double* xmax;
  const double* xs;
  double W_alpha, W_x, gamma_d;
};

// Per-tree node structure and inputs of the cost update, internal node order.
struct CostTreeDev {
  int32_t M, N;
  int32_t root;              // internal index of the root
  int32_t pad;
  const int32_t* stage;      // M
  const int32_t* parent;     // M: internal index of the parent, -1 for the root
  const int32_t* child_rp;   // M + 1: children of internal node n are
  const int32_t* child_ci;   //   child_ci[child_rp[n] .. child_rp[n + 1])
  const int32_t* perm;       // M: caller's index of internal node n
  const double* pi;          // M
  const double* d;           // M x nd demands, caller's node order
  const double* alpha2;      // N x nu pumping costs per stage
  const double* q;           // nu: input before the root (u_{a(root)})
  double* uhat;              // M x nu   outputs
  double* e;                 // M x nx
  double* beta;              // M x nu
  double* beta_root0;        // nu: the root's beta without its q term
  float* uhat32;             // float32 copies (nullptr: none)
  float* e32;
  float* beta32;
};

// Iterates of one solve for the objectives (float64, internal order).
struct ObjDev {
  const double* z;      // M x (nx + nu): x_n | u_n
  const double* yn;     // y^{nu+1} (scaled)
  const double* yc;     // y^nu
  const double* yp;     // y^{nu-1}
  const double* scale;  // M x 3
  double c;             // extrapolation coefficient of the last iteration
  double lam;           // step size
};

// Partial sums of the objective kernels: slots per workgroup and the
// workgroups of one launch at most (the scratch holds kObjSlots * blocks
// doubles plus kObjSlots results).
constexpr int kObjSlots = 8;
constexpr int kObjMaxBlocks = 1024;

// Cost update: uhat, e, beta (root without its q term) of every node, float64
// and, where the float32 pointers are set, float32.
hipError_t launch_cost_update(const CostSysDev& s, const CostTreeDev& t, hipStream_t st);
// The root's beta for the input q in t.q: beta_root0 - 2 pi_root Wu q.
hipError_t launch_root_beta(const CostSysDev& s, const CostTreeDev& t, hipStream_t st);
// Objectives at the iterates of a finished solve, reduced into out[0..7]:
// primal: [0] stage cost of u, [1] soft cost of t, [2] soft cost of x (t = Hz);
// dual (after a solve step at the unscaled dual, z = z(y)):
// [3] stage cost of u, [4] <y, H z>, [5] support function of the sets of g,
// [6] largest violation of dom g*.  `part` holds kObjSlots * blocks doubles.
hipError_t launch_objective(const CostSysDev& s, const CostTreeDev& t, const ObjDev& o, bool dual, double* part,
                            int blocks, double* out, hipStream_t st);
// dst = S src per dual block (M x (2 nx + nu), scale M x 3).
hipError_t launch_scale_dual(const double* src, double* dst, const double* scale, int M, int nx, int nu,
                             hipStream_t st);
hipError_t launch_narrow(const double* src, float* dst, size_t n, hipStream_t st);

// Row stride of the zero-padded P on the device (and of the staged rho rows),
// and the dynamic LDS of the two kernels.
__host__ __device__ inline int p_stride(int nu) { return nu <= 64 ? 64 : 128; }

__host__ __device__ inline size_t lds_bytes_backward(int nx, int nu, size_t elem, int chunk) {
  // the two Q parts of the chunk (2 x chunk x padded nx), rho transposed (P-stride
  // rows of chunk + 1 entries), -1/(2 pi) for two chunks, two Q carries
  // (general A), the chain-top exchange
  const size_t ch = (size_t)chunk;
  const size_t xs = nx <= 64 ? 64 : 128;
  return elem * (2 * ch * xs + (size_t)p_stride(nu) * (ch + 1) + 2 * ch + 3 * (size_t)nx);
}

// LDS per CU on gfx950, and where the forward layout starts when the fused
// iteration keeps the backward layout beside it (16-byte aligned).
constexpr size_t kLdsPerCu = 160 * 1024;
__host__ __device__ inline size_t lds_stash_offset(int nx, int nu, size_t elem, int chunk) {
  return (lds_bytes_backward(nx, nu, elem, chunk) + 15) & ~(size_t)15;
}

__host__ __device__ inline size_t lds_bytes_forward(int nx, int nu, size_t elem, int chunk) {
  // ut of two chunks (2 x chunk x padded nu), the scales of two chunks, the
  // x carries of waves 0 and 1 (general A), the per-node prox scalars of two
  // chunks (4 per node, room for float64), 32 float64 reduction slots
  const size_t ch = (size_t)chunk;
  return elem * (2 * ch * (size_t)p_stride(nu) + 8 * ch + 2 * (size_t)nx) + 8 * ch * sizeof(double) +
         32 * sizeof(double);
}


}  // namespace smpc
