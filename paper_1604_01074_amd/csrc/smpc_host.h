// Host-side objects behind the C ABI handles.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <map>
#include <tuple>
#include <string>
#include <vector>

#include "../../include/smpc.h"
#include "smpc_internal.h"

namespace smpc {

// ----------------------------------------------------------------- errors
int set_error(int code, const char* fmt, ...);
const char* last_error_text();  // this thread's last message

// Propagate a HIP error as SMPC_EDEVICE, or a negative library status.
#define HIP_TRY(expr)                                                                      \
  do {                                                                                     \
    hipError_t e_ = (expr);                                                                \
    if (e_ != hipSuccess)                                                                  \
      return set_error(SMPC_EDEVICE, "%s failed: %s (%s:%d)", #expr, hipGetErrorString(e_), \
                       __FILE__, __LINE__);                                                \
  } while (0)

#define SMPC_TRY(expr)        \
  do {                        \
    int r_ = (expr);          \
    if (r_ < 0) return r_;    \
  } while (0)

// ----------------------------------------------------------------- dense FP64 helpers
// Row-major n x n Cholesky (lower factor in place).  False if a pivot is not
// positive relative to the largest diagonal entry.
bool cholesky(std::vector<double>& a, int n);
// Solve (L L') x = b in place for a factor from cholesky().
void chol_solve(const std::vector<double>& l, int n, double* b);

struct Csr {
  std::vector<int32_t> rp, ci;
  std::vector<double> v;
};
Csr dense_to_csr(const double* a, int rows, int cols);
Csr dense_to_csr_transposed(const double* a, int rows, int cols);

// ----------------------------------------------------------------- device buffers
struct DevBuf {
  void* ptr = nullptr;
  size_t bytes = 0;
};

struct ProfRec {
  const char* name;
  hipEvent_t a, b;
};

}  // namespace smpc

struct smpc_ctx {
  int device = 0;
  hipStream_t stream = nullptr;
  bool own_stream = false;
  size_t budget = 0;
  size_t used = 0;
  int n_sys = 0;
  // c_nu = theta_nu (1/theta_{nu-1} - 1) for nu = 0..ctab_len-1
  double* ctab = nullptr;
  int ctab_len = 0;
  // profiling
  bool profiling = false;
  std::vector<smpc::ProfRec> prof;
  std::vector<hipEvent_t> ev_pool;
  std::map<std::string, std::pair<int, double>> stats;
  int ctab_gen = 0;  // bumped whenever ctab is reallocated (captured graphs hold its address)
  std::vector<double> ctab_host;  // host copy of ctab
  // cached batch launch plan
  struct Plan* batch_plan = nullptr;

  int alloc(smpc::DevBuf& b, size_t bytes);
  void release(smpc::DevBuf& b);
  int ensure_ctab(int n);
  hipEvent_t get_event();
  void flush_profile();
};

template <typename T>
struct SysBuffers {
  smpc::DevBuf P, b_rp, b_ci, b_v, bt_rp, bt_ci, bt_v, a_rp, a_ci, a_v, at_rp, at_ci, at_v;
  smpc::DevBuf umin, umax, xmin, xmax, xs;
  smpc::SysDev<T> view{};
};

struct smpc_sys {
  smpc_ctx* ctx = nullptr;
  int nx = 0, nu = 0, nd = 0, ne = 0;
  std::vector<double> A, B, Gd, E, Ed, umin, umax, xmin, xmax, xs, alpha1, Wu;
  double W_alpha = 0, W_x = 0, gamma_d = 0;
  int safety_by_prob = 1;
  // tree-independent factor products
  std::vector<double> P;   // nu x nu:  L (L' Wu L)^{-1} L'
  std::vector<double> Mu;  // nu x nd:  uhat = Mu d (minimum-norm)
  smpc::Csr Bc, Btc, Ac, Atc;
  int a_identity = 0;
  SysBuffers<double> d64;
  SysBuffers<float> d32;
  // float64 matrices of the cost update and the objectives (dense Mu, Wu, Gd)
  smpc::DevBuf c_Mu, c_Wu, c_Gd, c_alpha1;
  smpc::CostSysDev cview{};
  bool has32 = false;
  int n_trees = 0;
  // chunk lengths {backward, forward} chosen by the last tuned solve, per
  // precision ([0] float64, [1] float32, [2] float32 solve steps on a
  // float64 dual); used by servers with tune 1
  int tuned_chunk[3][2] = {{0, 0}, {0, 0}, {0, 0}};
  bool has_tuned[3] = {false, false, false};
};

template <typename T>
struct TreeBuffers {
  smpc::DevBuf y[3], beta, uhat, e, pi, scale, p, du, z, ctopQ, ctopR;
  smpc::TreeDev<T> view{};
  bool allocated = false;
};

struct smpc_tree {
  smpc_sys* sys = nullptr;
  int N = 0, M = 0;
  std::vector<int32_t> stage, parent;
  std::vector<double> prob;
  // internal (chain-major) order
  std::vector<int32_t> perm;   // internal -> caller index
  std::vector<int32_t> iperm;  // caller -> internal index
  std::vector<smpc::ChainDesc> chains;
  int n_levels = 0;
  std::vector<int32_t> leaves;    // chains that end at a leaf
  std::vector<int32_t> path_off;  // per chain: range in `path`
  std::vector<int32_t> path;      // ancestor nodes of each leaf chain (root first); -1-node = owned
  std::vector<double> scale;  // M x 3 or empty
  bool has_data = false;
  bool factored = false;
  double lambda = 0.0;
  double lmax = 0.0;
  int power_steps = 0;  // power-iteration steps the last smpc_factor ran
  // device
  TreeBuffers<double> b64;
  TreeBuffers<float> b32;
  smpc::DevBuf cstat, st, chains_dev, cnt, leaves_dev, path_off_dev, path_dev;
  // node structure and inputs of the device cost update (internal order,
  // demands in the caller's order through perm)
  smpc::DevBuf n_stage, n_parent, n_crp, n_cci, n_perm, d_dev, a2_dev, q_dev, broot0;
  // objective partial sums (kObjSlots per workgroup) and results
  smpc::DevBuf obj_part, obj_out;
  bool obj_valid = false;  // obj_cache holds the objectives of the resident solve
  smpc_objective obj_cache{};
  struct Plan* plan = nullptr;  // single-tree launch plan
  // resident dual of the last solve (slot of y^{nu+1} and its precision;
  // -1 when no solve has left one), whether its last primal iterate is in
  // the float32 buffers, and a pending warm-start shift
  int res_slot = -1;
  int res_prec = 0;
  bool res_z32 = false;
  bool shift_ready = false;
  smpc::DevBuf shift_src, shift_f;  // per internal node: source node, 3 factors
};

// Launch plan: the work lists of one set of trees solved together.
struct Plan {
  std::vector<smpc_tree*> trees;
  int n_items = 0;  // leaf chains of all trees
  smpc::DevBuf items, td64, td32, tdmix, done;  // tdmix: float32 data, float64 dual
  std::vector<int32_t> done_host;
  // two pinned host copies of the stop flags and the events behind them
  // (made on the solve driver's first use): it reads one block's flags while
  // the next block runs
  int32_t* done_pinned = nullptr;
  hipEvent_t done_ev[2] = {nullptr, nullptr};
  bool has32 = false;
  // chunk lengths {backward, forward} in use per precision ([0] float64,
  // [1] float32) and whether they were chosen by timing
  int chunk[3][2] = {{0, 0}, {0, 0}, {0, 0}};
  bool tuned[3] = {false, false, false};
  // APG iterations as one fused launch each (forward nu + backward nu + 1);
  // bwd_ready: the backward of every tree's current iteration is done (set
  // by a backward launch or a fused launch, cleared whenever a tree of the
  // plan restarts or another mode runs on it)
  bool fused = true;
  bool bwd_ready[3] = {false, false, false};
  // instantiated graphs of `iters` iterations, keyed by (element size, mode,
  // iters, backward chunk, forward chunk)
  std::map<std::tuple<int, int, int, int, int, int>, hipGraphExec_t> graphs;
  int graphs_ctab_gen = -1;
};

namespace smpc {
// smpc_api.cpp: plans and the per-tree solve steps (shared with the server)
// The phases of a solve: run32 -- a first phase with float32 solve steps
// (mixed: on a float64 dual, else on a float32 dual), run64 -- float64
// iterations (the whole solve, or the polish / the finish after a stall).
struct SolvePhases {
  int polish = 0, max32 = 0;
  bool run32 = false, run64 = false, mixed = false;
};
// Launch-plan precision of a block of iterations: 0 float64, 1 float32,
// 2 float32 solve steps on a float64 dual.
enum { kPrec64 = 0, kPrec32 = 1, kPrecMix = 2 };
SolvePhases phases(const smpc_solve_opts* o);
int check_opts(const smpc_solve_opts* o);
int tree_check_ready(smpc_tree* t, bool need_data);
int prepare32(smpc_tree* t);
int plan_build(smpc_ctx* ctx, const std::vector<smpc_tree*>& trees, bool need32, Plan** out);
void plan_free(smpc_ctx* ctx, Plan* p);
int tree_begin(smpc_tree* t, const double* p, const double* q, const smpc_solve_opts* o, const double* y0,
               const double* yp0);
int tree_to_fp64(smpc_tree* t, const smpc_solve_opts* o, int fp32_iters, int status32);
int tree_result(smpc_tree* t, const smpc_solve_opts* o, int fp32_iters, int status32, smpc_result* r);
int read_state(smpc_tree* t, TreeState* h);
int run_block_prec(smpc_ctx* ctx, smpc_sys* sys, Plan* p, int prec, int iters, bool eager);
void choose_chunks(const smpc_sys* sys, const smpc_solve_opts* o, bool from_sys, int (&chunk)[3][2],
                   bool (&tuned)[3]);
void result_chunks(const int (&chunk)[3][2], const smpc_solve_opts* o, smpc_result* r);
int read_done(smpc_ctx* ctx, Plan* p);
int ensure_single_plan(smpc_tree* t, bool need32);
// Device bytes of a tree's float32 buffers and of a system's float32 copy,
// and the release of a tree's float32 buffers (with the plans that use them).
size_t tree32_bytes(const smpc_tree* t);
size_t sys32_bytes(const smpc_sys* s);
int tree_release32(smpc_tree* t);
CostTreeDev cost_tree_view(smpc_tree* t);
int upload_q(smpc_tree* t, const double* q);
int tree_objective(smpc_tree* t, double* part, double* out_dev, smpc_objective* out);
// The device address of the no-allocation objective scratch on the current
// device (smpc_data.hip): kObjSlots * (kObjMaxBlocks + 1) doubles.
hipError_t objective_scratch(double** ptr);

// smpc_setup.cpp
int sys_factor(smpc_sys* s);
void single_branch_precond(const smpc_sys* s, int N, std::vector<double>& diag);  // N x 3
}  // namespace smpc
