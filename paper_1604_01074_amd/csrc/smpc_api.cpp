// C ABI of the scenario-tree SMPC solver: handles, validation, device buffers,
// chain decomposition of the tree, launch plans and the iteration driver.
#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <deque>
#include <iterator>
#include <new>
#include <string>
#include <vector>

#include "smpc_host.h"

using namespace smpc;

namespace {

thread_local std::string g_last_error;

}  // namespace

namespace smpc {

const char* last_error_text() { return g_last_error.c_str(); }

int set_error(int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_last_error = buf;
  return code;
}

}  // namespace smpc



// ------------------------------------------------------------------ context

int smpc_ctx::alloc(DevBuf& b, size_t bytes) {
  if (b.ptr && b.bytes == bytes) return SMPC_OK;
  release(b);
  if (bytes == 0) return SMPC_OK;
  if (budget && used + bytes > budget)
    return set_error(SMPC_ENOMEM, "HBM budget exceeded: %zu + %zu > %zu bytes", used, bytes, budget);
  hipError_t e = hipMalloc(&b.ptr, bytes);
  if (e != hipSuccess) {
    b.ptr = nullptr;
    return set_error(SMPC_ENOMEM, "hipMalloc(%zu) failed: %s", bytes, hipGetErrorString(e));
  }
  b.bytes = bytes;
  used += bytes;
  return SMPC_OK;
}

void smpc_ctx::release(DevBuf& b) {
  if (b.ptr) {
    (void)hipFree(b.ptr);
    used -= b.bytes;
  }
  b.ptr = nullptr;
  b.bytes = 0;
}

int smpc_ctx::ensure_ctab(int n) {
  if (n <= ctab_len) return SMPC_OK;
  int len = std::max(n, 2 * ctab_len);
  len = std::max(len, 1024);
  std::vector<double> h(len);
  // theta_0 = theta_{-1} = 1, theta_{k+1} = (sqrt(theta^4 + 4 theta^2) - theta^2) / 2
  double th_prev = 1.0, th = 1.0;
  for (int k = 0; k < len; ++k) {
    h[k] = th * (1.0 / th_prev - 1.0);
    const double nt = 0.5 * (std::sqrt(th * th * th * th + 4.0 * th * th) - th * th);
    th_prev = th;
    th = nt;
  }
  HIP_TRY(hipStreamSynchronize(stream));
  if (ctab) {
    (void)hipFree(ctab);
    used -= sizeof(double) * (size_t)ctab_len;
  }
  ctab = nullptr;
  ctab_len = 0;
  if (budget && used + sizeof(double) * len > budget) return set_error(SMPC_ENOMEM, "HBM budget exceeded");
  HIP_TRY(hipMalloc(&ctab, sizeof(double) * len));
  used += sizeof(double) * len;
  HIP_TRY(hipMemcpy(ctab, h.data(), sizeof(double) * len, hipMemcpyHostToDevice));
  ctab_host = h;
  ctab_len = len;
  ++ctab_gen;
  return SMPC_OK;
}

hipEvent_t smpc_ctx::get_event() {
  if (!ev_pool.empty()) {
    hipEvent_t e = ev_pool.back();
    ev_pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  (void)hipEventCreate(&e);
  return e;
}

void smpc_ctx::flush_profile() {
  if (prof.empty()) return;
  (void)hipStreamSynchronize(stream);
  for (auto& r : prof) {
    float ms = 0.f;
    (void)hipEventElapsedTime(&ms, r.a, r.b);
    auto& s = stats[r.name];
    s.first += 1;
    s.second += ms;
    ev_pool.push_back(r.a);
    ev_pool.push_back(r.b);
  }
  prof.clear();
}

// Library internals (declared in smpc_host.h where other sources use them).
namespace smpc {

// Bracket one launch with events when profiling is on.
template <typename F>
hipError_t timed(smpc_ctx* ctx, const char* name, F&& f) {
  if (!ctx->profiling) return f();
  hipEvent_t a = ctx->get_event(), b = ctx->get_event();
  (void)hipEventRecord(a, ctx->stream);
  hipError_t e = f();
  (void)hipEventRecord(b, ctx->stream);
  ctx->prof.push_back({name, a, b});
  if (ctx->prof.size() > 4096) ctx->flush_profile();
  return e;
}

bool all_finite(const double* p, size_t n) {
  for (size_t i = 0; i < n; ++i)
    if (!std::isfinite(p[i])) return false;
  return true;
}

template <typename T>
int upload(smpc_ctx* ctx, DevBuf& b, const double* src, size_t n) {
  SMPC_TRY(ctx->alloc(b, sizeof(T) * std::max<size_t>(n, 1)));
  if (n == 0) return SMPC_OK;
  std::vector<T> h(n);
  for (size_t i = 0; i < n; ++i) h[i] = (T)src[i];
  HIP_TRY(hipMemcpyAsync(b.ptr, h.data(), sizeof(T) * n, hipMemcpyHostToDevice, ctx->stream));
  HIP_TRY(hipStreamSynchronize(ctx->stream));
  return SMPC_OK;
}

int upload_i32(smpc_ctx* ctx, DevBuf& b, const std::vector<int32_t>& v) {
  SMPC_TRY(ctx->alloc(b, sizeof(int32_t) * std::max<size_t>(v.size(), 1)));
  if (v.empty()) return SMPC_OK;
  HIP_TRY(hipMemcpyAsync(b.ptr, v.data(), sizeof(int32_t) * v.size(), hipMemcpyHostToDevice, ctx->stream));
  HIP_TRY(hipStreamSynchronize(ctx->stream));
  return SMPC_OK;
}

template <typename T>
int sys_upload(smpc_sys* s, SysBuffers<T>& d) {
  smpc_ctx* ctx = s->ctx;
  {
    const int kp = p_stride(s->nu);
    std::vector<double> pp((size_t)kp * kp, 0.0);
    for (int i = 0; i < s->nu; ++i)
      for (int j = 0; j < s->nu; ++j) pp[(size_t)i * kp + j] = s->P[(size_t)i * s->nu + j];
    SMPC_TRY(upload<T>(ctx, d.P, pp.data(), pp.size()));
  }
  SMPC_TRY(upload_i32(ctx, d.b_rp, s->Bc.rp));
  SMPC_TRY(upload_i32(ctx, d.b_ci, s->Bc.ci));
  SMPC_TRY(upload<T>(ctx, d.b_v, s->Bc.v.data(), s->Bc.v.size()));
  SMPC_TRY(upload_i32(ctx, d.bt_rp, s->Btc.rp));
  SMPC_TRY(upload_i32(ctx, d.bt_ci, s->Btc.ci));
  SMPC_TRY(upload<T>(ctx, d.bt_v, s->Btc.v.data(), s->Btc.v.size()));
  SMPC_TRY(upload_i32(ctx, d.a_rp, s->Ac.rp));
  SMPC_TRY(upload_i32(ctx, d.a_ci, s->Ac.ci));
  SMPC_TRY(upload<T>(ctx, d.a_v, s->Ac.v.data(), s->Ac.v.size()));
  SMPC_TRY(upload_i32(ctx, d.at_rp, s->Atc.rp));
  SMPC_TRY(upload_i32(ctx, d.at_ci, s->Atc.ci));
  SMPC_TRY(upload<T>(ctx, d.at_v, s->Atc.v.data(), s->Atc.v.size()));
  SMPC_TRY(upload<T>(ctx, d.umin, s->umin.data(), s->nu));
  SMPC_TRY(upload<T>(ctx, d.umax, s->umax.data(), s->nu));
  SMPC_TRY(upload<T>(ctx, d.xmin, s->xmin.data(), s->nx));
  SMPC_TRY(upload<T>(ctx, d.xmax, s->xmax.data(), s->nx));
  SMPC_TRY(upload<T>(ctx, d.xs, s->xs.data(), s->nx));
  SysDev<T>& v = d.view;
  v.nx = s->nx;
  v.nu = s->nu;
  v.D = 2 * s->nx + s->nu;
  v.a_identity = s->a_identity;
  v.P = (const T*)d.P.ptr;
  v.b_rp = (const int32_t*)d.b_rp.ptr;
  v.b_ci = (const int32_t*)d.b_ci.ptr;
  v.b_v = (const T*)d.b_v.ptr;
  v.bt_rp = (const int32_t*)d.bt_rp.ptr;
  v.bt_ci = (const int32_t*)d.bt_ci.ptr;
  v.bt_v = (const T*)d.bt_v.ptr;
  v.a_rp = (const int32_t*)d.a_rp.ptr;
  v.a_ci = (const int32_t*)d.a_ci.ptr;
  v.a_v = (const T*)d.a_v.ptr;
  v.at_rp = (const int32_t*)d.at_rp.ptr;
  v.at_ci = (const int32_t*)d.at_ci.ptr;
  v.at_v = (const T*)d.at_v.ptr;
  v.umin = (const T*)d.umin.ptr;
  v.umax = (const T*)d.umax.ptr;
  v.xmin = (const T*)d.xmin.ptr;
  v.xmax = (const T*)d.xmax.ptr;
  v.xs = (const T*)d.xs.ptr;
  v.W_x = s->W_x;
  v.gamma_d = s->gamma_d;
  v.safety_by_prob = s->safety_by_prob;
  return SMPC_OK;
}

template <typename T>
void sys_free(smpc_ctx* ctx, SysBuffers<T>& d) {
  DevBuf* all[] = {&d.P, &d.b_rp, &d.b_ci, &d.b_v, &d.bt_rp, &d.bt_ci, &d.bt_v, &d.a_rp, &d.a_ci,
                   &d.a_v, &d.at_rp, &d.at_ci, &d.at_v, &d.umin, &d.umax, &d.xmin, &d.xmax, &d.xs};
  for (DevBuf* b : all) ctx->release(*b);
}

template <typename T>
SysBuffers<T>& sysbuf(smpc_sys* s);
template <>
SysBuffers<double>& sysbuf<double>(smpc_sys* s) { return s->d64; }
template <>
SysBuffers<float>& sysbuf<float>(smpc_sys* s) { return s->d32; }

template <typename T>
TreeBuffers<T>& treebuf(smpc_tree* t);
template <>
TreeBuffers<double>& treebuf<double>(smpc_tree* t) { return t->b64; }
template <>
TreeBuffers<float>& treebuf<float>(smpc_tree* t) { return t->b32; }

int ensure_sys32(smpc_sys* s) {
  if (s->has32) return SMPC_OK;
  SMPC_TRY(sys_upload<float>(s, s->d32));
  s->has32 = true;
  return SMPC_OK;
}

// Allocate the per-precision node buffers of a tree and upload what is known.
template <typename T>
int tree_upload_scale(smpc_tree* t);

template <typename T>
int tree_alloc(smpc_tree* t) {
  TreeBuffers<T>& b = treebuf<T>(t);
  smpc_ctx* ctx = t->sys->ctx;
  const size_t M = t->M, nx = t->sys->nx, nu = t->sys->nu, D = 2 * nx + nu, C = t->chains.size();
  if (!b.allocated) {
    for (int k = 0; k < 3; ++k) SMPC_TRY(ctx->alloc(b.y[k], sizeof(T) * M * D));
    SMPC_TRY(ctx->alloc(b.beta, sizeof(T) * M * nu));
    SMPC_TRY(ctx->alloc(b.uhat, sizeof(T) * M * nu));
    SMPC_TRY(ctx->alloc(b.e, sizeof(T) * M * nx));
    SMPC_TRY(ctx->alloc(b.pi, sizeof(T) * M));
    SMPC_TRY(ctx->alloc(b.scale, sizeof(T) * M * 3));
    SMPC_TRY(ctx->alloc(b.p, sizeof(T) * nx));
    SMPC_TRY(ctx->alloc(b.du, sizeof(T) * M * nu));
    SMPC_TRY(ctx->alloc(b.z, sizeof(T) * M * (nx + nu)));
    SMPC_TRY(ctx->alloc(b.ctopQ, sizeof(T) * C * nx));
    SMPC_TRY(ctx->alloc(b.ctopR, sizeof(T) * C * nu));
    for (int k = 0; k < 3; ++k) HIP_TRY(hipMemsetAsync(b.y[k].ptr, 0, sizeof(T) * M * D, ctx->stream));
    b.allocated = true;
    std::vector<double> pii(M);
    for (size_t i = 0; i < M; ++i) pii[i] = t->prob[t->perm[i]];
    SMPC_TRY(upload<T>(ctx, b.pi, pii.data(), M));
    SMPC_TRY(tree_upload_scale<T>(t));
  }
  TreeDev<T>& v = b.view;
  for (int k = 0; k < 3; ++k) v.y[k] = (T*)b.y[k].ptr;
  v.beta = (const T*)b.beta.ptr;
  v.uhat = (const T*)b.uhat.ptr;
  v.e = (const T*)b.e.ptr;
  v.pi = (const T*)b.pi.ptr;
  v.scale = (const T*)b.scale.ptr;  // ones when the tree is unscaled
  v.p = (const T*)b.p.ptr;
  v.du = (T*)b.du.ptr;
  v.z = (T*)b.z.ptr;
  v.ctopQ = (T*)b.ctopQ.ptr;
  v.ctopR = (T*)b.ctopR.ptr;
  v.cnt = (int32_t*)t->cnt.ptr;
  v.leaves = (const int32_t*)t->leaves_dev.ptr;
  v.path_off = (const int32_t*)t->path_off_dev.ptr;
  v.path = (const int32_t*)t->path_dev.ptr;
  v.n_leaves = (int32_t)t->leaves.size();
  v.cstat = (double*)t->cstat.ptr;
  v.chains = (const ChainDesc*)t->chains_dev.ptr;
  v.st = (TreeState*)t->st.ptr;
  v.n_chains = (int32_t)C;
  v.M = (int32_t)M;
  return SMPC_OK;
}

template <typename T>
void tree_free(smpc_ctx* ctx, TreeBuffers<T>& b) {
  DevBuf* all[] = {&b.y[0], &b.y[1], &b.y[2], &b.beta, &b.uhat, &b.e, &b.pi, &b.scale, &b.p,
                   &b.du, &b.z, &b.ctopQ, &b.ctopR};
  for (DevBuf* d : all) ctx->release(*d);
  b.allocated = false;
}

// The float32 copies of the node data from the float64 device buffers (the
// device cost update writes both precisions once the float32 buffers exist).
int tree_narrow_data(smpc_tree* t) {
  smpc_ctx* ctx = t->sys->ctx;
  const size_t M = t->M, nx = t->sys->nx, nu = t->sys->nu;
  HIP_TRY(launch_narrow((const double*)t->b64.beta.ptr, (float*)t->b32.beta.ptr, M * nu, ctx->stream));
  HIP_TRY(launch_narrow((const double*)t->b64.uhat.ptr, (float*)t->b32.uhat.ptr, M * nu, ctx->stream));
  HIP_TRY(launch_narrow((const double*)t->b64.e.ptr, (float*)t->b32.e.ptr, M * nx, ctx->stream));
  return SMPC_OK;
}

// The device scaling is always present: an unscaled tree holds ones, so the
// kernels multiply by it unconditionally (exactly).
template <typename T>
int tree_upload_scale(smpc_tree* t) {
  TreeBuffers<T>& b = treebuf<T>(t);
  if (t->scale.empty()) {
    const std::vector<double> ones((size_t)t->M * 3, 1.0);
    return upload<T>(t->sys->ctx, b.scale, ones.data(), ones.size());
  }
  return upload<T>(t->sys->ctx, b.scale, t->scale.data(), t->scale.size());
}

void plan_drop_graphs(Plan* p) {
  for (auto& kv : p->graphs) (void)hipGraphExecDestroy(kv.second);
  p->graphs.clear();
}

void plan_free(smpc_ctx* ctx, Plan* p) {
  if (!p) return;
  (void)hipStreamSynchronize(ctx->stream);
  plan_drop_graphs(p);
  ctx->release(p->items);
  ctx->release(p->td64);
  ctx->release(p->td32);
  ctx->release(p->tdmix);
  ctx->release(p->done);
  if (p->done_pinned) (void)hipHostFree(p->done_pinned);
  for (hipEvent_t& e : p->done_ev)
    if (e) (void)hipEventDestroy(e);
  delete p;
}

// The device view of a tree for float32 solve steps on its float64 dual: the
// float32 node data and work buffers with the float64 dual slots.
TreeDev<float, double> mixed_view(smpc_tree* t) {
  const TreeDev<float>& f = t->b32.view;
  TreeDev<float, double> m{};
  for (int k = 0; k < 3; ++k) m.y[k] = (double*)t->b64.y[k].ptr;
  m.beta = f.beta;
  m.uhat = f.uhat;
  m.e = f.e;
  m.pi = f.pi;
  m.scale = f.scale;
  m.p = f.p;
  m.du = f.du;
  m.z = f.z;
  m.ctopQ = f.ctopQ;
  m.ctopR = f.ctopR;
  m.cstat = f.cstat;
  m.chains = f.chains;
  m.st = f.st;
  m.cnt = f.cnt;
  m.leaves = f.leaves;
  m.path_off = f.path_off;
  m.path = f.path;
  m.n_chains = f.n_chains;
  m.n_leaves = f.n_leaves;
  m.M = f.M;
  return m;
}

// Build the launch plan of a set of trees: the leaf chains of all trees
// (longest first) and the device tree tables.
int plan_build(smpc_ctx* ctx, const std::vector<smpc_tree*>& trees, bool need32, Plan** out) {
  Plan* p = new (std::nothrow) Plan();
  if (!p) return set_error(SMPC_ENOMEM, "host allocation failed");
  p->trees = trees;
  std::vector<std::pair<int, WorkItem>> lv;
  for (size_t k = 0; k < trees.size(); ++k) {
    const smpc_tree* t = trees[k];
    for (int32_t c : t->leaves)
      lv.push_back({t->chains[c].len, WorkItem{(int32_t)k, c, t->chains[c].first, t->chains[c].len, t->path_off[c],
                                               t->path_off[c + 1] - t->path_off[c]}});
  }
  std::stable_sort(lv.begin(), lv.end(), [](const auto& a, const auto& b) { return a.first > b.first; });
  std::vector<WorkItem> items;
  for (auto& w : lv) items.push_back(w.second);
  p->n_items = (int)items.size();
  int rc = ctx->alloc(p->items, sizeof(WorkItem) * std::max<size_t>(items.size(), 1));
  if (rc >= 0) rc = ctx->alloc(p->done, sizeof(int32_t) * trees.size());
  if (rc < 0) { plan_free(ctx, p); return rc; }
  std::vector<TreeDev<double>> t64;
  std::vector<TreeDev<float>> t32;
  std::vector<TreeDev<float, double>> tmix;
  for (smpc_tree* t : trees) {
    t64.push_back(t->b64.view);
    if (need32) {
      t32.push_back(t->b32.view);
      tmix.push_back(mixed_view(t));
    }
  }
  rc = ctx->alloc(p->td64, sizeof(TreeDev<double>) * t64.size());
  if (rc >= 0 && need32) rc = ctx->alloc(p->td32, sizeof(TreeDev<float>) * t32.size());
  if (rc >= 0 && need32) rc = ctx->alloc(p->tdmix, sizeof(TreeDev<float, double>) * tmix.size());
  if (rc < 0) { plan_free(ctx, p); return rc; }
  hipStream_t s = ctx->stream;
  hipError_t e = hipSuccess;
  if (!items.empty()) e = hipMemcpyAsync(p->items.ptr, items.data(), sizeof(WorkItem) * items.size(), hipMemcpyHostToDevice, s);
  if (e == hipSuccess) e = hipMemcpyAsync(p->td64.ptr, t64.data(), sizeof(TreeDev<double>) * t64.size(), hipMemcpyHostToDevice, s);
  if (e == hipSuccess && need32) e = hipMemcpyAsync(p->td32.ptr, t32.data(), sizeof(TreeDev<float>) * t32.size(), hipMemcpyHostToDevice, s);
  if (e == hipSuccess && need32)
    e = hipMemcpyAsync(p->tdmix.ptr, tmix.data(), sizeof(TreeDev<float, double>) * tmix.size(), hipMemcpyHostToDevice, s);
  if (e == hipSuccess) e = hipMemsetAsync(p->done.ptr, 0, sizeof(int32_t) * trees.size(), s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) {
    plan_free(ctx, p);
    return set_error(SMPC_EDEVICE, "plan upload failed: %s", hipGetErrorString(e));
  }
  p->done_host.assign(trees.size(), 0);
  p->has32 = need32;
  p->chunk[0][0] = Chunks<double>::bwd[0];
  p->chunk[0][1] = Chunks<double>::fwd[0];
  p->chunk[1][0] = p->chunk[2][0] = Chunks<float>::bwd[0];
  p->chunk[1][1] = p->chunk[2][1] = Chunks<float>::fwd[0];
  *out = p;
  return SMPC_OK;
}

// The plan's device tree table for a (solve-step, dual) precision pair.
template <typename T, typename Y = T>
const TreeDev<T, Y>* plan_td(Plan* p) {
  if constexpr (sizeof(T) == 8) return (const TreeDev<T, Y>*)p->td64.ptr;
  if constexpr (sizeof(Y) == 8) return (const TreeDev<T, Y>*)p->tdmix.ptr;
  return (const TreeDev<T, Y>*)p->td32.ptr;
}

// Index of a precision pair in the per-plan tables: 0 float64, 1 float32,
// 2 float32 solve steps on a float64 dual.
template <typename T, typename Y = T>
constexpr int pix() {
  return sizeof(T) == 8 ? 0 : (sizeof(Y) == 8 ? 2 : 1);
}

template <typename T, typename Y = T>
const char* kname(int which) {
  static const char* names[3][3] = {{"backward_f64", "forward_f64", "iter_f64"},
                                    {"backward_f32", "forward_f32", "iter_f32"},
                                    {"backward_mix", "forward_mix", "iter_mix"}};
  return names[pix<T, Y>()][which];
}

// Enqueue one iteration of `mode` for every tree of the plan: the backward
// sweep over all chains, then the forward rollout with prox and the per-tree
// end of iteration -- or, for fused APG iterations, one launch that runs the
// forward rollout of this iteration and the backward sweep of the next (the
// caller has run the backward of the first one, see ensure_backward).
template <typename T, typename Y = T>
int enqueue_iteration(smpc_ctx* ctx, smpc_sys* sys, Plan* p, int mode) {
  const SysDev<T>& sv = sysbuf<T>(sys).view;
  const TreeDev<T, Y>* td = plan_td<T, Y>(p);
  const WorkItem* items = (const WorkItem*)p->items.ptr;
  hipStream_t s = ctx->stream;
  const int* ch = p->chunk[pix<T, Y>()];
  if (mode == kModeAPG && p->fused) {
    // forward of this iteration and backward of the next in one launch
    HIP_TRY(timed(ctx, kname<T, Y>(2), [&] {
      return launch_iter<T, Y>(sv, td, items, p->n_items, ctx->ctab, ch[0], ch[1], (int32_t*)p->done.ptr, s);
    }));
    return SMPC_OK;
  }
  HIP_TRY(timed(ctx, kname<T, Y>(0),
                [&] { return launch_backward<T, Y>(sv, td, items, p->n_items, ctx->ctab, mode, ch[0], s); }));
  HIP_TRY(timed(ctx, kname<T, Y>(1), [&] {
    return launch_forward<T, Y>(sv, td, items, p->n_items, ctx->ctab, mode, ch[1], (int32_t*)p->done.ptr, s);
  }));
  p->bwd_ready[pix<T, Y>()] = false;  // the next iteration starts with its backward
  return SMPC_OK;
}

// Before fused APG iterations: the backward of every tree's current
// iteration (one backward launch, outside any captured graph).
template <typename T, typename Y = T>
int ensure_backward(smpc_ctx* ctx, smpc_sys* sys, Plan* p) {
  if (!p->fused || p->bwd_ready[pix<T, Y>()]) return SMPC_OK;
  const SysDev<T>& sv = sysbuf<T>(sys).view;
  HIP_TRY(timed(ctx, kname<T, Y>(0), [&] {
    return launch_backward<T, Y>(sv, plan_td<T, Y>(p), (const WorkItem*)p->items.ptr, p->n_items, ctx->ctab,
                                 kModeAPG, p->chunk[pix<T, Y>()][0], ctx->stream);
  }));
  p->bwd_ready[pix<T, Y>()] = true;
  return SMPC_OK;
}

// Enqueue `iters` iterations.  Without profiling they are captured once into a
// hipGraph per (precision, mode, iters, chunk lengths) and replayed: the kernels take every
// per-iteration quantity from the device-side tree state, so one graph serves
// every block of a solve.
template <typename T, typename Y = T>
int run_block(smpc_ctx* ctx, smpc_sys* sys, Plan* p, int mode, int iters) {
  if (mode == kModeAPG) SMPC_TRY((ensure_backward<T, Y>(ctx, sys, p)));
  if (ctx->profiling) {
    for (int k = 0; k < iters; ++k) SMPC_TRY((enqueue_iteration<T, Y>(ctx, sys, p, mode)));
    return SMPC_OK;
  }
  if (p->graphs_ctab_gen != ctx->ctab_gen) {
    plan_drop_graphs(p);
    p->graphs_ctab_gen = ctx->ctab_gen;
  }
  const int* ch = p->chunk[pix<T, Y>()];
  const auto key = std::make_tuple(pix<T, Y>(), mode, iters, ch[0], ch[1], (int)(mode == kModeAPG && p->fused));
  auto found = p->graphs.find(key);
  if (found == p->graphs.end()) {
    HIP_TRY(hipStreamBeginCapture(ctx->stream, hipStreamCaptureModeThreadLocal));
    int rc = SMPC_OK;
    for (int k = 0; k < iters && rc >= 0; ++k) rc = enqueue_iteration<T, Y>(ctx, sys, p, mode);
    hipGraph_t graph = nullptr;
    hipError_t e = hipStreamEndCapture(ctx->stream, &graph);
    if (rc < 0) {
      if (graph) (void)hipGraphDestroy(graph);
      return rc;
    }
    if (e != hipSuccess) return set_error(SMPC_EDEVICE, "graph capture failed: %s", hipGetErrorString(e));
    hipGraphExec_t exec = nullptr;
    e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (e != hipSuccess) return set_error(SMPC_EDEVICE, "graph instantiation failed: %s", hipGetErrorString(e));
    found = p->graphs.emplace(key, exec).first;
  }
  HIP_TRY(hipGraphLaunch(found->second, ctx->stream));
  if (!(mode == kModeAPG && p->fused)) p->bwd_ready[pix<T, Y>()] = false;
  return SMPC_OK;
}

bool plan_all_done(const Plan* p) {
  for (int32_t d : p->done_host)
    if (!d) return false;
  return true;
}

int read_done(smpc_ctx* ctx, Plan* p) {
  HIP_TRY(hipMemcpyAsync(p->done_host.data(), p->done.ptr, sizeof(int32_t) * p->trees.size(), hipMemcpyDeviceToHost,
                         ctx->stream));
  HIP_TRY(hipStreamSynchronize(ctx->stream));
  return SMPC_OK;
}

// Stop flags through pinned slot `slot`: the copy behind the work enqueued so
// far, and the wait for it.  The two slots and their events are made on the
// plan's first use (plan_free releases them).
int ensure_done_slots(Plan* p) {
  if (!p->done_pinned)
    HIP_TRY(hipHostMalloc((void**)&p->done_pinned, 2 * sizeof(int32_t) * std::max<size_t>(p->trees.size(), 1)));
  for (hipEvent_t& ev : p->done_ev)
    if (!ev) HIP_TRY(hipEventCreateWithFlags(&ev, hipEventDisableTiming));
  return SMPC_OK;
}

int copy_done(smpc_ctx* ctx, Plan* p, int slot) {
  const size_t nt = p->trees.size();
  HIP_TRY(hipMemcpyAsync(p->done_pinned + slot * nt, p->done.ptr, sizeof(int32_t) * nt, hipMemcpyDeviceToHost,
                         ctx->stream));
  HIP_TRY(hipEventRecord(p->done_ev[slot], ctx->stream));
  return SMPC_OK;
}

int wait_done(Plan* p, int slot) {
  const size_t nt = p->trees.size();
  HIP_TRY(hipEventSynchronize(p->done_ev[slot]));
  std::copy(p->done_pinned + slot * nt, p->done_pinned + (slot + 1) * nt, p->done_host.begin());
  return SMPC_OK;
}

// Chunk-length autotuner: run the plan's next APG blocks with each listed
// (backward, forward) pair in turn -- one block to instantiate its graph and
// load its code, then two timed blocks -- and keep the pair with the
// shortest block.  The blocks are iterations of the running solve (the chunk
// length does not change the iterates).  Consumes up to 3 x pairs blocks of
// `rounds`; leaves the plan untuned when every tree stops first.
template <typename T, typename Y = T>
int tune_chunks(smpc_ctx* ctx, smpc_sys* sys, Plan* p, int iters, int max_rounds, int& rounds) {
  constexpr int K = pix<T, Y>();
  int* ch = p->chunk[K];
  hipEvent_t ev[2] = {nullptr, nullptr};
  HIP_TRY(hipEventCreate(&ev[0]));
  hipError_t e = hipEventCreate(&ev[1]);
  if (e != hipSuccess) {
    (void)hipEventDestroy(ev[0]);
    return set_error(SMPC_EDEVICE, "event creation failed: %s", hipGetErrorString(e));
  }
  int rc = SMPC_OK;
  float best = HUGE_VALF;
  int best_b = ch[0], best_f = ch[1];
  bool complete = true;
  for (int b : Chunks<T>::bwd) {
    for (int f : Chunks<T>::fwd) {
      ch[0] = b;
      ch[1] = f;
      float ms = HUGE_VALF;
      for (int rep = 0; rep < 3 && complete && rc >= 0; ++rep) {
        if (rounds >= max_rounds || plan_all_done(p)) {
          complete = false;
          break;
        }
        const bool timed_block = rep > 0;
        if (timed_block) e = hipEventRecord(ev[0], ctx->stream);
        if (e == hipSuccess) rc = run_block<T, Y>(ctx, sys, p, kModeAPG, iters);
        if (rc >= 0 && timed_block && e == hipSuccess) e = hipEventRecord(ev[1], ctx->stream);
        if (rc >= 0 && e == hipSuccess) rc = read_done(ctx, p);
        if (rc >= 0 && timed_block && e == hipSuccess) {
          float t = 0.f;
          e = hipEventElapsedTime(&t, ev[0], ev[1]);
          ms = std::min(ms, t);
        }
        if (e != hipSuccess && rc >= 0) rc = set_error(SMPC_EDEVICE, "autotune timing failed: %s", hipGetErrorString(e));
        ++rounds;
      }
      if (!complete || rc < 0) break;
      if (ms < best) {
        best = ms;
        best_b = b;
        best_f = f;
      }
    }
    if (!complete || rc < 0) break;
  }
  (void)hipEventDestroy(ev[0]);
  (void)hipEventDestroy(ev[1]);
  SMPC_TRY(rc);
  ch[0] = best_b;
  ch[1] = best_f;
  if (complete) {
    p->tuned[K] = true;
    sys->tuned_chunk[K][0] = best_b;
    sys->tuned_chunk[K][1] = best_f;
    sys->has_tuned[K] = true;
  }
  return SMPC_OK;
}

// Run APG iterations until every tree of the plan is done (after tuning the
// chunk lengths first when `tune` is set and the plan has no tuned pair).
template <typename T, typename Y = T>
int run_until_done(smpc_ctx* ctx, smpc_sys* sys, Plan* p, int check_every, int max_rounds, bool tune) {
  int round = 0;
  std::fill(p->done_host.begin(), p->done_host.end(), 0);
  if (tune && !p->tuned[pix<T, Y>()]) SMPC_TRY((tune_chunks<T, Y>(ctx, sys, p, check_every, max_rounds, round)));
  if (plan_all_done(p)) return SMPC_OK;
  if (round >= max_rounds) return set_error(SMPC_EDEVICE, "iteration driver did not terminate");
  // Blocks run one ahead of the host's read of the stop flags: the flags
  // behind block k are copied to pinned memory, block k + 1 is enqueued, and
  // only then does the host wait for the copy, so the device does not idle
  // while the host reads them.  A block enqueued after every tree has stopped
  // changes nothing (each kernel returns at once for a stopped tree) and is
  // ordered before whatever the caller enqueues next.
  SMPC_TRY(ensure_done_slots(p));
  int slot = 0;
  SMPC_TRY((run_block<T, Y>(ctx, sys, p, kModeAPG, check_every)));
  SMPC_TRY(copy_done(ctx, p, slot));
  for (++round;; ++round) {
    const bool more = round < max_rounds;
    if (more) SMPC_TRY((run_block<T, Y>(ctx, sys, p, kModeAPG, check_every)));
    SMPC_TRY(wait_done(p, slot));  // the flags behind the previous block
    if (plan_all_done(p)) return SMPC_OK;
    if (!more) break;
    slot ^= 1;
    SMPC_TRY(copy_done(ctx, p, slot));
  }
  return set_error(SMPC_EDEVICE, "iteration driver did not terminate");
}

int read_state(smpc_tree* t, TreeState* h) {
  HIP_TRY(hipMemcpyAsync(h, t->st.ptr, sizeof(TreeState), hipMemcpyDeviceToHost, t->sys->ctx->stream));
  HIP_TRY(hipStreamSynchronize(t->sys->ctx->stream));
  return SMPC_OK;
}

int write_state(smpc_tree* t, const TreeState& h) {
  HIP_TRY(hipMemcpyAsync(t->st.ptr, &h, sizeof(TreeState), hipMemcpyHostToDevice, t->sys->ctx->stream));
  HIP_TRY(hipStreamSynchronize(t->sys->ctx->stream));
  return SMPC_OK;
}

// Per-solve input of one precision: the root parent state p.
template <typename T>
int upload_root(smpc_tree* t, const double* p) {
  TreeBuffers<T>& b = treebuf<T>(t);
  smpc_ctx* ctx = t->sys->ctx;
  const int nx = t->sys->nx;
  std::vector<T> hp(nx);
  for (int i = 0; i < nx; ++i) hp[i] = (T)p[i];
  HIP_TRY(hipMemcpyAsync(b.p.ptr, hp.data(), sizeof(T) * nx, hipMemcpyHostToDevice, ctx->stream));
  HIP_TRY(hipStreamSynchronize(ctx->stream));
  return SMPC_OK;
}

// Warm start from the resident dual of the previous solve, shifted by the
// map prepared by smpc_shift_warm_start: y^0 = y^{-1} -> y[0], y[2] of the
// precision T of the coming phase.
template <typename Ts, typename Td>
int shift_resident(smpc_tree* t) {
  smpc_ctx* ctx = t->sys->ctx;
  const int nx = t->sys->nx, nu = t->sys->nu, D = 2 * nx + nu, M = t->M;
  TreeBuffers<Ts>& bs = treebuf<Ts>(t);
  TreeBuffers<Td>& bd = treebuf<Td>(t);
  const Ts* src = (const Ts*)bs.y[t->res_slot].ptr;
  if ((const void*)src == bd.y[0].ptr || (const void*)src == bd.y[2].ptr) {
    // the gather reads other nodes than it writes: move the source to the
    // free slot first (slot 1 is overwritten by the first iteration anyway)
    HIP_TRY(hipMemcpyAsync(bs.y[1].ptr, src, sizeof(Ts) * (size_t)M * D, hipMemcpyDeviceToDevice, ctx->stream));
    src = (const Ts*)bs.y[1].ptr;
  }
  hipError_t (*shift)(const Ts*, Td*, Td*, const int32_t*, const double*, int, int, int, hipStream_t) =
      launch_shift<Ts, Td>;
  HIP_TRY(shift(src, (Td*)bd.y[0].ptr, (Td*)bd.y[2].ptr, (const int32_t*)t->shift_src.ptr,
                (const double*)t->shift_f.ptr, M, nx, nu, ctx->stream));
  return SMPC_OK;
}

template <typename Td>
int start_from_resident(smpc_tree* t) {
  if (t->res_prec == 32) return shift_resident<float, Td>(t);
  return shift_resident<double, Td>(t);
}

// Initial dual iterates (scaled, internal order): y^0 -> y[0], y^{-1} -> y[2].
template <typename T>
int upload_dual_start(smpc_tree* t, const double* y0, const double* yprev0) {
  TreeBuffers<T>& b = treebuf<T>(t);
  smpc_ctx* ctx = t->sys->ctx;
  const int nx = t->sys->nx, nu = t->sys->nu, D = 2 * nx + nu, M = t->M;
  if (!y0) {
    HIP_TRY(hipMemsetAsync(b.y[0].ptr, 0, sizeof(T) * M * D, ctx->stream));
    HIP_TRY(hipMemsetAsync(b.y[2].ptr, 0, sizeof(T) * M * D, ctx->stream));
    return SMPC_OK;
  }
  std::vector<T> h((size_t)M * D);
  for (int pass = 0; pass < 2; ++pass) {
    const double* src = pass == 0 ? y0 : (yprev0 ? yprev0 : y0);
    for (int in = 0; in < M; ++in) {
      const int n = t->perm[in];
      for (int k = 0; k < D; ++k) {
        const int blk = k < nx ? 0 : (k < 2 * nx ? 1 : 2);
        const double s = t->scale.empty() ? 1.0 : t->scale[(size_t)in * 3 + blk];
        h[(size_t)in * D + k] = (T)(src[(size_t)n * D + k] / s);
      }
    }
    HIP_TRY(hipMemcpyAsync(b.y[pass == 0 ? 0 : 2].ptr, h.data(), sizeof(T) * M * D, hipMemcpyHostToDevice, ctx->stream));
    HIP_TRY(hipStreamSynchronize(ctx->stream));
  }
  return SMPC_OK;
}

template <typename T>
int download_primal(smpc_tree* t, double* x, double* u, double* u0) {
  TreeBuffers<T>& b = treebuf<T>(t);
  smpc_ctx* ctx = t->sys->ctx;
  const int nx = t->sys->nx, nu = t->sys->nu, M = t->M, nz = nx + nu;
  std::vector<T> h;
  if (x || u) {
    h.resize((size_t)M * nz);
    HIP_TRY(hipMemcpyAsync(h.data(), b.z.ptr, sizeof(T) * h.size(), hipMemcpyDeviceToHost, ctx->stream));
    HIP_TRY(hipStreamSynchronize(ctx->stream));
    for (int in = 0; in < M; ++in) {
      const int n = t->perm[in];
      if (x)
        for (int i = 0; i < nx; ++i) x[(size_t)n * nx + i] = (double)h[(size_t)in * nz + i];
      if (u)
        for (int j = 0; j < nu; ++j) u[(size_t)n * nu + j] = (double)h[(size_t)in * nz + nx + j];
    }
    if (u0) {
      const int r = t->iperm[0];
      for (int j = 0; j < nu; ++j) u0[j] = (double)h[(size_t)r * nz + nx + j];
    }
  } else if (u0) {
    std::vector<T> hr(nu);
    const size_t r = (size_t)t->iperm[0];
    HIP_TRY(hipMemcpyAsync(hr.data(), (T*)b.z.ptr + r * nz + nx, sizeof(T) * nu, hipMemcpyDeviceToHost, ctx->stream));
    HIP_TRY(hipStreamSynchronize(ctx->stream));
    for (int j = 0; j < nu; ++j) u0[j] = (double)hr[j];
  }
  return SMPC_OK;
}

template <typename T>
int download_dual(smpc_tree* t, int slot, double* y) {
  TreeBuffers<T>& b = treebuf<T>(t);
  smpc_ctx* ctx = t->sys->ctx;
  const int nx = t->sys->nx, nu = t->sys->nu, D = 2 * nx + nu, M = t->M;
  std::vector<T> h((size_t)M * D);
  HIP_TRY(hipMemcpyAsync(h.data(), b.y[slot].ptr, sizeof(T) * h.size(), hipMemcpyDeviceToHost, ctx->stream));
  HIP_TRY(hipStreamSynchronize(ctx->stream));
  for (int in = 0; in < M; ++in) {
    const int n = t->perm[in];
    for (int k = 0; k < D; ++k) {
      const int blk = k < nx ? 0 : (k < 2 * nx ? 1 : 2);
      const double s = t->scale.empty() ? 1.0 : t->scale[(size_t)in * 3 + blk];
      y[(size_t)n * D + k] = s * (double)h[(size_t)in * D + k];
    }
  }
  return SMPC_OK;
}

int check_opts(const smpc_solve_opts* o) {
  if (!o) return set_error(SMPC_EINVAL, "opts is NULL");
  if (o->max_iter < 1) return set_error(SMPC_EINVAL, "max_iter must be >= 1");
  if (o->check_every < 1) return set_error(SMPC_EINVAL, "check_every must be >= 1");
  if (o->precision != 64 && o->precision != 32) return set_error(SMPC_EINVAL, "precision must be 32 or 64");
  if (o->polish_iters < 0 || o->polish_iters > o->max_iter) return set_error(SMPC_EINVAL, "polish_iters out of range");
  if (!(o->tol >= 0.0) || !std::isfinite(o->tol)) return set_error(SMPC_EINVAL, "tol must be finite and >= 0");
  if (o->warm_start < 0 || o->warm_start > 2) return set_error(SMPC_EINVAL, "warm_start must be 0, 1 or 2");
  if (o->warm_start == 2 && !o->y0) return set_error(SMPC_EINVAL, "warm_start 2 needs y0");
  if (o->tune != 0 && o->tune != 1) return set_error(SMPC_EINVAL, "tune must be 0 or 1");
  if (o->dual64 != 0 && o->dual64 != 1) return set_error(SMPC_EINVAL, "dual64 must be 0 or 1");
  if (o->gap != 0 && o->gap != 1) return set_error(SMPC_EINVAL, "gap must be 0 or 1");
  for (int w = 0; w < 2; ++w) {
    if (o->chunk32[w] != 0 && !(w == 0 ? chunk_listed(Chunks<float>::bwd, o->chunk32[w])
                                       : chunk_listed(Chunks<float>::fwd, o->chunk32[w])))
      return set_error(SMPC_EINVAL, "chunk32[%d] = %d is not a built chunk length", w, o->chunk32[w]);
    if (o->chunk64[w] != 0 && !(w == 0 ? chunk_listed(Chunks<double>::bwd, o->chunk64[w])
                                       : chunk_listed(Chunks<double>::fwd, o->chunk64[w])))
      return set_error(SMPC_EINVAL, "chunk64[%d] = %d is not a built chunk length", w, o->chunk64[w]);
  }
  return SMPC_OK;
}

// Solve a set of trees (one plan) with the given options.
// ---------------------------------------------------------------- per-tree solve steps
// (shared by the batched solve and the server, so that both run the same
// arithmetic for a tree)

int stall_limit32(const smpc_solve_opts* o) {
  // a fixed iteration count (tol = 0) is never cut short; on a float64 dual
  // the float32 phase has no storage floor, so the rule applies only when
  // asked for explicitly
  if (o->tol <= 0.0 || o->stall_checks < 0) return 0;
  if (o->precision == 32 && o->dual64) return o->stall_checks;
  return o->stall_checks == 0 ? 100 : o->stall_checks;
}

// A float64 solve (precision 64) stops on a stall only when asked for
// (stall_checks > 0): its r_p has no storage floor, so a stall means no
// progress at all, as with an infeasible coupling, whose dual grows without
// bound.  (The float64 finish after a float32 stall runs to the stop test:
// the float32 window is short by design.)
int stall_limit64(const smpc_solve_opts* o) {
  return (o->tol > 0.0 && o->stall_checks > 0) ? o->stall_checks : 0;
}

int init_tree_state(smpc_tree* t, const smpc_solve_opts* o, int iter, int max_iter, double tol, int stall_limit) {
  TreeState h{};
  h.iter = iter;
  h.done = 0;
  h.max_iter = max_iter;
  h.check_every = o->check_every;
  h.status = 0;
  h.iters_done = 0;
  h.tol = tol;
  h.lambda = t->lambda;
  h.in_scale = 1.0;
  h.best_rp = HUGE_VAL;
  h.stall = 0;
  h.stall_limit = stall_limit;
  return write_state(t, h);
}

SolvePhases phases(const smpc_solve_opts* o) {
  SolvePhases ph;
  const bool use32 = o->precision == 32;
  ph.polish = use32 ? o->polish_iters : 0;
  ph.max32 = o->max_iter - ph.polish;
  ph.run32 = use32 && ph.max32 > 0;
  ph.run64 = !use32 || ph.polish > 0;
  ph.mixed = ph.run32 && o->dual64;
  return ph;
}

// Root data, dual start (y0 / y_prev0 for warm_start 2, the resident shifted
// dual for warm_start 1) and the state of the first phase.
int tree_begin(smpc_tree* t, const double* p, const double* q, const smpc_solve_opts* o, const double* y0,
               const double* yp0) {
  const SolvePhases ph = phases(o);
  SMPC_TRY(upload_root<double>(t, p));
  if (ph.run32) SMPC_TRY(upload_root<float>(t, p));
  SMPC_TRY(upload_q(t, q));
  if (o->warm_start == 1) {
    if (ph.run32 && !ph.mixed) SMPC_TRY(start_from_resident<float>(t));
    else SMPC_TRY(start_from_resident<double>(t));
    t->shift_ready = false;
  } else if (ph.run32 && !ph.mixed) {
    SMPC_TRY(upload_dual_start<float>(t, y0, yp0));
  } else {
    SMPC_TRY(upload_dual_start<double>(t, y0, yp0));
  }
  if (ph.run32) return init_tree_state(t, o, 0, ph.max32, o->tol, stall_limit32(o));
  return init_tree_state(t, o, 0, o->max_iter, o->tol, stall_limit64(o));
}

// After the float32 phase: continue in float64 from the float32 iterates
// (all three slots) -- polish after the stop test or the float32 budget, run
// on to the stop test after a stall (status 2), or record the divergence.
int tree_to_fp64(smpc_tree* t, const smpc_solve_opts* o, int fp32_iters, int status32) {
  smpc_ctx* ctx = t->sys->ctx;
  const SolvePhases ph = phases(o);
  const int D = 2 * t->sys->nx + t->sys->nu;
  if (!ph.mixed)  // (a float64 dual is already in place)
    for (int s = 0; s < 3; ++s)
      HIP_TRY(launch_widen<float>((const float*)t->b32.y[s].ptr, (double*)t->b64.y[s].ptr, (size_t)t->M * D,
                                  ctx->stream));
  if (status32 == -9) {
    SMPC_TRY(init_tree_state(t, o, fp32_iters, fp32_iters, 0.0, 0));
    TreeState h;
    SMPC_TRY(read_state(t, &h));
    h.done = 1;
    h.status = -9;
    h.iters_done = fp32_iters;
    return write_state(t, h);
  }
  if (status32 == 2) return init_tree_state(t, o, fp32_iters, o->max_iter, o->tol, 0);
  return init_tree_state(t, o, fp32_iters, fp32_iters + ph.polish, 0.0, 0);
}

// Final state of a tree: keep its last dual resident and fill `r` (may be
// NULL; outputs are downloaded when their pointers are set).
int tree_result(smpc_tree* t, const smpc_solve_opts* o, int fp32_iters, int status32, smpc_result* r) {
  const SolvePhases ph = phases(o);
  TreeState h;
  SMPC_TRY(read_state(t, &h));
  // the final dual y^{nu+1} stays resident for a shifted warm start
  t->res_slot = h.iters_done % 3;
  t->res_prec = (ph.run64 || ph.mixed) ? 64 : 32;
  t->res_z32 = !ph.run64;
  t->obj_valid = false;
  if (!r) return SMPC_OK;
  r->iterations = h.iters_done;
  r->fp32_iterations = ph.run32 ? fp32_iters : 0;
  r->r_primal = h.r_p;
  r->hz_t_max = h.hzt;
  // device status: 0 stop test passed, 1 iteration cap, 2 stalled, -9 diverged
  auto pub = [](int st) { return st == 0 ? SMPC_OK : (st == 2 ? SMPC_STALLED : SMPC_MAX_ITER); };
  int status;
  if (h.status == -9 || (ph.run32 && status32 == -9)) status = SMPC_EDIVERGED;
  else if (ph.run32 && ph.run64 && status32 != 2) status = pub(status32);  // float32 phase, then the polish
  else status = pub(h.status);
  r->status = status;
  if (ph.run64) SMPC_TRY(download_primal<double>(t, r->x, r->u, r->u0));
  else SMPC_TRY(download_primal<float>(t, r->x, r->u, r->u0));
  if (r->y && t->res_prec == 64) SMPC_TRY(download_dual<double>(t, h.iters_done % 3, r->y));
  else if (r->y) SMPC_TRY(download_dual<float>(t, h.iters_done % 3, r->y));
  return SMPC_OK;
}

template <typename T, typename Y>
int run_block_eager(smpc_ctx* ctx, smpc_sys* sys, Plan* p, int iters, bool eager) {
  if (!eager) return run_block<T, Y>(ctx, sys, p, kModeAPG, iters);
  SMPC_TRY((ensure_backward<T, Y>(ctx, sys, p)));
  for (int k = 0; k < iters; ++k) SMPC_TRY((enqueue_iteration<T, Y>(ctx, sys, p, kModeAPG)));
  return SMPC_OK;
}

int run_block_prec(smpc_ctx* ctx, smpc_sys* sys, Plan* p, int prec, int iters, bool eager) {
  if (prec == kPrec32) return run_block_eager<float, float>(ctx, sys, p, iters, eager);
  if (prec == kPrecMix) return run_block_eager<float, double>(ctx, sys, p, iters, eager);
  return run_block_eager<double, double>(ctx, sys, p, iters, eager);
}

// Chunk lengths for the options' precisions: explicit entries, else -- with
// tune and from_sys -- the system's tuned pair, else the default; with tune
// and without from_sys a pair already marked tuned is kept.
void choose_chunks(const smpc_sys* sys, const smpc_solve_opts* o, bool from_sys, int (&chunk)[3][2],
                   bool (&tuned)[3]) {
  const int* given[3] = {o->chunk64, o->chunk32, o->chunk32};
  const int defaults[3][2] = {{Chunks<double>::bwd[0], Chunks<double>::fwd[0]},
                              {Chunks<float>::bwd[0], Chunks<float>::fwd[0]},
                              {Chunks<float>::bwd[0], Chunks<float>::fwd[0]}};
  for (int k = 0; k < 3; ++k) {
    const bool explicit_pair = given[k][0] != 0 || given[k][1] != 0;
    if (explicit_pair) {
      for (int w = 0; w < 2; ++w) chunk[k][w] = given[k][w] ? given[k][w] : defaults[k][w];
      tuned[k] = false;
    } else if (o->tune && from_sys && sys->has_tuned[k]) {
      for (int w = 0; w < 2; ++w) chunk[k][w] = sys->tuned_chunk[k][w];
    } else if (!(o->tune && tuned[k])) {
      for (int w = 0; w < 2; ++w) chunk[k][w] = defaults[k][w];
      tuned[k] = false;
    }
  }
}

void result_chunks(const int (&chunk)[3][2], const smpc_solve_opts* o, smpc_result* r) {
  const SolvePhases ph = phases(o);
  for (int w = 0; w < 2; ++w) {
    r->chunk32[w] = ph.run32 ? chunk[ph.mixed ? kPrecMix : kPrec32][w] : 0;
    r->chunk64[w] = ph.run64 ? chunk[kPrec64][w] : 0;
  }
}

// Solve a set of trees (one plan) with the given options.
// ---------------------------------------------------------------- device cost update and objectives

// The float64 system matrices of the cost update and of the objectives.
int cost_sys_upload(smpc_sys* s) {
  smpc_ctx* ctx = s->ctx;
  SMPC_TRY(upload<double>(ctx, s->c_Mu, s->Mu.data(), s->Mu.size()));
  SMPC_TRY(upload<double>(ctx, s->c_Wu, s->Wu.data(), s->Wu.size()));
  SMPC_TRY(upload<double>(ctx, s->c_Gd, s->Gd.data(), s->Gd.size()));
  SMPC_TRY(upload<double>(ctx, s->c_alpha1, s->alpha1.data(), s->alpha1.size()));
  CostSysDev& v = s->cview;
  const SysDev<double>& d = s->d64.view;
  v.nx = s->nx;
  v.nu = s->nu;
  v.nd = s->nd;
  v.safety_by_prob = s->safety_by_prob;
  v.Mu = (const double*)s->c_Mu.ptr;
  v.Wu = (const double*)s->c_Wu.ptr;
  v.Gd = (const double*)s->c_Gd.ptr;
  v.b_rp = d.b_rp;
  v.b_ci = d.b_ci;
  v.b_v = d.b_v;
  v.alpha1 = (const double*)s->c_alpha1.ptr;
  v.umin = d.umin;
  v.umax = d.umax;
  v.xmin = d.xmin;
  v.xmax = d.xmax;
  v.xs = d.xs;
  v.W_alpha = s->W_alpha;
  v.W_x = s->W_x;
  v.gamma_d = s->gamma_d;
  return SMPC_OK;
}

// Node structure of the device cost update, internal order.
int cost_tree_upload(smpc_tree* t) {
  smpc_ctx* ctx = t->sys->ctx;
  const int M = t->M;
  std::vector<int32_t> st(M), par(M), crp(M + 1, 0), cci(M > 1 ? M - 1 : 1, 0);
  for (int in = 0; in < M; ++in) {
    const int n = t->perm[in];
    st[in] = t->stage[n];
    par[in] = t->parent[n] < 0 ? -1 : t->iperm[t->parent[n]];
  }
  for (int in = 0; in < M; ++in)
    if (par[in] >= 0) crp[par[in] + 1]++;
  for (int in = 0; in < M; ++in) crp[in + 1] += crp[in];
  std::vector<int32_t> fill(crp.begin(), crp.end() - 1);
  for (int in = 0; in < M; ++in)
    if (par[in] >= 0) cci[fill[par[in]]++] = in;
  SMPC_TRY(upload_i32(ctx, t->n_stage, st));
  SMPC_TRY(upload_i32(ctx, t->n_parent, par));
  SMPC_TRY(upload_i32(ctx, t->n_crp, crp));
  SMPC_TRY(upload_i32(ctx, t->n_cci, cci));
  SMPC_TRY(upload_i32(ctx, t->n_perm, t->perm));
  const smpc_sys* s = t->sys;
  SMPC_TRY(ctx->alloc(t->d_dev, sizeof(double) * (size_t)M * std::max(s->nd, 1)));
  SMPC_TRY(ctx->alloc(t->a2_dev, sizeof(double) * (size_t)t->N * s->nu));
  SMPC_TRY(ctx->alloc(t->q_dev, sizeof(double) * s->nu));
  SMPC_TRY(ctx->alloc(t->broot0, sizeof(double) * s->nu));
  HIP_TRY(hipMemsetAsync(t->q_dev.ptr, 0, sizeof(double) * s->nu, ctx->stream));
  HIP_TRY(hipMemsetAsync(t->broot0.ptr, 0, sizeof(double) * s->nu, ctx->stream));
  HIP_TRY(hipStreamSynchronize(ctx->stream));
  return SMPC_OK;
}

CostTreeDev cost_tree_view(smpc_tree* t) {
  CostTreeDev v{};
  v.M = t->M;
  v.N = t->N;
  v.root = t->iperm[0];
  v.stage = (const int32_t*)t->n_stage.ptr;
  v.parent = (const int32_t*)t->n_parent.ptr;
  v.child_rp = (const int32_t*)t->n_crp.ptr;
  v.child_ci = (const int32_t*)t->n_cci.ptr;
  v.perm = (const int32_t*)t->n_perm.ptr;
  v.pi = (const double*)t->b64.pi.ptr;
  v.d = (const double*)t->d_dev.ptr;
  v.alpha2 = (const double*)t->a2_dev.ptr;
  v.q = (const double*)t->q_dev.ptr;
  v.uhat = (double*)t->b64.uhat.ptr;
  v.e = (double*)t->b64.e.ptr;
  v.beta = (double*)t->b64.beta.ptr;
  v.beta_root0 = (double*)t->broot0.ptr;
  if (t->b32.allocated) {
    v.uhat32 = (float*)t->b32.uhat.ptr;
    v.e32 = (float*)t->b32.e.ptr;
    v.beta32 = (float*)t->b32.beta.ptr;
  }
  return v;
}

// The previous input q of a solve and the root's linear term it enters
// (both precisions).
int upload_q(smpc_tree* t, const double* q) {
  smpc_ctx* ctx = t->sys->ctx;
  HIP_TRY(hipMemcpyAsync(t->q_dev.ptr, q, sizeof(double) * t->sys->nu, hipMemcpyHostToDevice, ctx->stream));
  HIP_TRY(launch_root_beta(t->sys->cview, cost_tree_view(t), ctx->stream));
  HIP_TRY(hipStreamSynchronize(ctx->stream));
  return SMPC_OK;
}

int ensure_obj_scratch(smpc_tree* t) {
  smpc_ctx* ctx = t->sys->ctx;
  if (!t->obj_part.ptr) SMPC_TRY(ctx->alloc(t->obj_part, sizeof(double) * kObjSlots * kObjMaxBlocks));
  if (!t->obj_out.ptr) SMPC_TRY(ctx->alloc(t->obj_out, sizeof(double) * kObjSlots));
  return SMPC_OK;
}

// Objectives at the iterates of the tree's last solve (smpc_tree_objective),
// with the partial sums in `part` (kObjSlots * kObjMaxBlocks doubles) and the
// reduced values in `out_dev` (kObjSlots doubles).
int tree_objective(smpc_tree* t, double* part, double* out_dev, smpc_objective* out) {
  if (t->res_slot < 0)
    return set_error(SMPC_EINVAL, "no finished solve on the device (smpc_factor or smpc_solve_step ran since)");
  if (t->obj_valid) {
    *out = t->obj_cache;
    return SMPC_OK;
  }
  smpc_sys* s = t->sys;
  smpc_ctx* ctx = s->ctx;
  const int M = t->M, nx = s->nx, nu = s->nu, D = 2 * nx + nu;
  TreeState h;
  SMPC_TRY(read_state(t, &h));
  const int it_done = h.iters_done;
  if (it_done < 1 || it_done % 3 != t->res_slot || it_done > ctx->ctab_len)
    return set_error(SMPC_EINVAL, "the tree's iteration state does not match its resident solve");
  if (!t->plan) SMPC_TRY(ensure_single_plan(t, false));
  TreeBuffers<double>& b = t->b64;
  if (t->res_prec == 32) {
    // a solve that ended in float32: its dual iterates, widened (exactly)
    for (int k = 0; k < 3; ++k)
      HIP_TRY(launch_widen<float>((const float*)t->b32.y[k].ptr, (double*)b.y[k].ptr, (size_t)M * D, ctx->stream));
  }
  if (t->res_z32)  // and its last primal iterate
    HIP_TRY(launch_widen<float>((const float*)t->b32.z.ptr, (double*)b.z.ptr, (size_t)M * (nx + nu), ctx->stream));
  const int sl = t->res_slot;
  ObjDev o{};
  o.z = (const double*)b.z.ptr;
  o.yn = (const double*)b.y[sl].ptr;
  o.yc = (const double*)b.y[(sl + 2) % 3].ptr;
  o.yp = (const double*)b.y[(sl + 1) % 3].ptr;
  o.scale = (const double*)b.scale.ptr;
  o.c = ctx->ctab_host[it_done - 1];
  o.lam = t->lambda;
  const int blocks = std::min(M, kObjMaxBlocks);
  const CostTreeDev tv = cost_tree_view(t);
  HIP_TRY(launch_objective(s->cview, tv, o, false, part, blocks, out_dev, ctx->stream));
  // the solve step at the unscaled dual y = S y^{nu+1}, placed in the slot of
  // y^{nu-1}, which the solve-step mode reads at iteration it_done + 1
  HIP_TRY(launch_scale_dual((const double*)b.y[sl].ptr, (double*)b.y[(sl + 1) % 3].ptr, o.scale, M, nx, nu,
                            ctx->stream));
  TreeState hs = h;
  hs.iter = it_done + 1;
  hs.done = 0;
  SMPC_TRY(write_state(t, hs));
  SMPC_TRY(enqueue_iteration<double>(ctx, s, t->plan, kModeSolve));
  HIP_TRY(launch_objective(s->cview, tv, o, true, part, blocks, out_dev, ctx->stream));
  double r[kObjSlots];
  HIP_TRY(hipMemcpyAsync(r, out_dev, sizeof(r), hipMemcpyDeviceToHost, ctx->stream));
  HIP_TRY(hipStreamSynchronize(ctx->stream));
  SMPC_TRY(write_state(t, h));
  out->cost = r[0] + r[2];
  out->primal = r[0] + r[1];
  out->dual = -(r[3] + r[4]) + r[5];
  out->gap = out->primal + out->dual;
  out->dual_violation = r[6];
  t->obj_cache = *out;
  t->obj_valid = true;
  return SMPC_OK;
}

int solve_plan(Plan* plan, const double* const* p, const double* const* q, const smpc_solve_opts* o,
               smpc_result* res) {
  smpc_sys* sys = plan->trees[0]->sys;
  smpc_ctx* ctx = sys->ctx;
  const int n = (int)plan->trees.size();
  const int D = 2 * sys->nx + sys->nu;
  SMPC_TRY(ctx->ensure_ctab(o->max_iter + 2));
  const SolvePhases ph = phases(o);
  choose_chunks(sys, o, false, plan->chunk, plan->tuned);
  plan->fused = !o->unfused;
  plan->bwd_ready[0] = plan->bwd_ready[1] = plan->bwd_ready[2] = false;  // every tree starts over
  // tuning takes at most 3 blocks per chunk pair (they are iterations too)
  const int max_rounds = o->max_iter / o->check_every + 3 + 3 * 4;
  std::vector<int> fp32_iters(n, 0), status32(n, 0);
  size_t off = 0;
  for (int k = 0; k < n; ++k) {
    smpc_tree* t = plan->trees[k];
    const double* y0 = o->warm_start == 2 ? o->y0 + off : nullptr;
    const double* yp0 = (o->warm_start == 2 && o->y_prev0) ? o->y_prev0 + off : nullptr;
    SMPC_TRY(tree_begin(t, p[k], q[k], o, y0, yp0));
    off += (size_t)t->M * D;
  }
  if (ph.run32) {
    if (ph.mixed) SMPC_TRY((run_until_done<float, double>(ctx, sys, plan, o->check_every, max_rounds, o->tune != 0)));
    else SMPC_TRY((run_until_done<float, float>(ctx, sys, plan, o->check_every, max_rounds, o->tune != 0)));
    for (int k = 0; k < n; ++k) {
      TreeState h;
      SMPC_TRY(read_state(plan->trees[k], &h));
      fp32_iters[k] = h.iters_done;
      status32[k] = h.status;
      if (ph.run64) SMPC_TRY(tree_to_fp64(plan->trees[k], o, fp32_iters[k], status32[k]));
    }
    plan->bwd_ready[0] = false;
  }
  if (ph.run64)
    SMPC_TRY(run_until_done<double>(ctx, sys, plan, o->check_every, max_rounds + ph.polish + 2, o->tune != 0));
  for (int k = 0; k < n; ++k) {
    SMPC_TRY(tree_result(plan->trees[k], o, fp32_iters[k], status32[k], res ? &res[k] : nullptr));
    if (res) result_chunks(plan->chunk, o, &res[k]);
  }
  if (o->gap && res)
    for (int k = 0; k < n; ++k) {
      smpc_tree* t = plan->trees[k];
      SMPC_TRY(ensure_obj_scratch(t));
      smpc_objective ob{};
      SMPC_TRY(tree_objective(t, (double*)t->obj_part.ptr, (double*)t->obj_out.ptr, &ob));
      res[k].cost = ob.cost;
      res[k].gap = ob.gap;
    }
  return SMPC_OK;
}

uint64_t splitmix(uint64_t x) {
  x += 0x9e3779b97f4a7c15ULL;
  x = (x ^ (x >> 30)) * 0xbf58476d1ce4e5b9ULL;
  x = (x ^ (x >> 27)) * 0x94d049bb133111ebULL;
  return x ^ (x >> 31);
}

int tree_check_ready(smpc_tree* t, bool need_data) {
  if (!t) return set_error(SMPC_EINVAL, "tree is NULL");
  if (need_data && !t->has_data) return set_error(SMPC_ENOTFACTORED, "smpc_tree_set_data not called");
  if (need_data && !t->factored) return set_error(SMPC_ENOTFACTORED, "smpc_factor not called");
  return SMPC_OK;
}

int ensure_single_plan(smpc_tree* t, bool need32) {
  smpc_ctx* ctx = t->sys->ctx;
  if (t->plan && (!need32 || t->plan->has32)) return SMPC_OK;
  if (t->plan) {
    plan_free(ctx, t->plan);
    t->plan = nullptr;
  }
  return plan_build(ctx, {t}, need32, &t->plan);
}

size_t tree32_bytes(const smpc_tree* t) {
  const size_t M = t->M, nx = t->sys->nx, nu = t->sys->nu, D = 2 * nx + nu, C = t->chains.size();
  return sizeof(float) * (3 * M * D + 3 * M * nu + M * nx + M + 3 * M + nx + M * (nx + nu) + C * (nx + nu));
}

size_t sys32_bytes(const smpc_sys* s) {
  const size_t kp = p_stride(s->nu), nx = s->nx, nu = s->nu;
  const size_t nnz = s->Bc.v.size() + s->Btc.v.size() + s->Ac.v.size() + s->Atc.v.size();
  return sizeof(float) * (kp * kp + nnz + 2 * nu + 3 * nx) + sizeof(int32_t) * (nnz + 2 * (nx + 1) + 2 * (nu + 1));
}

int tree_release32(smpc_tree* t) {
  smpc_ctx* ctx = t->sys->ctx;
  if (!t->b32.allocated) return SMPC_OK;
  HIP_TRY(hipStreamSynchronize(ctx->stream));
  if (t->plan && t->plan->has32) {
    plan_free(ctx, t->plan);
    t->plan = nullptr;
  }
  if (ctx->batch_plan && ctx->batch_plan->has32 &&
      std::find(ctx->batch_plan->trees.begin(), ctx->batch_plan->trees.end(), t) != ctx->batch_plan->trees.end()) {
    plan_free(ctx, ctx->batch_plan);
    ctx->batch_plan = nullptr;
  }
  tree_free(ctx, t->b32);
  if (t->res_prec == 32) {
    t->res_slot = -1;
    t->shift_ready = false;
  }
  return SMPC_OK;
}

int prepare32(smpc_tree* t) {
  SMPC_TRY(ensure_sys32(t->sys));
  if (!t->b32.allocated) {
    SMPC_TRY(tree_alloc<float>(t));
    if (t->has_data) SMPC_TRY(tree_narrow_data(t));
    SMPC_TRY(tree_upload_scale<float>(t));
    SMPC_TRY(tree_alloc<float>(t));
    if (t->plan) {
      plan_free(t->sys->ctx, t->plan);
      t->plan = nullptr;
    }
  }
  return SMPC_OK;
}

}  // namespace smpc

// =================================================================== C ABI

extern "C" {

int smpc_chunk_lengths(int precision, int which, int* out, int cap, int* n) {
  if (precision != 32 && precision != 64) return set_error(SMPC_EINVAL, "precision must be 32 or 64");
  if (which != 0 && which != 1) return set_error(SMPC_EINVAL, "which must be 0 (backward) or 1 (forward)");
  if (!n || cap < 0 || (cap > 0 && !out)) return set_error(SMPC_EINVAL, "bad output arguments");
  std::vector<int> v;
  if (precision == 32) {
    if (which == 0) v.assign(std::begin(Chunks<float>::bwd), std::end(Chunks<float>::bwd));
    else v.assign(std::begin(Chunks<float>::fwd), std::end(Chunks<float>::fwd));
  } else {
    if (which == 0) v.assign(std::begin(Chunks<double>::bwd), std::end(Chunks<double>::bwd));
    else v.assign(std::begin(Chunks<double>::fwd), std::end(Chunks<double>::fwd));
  }
  for (int k = 0; k < cap && k < (int)v.size(); ++k) out[k] = v[k];
  *n = (int)v.size();
  return SMPC_OK;
}

int smpc_last_error(char* buf, size_t len) {
  if (buf && len) {
    std::strncpy(buf, g_last_error.c_str(), len - 1);
    buf[len - 1] = '\0';
  }
  return (int)g_last_error.size();
}

int smpc_ctx_create(int device, void* hip_stream, size_t hbm_budget, smpc_ctx** out) {
  if (!out) return set_error(SMPC_EINVAL, "out is NULL");
  *out = nullptr;
  int count = 0;
  if (hipGetDeviceCount(&count) != hipSuccess || device < 0 || device >= count)
    return set_error(SMPC_EDEVICE, "no HIP device %d (%d visible)", device, count);
  HIP_TRY(hipSetDevice(device));
  smpc_ctx* c = new (std::nothrow) smpc_ctx();
  if (!c) return set_error(SMPC_ENOMEM, "host allocation failed");
  c->device = device;
  c->budget = hbm_budget;
  if (hip_stream) {
    c->stream = (hipStream_t)hip_stream;
  } else {
    hipError_t e = hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking);
    if (e != hipSuccess) {
      delete c;
      return set_error(SMPC_EDEVICE, "hipStreamCreate failed: %s", hipGetErrorString(e));
    }
    c->own_stream = true;
  }
  *out = c;
  return SMPC_OK;
}

int smpc_ctx_destroy(smpc_ctx* ctx) {
  if (!ctx) return SMPC_OK;
  if (ctx->n_sys > 0) return set_error(SMPC_EINVAL, "context still has %d systems", ctx->n_sys);
  (void)hipStreamSynchronize(ctx->stream);
  ctx->flush_profile();
  if (ctx->batch_plan) plan_free(ctx, ctx->batch_plan);
  if (ctx->ctab) (void)hipFree(ctx->ctab);
  for (hipEvent_t e : ctx->ev_pool) (void)hipEventDestroy(e);
  if (ctx->own_stream) (void)hipStreamDestroy(ctx->stream);
  delete ctx;
  return SMPC_OK;
}

int smpc_ctx_mem_used(smpc_ctx* ctx, size_t* bytes) {
  if (!ctx || !bytes) return set_error(SMPC_EINVAL, "NULL argument");
  *bytes = ctx->used;
  return SMPC_OK;
}

int smpc_sys_create(smpc_ctx* ctx, const smpc_sys_desc* d, smpc_sys** out) {
  if (!ctx || !d || !out) return set_error(SMPC_EINVAL, "NULL argument");
  *out = nullptr;
  const int nx = d->nx, nu = d->nu, nd = d->nd, ne = d->ne;
  if (nx < 1 || nu < 1 || nd < 0 || ne < 0) return set_error(SMPC_EDIM, "dimensions must be positive");
  if (nu > 128) return set_error(SMPC_EDIM, "nu = %d exceeds the supported 128", nu);
  if (nx > 128) return set_error(SMPC_EDIM, "nx = %d exceeds the supported 128", nx);
  if (nd > 4096) return set_error(SMPC_EDIM, "nd = %d exceeds the supported 4096", nd);
  if (ne >= nu) return set_error(SMPC_EDIM, "ne = %d must be < nu = %d", ne, nu);
  if (!d->A || !d->B || (nd > 0 && !d->Gd) || !d->umin || !d->umax || !d->xmin || !d->xmax || !d->xs ||
      !d->alpha1 || !d->Wu)
    return set_error(SMPC_EINVAL, "missing system matrix");
  if (ne > 0 && (!d->E || (nd > 0 && !d->Ed))) return set_error(SMPC_EINVAL, "missing E / Ed");
  smpc_sys* s = new (std::nothrow) smpc_sys();
  if (!s) return set_error(SMPC_ENOMEM, "host allocation failed");
  s->ctx = ctx;
  s->nx = nx; s->nu = nu; s->nd = nd; s->ne = ne;
  auto cp = [](std::vector<double>& v, const double* p, size_t n) { v.assign(p ? p : nullptr, p ? p + n : nullptr); if (!p) v.assign(n, 0.0); };
  cp(s->A, d->A, (size_t)nx * nx);
  cp(s->B, d->B, (size_t)nx * nu);
  cp(s->Gd, d->Gd, (size_t)nx * nd);
  cp(s->E, ne ? d->E : nullptr, (size_t)ne * nu);
  cp(s->Ed, ne ? d->Ed : nullptr, (size_t)ne * nd);
  cp(s->umin, d->umin, nu);
  cp(s->umax, d->umax, nu);
  cp(s->xmin, d->xmin, nx);
  cp(s->xmax, d->xmax, nx);
  cp(s->xs, d->xs, nx);
  cp(s->alpha1, d->alpha1, nu);
  cp(s->Wu, d->Wu, (size_t)nu * nu);
  s->W_alpha = d->W_alpha;
  s->W_x = d->W_x;
  s->gamma_d = d->gamma_d;
  s->safety_by_prob = d->weight_safety_by_prob ? 1 : 0;
  const std::vector<double>* arrs[] = {&s->A, &s->B, &s->Gd, &s->E, &s->Ed, &s->umin, &s->umax,
                                       &s->xmin, &s->xmax, &s->xs, &s->alpha1, &s->Wu};
  bool fin = std::isfinite(s->W_alpha) && std::isfinite(s->W_x) && std::isfinite(s->gamma_d);
  for (auto* a : arrs) fin = fin && all_finite(a->data(), a->size());
  if (!fin) {
    delete s;
    return set_error(SMPC_ENAN, "NaN or Inf in the system description");
  }
  for (int j = 0; j < nu; ++j)
    if (s->umin[j] > s->umax[j]) {
      delete s;
      return set_error(SMPC_EINVAL, "umin > umax at %d", j);
    }
  for (int i = 0; i < nx; ++i)
    if (s->xmin[i] > s->xmax[i]) {
      delete s;
      return set_error(SMPC_EINVAL, "xmin > xmax at %d", i);
    }
  if (s->W_x < 0 || s->gamma_d < 0) {
    delete s;
    return set_error(SMPC_EINVAL, "W_x and gamma_d must be >= 0");
  }
  int rc = sys_factor(s);
  if (rc < 0) {
    delete s;
    return rc;
  }
  rc = sys_upload<double>(s, s->d64);
  if (rc >= 0) rc = cost_sys_upload(s);
  if (rc < 0) {
    sys_free(ctx, s->d64);
    DevBuf* cb[] = {&s->c_Mu, &s->c_Wu, &s->c_Gd, &s->c_alpha1};
    for (DevBuf* b : cb) ctx->release(*b);
    delete s;
    return rc;
  }
  ctx->n_sys++;
  *out = s;
  return SMPC_OK;
}

int smpc_sys_destroy(smpc_sys* s) {
  if (!s) return SMPC_OK;
  if (s->n_trees > 0) return set_error(SMPC_EINVAL, "system still has %d trees", s->n_trees);
  smpc_ctx* ctx = s->ctx;
  (void)hipStreamSynchronize(ctx->stream);
  if (ctx->batch_plan) {
    plan_free(ctx, ctx->batch_plan);
    ctx->batch_plan = nullptr;
  }
  sys_free(ctx, s->d64);
  sys_free(ctx, s->d32);
  DevBuf* cb[] = {&s->c_Mu, &s->c_Wu, &s->c_Gd, &s->c_alpha1};
  for (DevBuf* b : cb) ctx->release(*b);
  ctx->n_sys--;
  delete s;
  return SMPC_OK;
}

int smpc_tree_create(smpc_sys* sys, int N, int M, const int32_t* stage, const int32_t* parent,
                     const double* prob, smpc_tree** out) {
  if (!sys || !stage || !parent || !prob || !out) return set_error(SMPC_EINVAL, "NULL argument");
  *out = nullptr;
  if (N < 1 || M < 1) return set_error(SMPC_EINVAL, "need N >= 1 and M >= 1 (got N=%d, M=%d)", N, M);
  // kernels index the per-node arrays with 32-bit element offsets
  if ((int64_t)M * (2 * sys->nx + sys->nu) >= INT32_MAX)
    return set_error(SMPC_EDIM, "tree too large: M * (2 nx + nu) = %lld must stay below 2^31",
                     (long long)M * (2 * sys->nx + sys->nu));
  if (stage[0] != 0 || parent[0] != -1) return set_error(SMPC_EPROB, "node 0 must be the root");
  if (!(std::fabs(prob[0] - 1.0) <= 1e-12)) return set_error(SMPC_EPROB, "root probability must be 1");
  std::vector<int> nch(M, 0);
  std::vector<double> csum(M, 0.0);
  for (int n = 0; n < M; ++n) {
    if (!std::isfinite(prob[n])) return set_error(SMPC_ENAN, "probability %d is not finite", n);
    if (!(prob[n] > 0.0)) return set_error(SMPC_EPROB, "probability %d is not positive", n);
    if (stage[n] < 0 || stage[n] >= N) return set_error(SMPC_EPROB, "stage %d out of range", n);
    if (n > 0) {
      if (stage[n] < stage[n - 1]) return set_error(SMPC_EPROB, "nodes must be stage-sorted (node %d)", n);
      const int a = parent[n];
      if (a < 0 || a >= n) return set_error(SMPC_EPROB, "parent of node %d must be an earlier node", n);
      if (stage[a] != stage[n] - 1) return set_error(SMPC_EPROB, "parent of node %d is not one stage up", n);
      nch[a]++;
      csum[a] += prob[n];
    }
  }
  for (int n = 0; n < M; ++n) {
    if (stage[n] < N - 1 && nch[n] == 0) return set_error(SMPC_EPROB, "node %d at stage %d has no child", n, stage[n]);
    if (nch[n] > 0 && std::fabs(csum[n] - prob[n]) > 1e-9 * prob[n])
      return set_error(SMPC_EPROB, "children of node %d do not sum to its probability", n);
  }
  if (stage[M - 1] != N - 1) return set_error(SMPC_EPROB, "the last stage must be N-1");
  smpc_tree* t = new (std::nothrow) smpc_tree();
  if (!t) return set_error(SMPC_ENOMEM, "host allocation failed");
  t->sys = sys;
  t->N = N;
  t->M = M;
  t->stage.assign(stage, stage + M);
  t->parent.assign(parent, parent + M);
  t->prob.assign(prob, prob + M);
  // children lists
  std::vector<int> cstart(M + 1, 0), clist(M > 1 ? M - 1 : 0);
  for (int n = 0; n < M; ++n) cstart[n + 1] = cstart[n] + nch[n];
  {
    std::vector<int> fill(cstart.begin(), cstart.end() - 1);
    for (int n = 1; n < M; ++n) clist[fill[parent[n]]++] = n;
  }
  // chains, breadth-first; internal order = chain-major
  t->perm.reserve(M);
  std::deque<std::pair<int, int>> queue;  // (start node, parent chain)
  queue.push_back({0, -1});
  while (!queue.empty()) {
    auto [start, pc] = queue.front();
    queue.pop_front();
    ChainDesc cd{};
    cd.first = (int32_t)t->perm.size();
    cd.parent = pc;
    int nd = start;
    int len = 0;
    while (true) {
      t->perm.push_back(nd);
      ++len;
      if (nch[nd] != 1) break;
      nd = clist[cstart[nd]];
    }
    cd.len = len;
    const int id = (int)t->chains.size();
    cd.child_count = nch[nd];
    cd.child_begin = (int32_t)(t->chains.size() + queue.size() + 1);
    for (int k = 0; k < nch[nd]; ++k) queue.push_back({clist[cstart[nd] + k], id});
    t->chains.push_back(cd);
  }
  t->iperm.assign(M, 0);
  for (int i = 0; i < M; ++i) t->iperm[t->perm[i]] = i;
  // heights
  int H = 0;
  for (int c = (int)t->chains.size() - 1; c >= 0; --c) {
    ChainDesc& cd = t->chains[c];
    int h = 0;
    for (int k = 0; k < cd.child_count; ++k) h = std::max(h, t->chains[cd.child_begin + k].height + 1);
    cd.height = h;
    H = std::max(H, h + 1);
  }
  t->n_levels = H;
  // leaf chains; each inner chain is owned (its prox is done) by its first
  // leaf descendant; the root path of every leaf chain as internal node
  // indices, root first (-1 - node where that leaf chain owns the node)
  const int C0 = (int)t->chains.size();
  std::vector<int> first_leaf(C0, -1);
  for (int c = C0 - 1; c >= 0; --c) {
    const ChainDesc& cd = t->chains[c];
    first_leaf[c] = cd.child_count == 0 ? c : first_leaf[cd.child_begin];
    if (cd.child_count == 0) t->leaves.push_back(c);
  }
  std::reverse(t->leaves.begin(), t->leaves.end());
  t->path_off.assign(C0 + 1, 0);
  t->path.clear();
  for (int c = 0; c < C0; ++c) {
    t->path_off[c] = (int32_t)t->path.size();
    if (t->chains[c].child_count == 0) {
      std::vector<int32_t> anc;
      for (int a = t->chains[c].parent; a >= 0; a = t->chains[a].parent) anc.push_back(a);
      for (auto it = anc.rbegin(); it != anc.rend(); ++it)
        for (int k = 0; k < t->chains[*it].len; ++k) {
          const int32_t node = t->chains[*it].first + k;  // top to bottom
          t->path.push_back(first_leaf[*it] == c ? -1 - node : node);
        }
    }
  }
  t->path_off[C0] = (int32_t)t->path.size();
  // device state
  smpc_ctx* ctx = sys->ctx;
  const size_t C = t->chains.size();
  int rc = ctx->alloc(t->cstat, sizeof(double) * kStat * C);
  if (rc >= 0) rc = ctx->alloc(t->st, sizeof(TreeState));
  if (rc >= 0) rc = ctx->alloc(t->chains_dev, sizeof(ChainDesc) * C);
  if (rc >= 0) rc = ctx->alloc(t->cnt, sizeof(int32_t) * C);
  if (rc >= 0) rc = upload_i32(ctx, t->leaves_dev, t->leaves);
  if (rc >= 0) rc = upload_i32(ctx, t->path_off_dev, t->path_off);
  if (rc >= 0) rc = upload_i32(ctx, t->path_dev, t->path);
  if (rc >= 0) {
    hipError_t e = hipMemcpyAsync(t->chains_dev.ptr, t->chains.data(), sizeof(ChainDesc) * C, hipMemcpyHostToDevice, ctx->stream);
    if (e == hipSuccess) e = hipMemsetAsync(t->cstat.ptr, 0, sizeof(double) * kStat * C, ctx->stream);
    if (e == hipSuccess) e = hipMemsetAsync(t->st.ptr, 0, sizeof(TreeState), ctx->stream);
    if (e == hipSuccess) e = hipMemsetAsync(t->cnt.ptr, 0, sizeof(int32_t) * C, ctx->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
    if (e != hipSuccess) rc = set_error(SMPC_EDEVICE, "tree upload failed: %s", hipGetErrorString(e));
  }
  if (rc >= 0) rc = tree_alloc<double>(t);
  if (rc >= 0) rc = cost_tree_upload(t);
  if (rc < 0) {
    tree_free(ctx, t->b64);
    DevBuf* extra[] = {&t->cstat,  &t->st,       &t->chains_dev, &t->cnt,   &t->leaves_dev, &t->path_off_dev,
                       &t->path_dev, &t->n_stage, &t->n_parent,  &t->n_crp, &t->n_cci,      &t->n_perm,
                       &t->d_dev,  &t->a2_dev,   &t->q_dev,      &t->broot0};
    for (DevBuf* b : extra) ctx->release(*b);
    delete t;
    return rc;
  }
  sys->n_trees++;
  *out = t;
  return SMPC_OK;
}

int smpc_tree_destroy(smpc_tree* t) {
  if (!t) return SMPC_OK;
  smpc_ctx* ctx = t->sys->ctx;
  (void)hipStreamSynchronize(ctx->stream);
  if (ctx->batch_plan) {
    plan_free(ctx, ctx->batch_plan);
    ctx->batch_plan = nullptr;
  }
  if (t->plan) plan_free(ctx, t->plan);
  tree_free(ctx, t->b64);
  tree_free(ctx, t->b32);
  DevBuf* extra[] = {&t->cstat,    &t->st,       &t->chains_dev, &t->cnt,     &t->leaves_dev, &t->path_off_dev,
                     &t->path_dev, &t->shift_src, &t->shift_f,   &t->n_stage, &t->n_parent,   &t->n_crp,
                     &t->n_cci,    &t->n_perm,   &t->d_dev,      &t->a2_dev,  &t->q_dev,      &t->broot0,
                     &t->obj_part, &t->obj_out};
  for (DevBuf* b : extra) ctx->release(*b);
  t->sys->n_trees--;
  delete t;
  return SMPC_OK;
}

int smpc_tree_info(smpc_tree* t, int* M, int* N, int* n_chains, int* n_levels) {
  if (!t) return set_error(SMPC_EINVAL, "tree is NULL");
  if (M) *M = t->M;
  if (N) *N = t->N;
  if (n_chains) *n_chains = (int)t->chains.size();
  if (n_levels) *n_levels = t->n_levels;
  return SMPC_OK;
}

int smpc_tree_set_data(smpc_tree* t, const double* d, const double* alpha2) {
  if (!t) return set_error(SMPC_EINVAL, "tree is NULL");
  const smpc_sys* s = t->sys;
  if (s->nd > 0 && !d) return set_error(SMPC_EINVAL, "d is NULL");
  if (d && !all_finite(d, (size_t)t->M * s->nd)) return set_error(SMPC_ENAN, "NaN or Inf in d");
  if (alpha2 && !all_finite(alpha2, (size_t)t->N * s->nu)) return set_error(SMPC_ENAN, "NaN or Inf in alpha2");
  smpc_ctx* ctx = s->ctx;
  const size_t nd_bytes = sizeof(double) * (size_t)t->M * s->nd;
  const size_t a2_bytes = sizeof(double) * (size_t)t->N * s->nu;
  if (d && nd_bytes) HIP_TRY(hipMemcpyAsync(t->d_dev.ptr, d, nd_bytes, hipMemcpyHostToDevice, ctx->stream));
  else if (nd_bytes) HIP_TRY(hipMemsetAsync(t->d_dev.ptr, 0, nd_bytes, ctx->stream));
  if (alpha2) HIP_TRY(hipMemcpyAsync(t->a2_dev.ptr, alpha2, a2_bytes, hipMemcpyHostToDevice, ctx->stream));
  else HIP_TRY(hipMemsetAsync(t->a2_dev.ptr, 0, a2_bytes, ctx->stream));
  HIP_TRY(launch_cost_update(s->cview, cost_tree_view(t), ctx->stream));
  HIP_TRY(hipStreamSynchronize(ctx->stream));
  t->has_data = true;
  t->obj_valid = false;
  return SMPC_OK;
}

int smpc_tree_get_data(smpc_tree* t, double* uhat, double* e, double* beta) {
  if (!t) return set_error(SMPC_EINVAL, "tree is NULL");
  if (!t->has_data) return set_error(SMPC_ENOTFACTORED, "smpc_tree_set_data not called");
  smpc_ctx* ctx = t->sys->ctx;
  const int M = t->M;
  const int nx = t->sys->nx, nu = t->sys->nu;
  const struct {
    double* out;
    const DevBuf* buf;
    int w;
  } parts[] = {{uhat, &t->b64.uhat, nu}, {e, &t->b64.e, nx}, {beta, &t->b64.beta, nu}};
  for (const auto& pt : parts) {
    if (!pt.out) continue;
    std::vector<double> h((size_t)M * pt.w);
    HIP_TRY(hipMemcpyAsync(h.data(), pt.buf->ptr, sizeof(double) * h.size(), hipMemcpyDeviceToHost, ctx->stream));
    HIP_TRY(hipStreamSynchronize(ctx->stream));
    for (int in = 0; in < M; ++in)
      std::memcpy(pt.out + (size_t)t->perm[in] * pt.w, h.data() + (size_t)in * pt.w, sizeof(double) * pt.w);
  }
  return SMPC_OK;
}

int smpc_tree_objective(smpc_tree* t, smpc_objective* out) {
  if (!t || !out) return set_error(SMPC_EINVAL, "NULL argument");
  SMPC_TRY(ensure_obj_scratch(t));
  return tree_objective(t, (double*)t->obj_part.ptr, (double*)t->obj_out.ptr, out);
}

int smpc_tree_objective_noalloc(smpc_tree* t, smpc_objective* out) {
  if (!t || !out) return set_error(SMPC_EINVAL, "NULL argument");
  if (t->res_slot >= 0 && !t->obj_valid && !t->plan)
    return set_error(SMPC_EINVAL, "the tree has no single-tree launch plan (a smpc_solve of this tree creates it)");
  smpc_ctx* ctx = t->sys->ctx;
  double* sc = nullptr;
  HIP_TRY(hipSetDevice(ctx->device));
  HIP_TRY(objective_scratch(&sc));
  // no profiling events either: the kernels run untimed
  const bool prof = ctx->profiling;
  ctx->profiling = false;
  const int rc = tree_objective(t, sc, sc + (size_t)kObjSlots * kObjMaxBlocks, out);
  ctx->profiling = prof;
  return rc;
}

int smpc_factor(smpc_tree* t, const smpc_factor_opts* o) {
  if (t) {
    t->res_slot = -1;  // the power iteration overwrites the dual slots
    t->shift_ready = false;
  }
  if (!t) return set_error(SMPC_EINVAL, "tree is NULL");
  smpc_factor_opts def{};
  if (!o) o = &def;
  smpc_sys* s = t->sys;
  smpc_ctx* ctx = s->ctx;
  const int M = t->M, nx = s->nx, nu = s->nu, D = 2 * nx + nu;
  // dual scaling
  if (o->scale) {
    if (!all_finite(o->scale, (size_t)M * 3)) return set_error(SMPC_ENAN, "NaN or Inf in scale");
    t->scale.assign((size_t)M * 3, 1.0);
    for (int n = 0; n < M; ++n)
      for (int b = 0; b < 3; ++b) {
        const double v = o->scale[(size_t)n * 3 + b];
        if (!(v > 0.0)) return set_error(SMPC_EINVAL, "scale must be positive");
        t->scale[(size_t)t->iperm[n] * 3 + b] = v;
      }
  } else if (o->precond == 1 || o->precond == 2) {
    // the per-node block diagonal of the dual Hessian (single-branch model,
    // divided by pi_n) to the power -1/2 (1) or -1/4 (2)
    std::vector<double> diag;
    single_branch_precond(s, t->N, diag);
    t->scale.assign((size_t)M * 3, 1.0);
    for (int n = 0; n < M; ++n)
      for (int b = 0; b < 3; ++b) {
        const double dd = diag[(size_t)t->stage[n] * 3 + b];
        const double v = dd > 0.0 ? std::sqrt(t->prob[n] / dd) : 1.0;
        t->scale[(size_t)t->iperm[n] * 3 + b] = o->precond == 1 ? v : std::sqrt(v);
      }
  } else if (o->precond == 0) {
    t->scale.clear();
  } else {
    return set_error(SMPC_EINVAL, "precond must be 0, 1 or 2");
  }
  SMPC_TRY(tree_upload_scale<double>(t));
  SMPC_TRY(tree_alloc<double>(t));
  if (t->b32.allocated) {
    SMPC_TRY(tree_upload_scale<float>(t));
    SMPC_TRY(tree_alloc<float>(t));
  }
  if (t->plan) {
    plan_free(ctx, t->plan);
    t->plan = nullptr;
  }
  if (ctx->batch_plan) {
    plan_free(ctx, ctx->batch_plan);
    ctx->batch_plan = nullptr;
  }
  if (o->lambda_override > 0.0) {
    if (!std::isfinite(o->lambda_override)) return set_error(SMPC_EINVAL, "lambda_override not finite");
    t->lambda = o->lambda_override;
    t->lmax = 1.0 / o->lambda_override;
    t->factored = true;
    return SMPC_OK;
  }
  // power iteration on the (scaled) dual Hessian, float64 on the device
  SMPC_TRY(ensure_single_plan(t, false));
  std::vector<double> h((size_t)M * D);
  double nrm = 0.0;
  for (size_t i = 0; i < h.size(); ++i) {
    h[i] = 0.5 + (double)(splitmix(i + 0x5eedULL) >> 11) * (1.0 / 9007199254740992.0);
    nrm += h[i] * h[i];
  }
  HIP_TRY(hipMemcpyAsync(t->b64.y[0].ptr, h.data(), sizeof(double) * h.size(), hipMemcpyHostToDevice, ctx->stream));
  TreeState st{};
  st.iter = 0;
  st.done = 0;
  st.max_iter = 1 << 30;
  st.check_every = 1;
  st.lambda = 1.0;
  st.in_scale = 1.0 / std::sqrt(nrm);
  SMPC_TRY(write_state(t, st));
  // at least `iters` steps; then on until the Rayleigh quotient (which
  // approaches L from below) changes by less than kPowerTol over a block of
  // 10 steps, for at most 10 x iters steps in all
  const int iters = o->power_iters > 0 ? o->power_iters : 200;
  constexpr double kPowerTol = 1e-5;
  double prev = 0.0;
  int k = 0;
  while (true) {
    const int n = k < iters ? std::min(10, iters - k) : 10;
    SMPC_TRY(run_block<double>(ctx, s, t->plan, kModePower, n));
    k += n;
    if (k < iters) continue;
    SMPC_TRY(read_state(t, &st));
    if (!(st.lmax_est > 0.0) || !std::isfinite(st.lmax_est))
      return set_error(SMPC_EDEVICE, "power iteration failed (estimate %g)", st.lmax_est);
    if (std::fabs(st.lmax_est - prev) <= kPowerTol * st.lmax_est || k >= 10 * iters) break;
    prev = st.lmax_est;
  }
  t->power_steps = k;
  t->lmax = st.lmax_est;
  t->lambda = 1.0 / (st.lmax_est * 1.02);
  t->factored = true;
  return SMPC_OK;
}

int smpc_tree_get_factor(smpc_tree* t, double* lambda, double* scale) {
  if (!t) return set_error(SMPC_EINVAL, "tree is NULL");
  if (!t->factored) return set_error(SMPC_ENOTFACTORED, "smpc_factor not called");
  if (lambda) *lambda = t->lambda;
  if (scale) {
    for (int n = 0; n < t->M; ++n)
      for (int b = 0; b < 3; ++b)
        scale[(size_t)n * 3 + b] = t->scale.empty() ? 1.0 : t->scale[(size_t)t->iperm[n] * 3 + b];
  }
  return SMPC_OK;
}

int smpc_shift_warm_start(smpc_tree* t, int realized) {
  SMPC_TRY(tree_check_ready(t, false));
  if (t->res_slot < 0) return set_error(SMPC_EINVAL, "no resident dual: solve the tree first");
  smpc_sys* sys = t->sys;
  const int M = t->M;
  // children of every node in the caller's order (stage-sorted input)
  std::vector<std::vector<int32_t>> ch(M);
  for (int n = 1; n < M; ++n) ch[t->parent[n]].push_back(n);
  std::vector<int32_t> img(M);
  if (realized == -1) {
    for (int n = 0; n < M; ++n) img[n] = n;  // resume the same tree unshifted
  } else {
    if (realized < 0 || realized >= (int)ch[0].size())
      return set_error(SMPC_EINVAL, "realized child %d out of range (the root has %zu children)", realized,
                       ch[0].size());
    // the next root is the realised child; a deeper node follows the child
    // of its parent's image with its own child index (the last one when there
    // are fewer); below the last stage the image stays (last stage repeated)
    img[0] = ch[0][realized];
    std::vector<int32_t> rank(M, 0);
    for (int a = 0; a < M; ++a)
      for (size_t k = 0; k < ch[a].size(); ++k) rank[ch[a][k]] = (int32_t)k;
    for (int n = 1; n < M; ++n) {
      const std::vector<int32_t>& kids = ch[img[t->parent[n]]];
      img[n] = kids.empty() ? img[t->parent[n]] : kids[std::min<size_t>(rank[n], kids.size() - 1)];
    }
  }
  // internal order: source node and per-block factors pi_new / pi_old on the
  // probability-weighted blocks, times S_old / S_new for the scaled storage
  std::vector<int32_t> src(M);
  std::vector<double> f((size_t)M * 3);
  for (int in = 0; in < M; ++in) {
    const int n = t->perm[in];
    const int m = img[n];
    const int im = t->iperm[m];
    src[in] = im;
    const double ratio = t->prob[n] / t->prob[m];
    for (int b = 0; b < 3; ++b) {
      const bool weighted = (b == 0 && sys->safety_by_prob) || b == 2;
      double v = weighted ? ratio : 1.0;
      if (!t->scale.empty()) v *= t->scale[(size_t)im * 3 + b] / t->scale[(size_t)in * 3 + b];
      f[(size_t)in * 3 + b] = v;
    }
  }
  SMPC_TRY(upload_i32(sys->ctx, t->shift_src, src));
  SMPC_TRY(upload<double>(sys->ctx, t->shift_f, f.data(), f.size()));
  t->shift_ready = true;
  return SMPC_OK;
}

int smpc_solve(smpc_tree* t, const double* p, const double* q, const smpc_solve_opts* o, smpc_result* res) {
  SMPC_TRY(tree_check_ready(t, true));
  SMPC_TRY(check_opts(o));
  if (!p || !q) return set_error(SMPC_EINVAL, "p or q is NULL");
  if (!all_finite(p, t->sys->nx) || !all_finite(q, t->sys->nu)) return set_error(SMPC_ENAN, "NaN or Inf in p or q");
  if (o->warm_start == 2) {
    const size_t n = (size_t)t->M * (2 * t->sys->nx + t->sys->nu);
    if (!all_finite(o->y0, n) || (o->y_prev0 && !all_finite(o->y_prev0, n)))
      return set_error(SMPC_ENAN, "NaN or Inf in the warm start");
  }
  if (o->warm_start == 1 && !t->shift_ready)
    return set_error(SMPC_EINVAL, "warm_start 1 needs smpc_shift_warm_start after the previous solve");
  const bool need32 = o->precision == 32 && o->max_iter > o->polish_iters;
  if (need32) SMPC_TRY(prepare32(t));
  SMPC_TRY(ensure_single_plan(t, need32));
  smpc_result tmp{};
  smpc_result* r = res ? res : &tmp;
  SMPC_TRY(solve_plan(t->plan, &p, &q, o, r));
  if (r->status == SMPC_EDIVERGED)
    set_error(SMPC_EDIVERGED, "iteration diverged (residual non-finite or above 1e300) after %d iterations",
              r->iterations);
  return r->status;
}

int smpc_solve_batch(smpc_tree* const* trees, int n, const double* const* p, const double* const* q,
                     const smpc_solve_opts* o, smpc_result* res) {
  if (!trees || n < 1 || !p || !q) return set_error(SMPC_EINVAL, "bad batch arguments");
  SMPC_TRY(check_opts(o));
  smpc_sys* sys = trees[0] ? trees[0]->sys : nullptr;
  for (int k = 0; k < n; ++k) {
    SMPC_TRY(tree_check_ready(trees[k], true));
    if (trees[k]->sys != sys) return set_error(SMPC_EINVAL, "all trees of a batch must share one system");
    if (!p[k] || !q[k]) return set_error(SMPC_EINVAL, "p[%d] or q[%d] is NULL", k, k);
    if (!all_finite(p[k], sys->nx) || !all_finite(q[k], sys->nu)) return set_error(SMPC_ENAN, "NaN or Inf in p/q %d", k);
    for (int j = 0; j < k; ++j)
      if (trees[j] == trees[k]) return set_error(SMPC_EINVAL, "tree %d appears twice in the batch", k);
    if (o->warm_start == 1 && !trees[k]->shift_ready)
      return set_error(SMPC_EINVAL, "warm_start 1: tree %d has no prepared shift (smpc_shift_warm_start)", k);
  }
  smpc_ctx* ctx = sys->ctx;
  const bool need32 = o->precision == 32 && o->max_iter > o->polish_iters;
  if (need32)
    for (int k = 0; k < n; ++k) SMPC_TRY(prepare32(trees[k]));
  std::vector<smpc_tree*> tv(trees, trees + n);
  Plan* plan = ctx->batch_plan;
  if (!plan || plan->trees != tv || (need32 && !plan->has32)) {
    if (plan) plan_free(ctx, plan);
    ctx->batch_plan = nullptr;
    SMPC_TRY(plan_build(ctx, tv, need32, &ctx->batch_plan));
    plan = ctx->batch_plan;
  }
  std::vector<smpc_result> tmp(n);
  smpc_result* r = res ? res : tmp.data();
  SMPC_TRY(solve_plan(plan, p, q, o, r));
  int worst = SMPC_OK;
  for (int k = 0; k < n; ++k) {
    if (r[k].status < 0) worst = r[k].status;
    else if (worst == SMPC_OK && r[k].status > 0) worst = r[k].status;
  }
  if (worst == SMPC_EDIVERGED) set_error(SMPC_EDIVERGED, "at least one tree of the batch diverged");
  return worst;
}

int smpc_solve_step(smpc_tree* t, const double* p, const double* q, const double* w, int precision, double* x,
                    double* u) {
  SMPC_TRY(tree_check_ready(t, false));
  t->res_slot = -1;  // the solve step overwrites y[0]
  t->shift_ready = false;
  if (!t->has_data) return set_error(SMPC_ENOTFACTORED, "smpc_tree_set_data not called");
  if (!p || !q || !w) return set_error(SMPC_EINVAL, "NULL argument");
  if (precision != 64 && precision != 32) return set_error(SMPC_EINVAL, "precision must be 32 or 64");
  smpc_sys* s = t->sys;
  smpc_ctx* ctx = s->ctx;
  const int M = t->M, nx = s->nx, nu = s->nu, D = 2 * nx + nu;
  if (!all_finite(w, (size_t)M * D)) return set_error(SMPC_ENAN, "NaN or Inf in w");
  const bool use32 = precision == 32;
  if (use32) SMPC_TRY(prepare32(t));
  SMPC_TRY(ensure_single_plan(t, use32));
  SMPC_TRY(ctx->ensure_ctab(4));
  TreeState st{};
  st.iter = 0;
  st.done = 0;
  st.max_iter = 1;
  st.check_every = 1;
  st.lambda = 1.0;
  st.in_scale = 1.0;
  SMPC_TRY(write_state(t, st));
  // w in internal order, unscaled (the solve-step mode ignores the scaling)
  auto put = [&](auto tag) -> int {
    using T = decltype(tag);
    std::vector<T> h((size_t)M * D);
    for (int in = 0; in < M; ++in) {
      const int n = t->perm[in];
      for (int k = 0; k < D; ++k) h[(size_t)in * D + k] = (T)w[(size_t)n * D + k];
    }
    HIP_TRY(hipMemcpyAsync(treebuf<T>(t).y[0].ptr, h.data(), sizeof(T) * h.size(), hipMemcpyHostToDevice, ctx->stream));
    HIP_TRY(hipStreamSynchronize(ctx->stream));
    return SMPC_OK;
  };
  SMPC_TRY(upload_q(t, q));
  if (use32) {
    SMPC_TRY(upload_root<float>(t, p));
    SMPC_TRY(put(float{}));
    SMPC_TRY(enqueue_iteration<float>(ctx, s, t->plan, kModeSolve));
    HIP_TRY(hipStreamSynchronize(ctx->stream));
    SMPC_TRY(download_primal<float>(t, x, u, nullptr));
  } else {
    SMPC_TRY(upload_root<double>(t, p));
    SMPC_TRY(put(double{}));
    SMPC_TRY(enqueue_iteration<double>(ctx, s, t->plan, kModeSolve));
    HIP_TRY(hipStreamSynchronize(ctx->stream));
    SMPC_TRY(download_primal<double>(t, x, u, nullptr));
  }
  return SMPC_OK;
}

int smpc_ctx_set_profiling(smpc_ctx* ctx, int enable) {
  if (!ctx) return set_error(SMPC_EINVAL, "ctx is NULL");
  ctx->flush_profile();
  ctx->profiling = enable != 0;
  return SMPC_OK;
}

int smpc_ctx_kernel_stats(smpc_ctx* ctx, smpc_kernel_stat* out, int cap, int* n) {
  if (!ctx) return set_error(SMPC_EINVAL, "ctx is NULL");
  ctx->flush_profile();
  int k = 0;
  for (auto& kv : ctx->stats) {
    if (out && k < cap) {
      std::memset(out[k].name, 0, sizeof(out[k].name));
      std::strncpy(out[k].name, kv.first.c_str(), sizeof(out[k].name) - 1);
      out[k].launches = kv.second.first;
      out[k].total_ms = kv.second.second;
    }
    ++k;
  }
  if (n) *n = k;
  return SMPC_OK;
}

int smpc_ctx_reset_stats(smpc_ctx* ctx) {
  if (!ctx) return set_error(SMPC_EINVAL, "ctx is NULL");
  ctx->flush_profile();
  ctx->stats.clear();
  return SMPC_OK;
}

}  // extern "C"
