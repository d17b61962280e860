// Continuous batching of closed-loop MPC steps (the loop of Alg. 2, run for
// many controllers at once).
//
// One worker thread owns the context's stream.  Between iteration blocks it
// admits queued requests: each admitted request loads its demands into its
// tree (App. A cost update), starts the dual cold or from the tree's resident
// dual shifted one stage forward, and joins the launch group of its current
// precision (float32 bulk, then float64).  Every tree stops on its own stop
// test and leaves the group; a request's result is the same as that of
// smpc_solve on the same tree and inputs, since the kernels treat the trees
// of a launch independently.
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <new>
#include <set>
#include <string>
#include <thread>
#include <vector>

#include "smpc_host.h"

using namespace smpc;

namespace {

double now_ms() {
  using clk = std::chrono::steady_clock;
  return std::chrono::duration<double, std::milli>(clk::now().time_since_epoch()).count();
}

struct ServerReq {
  uint64_t id = 0;
  smpc_tree* t = nullptr;
  std::vector<double> d, a2, p, q;
  bool has_d = false, has_a2 = false;
  int warm = 0, realized = 0;
  double t_submit = 0, t_start = 0, t_done = 0;
  int phase = 0;  // 32 or 64 while iterating
  int fp32_iters = 0, status32 = 0;
  bool cancel = false;  // smpc_server_cancel on a running request (under the mutex)
  // outcome, written by the worker under the server mutex
  bool done = false;
  int code = SMPC_OK;
  std::string msg;
  smpc_result res{};
  std::vector<double> u0;
};

}  // namespace

struct smpc_server {
  smpc_sys* sys = nullptr;
  smpc_solve_opts o{};
  int max_active = 0;
  // chunk lengths of its launch groups ([0] float64, [1] float32, [2] float32
  // solve steps on a float64 dual)
  int chunk[3][2] = {{0, 0}, {0, 0}, {0, 0}};
  bool restarted[2] = {false, false};  // a tree of launch group g (0 float32, 1 float64) started over
  std::thread worker;
  std::mutex mu;
  std::condition_variable cv_work, cv_done;
  std::deque<ServerReq*> queue;
  std::map<uint64_t, ServerReq*> reqs;
  uint64_t next_id = 1;
  bool stop = false;
  // worker state
  std::vector<ServerReq*> active;
  std::map<smpc_tree*, uint64_t> last_done;  // finish order of each tree's last request
  uint64_t finished = 0;
  Plan* group[2] = {nullptr, nullptr};  // float32, float64 launch groups
  std::vector<smpc_tree*> members[2];
};

namespace {

void finish(smpc_server* S, ServerReq* r, int code, const char* msg) {
  r->t_done = now_ms();
  r->res.queue_ms = r->t_start - r->t_submit;
  r->res.run_ms = r->t_done - r->t_start;
  std::lock_guard<std::mutex> g(S->mu);
  r->code = code;
  if (msg) r->msg = msg;
  r->done = true;
  S->cv_done.notify_all();
}

bool is_active(const smpc_server* S, const smpc_tree* t) {
  for (const ServerReq* r : S->active)
    if (r->t == t) return true;
  return false;
}

// Device memory for the float32 buffers of the request's tree: they must fit
// the context's budget and the device's free memory (less a 1/16 reserve).
// Idle trees give up their float32 buffers, least recently finished first
// (a tree whose resident dual is float32 keeps them, a warm start may need
// it).  SMPC_ENOMEM when that is not enough.
int make_room(smpc_server* S, smpc_tree* t) {
  if (!phases(&S->o).run32 || t->b32.allocated) return SMPC_OK;
  smpc_ctx* ctx = S->sys->ctx;
  const size_t need = tree32_bytes(t) + (S->sys->has32 ? 0 : sys32_bytes(S->sys));
  while (true) {
    size_t freeb = 0, total = 0;
    if (hipMemGetInfo(&freeb, &total) != hipSuccess) return set_error(SMPC_EDEVICE, "hipMemGetInfo failed");
    const bool budget_ok = ctx->budget == 0 || ctx->used + need <= ctx->budget;
    if (budget_ok && freeb >= need + total / 16) return SMPC_OK;
    smpc_tree* victim = nullptr;
    uint64_t oldest = UINT64_MAX;
    for (const auto& kv : S->last_done) {
      smpc_tree* c = kv.first;
      if (c == t || !c->b32.allocated || c->res_prec == 32 || is_active(S, c)) continue;
      if (kv.second < oldest) {
        oldest = kv.second;
        victim = c;
      }
    }
    if (!victim)
      return set_error(SMPC_ENOMEM, "float32 buffers of %zu bytes do not fit (budget %zu, used %zu, device free %zu)",
                       need, ctx->budget, ctx->used, freeb);
    SMPC_TRY(tree_release32(victim));
  }
}

// Load the request's data and start its dual; SMPC_ENOMEM when its tree's
// float32 buffers do not fit yet (checked before any data moves).
int begin_request(smpc_server* S, ServerReq* r) {
  smpc_tree* t = r->t;
  const SolvePhases ph = phases(&S->o);
  SMPC_TRY(make_room(S, t));
  if (r->has_d) SMPC_TRY(smpc_tree_set_data(t, r->d.data(), r->has_a2 ? r->a2.data() : nullptr));
  SMPC_TRY(tree_check_ready(t, true));
  if (ph.run32) SMPC_TRY(prepare32(t));
  smpc_solve_opts o = S->o;
  o.warm_start = 0;
  o.y0 = o.y_prev0 = nullptr;
  if (r->warm) {
    SMPC_TRY(smpc_shift_warm_start(t, r->realized));
    o.warm_start = 1;
  }
  return tree_begin(t, r->p.data(), r->q.data(), &o, nullptr, nullptr);
}

// Rebuild the launch group of precision slot g (0: float32, 1: float64)
// when its members changed.
int sync_group(smpc_server* S, int g) {
  std::vector<smpc_tree*> want;
  for (ServerReq* r : S->active)
    if ((r->phase == 32) == (g == 0)) want.push_back(r->t);
  if (want == S->members[g] && (S->group[g] || want.empty())) return SMPC_OK;
  smpc_ctx* ctx = S->sys->ctx;
  if (S->group[g]) plan_free(ctx, S->group[g]);
  S->group[g] = nullptr;
  S->members[g] = want;
  if (want.empty()) return SMPC_OK;
  SMPC_TRY(plan_build(ctx, want, g == 0, &S->group[g]));
  for (int k = 0; k < 3; ++k)
    for (int w = 0; w < 2; ++w) S->group[g]->chunk[k][w] = S->chunk[k][w];
  S->group[g]->fused = !S->o.unfused;
  return SMPC_OK;
}

void worker_main(smpc_server* S) {
  smpc_ctx* ctx = S->sys->ctx;
  if (hipSetDevice(ctx->device) != hipSuccess) return;
  const SolvePhases ph = phases(&S->o);
  while (true) {
    std::vector<ServerReq*> start;
    {
      std::unique_lock<std::mutex> lk(S->mu);
      if (S->active.empty()) S->cv_work.wait(lk, [&] { return S->stop || !S->queue.empty(); });
      if (S->stop && S->queue.empty() && S->active.empty()) break;
      // admission in submission order: one request per tree at a time, at
      // most max_active trees iterating
      std::set<smpc_tree*> busy;
      for (ServerReq* r : S->active) busy.insert(r->t);
      for (auto it = S->queue.begin(); it != S->queue.end();) {
        if (S->max_active > 0 && (int)(S->active.size() + start.size()) >= S->max_active) break;
        ServerReq* r = *it;
        if (busy.count(r->t)) {
          busy.insert(r->t);
          ++it;
          continue;
        }
        busy.insert(r->t);
        start.push_back(r);
        it = S->queue.erase(it);
      }
    }
    std::vector<ServerReq*> blocked;
    for (ServerReq* r : start) {
      r->t_start = now_ms();
      const int rc = begin_request(S, r);
      if (rc == SMPC_ENOMEM && !S->active.empty()) {
        // wait for device memory, ahead of later requests
        blocked.push_back(r);
        continue;
      }
      if (rc < 0) {
        finish(S, r, rc, last_error_text());
        continue;
      }
      r->phase = ph.run32 ? 32 : 64;
      S->active.push_back(r);
    }
    if (!blocked.empty()) {
      std::lock_guard<std::mutex> g(S->mu);
      S->queue.insert(S->queue.begin(), blocked.begin(), blocked.end());
    }
    if (!start.empty()) S->restarted[ph.run32 ? 0 : 1] = true;
    if (S->active.empty()) continue;
    int rc = SMPC_OK;
    for (int g = 0; g < 2 && rc >= 0; ++g) {
      rc = sync_group(S, g);
      if (rc >= 0 && S->group[g] && S->restarted[g]) {
        // a tree of the group started over: its current backward is not done
        S->group[g]->bwd_ready[0] = S->group[g]->bwd_ready[1] = S->group[g]->bwd_ready[2] = false;
      }
      S->restarted[g] = false;
      const int prec = g == 1 ? kPrec64 : (ph.mixed ? kPrecMix : kPrec32);
      if (rc >= 0 && S->group[g]) rc = run_block_prec(ctx, S->sys, S->group[g], prec, S->o.check_every, true);
    }
    for (int g = 0; g < 2 && rc >= 0; ++g)
      if (S->group[g]) rc = read_done(ctx, S->group[g]);
    if (rc < 0) {
      // a device error ends every request in flight
      const std::string msg = last_error_text();
      for (ServerReq* r : S->active) finish(S, r, rc, msg.c_str());
      S->active.clear();
      continue;
    }
    std::vector<ServerReq*> still;
    for (ServerReq* r : S->active) {
      bool cancel;
      {
        std::lock_guard<std::mutex> g(S->mu);
        cancel = r->cancel;
      }
      if (cancel) {
        // withdrawn: the tree keeps no resident dual from this request
        r->t->res_slot = -1;
        r->t->shift_ready = false;
        r->t->obj_valid = false;
        S->last_done[r->t] = ++S->finished;
        finish(S, r, SMPC_ECANCELED, "request canceled");
        continue;
      }
      const int g = r->phase == 32 ? 0 : 1;
      const std::vector<smpc_tree*>& m = S->members[g];
      size_t k = 0;
      while (k < m.size() && m[k] != r->t) ++k;
      if (k == m.size() || !S->group[g]->done_host[k]) {
        still.push_back(r);
        continue;
      }
      int code = SMPC_OK;
      if (r->phase == 32) {
        TreeState h;
        code = read_state(r->t, &h);
        if (code >= 0) {
          r->fp32_iters = h.iters_done;
          r->status32 = h.status;
          if (ph.run64) {
            code = tree_to_fp64(r->t, &S->o, r->fp32_iters, r->status32);
            if (code >= 0) {
              r->phase = 64;
              S->restarted[1] = true;
              still.push_back(r);
              continue;
            }
          }
        }
      }
      if (code >= 0) {
        r->u0.assign(S->sys->nu, 0.0);
        r->res.u0 = r->u0.data();
        code = tree_result(r->t, &S->o, r->fp32_iters, r->status32, &r->res);
        r->res.u0 = nullptr;
        result_chunks(S->chunk, &S->o, &r->res);
      }
      if (code >= 0) code = r->res.status;
      S->last_done[r->t] = ++S->finished;
      finish(S, r, code, code < 0 ? last_error_text() : nullptr);
    }
    S->active.swap(still);
  }
  for (int g = 0; g < 2; ++g) {
    if (S->group[g]) plan_free(ctx, S->group[g]);
    S->group[g] = nullptr;
  }
}

}  // namespace

extern "C" {

int smpc_server_create(smpc_sys* sys, const smpc_server_opts* opts, smpc_server** out) {
  if (!sys || !opts || !out) return set_error(SMPC_EINVAL, "NULL argument");
  *out = nullptr;
  SMPC_TRY(check_opts(&opts->solve));
  if (opts->solve.warm_start != 0) return set_error(SMPC_EINVAL, "server options take no warm start (per request)");
  if (opts->max_active < 0) return set_error(SMPC_EINVAL, "max_active must be >= 0");
  SMPC_TRY(sys->ctx->ensure_ctab(opts->solve.max_iter + 2));
  smpc_server* S = new (std::nothrow) smpc_server();
  if (!S) return set_error(SMPC_ENOMEM, "host allocation failed");
  S->sys = sys;
  S->o = opts->solve;
  S->o.y0 = S->o.y_prev0 = nullptr;
  S->max_active = opts->max_active;
  bool tuned[3] = {false, false, false};
  choose_chunks(sys, &S->o, true, S->chunk, tuned);
  try {
    S->worker = std::thread(worker_main, S);
  } catch (...) {
    delete S;
    return set_error(SMPC_EDEVICE, "could not start the server thread");
  }
  *out = S;
  return SMPC_OK;
}

int smpc_server_submit(smpc_server* S, smpc_tree* t, const double* d, const double* alpha2, const double* p,
                       const double* q, int warm, int realized, uint64_t* ticket) {
  if (!S || !t || !p || !q || !ticket) return set_error(SMPC_EINVAL, "NULL argument");
  if (t->sys != S->sys) return set_error(SMPC_EINVAL, "the tree belongs to another system");
  if (warm != 0 && warm != 1) return set_error(SMPC_EINVAL, "warm must be 0 or 1");
  const smpc_sys* sys = S->sys;
  ServerReq* r = new (std::nothrow) ServerReq();
  if (!r) return set_error(SMPC_ENOMEM, "host allocation failed");
  r->t = t;
  r->p.assign(p, p + sys->nx);
  r->q.assign(q, q + sys->nu);
  if (d) {
    r->d.assign(d, d + (size_t)t->M * sys->nd);
    r->has_d = true;
    if (alpha2) {
      r->a2.assign(alpha2, alpha2 + (size_t)t->N * sys->nu);
      r->has_a2 = true;
    }
  }
  r->warm = warm;
  r->realized = realized;
  r->t_submit = now_ms();
  {
    std::lock_guard<std::mutex> g(S->mu);
    if (S->stop) {
      delete r;
      return set_error(SMPC_EINVAL, "server is shutting down");
    }
    r->id = S->next_id++;
    S->reqs[r->id] = r;
    S->queue.push_back(r);
  }
  S->cv_work.notify_one();
  *ticket = r->id;
  return SMPC_OK;
}

int smpc_server_poll(smpc_server* S, uint64_t ticket, smpc_result* res, int wait_ms) {
  if (!S) return set_error(SMPC_EINVAL, "server is NULL");
  if (res && (res->x || res->u || res->y)) return set_error(SMPC_EINVAL, "server results carry u0 only");
  std::unique_lock<std::mutex> lk(S->mu);
  auto it = S->reqs.find(ticket);
  if (it == S->reqs.end()) return set_error(SMPC_EINVAL, "unknown ticket %llu", (unsigned long long)ticket);
  ServerReq* r = it->second;
  auto ready = [&] { return r->done; };
  if (wait_ms < 0) S->cv_done.wait(lk, ready);
  else if (wait_ms > 0) S->cv_done.wait_for(lk, std::chrono::milliseconds(wait_ms), ready);
  if (!r->done) return SMPC_PENDING;
  const int code = r->code;
  if (res) {
    double* u0 = res->u0;
    *res = r->res;
    res->u0 = u0;
    res->x = res->u = res->y = nullptr;
    if (u0 && !r->u0.empty()) std::memcpy(u0, r->u0.data(), sizeof(double) * r->u0.size());
  }
  const std::string msg = r->msg;
  S->reqs.erase(it);
  delete r;
  lk.unlock();
  if (code < 0) return set_error(code, "%s", msg.c_str());
  if (code == SMPC_EDIVERGED) return set_error(code, "iteration diverged");
  return code;
}

int smpc_server_cancel(smpc_server* S, uint64_t ticket) {
  if (!S) return set_error(SMPC_EINVAL, "server is NULL");
  std::lock_guard<std::mutex> g(S->mu);
  auto it = S->reqs.find(ticket);
  if (it == S->reqs.end()) return set_error(SMPC_EINVAL, "unknown ticket %llu", (unsigned long long)ticket);
  ServerReq* r = it->second;
  if (r->done) return SMPC_OK;
  for (auto q = S->queue.begin(); q != S->queue.end(); ++q)
    if (*q == r) {
      // never started
      S->queue.erase(q);
      r->t_start = r->t_done = now_ms();
      r->res.queue_ms = r->t_done - r->t_submit;
      r->code = SMPC_ECANCELED;
      r->msg = "request canceled";
      r->done = true;
      S->cv_done.notify_all();
      return SMPC_OK;
    }
  r->cancel = true;  // running: the worker ends it after the current block
  return SMPC_OK;
}

int smpc_server_destroy(smpc_server* S) {
  if (!S) return SMPC_OK;
  {
    std::lock_guard<std::mutex> g(S->mu);
    S->stop = true;
  }
  S->cv_work.notify_all();
  if (S->worker.joinable()) S->worker.join();
  for (auto& kv : S->reqs) delete kv.second;
  delete S;
  return SMPC_OK;
}

}  // extern "C"
