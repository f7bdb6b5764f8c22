// kde_server.hip -- continuous-batching server for bandwidth-selection requests.
//
// One scheduler thread per context.  Clients submit requests (copied on
// submit), which queue in arrival order until admission: a free slot, room
// in the HBM budget and a place for the request's device block in the
// server's arena (one allocation of the whole budget, made when the server
// starts; kde_arena.h).  The first queued request that does not fit keeps its
// room, and later smaller requests pass it only within the rest of the
// budget (kde_admit.h), so a large request is not held up indefinitely and
// small ones are not held up behind it.  Admitted requests stay resident.
// Each scheduler iteration builds one executor pass over all resident
// requests: the moments of newly admitted ones, then plug-in stage units and
// LSCV units taken request by request, smallest remaining work first
// (optionally aged by the time waited), until the iteration's evaluation
// budget is used; a stage whose last units are in the pass is finished in it,
// and requests whose work is all done are finalised.  Iterations are
// pipelined two deep: the next iteration is planned, packed and enqueued
// while the previous one runs on the device, and only then is the previous
// one waited for and its finished requests copied back (on a second stream)
// and retired, so the device does not idle for the host's planning.
// Requests arriving while an iteration runs join the next one, so their work
// overlaps with the requests already on the device.  Every request keeps the
// work decomposition and reduction order it has alone, so its results are
// bitwise those of kde_batch.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <unordered_map>

#include "kde_admit.h"
#include "kde_arena.h"
#include "kde_runtime.h"

namespace kde {

namespace {

double now_s() {
  using namespace std::chrono;
  return duration<double>(steady_clock::now().time_since_epoch()).count();
}

}  // namespace

struct SrvReq {
  uint64_t ticket = 0;
  kde_request req;
  std::vector<char> host_x;  // copy of host samples
  void* dev_x = nullptr;     // copy of device samples
  ColPlan plan;
  uint64_t fp = 0;           // footprint in the arena (rounded block size)
  double work = 0.0;         // pair-term evaluations of the whole request
  char* block = nullptr;
  int64_t block_off = -1;    // the block's offset in the arena
  int slot = -1;
  bool stats_done = false, plugin_done = false, prep_done = false, lscv_done = false;
  int stage = 0;
  size_t psi_next = 0, lscv_next = 0;
  std::vector<Unit> psi_u, lscv_u;
  std::vector<UnitCost> psi_c, lscv_c;
  double remaining = 0.0;
  double key = 0.0;  // the scheduler's order of this iteration
  bool finishing = false, done = false;
  bool cancel = false;    // kde_cancel on an admitted request: dropped at the next iteration
  bool injected = false;  // the failure hook names this request
  bool dropped = false;   // cancelled while resident: leaves without a result
  int64_t retire_iter = -1;  // the iteration at whose end the request leaves (-1: still working)
  kde_result res;
  std::vector<double> g, gs;
  double t_submit = 0, t_admit = 0, t_done = 0;
};

struct Server {
  kde_ctx* c = nullptr;
  uint64_t budget = 0;
  int max_slots = 0;
  std::mutex mu;
  std::condition_variable cv_work, cv_done;
  std::deque<std::shared_ptr<SrvReq>> queue;
  std::vector<std::shared_ptr<SrvReq>> active;
  std::unordered_map<uint64_t, std::shared_ptr<SrvReq>> all;
  std::vector<int> free_slots;
  uint64_t next_ticket = 1;
  uint64_t used = 0;
  bool running = false, stopping = false;
  std::thread th;
  DevBuf<DevState> st;
  DevState* h_st = nullptr;
  DevBuf<char> arena_mem;  // the HBM budget, reserved at start
  Arena arena;
  hipStream_t copy_stream = nullptr;  // result copies of a finished iteration
  hipEvent_t ev[4] = {};              // start / end of the two iterations in the pipeline
  char* h_blob_alt = nullptr;         // second pinned staging blob (iterations alternate)
  size_t h_blob_alt_cap = 0;
  IterPlan it;
  // column table of a pass: slot s at s, for the slots below `top` (one past
  // the highest resident slot); with tile pruning, slot s's near-tile and
  // pruned-sweep descriptors at top + 2 s and top + 2 s + 1
  int top = 0;
  int extra_id(int slot) const { return top + 2 * slot; }
  // with serve_iter_ms: the counted evaluations an iteration takes, adapted
  // so that full iterations last about the target time
  double iter_budget = 0.0;
  void loop();
  void release_block(SrvReq& r);
};

namespace {

void finish_with(Server& s, const std::shared_ptr<SrvReq>& r, kde_status st) {
  r->res.status = st;
  r->t_done = now_s();
  r->res.t_queue_s = (r->t_admit > 0 ? r->t_admit : r->t_done) - r->t_submit;
  r->res.t_service_s = r->t_admit > 0 ? r->t_done - r->t_admit : 0.0;
  r->done = true;
  (void)s;
}

// Adds units [next, end) of one list to the pass while the budget lasts; at
// least one unit when `force`.  col >= 0 replaces the units' descriptor index.
void take_units(const std::vector<Unit>& u, const std::vector<UnitCost>& cu, size_t& next, double& budget,
                bool force, std::vector<Unit>& out, std::vector<UnitCost>& out_c, double& remaining, int col = -1) {
  while (next < u.size() && (budget > 0.0 || force)) {
    out.push_back(u[next]);
    if (col >= 0) out.back().col = col;
    out_c.push_back(cu[next]);
    budget -= cu[next].evals;
    remaining -= cu[next].evals;
    ++next;
    force = false;
  }
}

}  // namespace

// Returns a request's block to the arena and its slot (mu held).
void Server::release_block(SrvReq& r) {
  if (r.block_off >= 0) arena.release(r.block_off);
  r.block_off = -1;
  r.block = nullptr;
  used -= r.fp;
  free_slots.push_back(r.slot);
}

void Server::loop() {
  kde_ctx* ctx = c;
  (void)hipSetDevice(ctx->device);
  const bool cond = ctx->prec != KDE_PREC_FP64 && ctx->opt_fp64_kappa > 0.0;
  // the iteration in flight on the device (if any)
  struct Flight {
    bool on = false;
    int64_t id = -1;
    int ev = 0;  // its events: ev[ev], ev[ev + 1]
    bool full = false;
    double left0 = 0.0;
  } prev;
  int64_t iter_id = 0;
  int ev_next = 0;
  // Waits for the iteration in flight and retires the requests that leave at
  // its end; on a failure every resident request ends with KDE_E_DEVICE.
  auto retire = [&](const Flight& f, kde_status s) {
    if (s == KDE_OK && f.on) {
      const hipError_t e = hipEventSynchronize(ev[f.ev + 1]);
      if (e != hipSuccess) s = fail(ctx, KDE_E_DEVICE, std::string("server iteration: ") + hipGetErrorString(e));
    }
    if (s == KDE_OK) s = collect_ready_timing(ctx);
    // finished requests: state and curves, copied on the side stream (the
    // main stream already runs the next iteration)
    if (s == KDE_OK) {
      for (auto& r : active) {
        if (r->retire_iter != f.id || r->dropped || r->injected) continue;
        hipError_t e = hipMemcpyAsync(h_st + r->slot, st.p + r->slot, sizeof(DevState), hipMemcpyDeviceToHost,
                                      copy_stream);
        if (e == hipSuccess && r->plan.lscv) {
          ColDesc d;
          bind_column(r->plan, r->block, r->dev_x, st.p + r->slot, d);
          r->g.assign(r->plan.n_h, 0.0);
          r->gs.assign(r->plan.n_h, 0.0);
          e = hipMemcpyAsync(r->g.data(), d.g, sizeof(double) * r->plan.n_h, hipMemcpyDeviceToHost, copy_stream);
          if (e == hipSuccess)
            e = hipMemcpyAsync(r->gs.data(), d.gs, sizeof(double) * r->plan.n_h, hipMemcpyDeviceToHost, copy_stream);
        }
        if (e != hipSuccess) s = fail(ctx, KDE_E_DEVICE, std::string("result copy: ") + hipGetErrorString(e));
      }
      const hipError_t e = hipStreamSynchronize(copy_stream);
      if (s == KDE_OK && e != hipSuccess) s = fail(ctx, KDE_E_DEVICE, std::string("result copy: ") + hipGetErrorString(e));
    }
    if (s != KDE_OK) (void)hipStreamSynchronize(ctx->stream);  // nothing may still use the blocks
    if (s == KDE_OK && f.on && f.full && ctx->opt_serve_iter_s > 0.0) {
      // a full iteration: move the budget towards the target duration (by
      // the square root of the ratio, within [1, 64] x serve_iter_evals)
      float ms = 0.f;
      if (hipEventElapsedTime(&ms, ev[f.ev], ev[f.ev + 1]) == hipSuccess && ms > 0.1f) {
        const double want = f.left0 * std::sqrt(ctx->opt_serve_iter_s / (ms * 1e-3));
        iter_budget = std::min(64.0 * ctx->opt_serve_iter_evals, std::max(ctx->opt_serve_iter_evals, want));
      }
    }
    std::lock_guard<std::mutex> lk(mu);
    std::vector<std::shared_ptr<SrvReq>> keep;
    for (auto& r : active) {
      if (s == KDE_OK && r->retire_iter != f.id) {
        keep.push_back(r);
        continue;
      }
      if (s != KDE_OK || r->injected) {
        finish_with(*this, r, KDE_E_DEVICE);
      } else if (r->dropped) {
        finish_with(*this, r, KDE_E_CANCELLED);
      } else {
        fill_result(r->plan, h_st[r->slot], r->res);
        finish_with(*this, r, r->res.status);
      }
      release_block(*r);
    }
    active.swap(keep);
    cv_done.notify_all();
  };
  for (;;) {
    std::vector<std::shared_ptr<SrvReq>> admitted;
    {
      std::unique_lock<std::mutex> lk(mu);
      for (;;) {
        // requests larger than the whole budget never fit
        for (auto q = queue.begin(); q != queue.end();) {
          if ((*q)->fp > budget) {
            finish_with(*this, *q, KDE_E_NOMEM);
            q = queue.erase(q);
            cv_done.notify_all();
          } else {
            ++q;
          }
        }
        std::vector<uint64_t> fps;
        std::vector<double> work;
        for (auto& r : queue) {
          fps.push_back(r->fp);
          work.push_back(r->work);
        }
        std::vector<Resident> res;
        for (auto& r : active) res.push_back(Resident{r->fp, r->retire_iter >= 0 ? 0.0 : r->remaining});
        std::vector<int64_t> offs(queue.size(), -1);
        const std::vector<size_t> take = admit(fps, work, res, budget, used, (int)free_slots.size(), [&](size_t k) {
          offs[k] = arena.alloc(fps[k]);
          return offs[k] >= 0;
        });
        for (size_t t = 0; t < take.size(); ++t) {
          std::shared_ptr<SrvReq> r = queue[take[t]];
          r->block_off = offs[take[t]];
          r->block = arena_mem.p + r->block_off;
          r->slot = free_slots.back();
          free_slots.pop_back();
          admitted.push_back(r);
        }
        for (size_t t = take.size(); t-- > 0;) queue.erase(queue.begin() + (long)take[t]);
        bool busy_now = !admitted.empty() || prev.on;
        for (auto& r : active) busy_now = busy_now || r->retire_iter < 0;
        if (busy_now) break;
        if (stopping && active.empty()) return;
        cv_work.wait_for(lk, std::chrono::milliseconds(50));
      }
    }
    // initial state of newly admitted requests
    for (auto& r : admitted) {
      r->t_admit = now_s();
      init_state(r->plan, ctx->opt_fp64_kappa, h_st[r->slot]);
      (void)hipMemcpyAsync(st.p + r->slot, h_st + r->slot, sizeof(DevState), hipMemcpyHostToDevice, ctx->stream);
      psi_units_of(r->plan, r->slot, r->psi_u, r->psi_c);
      lscv_units_of(r->plan, r->slot, r->lscv_u, r->lscv_c);
      r->stage = r->plan.stages == 3 ? 0 : 1;
      r->remaining = 0.0;
      for (const UnitCost& u : r->psi_c) r->remaining += u.evals * (3 - r->stage);
      for (const UnitCost& u : r->lscv_c) r->remaining += u.evals;
      active.push_back(r);
    }
    // the requests this iteration works on: resident ones that do not leave
    // at the end of the iteration in flight; a cancelled one leaves now
    const int64_t cur = iter_id++;
    std::vector<std::shared_ptr<SrvReq>> work;
    {
      std::lock_guard<std::mutex> lk(mu);
      for (auto& r : active) {
        if (r->retire_iter >= 0) continue;
        if (r->cancel) {
          r->dropped = true;
          r->retire_iter = cur;
          continue;
        }
        work.push_back(r);
      }
    }
    // one executor pass over them, smallest remaining first; with aging (time
    // constant tau) a request's remaining work counts as
    // remaining / (1 + waited / tau), so long-waiting large requests move up
    it.clear();
    top = 0;
    for (auto& r : active) top = std::max(top, r->slot + 1);
    it.cols.assign((ctx->opt_prune ? 3 : 1) * (size_t)top, ColDesc());
    {
      const double now = now_s(), tau = ctx->opt_serve_aging_s;
      for (auto& r : work) r->key = tau > 0.0 ? r->remaining / (1.0 + (now - r->t_submit) / tau) : r->remaining;
    }
    std::sort(work.begin(), work.end(), [](const std::shared_ptr<SrvReq>& a, const std::shared_ptr<SrvReq>& b) {
      return a->key < b->key || (a->key == b->key && a->ticket < b->ticket);
    });
    // An iteration is one launch per pass, so it must hold many rounds of its
    // largest units or the launch tail idles the chip (about half a unit per
    // block at the end of every launch): at least 24 rounds of 1024 resident
    // blocks of the largest unit any resident request has next, which keeps
    // that idle share near 2% (at 6 rounds the served form lost ~3% of the
    // plain form's throughput on streams of large requests).
    double max_unit = 0.0;
    for (auto& r : work) {
      if (r->plan.plugin && !r->plugin_done && r->psi_next < r->psi_c.size())
        max_unit = std::max(max_unit, r->psi_c[r->psi_next].evals);
      if (r->plan.lscv && !r->lscv_done && r->lscv_next < r->lscv_c.size())
        max_unit = std::max(max_unit, r->lscv_c[r->lscv_next].evals);
    }
    const double base = ctx->opt_serve_iter_s > 0.0 ? std::max(iter_budget, ctx->opt_serve_iter_evals)
                                                    : ctx->opt_serve_iter_evals;
    double left = std::max(base, 24.0 * 1024.0 * max_unit);
    const double left0 = left;
    bool first = true;
    for (auto& r : work) {
      ColPlan& p = r->plan;
      ColDesc d;
      bind_column(p, r->block, r->dev_x, st.p + r->slot, d);
      it.cols[r->slot] = d;
      if (p.lscv && p.prune && r->prep_done && !r->lscv_done)
        prune_descs(p, d, it.cols[extra_id(r->slot)], it.cols[extra_id(r->slot) + 1]);
      if (!r->stats_done) {
        if (p.raw_in_block) it.uploads.push_back(Upload{(void*)d.raw, r->host_x.data(), p.raw_bytes});
        if (p.lscv && p.grid_kind == KDE_GRID_EXPLICIT)
          it.uploads.push_back(Upload{(void*)d.h_in, p.grid_h.data(), sizeof(double) * p.n_h});
        it.ids_stats.push_back(r->slot);
        it.max_stat_blocks = std::max(it.max_stat_blocks, std::min(kStatBlocks, (p.n + 2047) / 2048));
        r->stats_done = true;
      }
      if (p.plugin && !r->plugin_done) {
        while (r->stage < 3) {
          const int s = r->stage;
          if (r->psi_next == 0) it.ids_begin[s].push_back(r->slot);
          take_units(r->psi_u, r->psi_c, r->psi_next, left, first, it.psi_units[s], it.psi_cost[s], r->remaining);
          first = false;
          if (r->psi_next < r->psi_u.size()) break;
          it.ids_finish[s].push_back(r->slot);
          psi_rows_of(p, d, it.psi_rows[s]);
          if (cond) psi_units_of(p, r->slot, it.psi_cond_units[s], it.psi_cond_cost[s]);
          r->stage++;
          r->psi_next = 0;
          if (left <= 0.0) break;
        }
        if (r->stage == 3) {
          it.ids_plugin_final.push_back(r->slot);
          r->plugin_done = true;
        }
      }
      if (p.lscv && !r->lscv_done) {
        if (!r->prep_done) {
          it.ids_lscv_prep.push_back(r->slot);
          if (p.prune) add_prune_setup(p, d, r->slot, extra_id(r->slot), it);
          r->prep_done = true;
        }
        // a pruned column's sweep units name its pruned-sweep descriptor
        take_units(r->lscv_u, r->lscv_c, r->lscv_next, left, first, p.prune ? it.prune_units : it.lscv_units,
                   p.prune ? it.prune_cost : it.lscv_cost, r->remaining, p.prune ? extra_id(r->slot) + 1 : -1);
        first = false;
        if (r->lscv_next == r->lscv_u.size()) {
          lscv_rows_of(p, d, it.lscv_rows);
          it.ids_lscv_final.push_back(r->slot);
          r->lscv_done = true;
        }
      }
      r->finishing = (!p.plugin || r->plugin_done) && (!p.lscv || r->lscv_done);
      if (ctx->opt_serve_fail_ticket != 0 && r->ticket == ctx->opt_serve_fail_ticket) r->injected = true;
      if (r->finishing || r->injected) r->retire_iter = cur;
    }
    kde_status s = KDE_OK;
    Flight now;
    if (!work.empty()) {
      // iterations alternate between two pinned staging blobs: the previous
      // iteration's upload may still be pending
      std::swap(ctx->h_blob, h_blob_alt);
      std::swap(ctx->h_blob_cap, h_blob_alt_cap);
      now.on = true;
      now.id = cur;
      now.ev = ev_next;
      now.full = left <= 0.0;
      now.left0 = left0;
      ev_next ^= 2;
      hipError_t e = hipEventRecord(ev[now.ev], ctx->stream);
      if (e != hipSuccess) s = fail(ctx, KDE_E_DEVICE, std::string("event: ") + hipGetErrorString(e));
      if (s == KDE_OK) s = execute(ctx, it);
      if (s == KDE_OK) {
        e = hipEventRecord(ev[now.ev + 1], ctx->stream);
        if (e != hipSuccess) s = fail(ctx, KDE_E_DEVICE, std::string("event: ") + hipGetErrorString(e));
      }
    }
    if (s != KDE_OK) {
      // the pass could not be enqueued: every resident request fails
      Flight all;
      all.on = false;
      retire(all, s);
      prev.on = false;
      continue;
    }
    // the previous iteration ends while this one runs
    if (prev.on) retire(prev, KDE_OK);
    if (now.on) {
      prev = now;
    } else {
      prev.on = false;
      // requests that left with no iteration in flight (cancelled)
      Flight none;
      none.id = cur;
      retire(none, KDE_OK);
    }
  }
}

void ServerDeleter::operator()(Server* s) const {
  if (!s) return;
  for (auto& kv : s->all)
    if (kv.second->dev_x) (void)hipFree(kv.second->dev_x);
  (void)hipFree(s->st.p);
  (void)hipFree(s->arena_mem.p);
  if (s->h_st) (void)hipHostFree(s->h_st);
  if (s->h_blob_alt) (void)hipHostFree(s->h_blob_alt);
  for (hipEvent_t e : s->ev)
    if (e) (void)hipEventDestroy(e);
  if (s->copy_stream) (void)hipStreamDestroy(s->copy_stream);
  delete s;
}

bool server_running(const Server* s) { return s && s->running; }

}  // namespace kde

namespace {

using kde::fail;
using kde::Server;
using kde::SrvReq;

kde_status collect(kde_ctx* c, Server& s, uint64_t ticket, kde_result* out, std::unique_lock<std::mutex>& lk,
                   double timeout_s) {
  auto itr = s.all.find(ticket);
  if (itr == s.all.end()) return fail(c, KDE_E_INVAL, "unknown ticket");
  std::shared_ptr<SrvReq> r = itr->second;
  if (!r->done) {
    if (timeout_s == 0.0) return KDE_E_BUSY;
    auto pred = [&] { return r->done; };
    if (timeout_s < 0)
      s.cv_done.wait(lk, pred);
    else if (!s.cv_done.wait_for(lk, std::chrono::duration<double>(timeout_s), pred))
      return KDE_E_BUSY;
  }
  if (out) {
    double* g = out->g_out;
    double* gs = out->gscale_out;
    *out = r->res;
    out->g_out = g;
    out->gscale_out = gs;
    if (g && !r->g.empty()) std::memcpy(g, r->g.data(), sizeof(double) * r->g.size());
    if (gs && !r->gs.empty()) std::memcpy(gs, r->gs.data(), sizeof(double) * r->gs.size());
  }
  if (r->dev_x) (void)hipFree(r->dev_x);
  r->dev_x = nullptr;
  s.all.erase(itr);
  return KDE_OK;
}

}  // namespace

extern "C" {

kde_status kde_server_start(kde_ctx* c, uint64_t hbm_budget_bytes, int32_t max_slots) {
  if (!c) return KDE_E_INVAL;
  if (c->server && c->server->running) return fail(c, KDE_E_BUSY, "a server is already running");
  if (max_slots < 1 || max_slots > KDE_MAX_BATCH || hbm_budget_bytes == 0)
    return fail(c, KDE_E_INVAL, "max_slots must be in [1, KDE_MAX_BATCH] and the budget > 0");
  if (hipSetDevice(c->device) != hipSuccess) return fail(c, KDE_E_DEVICE, "hipSetDevice failed");
  c->server.reset();
  // served requests run the LSCV variant the options name (the variant does
  // not change any result, only the speed)
  c->job_hc = c->opt_hc;
  c->job_tj = c->opt_tj;
  c->job_mfma = c->opt_mfma;
  std::unique_ptr<Server, kde::ServerDeleter> s(new Server());
  s->c = c;
  s->budget = hbm_budget_bytes;
  s->max_slots = max_slots;
  kde_status st;
  if ((st = kde::ensure(c, s->st, (size_t)max_slots))) return st;
  if (hipHostMalloc((void**)&s->h_st, sizeof(kde::DevState) * max_slots, hipHostMallocDefault) != hipSuccess) {
    s->h_st = nullptr;
    return fail(c, KDE_E_NOMEM, "pinned host allocation failed");
  }
  // the whole budget, reserved once; request blocks are placed inside it
  const uint64_t arena_bytes = hbm_budget_bytes / kde::Arena::kAlign * kde::Arena::kAlign;
  if (arena_bytes == 0) return fail(c, KDE_E_INVAL, "the budget holds no block");
  if ((st = kde::ensure(c, s->arena_mem, (size_t)arena_bytes)))
    return fail(c, KDE_E_NOMEM, "the HBM budget could not be reserved on the device");
  s->arena.reset(arena_bytes);
  s->budget = arena_bytes;
  if (hipStreamCreateWithFlags(&s->copy_stream, hipStreamNonBlocking) != hipSuccess) {
    s->copy_stream = nullptr;
    return fail(c, KDE_E_DEVICE, "stream creation failed");
  }
  for (hipEvent_t& e : s->ev)
    if (hipEventCreate(&e) != hipSuccess) {
      e = nullptr;
      return fail(c, KDE_E_DEVICE, "event creation failed");
    }
  for (int k = max_slots - 1; k >= 0; --k) s->free_slots.push_back(k);
  s->running = true;
  Server* raw = s.get();
  c->server = std::move(s);
  raw->th = std::thread([raw] { raw->loop(); });
  return KDE_OK;
}

kde_status kde_submit(kde_ctx* c, const kde_request* req, uint64_t* ticket) {
  if (!c || !req || !ticket) return KDE_E_INVAL;
  Server* s = c->server.get();
  if (!s || !s->running) return fail(c, KDE_E_INVAL, "no server is running on this context");
  auto r = std::make_shared<SrvReq>();
  r->req = *req;
  // the plan copies an explicit grid; the samples are copied below
  std::string e;
  {
    // plan_column reads only the options, which cannot change while serving
    e = kde::plan_column(c, *req, r->plan);
  }
  if (!e.empty()) return fail(c, KDE_E_INVAL, e);
  r->fp = kde::Arena::round(r->plan.bytes);
  {
    const double pairs = 0.5 * (double)r->plan.n * (double)(r->plan.n - 1);
    r->work = pairs * ((r->plan.lscv ? r->plan.n_h : 0) + r->plan.stages);
  }
  const size_t bytes = r->plan.raw_bytes;
  if (req->x.on_device) {
    if (hipMalloc(&r->dev_x, bytes) != hipSuccess) return fail(c, KDE_E_NOMEM, "device copy of the column failed");
    if (hipMemcpy(r->dev_x, req->x.data, bytes, hipMemcpyDeviceToDevice) != hipSuccess) {
      (void)hipFree(r->dev_x);
      return fail(c, KDE_E_DEVICE, "device copy of the column failed");
    }
  } else {
    r->host_x.assign((const char*)req->x.data, (const char*)req->x.data + bytes);
  }
  r->req.x.data = req->x.on_device ? r->dev_x : (const void*)r->host_x.data();
  r->req.grid.h = r->plan.grid_h.empty() ? nullptr : r->plan.grid_h.data();
  r->res.g_out = r->res.gscale_out = nullptr;
  kde::init_result(r->res, KDE_OK);
  r->t_submit = kde::now_s();
  std::lock_guard<std::mutex> lk(s->mu);
  if (s->stopping) {
    if (r->dev_x) (void)hipFree(r->dev_x);
    return fail(c, KDE_E_CANCELLED, "server is stopping");
  }
  r->ticket = s->next_ticket++;
  s->queue.push_back(r);
  s->all[r->ticket] = r;
  *ticket = r->ticket;
  s->cv_work.notify_one();
  return KDE_OK;
}

kde_status kde_poll(kde_ctx* c, uint64_t ticket, kde_result* out) {
  if (!c) return KDE_E_INVAL;
  Server* s = c->server.get();
  if (!s) return fail(c, KDE_E_INVAL, "no server on this context");
  std::unique_lock<std::mutex> lk(s->mu);
  return collect(c, *s, ticket, out, lk, 0.0);
}

kde_status kde_wait(kde_ctx* c, uint64_t ticket, kde_result* out, double timeout_s) {
  if (!c) return KDE_E_INVAL;
  Server* s = c->server.get();
  if (!s) return fail(c, KDE_E_INVAL, "no server on this context");
  std::unique_lock<std::mutex> lk(s->mu);
  return collect(c, *s, ticket, out, lk, timeout_s);
}

kde_status kde_cancel(kde_ctx* c, uint64_t ticket) {
  if (!c) return KDE_E_INVAL;
  Server* s = c->server.get();
  if (!s) return fail(c, KDE_E_INVAL, "no server on this context");
  std::lock_guard<std::mutex> lk(s->mu);
  auto itr = s->all.find(ticket);
  if (itr == s->all.end()) return fail(c, KDE_E_INVAL, "unknown ticket");
  std::shared_ptr<SrvReq> r = itr->second;
  if (r->done) return KDE_OK;
  auto q = std::find(s->queue.begin(), s->queue.end(), r);
  if (q != s->queue.end()) {
    s->queue.erase(q);
    kde::finish_with(*s, r, KDE_E_CANCELLED);
    s->cv_done.notify_all();
  } else {
    r->cancel = true;
  }
  return KDE_OK;
}

kde_status kde_server_stop(kde_ctx* c) {
  if (!c) return KDE_E_INVAL;
  Server* s = c->server.get();
  if (!s || !s->running) return KDE_OK;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    s->stopping = true;
    while (!s->queue.empty()) {
      std::shared_ptr<SrvReq> r = s->queue.front();
      s->queue.pop_front();
      kde::finish_with(*s, r, KDE_E_CANCELLED);
    }
    s->cv_work.notify_all();
    s->cv_done.notify_all();
  }
  s->th.join();
  s->running = false;
  return KDE_OK;
}

}  // extern "C"
