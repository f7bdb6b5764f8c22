// kde_job.hip -- resumable requests: one bandwidth-selection request run on
// the caller's thread in slices of at most a given number of pair-term
// evaluations, with checkpoints that a later job (another context, another
// process) resumes from.
//
// A job owns its column's device block (the same plan and layout as in a
// batch or a server slot) and its device state, and walks the request's work
// in the server's order: moments, the plug-in stages unit by unit, the LSCV
// prep and units, the fixed-order row reductions and the finalisation.  Each
// work unit writes its own partial sums, and every reduction runs in a fixed
// order once the units it reads are complete, so the results do not depend
// on how the work was sliced or where it was interrupted: a job run in any
// slices, or checkpointed and resumed, gives results bitwise equal to the
// same request run through kde_batch.  A checkpoint is the job's cursor, its
// device state and a copy of its block (samples, working copies, partial
// sums); the samples travel with it.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "kde_runtime.h"

struct kde_job {
  kde_ctx* c = nullptr;
  kde::ColPlan plan;
  char* block = nullptr;
  kde::DevState* st = nullptr;  // device state of the column
  kde::DevState h_st{};
  int hc = 16, mfma = 0, cond = 0, prec = 0;
  bool started = false, failed = false;
  bool stats_done = false, plugin_done = false, prep_done = false, lscv_done = false, done = false;
  int stage = 0;
  size_t psi_next = 0, lscv_next = 0;
  std::vector<kde::Unit> psi_u, lscv_u;
  std::vector<kde::UnitCost> psi_c, lscv_c;
  double total = 0.0, remaining = 0.0;
  kde_result res{};
  std::vector<double> g, gs;
};

namespace {

using kde::fail;

// Checkpoint header; the block bytes, then g and gscale (n_h each) follow.
struct JobHeader {
  char magic[8];
  int32_t version, n, f64, plugin, lscv, stages, n_h, hc, mfma, cond, prec, grid_kind, prune;
  int64_t items_psi, items_lscv, block_bytes;
  int32_t stats_done, plugin_done, prep_done, lscv_done, done, stage;
  int64_t psi_next, lscv_next;
  double remaining, total;
  kde::DevState st;
  kde_result res;
};

constexpr char kMagic[8] = {'K', 'D', 'E', 'J', 'O', 'B', '\0', '\0'};
constexpr int32_t kVersion = 2;

bool serving(const kde_ctx* c) { return c->server && kde::server_running(c->server.get()); }

uint64_t ckpt_bytes(const kde_job* j) {
  return sizeof(JobHeader) + (uint64_t)j->plan.bytes + 16 * (uint64_t)j->plan.n_h;
}

void take(const std::vector<kde::Unit>& u, const std::vector<kde::UnitCost>& cu, size_t& next, double& budget,
          bool force, std::vector<kde::Unit>& out, std::vector<kde::UnitCost>& out_c, double& remaining) {
  while (next < u.size() && (budget > 0.0 || force)) {
    out.push_back(u[next]);
    out_c.push_back(cu[next]);
    budget -= cu[next].evals;
    remaining -= cu[next].evals;
    ++next;
    force = false;
  }
}

}  // namespace

extern "C" {

kde_status kde_job_create(kde_ctx* c, const kde_request* req, kde_job** out) {
  if (!c || !req || !out) return KDE_E_INVAL;
  *out = nullptr;
  if (serving(c)) return fail(c, KDE_E_BUSY, "a server is running");
  if (hipSetDevice(c->device) != hipSuccess) return fail(c, KDE_E_DEVICE, "hipSetDevice failed");
  std::unique_ptr<kde_job> j(new kde_job());
  j->c = c;
  j->hc = c->opt_hc;
  j->mfma = c->opt_mfma;
  j->prec = (int)c->prec;
  j->cond = c->prec != KDE_PREC_FP64 && c->opt_fp64_kappa > 0.0;
  c->job_hc = j->hc;
  c->job_tj = c->opt_tj;
  c->job_mfma = j->mfma;
  // plan as a host column so the block holds the samples (a checkpoint then
  // carries them); device samples are copied into the block below
  kde_request r = *req;
  r.x.on_device = 0;
  std::string e = kde::plan_column(c, r, j->plan);
  if (!e.empty()) return fail(c, KDE_E_INVAL, e);
  kde::ColPlan& p = j->plan;
  if (hipMalloc((void**)&j->block, p.bytes) != hipSuccess) {
    j->block = nullptr;
    return fail(c, KDE_E_NOMEM, "device allocation of the job's block failed");
  }
  if (hipMalloc((void**)&j->st, sizeof(kde::DevState)) != hipSuccess) {
    j->st = nullptr;
    (void)hipFree(j->block);
    return fail(c, KDE_E_NOMEM, "device allocation of the job's state failed");
  }
  kde_status s = KDE_OK;
  hipError_t he = hipMemcpy(j->block + p.off_raw, req->x.data, p.raw_bytes,
                            req->x.on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice);
  if (he == hipSuccess && p.lscv && p.grid_kind == KDE_GRID_EXPLICIT)
    he = hipMemcpy(j->block + p.off_hin, p.grid_h.data(), sizeof(double) * p.n_h, hipMemcpyHostToDevice);
  kde::init_state(p, c->opt_fp64_kappa, j->h_st);
  if (he == hipSuccess) he = hipMemcpy(j->st, &j->h_st, sizeof(kde::DevState), hipMemcpyHostToDevice);
  if (he != hipSuccess) s = fail(c, KDE_E_DEVICE, std::string("job setup copy failed: ") + hipGetErrorString(he));
  if (s) {
    (void)hipFree(j->block);
    (void)hipFree(j->st);
    return s;
  }
  kde::psi_units_of(p, 0, j->psi_u, j->psi_c);
  // with tile pruning the sweep units name the pruned-sweep descriptor (2)
  kde::lscv_units_of(p, p.prune ? 2 : 0, j->lscv_u, j->lscv_c);
  j->stage = p.stages == 3 ? 0 : 1;
  for (const kde::UnitCost& u : j->psi_c) j->total += u.evals * (3 - j->stage);
  for (const kde::UnitCost& u : j->lscv_c) j->total += u.evals;
  j->remaining = j->total;
  j->res.g_out = j->res.gscale_out = nullptr;
  kde::init_result(j->res, KDE_OK);
  c->jobs.push_back(j.get());
  *out = j.release();
  return KDE_OK;
}

void kde_job_destroy(kde_job* j) {
  if (!j) return;
  auto& v = j->c->jobs;
  v.erase(std::remove(v.begin(), v.end(), j), v.end());
  (void)hipSetDevice(j->c->device);
  if (j->block) (void)hipFree(j->block);
  if (j->st) (void)hipFree(j->st);
  delete j;
}

kde_status kde_job_run(kde_job* j, double max_evals, int* done_out) {
  if (!j || !(max_evals > 0.0)) return KDE_E_INVAL;
  kde_ctx* c = j->c;
  if (j->failed) return fail(c, KDE_E_DEVICE, "the job failed earlier");
  if (j->done) {
    if (done_out) *done_out = 1;
    return KDE_OK;
  }
  if (serving(c)) return fail(c, KDE_E_BUSY, "a server is running");
  if ((int)c->prec != j->prec) return fail(c, KDE_E_INVAL, "the context's precision changed since the job began");
  if (hipSetDevice(c->device) != hipSuccess) return fail(c, KDE_E_DEVICE, "hipSetDevice failed");
  c->job_hc = j->hc;
  c->job_tj = c->opt_tj;
  c->job_mfma = j->mfma;
  j->started = true;
  const kde::ColPlan& p = j->plan;
  kde::IterPlan& it = c->iter;
  it.clear();
  // column table: the column at 0; with tile pruning its near-tile and
  // pruned-sweep descriptors at 1 and 2
  it.cols.assign(p.prune ? 3 : 1, kde::ColDesc());
  kde::ColDesc d;
  kde::bind_column(p, j->block, nullptr, j->st, d);
  it.cols[0] = d;
  if (p.lscv && p.prune) kde::prune_descs(p, d, it.cols[1], it.cols[2]);
  double left = max_evals;
  bool first = true;
  if (!j->stats_done) {
    it.ids_stats.push_back(0);
    it.max_stat_blocks = std::min(kde::kStatBlocks, (p.n + 2047) / 2048);
    j->stats_done = true;
  }
  if (p.plugin && !j->plugin_done) {
    while (j->stage < 3) {
      const int s = j->stage;
      if (j->psi_next == 0) it.ids_begin[s].push_back(0);
      take(j->psi_u, j->psi_c, j->psi_next, left, first, it.psi_units[s], it.psi_cost[s], j->remaining);
      first = false;
      if (j->psi_next < j->psi_u.size()) break;
      it.ids_finish[s].push_back(0);
      kde::psi_rows_of(p, d, it.psi_rows[s]);
      if (j->cond) kde::psi_units_of(p, 0, it.psi_cond_units[s], it.psi_cond_cost[s]);
      j->stage++;
      j->psi_next = 0;
      if (left <= 0.0) break;
    }
    if (j->stage == 3) {
      it.ids_plugin_final.push_back(0);
      j->plugin_done = true;
    }
  }
  if (p.lscv && !j->lscv_done && (!p.plugin || j->plugin_done || left > 0.0)) {
    if (!j->prep_done) {
      it.ids_lscv_prep.push_back(0);
      if (p.prune) kde::add_prune_setup(p, d, 0, 1, it);
      j->prep_done = true;
    }
    take(j->lscv_u, j->lscv_c, j->lscv_next, left, first, p.prune ? it.prune_units : it.lscv_units,
         p.prune ? it.prune_cost : it.lscv_cost, j->remaining);
    if (j->lscv_next == j->lscv_u.size()) {
      kde::lscv_rows_of(p, d, it.lscv_rows);
      it.ids_lscv_final.push_back(0);
      j->lscv_done = true;
    }
  }
  const bool finishing = (!p.plugin || j->plugin_done) && (!p.lscv || j->lscv_done);
  kde_status s = kde::execute(c, it);
  if (!s && finishing) {
    if (p.lscv) {
      j->g.assign(p.n_h, 0.0);
      j->gs.assign(p.n_h, 0.0);
    }
    hipError_t he = hipMemcpyAsync(&j->h_st, j->st, sizeof(kde::DevState), hipMemcpyDeviceToHost, c->stream);
    if (he == hipSuccess && p.lscv)
      he = hipMemcpyAsync(j->g.data(), d.g, sizeof(double) * p.n_h, hipMemcpyDeviceToHost, c->stream);
    if (he == hipSuccess && p.lscv)
      he = hipMemcpyAsync(j->gs.data(), d.gs, sizeof(double) * p.n_h, hipMemcpyDeviceToHost, c->stream);
    if (he != hipSuccess) s = fail(c, KDE_E_DEVICE, std::string("job copy-back failed: ") + hipGetErrorString(he));
  }
  if (!s) s = kde::sync_and_check(c);
  if (s) {
    j->failed = true;
    return s;
  }
  if (finishing) {
    kde::fill_result(p, j->h_st, j->res);
    j->done = true;
  }
  if (done_out) *done_out = j->done ? 1 : 0;
  return KDE_OK;
}

kde_status kde_job_progress(const kde_job* j, double* evals_done, double* evals_total, int* done_out) {
  if (!j) return KDE_E_INVAL;
  if (evals_done) *evals_done = j->total - j->remaining;
  if (evals_total) *evals_total = j->total;
  if (done_out) *done_out = j->done ? 1 : 0;
  return KDE_OK;
}

kde_status kde_job_result(kde_job* j, kde_result* out) {
  if (!j || !out) return KDE_E_INVAL;
  if (!j->done) return KDE_E_BUSY;
  double* g = out->g_out;
  double* gs = out->gscale_out;
  *out = j->res;
  out->g_out = g;
  out->gscale_out = gs;
  if (g && !j->g.empty()) std::memcpy(g, j->g.data(), sizeof(double) * j->g.size());
  if (gs && !j->gs.empty()) std::memcpy(gs, j->gs.data(), sizeof(double) * j->gs.size());
  return KDE_OK;
}

kde_status kde_job_checkpoint_bytes(const kde_job* j, uint64_t* bytes) {
  if (!j || !bytes) return KDE_E_INVAL;
  *bytes = ckpt_bytes(j);
  return KDE_OK;
}

kde_status kde_job_checkpoint(kde_job* j, void* buf, uint64_t bytes) {
  if (!j || !buf) return KDE_E_INVAL;
  kde_ctx* c = j->c;
  if (bytes < ckpt_bytes(j)) return fail(c, KDE_E_INVAL, "checkpoint buffer smaller than kde_job_checkpoint_bytes");
  if (j->failed) return fail(c, KDE_E_DEVICE, "the job failed earlier");
  if (hipSetDevice(c->device) != hipSuccess) return fail(c, KDE_E_DEVICE, "hipSetDevice failed");
  const kde::ColPlan& p = j->plan;
  JobHeader h;
  std::memset(&h, 0, sizeof(h));
  std::memcpy(h.magic, kMagic, sizeof(kMagic));
  h.version = kVersion;
  h.n = p.n;
  h.f64 = p.f64;
  h.plugin = p.plugin;
  h.lscv = p.lscv;
  h.stages = p.stages;
  h.n_h = p.n_h;
  h.hc = j->hc;
  h.mfma = j->mfma;
  h.cond = j->cond;
  h.prec = j->prec;
  h.grid_kind = p.grid_kind;
  h.prune = p.prune;
  h.items_psi = (int64_t)p.psi_items.pairs.size();
  h.items_lscv = (int64_t)p.lscv_items.pairs.size();
  h.block_bytes = (int64_t)p.bytes;
  h.stats_done = j->stats_done;
  h.plugin_done = j->plugin_done;
  h.prep_done = j->prep_done;
  h.lscv_done = j->lscv_done;
  h.done = j->done;
  h.stage = j->stage;
  h.psi_next = (int64_t)j->psi_next;
  h.lscv_next = (int64_t)j->lscv_next;
  h.remaining = j->remaining;
  h.total = j->total;
  char* o = (char*)buf;
  KDE_HIP_TRY(c, hipMemcpy(&h.st, j->st, sizeof(kde::DevState), hipMemcpyDeviceToHost));
  KDE_HIP_TRY(c, hipMemcpy(o + sizeof(JobHeader), j->block, p.bytes, hipMemcpyDeviceToHost));
  h.res = j->res;
  h.res.g_out = h.res.gscale_out = nullptr;
  std::memcpy(o, &h, sizeof(h));
  double* tail = (double*)(o + sizeof(JobHeader) + p.bytes);
  for (int k = 0; k < p.n_h; ++k) {
    tail[k] = j->done && !j->g.empty() ? j->g[k] : 0.0;
    tail[p.n_h + k] = j->done && !j->gs.empty() ? j->gs[k] : 0.0;
  }
  return KDE_OK;
}

kde_status kde_job_resume(kde_job* j, const void* buf, uint64_t bytes) {
  if (!j || !buf) return KDE_E_INVAL;
  kde_ctx* c = j->c;
  if (j->started || j->failed) return fail(c, KDE_E_INVAL, "resume needs a job that has not run");
  if (bytes < sizeof(JobHeader)) return fail(c, KDE_E_INVAL, "checkpoint too short");
  JobHeader h;
  std::memcpy(&h, buf, sizeof(h));
  const kde::ColPlan& p = j->plan;
  const bool same = std::memcmp(h.magic, kMagic, sizeof(kMagic)) == 0 && h.version == kVersion && h.n == p.n &&
                    h.f64 == p.f64 && h.plugin == (int)p.plugin && h.lscv == (int)p.lscv && h.stages == p.stages &&
                    h.n_h == p.n_h && h.hc == j->hc && h.mfma == j->mfma && h.cond == j->cond &&
                    h.prec == j->prec && h.grid_kind == p.grid_kind && h.prune == (int)p.prune &&
                    h.items_psi == (int64_t)p.psi_items.pairs.size() &&
                    h.items_lscv == (int64_t)p.lscv_items.pairs.size() && h.block_bytes == (int64_t)p.bytes;
  if (!same)
    return fail(c, KDE_E_INVAL,
                "checkpoint does not belong to this request shape, precision and options (or is not a checkpoint)");
  if (bytes < ckpt_bytes(j)) return fail(c, KDE_E_INVAL, "checkpoint truncated");
  if (h.stage < 0 || h.stage > 3 || h.psi_next < 0 || h.psi_next > (int64_t)j->psi_u.size() || h.lscv_next < 0 ||
      h.lscv_next > (int64_t)j->lscv_u.size())
    return fail(c, KDE_E_INVAL, "checkpoint cursor out of range");
  if (hipSetDevice(c->device) != hipSuccess) return fail(c, KDE_E_DEVICE, "hipSetDevice failed");
  const char* in = (const char*)buf;
  KDE_HIP_TRY(c, hipMemcpy(j->block, in + sizeof(JobHeader), p.bytes, hipMemcpyHostToDevice));
  KDE_HIP_TRY(c, hipMemcpy(j->st, &h.st, sizeof(kde::DevState), hipMemcpyHostToDevice));
  j->h_st = h.st;
  j->stats_done = h.stats_done;
  j->plugin_done = h.plugin_done;
  j->prep_done = h.prep_done;
  j->lscv_done = h.lscv_done;
  j->done = h.done;
  j->stage = h.stage;
  j->psi_next = (size_t)h.psi_next;
  j->lscv_next = (size_t)h.lscv_next;
  j->remaining = h.remaining;
  j->total = h.total;
  j->started = true;
  if (j->done) {
    j->res = h.res;
    j->res.g_out = j->res.gscale_out = nullptr;
    const double* tail = (const double*)(in + sizeof(JobHeader) + p.bytes);
    if (p.lscv) {
      j->g.assign(tail, tail + p.n_h);
      j->gs.assign(tail + p.n_h, tail + 2 * p.n_h);
    }
  }
  return KDE_OK;
}

}  // extern "C"
