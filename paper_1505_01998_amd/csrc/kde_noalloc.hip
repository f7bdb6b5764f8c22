// kde_noalloc.hip -- kde_lscv_curve_noalloc: the LSCV objective curve of one
// column computed without allocating memory.
//
// The call runs exactly the job kde_lscv_curve runs (same planner, same
// kernels, same reduction order, so the same values bit for bit), with every
// device buffer of that job carved from one file-scope device array
// (`scratch`, KDE_NOALLOC_SCRATCH_BYTES per device, held from the library's
// load until the process ends) and the host staging in pageable vectors of
// the context, grown on their first use and reused after.  The context is switched to a fixed-workspace mode for
// the call: a buffer that would have to grow makes the call fail with
// KDE_E_NOMEM instead of allocating, and graph replay and kernel timing
// (which create graphs and events) are off.
//
// Host code never passes `scratch` itself to a kernel or a copy: the name is
// a host-side stand-in, not the device address.  The address is looked up
// once per device with hipGetSymbolAddress (at context creation, with the
// device current) and kept per device in g_dev_ptr[].
#include <hip/hip_runtime.h>

#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "kde_bw.h"
#include "kde_internal.h"
#include "kde_runtime.h"

static constexpr size_t kScratchBytes = (size_t)KDE_NOALLOC_SCRATCH_BYTES;

static __device__ __align__(256) char scratch[kScratchBytes];

namespace {

constexpr int kMaxDevices = 64;

std::mutex g_mu;
char* g_dev_ptr[kMaxDevices] = {};
hipError_t g_dev_err[kMaxDevices] = {};

size_t round256(size_t b) { return (b + 255) / 256 * 256; }

// The device address of this device's scratch, or null with *err saying why.
char* scratch_of(int device, hipError_t* err) {
  *err = hipErrorInvalidDevice;
  if (device < 0 || device >= kMaxDevices) return nullptr;
  std::lock_guard<std::mutex> lk(g_mu);
  *err = g_dev_ptr[device] ? hipSuccess : g_dev_err[device];
  return g_dev_ptr[device];
}

// Swaps the context's job buffers for slices of the scratch and the call's
// host buffers, and puts everything back on destruction (after the stream
// has drained, so no copy still reads or writes the call's host buffers).
struct FixedWorkspace {
  kde_ctx* c;
  kde::DevBuf<char> blocks, blob, sort_tmp;
  kde::DevBuf<kde::DevState> st;
  kde::DevState* h_st;
  size_t h_st_cap;
  double* h_out;
  size_t h_out_cap;
  char* h_blob;
  size_t h_blob_cap;
  int opt_graph;
  bool timing;

  FixedWorkspace(kde_ctx* ctx, char* base, size_t st_bytes, size_t block_bytes, size_t sort_bytes, size_t blob_bytes,
                 size_t out_doubles)
      : c(ctx),
        blocks(ctx->blocks),
        blob(ctx->blob),
        sort_tmp(ctx->sort_tmp),
        st(ctx->st),
        h_st(ctx->h_st),
        h_st_cap(ctx->h_st_cap),
        h_out(ctx->h_out),
        h_out_cap(ctx->h_out_cap),
        h_blob(ctx->h_blob),
        h_blob_cap(ctx->h_blob_cap),
        opt_graph(ctx->opt_graph),
        timing(ctx->timing) {
    // host staging: the context's pageable vectors, grown on first use only
    if (c->na_st.size() < 1) c->na_st.resize(1);
    if (c->na_out.size() < out_doubles) c->na_out.resize(out_doubles);
    if (c->na_blob.size() < blob_bytes) c->na_blob.resize(blob_bytes);
    size_t at = 0;
    c->st.p = reinterpret_cast<kde::DevState*>(base + at);
    c->st.cap = 1;
    at += st_bytes;
    c->blocks.p = base + at;
    c->blocks.cap = block_bytes;
    at += block_bytes;
    c->sort_tmp.p = sort_bytes ? base + at : nullptr;
    c->sort_tmp.cap = sort_bytes;
    at += sort_bytes;
    c->blob.p = base + at;
    c->blob.cap = blob_bytes;
    c->h_st = c->na_st.data();
    c->h_st_cap = sizeof(kde::DevState);
    c->h_out = c->na_out.data();
    c->h_out_cap = out_doubles;
    c->h_blob = c->na_blob.data();
    c->h_blob_cap = blob_bytes;
    c->opt_graph = 0;
    c->timing = false;
    c->no_alloc = true;
  }

  ~FixedWorkspace() {
    (void)hipStreamSynchronize(c->stream);
    c->blocks = blocks;
    c->blob = blob;
    c->sort_tmp = sort_tmp;
    c->st = st;
    c->h_st = h_st;
    c->h_st_cap = h_st_cap;
    c->h_out = h_out;
    c->h_out_cap = h_out_cap;
    c->h_blob = h_blob;
    c->h_blob_cap = h_blob_cap;
    c->opt_graph = opt_graph;
    c->timing = timing;
    c->no_alloc = false;
    // the job's plan and executor plan point into the scratch; drop them so
    // no later call mistakes them for the context's own
    c->plans.clear();
    c->plan_req.clear();
    c->iter.clear();
  }
};

}  // namespace

void kde::noalloc_setup(kde_ctx* c) {
  const int dev = c->device;
  if (dev < 0 || dev >= kMaxDevices) return;
  std::lock_guard<std::mutex> lk(g_mu);
  if (g_dev_ptr[dev]) return;
  void* p = nullptr;
  const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
  if (e == hipSuccess && p) {
    g_dev_ptr[dev] = static_cast<char*>(p);
    g_dev_err[dev] = hipSuccess;
  } else {
    g_dev_err[dev] = e == hipSuccess ? hipErrorInvalidSymbol : e;
    (void)hipGetLastError();  // the failure is reported by the entry point, not by the next call
  }
}

extern "C" kde_status kde_lscv_curve_noalloc(kde_ctx* c, kde_column x, const double* h_grid, int32_t n_h,
                                             double* g_out, double* gscale_out) {
  if (!c || !g_out) return KDE_E_INVAL;
  if (c->server && kde::server_running(c->server.get()))
    return kde::fail(c, KDE_E_BUSY, "a server is running on this context");
  if (hipSetDevice(c->device) != hipSuccess) return kde::fail(c, KDE_E_DEVICE, "hipSetDevice failed");
  hipError_t he;
  char* base = scratch_of(c->device, &he);
  if (!base)
    return kde::fail(c, KDE_E_DEVICE,
                     std::string("device address of the fixed scratch unavailable: ") + hipGetErrorString(he));
  if (c->opt_autotune && c->prec == KDE_PREC_MIXED)
    return kde::fail(c, KDE_E_INVAL, "the autotune option may allocate a trial buffer; switch it off for this call");
  if (!h_grid && n_h <= 0) n_h = 150;
  kde_request r;
  std::memset(&r, 0, sizeof(r));
  r.x = x;
  r.methods = KDE_METHOD_LSCV;
  r.stages = 2;
  if (h_grid) {
    r.grid.kind = KDE_GRID_EXPLICIT;
    r.grid.h = h_grid;
    r.grid.n_h = n_h;
  } else {
    r.grid.kind = KDE_GRID_PAPER;
    r.grid.n_h = n_h;
  }
  // size the job exactly as the executor will: the column's block, its state
  // and (with tile pruning) the sort's temporary; the blob (column table,
  // work units, rows) gets what is left
  kde::ColPlan p;
  std::string e = kde::plan_column(c, r, p);
  if (!e.empty()) return kde::fail(c, KDE_E_INVAL, e);
  const size_t st_bytes = round256(sizeof(kde::DevState));
  const size_t block_bytes = round256(p.bytes);
  const size_t sort_bytes = p.prune ? round256(kde::sort_temp_bytes((int)(p.n + kde::kPad))) : 0;
  const size_t fixed = st_bytes + block_bytes + sort_bytes;
  if (fixed + 4096 > kScratchBytes)
    return kde::fail(c, KDE_E_NOMEM,
                     "column needs " + std::to_string(fixed) + " bytes of device workspace; the fixed scratch of "
                     "kde_lscv_curve_noalloc holds " + std::to_string(kScratchBytes));
  kde_status s;
  {
    FixedWorkspace ws(c, base, st_bytes, block_bytes, sort_bytes, kScratchBytes - fixed, (size_t)3 * n_h);
    s = kde::lscv_curve_call(c, x, h_grid, n_h, g_out, gscale_out, nullptr);
  }
  return s;
}
