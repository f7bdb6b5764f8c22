// kde_probe.hip -- issue rates of the vector ALU on the device.
//
// The pair kernels of the selectors (Section 4.4: the psi_r double sums and
// the LSCV sums over all pairs, with the pair distance reused across
// bandwidths as in Section 4.5) keep everything in registers and LDS, so
// their speed is set by how many plain FP32 vector instructions and how many
// v_exp_f32 (the transcendental unit) a compute unit issues per clock.  This
// probe measures those rates: register-only loops of eight independent
// instruction chains per lane (so that neither dependency latency nor memory
// limits them), timed with HIP events on the caller's stream, and reported per
// clock and per compute unit at the device's nominal engine clock.  The
// roofline of the pair kernels is derived from unit counts and clock; this
// probe is the measured evidence behind the per-clock rates it assumes.
#include <hip/hip_runtime.h>

#include <string>

#include "kde_runtime.h"

namespace kde {

namespace {

constexpr int kProbeThreads = 256;
constexpr int kProbeBlocks = 4096;  // 16 blocks (64 waves) per CU on 256 CUs
constexpr int kChains = 8;          // independent chains per lane
constexpr int kPerIter = 4 * kChains;

enum ProbeOp { kOpAdd = 0, kOpMul, kOpFma, kOpExp, kOpMix };

// Each iteration issues kPerIter instructions of one kind per lane.  The
// operands b and a are kernel arguments, so nothing folds at compile time,
// and the chains stay finite (add grows slowly, mul by ~1, fma contracts,
// 2^-v has a fixed point).
template <int OP>
__global__ __launch_bounds__(kProbeThreads) void k_issue(float a, float b, int iters, float* __restrict__ out) {
  float v[kChains];
  const float lane = (float)(threadIdx.x & 63) * (1.0f / 64.0f);
#pragma unroll
  for (int k = 0; k < kChains; ++k) v[k] = a + lane + 0.125f * (float)k;
  for (int it = 0; it < iters; ++it) {
#pragma unroll
    for (int r = 0; r < 4; ++r) {
#pragma unroll
      for (int k = 0; k < kChains; ++k) {
        if (OP == kOpAdd) v[k] = v[k] + b;
        if (OP == kOpMul) v[k] = v[k] * b;
        if (OP == kOpFma) v[k] = __builtin_fmaf(v[k], b, a);
        if (OP == kOpExp) v[k] = __builtin_amdgcn_exp2f(-v[k]);
      }
    }
  }
  float s = 0.f;
#pragma unroll
  for (int k = 0; k < kChains; ++k) s += v[k];
  out[(size_t)blockIdx.x * kProbeThreads + threadIdx.x] = s;
}

// The LSCV term mix: for a pair distance t and 16 bandwidth coefficients
// c_k, e = exp2(t c_k), S1 += e, S2 += e e (one mul, one exp, one add, one
// fma per term), then the next distance t + dt (one add per 16 terms).  With
// t0 = dt = 0 every exponential is of zero.  Each term is issued in program
// order behind a scheduling barrier, with the wave's priority raised from the
// exponential to its consumers, as in the LSCV sweep's inner loop.
__global__ __launch_bounds__(kProbeThreads) void k_issue_mix(float t0, float dt, float c0, int iters,
                                                             float* __restrict__ out) {
  constexpr int HC = 16;
  float ck[HC], s1[HC], s2[HC];
#pragma unroll
  for (int k = 0; k < HC; ++k) {
    ck[k] = c0 * (float)(1 + k);
    s1[k] = 0.f;
    s2[k] = 0.f;
  }
  float t = t0 * (float)(threadIdx.x & 63) * (1.0f / 16.0f);
  for (int it = 0; it < iters; ++it) {
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      t = t + dt;
#pragma unroll
      for (int k = 0; k < HC; ++k) {
        __builtin_amdgcn_s_setprio(1);
        const float e = __builtin_amdgcn_exp2f(t * ck[k]);
        s1[k] += e;
        s2[k] = __builtin_fmaf(e, e, s2[k]);
        __builtin_amdgcn_s_setprio(0);
        __builtin_amdgcn_sched_barrier(0);
      }
    }
  }
  float s = 0.f;
#pragma unroll
  for (int k = 0; k < HC; ++k) s += s1[k] + s2[k];
  out[(size_t)blockIdx.x * kProbeThreads + threadIdx.x] = s;
}

void launch_issue(hipStream_t st, int op, int iters, float* out, float t0) {
  switch (op) {
    case kOpAdd: k_issue<kOpAdd><<<kProbeBlocks, kProbeThreads, 0, st>>>(0.5f, 1e-7f, iters, out); break;
    case kOpMul: k_issue<kOpMul><<<kProbeBlocks, kProbeThreads, 0, st>>>(0.5f, 1.0000001f, iters, out); break;
    case kOpFma: k_issue<kOpFma><<<kProbeBlocks, kProbeThreads, 0, st>>>(0.5f, 0.5f, iters, out); break;
    case kOpExp: k_issue<kOpExp><<<kProbeBlocks, kProbeThreads, 0, st>>>(0.5f, 0.f, iters, out); break;
    default:
      // distances spread over [0, 4) with per-lane offsets; coefficients of
      // bandwidths between 0.06 and 0.25, so the exponentials range over
      // (2^-50, 1] like a real grid's
      k_issue_mix<<<kProbeBlocks, kProbeThreads, 0, st>>>(t0, t0 * 1e-4f, -0.2f, iters, out);
      break;
  }
}

}  // namespace

}  // namespace kde

extern "C" kde_status kde_issue_rates(kde_ctx* c, kde_issue_info* out) {
  using namespace kde;
  if (!c || !out) return KDE_E_INVAL;
  if (c->server && server_running(c->server.get())) return fail(c, KDE_E_BUSY, "a server is running on this context");
  if (hipSetDevice(c->device) != hipSuccess) return fail(c, KDE_E_DEVICE, "hipSetDevice failed");
  hipDeviceProp_t prop;
  KDE_HIP_TRY(c, hipGetDeviceProperties(&prop, c->device));
  const double clock = (double)prop.clockRate * 1e3;  // reported in kHz
  const int cus = prop.multiProcessorCount;
  if (!(clock > 0.0) || cus <= 0) return fail(c, KDE_E_DEVICE, "device reports no clock or compute units");
  kde_status s;
  const size_t bytes = sizeof(float) * (size_t)kProbeBlocks * kProbeThreads;
  if ((s = ensure(c, c->tune_buf, bytes))) return s;
  float* buf = (float*)c->tune_buf.p;
  hipEvent_t ev[2];
  int made = 0;
  hipError_t he = hipSuccess;
  for (; made < 2 && he == hipSuccess; ++made) he = hipEventCreate(&ev[made]);
  if (he != hipSuccess) --made;
  // (op, iterations, instructions or terms per lane and iteration, t0)
  struct Case {
    int op, iters;
    double per_iter;
    float t0;
    double* dst;
  };
  const Case cases[] = {
      {kOpAdd, 65536, (double)kPerIter, 0.f, &out->add_f32},
      {kOpMul, 65536, (double)kPerIter, 0.f, &out->mul_f32},
      {kOpFma, 65536, (double)kPerIter, 0.f, &out->fma_f32},
      {kOpExp, 16384, (double)kPerIter, 0.f, &out->exp_f32},
      {kOpMix, 4096, 64.0, 4.0f, &out->lscv_mix},
      {kOpMix, 4096, 64.0, 0.0f, &out->lscv_mix_zero},
  };
  for (const Case& k : cases) {
    if (he != hipSuccess) break;
    launch_issue(c->stream, k.op, k.iters / 8, buf, k.t0);  // warm-up
    he = hipEventRecord(ev[0], c->stream);
    if (he == hipSuccess) {
      launch_issue(c->stream, k.op, k.iters, buf, k.t0);
      he = hipEventRecord(ev[1], c->stream);
    }
    if (he == hipSuccess) he = hipGetLastError();
    if (he == hipSuccess) he = hipEventSynchronize(ev[1]);
    float ms = 0.f;
    if (he == hipSuccess) he = hipEventElapsedTime(&ms, ev[0], ev[1]);
    const double lanes = (double)kProbeBlocks * kProbeThreads * k.iters * k.per_iter;
    *k.dst = (he == hipSuccess && ms > 0.f) ? lanes / (ms * 1e-3) / (clock * cus) : 0.0;
  }
  for (int k = 0; k < made; ++k) (void)hipEventDestroy(ev[k]);
  if (he != hipSuccess) return fail(c, KDE_E_DEVICE, std::string("issue-rate probe: ") + hipGetErrorString(he));
  out->clock_hz = clock;
  out->cus = cus;
  out->pad0 = 0;
  return KDE_OK;
}
