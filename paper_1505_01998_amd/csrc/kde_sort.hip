// kde_sort.hip -- ascending sort of a column's FP32 working copy for tile
// pruning (the pair sums do not depend on the order of the samples, so only
// the keys are sorted).
//
// Least-significant-digit radix sort over 4-bit digits (eight passes of the
// 32-bit key).  Each float is first mapped to an unsigned key with the same
// order (sign bit set: all bits flipped; clear: sign bit set), so +inf
// padding sorts last.  A pass is three kernels: every block of
// kTile = 2048 keys counts its digits (16 bins); one block turns the
// counts, taken digit-major over the blocks, into exclusive offsets; every
// block then writes its keys to offset[digit][block] + the key's rank among
// the block's keys of that digit, which keeps equal digits in input order
// (the stability an LSD sort needs).  The passes ping-pong between the
// temporary buffer and the output; the first reads the input floats and the
// last writes floats back.  All work is in kernels on the caller's stream.
#include <hip/hip_runtime.h>

#include <stdint.h>

#include "kde_internal.h"

namespace kde {

namespace {

constexpr int kSortThreads = 256;
constexpr int kKeysPerThread = 8;
constexpr int kTile = kSortThreads * kKeysPerThread;
constexpr int kBins = 16;
constexpr int kPasses = 8;
constexpr int kScanThreads = 1024;

__device__ __forceinline__ uint32_t to_key(uint32_t f) { return (f & 0x80000000u) ? ~f : (f | 0x80000000u); }
__device__ __forceinline__ uint32_t from_key(uint32_t k) { return (k & 0x80000000u) ? (k & 0x7FFFFFFFu) : ~k; }

// Digit counts of each block's tile: counts[bin * nblocks + block].
template <bool FIRST>
__global__ __launch_bounds__(kSortThreads) void k_sort_count(const uint32_t* __restrict__ src, int count, int shift,
                                                             int* __restrict__ counts, int nblocks) {
  __shared__ int hist[kBins];
  if (threadIdx.x < kBins) hist[threadIdx.x] = 0;
  __syncthreads();
  const int64_t base = (int64_t)blockIdx.x * kTile;
  for (int q = 0; q < kKeysPerThread; ++q) {
    const int64_t i = base + (int64_t)q * kSortThreads + threadIdx.x;
    if (i < count) {
      const uint32_t k = FIRST ? to_key(src[i]) : src[i];
      atomicAdd(&hist[(k >> shift) & (kBins - 1)], 1);
    }
  }
  __syncthreads();
  if (threadIdx.x < kBins) counts[(int64_t)threadIdx.x * nblocks + blockIdx.x] = hist[threadIdx.x];
}

// In-place exclusive scan of counts[0 .. m) by one block.
__global__ __launch_bounds__(kScanThreads) void k_sort_scan(int* __restrict__ counts, int64_t m) {
  __shared__ int64_t part[kScanThreads];
  const int t = threadIdx.x;
  const int64_t per = (m + kScanThreads - 1) / kScanThreads;
  const int64_t a = min(m, (int64_t)t * per), b = min(m, a + per);
  int64_t s = 0;
  for (int64_t i = a; i < b; ++i) s += counts[i];
  part[t] = s;
  __syncthreads();
  for (int d = 1; d < kScanThreads; d <<= 1) {  // inclusive Hillis-Steele scan of the chunk sums
    const int64_t v = t >= d ? part[t - d] : 0;
    __syncthreads();
    part[t] += v;
    __syncthreads();
  }
  int64_t run = part[t] - s;  // exclusive prefix of this chunk
  for (int64_t i = a; i < b; ++i) {
    const int c = counts[i];
    counts[i] = (int)run;
    run += c;
  }
}

// Stable scatter of each block's tile.  Thread t holds the block's keys
// t * 8 .. t * 8 + 7 (consecutive, so thread order is input order).
template <bool FIRST, bool LAST>
__global__ __launch_bounds__(kSortThreads) void k_sort_scatter(const uint32_t* __restrict__ src,
                                                               uint32_t* __restrict__ dst, int count, int shift,
                                                               const int* __restrict__ offsets, int nblocks) {
  // per (bin, thread) counts, digit-major, then their exclusive scan
  __shared__ int cnt[kBins * kSortThreads];
  __shared__ int tsum[kSortThreads];
  const int t = threadIdx.x;
  const int64_t base = (int64_t)blockIdx.x * kTile + (int64_t)t * kKeysPerThread;
  uint32_t key[kKeysPerThread];
  int dig[kKeysPerThread];
#pragma unroll
  for (int b = 0; b < kBins; ++b) cnt[b * kSortThreads + t] = 0;
#pragma unroll
  for (int q = 0; q < kKeysPerThread; ++q) {
    const int64_t i = base + q;
    if (i < count) {
      key[q] = FIRST ? to_key(src[i]) : src[i];
      dig[q] = (int)((key[q] >> shift) & (kBins - 1));
      cnt[dig[q] * kSortThreads + t] += 1;
    } else {
      dig[q] = -1;
    }
  }
  __syncthreads();
  // exclusive scan of cnt (4096 entries) in flat order: thread t owns
  // entries [16 t, 16 t + 16)
  int own[kBins];
  int s = 0;
#pragma unroll
  for (int e = 0; e < kBins; ++e) {
    own[e] = cnt[t * kBins + e];
    s += own[e];
  }
  tsum[t] = s;
  __syncthreads();
  for (int d = 1; d < kSortThreads; d <<= 1) {
    const int v = t >= d ? tsum[t - d] : 0;
    __syncthreads();
    tsum[t] += v;
    __syncthreads();
  }
  int run = tsum[t] - s;
  __syncthreads();
#pragma unroll
  for (int e = 0; e < kBins; ++e) {
    cnt[t * kBins + e] = run;
    run += own[e];
  }
  __syncthreads();
  // a key's place: its digit's global offset for this block, plus the keys of
  // that digit in earlier threads (flat prefix minus the prefix at thread 0,
  // which counts the lower digits), plus the earlier keys of that digit here
#pragma unroll
  for (int q = 0; q < kKeysPerThread; ++q) {
    const int dg = dig[q];
    if (dg < 0) continue;
    int mine = 0;
#pragma unroll
    for (int q2 = 0; q2 < q; ++q2) mine += dig[q2] == dg ? 1 : 0;
    const int local = cnt[dg * kSortThreads + t] - cnt[dg * kSortThreads] + mine;
    const int64_t pos = (int64_t)offsets[(int64_t)dg * nblocks + blockIdx.x] + local;
    if (pos >= 0 && pos < count) dst[pos] = LAST ? from_key(key[q]) : key[q];
  }
}

}  // namespace

size_t sort_temp_bytes(int count) {
  if (count <= 0) return 0;
  const int64_t nblocks = ((int64_t)count + kTile - 1) / kTile;
  return ((size_t)count * 4 + 255) / 256 * 256 + (size_t)kBins * nblocks * 4;
}

hipError_t sort_keys(void* tmp, size_t tmp_bytes, const float* in, float* out, int count, hipStream_t s) {
  if (count <= 0) return hipSuccess;
  if (!tmp || !in || !out || tmp_bytes < sort_temp_bytes(count)) return hipErrorInvalidValue;
  const int nblocks = (int)(((int64_t)count + kTile - 1) / kTile);
  uint32_t* keys = static_cast<uint32_t*>(tmp);
  int* counts = reinterpret_cast<int*>(static_cast<char*>(tmp) + ((size_t)count * 4 + 255) / 256 * 256);
  const uint32_t* src0 = reinterpret_cast<const uint32_t*>(in);
  uint32_t* o = reinterpret_cast<uint32_t*>(out);
  // pass p reads from (p == 0 ? in : p odd ? keys : out) and writes to
  // (p even ? keys : out); with eight passes the last writes out
  for (int p = 0; p < kPasses; ++p) {
    const int shift = 4 * p;
    const uint32_t* src = p == 0 ? src0 : (p % 2 ? keys : o);
    uint32_t* dst = p % 2 ? o : keys;
    if (p == 0)
      k_sort_count<true><<<nblocks, kSortThreads, 0, s>>>(src, count, shift, counts, nblocks);
    else
      k_sort_count<false><<<nblocks, kSortThreads, 0, s>>>(src, count, shift, counts, nblocks);
    k_sort_scan<<<1, kScanThreads, 0, s>>>(counts, (int64_t)kBins * nblocks);
    if (p == 0)
      k_sort_scatter<true, false><<<nblocks, kSortThreads, 0, s>>>(src, dst, count, shift, counts, nblocks);
    else if (p == kPasses - 1)
      k_sort_scatter<false, true><<<nblocks, kSortThreads, 0, s>>>(src, dst, count, shift, counts, nblocks);
    else
      k_sort_scatter<false, false><<<nblocks, kSortThreads, 0, s>>>(src, dst, count, shift, counts, nblocks);
  }
  return hipGetLastError();
}

}  // namespace kde
