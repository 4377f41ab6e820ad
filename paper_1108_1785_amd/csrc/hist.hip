// Rate histograms (§III.B.2, TransRate Kernel: per-rate frequency counts in
// 10 kbps buckets per site and direction, from which the median is read),
// gathered without device-scope atomics.
//
// A histogram cell is touched by few flows (a 10 M-record window of 1,000
// sites fills about 180 thousand of its 20 million cells), so a workgroup's
// LDS cache of (row, bucket) counters keeps missing, and the misses and the
// flushes then cost one device-scope atomic each.  Here the classify kernel
// only stages a 32-bit key per bulk flow (hist.h) and, when its LDS has room,
// counts its keys per partition (a range of 2^shift rows); then
//   1. (only when the classify kernel did not count) part_count_kernel;
//   2. part_scan_kernel: per partition, the offset of every classify
//      workgroup's share, and the totals.  A partition with more keys than
//      one reduce slice holds (the rows of the most popular sites) gets
//      overflow slices, numbered from a counter;
//   3. part_scatter_kernel: every key to its partition's range; unless the
//      call accumulates, every scatter workgroup also zeroes its share of
//      the rows of the partitions with overflow slices;
//   4. hist_reduce_kernel: one workgroup per partition (its first slice) and
//      per overflow slice counts its keys in an LDS copy of the partition's
//      rows (LDS atomics).  The only slice of a partition then writes the
//      rows whole (16-byte stores, zeros included), or adds its counts into
//      them when the call accumulates; the slices of a split partition add
//      their non-zero counts with device atomics.
// The histograms need no zeroing pass of their own: every row of a call is
// written by the reduce, or zeroed by the scatter.  (Zeroing them in the
// classify kernel instead, a few 16-byte stores per tile, measured 15 us
// slower there and saved only 3 us in the reduce.)
#include <hip/hip_runtime.h>

#include <cstdint>
#include <mutex>
#include <string>

#include "gnm_device.h"
#include "hist.h"
#include "partition.h"
#include "registry.h"

namespace gnm {

namespace {

constexpr uint32_t kSliceEntries = 16384;  // keys per reduce slice, all of a lane's loads in flight at once
constexpr uint32_t kRowsMax = 65536;      // rows over all windows of a staged call (2^shift <= 4 per partition)
constexpr uint32_t kPartsTarget = 4096;   // partitions above which 2 (then 4) rows share one
constexpr uint32_t kOwnerPartBits = 14;   // overflow slice owner: slice << 14 | partition (< 16,384)
constexpr uint32_t kBucketMask = (1u << kHistBucketBits) - 1u;

static_assert(kBuckets <= kBucketMask + 1u, "a bucket fits the key's low bits");

// log2 of the rows per partition: the fewest that keep the partitions
// within kPartsTarget (the classify kernel's LDS counters, the count
// matrix), and within the partition kernels' limit.
uint32_t row_shift(uint32_t total_rows) {
  uint32_t s = 0;
  while (s < 2u && ((total_rows + (1u << s) - 1u) >> s) > kPartsTarget) ++s;
  return s;
}

struct Plan {
  uint32_t total_rows, shift, real, nparts;
  uint64_t over;  // most overflow slices a call can have: one per kSliceEntries keys
};

Plan plan(uint64_t n, uint32_t n_windows, uint32_t hist_rows) {
  Plan q{};
  q.total_rows = n_windows * hist_rows;
  q.shift = row_shift(q.total_rows);
  q.real = (q.total_rows + (1u << q.shift) - 1u) >> q.shift;
  q.nparts = (q.real + 63u) & ~63u;  // the scan kernel takes partitions 64 at a time
  q.over = (n + kSliceEntries - 1u) / kSliceEntries;
  return q;
}

// The partition kernels' arrays, then the overflow-slice counter and the
// overflow slices' owners.
struct Layout {
  PartLayout part;
  uint64_t over, owner, end;
};

Layout layout(uint64_t n, uint64_t grid, const Plan &q) {
  Layout L{};
  L.part = part_layout(n, grid, q.nparts, 4u);
  L.over = L.part.end;
  L.owner = part_align256(L.over + 8u);
  L.end = part_align256(L.owner + 4u * q.over);
  return L;
}

// Partition of a staged key: its range of 2^shift rows.
struct HistPart {
  uint32_t shift, real, total_rows, accumulate;
  uint32_t *hist;
  u64 *over;        // overflow slices handed out
  uint32_t *owner;  // overflow slice o: (slice within its partition) << 14 | partition
  static constexpr bool kTotalsHook = true;
  static __device__ __forceinline__ uint32_t part(const uint32_t &key, const HistPart &t) {
    return key >> (kHistBucketBits + t.shift);
  }
  // Partitions p0 .. p0 + 63 of one scan workgroup with more keys than a
  // slice: their overflow slices, numbered with one device atomic for the
  // workgroup.
  static __device__ __forceinline__ void totals(const uint32_t *tot, uint32_t p0, const HistPart &t) {
    if (threadIdx.x >= 64u) return;
    const uint32_t c = tot[threadIdx.x], p = p0 + threadIdx.x;
    const uint32_t extra = (c > kSliceEntries && p < t.real) ? (c - 1u) / kSliceEntries : 0u;
    uint32_t x = extra;  // inclusive prefix over the 64 partitions
#pragma unroll
    for (uint32_t o = 1; o < 64u; o <<= 1) {
      const uint32_t y = __shfl_up(x, o, 64);
      if (threadIdx.x >= o) x += y;
    }
    const uint32_t all = __shfl(x, 63, 64);
    uint32_t base = 0;
    if (all && threadIdx.x == 0)
      base = (uint32_t)__hip_atomic_fetch_add(t.over, (u64)all, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    base = __shfl(base, 0, 64) + x - extra;
    for (uint32_t j = 1; j <= extra; ++j) t.owner[base + j - 1u] = (j << kOwnerPartBits) | p;
  }
  // Unless accumulating, scatter workgroup b of `grid` zeroes its share of
  // the rows of every partition split into several slices (for the slices'
  // atomics); tot: every partition's keys.
  static __device__ __forceinline__ void scatter_share(const uint32_t *tot, uint32_t P, const HistPart &t,
                                                       uint32_t b, uint32_t grid) {
    if (t.accumulate) return;
    for (uint32_t p = threadIdx.x; p < P && p < t.real; p += kPartThreads) {
      if (tot[p] <= kSliceEntries) continue;
      const uint64_t r0 = (uint64_t)p << t.shift;
      const uint64_t r1 = r0 + (1u << t.shift) < t.total_rows ? r0 + (1u << t.shift) : t.total_rows;
      const uint64_t w0 = r0 * kBuckets, len = (r1 - r0) * kBuckets;
      const uint64_t a = w0 + (uint64_t)b * len / grid, e = w0 + (uint64_t)(b + 1u) * len / grid;
      for (uint64_t i = a; i < e; ++i) t.hist[i] = 0u;
    }
  }
};

struct Reduce {
  const uint32_t *part, *ptotal, *pbase, *owner;
  const u64 *over;
  uint32_t *hist;
  uint32_t shift, total_rows, real, accumulate;
};

// Workgroup i < real: partition i, its first slice; beyond: overflow slice
// i - real, while there are that many.  LDS word pad + k stands for
// histogram word w0 + k, where w0 is the partition's first word and pad =
// w0 mod 4, so that 16-byte aligned histogram words are 16-byte aligned in
// LDS.  THREADS: 512 for partitions of one row (four workgroups of 40 KB
// per CU), 1024 for wider ones.
template <uint32_t THREADS>
__global__ __launch_bounds__(THREADS) void hist_reduce_kernel(const Reduce q) {
  constexpr uint32_t kSliceQuads = kSliceEntries / 4u / THREADS;  // 16-byte loads per lane
  static_assert(kSliceQuads * 4u * THREADS == kSliceEntries, "slices are whole 16-byte loads per lane");
  extern __shared__ __align__(16) uint32_t h[];
  uint32_t p = blockIdx.x, slice = 0;
  if (p >= q.real) {
    const uint64_t o = p - q.real;
    if (o >= *q.over) return;
    const uint32_t w = q.owner[o];
    p = w & ((1u << kOwnerPartBits) - 1u);
    slice = w >> kOwnerPartBits;
  }
  const uint32_t n = q.ptotal[p];
  if (n == 0u && q.accumulate) return;  // nothing to add
  const uint32_t first = slice * kSliceEntries;
  const uint32_t cnt = n > first ? (n - first < kSliceEntries ? n - first : kSliceEntries) : 0u;
  const uint64_t r0 = (uint64_t)p << q.shift;
  const uint32_t nr = r0 + (1u << q.shift) < q.total_rows ? (1u << q.shift) : q.total_rows - (uint32_t)r0;
  const uint64_t w0 = r0 * kBuckets;
  const uint32_t pad = (uint32_t)(w0 & 3u), words = nr * kBuckets;
  const uint32_t quads = (pad + words + 3u) / 4u;
  for (uint32_t i = threadIdx.x; i < quads; i += THREADS) ((u32x4 *)h)[i] = u32x4{0u, 0u, 0u, 0u};
  __syncthreads();
  // the slice's keys: up to 3 before the first 16-byte boundary, then 16-byte
  // loads (all of a lane's in flight at once), then up to 3 after the last
  const uint32_t *e = q.part + q.pbase[p] + first;
  const uint32_t head = (uint32_t)((16u - ((uintptr_t)e & 15u)) & 15u) / 4u;
  const uint32_t lead = head < cnt ? head : cnt;
  const uint32_t body = (cnt - lead) / 4u;
  const uint32_t base = pad - (uint32_t)r0 * kBuckets;  // LDS word of row r0 + r, bucket c: base + (r0 + r) * kBuckets + c
  auto add = [&](uint32_t key) {
    atomicAdd(&h[base + (key >> kHistBucketBits) * kBuckets + (key & kBucketMask)], 1u);
  };
  if (threadIdx.x < lead) add(e[threadIdx.x]);
  const u32x4 *e4 = (const u32x4 *)(e + lead);
  u32x4 v[kSliceQuads];
#pragma unroll
  for (uint32_t j = 0; j < kSliceQuads; ++j) {
    const uint32_t i = j * THREADS + threadIdx.x;
    if (i < body) v[j] = e4[i];
  }
#pragma unroll
  for (uint32_t j = 0; j < kSliceQuads; ++j) {
    if (j * THREADS + threadIdx.x < body) {
      add(v[j].x);
      add(v[j].y);
      add(v[j].z);
      add(v[j].w);
    }
  }
  const uint32_t done = lead + 4u * body;
  if (threadIdx.x < cnt - done) add(e[done + threadIdx.x]);
  __syncthreads();
  uint32_t *out = q.hist + (w0 - pad);  // 16-byte aligned: hist is, and w0 - pad is a multiple of 4
  if (n > kSliceEntries) {
    // one of several slices: non-zero counts, device-scope atomics
    for (uint32_t i = pad + threadIdx.x; i < pad + words; i += THREADS) {
      const uint32_t c = h[i];
      if (c) __hip_atomic_fetch_add(out + i, c, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
  } else if (q.accumulate) {
    for (uint32_t i = pad + threadIdx.x; i < pad + words; i += THREADS) {
      const uint32_t c = h[i];
      if (c) out[i] += c;
    }
  } else {
    // the rows whole: 16-byte stores, single words at the ends
    for (uint32_t i = threadIdx.x; i < quads; i += THREADS) {
      const u32x4 c = ((const u32x4 *)h)[i];
      if (4u * i >= pad && 4u * i + 4u <= pad + words) {
        ((u32x4 *)out)[i] = c;
      } else {
        const uint32_t cw[4] = {c.x, c.y, c.z, c.w};
#pragma unroll
        for (uint32_t j = 0; j < 4u; ++j)
          if (4u * i + j >= pad && 4u * i + j < pad + words) out[4u * i + j] = cw[j];
      }
    }
  }
}

uint32_t reduce_lds_bytes(uint32_t shift) { return ((3u + (kBuckets << shift) + 3u) / 4u) * 16u; }

}  // namespace

bool hist_stage_fits(uint64_t n, uint32_t n_windows, uint32_t hist_rows) {
  const uint64_t rows = (uint64_t)n_windows * hist_rows;
  return rows > 0 && rows <= kRowsMax && n < (1ull << 32);
}

uint64_t hist_work_bytes(uint64_t n, uint64_t grid, uint32_t n_windows, uint32_t hist_rows) {
  return layout(n, grid, plan(n, n_windows, hist_rows)).end;
}

HistStage hist_stage(void *work, uint64_t n, uint64_t grid, uint32_t n_windows, uint32_t hist_rows) {
  const Plan pl = plan(n, n_windows, hist_rows);
  const Layout L = layout(n, grid, pl);
  char *w = (char *)work;
  return HistStage{(uint32_t *)(w + L.part.stage), (uint32_t *)(w + L.part.scount), (uint32_t *)(w + L.part.phist),
                   (unsigned long long *)(w + L.over), pl.shift, pl.nparts};
}

hipError_t hist_prepare(int dev) {
  static std::mutex mu;
  static bool done[64] = {};
  std::lock_guard<std::mutex> g(mu);
  if (dev >= 0 && dev < 64 && done[dev]) return hipSuccess;
  hipError_t e = hipFuncSetAttribute((const void *)hist_reduce_kernel<512>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                     (int)reduce_lds_bytes(0));
  if (e == hipSuccess)
    e = hipFuncSetAttribute((const void *)hist_reduce_kernel<1024>, hipFuncAttributeMaxDynamicSharedMemorySize,
                            (int)reduce_lds_bytes(2));
  if (e == hipSuccess && dev >= 0 && dev < 64) done[dev] = true;
  return e;
}

int hist_pipeline_launch(void *work, uint64_t n, uint64_t grid, uint32_t n_windows, uint32_t hist_rows,
                         uint32_t *hist, bool accumulate, bool counted, hipStream_t stream) {
  const Plan pl = plan(n, n_windows, hist_rows);
  const Layout L = layout(n, grid, pl);
  char *w = (char *)work;
  PartArgs<uint32_t> pa{};
  pa.stage = (const uint32_t *)(w + L.part.stage);
  pa.scount = (const uint32_t *)(w + L.part.scount);
  pa.n = n;
  pa.grid = (uint32_t)grid;
  pa.nparts = pl.nparts;
  pa.phist = (uint32_t *)(w + L.part.phist);
  pa.ptotal = (uint32_t *)(w + L.part.ptotal);
  pa.pbase = (uint32_t *)(w + L.part.pbase);
  pa.part = (uint32_t *)(w + L.part.part);
  pa.clear = (u64 *)(w + L.over);  // the overflow-slice counter, when the count kernel runs
  pa.nclear = 1;
  HistPart hp{};
  hp.shift = pl.shift;
  hp.real = pl.real;
  hp.total_rows = pl.total_rows;
  hp.accumulate = accumulate ? 1u : 0u;
  hp.hist = hist;
  hp.over = (u64 *)(w + L.over);
  hp.owner = (uint32_t *)(w + L.owner);
  Reduce q{};
  q.part = pa.part;
  q.ptotal = pa.ptotal;
  q.pbase = pa.pbase;
  q.owner = hp.owner;
  q.over = hp.over;
  q.hist = hist;
  q.shift = pl.shift;
  q.total_rows = pl.total_rows;
  q.real = pl.real;
  q.accumulate = hp.accumulate;
  const uint32_t P = pl.nparts;
  if (!counted)
    hipLaunchKernelGGL((part_count_kernel<uint32_t, HistPart>), dim3((uint32_t)grid), dim3(kPartThreads), P * 4u,
                       stream, pa, hp);
  hipLaunchKernelGGL((part_scan_kernel<uint32_t, HistPart>), dim3(P / 64u), dim3(64 * kPartScanWaves), 0, stream, pa,
                     hp);
  hipLaunchKernelGGL((part_scatter_kernel<uint32_t, HistPart>), dim3((uint32_t)grid), dim3(kPartThreads), P * 4u,
                     stream, pa, hp);
  const dim3 rgrid((uint32_t)(pl.real + pl.over));
  if (pl.shift == 0)
    hipLaunchKernelGGL(hist_reduce_kernel<512>, rgrid, dim3(512), reduce_lds_bytes(0), stream, q);
  else
    hipLaunchKernelGGL(hist_reduce_kernel<1024>, rgrid, dim3(1024), reduce_lds_bytes(pl.shift), stream, q);
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) {
    set_last_error(std::string("histogram kernels: ") + hipGetErrorString(e));
    return GNM_E_HIP;
  }
  return GNM_OK;
}

}  // namespace gnm
