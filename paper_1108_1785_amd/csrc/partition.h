// Partitioning of staged entries, shared by the per-host statistics
// (hosts.hip) and the spilled accumulator tables (table.hip).
//
// A classify workgroup b stages entries in its own range [lo_b, lo_b +
// count[b]) of an entry array, [lo_b, hi_b) being its slice of the records.
// Three kernels put every entry into its partition's range of a second array:
//   part_count_kernel    per workgroup b, its entries in each of P partitions;
//   part_scan_kernel     per partition, the offset of every workgroup's share
//                        (a column prefix sum of the grid x P count matrix)
//                        and the partition totals;
//   part_scatter_kernel  every entry to its place (partition base, the
//                        workgroup's offset, an LDS cursor).
// The Traits template argument provides `static uint32_t part(const Entry &,
// const Traits &)` and `static constexpr bool kTotalsHook`; with the hook,
// every scan workgroup also calls `Traits::totals(tot, p0, t)` with all its
// threads once the totals tot[0..64) of partitions p0 .. p0 + 63 are in LDS,
// and every scatter workgroup b of `grid` calls `Traits::scatter_share(tot,
// P, t, b, grid)` with all the totals in LDS.
// Entries of 16-byte multiples are copied as 16-byte words, smaller ones
// whole.  The count kernel can be left out when the producer writes the
// count matrix itself.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "gnm_device.h"

namespace gnm {

constexpr uint32_t kPartThreads = 1024;  // count and scatter workgroups (16 waves: one per classify workgroup)
constexpr uint32_t kPartScanWaves = 16;  // scan: waves sharing one group of 64 partitions
constexpr uint32_t kPartUnroll = 4;      // count and scatter: entries per lane in flight

template <class E>
struct PartArgs {
  const E *stage;
  const uint32_t *scount;  // [grid]
  uint64_t n;              // records of the classify launch
  uint64_t extra;          // entries each workgroup's range holds beyond its records
  uint32_t grid, nparts;   // classify workgroups; partitions (a multiple of 64)
  uint32_t *phist;         // [grid][nparts]: counts, then each workgroup's offset within the partition
  uint32_t *ptotal, *pbase;  // [nparts]
  E *part;                 // entries in partition order
  u64 *staged;             // NULL, or a word that receives the number of staged entries
  u64 *clear;              // words set to 0 by the count kernel before anything else reads them
  uint32_t nclear;
};

// First staged entry of classify workgroup b: its first record, plus the
// extra room of the workgroups before it.
__device__ __forceinline__ uint64_t part_stage_lo(uint32_t b, uint64_t n, uint32_t grid, uint64_t extra) {
  return (uint64_t)b * n / grid + (uint64_t)b * extra;
}

// Partition counts of classify workgroup b's entries (dynamic LDS: nparts
// counters).  Workgroup 0 also clears the caller's counter words.
template <class E, class T>
__global__ __launch_bounds__(kPartThreads) void part_count_kernel(const PartArgs<E> q, const T t) {
  extern __shared__ uint32_t h[];
  const uint32_t P = q.nparts, b = blockIdx.x;
  for (uint32_t p = threadIdx.x; p < P; p += kPartThreads) h[p] = 0u;
  if (b == 0 && threadIdx.x < q.nclear) q.clear[threadIdx.x] = 0;
  __syncthreads();
  const uint64_t lo = part_stage_lo(b, q.n, q.grid, q.extra);
  const uint32_t cnt = q.scount[b];
  // kPartUnroll entries per lane loaded before their counts are added
  for (uint32_t i0 = 0; i0 < cnt; i0 += kPartUnroll * kPartThreads) {
    uint32_t pp[kPartUnroll];
#pragma unroll
    for (uint32_t j = 0; j < kPartUnroll; ++j) {
      const uint32_t i = i0 + j * kPartThreads + threadIdx.x;
      pp[j] = i < cnt ? T::part(q.stage[lo + i], t) : ~0u;
    }
#pragma unroll
    for (uint32_t j = 0; j < kPartUnroll; ++j)
      if (pp[j] != ~0u) atomicAdd(&h[pp[j]], 1u);
  }
  __syncthreads();
  uint32_t *row = q.phist + (uint64_t)b * P;
  for (uint32_t p = threadIdx.x; p < P; p += kPartThreads) row[p] = h[p];
}

// Column prefix sums of the count matrix: workgroup x owns partitions
// 64x .. 64x + 63 (lane j: partition 64x + j); its 16 waves each take a
// sixteenth of the classify workgroups, sum their counts (8 loads in flight
// per lane), meet in LDS, and then rewrite the counts as exclusive offsets.
// Also the partition totals, and the number of staged entries.
template <class E, class T>
__global__ __launch_bounds__(64 * kPartScanWaves) void part_scan_kernel(const PartArgs<E> q, const T t) {
  __shared__ uint32_t part[kPartScanWaves][64];
  __shared__ uint32_t tot[64];
  const uint32_t P = q.nparts, lane = threadIdx.x % 64u, w = threadIdx.x / 64u;
  const uint32_t p = blockIdx.x * 64u + lane;
  const uint32_t chunk = (q.grid + kPartScanWaves - 1u) / kPartScanWaves;
  const uint32_t b0 = w * chunk < q.grid ? w * chunk : q.grid;
  const uint32_t b1 = b0 + chunk < q.grid ? b0 + chunk : q.grid;
  uint32_t s = 0;
  for (uint32_t b = b0; b < b1; b += 8u) {
    uint32_t v[8];
#pragma unroll
    for (uint32_t j = 0; j < 8u; ++j) v[j] = b + j < b1 ? q.phist[(uint64_t)(b + j) * P + p] : 0u;
#pragma unroll
    for (uint32_t j = 0; j < 8u; ++j) s += v[j];
  }
  part[w][lane] = s;
  __syncthreads();
  uint32_t run = 0, total = 0;
  for (uint32_t v = 0; v < kPartScanWaves; ++v) {
    run += v < w ? part[v][lane] : 0u;
    total += part[v][lane];
  }
  for (uint32_t b = b0; b < b1; b += 8u) {
    uint32_t v[8];
#pragma unroll
    for (uint32_t j = 0; j < 8u; ++j) v[j] = b + j < b1 ? q.phist[(uint64_t)(b + j) * P + p] : 0u;
#pragma unroll
    for (uint32_t j = 0; j < 8u; ++j) {
      if (b + j < b1) q.phist[(uint64_t)(b + j) * P + p] = run;
      run += v[j];
    }
  }
  if (w == 0) {
    q.ptotal[p] = total;
    tot[lane] = total;
    if (q.staged) {
      u64 c = total;
#pragma unroll
      for (uint32_t o = 32; o > 0; o >>= 1) c += __shfl_xor(c, o, 64);
      if (lane == 0 && c) __hip_atomic_fetch_add(q.staged, c, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
  }
  if constexpr (T::kTotalsHook) {
    __syncthreads();
    T::totals(tot, blockIdx.x * 64u, t);
  }
}

// Exclusive prefix sum of v[0..P) in LDS: every thread scans a run of
// ceil(P / kPartThreads) consecutive values.
__device__ __forceinline__ void part_exclusive_scan(uint32_t *v, uint32_t P, uint32_t *wsum) {
  const uint32_t per = (P + kPartThreads - 1u) / kPartThreads;
  const uint32_t start = threadIdx.x * per;
  uint32_t s = 0;
  for (uint32_t j = 0; j < per && start + j < P; ++j) s += v[start + j];
  const uint32_t lane = threadIdx.x % 64u, w = threadIdx.x / 64u;
  uint32_t x = s;
#pragma unroll
  for (uint32_t o = 1; o < 64; o <<= 1) {
    const uint32_t y = __shfl_up(x, o, 64);
    if (lane >= o) x += y;
  }
  if (lane == 63u) wsum[w] = x;
  __syncthreads();
  uint32_t before = x - s;
  for (uint32_t v2 = 0; v2 < w; ++v2) before += wsum[v2];
  uint32_t run = before;
  for (uint32_t j = 0; j < per && start + j < P; ++j) {
    const uint32_t c = v[start + j];
    v[start + j] = run;
    run += c;
  }
  __syncthreads();
}

// Every entry of classify workgroup b to its place in partition order: the
// partition's base (a scan of the totals, recomputed by every workgroup in
// LDS) plus b's offset within the partition, plus an LDS cursor.  Workgroup 0
// also stores the bases for the reduce kernels.
template <class E, class T>
__global__ __launch_bounds__(kPartThreads) void part_scatter_kernel(const PartArgs<E> q, const T t) {
  extern __shared__ uint32_t cur[];
  __shared__ uint32_t wsum[kPartThreads / 64];
  const uint32_t P = q.nparts, b = blockIdx.x;
  for (uint32_t p = threadIdx.x; p < P; p += kPartThreads) cur[p] = q.ptotal[p];
  __syncthreads();
  if constexpr (T::kTotalsHook) T::scatter_share(cur, P, t, b, q.grid);
  part_exclusive_scan(cur, P, wsum);
  if (b == 0)
    for (uint32_t p = threadIdx.x; p < P; p += kPartThreads) q.pbase[p] = cur[p];
  const uint32_t *off = q.phist + (uint64_t)b * P;
  for (uint32_t p = threadIdx.x; p < P; p += kPartThreads) cur[p] += off[p];
  __syncthreads();
  const uint64_t lo = part_stage_lo(b, q.n, q.grid, q.extra);
  const uint32_t cnt = q.scount[b];
  if constexpr (sizeof(E) % 16 != 0) {
    // small entries: kPartUnroll per lane in flight, copied whole
    for (uint32_t i0 = 0; i0 < cnt; i0 += kPartUnroll * kPartThreads) {
      E v[kPartUnroll];
      uint32_t pos[kPartUnroll];
#pragma unroll
      for (uint32_t j = 0; j < kPartUnroll; ++j) {
        const uint32_t i = i0 + j * kPartThreads + threadIdx.x;
        if (i < cnt) v[j] = q.stage[lo + i];
      }
#pragma unroll
      for (uint32_t j = 0; j < kPartUnroll; ++j) {
        const uint32_t i = i0 + j * kPartThreads + threadIdx.x;
        pos[j] = i < cnt ? atomicAdd(&cur[T::part(v[j], t)], 1u) : 0u;
      }
#pragma unroll
      for (uint32_t j = 0; j < kPartUnroll; ++j)
        if (i0 + j * kPartThreads + threadIdx.x < cnt) q.part[pos[j]] = v[j];
    }
    return;
  }
  // kPartUnroll entries per lane in flight: loaded, then placed, then stored
  typedef u64 u64x2p __attribute__((ext_vector_type(2)));
  constexpr uint32_t W = sizeof(E) / 16 ? sizeof(E) / 16 : 1u;
  for (uint32_t i0 = 0; i0 < cnt; i0 += kPartUnroll * kPartThreads) {
    u64x2p v[kPartUnroll][W];
    uint32_t pos[kPartUnroll];
#pragma unroll
    for (uint32_t j = 0; j < kPartUnroll; ++j) {
      const uint32_t i = i0 + j * kPartThreads + threadIdx.x;
      if (i < cnt) {
#pragma unroll
        for (uint32_t k = 0; k < W; ++k) v[j][k] = ((const u64x2p *)(q.stage + lo + i))[k];
      }
    }
#pragma unroll
    for (uint32_t j = 0; j < kPartUnroll; ++j) {
      const uint32_t i = i0 + j * kPartThreads + threadIdx.x;
      pos[j] = i < cnt ? atomicAdd(&cur[T::part(*(const E *)v[j], t)], 1u) : 0u;
    }
#pragma unroll
    for (uint32_t j = 0; j < kPartUnroll; ++j) {
      const uint32_t i = i0 + j * kPartThreads + threadIdx.x;
      if (i < cnt) {
#pragma unroll
        for (uint32_t k = 0; k < W; ++k) ((u64x2p *)(q.part + pos[j]))[k] = v[j][k];
      }
    }
  }
}

// Work-buffer layout of one staged pipeline: stage entries (room for
// `entries`), per-workgroup counts, the count matrix, totals and bases, the
// partitioned entries; every section 256-byte aligned.
struct PartLayout {
  uint64_t stage, scount, phist, ptotal, pbase, part, end;
};

inline uint64_t part_align256(uint64_t x) { return (x + 255u) & ~255ull; }

inline PartLayout part_layout(uint64_t entries, uint64_t grid, uint64_t nparts, uint64_t entry_bytes,
                              uint64_t base = 0) {
  PartLayout L{};
  const uint64_t n = entries;
  uint64_t o = part_align256(base);
  L.stage = o; o = part_align256(o + entry_bytes * n);
  L.scount = o; o = part_align256(o + 4u * grid);
  L.phist = o; o = part_align256(o + 4u * grid * nparts);
  L.ptotal = o; o = part_align256(o + 4u * nparts);
  L.pbase = o; o = part_align256(o + 4u * nparts);
  L.part = o; o = part_align256(o + entry_bytes * n);
  L.end = o;
  return L;
}

}  // namespace gnm
