// Merge of spilled accumulator rows (§III.B.2, TransRate Kernel: per-site
// statistics; here for registries whose table does not fit LDS).
//
// The classify kernel stages the rows that miss its LDS row cache, and the
// cached rows it flushes at window changes, as 64-byte partial rows (see
// table.h).  The partition kernels of partition.h order them by (window,
// range of 256 table rows); table_reduce_kernel then gives each range one
// workgroup, which owns those rows: it sums the partial rows in an LDS
// table (one LDS atomic per field), adds them into its rows of the device
// table (initialised before the classify kernel unless the call accumulates,
// and holding whatever a workgroup flushed there with device atomics because
// its range had no room) and applies the mean-rate flag test to the sites of
// its rows.  Device-scope atomics, which
// run at about 23 G/s on MI355X, are left out entirely.
#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>

#include "gnm_device.h"
#include "partition.h"
#include "registry.h"
#include "table.h"

namespace gnm {

namespace {

constexpr uint32_t kTableThreads = 1024;

// Partition of a partial row: its window's range of kTableTileRows rows.
struct TablePart {
  uint32_t tiles;  // row ranges per window
  static constexpr bool kTotalsHook = false;
  static __device__ __forceinline__ uint32_t part(const TableEntry &e, const TablePart &t) {
    return (e.w & kWindowMask) * t.tiles + (e.row & kRowMask) / kTableTileRows;
  }
};

uint32_t tiles_per_window(uint32_t rows) { return (rows + kTableTileRows - 1u) / kTableTileRows; }

uint32_t table_parts(uint32_t n_windows, uint32_t rows) {
  const uint64_t p = (uint64_t)n_windows * tiles_per_window(rows);
  return (uint32_t)((p + 63u) & ~63ull);  // the scan kernel takes partitions 64 at a time (at most 16,384)
}

struct Merge {
  const TableEntry *part;
  const uint32_t *ptotal, *pbase;
  u64 *acc;
  uint32_t rows, tiles, n_windows;
  TableFlags fl;
};

// One workgroup per (window, row range).  LDS rows of eight u64 words:
// flows, bulk flows, bytes, packets, duration, rate sum, min, max (the
// device-table order).
__global__ __launch_bounds__(kTableThreads) void table_reduce_kernel(const Merge q) {
  __shared__ u64 t[kTableTileRows][8];
  const uint32_t p = blockIdx.x, w = p / q.tiles, tile = p - w * q.tiles;
  if (w >= q.n_windows) return;  // padding partitions
  const uint32_t r0 = tile * kTableTileRows;
  const uint32_t nr = q.rows - r0 < kTableTileRows ? q.rows - r0 : kTableTileRows;
  for (uint32_t r = threadIdx.x; r < kTableTileRows; r += kTableThreads) {
#pragma unroll
    for (uint32_t f = 0; f < 8u; ++f) t[r][f] = f == 6u ? ~0ull : 0ull;
  }
  __syncthreads();
  const TableEntry *e = q.part + q.pbase[p];
  const uint32_t n = q.ptotal[p];
  // four entries per lane loaded before their LDS atomics
  constexpr uint32_t U = 4;
  for (uint32_t i0 = 0; i0 < n; i0 += U * kTableThreads) {
    TableEntry x[U];
#pragma unroll
    for (uint32_t j = 0; j < U; ++j) {
      const uint32_t i = i0 + j * kTableThreads + threadIdx.x;
      if (i < n) x[j] = e[i];
    }
#pragma unroll
    for (uint32_t j = 0; j < U; ++j) {
      if (i0 + j * kTableThreads + threadIdx.x >= n) continue;
      const TableEntry &y = x[j];
      u64 *o = t[(y.row & kRowMask) - r0];
      switch (y.row >> kRowKindShift) {
        case kRec:  // one record
          atomicAdd(&o[0], 1ull);
          atomicAdd(&o[1], y.y);
          atomicAdd(&o[2], y.x & 0xFFFFFFFFull);
          atomicAdd(&o[3], y.x >> 32);
          if (y.w & kRecBulk) {
            atomicAdd(&o[4], 1ull);
            atomicAdd(&o[5], y.z);
            atomicMin(&o[6], y.z);
            atomicMax(&o[7], y.z);
          }
          break;
        case kRowA:  // flows | bulk flows << 32, bytes, packets
          atomicAdd(&o[0], y.x & 0xFFFFFFFFull);
          if (y.x >> 32) atomicAdd(&o[4], y.x >> 32);
          atomicAdd(&o[1], y.y);
          atomicAdd(&o[2], y.z);
          break;
        case kRowB:  // duration, rate sum, rate minimum
          atomicAdd(&o[3], y.x);
          atomicAdd(&o[5], y.y);
          atomicMin(&o[6], y.z);
          break;
        default:  // kRowC: rate maximum
          atomicMax(&o[7], y.x);
          break;
      }
    }
  }
  __syncthreads();
  // the rows of the device table: word f of row r of window w, one word per
  // lane, consecutive lanes on consecutive words
  u64 *acc = q.acc + ((uint64_t)w * q.rows + r0) * 8u;
  for (uint32_t i = threadIdx.x; i < nr * 8u; i += kTableThreads) {
    const uint32_t r = i / 8u, f = i % 8u;
    const u64 c = acc[i], s2 = t[r][f];
    const u64 v = f == 6u ? (s2 < c ? s2 : c) : (f == 7u ? (s2 > c ? s2 : c) : s2 + c);
    acc[i] = v;
    if (q.fl.flags) t[r][f] = v;  // the final row, for the flag test
  }
  if (!q.fl.flags) return;
  __syncthreads();
  // mean-rate test of the registered sites whose rows lie in this range
  for (uint32_t j = threadIdx.x; 2u * j < nr; j += kTableThreads) {
    const uint32_t site = r0 / 2u + j;
    if (site >= q.fl.n_sites) continue;
    uint8_t fv = 0;
    for (uint32_t d = 0; d < 2u; ++d) {
      const u64 nb = t[2u * j + d][4], sum = t[2u * j + d][5];
      if (nb >= q.fl.need && sum / nb < q.fl.threshold) fv |= (uint8_t)(1u << d);
    }
    q.fl.flags[(uint64_t)w * q.fl.n_sites + site] = fv;
  }
}

PartLayout layout(uint64_t n, uint64_t grid, uint32_t n_windows, uint32_t rows, uint32_t slots) {
  return part_layout(n + grid * table_extra(slots), grid, table_parts(n_windows, rows), sizeof(TableEntry));
}

}  // namespace

bool table_fits(uint32_t n_windows, uint32_t rows) {
  return (uint64_t)n_windows * tiles_per_window(rows) <= 16384u;
}

uint64_t table_spill_bytes(uint64_t n, uint64_t grid, uint32_t n_windows, uint32_t rows, uint32_t slots) {
  return layout(n, grid, n_windows, rows, slots).end;
}

TableStage table_stage(void *work, uint64_t n, uint64_t grid, uint32_t n_windows, uint32_t rows, uint32_t slots) {
  const PartLayout L = layout(n, grid, n_windows, rows, slots);
  char *wb = (char *)work;
  return TableStage{(TableEntry *)(wb + L.stage), (uint32_t *)(wb + L.scount)};
}

int table_merge_launch(void *work, uint64_t n, uint64_t grid, uint32_t n_windows, uint32_t rows, uint32_t slots,
                       unsigned long long *acc, const TableFlags &fl, hipStream_t stream) {
  const PartLayout L = layout(n, grid, n_windows, rows, slots);
  char *wb = (char *)work;
  PartArgs<TableEntry> pa{};
  pa.stage = (const TableEntry *)(wb + L.stage);
  pa.scount = (const uint32_t *)(wb + L.scount);
  pa.n = n;
  pa.extra = table_extra(slots);
  pa.grid = (uint32_t)grid;
  pa.nparts = table_parts(n_windows, rows);
  pa.phist = (uint32_t *)(wb + L.phist);
  pa.ptotal = (uint32_t *)(wb + L.ptotal);
  pa.pbase = (uint32_t *)(wb + L.pbase);
  pa.part = (TableEntry *)(wb + L.part);
  const TablePart tp{tiles_per_window(rows)};
  Merge q{};
  q.part = pa.part;
  q.ptotal = pa.ptotal;
  q.pbase = pa.pbase;
  q.acc = (u64 *)acc;
  q.rows = rows;
  q.tiles = tp.tiles;
  q.n_windows = n_windows;
  q.fl = fl;
  const uint32_t P = pa.nparts;
  hipLaunchKernelGGL((part_count_kernel<TableEntry, TablePart>), dim3((uint32_t)grid), dim3(kPartThreads), P * 4u,
                     stream, pa, tp);
  hipLaunchKernelGGL((part_scan_kernel<TableEntry, TablePart>), dim3(P / 64u), dim3(64 * kPartScanWaves), 0, stream,
                     pa, tp);
  hipLaunchKernelGGL((part_scatter_kernel<TableEntry, TablePart>), dim3((uint32_t)grid), dim3(kPartThreads),
                     P * 4u, stream, pa, tp);
  hipLaunchKernelGGL(table_reduce_kernel, dim3(P), dim3(kTableThreads), 0, stream, q);
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) {
    set_last_error(std::string("table merge kernels: ") + hipGetErrorString(e));
    return GNM_E_HIP;
  }
  return GNM_OK;
}

}  // namespace gnm
