// Spilled accumulator tables: the interface between the classify launcher
// (kernels.hip) and the kernels that merge the spilled rows (table.hip).
//
// When a registry's table does not fit LDS, a classify workgroup keeps its
// hot rows in an LDS cache.  With a workspace, the rows that miss the cache
// and the cached rows flushed at the end of each window segment are not added
// to the device table with device-scope atomics: each becomes one 64-byte
// partial row staged in the workgroup's own range of the workspace (a record
// adds at most one, so the range always has room).  The partial rows are then
// partitioned by (window, range of kTableTileRows rows), and one workgroup
// per partition sums them in LDS and writes its rows of the table, and their
// flag bytes, directly: no initialisation and no device-scope atomics.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "gnm.h"

namespace gnm {

constexpr uint32_t kTableTileRows = 256;  // table rows per partition (even: a site's two rows stay together)

// One staged 32-byte entry: a header (window, row) and three words; the two
// top bits of `row` give the kind.  A record that missed the LDS row cache is
// one entry of kind kRec: word 0 holds its packets (low half) and duration
// (high half), word 1 its bytes, word 2 its rate, and the top bit of `w` marks
// a bulk flow.  A cached row flushed at a window change is three entries:
// kRowA (flows and bulk flows packed as in the LDS table, bytes, packets),
// kRowB (duration, rate sum, rate minimum) and kRowC (rate maximum).
struct __attribute__((aligned(16))) TableEntry {
  uint32_t w, row;
  unsigned long long x, y, z;
};
constexpr uint32_t kRowKindShift = 30;
constexpr uint32_t kRowMask = (1u << kRowKindShift) - 1u;
constexpr uint32_t kRec = 0u, kRowA = 1u, kRowB = 2u, kRowC = 3u;
constexpr uint32_t kRecBulk = 0x80000000u;  // in `w` of a kRec entry
constexpr uint32_t kWindowMask = 0x7FFFFFFFu;

struct TableStage {
  TableEntry *entry;
  uint32_t *count;  // [grid]: partial rows staged by each classify workgroup
};

// Entries each classify workgroup's range holds beyond one per record: the
// three entries per cached row of two flushes (a workgroup whose slice has
// more segments flushes the rest with device atomics).
inline uint64_t table_extra(uint32_t slots) { return 6ull * slots; }

// Bytes of the spill area of a launch over n records on `grid` workgroups
// with n_windows windows of `rows` rows and `slots` LDS cache slots.
uint64_t table_spill_bytes(uint64_t n, uint64_t grid, uint32_t n_windows, uint32_t rows, uint32_t slots);

TableStage table_stage(void *work, uint64_t n, uint64_t grid, uint32_t n_windows, uint32_t rows, uint32_t slots);

// Whether a call of n_windows windows of `rows` rows can spill: at most 16,384
// partitions (the partition kernels keep one LDS counter per partition), so
// fewer than 2^31 windows and rows.
bool table_fits(uint32_t n_windows, uint32_t rows);

// Flag test fused into the merge (threshold in bits/s; need = max(1, min bulk flows)).
struct TableFlags {
  uint8_t *flags;  // NULL: no flags
  uint64_t threshold, need;
  uint32_t n_sites;
};

// Enqueue the merge after the classify kernel: partition counts, their scan,
// the scatter and one workgroup per (window, row range) that adds its sums
// into acc (initialised before the classify kernel, or accumulated into) and
// writes the flags.
int table_merge_launch(void *work, uint64_t n, uint64_t grid, uint32_t n_windows, uint32_t rows, uint32_t slots,
                       unsigned long long *acc, const TableFlags &fl, hipStream_t stream);

}  // namespace gnm
