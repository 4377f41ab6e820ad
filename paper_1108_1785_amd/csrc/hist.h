// Rate histograms gathered without device-scope atomics: the interface
// between the classify launcher (kernels.hip) and the histogram kernels
// (hist.hip).
//
// With a workspace that holds them, the classify kernel appends one 32-bit
// key per bulk flow of a registered site to its workgroup's staging range
// (workgroup b owns keys [lo_b, lo_b + count[b]), [lo_b, hi_b) being its
// slice of the records, so the range always has room): the flow's histogram
// row over all windows of the call, window * hist_rows + row, above its
// 14-bit rate bucket.  The partition kernels of partition.h then order the
// keys by ranges of rows, and the reduce kernel counts each range in LDS and
// writes its rows of the histograms.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace gnm {

constexpr uint32_t kHistBucketBits = 14;  // staged key: global row << 14 | bucket

struct HistStage {
  uint32_t *key;
  uint32_t *count;           // [grid]: keys staged by each classify workgroup
  uint32_t *phist;           // [grid][nparts]: each classify workgroup's keys per partition
  unsigned long long *over;  // the overflow-slice counter (cleared by the classify kernel when it counts)
  uint32_t shift;            // a partition holds 2^shift rows
  uint32_t nparts;           // partitions (a multiple of 64)
};

// Whether a call over n records in n_windows windows of hist_rows histogram
// rows can stage its keys (at most 65,536 rows over all windows, fewer than
// 2^32 records).
bool hist_stage_fits(uint64_t n, uint32_t n_windows, uint32_t hist_rows);

// Workspace bytes of the staged histograms of such a call on `grid` classify
// workgroups.
uint64_t hist_work_bytes(uint64_t n, uint64_t grid, uint32_t n_windows, uint32_t hist_rows);

// Staging arrays inside a work area laid out for (n, grid, n_windows, hist_rows).
HistStage hist_stage(void *work, uint64_t n, uint64_t grid, uint32_t n_windows, uint32_t hist_rows);

// Kernel attributes of the reduce kernel on device dev (once per device,
// outside any graph capture).
hipError_t hist_prepare(int dev);

// Enqueue the histogram kernels after the classify kernel: partition counts
// (left out when the classify kernel counted its keys per partition itself:
// `counted`), their scan (which also sizes the slices of the most popular
// rows), the scatter into row order, and the reduce into hist (n_windows *
// hist_rows rows of 10,001 counts), which overwrites the rows or, with
// accumulate, adds into them.
int hist_pipeline_launch(void *work, uint64_t n, uint64_t grid, uint32_t n_windows, uint32_t hist_rows,
                         uint32_t *hist, bool accumulate, bool counted, hipStream_t stream);

}  // namespace gnm
