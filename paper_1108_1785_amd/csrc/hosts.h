// Per-host statistics and medians: the interface between the classify
// launcher (kernels.hip) and the per-host kernels (hosts.hip).
//
// The classify kernel appends one entry (host key, bytes, rate, bucket) per bulk flow
// of a registered site to its workgroup's staging range: workgroup b owns
// entries [lo_b, lo_b + count[b]) of the staging arrays, where [lo_b, hi_b)
// is its slice of the records (a record gives at most one entry, so the range
// always has room).  The per-host kernels then partition the entries by a
// hash of the key and reduce each partition in LDS.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "gnm.h"

namespace gnm {

// One staged bulk flow: 32 bytes, written and read as two 16-byte words.
struct __attribute__((aligned(32))) HostEntry {
  unsigned long long key;    // remote address << 32 | row (2 * site + direction)
  unsigned long long bytes;
  unsigned long long rate;   // bits/s
  unsigned long long bucket; // the rate's 10 kbps bucket
};

// Staging arrays written by the classify kernel (device pointers into the
// caller's work buffer).
struct HostStage {
  HostEntry *entry;
  uint32_t *count;  // [grid]: entries staged by each classify workgroup
  uint32_t *phist;  // [grid][2^pbits]: each classify workgroup's entries per partition
  uint32_t pbits;   // partition of an entry: mix64(key) >> (64 - pbits)
};

// log2 of the partition count for a call over n records: the power of two
// nearest n / 2048, between 2^6 and 2^14.
uint32_t host_part_bits(uint64_t n);

// Bytes of the work buffer for n records on `grid` classify workgroups.
uint64_t host_work_bytes(uint64_t n, uint64_t grid);

// Staging arrays inside a work buffer laid out for (n, grid).
HostStage host_stage(void *work, uint64_t n, uint64_t grid);

// Enqueue the per-host kernels after the classify kernel: partition counts
// (left out when the classify kernel counted its entries per partition and
// cleared ht->counters itself: `counted`), their scan, the scatter into
// partition order and the per-partition reduction into ht's arrays.  With
// n == 0 only the counters are cleared.
int host_pipeline_launch(const gnm_host_table *ht, uint64_t n, uint64_t grid, bool counted, hipStream_t stream);

}  // namespace gnm
