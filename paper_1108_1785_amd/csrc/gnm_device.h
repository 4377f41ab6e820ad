// Device helpers shared by the classify kernels (kernels.hip), the histogram
// kernels (hist.hip) and the per-host statistics kernels (hosts.hip).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace gnm {

typedef unsigned long long u64;
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

constexpr uint32_t kBuckets = 10001;  // rate histogram: 10 kbps buckets, the last for >= 100 Mbps
constexpr uint32_t kBucketBps = 10000;

// Histogram bucket of a rate (§III.B.2, TransRate Kernel): floor(rate /
// 10 kbps), every rate of 100 Mbps and above in the last bucket.
__device__ __forceinline__ uint32_t rate_bucket(uint64_t rate) {
  constexpr uint64_t kTop = (uint64_t)kBucketBps * (kBuckets - 1u);  // 100 Mbps
  return rate >= kTop ? kBuckets - 1u : (uint32_t)rate / kBucketBps;
}

// Finalizer of splitmix64: spreads host keys over partitions and LDS slots.
__device__ __forceinline__ uint64_t mix64(uint64_t x) {
  x ^= x >> 30;
  x *= 0xBF58476D1CE4E5B9ull;
  x ^= x >> 27;
  x *= 0x94D049BB133111EBull;
  return x ^ (x >> 31);
}

}  // namespace gnm
