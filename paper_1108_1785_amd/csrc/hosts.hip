// Per-host rate statistics and medians (§III.B.2, TransRate Kernel: maximum,
// minimum, average and median transfer rates for each host in a registered
// site, the median read from the host's 10 kbps bucket array).
//
// Dense bucket arrays per host do not fit (a 10 M-record window has about
// half a million hosts with bulk flows; 10,001 buckets each would be 21 GB),
// and hash-table updates with device-scope atomics are bound by the rate of
// those atomics.  Here the classify kernel only appends one 32-byte entry
// (host key, bytes, rate, bucket) per bulk flow of a registered site to its
// workgroup's staging range, and four kernels finish the job with no
// per-flow device atomics:
//   1. host_count_kernel: per classify workgroup, the number of its entries
//      in each of P partitions (a partition is the top bits of a hash of the
//      key, so all entries of a host land in one partition);
//   2. host_scan_kernel: for each partition, the offset of every workgroup's
//      share within the partition (a column prefix sum) and the totals;
//   3. host_scatter_kernel: every entry to its partition's range;
//   4. host_reduce_kernel: one workgroup per partition gathers its hosts in
//      an LDS hash map with their statistics (LDS atomics), then finds each
//      host's lower median bucket (the ceil(N/2)-th smallest of its N flows'
//      buckets) by a radix selection over the 14-bit bucket: four rounds,
//      each counting the candidates' next 4-bit digit in 16 LDS bins per
//      host and keeping the digit where the running count reaches the rank.
//      A partition with more hosts than the map holds is done in batches: the
//      entries of hosts not yet in the map are compacted in place and
//      reduced by the next batch.
// Each host is written once, at an index taken from counters[0]; the order
// of hosts therefore depends on timing, the set of (key, statistics, median)
// does not.
#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>

#include "gnm_device.h"
#include "hosts.h"
#include "partition.h"
#include "registry.h"

namespace gnm {

namespace {

constexpr uint32_t kHostThreads = 256;
constexpr uint32_t kHostSlots = 256;        // LDS hash-map slots per reduce workgroup (a power of two)
constexpr uint32_t kEntryCap = 2048;        // entries of a partition whose (slot, bucket) stay in LDS
constexpr uint64_t kHostEmpty = ~0ull;      // free map slot (no key has all low 32 bits set)
constexpr uint32_t kDigitBins = 16;         // radix selection: 4 bits per round
constexpr uint32_t kDigitRounds = 4;        // buckets < 2^14: digits at bits 12, 8, 4, 0
constexpr uint32_t kPartBitsMin = 6, kPartBitsMax = 14;
constexpr uint32_t kNoSlot = 0xFFFFFFFFu;

typedef u64 u64x2 __attribute__((ext_vector_type(2)));

// Partition of a host entry: the top pbits of a hash of its key, so all
// entries of a host land in one partition.
struct HostPart {
  uint32_t pbits;
  static constexpr bool kTotalsHook = false;
  static __device__ __forceinline__ uint32_t part(const HostEntry &e, const HostPart &t) {
    return (uint32_t)(mix64(e.key) >> (64u - t.pbits));
  }
};

struct Parts {
  HostEntry *part;
  const uint32_t *ptotal, *pbase;
  u64 *keys, *stats;
  uint32_t *median;
  uint64_t capacity;
  u64 *counters;
};

__device__ __forceinline__ void load_entry(const HostEntry *e, u64 &key, u64 &bytes, u64 &rate, uint32_t &bucket) {
  const u64x2 a = *(const u64x2 *)e, b = *((const u64x2 *)e + 1);
  key = a.x;
  bytes = a.y;
  rate = b.x;
  bucket = (uint32_t)b.y;
}

__device__ __forceinline__ void store_entry(HostEntry *e, u64 key, u64 bytes, u64 rate, uint32_t bucket) {
  *(u64x2 *)e = u64x2{key, bytes};
  *((u64x2 *)e + 1) = u64x2{rate, (u64)bucket};
}

struct HostMap {
  u64 key[kHostSlots];
  u64 bytes[kHostSlots], rsum[kHostSlots], rmin[kHostSlots], rmax[kHostSlots];
  uint32_t flows[kHostSlots];
  uint32_t bins[kDigitBins][kHostSlots];  // digit counts, bin-major so a slot's walk is bank-conflict free
  uint32_t want[kHostSlots];    // rank of the median among the candidates still in play
  uint32_t prefix[kHostSlots];  // digits of the median bucket chosen so far
  uint32_t out[kHostSlots];     // output index of the slot's host within the batch
};

__device__ __forceinline__ uint32_t slot_hash(u64 key) { return (uint32_t)mix64(key) & (kHostSlots - 1u); }

// Slot of key in the map, inserting it when absent; kNoSlot when the map is
// full.  Keys are never removed within a batch, so a slot seen holding
// another key stays that way and linear probing needs no locks.
__device__ __forceinline__ uint32_t map_insert(HostMap &m, u64 key) {
  uint32_t s = slot_hash(key);
  for (uint32_t probe = 0; probe < kHostSlots; ++probe) {
    u64 cur = m.key[s];
    if (cur == kHostEmpty) cur = atomicCAS(&m.key[s], kHostEmpty, key);
    if (cur == kHostEmpty || cur == key) return s;
    s = (s + 1u) & (kHostSlots - 1u);
  }
  return kNoSlot;
}

__device__ __forceinline__ uint32_t map_find(const HostMap &m, u64 key) {
  uint32_t s = slot_hash(key);
  for (uint32_t probe = 0; probe < kHostSlots; ++probe) {
    const u64 cur = m.key[s];
    if (cur == key) return s;
    if (cur == kHostEmpty) return kNoSlot;
    s = (s + 1u) & (kHostSlots - 1u);
  }
  return kNoSlot;
}

// Choose slot s's next digit: the bin where the running count of its
// candidates reaches its rank (the rank becomes the rank within that bin),
// from the 16 bins read at once; the bins are cleared for the next round.
__device__ __forceinline__ void pick_digit(HostMap &m, uint32_t s) {
  uint32_t b[kDigitBins];
#pragma unroll
  for (uint32_t j = 0; j < kDigitBins; ++j) b[j] = m.bins[j][s];
  const uint32_t want = m.want[s];
  uint32_t c = 0, d = 0, before = 0;
#pragma unroll
  for (uint32_t j = 0; j < kDigitBins - 1u; ++j) {
    c += b[j];
    const bool below = c < want;  // the target lies beyond bin j
    d += below;
    before = below ? c : before;
  }
  m.want[s] = want - before;
  m.prefix[s] = (m.prefix[s] << 4) | d;
#pragma unroll
  for (uint32_t j = 0; j < kDigitBins; ++j) m.bins[j][s] = 0u;
}

constexpr uint32_t kPerThread = 4;  // entries a thread loads before working on them

// One workgroup per partition.  A partition of at most kEntryCap entries
// keeps each entry's (slot, bucket) in LDS after the first pass, so the
// three later digit rounds read no device memory; a larger one (a hot host)
// re-reads its entries and looks their keys up again.
__global__ __launch_bounds__(kHostThreads) void host_reduce_kernel(const Parts q) {
  static_assert(kHostSlots == kHostThreads, "one map slot per thread");
  __shared__ HostMap m;
  __shared__ uint32_t e_sb[kEntryCap];  // slot << 14 | bucket, kNoSlot for a host left to the next batch
  __shared__ uint32_t s_overflow, s_deferred, s_wave[kHostThreads / 64];
  __shared__ u64 s_out;
  const uint32_t p = blockIdx.x, tid = threadIdx.x, lane = tid % 64u, wv = tid / 64u;
  HostEntry *ent = q.part + q.pbase[p];
  uint32_t n = q.ptotal[p];
  while (n > 0) {
    const bool in_lds = n <= kEntryCap;
    m.key[tid] = kHostEmpty;
    m.flows[tid] = 0u;
    m.bytes[tid] = m.rsum[tid] = m.rmax[tid] = 0;
    m.rmin[tid] = ~0ull;
    m.prefix[tid] = 0u;
#pragma unroll
    for (uint32_t j = 0; j < kDigitBins; ++j) m.bins[j][tid] = 0u;
    if (tid == 0) {
      s_overflow = 0u;
      s_deferred = 0u;
    }
    __syncthreads();
    // hosts, statistics and the first digit (bits 13..12) of every bucket;
    // each thread loads kPerThread entries before it works on them
    for (uint32_t i0 = 0; i0 < n; i0 += kPerThread * kHostThreads) {
      u64 key[kPerThread], by[kPerThread], rt[kPerThread];
      uint32_t bk[kPerThread];
#pragma unroll
      for (uint32_t j = 0; j < kPerThread; ++j) {
        const uint32_t i = i0 + j * kHostThreads + tid;
        if (i < n) load_entry(ent + i, key[j], by[j], rt[j], bk[j]);
      }
#pragma unroll
      for (uint32_t j = 0; j < kPerThread; ++j) {
        const uint32_t i = i0 + j * kHostThreads + tid;
        if (i >= n) continue;
        const uint32_t s = map_insert(m, key[j]);
        if (in_lds) e_sb[i] = s == kNoSlot ? kNoSlot : (s << 14) | bk[j];
        if (s == kNoSlot) {
          s_overflow = 1u;
          continue;
        }
        atomicAdd(&m.flows[s], 1u);
        atomicAdd(&m.bytes[s], (u64)by[j]);
        atomicAdd(&m.rsum[s], (u64)rt[j]);
        atomicMin(&m.rmin[s], (u64)rt[j]);
        atomicMax(&m.rmax[s], (u64)rt[j]);
        atomicAdd(&m.bins[bk[j] >> 12][s], 1u);
      }
    }
    __syncthreads();
    // reserve the batch's output indexes now, so the atomic's round trip
    // overlaps the digit rounds
    const bool used = m.key[tid] != kHostEmpty;
    const u64 bal = __ballot(used);
    if (lane == 0) s_wave[wv] = (uint32_t)__popcll(bal);
    if (used) m.want[tid] = (m.flows[tid] + 1u) / 2u;
    __syncthreads();
    if (tid == 0) {
      uint32_t t = 0;
      for (uint32_t v = 0; v < kHostThreads / 64u; ++v) {
        const uint32_t c = s_wave[v];
        s_wave[v] = t;
        t += c;
      }
      s_out = t ? __hip_atomic_fetch_add(&q.counters[0], (u64)t, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) : 0ull;
    }
    if (used) {
      pick_digit(m, tid);
      m.out[tid] = (uint32_t)__popcll(bal & ((1ull << lane) - 1ull));  // plus s_wave[wv], known after the barrier
    }
    __syncthreads();
    // the other three digits, among the candidates that share the digits so far
    for (uint32_t r = 1; r < kDigitRounds; ++r) {
      const uint32_t shift = 12u - 4u * r;
      for (uint32_t i = tid; i < n; i += kHostThreads) {
        uint32_t s, bk;
        if (in_lds) {
          const uint32_t sb = e_sb[i];
          s = sb == kNoSlot ? kNoSlot : sb >> 14;
          bk = sb & 0x3FFFu;
        } else {
          u64 key, by, rate;
          load_entry(ent + i, key, by, rate, bk);
          s = map_find(m, key);
        }
        if (s == kNoSlot) continue;
        if ((bk >> (shift + 4u)) == m.prefix[s]) atomicAdd(&m.bins[(bk >> shift) & 15u][s], 1u);
      }
      __syncthreads();
      if (used) pick_digit(m, tid);
      __syncthreads();
    }
    // write the batch's hosts
    if (used) {
      const uint64_t idx = s_out + s_wave[wv] + m.out[tid];
      if (idx < q.capacity) {
        q.keys[idx] = m.key[tid];
        u64 *st = q.stats + idx * 5u;
        st[0] = m.flows[tid];
        st[1] = m.bytes[tid];
        st[2] = m.rsum[tid];
        st[3] = m.rmin[tid];
        st[4] = m.rmax[tid];
        if (q.median) q.median[idx] = m.prefix[tid];
      }
    }
    if (!s_overflow) break;
    // entries of hosts that found no slot, compacted to the front for the
    // next batch: each round reads a block of entries, waits, then writes
    // them at or before the block's end, so no entry is overwritten unread
    for (uint32_t i0 = 0; i0 < n; i0 += kHostThreads) {
      const uint32_t i = i0 + tid;
      u64 key = 0, by = 0, rt = 0;
      uint32_t bk = 0;
      bool keep = false;
      if (i < n) {
        load_entry(ent + i, key, by, rt, bk);
        keep = in_lds ? e_sb[i] == kNoSlot : map_find(m, key) == kNoSlot;
      }
      __syncthreads();
      if (keep) store_entry(ent + atomicAdd(&s_deferred, 1u), key, by, rt, bk);
      __syncthreads();
    }
    n = s_deferred;
    __syncthreads();
  }
}

// n == 0: no classify launch and no entries; the counters still start at 0.
__global__ void host_clear_kernel(u64 *counters) {
  counters[0] = 0;
  counters[1] = 0;
}

PartLayout layout(uint64_t n, uint64_t grid) {
  return part_layout(n, grid, 1ull << host_part_bits(n), sizeof(HostEntry));
}

}  // namespace

uint32_t host_part_bits(uint64_t n) {
  // the power of two nearest n / 2048: a generated window's partitions then
  // hold about 300 entries of about 130 hosts, half the LDS map
  uint32_t b = kPartBitsMin;
  while (b < kPartBitsMax && (1ull << b) * 2896u <= n) ++b;
  return b;
}

uint64_t host_work_bytes(uint64_t n, uint64_t grid) { return layout(n, grid).end; }

HostStage host_stage(void *work, uint64_t n, uint64_t grid) {
  const PartLayout L = layout(n, grid);
  char *w = (char *)work;
  return HostStage{(HostEntry *)(w + L.stage), (uint32_t *)(w + L.scount), (uint32_t *)(w + L.phist),
                   host_part_bits(n)};
}

int host_pipeline_launch(const gnm_host_table *ht, uint64_t n, uint64_t grid, bool counted, hipStream_t stream) {
  if (n == 0) {
    hipLaunchKernelGGL(host_clear_kernel, dim3(1), dim3(1), 0, stream, (u64 *)ht->counters);
  } else {
    const PartLayout L = layout(n, grid);
    char *w = (char *)ht->work;
    PartArgs<HostEntry> pa{};
    pa.stage = (const HostEntry *)(w + L.stage);
    pa.scount = (const uint32_t *)(w + L.scount);
    pa.n = n;
    pa.grid = (uint32_t)grid;
    const HostPart hp{host_part_bits(n)};
    pa.nparts = 1u << hp.pbits;
    pa.phist = (uint32_t *)(w + L.phist);
    pa.ptotal = (uint32_t *)(w + L.ptotal);
    pa.pbase = (uint32_t *)(w + L.pbase);
    pa.part = (HostEntry *)(w + L.part);
    pa.staged = (u64 *)ht->counters + 1;
    pa.clear = (u64 *)ht->counters;
    pa.nclear = 2;
    Parts q{};
    q.part = pa.part;
    q.ptotal = pa.ptotal;
    q.pbase = pa.pbase;
    q.keys = (u64 *)ht->keys;
    q.stats = (u64 *)ht->stats;
    q.median = ht->median;
    q.capacity = ht->capacity;
    q.counters = (u64 *)ht->counters;
    const uint32_t P = pa.nparts;
    if (!counted)
      hipLaunchKernelGGL((part_count_kernel<HostEntry, HostPart>), dim3((uint32_t)grid), dim3(kPartThreads), P * 4u,
                         stream, pa, hp);
    hipLaunchKernelGGL((part_scan_kernel<HostEntry, HostPart>), dim3(P / 64u), dim3(64 * kPartScanWaves), 0, stream,
                       pa, hp);
    hipLaunchKernelGGL((part_scatter_kernel<HostEntry, HostPart>), dim3((uint32_t)grid), dim3(kPartThreads),
                       P * 4u, stream, pa, hp);
    hipLaunchKernelGGL(host_reduce_kernel, dim3(P), dim3(kHostThreads), 0, stream, q);
  }
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) {
    set_last_error(std::string("per-host kernels: ") + hipGetErrorString(e));
    return GNM_E_HIP;
  }
  return GNM_OK;
}

}  // namespace gnm
