// gfx950 kernels of the flow classify/aggregate path and their C-ABI launchers.
//
// The paper's TransRate Kernel (§III.B.2) gives every GPU thread one flow
// record: the record is assigned to a site by its source or destination
// address, its transfer rate is derived from bytes and the first/last packet
// timestamps, and per-site statistics are accumulated with atomics; shared
// memory is used as much as possible and the record store is read with
// non-caching loads (§III.B.2, GPU Kernel Optimization).  On CDNA4 the same
// method is laid out as:
//   * workgroups of 1024 lanes (16 wave64s) that each own a balanced,
//     contiguous slice of the records, streamed with non-temporal 16-byte
//     loads (4 consecutive records per lane per field), the next tile's loads
//     in flight while the current tile is classified;
//   * an LDS-resident trie root whose 64-bit entries also carry the locality
//     of 16 sub-blocks per cell (one read per endpoint), and the trie's
//     64-byte leaf lines as well when they fit; otherwise wide inner nodes
//     whose 16-byte entries usually hold a whole cell, so one cached read
//     resolves a lookup; the R lookups of a lane advance in lockstep so their
//     memory accesses overlap;
//   * a per-workgroup accumulator table in LDS (rows of seven u64 words,
//     ds_add/ds_min/ds_max_u64); a table too large for LDS lives in device
//     memory behind a 4-way LDS cache of its hot rows;
//   * an exact integer rate: a correctly rounded f64 quotient, within one of
//     the answer for 8000*bytes < 2^53, corrected by one integer
//     multiply-compare; a 64-bit long division covers larger byte counts;
//   * each workgroup's final table written with plain coalesced stores to a
//     caller workspace and combined by a small reduce kernel (device-scope
//     atomics, which serialise across the chip, are used only for tables
//     flushed mid-launch at window changes, or when no workspace is given).
// Several windows go through one persistent launch: workgroups cut the
// concatenated records into equal slices and flush at window boundaries.
// On request the same pass also counts every bulk flow of a registered
// (site, direction) in that row's 10 kbps rate histogram in device memory
// (the paper's bucket arrays behind its median statistic, §III.B.2), and
// two small kernels read each histogram's lower median and apply the
// two-window warning (§III.B.1, §IV.B).
#include <hip/hip_runtime.h>

#include <cstdint>
#include <mutex>
#include <string>

#include "gnm_device.h"
#include "hist.h"
#include "hosts.h"
#include "registry.h"
#include "table.h"

namespace gnm {

typedef uint64_t u64x2 __attribute__((ext_vector_type(2)));
// Pointers into the global address space (not flat).
typedef __attribute__((address_space(1))) const uint32_t gu32;
typedef __attribute__((address_space(1))) const uint64_t gu64;

constexpr uint32_t kThreads = 1024;
constexpr uint32_t kRedRows = 8;     // reduce kernel: table rows (4 sites) per workgroup
constexpr uint32_t kRedWords = kRedRows * kAccFields;  // reduce kernel: 56 table words, one per lane
constexpr uint32_t kRedGroups = 16;  // reduce kernel: at most 16 waves, each summing every G-th slot
constexpr uint32_t kRedUnroll = 8;   // reduce kernel: slot loads in flight per lane
constexpr uint32_t kFeatHist = 1;         // classify_kernel FEAT bits: rate histograms,
constexpr uint32_t kFeatHosts = 2;        //   per-host statistics
constexpr uint32_t kHistKeyBits = 14;     // LDS histogram cache key: row << 14 | bucket
constexpr uint32_t kHistSlotsMax = 4096;  // LDS histogram cache slots (8 bytes each, 4-way sets)
constexpr uint32_t kMedWaves = 4;         // median kernel: waves sharing one (window, site) item
constexpr uint32_t kMedRun = 16;          // buckets per lane per batch: 64 * 16 = 1024 per batch
constexpr uint32_t kMedBatchWords = 64u * kMedRun;
constexpr uint32_t kMedBatches = (kBuckets + kMedBatchWords - 1u) / kMedBatchWords;  // 5
static_assert((1u << kHistKeyBits) > kBuckets, "bucket must fit the key's low bits");
constexpr uint32_t kMedFullBatches = kBuckets / kMedBatchWords;  // batches with no bucket past the row
static_assert(kMedBatches <= 64, "batch sums are held one per lane");

struct LocalRanges {
  uint32_t n;
  uint32_t lo[kMaxLocalRanges];
  uint32_t span[kMaxLocalRanges];  // hi - lo
};

struct ClassifyArgs {
  const uint32_t *src, *dst;
  const uint64_t *bytes;
  const uint32_t *packets, *first, *last;
  uint64_t n;
  uint64_t flush_records;  // records aggregated in LDS between two table flushes (<= kMaxRecordsPerFlush)
  gu64 *woff;  // NULL: one window [0, n)
  uint32_t n_windows;
  uint32_t rows;
  uint64_t bulk_bytes;
  u64 *acc;  // n_windows * rows * 8 words
  gu64 *root;  // trie entry | locality masks << 32
  gu32 *wide, *lines;
  uint32_t root_bits, node_bits;
  uint32_t n_line_words;
  uint32_t lds_off_acc, lds_off_lines;
  uint32_t cache_slots;  // LDS cache slots for a table that does not fit in LDS
  u64 *ws;             // NULL: every table is flushed with atomics
  uint32_t *ws_meta;   // per workgroup: window of the table it left in ws
  uint32_t *hist;      // rate histograms: n_windows * hist_rows * kBuckets counts (FEAT & kFeatHist)
  uint32_t hist_rows;  // 2 * n_sites: rows of registered sites
  uint32_t lds_off_hist, hist_slots;  // LDS histogram cache (0 slots: every count goes to device memory)
  HostEntry *hs_entry;                // per-host staging (FEAT & kFeatHosts): workgroup b's entries
  uint32_t *hs_count;                 //   at [lo_b, lo_b + hs_count[b]) of its record slice [lo_b, hi_b)
  TableEntry *ts_entry;               // spilled rows (a table beyond LDS, with a workspace; NULL: device
  uint32_t *ts_count;                 //   atomics): workgroup b's entries at [s_b, s_b + ts_count[b]),
  uint32_t ts_extra;                  //   s_b = lo_b + b * ts_extra, room for hi_b - lo_b + ts_extra
  uint32_t *ks_key;                   // staged histogram keys (FEAT & kFeatHist, with a workspace; NULL: the
  uint32_t *ks_count;                 //   LDS cache and device atomics): workgroup b's at [lo_b, lo_b + ks_count[b])
  uint32_t *kp_hist;                  // staged keys counted per partition here: [grid][kp_parts] (NULL: not here)
  unsigned long long *kp_over;        //   a word workgroup 0 clears (the histogram kernels' overflow slices)
  uint32_t kp_shift, kp_parts;        //   partition of a key: key >> (14 + kp_shift), kp_parts of them
  uint32_t lds_off_kp;                //   LDS counters
  uint32_t *hp_hist;                  // per-host entries counted per partition here: [grid][2^hp_bits] (NULL: not
  uint32_t hp_bits, lds_off_hp;       //   here); partition mix64(key) >> (64 - hp_bits); LDS counters
  unsigned long long *hp_clear;       //   the host table's two counters, cleared by workgroup 0
  uint32_t lds_off_ctr;               // LDS words: the workgroup's staging cursors (hosts, spilled rows, keys)
  uint32_t filters;                   // any exclusion filter set
  uint32_t min_avg_packet_bytes, min_packets, min_duration_ms;
  LocalRanges local;
};

// ---------------------------------------------------------------- device helpers

__device__ __forceinline__ bool in_ranges(const LocalRanges &L, uint32_t ip) {
  bool r = false;
  for (uint32_t j = 0; j < L.n; ++j) r |= (ip - L.lo[j]) <= L.span[j];
  return r;
}


// Longest-prefix match of R addresses at once, from the root trie entries of
// their cells: site codes of the intervals containing ip[k] for lanes with
// act[k].  The R walks advance in lockstep
// so that their memory accesses are in flight together.  A wide-node entry
// costs one 16-byte read and usually resolves the address; a leaf line costs
// one 64-byte line read (keys) and one read of the same line (site).  Lanes
// with nothing to resolve read the dummy entry 0 rather than branching.
template <int R, bool LINES_LDS>
__device__ __forceinline__ void lookup_sites(const uint32_t (&ip)[R], const uint32_t (&root_e)[R],
                                             const bool (&act)[R], uint32_t (&site)[R], gu32 *wide,
                                             const uint32_t *s_lines, gu32 *g_lines, uint32_t root_bits,
                                             uint32_t node_bits) {
  uint32_t node[R], line[R];
  bool any = false, any_line = false;
  // every lane still walking at depth d has the same number of unresolved
  // address bits, so the shift is wave-uniform
  uint32_t shift = 32u - root_bits;
#pragma unroll
  for (int k = 0; k < R; ++k) {
    const uint32_t e = root_e[k];
    const uint32_t kind = act[k] ? e >> kKindShift : kKindLeaf, pay = e & kPayloadMask;
    site[k] = pay;
    node[k] = kind == kKindNode ? pay : 0u;
    line[k] = kind == kKindLine ? pay : 0u;
    any |= node[k] != 0u;
    any_line |= line[k] != 0u;
  }
  // wide nodes: first level node_bits (>= 4) wide, then 8 bits, so at most
  // 1 + ceil(20 / 8) = 4 levels below a root of >= 8 bits
  for (int depth = 0; depth < 4 && __builtin_amdgcn_ballot_w64(any); ++depth) {
    const uint32_t smax = depth == 0 ? node_bits : kNodeStrideMax;
    const uint32_t ns = shift > smax ? shift - smax : 0u;
    const uint32_t mask = (1u << (shift - ns)) - 1u;
    u32x4 q[R];
#pragma unroll
    for (int k = 0; k < R; ++k) {
      const uint32_t idx = node[k] ? (ip[k] >> ns) & mask : 0u;
      q[k] = *(__attribute__((address_space(1))) const u32x4 *)(wide + 4ull * (node[k] + idx));
    }
    shift = ns;
    any = false;
    // QUAD entries (leaves too, when site codes fit 16 bits) resolve here:
    // the position is 3 minus the number of split offsets above the
    // address's offset, each found from the sign of a difference (offsets
    // are < 2^24); the site is that 16-bit field of z:w.
    const uint32_t low = (1u << ns) - 1u;
    bool odd = false;
#pragma unroll
    for (int k = 0; k < R; ++k) {
      const bool walk = node[k] != 0u;
      const uint32_t off = ip[k] & low;
      const uint32_t gt = ((off - (q[k].x & 0xFFFFu)) >> 31) + ((off - (q[k].x >> 16)) >> 31) +
                          ((off - (q[k].y & 0xFFFFu)) >> 31);
      const uint64_t packed = ((uint64_t)q[k].w << 32) | q[k].z;
      const uint32_t qs = (uint32_t)(packed >> (48u - 16u * gt)) & 0xFFFFu;
      const bool quad = (q[k].y >> kKindShift) == kKindQuad;
      site[k] = walk && quad ? qs : site[k];
      odd |= walk && !quad;
    }
    // the rest: leaves with wide site codes, leaf lines, deeper nodes
    if (__builtin_amdgcn_ballot_w64(odd)) {
#pragma unroll
      for (int k = 0; k < R; ++k) {
        const bool walk = node[k] != 0u;
        const uint32_t kind = q[k].y >> kKindShift;
        site[k] = walk && kind == kKindLeaf ? q[k].z : site[k];
        line[k] = walk && kind == kKindLine ? q[k].z : line[k];
        node[k] = walk && kind == kKindNode ? q[k].z : 0u;
        any |= node[k] != 0u;
        any_line |= line[k] != 0u;
      }
    } else {
#pragma unroll
      for (int k = 0; k < R; ++k) node[k] = 0u;
    }
  }
  // leaf lines: position = number of starts 1..7 that are <= ip
  if (LINES_LDS) {
    // LDS: the keys, then the one site code at the position
    if (!__builtin_amdgcn_ballot_w64(any_line)) return;
    u32x4 k0[R], k1[R];
#pragma unroll
    for (int k = 0; k < R; ++k) {
      const uint32_t w = line[k] * kLineWords;
      k0[k] = *(const u32x4 *)(s_lines + w);
      k1[k] = *(const u32x4 *)(s_lines + w + 4);
    }
#pragma unroll
    for (int k = 0; k < R; ++k) {
      const uint32_t x = ip[k];
      const uint32_t pos = (k0[k].y <= x) + (k0[k].z <= x) + (k0[k].w <= x) + (k1[k].x <= x) +
                           (k1[k].y <= x) + (k1[k].z <= x) + (k1[k].w <= x);
      const uint32_t ls = s_lines[line[k] * kLineWords + kLineKeys + pos];
      if (line[k]) site[k] = ls;
    }
  } else if (R == 4) {
    // device memory, four walks per lane: the keys, then the one site code
    // (the whole line for four walks at once would not fit the registers)
    if (!__builtin_amdgcn_ballot_w64(any_line)) return;
    u32x4 k0[R], k1[R];
#pragma unroll
    for (int k = 0; k < R; ++k) {
      typedef __attribute__((address_space(1))) const u32x4 gq;
      const gq *l = (const gq *)(g_lines + line[k] * kLineWords);
      k0[k] = l[0];
      k1[k] = l[1];
    }
#pragma unroll
    for (int k = 0; k < R; ++k) {
      const uint32_t x = ip[k];
      const uint32_t pos = (k0[k].y <= x) + (k0[k].z <= x) + (k0[k].w <= x) + (k1[k].x <= x) +
                           (k1[k].y <= x) + (k1[k].z <= x) + (k1[k].w <= x);
      const uint32_t ls = g_lines[line[k] * kLineWords + kLineKeys + pos];
      if (line[k]) site[k] = ls;
    }
  } else if (__builtin_amdgcn_ballot_w64(any_line)) {
    // device memory: the whole 64-byte line in one round trip, the site
    // code selected in registers
    u32x4 k0[R], k1[R], s0[R], s1[R];
#pragma unroll
    for (int k = 0; k < R; ++k) {
      typedef __attribute__((address_space(1))) const u32x4 gq;
      const gq *l = (const gq *)(g_lines + line[k] * kLineWords);
      k0[k] = l[0];
      k1[k] = l[1];
      s0[k] = l[2];
      s1[k] = l[3];
    }
#pragma unroll
    for (int k = 0; k < R; ++k) {
      const uint32_t x = ip[k];
      const uint32_t hi = k1[k].x <= x;  // position >= 4
      const u32x4 kk = hi ? k1[k] : k0[k];
      const u32x4 ss = hi ? s1[k] : s0[k];
      // position within the half: starts 1..3 of that half that are <= ip
      // (start 0 of the low half is the cell start, <= ip by construction)
      const uint32_t p = (kk.y <= x) + (kk.z <= x) + (kk.w <= x);
      const uint32_t ls = p == 0 ? ss.x : (p == 1 ? ss.y : (p == 2 ? ss.z : ss.w));
      if (line[k]) site[k] = ls;
    }
  }
}

// floor(b * 8000 / d) for b with 8000*b < 2^53, d >= 1.
constexpr uint64_t kFastBytesMax = ((1ull << 53) - 1ull) / 8000ull;

__device__ __noinline__ uint64_t rate_bps_wide(uint64_t b, uint32_t d) {
  // floor(8000 b / d) = 8000 floor(b/d) + floor(8000 (b mod d) / d), saturated.
  const uint64_t q1 = b / d, r1 = b % d;
  if (q1 > ~0ull / 8000ull) return ~0ull;
  const uint64_t hi = q1 * 8000ull;
  const uint64_t lo = (r1 * 8000ull) / d;  // r1 * 8000 < 2^45
  const uint64_t s = hi + lo;
  return s < hi ? ~0ull : s;
}

__device__ __forceinline__ uint64_t rate_bps(uint64_t b, uint32_t d) {
  if (b <= kFastBytesMax) {
    const uint64_t num = b * 8000ull;  // < 2^53: exact as a double
    // The correctly rounded quotient is within one of floor(num/d) and never
    // below it; one integer check removes the rounding step up.
    uint64_t q = (uint64_t)((double)num / (double)d);
    const uint64_t prod = q * (uint64_t)d;
    if (prod > num) q -= 1;
    else if (num - prod >= d) q += 1;
    return q;
  }
  return rate_bps_wide(b, d);
}

__device__ __forceinline__ uint32_t ldg_nt(const uint32_t *p) { return __builtin_nontemporal_load(p); }
__device__ __forceinline__ uint64_t ldg_nt(const uint64_t *p) { return __builtin_nontemporal_load(p); }
__device__ __forceinline__ u32x4 ldg_nt4(const uint32_t *p) { return __builtin_nontemporal_load((const u32x4 *)p); }
__device__ __forceinline__ u64x2 ldg_nt2(const uint64_t *p) { return __builtin_nontemporal_load((const u64x2 *)p); }

// Window containing record i: largest w with offsets[w] <= i (offsets clamped
// to [0, n]); also returns the end of that window, at least i + 1.
__device__ __forceinline__ uint32_t window_of(const ClassifyArgs &a, uint64_t i, uint64_t &wend) {
  if (!a.woff) { wend = a.n; return 0; }
  uint32_t lo = 0, len = a.n_windows;
  while (len > 1) {
    const uint32_t half = len >> 1;
    uint64_t o = a.woff[lo + half];
    o = o < a.n ? o : a.n;
    if (o <= i) lo += half;
    len -= half;
  }
  uint64_t e = (lo + 1 < a.n_windows) ? a.woff[lo + 1] : a.n;
  e = e < a.n ? e : a.n;
  wend = e > i ? e : i + 1;
  return lo;
}

// ---------------------------------------------------------------- accumulation

struct Lds {
  const uint64_t *root;
  const uint32_t *lines;
  u64 *acc;        // the accumulator table, or the cache slots' rows
  uint32_t *tags;  // cache slots: row + 1 of the owner, 0 = free
  uint32_t slots;  // cache slots (0 when the table is in LDS)
  uint32_t *htags;  // histogram cache: key + 1 of the owner, 0 = free
  uint32_t *hcnt;   // histogram cache: counts
  uint32_t hslots;  // histogram cache slots (0 = none)
  uint32_t *hcur;   // per-host staging: entries this workgroup has staged
  HostEntry *se;    // per-host staging: this workgroup's range
  uint32_t *tcur;   // spilled rows: partial rows this workgroup has staged
  TableEntry *te;   // spilled rows: this workgroup's range (NULL: misses and flushes use device atomics)
  uint32_t *kcur;   // staged histogram keys: keys this workgroup has staged (without per-host staging)
  uint32_t *ke;     // staged histogram keys: this workgroup's range (NULL: the histogram cache)
  uint32_t *kp;     // staged histogram keys per partition (NULL: counted by the histogram kernels)
  uint32_t kshift;  // partition of a key: key >> (14 + kshift)
  uint32_t *hp;     // per-host entries per partition (NULL: counted by the count kernel)
  uint32_t hpbits;  // partition of a host entry: mix64(key) >> (64 - hpbits)
  uint32_t win;     // window of the current segment
  uint32_t kbase;   // histogram row of the current segment's window: win * hist_rows
};

// Staging code of a record whose row lives in an LDS cache slot.
constexpr uint32_t kInSlot = 0x80000000u;

// LDS cache set of a row (any set count): multiplicative hash, then the
// high half of hash * sets.
__device__ __forceinline__ uint32_t cache_set(uint32_t row, uint32_t sets) {
  return __umulhi(row * 0x9E3779B1u, sets);
}

// Fields every record updates (the bulk count rides in the packed `cnt`).
// With the whole table in LDS the row is the LDS row.  Otherwise (a table
// too large for LDS) the row goes to an LDS cache: 4-way sets, each way owned
// by the first row that claims it in this workgroup's current window segment
// (ways are claimed in order and never released before the segment ends, so
// a row holds at most one way); records of rows whose set is full update the
// device table with device-scope atomics.  Returns the code the bulk pass
// needs: the LDS row, kInSlot | slot, or the device-table row.
template <bool ACC_LDS>
__device__ __forceinline__ uint32_t accumulate(const Lds &L, u64 *g_row, uint32_t row, uint64_t b, uint32_t pk,
                                               uint32_t dur, bool bulk) {
  if (ACC_LDS) {
    u64 *t = L.acc + row * kAccFields;  // one address, immediate field offsets
    atomicAdd(&t[kCnt], 1ull | ((u64)bulk << 32));
    atomicAdd(&t[kBytes], (u64)b);
    atomicAdd(&t[kPackets], (u64)pk);
    atomicAdd(&t[kDur], (u64)dur);
    return row;
  }
  bool hit = false;
  uint32_t slot = 0;
  if (L.slots) {
    const uint32_t set = cache_set(row, L.slots >> 2);
    uint32_t *tg = L.tags + 4u * set;
    const uint32_t tag = row + 1u;
    const u32x4 t4 = *(const u32x4 *)tg;
    uint32_t w[4] = {t4.x, t4.y, t4.z, t4.w};
    uint32_t way = 4;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      if (way == 4u && w[j] == 0u) w[j] = atomicCAS(&tg[j], 0u, tag) ?: tag;  // claimed, or its owner
      if (way == 4u && w[j] == tag) way = j;
    }
    hit = way < 4u;
    slot = 4u * set + way;
  }
  if (hit) {
    u64 *t = L.acc + slot * kAccFields;
    atomicAdd(&t[kCnt], 1ull | ((u64)bulk << 32));
    atomicAdd(&t[kBytes], (u64)b);
    atomicAdd(&t[kPackets], (u64)pk);
    atomicAdd(&t[kDur], (u64)dur);
    return kInSlot | slot;
  }
  if (L.te) return row;  // spilled: the caller stages the record as a partial row
  u64 *g = g_row + (uint64_t)row * 8u;
  atomicAdd(&g[0], 1ull);
  atomicAdd(&g[1], (u64)b);
  atomicAdd(&g[2], (u64)pk);
  atomicAdd(&g[3], (u64)dur);
  return row;
}

// Rate fields of a bulk record, at the place accumulate() returned.
template <bool ACC_LDS>
__device__ __forceinline__ void add_rate(const Lds &L, u64 *g_row, uint32_t code, uint64_t rate) {
  if (ACC_LDS || (code & kInSlot)) {
    u64 *t = L.acc + (code & ~kInSlot) * kAccFields;
    atomicAdd(&t[kRateSum], (u64)rate);
    atomicMin(&t[kRateMin], (u64)rate);
    atomicMax(&t[kRateMax], (u64)rate);
  } else {
    u64 *g = g_row + (uint64_t)code * 8u;
    atomicAdd(&g[4], 1ull);
    atomicAdd(&g[5], (u64)rate);
    atomicMin(&g[6], (u64)rate);
    atomicMax(&g[7], (u64)rate);
  }
}

// Flush the workgroup's LDS table into window table g (rows x 8 words) with
// device-scope atomics and reset it.  Only touched rows, and only non-empty
// bulk fields, are sent.
__device__ __forceinline__ void flush_atomic(u64 *s_acc, u64 *__restrict__ g, uint32_t rows) {
  __syncthreads();
  for (uint32_t r = threadIdx.x; r < rows; r += kThreads) {
    u64 *t = s_acc + r * kAccFields;
    const u64 cnt = t[kCnt];
    if (cnt == 0) continue;
    u64 *o = g + (uint64_t)r * 8u;
    atomicAdd(&o[0], cnt & 0xFFFFFFFFull);
    atomicAdd(&o[1], t[kBytes]);
    atomicAdd(&o[2], t[kPackets]);
    atomicAdd(&o[3], t[kDur]);
    const u64 nb = cnt >> 32;
    if (nb) {
      atomicAdd(&o[4], nb);
      atomicAdd(&o[5], t[kRateSum]);
      atomicMin(&o[6], t[kRateMin]);
      atomicMax(&o[7], t[kRateMax]);
    }
    t[kCnt] = t[kBytes] = t[kPackets] = t[kDur] = t[kRateSum] = t[kRateMax] = 0;
    t[kRateMin] = ~0ull;
  }
  __syncthreads();
}

// Count one bulk flow in bucket `bucket` of row `row` of window histogram h.
// Counts are gathered per workgroup in an LDS cache of (row, bucket) keys
// with the accumulator cache's discipline (4-way sets, ways claimed in order
// and kept until the segment ends); a key whose set is full, or a row beyond
// the key's range, goes to device memory directly.  Device-scope atomics on
// a few popular buckets serialise in the memory system, so gathering them
// first matters more than their number.
__device__ __forceinline__ void hist_add(const Lds &L, uint32_t *h, uint32_t row, uint32_t bucket) {
  if (L.hslots && row < (1u << (32 - kHistKeyBits)) - 1u) {
    const uint32_t tag = ((row << kHistKeyBits) | bucket) + 1u;
    const uint32_t set = cache_set(tag, L.hslots >> 2);
    uint32_t *tg = L.htags + 4u * set;
    const u32x4 t4 = *(const u32x4 *)tg;
    uint32_t w[4] = {t4.x, t4.y, t4.z, t4.w};
    uint32_t way = 4;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      if (way == 4u && w[j] == 0u) w[j] = atomicCAS(&tg[j], 0u, tag) ?: tag;  // claimed, or its owner
      if (way == 4u && w[j] == tag) way = j;
    }
    if (way < 4u) {
      atomicAdd(&L.hcnt[4u * set + way], 1u);
      return;
    }
  }
  __hip_atomic_fetch_add(h + (uint64_t)row * kBuckets + bucket, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Add the histogram cache into window histogram h and free its slots.
__device__ __forceinline__ void flush_hist(const Lds &L, uint32_t *h) {
  __syncthreads();
  for (uint32_t sl = threadIdx.x; sl < L.hslots; sl += kThreads) {
    const uint32_t tag = L.htags[sl];
    if (tag == 0u) continue;
    const uint32_t key = tag - 1u;
    __hip_atomic_fetch_add(h + (uint64_t)(key >> kHistKeyBits) * kBuckets + (key & ((1u << kHistKeyBits) - 1u)),
                           L.hcnt[sl], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    L.htags[sl] = 0u;
    L.hcnt[sl] = 0u;
  }
  __syncthreads();
}

// One staged 32-byte entry of window L.win (two 16-byte stores).
__device__ __forceinline__ void stage_entry(const Lds &L, uint32_t pos, uint32_t w, uint32_t row_kind, u64 x, u64 y,
                                            u64 z) {
  typedef u64 u64x2_ __attribute__((ext_vector_type(2)));
  u64x2_ *e = (u64x2_ *)(L.te + pos);
  e[0] = u64x2_{(u64)w | ((u64)row_kind << 32), x};
  e[1] = u64x2_{y, z};
}

// Entries reserved for the wave's lanes with `want`: the first entry of the
// wave's run (one LDS atomic by the first active lane); bal = the lanes.
__device__ __forceinline__ uint32_t reserve_rows(uint32_t *cursor, bool want, uint64_t &bal, uint32_t per = 1u) {
  bal = __builtin_amdgcn_ballot_w64(want);
  if (!bal) return 0u;
  uint32_t base = 0;
  if (__lane_id() == (uint32_t)__builtin_ctzll(__builtin_amdgcn_read_exec()))
    base = atomicAdd(cursor, per * (uint32_t)__builtin_popcountll(bal));
  return __builtin_amdgcn_readfirstlane(base);
}

// Flush the LDS cache slots into window table g with device-scope atomics,
// or, when the table spills and the workgroup's range has room for three
// entries per claimed slot below `room`, stage them; then free them.
__device__ __forceinline__ void flush_cache(const Lds &L, u64 *__restrict__ g, uint32_t room) {
  __syncthreads();
  bool stage = false;
  if (L.te) {
    // claimed slots, counted by every wave into the spare LDS counter word
    uint32_t *claimed = L.tcur + 1;
    if (threadIdx.x == 0) *claimed = 0u;
    __syncthreads();
    uint32_t c = 0;
    for (uint32_t sl = threadIdx.x; sl < L.slots; sl += kThreads) c += L.tags[sl] != 0u;
    for (uint32_t o = 32; o > 0; o >>= 1) c += __shfl_xor(c, o, 64);
    if (__lane_id() == 0 && c) atomicAdd(claimed, c);
    __syncthreads();
    stage = *L.tcur + 3u * *claimed <= room;
  }
  if (stage) {
    const uint64_t below = (1ull << __lane_id()) - 1ull;
    for (uint32_t s0 = 0; s0 < L.slots; s0 += kThreads) {  // whole waves, so the reservation is uniform
      const uint32_t sl = s0 + threadIdx.x;
      const uint32_t tag = sl < L.slots ? L.tags[sl] : 0u;
      uint64_t bal;
      const uint32_t base = reserve_rows(L.tcur, tag != 0u, bal, 3u);
      if (tag == 0u) continue;
      u64 *t = L.acc + sl * kAccFields;
      const uint32_t pos = base + 3u * (uint32_t)__builtin_popcountll(bal & below), row = tag - 1u;
      stage_entry(L, pos, L.win, row | (kRowA << kRowKindShift), t[kCnt], t[kBytes], t[kPackets]);
      stage_entry(L, pos + 1u, L.win, row | (kRowB << kRowKindShift), t[kDur], t[kRateSum], t[kRateMin]);
      stage_entry(L, pos + 2u, L.win, row | (kRowC << kRowKindShift), t[kRateMax], 0ull, 0ull);
      t[kCnt] = t[kBytes] = t[kPackets] = t[kDur] = t[kRateSum] = t[kRateMax] = 0;
      t[kRateMin] = ~0ull;
      L.tags[sl] = 0u;
    }
    __syncthreads();
    return;
  }
  for (uint32_t sl = threadIdx.x; sl < L.slots; sl += kThreads) {
    const uint32_t tag = L.tags[sl];
    if (tag == 0u) continue;
    u64 *t = L.acc + sl * kAccFields;
    u64 *o = g + (uint64_t)(tag - 1u) * 8u;
    const u64 cnt = t[kCnt];
    atomicAdd(&o[0], cnt & 0xFFFFFFFFull);
    atomicAdd(&o[1], t[kBytes]);
    atomicAdd(&o[2], t[kPackets]);
    atomicAdd(&o[3], t[kDur]);
    const u64 nb = cnt >> 32;
    if (nb) {
      atomicAdd(&o[4], nb);
      atomicAdd(&o[5], t[kRateSum]);
      atomicMin(&o[6], t[kRateMin]);
      atomicMax(&o[7], t[kRateMax]);
    }
    t[kCnt] = t[kBytes] = t[kPackets] = t[kDur] = t[kRateSum] = t[kRateMax] = 0;
    t[kRateMin] = ~0ull;
    L.tags[sl] = 0u;
  }
  __syncthreads();
}

// Copy the workgroup's LDS table (same row layout) to its workspace slot and
// record which window it belongs to.  The kernel ends right after.
__device__ __forceinline__ void flush_partial(const ClassifyArgs &a, const u64 *s_acc, uint32_t w) {
  __syncthreads();
  const uint32_t words = kAccFields * a.rows;
  u64 *dst = a.ws + (uint64_t)blockIdx.x * words;
  for (uint32_t i = threadIdx.x; i < words; i += kThreads) dst[i] = s_acc[i];
  if (threadIdx.x == 0) a.ws_meta[blockIdx.x] = w;
}

// ---------------------------------------------------------------- record tiles

// R records per lane, in two parts loaded at different times: the endpoint
// addresses (needed first, for locality and the trie walk) and the rest.
// Strided tiles: lane t of a tile at `base` holds records base + k*kThreads + t.
// Vector tiles (R = 4): lane t holds base + 4t + k, one 16-byte load per field.
template <int R>
struct Addr {
  uint32_t s[R], d[R];
  bool v[R];
};
template <int R>
struct Rest {
  uint32_t pk[R], f[R], l[R];
  uint64_t b[R];
};

template <int R, bool VEC>
__device__ __forceinline__ void load_addr(Addr<R> &t, const ClassifyArgs &a, uint64_t base, uint64_t end) {
  // Lanes past the end load the range's last records (always valid, since
  // ranges are non-empty) and are marked invalid: unconditional loads keep
  // the code straight-line.
  if (VEC) {
    const uint64_t idx = base + 4ull * threadIdx.x;
    const bool ok = idx < end;  // end is base + a multiple of 4, and end - 4 >= the range start
    const uint64_t at = ok ? idx : end - 4;
    const u32x4 s = ldg_nt4(a.src + at), d = ldg_nt4(a.dst + at);
    t.s[0] = s.x; t.s[1] = s.y; t.s[2] = s.z; t.s[3] = s.w;
    t.d[0] = d.x; t.d[1] = d.y; t.d[2] = d.z; t.d[3] = d.w;
#pragma unroll
    for (int k = 0; k < R; ++k) t.v[k] = ok;
  } else {
#pragma unroll
    for (int k = 0; k < R; ++k) {
      const uint64_t idx = base + (uint64_t)k * kThreads + threadIdx.x;
      t.v[k] = idx < end;
      const uint64_t at = t.v[k] ? idx : end - 1;
      t.s[k] = ldg_nt(a.src + at);
      t.d[k] = ldg_nt(a.dst + at);
    }
  }
}

template <int R, bool VEC>
__device__ __forceinline__ void load_rest(Rest<R> &t, const ClassifyArgs &a, uint64_t base, uint64_t end) {
  // (lanes past the end load the range's last records, as in load_addr)
  if (VEC) {
    const uint64_t idx = base + 4ull * threadIdx.x;
    const uint64_t at = idx < end ? idx : end - 4;
    const u32x4 pk = ldg_nt4(a.packets + at), f = ldg_nt4(a.first + at), l = ldg_nt4(a.last + at);
    const u64x2 b0 = ldg_nt2(a.bytes + at), b1 = ldg_nt2(a.bytes + at + 2);
    t.pk[0] = pk.x; t.pk[1] = pk.y; t.pk[2] = pk.z; t.pk[3] = pk.w;
    t.f[0] = f.x; t.f[1] = f.y; t.f[2] = f.z; t.f[3] = f.w;
    t.l[0] = l.x; t.l[1] = l.y; t.l[2] = l.z; t.l[3] = l.w;
    t.b[0] = b0.x; t.b[1] = b0.y; t.b[2] = b1.x; t.b[3] = b1.y;
  } else {
#pragma unroll
    for (int k = 0; k < R; ++k) {
      const uint64_t idx = base + (uint64_t)k * kThreads + threadIdx.x;
      const uint64_t at = idx < end ? idx : end - 1;
      t.pk[k] = ldg_nt(a.packets + at);
      t.f[k] = ldg_nt(a.first + at);
      t.l[k] = ldg_nt(a.last + at);
      t.b[k] = ldg_nt(a.bytes + at);
    }
  }
}

// One record per lane at an arbitrary index (segment heads and tails).
template <int R>
__device__ __forceinline__ void load_single(Addr<R> &t, Rest<R> &r, const ClassifyArgs &a, uint64_t idx,
                                            bool ok) {
#pragma unroll
  for (int k = 0; k < R; ++k) {
    t.v[k] = false;
    t.s[k] = t.d[k] = r.pk[k] = r.f[k] = r.l[k] = 0;
    r.b[k] = 0;
  }
  if (ok) {
    t.v[0] = true;
    t.s[0] = ldg_nt(a.src + idx);
    t.d[0] = ldg_nt(a.dst + idx);
    r.pk[0] = ldg_nt(a.packets + idx);
    r.f[0] = ldg_nt(a.first + idx);
    r.l[0] = ldg_nt(a.last + idx);
    r.b[0] = ldg_nt(a.bytes + idx);
  }
}


// Classify the tile's records from their addresses: the accumulator row of
// each (2 * site + direction, or the NODIR row).
template <int R, bool LINES_LDS>
__device__ __forceinline__ void classify_tile(const Addr<R> &t, const ClassifyArgs &a, const Lds &L,
                                              uint32_t (&row)[R]) {
  const uint32_t rows = a.rows;
  // one root read per endpoint gives its locality and, for the remote one,
  // the first trie entry of its walk
  const uint32_t sh = 32u - a.root_bits, sb = 28u - a.root_bits;
  uint32_t remote[R], re[R], site[R];
  bool one[R], inbound[R], ls[R], ld[R], part = false;
#pragma unroll
  for (int k = 0; k < R; ++k) {
    const uint64_t es = L.root[t.s[k] >> sh], ed = L.root[t.d[k] >> sh];
    const uint32_t ms = (uint32_t)(es >> 32) >> ((t.s[k] >> sb) & 15u);
    const uint32_t md = (uint32_t)(ed >> 32) >> ((t.d[k] >> sb) & 15u);
    ls[k] = ms & 1u;
    ld[k] = md & 1u;
    part |= ((ms | md) >> kLocalSubBlocks) & 1u;
    re[k] = ld[k] ? (uint32_t)es : (uint32_t)ed;
  }
  if (__builtin_amdgcn_ballot_w64(part)) {  // partly local sub-blocks: exact ranges
#pragma unroll
    for (int k = 0; k < R; ++k) {
      const uint64_t es = L.root[t.s[k] >> sh], ed = L.root[t.d[k] >> sh];
      if (((uint32_t)(es >> 32) >> (16u + ((t.s[k] >> sb) & 15u))) & 1u) ls[k] = in_ranges(a.local, t.s[k]);
      if (((uint32_t)(ed >> 32) >> (16u + ((t.d[k] >> sb) & 15u))) & 1u) ld[k] = in_ranges(a.local, t.d[k]);
      re[k] = ld[k] ? (uint32_t)es : (uint32_t)ed;
    }
  }
#pragma unroll
  for (int k = 0; k < R; ++k) {
    one[k] = t.v[k] && ls[k] != ld[k];
    inbound[k] = ld[k];
    remote[k] = ld[k] ? t.s[k] : t.d[k];
  }
  lookup_sites<R, LINES_LDS>(remote, re, one, site, a.wide, L.lines, a.lines, a.root_bits, a.node_bits);
#pragma unroll
  for (int k = 0; k < R; ++k) row[k] = one[k] ? 2u * site[k] + (inbound[k] ? 0u : 1u) : rows - 1u;
}

// Per-host (or histogram key) staging of a tile: the wave's entries for all
// R record slots are reserved with one LDS atomic on `cursor` before the
// rates are computed (the bulk test and the row decide which records have
// one), so each entry can be written as soon as its rate is known.  hb[k]:
// the wave's lanes with an entry in slot k; returns the first entry of slot
// 0.  Called by the whole wave.
template <int R>
__device__ __forceinline__ uint32_t reserve_hosts(uint32_t *cursor, const bool (&want)[R], uint64_t (&hb)[R]) {
  uint32_t total = 0;
#pragma unroll
  for (int k = 0; k < R; ++k) {
    hb[k] = __builtin_amdgcn_ballot_w64(want[k]);
    total += (uint32_t)__builtin_popcountll(hb[k]);
  }
  if (total == 0u) return 0u;
  uint32_t base = 0;
  if (__lane_id() == (uint32_t)__builtin_ctzll(__builtin_amdgcn_read_exec())) base = atomicAdd(cursor, total);
  return __builtin_amdgcn_readfirstlane(base);
}

// One staged entry: two 16-byte stores.
__device__ __forceinline__ void stage_host(const Lds &L, uint32_t pos, uint64_t key, uint64_t bytes, uint64_t rate) {
  typedef u64 u64x2_ __attribute__((ext_vector_type(2)));
  u64x2_ *e = (u64x2_ *)(L.se + pos);
  e[0] = u64x2_{(u64)key, (u64)bytes};
  e[1] = u64x2_{(u64)rate, (u64)rate_bucket(rate)};
}

// Aggregate the tile's classified records.
template <int R, bool ACC_LDS, uint32_t FEAT>
__device__ __forceinline__ void aggregate_tile(const Addr<R> &t, const uint32_t (&row)[R], const Rest<R> &r,
                                               const ClassifyArgs &a, const Lds &L, u64 *g_tab,
                                               uint32_t *h_tab) {
  const bool(&valid)[R] = t.v;
  uint32_t durv[R];
  bool bulkv[R];
#pragma unroll
  for (int k = 0; k < R; ++k) {
    const uint32_t dur = r.l[k] - r.f[k];
    // (bitwise, not short-circuit: no branches)
    bool bulk = valid[k] & (r.b[k] > a.bulk_bytes) & (dur != 0u);
    // exclusion filters: average packet size, packet count, duration (one
    // wave-uniform branch when none is set)
    if (a.filters)
      bulk = bulk & (r.b[k] >= (uint64_t)a.min_avg_packet_bytes * r.pk[k]) & (r.pk[k] >= a.min_packets) &
             (dur >= a.min_duration_ms);
    durv[k] = dur;
    bulkv[k] = bulk;
  }
  // per-host statistics and staged histogram keys: bulk flows of registered
  // sites (not the "no site" rows or NODIR); a host is keyed by the remote
  // endpoint (the source of an inbound flow, the destination of an outbound
  // one).  With both, one reservation serves the two ranges.
  constexpr bool HOSTS = (FEAT & kFeatHosts) != 0;
  const bool kst = (FEAT & kFeatHist) && L.ke != nullptr;
  uint64_t hb[R];
  uint32_t hpos = 0;
  if (HOSTS || kst) {
    bool want[R];
#pragma unroll
    for (int k = 0; k < R; ++k) want[k] = bulkv[k] & (row[k] < a.hist_rows);
    hpos = reserve_hosts<R>(HOSTS ? L.hcur : L.kcur, want, hb);
  }
  const uint64_t below = (1ull << __lane_id()) - 1ull;
#pragma unroll
  for (int k = 0; k < R; ++k) {
    const uint32_t dur = durv[k];
    const bool bulk = bulkv[k];
    uint32_t code = row[k];
    // (a spare LDS row for invalid records instead of this branch measured
    // 10 % slower on the 64-site registry)
    if (valid[k]) code = accumulate<ACC_LDS>(L, g_tab, row[k], r.b[k], r.pk[k], dur, bulk);
    // a spilled table: a record that missed the cache becomes a partial row
    const bool spill = !ACC_LDS && L.te != nullptr;
    const bool miss = spill && valid[k] && !(code & kInSlot);
    uint64_t sbal = 0;
    uint32_t sbase = 0;
    if (spill) sbase = reserve_rows(L.tcur, miss, sbal);
    uint64_t rate = 0;
    if (bulk) rate = rate_bps(r.b[k], dur);
    if (miss)
      stage_entry(L, sbase + (uint32_t)__builtin_popcountll(sbal & below), L.win | (bulk ? kRecBulk : 0u),
                  row[k] | (kRec << kRowKindShift), (u64)r.pk[k] | ((u64)dur << 32), r.b[k], rate);
    if (bulk) {
      if (!miss) add_rate<ACC_LDS>(L, g_tab, code, rate);
      // count in the row's histogram: registered sites only
      if ((FEAT & kFeatHist) && row[k] < a.hist_rows) {
        if (kst) {
          const uint32_t grow = L.kbase + row[k];
          L.ke[hpos + (uint32_t)__builtin_popcountll(hb[k] & below)] = (grow << kHistBucketBits) | rate_bucket(rate);
          if (L.kp) atomicAdd(&L.kp[grow >> L.kshift], 1u);
        } else
          hist_add(L, h_tab, row[k], rate_bucket(rate));
      }
      if (HOSTS && row[k] < a.hist_rows) {
        const uint64_t key = ((uint64_t)((row[k] & 1u) ? t.d[k] : t.s[k]) << 32) | row[k];
        stage_host(L, hpos + (uint32_t)__builtin_popcountll(hb[k] & below), key, r.b[k], rate);
        if (L.hp) atomicAdd(&L.hp[(uint32_t)(mix64(key) >> (64u - L.hpbits))], 1u);
      }
    }
    if (HOSTS || kst) hpos += (uint32_t)__builtin_popcountll(hb[k]);
  }
}

template <int R, bool LINES_LDS, bool ACC_LDS, uint32_t FEAT>
__device__ __forceinline__ void process_tile(const Addr<R> &t, const Rest<R> &r, const ClassifyArgs &a,
                                             const Lds &L, u64 *g_tab, uint32_t *h_tab) {
  uint32_t row[R];
  classify_tile<R, LINES_LDS>(t, a, L, row);
  aggregate_tile<R, ACC_LDS, FEAT>(t, row, r, a, L, g_tab, h_tab);
}

// Records [lo, hi) of one window: tiles whose addresses are prefetched one
// tile ahead; the other fields load when their tile starts, so their latency
// overlaps the locality tests and the trie walk.  (Measured: prefetching the
// other fields a tile ahead as well, or in the middle of the walk, gained
// nothing at 4 waves per SIMD.)
template <int R, bool VEC, bool LINES_LDS, bool ACC_LDS, uint32_t FEAT>
__device__ __forceinline__ void process_range(const ClassifyArgs &a, const Lds &L, u64 *g_tab, uint32_t *h_tab,
                                              uint64_t lo, uint64_t hi) {
  constexpr uint64_t T = (uint64_t)kThreads * R;
  Addr<R> cur;
  load_addr<R, VEC>(cur, a, lo, hi);
  for (uint64_t base = lo; base < hi; base += T) {
    Rest<R> rest;
    load_rest<R, VEC>(rest, a, base, hi);
    Addr<R> nxt;
    load_addr<R, VEC>(nxt, a, base + T, hi);  // past the end: reloads the last records, marked invalid
    uint32_t row[R];
    classify_tile<R, LINES_LDS>(cur, a, L, row);
    aggregate_tile<R, ACC_LDS, FEAT>(cur, row, rest, a, L, g_tab, h_tab);
    cur = nxt;
  }
}

// ---------------------------------------------------------------- kernels

__global__ void init_acc_kernel(u64 *__restrict__ acc, uint64_t words) {
  const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < words) acc[i] = ((i & 7u) == 6u) ? ~0ull : 0ull;
}

// Zero n 32-bit words at a 16-byte aligned address: four per lane, grid-stride.
__global__ void zero_words_kernel(uint32_t *__restrict__ p, uint64_t n) {
  const uint64_t quads = (n + 3u) / 4u;
  for (uint64_t q = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; q < quads;
       q += (uint64_t)gridDim.x * blockDim.x) {
    if (4u * q + 4u <= n) {
      *(u32x4 *)(p + 4u * q) = u32x4{0u, 0u, 0u, 0u};
    } else {
      for (uint64_t j = 4u * q; j < n; ++j) p[j] = 0u;
    }
  }
}

template <int R, bool VEC, bool LINES_LDS, bool ACC_LDS, uint32_t FEAT>
__global__ __launch_bounds__(kThreads) void classify_kernel(const ClassifyArgs a) {
  constexpr bool HIST = (FEAT & kFeatHist) != 0;
  extern __shared__ __align__(16) unsigned char lds[];
  uint64_t *s_root = (uint64_t *)lds;
  u64 *s_acc = (u64 *)(lds + a.lds_off_acc);
  uint32_t *s_lines = (uint32_t *)(lds + a.lds_off_lines);
  const uint32_t tid = threadIdx.x;
  const uint32_t rows = a.rows;

  // stage the trie root (with locality masks) and, when they fit, the leaf lines
  const uint32_t nroot = 1u << a.root_bits;
  for (uint32_t i = tid; i < nroot; i += kThreads) s_root[i] = a.root[i];
  if (LINES_LDS)
    for (uint32_t i = tid; i < a.n_line_words; i += kThreads) s_lines[i] = a.lines[i];
  // the table, or the cache slots' rows and their tags
  const uint32_t slots = ACC_LDS ? 0u : a.cache_slots;
  uint32_t *s_tags = (uint32_t *)(s_acc + (uint64_t)slots * kAccFields);
  const uint32_t acc_words = kAccFields * (ACC_LDS ? rows : slots);
  for (uint32_t i = tid; i < acc_words; i += kThreads) s_acc[i] = (i % kAccFields == kRateMin) ? ~0ull : 0ull;
  for (uint32_t i = tid; i < slots; i += kThreads) s_tags[i] = 0u;
  const uint32_t hslots = HIST ? a.hist_slots : 0u;
  uint32_t *s_htags = (uint32_t *)(lds + a.lds_off_hist);
  for (uint32_t i = tid; i < 2u * hslots; i += kThreads) s_htags[i] = 0u;  // tags, then counts
  constexpr bool HOSTS = (FEAT & kFeatHosts) != 0;
  const bool spill = !ACC_LDS && a.ts_entry != nullptr;
  const bool kst = HIST && a.ks_key != nullptr;
  // cursors: per-host entries, spilled rows, the spilled-row flush's claimed
  // slots, histogram keys
  uint32_t *s_hcur = (uint32_t *)(lds + a.lds_off_ctr), *s_tcur = s_hcur + 1, *s_kcur = s_hcur + 3;
  if ((HOSTS || spill || kst) && tid < 4u) s_hcur[tid] = 0u;
  uint32_t *s_kp = (uint32_t *)(lds + a.lds_off_kp);
  const bool kcount = kst && a.kp_hist != nullptr;
  if (kcount) {
    for (uint32_t i = tid; i < a.kp_parts; i += kThreads) s_kp[i] = 0u;
    if (blockIdx.x == 0 && tid == 0) *a.kp_over = 0ull;
  }
  uint32_t *s_hp = (uint32_t *)(lds + a.lds_off_hp);
  const bool hcount = HOSTS && a.hp_hist != nullptr;
  const uint32_t hparts = 1u << a.hp_bits;
  if (hcount) {
    for (uint32_t i = tid; i < hparts; i += kThreads) s_hp[i] = 0u;
    if (blockIdx.x == 0 && tid < 2u) a.hp_clear[tid] = 0ull;
  }
  __syncthreads();
  // this workgroup's balanced slice of all records
  const uint64_t lo = (uint64_t)blockIdx.x * a.n / gridDim.x;
  const uint64_t hi = (uint64_t)(blockIdx.x + 1) * a.n / gridDim.x;
  Lds L{s_root, s_lines, s_acc, s_tags, slots, s_htags, s_htags + hslots, hslots, s_hcur,
        HOSTS ? a.hs_entry + lo : nullptr, s_tcur, spill ? a.ts_entry + lo + (uint64_t)blockIdx.x * a.ts_extra : nullptr,
        s_kcur, kst ? a.ks_key + lo : nullptr, kcount ? s_kp : nullptr, a.kp_shift, hcount ? s_hp : nullptr, a.hp_bits,
        0u, 0u};
  // spilled rows: the entries this workgroup's range holds
  const uint32_t t_cap = (uint32_t)(hi - lo) + a.ts_extra;
  if (lo == hi) {
    // empty slice: leave an empty table whose window keeps the slots ordered
    if (ACC_LDS && a.ws) {
      uint64_t we;
      flush_partial(a, s_acc, window_of(a, lo ? lo - 1 : 0, we));
    }
    if (HOSTS && tid == 0) a.hs_count[blockIdx.x] = 0u;
    if (spill && tid == 0) a.ts_count[blockIdx.x] = 0u;
    if (kst && tid == 0) a.ks_count[blockIdx.x] = 0u;
    if (kcount)
      for (uint32_t j = tid; j < a.kp_parts; j += kThreads) a.kp_hist[(uint64_t)blockIdx.x * a.kp_parts + j] = 0u;
    if (hcount)
      for (uint32_t j = tid; j < hparts; j += kThreads) a.hp_hist[(uint64_t)blockIdx.x * hparts + j] = 0u;
    return;
  }
  uint64_t i = lo;
  while (i < hi) {
    uint64_t wend;
    const uint32_t w = window_of(a, i, wend);
    uint64_t seg_end = wend < hi ? wend : hi;
    if (seg_end - i > a.flush_records) seg_end = i + a.flush_records;
    u64 *g_tab = a.acc + (uint64_t)w * rows * 8u;
    L.win = w;
    L.kbase = w * a.hist_rows;
    uint32_t *h_tab = HIST ? a.hist + (uint64_t)w * a.hist_rows * kBuckets : nullptr;

    if (VEC) {
      // whole groups of 4 records with vector loads; up to 3 records before
      // and after them in one single-record mini-tile
      const uint64_t a0 = ((i + 3) & ~3ull) < seg_end ? ((i + 3) & ~3ull) : seg_end;
      const uint64_t a1 = a0 + ((seg_end - a0) & ~3ull);
      if (i < a0 || a1 < seg_end) {
        Addr<R> m;
        Rest<R> mr;
        const bool head = tid < a0 - i, tail = tid >= 3 && tid - 3 < seg_end - a1;
        load_single(m, mr, a, head ? i + tid : a1 + (tid - 3), head || tail);
        process_tile<R, LINES_LDS, ACC_LDS, FEAT>(m, mr, a, L, g_tab, h_tab);
      }
      if (a0 < a1) process_range<4, true, LINES_LDS, ACC_LDS, FEAT>(a, L, g_tab, h_tab, a0, a1);
    } else {
      process_range<R, false, LINES_LDS, ACC_LDS, FEAT>(a, L, g_tab, h_tab, i, seg_end);
    }
    if (ACC_LDS) {
      if (seg_end >= hi && a.ws) flush_partial(a, s_acc, w);
      else flush_atomic(s_acc, g_tab, rows);
    } else if (slots) {
      // room for this flush: what the range holds less one entry for each
      // record still to come
      flush_cache(L, g_tab, t_cap - (uint32_t)(hi - seg_end));
    }
    if (HIST && hslots) flush_hist(L, h_tab);
    i = seg_end;
  }
  if (HOSTS || spill || kst) {
    __syncthreads();
    if (HOSTS && tid == 0) a.hs_count[blockIdx.x] = *s_hcur;
    if (spill && tid == 0) a.ts_count[blockIdx.x] = *s_tcur;
    // with per-host staging the keys share its cursor
    if (kst && tid == 0) a.ks_count[blockIdx.x] = HOSTS ? *s_hcur : *s_kcur;
    if (kcount)
      for (uint32_t j = tid; j < a.kp_parts; j += kThreads) a.kp_hist[(uint64_t)blockIdx.x * a.kp_parts + j] = s_kp[j];
    if (hcount)
      for (uint32_t j = tid; j < hparts; j += kThreads) a.hp_hist[(uint64_t)blockIdx.x * hparts + j] = s_hp[j];
  }
}

// Mean-rate test of gnm_flag_suboptimal, fused into the reduce kernel when a
// call asks for both: flags[w * n_sites + s] for every window w and site s.
struct FlagArgs {
  uint8_t *flags;  // NULL: no flags
  uint64_t threshold, need;
  uint32_t n_sites;
};

// Combine the workgroups' final tables.  The slots whose window is w form a
// contiguous range (slot windows never decrease).  Workgroup
// w * row_tiles + x owns rows 8x .. 8x + 7 (sites 4x .. 4x + 3) of window w's
// table, 56 consecutive words of the flattened table (rows of kAccFields
// words): lane j < 56 of each of its G waves (G = blockDim.x / 64, 1..16, set
// by the host from the slots per window) reads word j of every G-th slot, so
// each wave load is one contiguous 448-byte run, and the waves' partial
// results meet in LDS.  Adds into acc, or overwrites it when the classify
// launch left no other contribution.  With flags, wave 0 then holds the final
// bulk-flow counts and rate sums of the tile's rows and applies the mean-rate
// test to its four sites, reading acc as it stands where no slot belongs to
// the window.
__global__ __launch_bounds__(64 * kRedGroups) void reduce_partials_kernel(
    const u64 *__restrict__ ws, const uint32_t *__restrict__ meta, uint32_t slots, uint32_t rows,
    u64 *__restrict__ acc, uint32_t row_tiles, uint32_t overwrite, uint32_t one_window, FlagArgs fl) {
  const uint32_t w = blockIdx.x / row_tiles, tile = blockIdx.x - w * row_tiles;
  // window w's slots [b0, b1): the slot windows are sorted, so b0 counts the
  // slots of earlier windows and b1 adds w's own; every lane counts a strided
  // share, eight independent loads at a time.  A single window owns them all.
  uint32_t b0 = 0, b1 = slots;
  if (!one_window) {
    __shared__ uint32_t counts[2];
    if (threadIdx.x < 2u) counts[threadIdx.x] = 0u;
    __syncthreads();
    uint32_t lt = 0, le = 0;
    for (uint32_t k0 = threadIdx.x; k0 < slots; k0 += 8u * blockDim.x) {
      uint32_t m[8];  // eight loads in flight; past the end, a tag above every window
#pragma unroll
      for (uint32_t j = 0; j < 8u; ++j) {
        const uint32_t k = k0 + j * blockDim.x;
        m[j] = k < slots ? meta[k] : ~0u;
      }
#pragma unroll
      for (uint32_t j = 0; j < 8u; ++j) {
        lt += m[j] < w;
        le += m[j] <= w;
      }
    }
#pragma unroll
    for (uint32_t o = 32; o > 0; o >>= 1) {
      lt += __shfl_xor(lt, o, 64);
      le += __shfl_xor(le, o, 64);
    }
    if (threadIdx.x % 64u == 0u && le) {
      atomicAdd(&counts[0], lt);
      atomicAdd(&counts[1], le);
    }
    __syncthreads();
    b0 = counts[0];
    b1 = counts[1];
  }
  const bool any = b0 < b1;
  if (!any && !fl.flags) return;
  const uint32_t lane = threadIdx.x % 64u, g = threadIdx.x / 64u, groups = blockDim.x / 64u;
  const uint32_t words = kAccFields * rows;
  const uint32_t i = tile * kRedWords + lane;
  const bool mine = lane < kRedWords && i < words;
  const uint32_t f = lane % kAccFields;  // = i % kAccFields: tiles start on a row
  const bool is_cnt = f == kCnt, is_min = f == kRateMin, is_max = f == kRateMax;
  // x: sum (or min / max) of the word; y: bulk flows, for the packed count word
  u64 xs = 0, y = 0, xmin = ~0ull, xmax = 0;
  if (mine) {
    const u64 *p = ws + i;
    // kRedUnroll loads in flight per lane (indexes past the range reload its
    // last slot and are masked), then branch-free combining
    for (uint32_t base = b0 + g; base < b1; base += groups * kRedUnroll) {
      u64 v[kRedUnroll];
#pragma unroll
      for (uint32_t j = 0; j < kRedUnroll; ++j) {
        const uint32_t b = base + j * groups;
        v[j] = __builtin_nontemporal_load(p + (uint64_t)(b < b1 ? b : b1 - 1u) * words);
      }
#pragma unroll
      for (uint32_t j = 0; j < kRedUnroll; ++j) {
        const bool ok = base + j * groups < b1;
        const u64 val = v[j];
        xs += ok ? (is_cnt ? (val & 0xFFFFFFFFull) : val) : 0ull;
        y += ok && is_cnt ? val >> 32 : 0ull;
        xmin = ok && val < xmin ? val : xmin;
        xmax = ok && val > xmax ? val : xmax;
      }
    }
  }
  u64 x = is_min ? xmin : (is_max ? xmax : xs);
  // the waves' partial results: 1 KB of dynamic LDS per wave (a small
  // workgroup takes little LDS, so many fit a CU at once)
  extern __shared__ u64 red[];  // [groups][2][64]
  red[(2u * g) * 64u + lane] = x;
  red[(2u * g + 1u) * 64u + lane] = y;
  __syncthreads();
  if (g != 0) return;
  for (uint32_t s = 1; s < groups; ++s) {
    const u64 v = red[(2u * s) * 64u + lane];
    if (f == kRateMin) x = v < x ? v : x;
    else if (f == kRateMax) x = v > x ? v : x;
    else x += v;
    y += red[(2u * s + 1u) * 64u + lane];
  }
  // table word (row, f) -> acc fields: cnt -> flows (0) and bulk flows (4);
  // bytes, packets, duration -> 1..3; rate sum, min, max -> 5..7.  fx, fy:
  // the word's final value, and the bulk flows beside a count word.
  u64 fx = 0, fy = 0;
  if (mine) {
    const uint32_t r = i / kAccFields;
    u64 *o = acc + ((uint64_t)w * rows + r) * 8u;
    const uint32_t of = f == kCnt ? 0u : (f < kRateSum ? f : f + 1u);
    if (!any) {
      fx = o[of];
      fy = f == kCnt ? o[4] : 0ull;
    } else if (overwrite) {
      fx = x;
      fy = y;
    } else if (f == kRateMin) {
      const u64 c = o[of];
      fx = x < c ? x : c;
    } else if (f == kRateMax) {
      const u64 c = o[of];
      fx = x > c ? x : c;
    } else {
      fx = o[of] + x;
      fy = f == kCnt ? o[4] + y : 0ull;
    }
    if (any) {
      o[of] = fx;
      if (f == kCnt) o[4] = fy;
    }
  }
  if (!fl.flags) return;
  // lane j < 4 tests site 4 * tile + j: rows 2j (inbound) and 2j + 1
  // (outbound) of the tile; every lane takes part in the exchanges
  const uint32_t j = lane & 3u;
  const uint32_t c0 = 2u * j * kAccFields;
  const u64 nb0 = __shfl(fy, (int)(c0 + kCnt), 64), sum0 = __shfl(fx, (int)(c0 + kRateSum), 64);
  const u64 nb1 = __shfl(fy, (int)(c0 + kAccFields + kCnt), 64);
  const u64 sum1 = __shfl(fx, (int)(c0 + kAccFields + kRateSum), 64);
  const uint32_t site = tile * (kRedRows / 2u) + j;
  if (lane < 4u && site < fl.n_sites) {
    uint8_t fv = 0;
    if (nb0 >= fl.need && sum0 / nb0 < fl.threshold) fv |= 1u;
    if (nb1 >= fl.need && sum1 / nb1 < fl.threshold) fv |= 2u;
    fl.flags[(uint64_t)w * fl.n_sites + site] = fv;
  }
}

__global__ void flag_kernel(const u64 *__restrict__ acc, uint32_t n_windows, uint32_t n_sites,
                            uint32_t rows, uint64_t threshold, uint64_t need,
                            uint8_t *__restrict__ flags) {
  const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (uint64_t)n_windows * n_sites) return;
  const uint64_t w = i / n_sites, s = i - w * n_sites;
  const u64 *row = acc + (w * rows + 2u * s) * 8u;
  uint8_t f = 0;
  for (uint32_t dir = 0; dir < 2; ++dir) {
    const u64 nb = row[dir * 8 + 4], sum = row[dir * 8 + 5];
    if (nb >= need && sum / nb < threshold) f |= (uint8_t)(1u << dir);
  }
  flags[i] = f;
}

__device__ __forceinline__ u64 wave_sum(u64 x) {
#pragma unroll
  for (uint32_t o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o, 64);
  return x;
}

__device__ __forceinline__ u64 wave_inclusive_scan(u64 x, uint32_t lane) {
#pragma unroll
  for (uint32_t o = 1; o < 64; o <<= 1) {
    const u64 y = __shfl_up(x, o, 64);
    if (lane >= o) x += y;
  }
  return x;
}

// Lower-median bucket of one histogram row: the bucket holding the
// ceil(total/2)-th smallest count.  `bsum` holds, on lane b, the total of
// batch b (1024 buckets), 0 on lanes past the last batch.  The batch holding
// the target is found by a scan over the lanes, reloaded as 16 consecutive
// buckets per lane, and the lane whose run holds the target walks it.
__device__ __forceinline__ uint32_t row_median(const uint32_t *row, u64 bsum, u64 total, uint32_t lane) {
  if (total == 0u) return 0xFFFFFFFFu;
  const u64 target = total - total / 2u;
  const u64 incl = wave_inclusive_scan(bsum, lane);
  const uint32_t b = (uint32_t)__ffsll((unsigned long long)__ballot(incl >= target)) - 1u;
  const u64 before = __shfl(incl - bsum, b, 64);
  const uint32_t base = b * kMedBatchWords + lane * kMedRun;
  uint32_t v[kMedRun];
  u64 s = 0;
#pragma unroll
  for (uint32_t j = 0; j < kMedRun; ++j) {
    v[j] = base + j < kBuckets ? row[base + j] : 0u;
    s += v[j];
  }
  const u64 li = wave_inclusive_scan(s, lane) + before;
  const uint32_t owner = (uint32_t)__ffsll((unsigned long long)__ballot(li >= target)) - 1u;
  uint32_t m = 0;
  if (lane == owner) {
    u64 c = li - s;
#pragma unroll
    for (uint32_t j = 0; j < kMedRun; ++j) {
      c += v[j];
      if (c >= target) { m = base + j; break; }
    }
  }
  return __shfl(m, owner, 64);
}

// This lane's part of the totals of batch b of two rows (buckets b*1024 +
// 64j + lane), streamed with coalesced loads, 32 in flight per lane.  The
// last, partial batch is read as the row's final 1024 buckets (in bounds,
// same immediate offsets) and counts only its own buckets.
__device__ __forceinline__ void batch_sums(const uint32_t *r0, const uint32_t *r1, uint32_t b, uint32_t lane,
                                           u64 &s0, u64 &s1) {
  const uint32_t lo = b * kMedBatchWords;
  const uint32_t start = b < kMedFullBatches ? lo : kBuckets - kMedBatchWords;
  const uint32_t *p0 = r0 + start + lane, *p1 = r1 + start + lane;
  uint32_t v0[kMedRun], v1[kMedRun];
#pragma unroll
  for (uint32_t j = 0; j < kMedRun; ++j) {
    v0[j] = __builtin_nontemporal_load(p0 + j * 64u);
    v1[j] = __builtin_nontemporal_load(p1 + j * 64u);
  }
  s0 = 0;
  s1 = 0;
#pragma unroll
  for (uint32_t j = 0; j < kMedRun; ++j) {
    const bool mine = start + j * 64u + lane >= lo;
    s0 += mine ? v0[j] : 0u;
    s1 += mine ? v1[j] : 0u;
  }
}

// Lower medians of the rate histograms: one workgroup of 4 waves per (window,
// site) item.  The waves share the item's two rows (inbound, outbound): each
// streams every 4th 1024-bucket batch of both rows once (32 loads in flight
// per lane) and leaves the batch totals in LDS; then wave d walks row d from
// those totals, re-reading only the batch that holds the median.  (One wave
// per item left a single window's 1,000 items too few waves to cover the
// memory latency.)  Writes the median buckets (NO_MEDIAN when a row has no
// bulk flow) when `median` is not NULL, and bits 0/1 of the item's flag
// byte: total >= need and bucket * 10 kbps < threshold.
__global__ __launch_bounds__(64 * kMedWaves) void median_kernel(const uint32_t *__restrict__ hist, uint64_t items,
                                                               uint64_t threshold, uint64_t need,
                                                               uint32_t *__restrict__ median,
                                                               uint8_t *__restrict__ flags) {
  __shared__ u64 s_bsum[2][kMedBatches];
  __shared__ uint32_t s_med[2];
  __shared__ u64 s_total[2];
  const uint32_t lane = threadIdx.x % 64u, wave = threadIdx.x / 64u;
  for (uint64_t item = blockIdx.x; item < items; item += gridDim.x) {
    const uint32_t *r0 = hist + 2u * item * kBuckets, *r1 = r0 + kBuckets;
#pragma unroll 1
    for (uint32_t b = wave; b < kMedBatches; b += kMedWaves) {
      u64 s0, s1;
      batch_sums(r0, r1, b, lane, s0, s1);
      s0 = wave_sum(s0);
      s1 = wave_sum(s1);
      if (lane == 0u) {
        s_bsum[0][b] = s0;
        s_bsum[1][b] = s1;
      }
    }
    __syncthreads();
    if (wave < 2u) {
      const u64 bs = lane < kMedBatches ? s_bsum[wave][lane] : 0u;
      const u64 total = wave_sum(bs);
      const uint32_t m = row_median(wave ? r1 : r0, bs, total, lane);
      if (lane == 0u) {
        s_med[wave] = m;
        s_total[wave] = total;
      }
    }
    __syncthreads();
    if (threadIdx.x == 0u) {
      uint8_t f = 0;
      for (uint32_t d = 0; d < 2; ++d) {
        if (median) median[2u * item + d] = s_med[d];
        if (s_total[d] >= need && (u64)s_med[d] * kBucketBps < threshold) f |= (uint8_t)(1u << d);
      }
      flags[item] = f;
    }
  }
}

// The two-window rule, one lane per site walking the windows in order: bit
// 2 + d is set when bit d (low median) is set in this window and in the one
// before it (the caller's `prev` byte for the first window).  Flag bytes are
// read in independent batches ahead of the rewrites.
__global__ void warn_kernel(uint8_t *__restrict__ flags, uint32_t n_windows, uint32_t n_sites,
                            const uint8_t *__restrict__ prev) {
  constexpr uint32_t kBatch = 32;
  const uint64_t s = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= n_sites) return;
  uint32_t before = prev ? prev[s] & 3u : 0u;
  for (uint32_t w0 = 0; w0 < n_windows; w0 += kBatch) {
    uint32_t low[kBatch];
#pragma unroll
    for (uint32_t j = 0; j < kBatch; ++j)
      low[j] = w0 + j < n_windows ? flags[(uint64_t)(w0 + j) * n_sites + s] & 3u : 0u;
#pragma unroll
    for (uint32_t j = 0; j < kBatch; ++j) {
      if (w0 + j < n_windows) {
        flags[(uint64_t)(w0 + j) * n_sites + s] = (uint8_t)(low[j] | ((low[j] & before) << 2));
        before = low[j];
      }
    }
  }
}

// ---------------------------------------------------------------- launch plumbing

namespace {

int hip_fail(hipError_t e, const char *where) {
  set_last_error(std::string(where) + ": " + hipGetErrorString(e));
  return GNM_E_HIP;
}

int device_cus(int dev) {
  static std::mutex mu;
  static int cus[64] = {};
  std::lock_guard<std::mutex> g(mu);
  if (dev < 0 || dev >= 64) return 256;
  if (cus[dev] == 0) {
    int c = 0;
    if (hipDeviceGetAttribute(&c, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || c <= 0) c = 256;
    cus[dev] = c;
  }
  return cus[dev];
}

typedef void (*KernelFn)(const ClassifyArgs);

// variant slot: feat * 16 + shape * 4 + lists * 2 + acc; shapes: R=1, R=2, R=4 strided, R=4 vector
template <int R, bool V, uint32_t F>
KernelFn pick_la(bool lists, bool acc) {
  if (lists) return acc ? classify_kernel<R, V, true, true, F> : classify_kernel<R, V, true, false, F>;
  return acc ? classify_kernel<R, V, false, true, F> : classify_kernel<R, V, false, false, F>;
}

template <uint32_t F>
KernelFn pick_shape(int shape, bool lists, bool acc) {
  switch (shape) {
    case 0: return pick_la<1, false, F>(lists, acc);
    case 1: return pick_la<2, false, F>(lists, acc);
    case 2: return pick_la<4, false, F>(lists, acc);
    default: return pick_la<4, true, F>(lists, acc);
  }
}

KernelFn pick(int shape, bool lists, bool acc, uint32_t feat) {
  switch (feat) {
    case 0: return pick_shape<0>(shape, lists, acc);
    case kFeatHist: return pick_shape<kFeatHist>(shape, lists, acc);
    case kFeatHosts: return pick_shape<kFeatHosts>(shape, lists, acc);
    default: return pick_shape<kFeatHist | kFeatHosts>(shape, lists, acc);
  }
}

// Allow every kernel variant the full 160 KB of LDS, once per device.
hipError_t allow_lds(KernelFn fn, int slot, int dev) {
  static std::mutex mu;
  static bool done[64][64] = {};
  std::lock_guard<std::mutex> g(mu);
  if (dev >= 0 && dev < 64 && done[dev][slot]) return hipSuccess;
  hipError_t e = hipFuncSetAttribute((const void *)fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)kLdsMax);
  if (e == hipSuccess && dev >= 0 && dev < 64) done[dev][slot] = true;
  return e;
}

uint32_t blocks_per_cu(const gnm_registry *reg) { return reg->lds_bytes <= kLdsMax / 2 ? 2u : 1u; }

uint64_t partial_bytes(const gnm_registry *reg, uint64_t grid) {
  const uint64_t tables = grid * kAccFields * reg->rows() * 8u;
  return tables + ((grid * 4u + 255u) & ~255ull);
}

bool aligned16(const void *p) { return ((uintptr_t)p & 15u) == 0; }

// Workgroups of a classify launch over n records with R records per lane:
// the caller's count, else one resident wave of workgroups (fewer for short
// runs).
uint64_t launch_grid(const gnm_registry *reg, uint64_t n, uint32_t R, uint32_t grid_blocks, int dev) {
  const uint64_t resident = (uint64_t)device_cus(dev) * blocks_per_cu(reg);
  const uint64_t tiles = (n + (uint64_t)kThreads * R - 1) / ((uint64_t)kThreads * R);
  uint64_t grid = grid_blocks ? grid_blocks : (tiles < resident ? tiles : resident);
  if (grid == 0) grid = 1;
  if (grid > 65535u * 16u) grid = 65535u * 16u;
  return grid;
}

}  // namespace
}  // namespace gnm

using namespace gnm;

extern "C" gnm_params gnm_params_default(void) {
  gnm_params p{};
  p.bulk_bytes = 1000000ull;
  return p;
}

extern "C" uint64_t gnm_host_work_bytes(const gnm_registry *reg, uint64_t n_records, uint32_t grid_blocks) {
  if (!reg) return 0;
  // an automatic launch uses at most one resident wave of workgroups
  const uint64_t grid = grid_blocks ? grid_blocks : (uint64_t)device_cus(reg->device) * blocks_per_cu(reg);
  return host_work_bytes(n_records, grid);
}

extern "C" uint64_t gnm_workspace_bytes_n(const gnm_registry *reg, uint64_t n_records, uint32_t n_windows,
                                          uint32_t grid_blocks) {
  if (!reg) return 0;
  const uint64_t grid = grid_blocks ? grid_blocks : (uint64_t)device_cus(reg->device) * blocks_per_cu(reg);
  if (reg->acc_in_lds) return partial_bytes(reg, grid);
  if (n_windows == 0 || !table_fits(n_windows, (uint32_t)reg->rows())) return 0;
  return table_spill_bytes(n_records, grid, n_windows, (uint32_t)reg->rows(), reg->cache_slots);
}

extern "C" uint64_t gnm_workspace_bytes_hist(const gnm_registry *reg, uint64_t n_records, uint32_t n_windows,
                                             uint32_t grid_blocks) {
  if (!reg || n_windows == 0) return 0;
  const uint64_t grid = grid_blocks ? grid_blocks : (uint64_t)device_cus(reg->device) * blocks_per_cu(reg);
  const uint64_t tables = (gnm_workspace_bytes_n(reg, n_records, n_windows, grid_blocks) + 255u) & ~255ull;
  const uint32_t hist_rows = 2u * reg->n_sites;
  if (!hist_stage_fits(n_records, n_windows, hist_rows)) return tables;
  return tables + hist_work_bytes(n_records, grid, n_windows, hist_rows);
}

extern "C" uint64_t gnm_workspace_bytes(const gnm_registry *reg, uint32_t grid_blocks) {
  if (!reg) return 0;
  const uint64_t grid = grid_blocks ? grid_blocks : (uint64_t)device_cus(reg->device) * blocks_per_cu(reg);
  return partial_bytes(reg, grid);
}

namespace {

// gnm_classify_aggregate, and with fl.flags also gnm_flag_suboptimal on the
// result: fused into the reduce kernel when the workspace is used, otherwise
// the flag kernel after the classify launch.  Every argument is validated and
// the kernel attributes are set before anything is enqueued; with
// launch == false the call stops there (a graph's validation, outside
// capture).
int classify_impl(const gnm_registry *reg, const gnm_records *rec, const uint64_t *window_offsets,
                  uint32_t n_windows, const gnm_params *pp, gnm_acc *acc, const FlagArgs &fl,
                  hipStream_t stream, bool launch) {
  if (!reg || !rec || !acc) { set_last_error("NULL argument"); return GNM_E_INVAL; }
  if (reg->host_only) { set_last_error("registry was built host-only"); return GNM_E_UNSUPPORTED; }
  if (n_windows == 0) { set_last_error("n_windows must be >= 1"); return GNM_E_INVAL; }
  if (!window_offsets && n_windows != 1) { set_last_error("several windows need offsets"); return GNM_E_INVAL; }
  if (rec->n > 0 && (!rec->src_ip || !rec->dst_ip || !rec->bytes || !rec->packets || !rec->first_ms ||
                     !rec->last_ms)) {
    set_last_error("NULL record field");
    return GNM_E_INVAL;
  }
  const gnm_params p = pp ? *pp : gnm_params_default();
  const uint64_t flush_records =
      p.flush_records && p.flush_records < kMaxRecordsPerFlush ? p.flush_records : kMaxRecordsPerFlush;
  const uint32_t R = p.records_per_thread ? p.records_per_thread : 4u;
  if (R != 1 && R != 2 && R != 4) { set_last_error("records_per_thread must be 0, 1, 2 or 4"); return GNM_E_INVAL; }
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
  if (dev != reg->device) { set_last_error("registry belongs to another device"); return GNM_E_INVAL; }

  const uint64_t rows = reg->rows();
  const uint64_t grid = launch_grid(reg, rec->n, R, p.grid_blocks, dev);
  if ((uint64_t)n_windows * rows * 8u > (uint64_t)INT32_MAX * 256u) {
    set_last_error("accumulator tables too large");
    return GNM_E_INVAL;
  }
  const uint64_t hist_words = (uint64_t)n_windows * 2u * reg->n_sites * kBuckets;
  if (p.rate_hist && !aligned16(p.rate_hist)) {
    set_last_error("rate_hist must be 16-byte aligned");
    return GNM_E_INVAL;
  }
  const gnm_host_table *ht = p.hosts;
  if (ht) {
    if ((ht->capacity && (!ht->keys || !ht->stats)) || !ht->counters || !ht->work ||
        ((uintptr_t)ht->keys & 7u) || ((uintptr_t)ht->stats & 7u) || ((uintptr_t)ht->counters & 7u) ||
        ((uintptr_t)ht->median & 3u) || ((uintptr_t)ht->work & 255u)) {
      set_last_error("host table: NULL or misaligned arrays or work buffer");
      return GNM_E_INVAL;
    }
    if (p.flags & GNM_ACCUMULATE) {
      set_last_error("per-host statistics cover one call's records: GNM_ACCUMULATE cannot be combined with hosts");
      return GNM_E_INVAL;
    }
    if (rec->n >= (1ull << 32)) {
      set_last_error("per-host statistics need fewer than 2^32 records per call");
      return GNM_E_INVAL;
    }
    if (ht->work_bytes < host_work_bytes(rec->n, grid)) {
      set_last_error("host table: work buffer of " + std::to_string(ht->work_bytes) + " bytes, " +
                     std::to_string(host_work_bytes(rec->n, grid)) + " needed (gnm_host_work_bytes)");
      return GNM_E_INVAL;
    }
  }
  const uint64_t row_tiles = (rows + kRedRows - 1) / kRedRows;
  const bool use_ws = rec->n > 0 && reg->acc_in_lds && p.workspace &&
                      p.workspace_bytes >= partial_bytes(reg, grid) && aligned16(p.workspace) &&
                      row_tiles * n_windows <= (uint64_t)INT32_MAX;
  // With one window, a workspace, no accumulation and slices short enough to
  // need no mid-launch flush, the reduce kernel writes every row of the
  // table, so it needs no initialisation.
  const bool overwrite = use_ws && n_windows == 1 && !(p.flags & GNM_ACCUMULATE) &&
                         (rec->n + grid - 1) / grid <= flush_records;

  ClassifyArgs a{};
  a.src = rec->src_ip; a.dst = rec->dst_ip; a.bytes = rec->bytes; a.packets = rec->packets;
  a.first = rec->first_ms; a.last = rec->last_ms; a.n = rec->n;
  a.flush_records = flush_records;
  a.woff = (gu64 *)window_offsets; a.n_windows = n_windows; a.rows = (uint32_t)rows;
  a.bulk_bytes = p.bulk_bytes; a.acc = (u64 *)acc;
  a.min_avg_packet_bytes = p.min_avg_packet_bytes; a.min_packets = p.min_packets;
  a.min_duration_ms = p.min_duration_ms;
  a.filters = (p.min_avg_packet_bytes | p.min_packets | p.min_duration_ms) != 0u;
  a.root = (gu64 *)reg->d_root; a.wide = (gu32 *)reg->d_wide; a.lines = (gu32 *)reg->d_lines;
  a.root_bits = reg->root_bits; a.node_bits = reg->node_bits; a.n_line_words = (uint32_t)reg->lines.size();
  a.lds_off_acc = reg->lds_off_acc; a.lds_off_lines = reg->lds_off_lines;
  a.cache_slots = reg->acc_in_lds ? 0u : reg->cache_slots;
  a.hist = p.rate_hist;
  a.hist_rows = 2u * reg->n_sites;
  if (ht) {
    const HostStage st = host_stage(ht->work, rec->n, grid);
    a.hs_entry = st.entry;
    a.hs_count = st.count;
  }
  // a table beyond LDS with a workspace that holds its spilled rows: the
  // misses of the row cache and its flushes are staged and merged by the
  // table kernels instead of device-scope atomics
  const bool spill = !reg->acc_in_lds && rec->n > 0 && rec->n < (1ull << 32) && p.workspace &&
                     ((uintptr_t)p.workspace & 255u) == 0 && table_fits(n_windows, (uint32_t)rows) &&
                     p.workspace_bytes >= table_spill_bytes(rec->n, grid, n_windows, (uint32_t)rows, reg->cache_slots);
  if (spill) {
    const TableStage ts = table_stage(p.workspace, rec->n, grid, n_windows, (uint32_t)rows, reg->cache_slots);
    a.ts_entry = ts.entry;
    a.ts_count = ts.count;
    a.ts_extra = (uint32_t)table_extra(reg->cache_slots);
  }
  // histograms with a workspace that also holds their keys, after what the
  // tables use of it: staged keys and the histogram kernels instead of the
  // LDS cache, device-scope atomics and the zeroing pass
  char *hist_work = nullptr;
  HistStage ks{};
  if (p.rate_hist && rec->n > 0 && p.workspace && ((uintptr_t)p.workspace & 255u) == 0 &&
      hist_stage_fits(rec->n, n_windows, a.hist_rows)) {
    const uint64_t used = spill ? table_spill_bytes(rec->n, grid, n_windows, (uint32_t)rows, reg->cache_slots)
                                : (use_ws ? partial_bytes(reg, grid) : 0u);
    const uint64_t off = (used + 255u) & ~255ull;
    if (p.workspace_bytes >= off + hist_work_bytes(rec->n, grid, n_windows, a.hist_rows)) {
      hist_work = (char *)p.workspace + off;
      ks = hist_stage(hist_work, rec->n, grid, n_windows, a.hist_rows);
      a.ks_key = ks.key;
      a.ks_count = ks.count;
    }
  }
  uint32_t lds_launch = reg->lds_bytes;
  if (p.rate_hist && !hist_work) {
    // the histogram cache takes the LDS the registry leaves free, within the
    // budget that keeps the registry's workgroups per CU
    const uint32_t off = (reg->lds_bytes + 15u) & ~15u;
    const uint32_t budget = (reg->lds_bytes <= kLdsMax / 2 ? kLdsMax / 2 : kLdsMax) - kLdsReserve;
    uint32_t hs = budget > off ? (budget - off) / 8u : 0u;
    hs = (hs < kHistSlotsMax ? hs : kHistSlotsMax) & ~3u;
    if (hs < 64u) hs = 0;
    a.lds_off_hist = off;
    a.hist_slots = hs;
    lds_launch = off + hs * 8u;
  }
  if (hist_work) {
    // the keys' partition counts in LDS too, when they fit that budget
    // (otherwise the count kernel counts them)
    const uint32_t off = (lds_launch + 15u) & ~15u;
    const uint32_t budget = (reg->lds_bytes <= kLdsMax / 2 ? kLdsMax / 2 : kLdsMax) - kLdsReserve;
    if (off + 4u * ks.nparts <= budget) {
      a.kp_hist = ks.phist;
      a.kp_over = ks.over;
      a.kp_shift = ks.shift;
      a.kp_parts = ks.nparts;
      a.lds_off_kp = off;
      lds_launch = off + 4u * ks.nparts;
    }
  }
  if (ht) {
    // the per-host entries' partition counts in LDS too, when they fit
    // (otherwise the count kernel counts them)
    const HostStage st = host_stage(ht->work, rec->n, grid);
    const uint32_t off = (lds_launch + 15u) & ~15u;
    const uint32_t budget = (reg->lds_bytes <= kLdsMax / 2 ? kLdsMax / 2 : kLdsMax) - kLdsReserve;
    if (rec->n > 0 && off + (4u << st.pbits) <= budget) {
      a.hp_hist = st.phist;
      a.hp_bits = st.pbits;
      a.hp_clear = (unsigned long long *)ht->counters;
      a.lds_off_hp = off;
      lds_launch = off + (4u << st.pbits);
    }
  }
  if (ht || spill || hist_work) {
    // the staging cursors: words in the bytes every LDS plan leaves free
    a.lds_off_ctr = (lds_launch + 15u) & ~15u;
    lds_launch = a.lds_off_ctr + 16u;
  }
  if (use_ws) {
    a.ws = (u64 *)p.workspace;
    a.ws_meta = (uint32_t *)((char *)p.workspace + grid * kAccFields * rows * 8u);
  }
  a.local.n = (uint32_t)reg->local_lo.size();
  for (uint32_t j = 0; j < a.local.n; ++j) {
    a.local.lo[j] = reg->local_lo[j];
    a.local.span[j] = reg->local_hi[j] - reg->local_lo[j];
  }

  const bool vec = R == 4 && aligned16(rec->src_ip) && aligned16(rec->dst_ip) && aligned16(rec->bytes) &&
                   aligned16(rec->packets) && aligned16(rec->first_ms) && aligned16(rec->last_ms);
  const int shape = vec ? 3 : (R == 1 ? 0 : (R == 2 ? 1 : 2));
  const uint32_t feat = (p.rate_hist ? kFeatHist : 0u) | (p.hosts ? kFeatHosts : 0u);
  KernelFn fn = pick(shape, reg->lines_in_lds, reg->acc_in_lds, feat);
  if (rec->n > 0) {
    e = allow_lds(fn, (int)feat * 16 + shape * 4 + (reg->lines_in_lds ? 2 : 0) + (reg->acc_in_lds ? 1 : 0), dev);
    if (e != hipSuccess) return hip_fail(e, "hipFuncSetAttribute");
  }
  if (hist_work) {
    e = hist_prepare(dev);
    if (e != hipSuccess) return hip_fail(e, "hipFuncSetAttribute (histograms)");
  }
  if (!launch) return GNM_OK;

  if (!(p.flags & GNM_ACCUMULATE) && !overwrite) {
    const uint64_t words = (uint64_t)n_windows * rows * 8u;
    const uint64_t blocks = (words + 255) / 256;
    hipLaunchKernelGGL(init_acc_kernel, dim3((uint32_t)blocks), dim3(256), 0, stream, (u64 *)acc, words);
    e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(e, "init launch");
  }
  if (p.rate_hist && !(p.flags & GNM_ACCUMULATE) && !hist_work) {
    const uint64_t quads = (hist_words + 3u) / 4u;
    const uint64_t cap = (uint64_t)device_cus(dev) * 64u;
    const uint64_t blocks = (quads + 255u) / 256u < cap ? (quads + 255u) / 256u : cap;
    hipLaunchKernelGGL(zero_words_kernel, dim3((uint32_t)(blocks ? blocks : 1u)), dim3(256), 0, stream,
                       p.rate_hist, hist_words);
    e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(e, "histogram init launch");
  }
  // the per-host kernels, after the classify launch (and on an empty run)
  auto count_hosts = [&]() -> int {
    if (!ht) return GNM_OK;
    return host_pipeline_launch(ht, rec->n, grid, a.hp_hist != nullptr, stream);
  };
  // the mean-rate flags, when the reduce kernel does not apply them
  auto flag_launch = [&]() -> int {
    if (!fl.flags) return GNM_OK;
    const uint64_t items = (uint64_t)n_windows * reg->n_sites;
    hipLaunchKernelGGL(flag_kernel, dim3((uint32_t)((items + 255) / 256)), dim3(256), 0, stream, (const u64 *)acc,
                       n_windows, reg->n_sites, (uint32_t)rows, fl.threshold, fl.need, fl.flags);
    const hipError_t e2 = hipGetLastError();
    return e2 == hipSuccess ? GNM_OK : hip_fail(e2, "flag launch");
  };
  if (rec->n == 0) {
    const int rc = flag_launch();
    return rc == GNM_OK ? count_hosts() : rc;
  }

  hipLaunchKernelGGL(fn, dim3((uint32_t)grid), dim3(kThreads), lds_launch, stream, a);
  e = hipGetLastError();
  if (e != hipSuccess) return hip_fail(e, "classify launch");
  if (spill) {
    const TableFlags tf{fl.flags, fl.threshold, fl.need, fl.n_sites};
    const int rc = table_merge_launch(p.workspace, rec->n, grid, n_windows, (uint32_t)rows, reg->cache_slots,
                                      (unsigned long long *)acc, tf, stream);
    if (rc != GNM_OK) return rc;
  } else if (use_ws) {
    // waves per reduce workgroup: enough for one round of kRedUnroll loads per
    // lane over the mean slots per window, rounded up to a power of two, at
    // most kRedGroups (smaller workgroups fit more per CU at once)
    const uint64_t rounds = ((grid + n_windows - 1) / n_windows + kRedUnroll - 1) / kRedUnroll;
    uint32_t groups = 1;
    while (groups < kRedGroups && groups < rounds) groups *= 2;
    hipLaunchKernelGGL(reduce_partials_kernel, dim3((uint32_t)(row_tiles * n_windows)), dim3(64 * groups),
                       groups * 2u * 64u * sizeof(u64),
                       stream, (const u64 *)a.ws, (const uint32_t *)a.ws_meta, (uint32_t)grid, (uint32_t)rows,
                       (u64 *)acc, (uint32_t)row_tiles, overwrite ? 1u : 0u, n_windows == 1 ? 1u : 0u, fl);
    e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(e, "reduce launch");
  } else {
    const int rc = flag_launch();
    if (rc != GNM_OK) return rc;
  }
  if (hist_work) {
    const int rc = hist_pipeline_launch(hist_work, rec->n, grid, n_windows, a.hist_rows, p.rate_hist,
                                        (p.flags & GNM_ACCUMULATE) != 0, a.kp_hist != nullptr, stream);
    if (rc != GNM_OK) return rc;
  }
  return count_hosts();
}

}  // namespace

namespace gnm {
// Validation and kernel set-up of a classify step without enqueueing it
// (gnm_graph_create runs this outside capture, then captures the step).
int classify_prepare(const gnm_registry *reg, const gnm_records *rec, const uint64_t *window_offsets,
                     uint32_t n_windows, const gnm_params *p, gnm_acc *acc, uint8_t *flags) {
  if (flags && !reg) { set_last_error("NULL argument"); return GNM_E_INVAL; }
  FlagArgs fl{};
  if (flags) fl = FlagArgs{flags, 0, 1, reg->n_sites};
  return classify_impl(reg, rec, window_offsets, n_windows, p, acc, fl, nullptr, false);
}
}  // namespace gnm

extern "C" int gnm_classify_aggregate(const gnm_registry *reg, const gnm_records *rec,
                                      const uint64_t *window_offsets, uint32_t n_windows,
                                      const gnm_params *pp, gnm_acc *acc, hipStream_t stream) {
  return classify_impl(reg, rec, window_offsets, n_windows, pp, acc, FlagArgs{}, stream, true);
}

extern "C" int gnm_classify_flag(const gnm_registry *reg, const gnm_records *rec, const uint64_t *window_offsets,
                                 uint32_t n_windows, const gnm_params *p, gnm_acc *acc, uint64_t threshold_bps,
                                 uint64_t min_bulk_flows, uint8_t *flags, hipStream_t stream) {
  if (!flags) { set_last_error("NULL argument"); return GNM_E_INVAL; }
  if (!reg) { set_last_error("NULL argument"); return GNM_E_INVAL; }
  const FlagArgs fl{flags, threshold_bps, min_bulk_flows > 1 ? min_bulk_flows : 1, reg->n_sites};
  return classify_impl(reg, rec, window_offsets, n_windows, p, acc, fl, stream, true);
}

extern "C" int gnm_flag_suboptimal(const gnm_registry *reg, const gnm_acc *acc, uint32_t n_windows,
                                   uint64_t threshold_bps, uint64_t min_bulk_flows, uint8_t *flags,
                                   hipStream_t stream) {
  if (!reg || !acc || !flags) { set_last_error("NULL argument"); return GNM_E_INVAL; }
  if (reg->host_only) { set_last_error("registry was built host-only"); return GNM_E_UNSUPPORTED; }
  if (n_windows == 0) { set_last_error("n_windows must be >= 1"); return GNM_E_INVAL; }
  int dev = -1;
  hipError_t e0 = hipGetDevice(&dev);
  if (e0 != hipSuccess) return hip_fail(e0, "hipGetDevice");
  if (dev != reg->device) { set_last_error("registry belongs to another device"); return GNM_E_INVAL; }
  const uint64_t items = (uint64_t)n_windows * reg->n_sites;
  const uint64_t need = min_bulk_flows > 1 ? min_bulk_flows : 1;
  const uint64_t blocks = (items + 255) / 256;
  hipLaunchKernelGGL(flag_kernel, dim3((uint32_t)blocks), dim3(256), 0, stream, (const u64 *)acc, n_windows,
                     reg->n_sites, (uint32_t)reg->rows(), threshold_bps, need, flags);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return hip_fail(e, "flag launch");
  return GNM_OK;
}

extern "C" int gnm_median_flags(const gnm_registry *reg, const uint32_t *rate_hist, uint32_t n_windows,
                                uint64_t threshold_bps, uint64_t min_bulk_flows, const uint8_t *prev_flags,
                                uint32_t *median_bucket, uint8_t *flags, hipStream_t stream) {
  if (!reg || !rate_hist || !flags) { set_last_error("NULL argument"); return GNM_E_INVAL; }
  if (reg->host_only) { set_last_error("registry was built host-only"); return GNM_E_UNSUPPORTED; }
  if (n_windows == 0) { set_last_error("n_windows must be >= 1"); return GNM_E_INVAL; }
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
  if (dev != reg->device) { set_last_error("registry belongs to another device"); return GNM_E_INVAL; }
  const uint64_t items = (uint64_t)n_windows * reg->n_sites;
  const uint64_t cap = (uint64_t)device_cus(dev) * 16u;
  const uint64_t blocks = items;
  const uint64_t need = min_bulk_flows > 1 ? min_bulk_flows : 1;
  hipLaunchKernelGGL(median_kernel, dim3((uint32_t)(blocks < cap ? blocks : cap)), dim3(64 * kMedWaves), 0, stream,
                     rate_hist, items, threshold_bps, need, median_bucket, flags);
  e = hipGetLastError();
  if (e != hipSuccess) return hip_fail(e, "median launch");
  hipLaunchKernelGGL(warn_kernel, dim3((reg->n_sites + 255u) / 256u), dim3(256), 0, stream, flags, n_windows,
                     reg->n_sites, prev_flags);
  e = hipGetLastError();
  if (e != hipSuccess) return hip_fail(e, "warn launch");
  return GNM_OK;
}

// ---------------------------------------------------------------- no-allocation variant

namespace gnm {

// Workspace of gnm_classify_flag_static: the per-workgroup partial tables and
// their window tags (and, when they fit, spilled rows or staged histogram
// keys), in a file-scope device array.  Each GPU the library runs on holds
// its own copy until the process ends; every call on that GPU shares it.
// Nothing in it needs to start at zero: each classify workgroup writes its
// whole slot and tag (and its staging counts) before the kernels after it
// read them.
constexpr uint64_t kStaticScratchBytes = 32ull << 20;
__device__ __align__(256) unsigned char scratch[kStaticScratchBytes];

namespace {

// Device address of `scratch` on device dev, which must be the current
// device: looked up once per device with hipGetSymbolAddress (in host code
// the array's name is only a stand-in, never a device address).
int static_scratch(int dev, void **out) {
  static std::mutex mu;
  static void *ptr[64] = {};
  std::lock_guard<std::mutex> g(mu);
  if (dev < 0 || dev >= 64) { set_last_error("device ordinal out of range"); return GNM_E_INVAL; }
  if (!ptr[dev]) {
    void *p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return hip_fail(e, "hipGetSymbolAddress(scratch)");
    if (!p) { set_last_error("hipGetSymbolAddress(scratch) gave NULL"); return GNM_E_HIP; }
    ptr[dev] = p;
  }
  *out = ptr[dev];
  return GNM_OK;
}

}  // namespace
}  // namespace gnm

extern "C" uint64_t gnm_static_scratch_bytes(void) { return kStaticScratchBytes; }

extern "C" int gnm_classify_flag_static(const gnm_registry *reg, const gnm_records *rec,
                                        const uint64_t *window_offsets, uint32_t n_windows, const gnm_params *pp,
                                        gnm_acc *acc, uint64_t threshold_bps, uint64_t min_bulk_flows,
                                        uint8_t *flags, hipStream_t stream) {
  if (!reg || !rec || !acc || !flags) { set_last_error("NULL argument"); return GNM_E_INVAL; }
  if (reg->host_only) { set_last_error("registry was built host-only"); return GNM_E_UNSUPPORTED; }
  if (pp && pp->workspace) {
    set_last_error("gnm_classify_flag_static takes its workspace from the library's static scratch: "
                   "p->workspace must be NULL");
    return GNM_E_INVAL;
  }
  gnm_params p = pp ? *pp : gnm_params_default();
  const uint32_t R = p.records_per_thread ? p.records_per_thread : 4u;
  if (R != 1 && R != 2 && R != 4) { set_last_error("records_per_thread must be 0, 1, 2 or 4"); return GNM_E_INVAL; }
  int dev = -1;
  const hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
  if (dev != reg->device) { set_last_error("registry belongs to another device"); return GNM_E_INVAL; }
  if (reg->acc_in_lds && rec->n > 0) {
    const uint64_t grid = launch_grid(reg, rec->n, R, p.grid_blocks, dev);
    const uint64_t need = partial_bytes(reg, grid);
    if (need > kStaticScratchBytes) {
      set_last_error("the partial tables of " + std::to_string(grid) + " workgroups x " +
                     std::to_string(reg->rows()) + " rows need " + std::to_string(need) +
                     " bytes; the static scratch holds " + std::to_string(kStaticScratchBytes) +
                     " (lower grid_blocks)");
      return GNM_E_INVAL;
    }
  }
  void *ws = nullptr;
  const int rc = static_scratch(dev, &ws);
  if (rc != GNM_OK) return rc;
  p.workspace = ws;
  p.workspace_bytes = kStaticScratchBytes;
  const FlagArgs fl{flags, threshold_bps, min_bulk_flows > 1 ? min_bulk_flows : 1, reg->n_sites};
  return classify_impl(reg, rec, window_offsets, n_windows, &p, acc, fl, stream, true);
}
