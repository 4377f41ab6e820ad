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
//     contiguous slice of the records and stream it with coalesced
//     non-temporal SoA loads, R records per lane in flight;
//   * the top level of the prefix trie (and, when small, the whole trie)
//     staged once per workgroup into LDS;
//   * a per-workgroup accumulator table in LDS (structure of arrays of u64,
//     updated with ds_add/ds_min/ds_max_u64) flushed to the caller's HBM
//     table with 64-bit global atomics once per (workgroup, window);
//   * an exact integer rate: a correctly rounded f64 quotient, which is exact
//     to within one unit for 8000*bytes < 2^53, corrected by one integer
//     multiply-compare; a 64-bit integer long division covers larger byte
//     counts.
// Several windows go through one persistent launch: workgroups cut the
// concatenated records into equal slices and flush at window boundaries.
#include <hip/hip_runtime.h>

#include <cstdint>
#include <mutex>
#include <string>

#include "registry.h"

namespace gnm {

typedef unsigned long long u64;

constexpr uint32_t kThreads = 1024;

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
  const uint64_t *woff;  // NULL: one window [0, n)
  uint32_t n_windows;
  uint32_t rows;
  uint64_t bulk_bytes;
  u64 *acc;  // n_windows * rows * 8 words
  const uint32_t *root, *nodes, *keys, *vals;
  uint32_t root_bits;
  uint32_t n_list;
  uint32_t lds_off_acc, lds_off_keys, lds_off_vals;
  LocalRanges local;
};

// ---------------------------------------------------------------- device helpers

// Membership of ip in the local set (disjoint ranges in kernel arguments, so
// the loop bound and operands are wave-uniform scalars).
__device__ __forceinline__ bool is_local(const LocalRanges &L, uint32_t ip) {
  bool r = false;
  for (uint32_t j = 0; j < L.n; ++j) r |= (ip - L.lo[j]) <= L.span[j];
  return r;
}

// Longest-prefix match: site code of the interval containing ip.
template <bool LISTS_LDS>
__device__ __forceinline__ uint32_t lookup_site(uint32_t ip, const uint32_t *s_root,
                                                const uint32_t *__restrict__ nodes,
                                                const uint32_t *keys, const uint32_t *vals,
                                                uint32_t root_bits) {
  uint32_t shift = 32u - root_bits;
  uint32_t e = s_root[ip >> shift];
  // at most ceil(24 / 8) = 3 node levels lie below a root of >= 8 bits
  for (int depth = 0; depth < 3 && (e >> kKindShift) == kKindNode; ++depth) {
    const uint32_t ns = shift > kNodeStrideMax ? shift - kNodeStrideMax : 0u;
    const uint32_t idx = (ip >> ns) & ((1u << (shift - ns)) - 1u);
    e = nodes[(e & kPayloadMask) + idx];
    shift = ns;
  }
  if ((e >> kKindShift) == kKindLeaf) return e & kPayloadMask;
  const uint32_t off = e & kListOffsetMask;
  uint32_t len = ((e >> kListOffsetBits) & 63u) + 1u;
  uint32_t lo = 0;
  while (len > 1) {  // keys[off] is the cell base <= ip
    const uint32_t half = len >> 1;
    if (keys[off + lo + half] <= ip) lo += half;
    len -= half;
  }
  return vals[off + lo];
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

// ---------------------------------------------------------------- kernels

__global__ void init_acc_kernel(u64 *__restrict__ acc, uint64_t words) {
  const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < words) acc[i] = ((i & 7u) == 6u) ? ~0ull : 0ull;
}

template <bool ACC_LDS>
__device__ __forceinline__ void accumulate(u64 *s_acc, u64 *g_row, uint32_t rows, uint32_t row,
                                           uint64_t b, uint32_t pk, uint32_t dur, bool bulk,
                                           uint64_t rate) {
  if (ACC_LDS) {
    atomicAdd(&s_acc[kCnt * rows + row], 1ull | ((u64)bulk << 32));
    atomicAdd(&s_acc[kBytes * rows + row], (u64)b);
    atomicAdd(&s_acc[kPackets * rows + row], (u64)pk);
    atomicAdd(&s_acc[kDur * rows + row], (u64)dur);
    if (bulk) {
      atomicAdd(&s_acc[kRateSum * rows + row], (u64)rate);
      atomicMin(&s_acc[kRateMin * rows + row], (u64)rate);
      atomicMax(&s_acc[kRateMax * rows + row], (u64)rate);
    }
  } else {
    u64 *g = g_row + (uint64_t)row * 8u;
    atomicAdd(&g[0], 1ull);
    atomicAdd(&g[1], (u64)b);
    atomicAdd(&g[2], (u64)pk);
    atomicAdd(&g[3], (u64)dur);
    if (bulk) {
      atomicAdd(&g[4], 1ull);
      atomicAdd(&g[5], (u64)rate);
      atomicMin(&g[6], (u64)rate);
      atomicMax(&g[7], (u64)rate);
    }
  }
}

// Flush the workgroup's LDS table into window table g (rows x 8 words) and
// reset it.  Only touched rows, and only non-empty bulk fields, are sent.
__device__ __forceinline__ void flush_acc(u64 *s_acc, u64 *__restrict__ g, uint32_t rows) {
  __syncthreads();
  for (uint32_t r = threadIdx.x; r < rows; r += blockDim.x) {
    const u64 cnt = s_acc[kCnt * rows + r];
    if (cnt == 0) continue;
    u64 *o = g + (uint64_t)r * 8u;
    atomicAdd(&o[0], cnt & 0xFFFFFFFFull);
    atomicAdd(&o[1], s_acc[kBytes * rows + r]);
    atomicAdd(&o[2], s_acc[kPackets * rows + r]);
    atomicAdd(&o[3], s_acc[kDur * rows + r]);
    const u64 nb = cnt >> 32;
    if (nb) {
      atomicAdd(&o[4], nb);
      atomicAdd(&o[5], s_acc[kRateSum * rows + r]);
      atomicMin(&o[6], s_acc[kRateMin * rows + r]);
      atomicMax(&o[7], s_acc[kRateMax * rows + r]);
    }
    s_acc[kCnt * rows + r] = 0;
    s_acc[kBytes * rows + r] = 0;
    s_acc[kPackets * rows + r] = 0;
    s_acc[kDur * rows + r] = 0;
    s_acc[kRateSum * rows + r] = 0;
    s_acc[kRateMin * rows + r] = ~0ull;
    s_acc[kRateMax * rows + r] = 0;
  }
  __syncthreads();
}

template <int R, bool LISTS_LDS, bool ACC_LDS>
__global__ __launch_bounds__(kThreads) void classify_kernel(const ClassifyArgs a) {
  extern __shared__ __align__(16) unsigned char lds[];
  uint32_t *s_root = (uint32_t *)lds;
  u64 *s_acc = (u64 *)(lds + a.lds_off_acc);
  uint32_t *s_keys = (uint32_t *)(lds + a.lds_off_keys);
  uint32_t *s_vals = (uint32_t *)(lds + a.lds_off_vals);
  const uint32_t tid = threadIdx.x;
  const uint32_t rows = a.rows;

  // stage the trie top (and the leaf lists when they fit) into LDS
  const uint32_t nroot = 1u << a.root_bits;
  for (uint32_t i = tid; i < nroot; i += kThreads) s_root[i] = a.root[i];
  if (LISTS_LDS) {
    for (uint32_t i = tid; i < a.n_list; i += kThreads) {
      s_keys[i] = a.keys[i];
      s_vals[i] = a.vals[i];
    }
  }
  if (ACC_LDS) {
    for (uint32_t r = tid; r < rows; r += kThreads) {
      for (uint32_t f = 0; f < kAccFields; ++f) s_acc[f * rows + r] = (f == kRateMin) ? ~0ull : 0ull;
    }
  }
  __syncthreads();
  const uint32_t *keys = LISTS_LDS ? s_keys : a.keys;
  const uint32_t *vals = LISTS_LDS ? s_vals : a.vals;
  const uint32_t nodir = rows - 1u;

  // this workgroup's balanced slice of all records
  const uint64_t lo = (uint64_t)blockIdx.x * a.n / gridDim.x;
  const uint64_t hi = (uint64_t)(blockIdx.x + 1) * a.n / gridDim.x;
  uint64_t i = lo;
  while (i < hi) {
    uint64_t wend;
    const uint32_t w = window_of(a, i, wend);
    uint64_t seg_end = wend < hi ? wend : hi;
    if (seg_end - i > kMaxRecordsPerFlush) seg_end = i + kMaxRecordsPerFlush;
    u64 *g_tab = a.acc + (uint64_t)w * rows * 8u;

    for (uint64_t base = i; base < seg_end; base += (uint64_t)kThreads * R) {
      uint32_t s[R], d[R], pk[R], f[R], l[R];
      uint64_t b[R];
      bool v[R];
#pragma unroll
      for (int k = 0; k < R; ++k) {
        const uint64_t idx = base + (uint64_t)k * kThreads + tid;
        v[k] = idx < seg_end;
        if (v[k]) {
          s[k] = ldg_nt(a.src + idx);
          d[k] = ldg_nt(a.dst + idx);
          b[k] = ldg_nt(a.bytes + idx);
          pk[k] = ldg_nt(a.packets + idx);
          f[k] = ldg_nt(a.first + idx);
          l[k] = ldg_nt(a.last + idx);
        }
      }
#pragma unroll
      for (int k = 0; k < R; ++k) {
        if (!v[k]) continue;
        const bool ls = is_local(a.local, s[k]);
        const bool ld = is_local(a.local, d[k]);
        uint32_t row = nodir;
        if (ls != ld) {
          const uint32_t remote = ld ? s[k] : d[k];
          const uint32_t site = lookup_site<LISTS_LDS>(remote, s_root, a.nodes, keys, vals, a.root_bits);
          row = 2u * site + (ld ? 0u : 1u);
        }
        const uint32_t dur = l[k] - f[k];
        const bool bulk = b[k] > a.bulk_bytes && dur > 0u;
        uint64_t rate = 0;
        if (bulk) rate = rate_bps(b[k], dur);
        accumulate<ACC_LDS>(s_acc, g_tab, rows, row, b[k], pk[k], dur, bulk, rate);
      }
    }
    if (ACC_LDS) flush_acc(s_acc, g_tab, rows);
    i = seg_end;
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

// ---------------------------------------------------------------- launch plumbing

namespace {

int hip_fail(hipError_t e, const char *where) {
  set_last_error(std::string(where) + ": " + hipGetErrorString(e));
  return GNM_E_HIP;
}

struct DeviceFacts {
  int cus = 0;
};

DeviceFacts device_facts(int dev) {
  static std::mutex mu;
  static DeviceFacts facts[64];
  std::lock_guard<std::mutex> g(mu);
  if (dev < 0 || dev >= 64) return DeviceFacts{256};
  if (facts[dev].cus == 0) {
    int cus = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus <= 0)
      cus = 256;
    facts[dev].cus = cus;
  }
  return facts[dev];
}

typedef void (*KernelFn)(const ClassifyArgs);

template <int R, bool L, bool A>
KernelFn pick3() { return classify_kernel<R, L, A>; }

template <int R>
KernelFn pick2(bool lists, bool acc) {
  if (lists) return acc ? pick3<R, true, true>() : pick3<R, true, false>();
  return acc ? pick3<R, false, true>() : pick3<R, false, false>();
}

KernelFn pick(int r, bool lists, bool acc) {
  switch (r) {
    case 1: return pick2<1>(lists, acc);
    case 2: return pick2<2>(lists, acc);
    case 4: return pick2<4>(lists, acc);
    default: return pick2<8>(lists, acc);
  }
}

// Allow every kernel variant the full 160 KB of LDS, once per device.
hipError_t allow_lds(KernelFn fn, int dev) {
  static std::mutex mu;
  static bool done[64][32] = {};
  int slot = -1;
  for (int r = 0, k = 0; r < 4; ++r)
    for (int l = 0; l < 2; ++l)
      for (int c = 0; c < 2; ++c, ++k)
        if (fn == pick((1 << r), l, c)) slot = k;
  std::lock_guard<std::mutex> g(mu);
  if (dev >= 0 && dev < 64 && slot >= 0 && done[dev][slot]) return hipSuccess;
  hipError_t e = hipFuncSetAttribute((const void *)fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)kLdsMax);
  if (e == hipSuccess && dev >= 0 && dev < 64 && slot >= 0) done[dev][slot] = true;
  return e;
}

}  // namespace
}  // namespace gnm

using namespace gnm;

extern "C" gnm_params gnm_params_default(void) {
  gnm_params p{};
  p.bulk_bytes = 1000000ull;
  return p;
}

extern "C" int gnm_classify_aggregate(const gnm_registry *reg, const gnm_records *rec,
                                      const uint64_t *window_offsets, uint32_t n_windows,
                                      const gnm_params *pp, gnm_acc *acc, hipStream_t stream) {
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
  const uint32_t R = p.records_per_thread ? p.records_per_thread : 4u;
  if (R != 1 && R != 2 && R != 4 && R != 8) { set_last_error("records_per_thread must be 0,1,2,4,8"); return GNM_E_INVAL; }
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
  if (dev != reg->device) { set_last_error("registry belongs to another device"); return GNM_E_INVAL; }

  const uint64_t rows = reg->rows();
  if (!(p.flags & GNM_ACCUMULATE)) {
    const uint64_t words = (uint64_t)n_windows * rows * 8u;
    const uint64_t blocks = (words + 255) / 256;
    hipLaunchKernelGGL(init_acc_kernel, dim3((uint32_t)blocks), dim3(256), 0, stream, (u64 *)acc, words);
    e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(e, "init launch");
  }
  if (rec->n == 0) return GNM_OK;

  ClassifyArgs a{};
  a.src = rec->src_ip; a.dst = rec->dst_ip; a.bytes = rec->bytes; a.packets = rec->packets;
  a.first = rec->first_ms; a.last = rec->last_ms; a.n = rec->n;
  a.woff = window_offsets; a.n_windows = n_windows; a.rows = (uint32_t)rows;
  a.bulk_bytes = p.bulk_bytes; a.acc = (u64 *)acc;
  a.root = reg->d_root; a.nodes = reg->d_nodes; a.keys = reg->d_keys; a.vals = reg->d_vals;
  a.root_bits = reg->root_bits; a.n_list = (uint32_t)reg->keys.size();
  a.lds_off_acc = reg->lds_off_acc; a.lds_off_keys = reg->lds_off_keys; a.lds_off_vals = reg->lds_off_vals;
  a.local.n = (uint32_t)reg->local_lo.size();
  for (uint32_t j = 0; j < a.local.n; ++j) {
    a.local.lo[j] = reg->local_lo[j];
    a.local.span[j] = reg->local_hi[j] - reg->local_lo[j];
  }

  const DeviceFacts df = device_facts(dev);
  const uint32_t per_cu = reg->lds_bytes <= kLdsMax / 2 ? 2u : 1u;
  const uint64_t resident = (uint64_t)df.cus * per_cu;
  const uint64_t tiles = (rec->n + (uint64_t)kThreads * R - 1) / ((uint64_t)kThreads * R);
  uint64_t grid = p.grid_blocks ? p.grid_blocks : (tiles < resident ? tiles : resident);
  if (grid == 0) grid = 1;
  if (grid > 65535u * 16u) grid = 65535u * 16u;

  KernelFn fn = pick((int)R, reg->lists_in_lds, reg->acc_in_lds);
  e = allow_lds(fn, dev);
  if (e != hipSuccess) return hip_fail(e, "hipFuncSetAttribute");
  hipLaunchKernelGGL(fn, dim3((uint32_t)grid), dim3(kThreads), reg->lds_bytes, stream, a);
  e = hipGetLastError();
  if (e != hipSuccess) return hip_fail(e, "classify launch");
  return GNM_OK;
}

extern "C" int gnm_flag_suboptimal(const gnm_registry *reg, const gnm_acc *acc, uint32_t n_windows,
                                   uint64_t threshold_bps, uint64_t min_bulk_flows, uint8_t *flags,
                                   hipStream_t stream) {
  if (!reg || !acc || !flags) { set_last_error("NULL argument"); return GNM_E_INVAL; }
  if (reg->host_only) { set_last_error("registry was built host-only"); return GNM_E_UNSUPPORTED; }
  if (n_windows == 0) { set_last_error("n_windows must be >= 1"); return GNM_E_INVAL; }
  const uint64_t items = (uint64_t)n_windows * reg->n_sites;
  const uint64_t need = min_bulk_flows > 1 ? min_bulk_flows : 1;
  const uint64_t blocks = (items + 255) / 256;
  hipLaunchKernelGGL(flag_kernel, dim3((uint32_t)blocks), dim3(256), 0, stream, (const u64 *)acc, n_windows,
                     reg->n_sites, (uint32_t)reg->rows(), threshold_bps, need, flags);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return hip_fail(e, "flag launch");
  return GNM_OK;
}
