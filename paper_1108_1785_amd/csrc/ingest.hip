// gfx950 kernels of the NetFlow v5 decode step and its C-ABI launcher.
//
// The paper's border routers export NetFlow V5 datagrams over UDP (48-byte
// records, at most 30 per datagram) and a receiver thread stores the records
// in a host buffer (§III.B.1, FlowData Receiver Thread; §IV.A.3).  Here the
// datagrams, as received back to back, are decoded on the GPU into the
// structure-of-arrays window that the classify path reads:
//   1. v5_count_kernel: one lane per datagram checks its header and span and
//      writes the number of records it carries (0 = rejected);
//   2. v5_reduce_kernel, v5_top_kernel, v5_down_kernel: exclusive prefix
//      sums of the counts (per-block totals, a one-block scan of those, then
//      per-block rescans) give each datagram's first output record, and the
//      totals of records and rejected datagrams;
//   3. v5_decode_kernel: one half-wave per datagram, lane k decoding record
//      k (eight of its twelve big-endian words, with 8-byte loads when the
//      record is 8-byte aligned, as back-to-back datagrams are) and writing
//      each field with coalesced stores.
// Field layout (public NetFlow version 5 export format, big-endian): header
// of 24 bytes starting with version u16 and count u16; records of 48 bytes:
// srcaddr, dstaddr, nexthop u32; input, output u16; dPkts, dOctets, First,
// Last u32; srcport, dstport u16; pad1, tcp_flags, prot, tos u8; src_as,
// dst_as u16; src_mask, dst_mask u8; pad2 u16.
#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>

#include "registry.h"

namespace gnm {
namespace {

typedef unsigned long long u64;

constexpr uint32_t kV5Header = 24;
constexpr uint32_t kV5Record = 48;
constexpr uint32_t kV5MaxRecords = 30;
constexpr uint32_t kScanThreads = 1024;  // threads of the scan kernels
constexpr uint32_t kScanBlocks = 1024;   // most blocks of the reduce and down-sweep passes
constexpr uint32_t kDecodeThreads = 256;                  // decode workgroup
constexpr uint32_t kDecodeSlots = kDecodeThreads / 32u;   // one datagram per half-wave

struct V5Out {
  uint32_t *src, *dst;
  uint16_t *sport, *dport;  // may be NULL
  uint8_t *proto;           // may be NULL
  uint64_t *bytes;
  uint32_t *packets, *first, *last;
  uint64_t capacity;
};

__device__ __forceinline__ uint32_t be32(uint32_t x) { return __builtin_bswap32(x); }

// Records datagram d carries: its span [off[d], off[d+1]) lies in the
// buffer, starts at a multiple of 4, holds the header, version 5, count
// 1..30, and room for count records.  0 = rejected.
__global__ void v5_count_kernel(const uint8_t *__restrict__ buf, uint64_t buf_bytes,
                                const uint64_t *__restrict__ off, uint64_t n, uint32_t *__restrict__ cnt) {
  const uint64_t d = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (d >= n) return;
  const uint64_t s = off[d], e = off[d + 1];
  uint32_t c = 0;
  if (e >= s && e <= buf_bytes && e - s >= kV5Header && (s & 3u) == 0u) {
    const uint32_t h = be32(*(const uint32_t *)(buf + s));
    const uint32_t version = h >> 16, count = h & 0xFFFFu;
    if (version == 5u && count >= 1u && count <= kV5MaxRecords &&
        e - s >= kV5Header + (uint64_t)kV5Record * count)
      c = count;
  }
  cnt[d] = c;
}

__device__ __forceinline__ u64 wave_reduce(u64 x) {
#pragma unroll
  for (uint32_t o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o, 64);
  return x;
}

// Inclusive scan over a 1024-lane block; `total` receives the block's sum.
__device__ __forceinline__ u64 block_scan(u64 x, u64 &total) {
  __shared__ u64 wsum[kScanThreads / 64];
  const uint32_t lane = threadIdx.x % 64u, wave = threadIdx.x / 64u;
#pragma unroll
  for (uint32_t o = 1; o < 64; o <<= 1) {
    const u64 y = __shfl_up(x, o, 64);
    if (lane >= o) x += y;
  }
  __syncthreads();  // earlier readers of wsum are done
  if (lane == 63u) wsum[wave] = x;
  __syncthreads();
  u64 before = 0, t = 0;
#pragma unroll
  for (uint32_t v = 0; v < kScanThreads / 64; ++v) {
    if (v < wave) before += wsum[v];
    t += wsum[v];
  }
  total = t;
  return x + before;
}

// Block b's chunk [b*n/G, (b+1)*n/G): total records (sums[b]) and rejected
// datagrams (sums[G + b]).
__global__ __launch_bounds__(kScanThreads) void v5_reduce_kernel(const uint32_t *__restrict__ cnt, uint64_t n,
                                                                 u64 *__restrict__ sums) {
  __shared__ u64 part[2][kScanThreads / 64];
  const uint64_t G = gridDim.x, b = blockIdx.x;
  const uint64_t lo = b * n / G, hi = (b + 1) * n / G;
  u64 s = 0, z = 0;
  for (uint64_t i = lo + threadIdx.x; i < hi; i += kScanThreads) {
    const uint32_t c = cnt[i];
    s += c;
    z += c == 0u;
  }
  s = wave_reduce(s);
  z = wave_reduce(z);
  const uint32_t lane = threadIdx.x % 64u, wave = threadIdx.x / 64u;
  if (lane == 0u) {
    part[0][wave] = s;
    part[1][wave] = z;
  }
  __syncthreads();
  if (threadIdx.x == 0u) {
    u64 ts = 0, tz = 0;
    for (uint32_t v = 0; v < kScanThreads / 64; ++v) {
      ts += part[0][v];
      tz += part[1][v];
    }
    sums[b] = ts;
    sums[G + b] = tz;
  }
}

// One block: sums[0..G) become exclusive prefix sums; the totals go out.
__global__ __launch_bounds__(kScanThreads) void v5_top_kernel(u64 *__restrict__ sums, uint32_t G,
                                                              u64 *__restrict__ n_records,
                                                              u64 *__restrict__ n_rejected) {
  const uint32_t t = threadIdx.x;
  const u64 v = t < G ? sums[t] : 0u;
  const u64 z = t < G ? sums[G + t] : 0u;
  u64 total, rejected;
  const u64 incl = block_scan(v, total);
  block_scan(z, rejected);
  if (t < G) sums[t] = incl - v;
  if (t == 0u) {
    *n_records = total;
    *n_rejected = rejected;
  }
}

// Block b rescans its chunk from its exclusive offset: base[i] = first
// output record of datagram i.
__global__ __launch_bounds__(kScanThreads) void v5_down_kernel(const uint32_t *__restrict__ cnt, uint64_t n,
                                                               const u64 *__restrict__ sums,
                                                               u64 *__restrict__ base) {
  const uint64_t G = gridDim.x, b = blockIdx.x;
  const uint64_t lo = b * n / G, hi = (b + 1) * n / G;
  u64 running = sums[b];
  for (uint64_t start = lo; start < hi; start += kScanThreads) {
    const uint64_t i = start + threadIdx.x;
    const u64 c = i < hi ? cnt[i] : 0u;
    u64 total;
    const u64 incl = block_scan(c, total);
    if (i < hi) base[i] = running + incl - c;
    running += total;
  }
}

// One half-wave per datagram; lane k < count of the half decodes record k
// of an accepted datagram and writes it at base[d] + k (records past the
// capacity are dropped; the reported total still counts them).
__global__ __launch_bounds__(kDecodeThreads) void v5_decode_kernel(const uint8_t *__restrict__ buf,
                                                                   const uint64_t *__restrict__ off, uint64_t n,
                                                                   const uint32_t *__restrict__ cnt,
                                                                   const u64 *__restrict__ base, V5Out o) {
  const uint32_t k = threadIdx.x % 32u, slot = threadIdx.x / 32u;
  for (uint64_t d = (uint64_t)blockIdx.x * kDecodeSlots + slot; d < n; d += (uint64_t)gridDim.x * kDecodeSlots) {
    // the three per-datagram loads issue together (the offset and base of a
    // rejected datagram are read but unused)
    const uint32_t c = cnt[d];
    const uint64_t start = off[d], first = base[d];
    if (k >= c) continue;
    const uint8_t *rp = buf + start + kV5Header + (uint64_t)kV5Record * k;
    uint32_t w0, w1, w4, w5, w6, w7, w8, w9;
    if (((uintptr_t)rp & 7u) == 0u) {
      const uint64_t *q = (const uint64_t *)rp;
      const uint64_t a = __builtin_nontemporal_load(q), b = __builtin_nontemporal_load(q + 2),
                     e = __builtin_nontemporal_load(q + 3), f = __builtin_nontemporal_load(q + 4);
      w0 = (uint32_t)a; w1 = (uint32_t)(a >> 32);
      w4 = (uint32_t)b; w5 = (uint32_t)(b >> 32);
      w6 = (uint32_t)e; w7 = (uint32_t)(e >> 32);
      w8 = (uint32_t)f; w9 = (uint32_t)(f >> 32);
    } else {
      const uint32_t *r = (const uint32_t *)rp;
      w0 = r[0]; w1 = r[1]; w4 = r[4]; w5 = r[5]; w6 = r[6]; w7 = r[7]; w8 = r[8]; w9 = r[9];
    }
    const uint64_t i = first + k;
    if (i >= o.capacity) continue;
    o.src[i] = be32(w0);
    o.dst[i] = be32(w1);
    o.packets[i] = be32(w4);
    o.bytes[i] = be32(w5);
    o.first[i] = be32(w6);
    o.last[i] = be32(w7);
    const uint32_t ports = be32(w8);
    if (o.sport) o.sport[i] = (uint16_t)(ports >> 16);
    if (o.dport) o.dport[i] = (uint16_t)(ports & 0xFFFFu);
    if (o.proto) o.proto[i] = (uint8_t)(w9 >> 16);  // bytes pad1, tcp_flags, prot, tos: prot is the third
  }
}

int fail(hipError_t e, const char *where) {
  set_last_error(std::string(where) + ": " + hipGetErrorString(e));
  return GNM_E_HIP;
}

uint64_t align256(uint64_t x) { return (x + 255u) & ~255ull; }

}  // namespace
}  // namespace gnm

using namespace gnm;

extern "C" uint64_t gnm_netflow_v5_workspace_bytes(uint64_t n_datagrams) {
  return align256(n_datagrams * 4u) + align256(n_datagrams * 8u) + 2u * kScanBlocks * 8u;
}

extern "C" int gnm_netflow_v5_decode(const uint8_t *datagrams, uint64_t buf_bytes, const uint64_t *offsets,
                                     uint64_t n_datagrams, void *workspace, uint64_t workspace_bytes,
                                     const gnm_records_out *out, uint64_t *n_records, uint64_t *n_rejected,
                                     hipStream_t stream) {
  if (!offsets || !out || !n_records || !n_rejected || !workspace) {
    set_last_error("NULL argument");
    return GNM_E_INVAL;
  }
  if (n_datagrams > 0 && !datagrams) { set_last_error("NULL datagram buffer"); return GNM_E_INVAL; }
  if ((uintptr_t)datagrams & 3u) { set_last_error("datagram buffer not 4-byte aligned"); return GNM_E_INVAL; }
  if (((uintptr_t)offsets | (uintptr_t)n_records | (uintptr_t)n_rejected) & 7u) {
    set_last_error("offsets or counters not 8-byte aligned");
    return GNM_E_INVAL;
  }
  if (n_datagrams > (1ull << 31)) { set_last_error("more than 2^31 datagrams"); return GNM_E_INVAL; }
  if (!out->src_ip || !out->dst_ip || !out->bytes || !out->packets || !out->first_ms || !out->last_ms) {
    set_last_error("NULL output field");
    return GNM_E_INVAL;
  }
  if (workspace_bytes < gnm_netflow_v5_workspace_bytes(n_datagrams) || ((uintptr_t)workspace & 255u)) {
    set_last_error("workspace too small or not 256-byte aligned");
    return GNM_E_INVAL;
  }
  uint8_t *ws = (uint8_t *)workspace;
  uint32_t *cnt = (uint32_t *)ws;
  u64 *base = (u64 *)(ws + align256(n_datagrams * 4u));
  u64 *sums = (u64 *)(ws + align256(n_datagrams * 4u) + align256(n_datagrams * 8u));
  const uint64_t n = n_datagrams;
  const uint32_t G = (uint32_t)(n == 0 ? 0 : ((n + kScanThreads - 1) / kScanThreads < kScanBlocks
                                                  ? (n + kScanThreads - 1) / kScanThreads
                                                  : kScanBlocks));
  hipError_t e;
  if (n > 0) {
    hipLaunchKernelGGL(v5_count_kernel, dim3((uint32_t)((n + 255) / 256)), dim3(256), 0, stream, datagrams,
                       buf_bytes, offsets, n, cnt);
    if ((e = hipGetLastError()) != hipSuccess) return fail(e, "count launch");
    hipLaunchKernelGGL(v5_reduce_kernel, dim3(G), dim3(kScanThreads), 0, stream, (const uint32_t *)cnt, n, sums);
    if ((e = hipGetLastError()) != hipSuccess) return fail(e, "reduce launch");
  }
  hipLaunchKernelGGL(v5_top_kernel, dim3(1), dim3(kScanThreads), 0, stream, sums, G, (u64 *)n_records,
                     (u64 *)n_rejected);
  if ((e = hipGetLastError()) != hipSuccess) return fail(e, "scan launch");
  if (n == 0) return GNM_OK;
  hipLaunchKernelGGL(v5_down_kernel, dim3(G), dim3(kScanThreads), 0, stream, (const uint32_t *)cnt, n,
                     (const u64 *)sums, base);
  if ((e = hipGetLastError()) != hipSuccess) return fail(e, "scan launch");
  V5Out o{out->src_ip, out->dst_ip, out->src_port, out->dst_port, out->proto, out->bytes,
          out->packets, out->first_ms, out->last_ms, out->capacity};
  int dev = 0, cus = 256;
  if (hipGetDevice(&dev) == hipSuccess) {
    int c = 0;
    if (hipDeviceGetAttribute(&c, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && c > 0) cus = c;
  }
  const uint64_t want = (n + kDecodeSlots - 1) / kDecodeSlots, cap = (uint64_t)cus * 32u;
  hipLaunchKernelGGL(v5_decode_kernel, dim3((uint32_t)(want < cap ? want : cap)), dim3(kDecodeThreads), 0,
                     stream, datagrams, offsets, n, (const uint32_t *)cnt, (const u64 *)base, o);
  if ((e = hipGetLastError()) != hipSuccess) return fail(e, "decode launch");
  return GNM_OK;
}
