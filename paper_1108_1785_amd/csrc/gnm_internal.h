// Internal layout shared by the host registry builder and the HIP kernels.
//
// Longest-prefix-match structure (built once per registry on the host, read
// only on the device; the paper's Catalog Kernel likewise builds a read-only
// table that is rebuilt from scratch on change, §III.B.2).
//
// The registry's answer is a step function over the 32-bit address space: it
// is constant on maximal intervals between prefix starts and ends.  It is laid
// out as a direct-indexed trie whose entries are 32-bit words:
//
//   root[2^root_bits]   indexed by the top root_bits of the address (staged
//                       into LDS by every classify workgroup);
//   nodes[]             inner nodes, each indexed by the next up-to-8 bits;
//   keys[] / vals[]     leaf lists: the sorted interval starts falling in one
//                       trie cell (first entry = the cell's base address) and
//                       the site code of each interval.
//
// Entry encoding (bits 31..30 = kind):
//   LEAF  (2): bits 29..0 = site code (site id, or n_sites = no site);
//   LIST  (0): bits 23..0 = offset into keys/vals, bits 29..24 = count - 1;
//   NODE  (1): bits 29..0 = offset of the child node's first entry in nodes[].
// A node below a cell that leaves `shift` address bits unresolved indexes
// min(8, shift) bits; its children then leave shift - that many.
#pragma once

#include <cstdint>

namespace gnm {

constexpr uint32_t kKindShift = 30;
constexpr uint32_t kKindList = 0u;
constexpr uint32_t kKindNode = 1u;
constexpr uint32_t kKindLeaf = 2u;
constexpr uint32_t kPayloadMask = (1u << 30) - 1u;
constexpr uint32_t kListOffsetBits = 24;
constexpr uint32_t kListOffsetMask = (1u << kListOffsetBits) - 1u;
constexpr uint32_t kListCountMax = 64;  // count - 1 fits 6 bits
constexpr uint32_t kNodeStrideMax = 8;

constexpr uint32_t kMaxLocalRanges = 32;
constexpr uint32_t kMaxSites = 1u << 28;
constexpr uint32_t kLdsMax = 160u * 1024u;

// Accumulator table held in LDS by a classify workgroup, structure of arrays
// of `rows` 64-bit words each.  `cnt` packs flows (low 32 bits) and bulk
// flows (high 32 bits); a workgroup flushes before either can reach 2^32.
enum AccField : uint32_t { kCnt = 0, kBytes, kPackets, kDur, kRateSum, kRateMin, kRateMax, kAccFields };

constexpr uint64_t kMaxRecordsPerFlush = 1ull << 31;

inline uint32_t make_leaf(uint32_t site) { return (kKindLeaf << kKindShift) | site; }
inline uint32_t make_list(uint32_t off, uint32_t count) {
  return (kKindList << kKindShift) | ((count - 1u) << kListOffsetBits) | off;
}
inline uint32_t make_node(uint32_t off) { return (kKindNode << kKindShift) | off; }

}  // namespace gnm
