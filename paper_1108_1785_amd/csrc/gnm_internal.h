// Internal layout shared by the host registry builder and the HIP kernels.
//
// Longest-prefix-match structure (built once per registry on the host, read
// only on the device; the paper's Catalog Kernel likewise builds a read-only
// table that is rebuilt from scratch on change, §III.B.2).
//
// The registry's answer is a step function over the 32-bit address space: it
// is constant on maximal intervals between prefix starts and ends.  It is laid
// out as a direct-indexed trie:
//
//   root[2^root_bits]   64-bit entries indexed by the top root_bits of the
//                       address (staged into LDS by every classify workgroup):
//                       the low word is the trie entry below, the high word
//                       the locality of the cell's 16 equal sub-blocks (bit j
//                       = sub-block j entirely local, bit 16 + j = partly
//                       local, decided by the local ranges);
//   wide[]              inner nodes: arrays of 16-byte entries indexed by the
//                       next address bits (node_bits of them just below the
//                       root, up to 8 further down);
//   lines[]             leaf lines of 64 bytes for cells holding 2..8
//                       intervals: 8 sorted interval starts (the first is the
//                       cell's base address) then their 8 site codes; unused
//                       slots repeat the last interval, so the answer is
//                       sites[number of starts 1..7 that are <= address].
//
// Root trie entry (bits 31..30 = kind, bits 29..0 = payload):
//   LEAF (2): site code (site id, or n_sites = no site);
//   LINE (0): index of the cell's leaf line;
//   NODE (1): index (in 16-byte entries) of the cell's wide node.
// Wide-node entry, four 32-bit words x, y, z, w; kind = y >> 30:
//   LEAF (2): z = site code (only when site codes need more than 16 bits;
//             otherwise a leaf is a QUAD with offsets 0 and four equal codes);
//   LINE (0): z = leaf line index;
//   NODE (1): z = index of the next wide node;
//   QUAD (3): up to 4 intervals of a cell of at most 2^16 addresses (or
//             one interval of any cell):
//             starts as offsets from the cell base k1 = x & 0xFFFF,
//             k2 = x >> 16, k3 = y & 0xFFFF (k0 = 0 implicit), sites as
//             16-bit codes s0 = z & 0xFFFF, s1 = z >> 16, s2 = w & 0xFFFF,
//             s3 = w >> 16; unused slots repeat the last interval.
// A node below a cell that leaves `shift` address bits unresolved indexes
// min(node_bits, shift) bits just below the root and min(8, shift) bits
// further down; its children then leave shift - that many.  Entry 0 of
// wide[] and line 0 of lines[] are dummies (site 0) that are never referenced
// by the trie; lanes with no lookup to do read them instead of branching.

#pragma once

#include <cstdint>

namespace gnm {

constexpr uint32_t kKindShift = 30;
constexpr uint32_t kKindLine = 0u;
constexpr uint32_t kKindNode = 1u;
constexpr uint32_t kKindLeaf = 2u;
constexpr uint32_t kKindQuad = 3u;  // wide-node entries only
constexpr uint32_t kPayloadMask = (1u << 30) - 1u;
constexpr uint32_t kLineKeys = 8;     // interval starts per leaf line
constexpr uint32_t kLineWords = 16;   // 8 starts + 8 site codes = 64 bytes
constexpr uint32_t kNodeStrideMax = 8;    // index bits of wide nodes below the first level
constexpr uint32_t kNodeStride1Max = 12;  // index bits of first-level nodes (just below the root)
// first-level node bytes above which the automatic layout uses 8-bit first-level nodes
constexpr uint64_t kLevel1Bytes = 256ull << 20;
// bytes of wide nodes below the first level above which cells of <=
// list_max intervals there use leaf lines rather than deeper nodes
constexpr uint64_t kDeepNodeBytes = 64ull << 20;

constexpr uint32_t kMaxLocalRanges = 32;
constexpr uint32_t kLocalSubBlocks = 16;  // locality sub-blocks per root cell
constexpr uint32_t kMaxSites = 1u << 28;
constexpr uint32_t kLdsMax = 160u * 1024u;
// LDS that every registry plan leaves free at the top of the 160 KB, for a
// classify workgroup's counters (the per-host staging cursor)
constexpr uint32_t kLdsReserve = 16u;

// Accumulator table held in LDS by a classify workgroup: rows of kAccFields
// 64-bit words (56 bytes, so rows fall on 32 distinct banks).  `cnt` packs
// flows (low 32 bits) and bulk flows (high 32 bits); a workgroup flushes
// before either can reach 2^32.
enum AccField : uint32_t { kCnt = 0, kBytes, kPackets, kDur, kRateSum, kRateMin, kRateMax, kAccFields };

constexpr uint64_t kMaxRecordsPerFlush = 1ull << 31;
constexpr uint32_t kMaxCacheSlots = 4096;  // LDS cache (4-way sets) of a table too large for LDS

inline uint32_t make_leaf(uint32_t site) { return (kKindLeaf << kKindShift) | site; }
inline uint32_t make_line(uint32_t index) { return (kKindLine << kKindShift) | index; }
inline uint32_t make_node(uint32_t off) { return (kKindNode << kKindShift) | off; }

}  // namespace gnm
