// Host-side registry builder: validation, normalisation, longest-prefix-match
// resolution into disjoint address intervals, and the direct-indexed trie
// layout uploaded to the device.
//
// §III.B.1 (Site Registration Thread): registered subnets identify transfers
// between the local site and its collaboration sites.  §III.B.2 (Catalog
// Kernel): the lookup structure is read-only on the device and rebuilt from
// scratch on any change.  The paper expands every subnet into /24 hash
// entries; here any length /0../32 is supported and overlapping prefixes
// resolve to the longest one.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "registry.h"

namespace gnm {

thread_local std::string g_last_error;
void set_last_error(const std::string &s) { g_last_error = s; }

namespace {

inline uint32_t mask_of(uint32_t len) { return len == 0 ? 0u : (0xFFFFFFFFu << (32u - len)); }

struct Pfx {
  uint32_t addr, len, site;
};

// Sorted by start address, then shorter (enclosing) first.
bool pfx_less(const Pfx &a, const Pfx &b) {
  if (a.addr != b.addr) return a.addr < b.addr;
  if (a.len != b.len) return a.len < b.len;
  return a.site < b.site;
}

struct Interval {
  uint32_t start;
  uint32_t site;
};

// Append an interval [x, ...) answering `site`, keeping the list minimal:
// a zero-length predecessor is replaced and equal neighbours are merged.
void emit(std::vector<Interval> &out, uint64_t x, uint32_t site) {
  if (!out.empty() && out.back().start == (uint32_t)x) {
    out.back().site = site;
    if (out.size() >= 2 && out[out.size() - 2].site == site) out.pop_back();
    return;
  }
  if (!out.empty() && out.back().site == site) return;
  out.push_back({(uint32_t)x, site});
}

// Resolve prefixes (normalised, distinct, sorted by pfx_less) into the
// maximal intervals of the longest-match function.  Prefixes are either
// nested or disjoint, so a stack of enclosing prefixes gives the answer of
// every address between consecutive prefix boundaries.
std::vector<Interval> resolve(const std::vector<Pfx> &p, uint32_t none) {
  struct Open {
    uint64_t end;  // inclusive
    uint32_t site;
  };
  std::vector<Interval> out;
  std::vector<Open> stack;
  uint64_t cur = 0;  // first address not yet emitted
  for (const Pfx &q : p) {
    const uint64_t start = q.addr;
    while (!stack.empty() && stack.back().end < start) {
      const Open top = stack.back();
      stack.pop_back();
      if (cur <= top.end) {
        emit(out, cur, top.site);
        cur = top.end + 1;
      }
    }
    if (cur < start) {
      emit(out, cur, stack.empty() ? none : stack.back().site);
      cur = start;
    }
    stack.push_back({start + ((uint64_t)1 << (32 - q.len)) - 1, q.site});
  }
  while (!stack.empty()) {
    const Open top = stack.back();
    stack.pop_back();
    if (cur <= top.end) {
      emit(out, cur, top.site);
      cur = top.end + 1;
    }
  }
  if (cur <= 0xFFFFFFFFull) emit(out, cur, none);
  if (out.empty() || out.front().start != 0) out.insert(out.begin(), {0u, none});
  return out;
}

// index of the interval containing address a (intervals sorted, first starts at 0)
size_t find_index(const std::vector<Interval> &v, uint64_t a) {
  size_t lo = 0, hi = v.size();
  while (hi - lo > 1) {
    const size_t mid = (lo + hi) / 2;
    if ((uint64_t)v[mid].start <= a) lo = mid; else hi = mid;
  }
  return lo;
}

struct Layout {
  const std::vector<Interval> *iv;
  uint32_t list_max;
  bool root_lines;  // root cells with <= list_max intervals become leaf lines
  bool quad_ok;     // site codes fit 16 bits
  bool deep;        // cells of 5..list_max intervals get deeper nodes, not lines
  uint32_t stride1; // index bits of first-level nodes
  std::vector<uint32_t> wide, lines;
  uint64_t n_wide_nodes = 0;
  uint64_t level1_entries = 0, deeper_entries = 0;
  bool overflow = false;

  // index of the interval containing address a
  size_t find(uint64_t a) const {
    const auto &v = *iv;
    size_t lo = 0, hi = v.size();  // v[0].start == 0 <= a
    while (hi - lo > 1) {
      size_t mid = (lo + hi) / 2;
      if ((uint64_t)v[mid].start <= a) lo = mid; else hi = mid;
    }
    return lo;
  }

  // the intervals overlapping cell [lo, lo + 2^shift): first index, count
  size_t span(uint64_t lo, uint32_t shift, size_t &count) const {
    const size_t i0 = find(lo), i1 = find(lo + ((uint64_t)1 << shift) - 1);
    count = i1 - i0 + 1;
    return i0;
  }

  uint32_t add_line(uint64_t lo, size_t i0, size_t count) {
    const size_t index = lines.size() / kLineWords;
    if (index > kPayloadMask) { overflow = true; return 0; }
    const auto &v = *iv;
    uint32_t key[kLineKeys], site[kLineKeys];
    for (uint32_t j = 0; j < kLineKeys; ++j) {
      const size_t src = i0 + (j < count ? j : count - 1);
      key[j] = j == 0 ? (uint32_t)lo : v[src].start;
      site[j] = v[src].site;
    }
    lines.insert(lines.end(), key, key + kLineKeys);
    lines.insert(lines.end(), site, site + kLineKeys);
    return (uint32_t)index;
  }

  // 32-bit root entry for the cell [lo, lo + 2^shift)
  uint32_t root_cell(uint64_t lo, uint32_t shift) {
    size_t count;
    const size_t i0 = span(lo, shift, count);
    if (count == 1) return make_leaf((*iv)[i0].site);
    if (root_lines && count <= list_max) return make_line(add_line(lo, i0, count));
    return make_node(wide_node(lo, shift, 0));
  }

  // wide node for the cell [lo, lo + 2^shift): returns its first entry index
  uint32_t wide_node(uint64_t lo, uint32_t shift, uint32_t depth) {
    const uint32_t smax = depth == 0 ? stride1 : kNodeStrideMax;
    const uint32_t ns = shift > smax ? shift - smax : 0u;
    const uint32_t stride = shift - ns;
    const size_t base = wide.size() / 4;
    if (base + ((size_t)1 << stride) > kPayloadMask) { overflow = true; return 0; }
    wide.resize(wide.size() + 4 * ((size_t)1 << stride));
    ++n_wide_nodes;
    (depth == 0 ? level1_entries : deeper_entries) += (uint64_t)1 << stride;
    for (uint64_t c = 0; c < ((uint64_t)1 << stride); ++c) {
      uint32_t q[4];
      wide_entry(lo + (c << ns), ns, depth, q);
      for (int j = 0; j < 4; ++j) wide[(base + c) * 4 + j] = q[j];
    }
    return (uint32_t)base;
  }

  // 16-byte wide-node entry for the cell [lo, lo + 2^shift)
  void wide_entry(uint64_t lo, uint32_t shift, uint32_t depth, uint32_t q[4]) {
    size_t count;
    const size_t i0 = span(lo, shift, count);
    const auto &v = *iv;
    q[0] = q[1] = q[2] = q[3] = 0;
    if (count == 1 && quad_ok) {
      // a leaf as a QUAD entry: split offsets 0, four equal site codes (the
      // device decodes every QUAD the same way, whatever the offset)
      const uint32_t st = v[i0].site;
      q[1] = kKindQuad << kKindShift;
      q[2] = q[3] = st | (st << 16);
    } else if (count == 1) {
      q[1] = kKindLeaf << kKindShift;
      q[2] = v[i0].site;
    } else if (count <= 4 && quad_ok && shift <= 16) {
      uint32_t k[4], st[4];
      for (uint32_t j = 0; j < 4; ++j) {
        const size_t src = i0 + (j < count ? j : count - 1);
        k[j] = j == 0 ? 0u : (uint32_t)(v[src].start - lo);
        st[j] = v[src].site;
      }
      q[0] = k[1] | (k[2] << 16);
      q[1] = k[3] | (kKindQuad << kKindShift);
      q[2] = st[0] | (st[1] << 16);
      q[3] = st[2] | (st[3] << 16);
    } else if (count <= list_max && (!quad_ok || !deep)) {
      // a leaf line (32-bit site codes): when 16-bit codes do not fit, or
      // when deeper nodes everywhere would outgrow the caches
      q[1] = kKindLine << kKindShift;
      q[2] = add_line(lo, i0, count);
    } else {
      // a deeper wide node, whose entries are again mostly leaves or quads
      const uint32_t child = wide_node(lo, shift, depth + 1);
      q[1] = kKindNode << kKindShift;
      q[2] = child;
    }
  }
};

int fail(int code, const char *msg) {
  set_last_error(msg);
  return code;
}

}  // namespace

uint32_t line_site(const gnm_registry *r, uint32_t index, uint32_t ip) {
  const uint32_t *line = &r->lines[(size_t)index * kLineWords];
  uint32_t pos = 0;
  for (uint32_t j = 1; j < kLineKeys; ++j) pos += line[j] <= ip ? 1u : 0u;
  return line[kLineKeys + pos];
}

// Walk of the host copy; mirrors the device walk in kernels.hip.
uint32_t host_lookup(const gnm_registry *r, uint32_t ip) {
  uint32_t shift = 32u - r->root_bits;
  const uint32_t e = r->root[ip >> shift];
  if ((e >> kKindShift) == kKindLeaf) return e & kPayloadMask;
  if ((e >> kKindShift) == kKindLine) return line_site(r, e & kPayloadMask, ip);
  uint32_t base = e & kPayloadMask;
  for (uint32_t depth = 0;; ++depth) {
    const uint32_t smax = depth == 0 ? r->node_bits : kNodeStrideMax;
    const uint32_t ns = shift > smax ? shift - smax : 0u;
    const uint32_t idx = (ip >> ns) & ((1u << (shift - ns)) - 1u);
    const uint32_t *q = &r->wide[((size_t)base + idx) * 4];
    shift = ns;
    switch (q[1] >> kKindShift) {
      case kKindLeaf: return q[2];
      case kKindLine: return line_site(r, q[2], ip);
      case kKindQuad: {
        const uint32_t off = ip & (uint32_t)(((uint64_t)1 << ns) - 1);
        const uint32_t pos = ((q[0] & 0xFFFFu) <= off) + ((q[0] >> 16) <= off) + ((q[1] & 0xFFFFu) <= off);
        const uint32_t sites[4] = {q[2] & 0xFFFFu, q[2] >> 16, q[3] & 0xFFFFu, q[3] >> 16};
        return sites[pos];
      }
      default: base = q[2];
    }
  }
}

bool host_in_ranges(const gnm_registry *r, uint32_t ip) {
  for (size_t j = 0; j < r->local_lo.size(); ++j)
    if (ip - r->local_lo[j] <= r->local_hi[j] - r->local_lo[j]) return true;
  return false;
}

// Locality through the root cell's sub-block masks, as the device decides it.
bool host_is_local(const gnm_registry *r, uint32_t ip) {
  const uint32_t m = r->root_local[ip >> (32u - r->root_bits)];
  const uint32_t sub = (ip >> (28u - r->root_bits)) & 15u;
  if ((m >> (16u + sub)) & 1u) return host_in_ranges(r, ip);
  return (m >> sub) & 1u;
}

// Per root cell, 16 sub-blocks of 2^(28 - root_bits) addresses each: bit j
// if a local range covers sub-block j entirely, bit 16 + j if local ranges
// cover part of it.  The ranges are disjoint and coalesced, so a sub-block is
// entirely local only if one range covers it.
void build_local_masks(gnm_registry *r) {
  r->root_local.assign((size_t)1 << r->root_bits, 0u);
  const uint32_t sb_shift = 28u - r->root_bits;
  for (size_t j = 0; j < r->local_lo.size(); ++j) {
    const uint64_t lo = r->local_lo[j], hi = r->local_hi[j];
    for (uint64_t b = lo >> sb_shift; b <= (hi >> sb_shift); ++b) {
      const uint64_t blo = b << sb_shift, bhi = blo + ((uint64_t)1 << sb_shift) - 1;
      const bool full = lo <= blo && hi >= bhi;
      uint32_t &m = r->root_local[b >> 4];
      const uint32_t sub = (uint32_t)(b & 15u);
      if (full) m = (m | (1u << sub)) & ~(1u << (16u + sub));
      else if (!((m >> sub) & 1u)) m |= 1u << (16u + sub);
    }
  }
}

// LDS plan for a classify workgroup: the root (with locality masks), then (if
// it fits) the accumulator table, then (if they fit) the leaf lines.
void plan_lds(gnm_registry *r, uint32_t lds_budget) {
  // The budget covers root, accumulator table (or its cache) and leaf lines;
  // the top kLdsReserve bytes of LDS stay free.
  if (lds_budget > kLdsMax - kLdsReserve) lds_budget = kLdsMax - kLdsReserve;
  const uint64_t root_b = 8ull << r->root_bits;
  const uint64_t line_b = 4ull * r->lines.size();
  const uint64_t acc_b = 8ull * kAccFields * r->rows();
  uint64_t used = root_b;
  r->acc_in_lds = used + acc_b <= lds_budget;
  if (r->acc_in_lds) used += acc_b;
  used = (used + 15u) & ~15ull;  // 16-byte loads of line keys
  r->lines_in_lds = used + line_b <= lds_budget;
  // A table that does not fit gets as many cache slots (a 56-byte row and a
  // 4-byte tag each) as the rest of the budget holds.
  uint64_t cache_b = 0;
  r->cache_slots = 0;
  if (!r->acc_in_lds) {
    const uint64_t rest = lds_budget - used - (r->lines_in_lds ? line_b : 0);
    uint64_t slots = rest / (8ull * kAccFields + 4ull);
    if (slots > kMaxCacheSlots) slots = kMaxCacheSlots;
    slots &= ~3ull;  // 4-way sets
    r->cache_slots = (uint32_t)slots;
    cache_b = (slots * (8ull * kAccFields + 4ull) + 15u) & ~15ull;
  }
  // layout: root | table, or cache rows and tags | lines
  r->lds_off_acc = (uint32_t)root_b;
  r->lds_off_lines = (uint32_t)(used + cache_b);
  r->lds_bytes = (uint32_t)(r->lds_off_lines + (r->lines_in_lds ? line_b : 0));
}

}  // namespace gnm

using namespace gnm;

extern "C" int gnm_registry_build(const gnm_prefix *sites, uint64_t n_prefixes, uint32_t n_sites,
                                  const gnm_prefix *local, uint32_t n_local,
                                  const gnm_registry_opts *opts, hipStream_t stream,
                                  gnm_registry **out) {
  if (!out) return fail(GNM_E_INVAL, "out is NULL");
  *out = nullptr;
  if (n_prefixes > 0 && !sites) return fail(GNM_E_INVAL, "sites is NULL");
  if (n_local > 0 && !local) return fail(GNM_E_INVAL, "local is NULL");
  if (n_sites == 0 || n_sites > kMaxSites) return fail(GNM_E_INVAL, "n_sites out of range");
  gnm_registry_opts o{};
  if (opts) o = *opts;
  const uint32_t root_bits = o.root_bits ? o.root_bits : 12u;
  const uint32_t list_max = o.list_max ? o.list_max : kLineKeys;
  if (o.node_bits && (o.node_bits < 4 || o.node_bits > 16)) return fail(GNM_E_INVAL, "node_bits must be 4..16");
  const uint32_t lds_budget = o.lds_bytes ? o.lds_bytes : kLdsMax;
  if (root_bits < 8 || root_bits > 14) return fail(GNM_E_INVAL, "root_bits must be 8..14");
  if (list_max < 2 || list_max > kLineKeys) return fail(GNM_E_INVAL, "list_max must be 2..8");
  if (lds_budget > kLdsMax || lds_budget < (8u << root_bits))
    return fail(GNM_E_INVAL, "lds_bytes must hold the root table and be at most 163840");

  gnm_registry *r = new (std::nothrow) gnm_registry();
  if (!r) return fail(GNM_E_NOMEM, "host allocation failed");
  try {
    r->n_sites = n_sites;
    r->root_bits = root_bits;
    r->list_max = list_max;
    r->info.n_prefixes_in = n_prefixes;

    // validate and normalise
    std::vector<Pfx> p;
    p.reserve(n_prefixes);
    for (uint64_t i = 0; i < n_prefixes; ++i) {
      const gnm_prefix &s = sites[i];
      if (s.len > 32) { delete r; return fail(GNM_E_INVAL, "prefix length > 32"); }
      if (s.site >= n_sites) { delete r; return fail(GNM_E_INVAL, "site id >= n_sites"); }
      const uint32_t a = s.addr & mask_of(s.len);
      if (a != s.addr) r->info.n_host_bits++;
      p.push_back({a, s.len, s.site});
    }
    std::sort(p.begin(), p.end(), pfx_less);
    std::vector<Pfx> d;
    d.reserve(p.size());
    for (const Pfx &q : p) {
      if (!d.empty() && d.back().addr == q.addr && d.back().len == q.len) {
        if (d.back().site != q.site) { delete r; return fail(GNM_E_CONFLICT, "prefix registered to two sites"); }
        r->info.n_duplicates++;
        continue;
      }
      d.push_back(q);
    }
    r->info.n_prefixes = d.size();

    // local set -> disjoint inclusive ranges
    std::vector<std::pair<uint32_t, uint32_t>> lr;
    for (uint32_t j = 0; j < n_local; ++j) {
      if (local[j].len > 32) { delete r; return fail(GNM_E_INVAL, "local prefix length > 32"); }
      const uint32_t m = mask_of(local[j].len);
      lr.push_back({local[j].addr & m, (local[j].addr & m) | ~m});
    }
    std::sort(lr.begin(), lr.end());
    for (const auto &x : lr) {
      if (!r->local_lo.empty() && (uint64_t)x.first <= (uint64_t)r->local_hi.back() + 1ull) {
        r->local_hi.back() = std::max(r->local_hi.back(), x.second);
      } else {
        r->local_lo.push_back(x.first);
        r->local_hi.push_back(x.second);
      }
    }
    if (r->local_lo.size() > kMaxLocalRanges) {
      delete r;
      return fail(GNM_E_UNSUPPORTED, "local set needs more than 32 disjoint ranges");
    }

    // longest-prefix-match intervals and the trie layout.  Root cells of up
    // to list_max intervals become leaf lines when all lines fit in LDS
    // beside the root, locality map and accumulator table; otherwise every
    // multi-interval root cell gets a wide node (one 16-byte read resolves
    // most lookups).
    const std::vector<Interval> iv = resolve(d, n_sites);
    r->info.n_intervals = iv.size();
    build_local_masks(r);
    const bool force_wide = (o.flags & GNM_REG_FORCE_WIDE) != 0;
    const bool force_lines = (o.flags & GNM_REG_FORCE_LINES) != 0;
    // Deeper wide nodes resolve a lookup in one 16-byte read per level, but
    // each costs 2^stride entries; past kDeepNodeBytes the structure would
    // no longer stay cache-resident, so cells of up to list_max intervals
    // below the root become 64-byte leaf lines instead.
    bool root_lines = !force_wide, deep = (o.flags & GNM_REG_SHALLOW) == 0;
    // First-level nodes index 12 bits by default, so below a 12-bit root one
    // 16-byte entry covers a /24 and resolves almost every lookup; they cost
    // 64 KiB each, and past kLevel1Bytes the automatic layout uses 8 bits.
    const uint32_t sub_bits = 32u - root_bits;
    uint32_t stride1 = o.node_bits ? o.node_bits : kNodeStride1Max;
    if (stride1 > sub_bits) stride1 = sub_bits;
    if (!o.node_bits) {
      uint64_t multi = 0;
      for (uint64_t b = 0; b < ((uint64_t)1 << root_bits); ++b) {
        const uint64_t lo = b << sub_bits, hi = lo + ((uint64_t)1 << sub_bits) - 1;
        if (r->n_sites && find_index(iv, hi) != find_index(iv, lo)) ++multi;
      }
      if (multi * (16ull << stride1) > kLevel1Bytes) stride1 = std::min(kNodeStrideMax, sub_bits);
    }
    r->node_bits = stride1;
    for (int attempt = 0; attempt < 4; ++attempt) {
      Layout lay{&iv, list_max, root_lines, n_sites < 0xFFFFu, deep, stride1, {}, {}};
      // entry 0 of each array is a harmless dummy (a leaf of site 0) that lanes
      // with nothing to look up may read instead of branching around the load
      lay.wide.assign(4, 0u);
      lay.wide[1] = kKindLeaf << kKindShift;
      lay.lines.assign(kLineWords, 0u);
      r->root.assign((size_t)1 << root_bits, 0u);
      for (uint64_t b = 0; b < ((uint64_t)1 << root_bits); ++b) {
        const uint32_t e = lay.root_cell(b << (32 - root_bits), 32 - root_bits);
        r->root[b] = e;
      }
      if (lay.overflow) { delete r; return fail(GNM_E_NOMEM, "lookup structure exceeds its index range"); }
      r->wide.swap(lay.wide);
      r->lines.swap(lay.lines);
      r->info.n_nodes = lay.n_wide_nodes;
      if (deep && 16ull * lay.deeper_entries > kDeepNodeBytes) {
        deep = false;
        continue;
      }
      plan_lds(r, lds_budget);
      if (!root_lines || force_lines || r->lines_in_lds) break;
      root_lines = false;
    }
    r->info.n_leaf_lines = r->lines.size() / kLineWords - 1;
  } catch (const std::bad_alloc &) {
    delete r;
    return fail(GNM_E_NOMEM, "host allocation failed");
  }

  r->info.n_sites = n_sites;
  r->info.n_local_ranges = (uint32_t)r->local_lo.size();
  r->info.root_bits = r->root_bits;
  r->info.list_max = r->list_max;
  r->info.lines_in_lds = r->lines_in_lds;
  r->info.acc_in_lds = r->acc_in_lds;
  r->info.lds_bytes = r->lds_bytes;
  r->info.cache_slots = r->cache_slots;
  r->info.node_bits = r->node_bits;

  if (o.flags & GNM_REG_HOST_ONLY) {
    *out = r;
    return GNM_OK;
  }

  // device upload: root (64-bit: trie entry | locality masks << 32) | wide |
  // lines, each 256-byte aligned
  std::vector<uint64_t> root64(r->root.size());
  for (size_t b = 0; b < root64.size(); ++b) root64[b] = (uint64_t)r->root[b] | ((uint64_t)r->root_local[b] << 32);
  auto al = [](uint64_t x) { return (x + 255) & ~255ull; };
  const uint64_t b_root = 8ull * root64.size(), b_nodes = 4ull * r->wide.size();
  const uint64_t b_lines = 4ull * r->lines.size();
  const uint64_t o_nodes = al(b_root), o_lines = o_nodes + al(b_nodes);
  const uint64_t total = o_lines + al(b_lines) + 256;
  hipError_t e = hipGetDevice(&r->device);
  if (e == hipSuccess) e = hipMalloc(&r->d_buf, total);
  if (e != hipSuccess) {
    set_last_error(std::string("registry upload: ") + hipGetErrorString(e));
    delete r;
    return e == hipErrorOutOfMemory ? GNM_E_NOMEM : GNM_E_HIP;
  }
  char *base = (char *)r->d_buf;
  r->d_root = (const uint64_t *)base;
  r->d_wide = (const uint32_t *)(base + o_nodes);
  r->d_lines = (const uint32_t *)(base + o_lines);
  r->d_bytes = total;
  struct Part { const void *h; void *d; uint64_t b; } parts[] = {
      {root64.data(), (void *)r->d_root, b_root}, {r->wide.data(), (void *)r->d_wide, b_nodes},
      {r->lines.data(), (void *)r->d_lines, b_lines}};
  for (const Part &q : parts) {
    if (q.b == 0) continue;
    e = hipMemcpyAsync(q.d, q.h, q.b, hipMemcpyHostToDevice, stream);
    if (e != hipSuccess) break;
  }
  if (e == hipSuccess) e = hipStreamSynchronize(stream);
  if (e != hipSuccess) {
    set_last_error(std::string("registry upload: ") + hipGetErrorString(e));
    (void)hipFree(r->d_buf);
    delete r;
    return GNM_E_HIP;
  }
  r->host_only = false;
  r->info.device_bytes = total;
  *out = r;
  return GNM_OK;
}

extern "C" int gnm_registry_free(gnm_registry *reg) {
  if (!reg) return GNM_OK;
  int rc = GNM_OK;
  if (reg->d_buf) {
    int cur = -1;
    (void)hipGetDevice(&cur);
    if (cur != reg->device) (void)hipSetDevice(reg->device);
    hipError_t e = hipFree(reg->d_buf);
    if (cur != reg->device && cur >= 0) (void)hipSetDevice(cur);
    if (e != hipSuccess) {
      set_last_error(std::string("registry free: ") + hipGetErrorString(e));
      rc = GNM_E_HIP;
    }
  }
  delete reg;
  return rc;
}

extern "C" int gnm_registry_info_get(const gnm_registry *reg, gnm_registry_info *info) {
  if (!reg || !info) return fail(GNM_E_INVAL, "NULL argument");
  *info = reg->info;
  return GNM_OK;
}

extern "C" uint64_t gnm_acc_rows(const gnm_registry *reg) { return reg ? reg->rows() : 0; }

extern "C" int gnm_registry_lookup_host(const gnm_registry *reg, const uint32_t *ip, uint64_t n,
                                        uint32_t *site_out, uint8_t *local_out) {
  if (!reg || (n > 0 && !ip)) return fail(GNM_E_INVAL, "NULL argument");
  for (uint64_t i = 0; i < n; ++i) {
    if (site_out) site_out[i] = host_lookup(reg, ip[i]);
    if (local_out) local_out[i] = host_is_local(reg, ip[i]) ? 1 : 0;
  }
  return GNM_OK;
}

extern "C" const char *gnm_strerror(int code) {
  switch (code) {
    case GNM_OK: return "ok";
    case GNM_E_INVAL: return "invalid argument";
    case GNM_E_CONFLICT: return "prefix registered to two different sites";
    case GNM_E_NOMEM: return "out of memory";
    case GNM_E_HIP: return "HIP runtime error";
    case GNM_E_UNSUPPORTED: return "unsupported configuration";
    default: return "unknown error";
  }
}

extern "C" const char *gnm_last_error(void) { return gnm::g_last_error.c_str(); }

extern "C" const char *gnm_version(void) { return "gnm 0.1.0 (gfx950)"; }
