// Host-only registry build and walk under AddressSanitizer and
// UndefinedBehaviorSanitizer (built with g++ by tests/test_sanitize_host.py;
// no GPU is touched: every registry is built with GNM_REG_HOST_ONLY).
//
// Each registry's host walk is compared with a linear longest-match scan at
// every interval boundary (start - 1, start, end + 1 of every prefix) and at
// both ends of the address space; the edge registries include /0 (a mask
// computed with a shift by 32 would be undefined), /32, host bits,
// duplicates, overlaps and invalid inputs.
#include <cstdio>
#include <cstdint>
#include <cstdlib>
#include <vector>

#include "gnm.h"

static int failures = 0;
#define EXPECT(c)                                                   \
  do {                                                              \
    if (!(c)) {                                                     \
      std::printf("FAILED %s:%d: %s\n", __FILE__, __LINE__, #c);    \
      ++failures;                                                   \
    }                                                               \
  } while (0)

static uint32_t mask_len(uint32_t len) { return len == 0 ? 0u : 0xFFFFFFFFu << (32u - len); }

// Longest containing prefix by a linear scan (the definition, written out).
static uint32_t scan_lpm(const std::vector<gnm_prefix> &p, uint32_t n_sites, uint32_t ip) {
  int best = -1;
  uint32_t site = n_sites;
  for (const gnm_prefix &q : p) {
    const uint32_t m = mask_len(q.len);
    if ((ip & m) == (q.addr & m) && (int)q.len > best) {
      best = (int)q.len;
      site = q.site;
    }
  }
  return site;
}

static bool scan_local(const std::vector<gnm_prefix> &l, uint32_t ip) {
  for (const gnm_prefix &q : l)
    if ((ip & mask_len(q.len)) == (q.addr & mask_len(q.len))) return true;
  return false;
}

static uint64_t rng = 0x9E3779B97F4A7C15ull;
static uint32_t next32() {
  rng ^= rng << 13;
  rng ^= rng >> 7;
  rng ^= rng << 17;
  return (uint32_t)(rng >> 16);
}

static void check_registry(const char *name, const std::vector<gnm_prefix> &p, uint32_t n_sites,
                           const std::vector<gnm_prefix> &local, const gnm_registry_opts &o) {
  gnm_registry *reg = nullptr;
  gnm_registry_opts opts = o;
  opts.flags |= GNM_REG_HOST_ONLY;
  const int rc = gnm_registry_build(p.data(), p.size(), n_sites, local.data(), (uint32_t)local.size(), &opts,
                                    nullptr, &reg);
  if (rc != GNM_OK) {
    std::printf("FAILED %s: build rc %d (%s)\n", name, rc, gnm_last_error());
    ++failures;
    return;
  }
  std::vector<uint32_t> ips = {0u, 1u, 0x7FFFFFFFu, 0x80000000u, 0xFFFFFFFEu, 0xFFFFFFFFu};
  for (const gnm_prefix &q : p) {
    const uint32_t lo = q.addr & mask_len(q.len), hi = lo | ~mask_len(q.len);
    ips.push_back(lo);
    ips.push_back(lo - 1u);
    ips.push_back(hi);
    ips.push_back(hi + 1u);
  }
  for (const gnm_prefix &q : local) {
    const uint32_t lo = q.addr & mask_len(q.len), hi = lo | ~mask_len(q.len);
    ips.push_back(lo);
    ips.push_back(lo - 1u);
    ips.push_back(hi);
    ips.push_back(hi + 1u);
  }
  for (int k = 0; k < 2000; ++k) ips.push_back(next32());
  std::vector<uint32_t> site(ips.size());
  std::vector<uint8_t> loc(ips.size());
  EXPECT(gnm_registry_lookup_host(reg, ips.data(), ips.size(), site.data(), loc.data()) == GNM_OK);
  int bad = 0;
  for (size_t i = 0; i < ips.size(); ++i) {
    if (site[i] != scan_lpm(p, n_sites, ips[i]) || (loc[i] != 0) != scan_local(local, ips[i])) {
      if (bad++ < 3)
        std::printf("  %s: ip %08x site %u (scan %u) local %u\n", name, ips[i], site[i],
                    scan_lpm(p, n_sites, ips[i]), (unsigned)loc[i]);
    }
  }
  if (bad) {
    std::printf("FAILED %s: %d of %zu lookups differ from the scan\n", name, bad, ips.size());
    ++failures;
  }
  gnm_registry_info info{};
  EXPECT(gnm_registry_info_get(reg, &info) == GNM_OK);
  EXPECT(info.n_sites == n_sites);
  EXPECT(gnm_acc_rows(reg) == 2ull * (n_sites + 1ull) + 1ull);
  EXPECT(gnm_registry_free(reg) == GNM_OK);
}

static std::vector<gnm_prefix> random_prefixes(uint32_t n, uint32_t n_sites, uint32_t min_len, uint32_t max_len) {
  std::vector<gnm_prefix> p;
  for (uint32_t i = 0; i < n; ++i) {
    gnm_prefix q{};
    q.len = (uint8_t)(min_len + next32() % (max_len - min_len + 1u));
    q.addr = next32() & mask_len(q.len);
    q.site = next32() % n_sites;
    p.push_back(q);
  }
  // distinct (addr, len): later duplicates take the first one's site
  for (size_t i = 0; i < p.size(); ++i)
    for (size_t j = 0; j < i; ++j)
      if (p[j].addr == p[i].addr && p[j].len == p[i].len) p[i].site = p[j].site;
  return p;
}

int main() {
  const std::vector<gnm_prefix> local = {{0xC6120000u, 16, 0}, {0x0A010000u, 16, 0}};
  gnm_registry_opts dflt{};

  // the worked example of the definition: a /8, a /24 and a /25 nested, and a
  // /24 inside the local /16
  std::vector<gnm_prefix> ex = {{0xCB000000u, 8, 0}, {0xCB007100u, 24, 1}, {0xCB007180u, 25, 2},
                                {0xC6120500u, 24, 1}};
  check_registry("worked example", ex, 3, {{0xC6120000u, 16, 0}}, dflt);

  // /0 and /32 together, host bits set, exact duplicates for one site
  std::vector<gnm_prefix> edge = {{0x12345678u, 0, 3}, {0x0A000001u, 32, 1}, {0xFFFFFFFFu, 32, 2},
                                  {0x00000000u, 32, 0}, {0x0B0C0D0Eu, 8, 4}, {0x0B000000u, 8, 4},
                                  {0xC0A80001u, 24, 5}};
  check_registry("/0 and /32", edge, 6, local, dflt);
  check_registry("/0 only", {{0u, 0, 0}}, 1, {}, dflt);
  check_registry("empty registry", {}, 1, local, dflt);
  check_registry("local /0", {{0x0B000000u, 8, 0}}, 1, {{0u, 0, 0}}, dflt);

  // random registries under every layout option
  const uint32_t opt_flags[] = {0u, GNM_REG_FORCE_WIDE, GNM_REG_FORCE_LINES, GNM_REG_SHALLOW};
  for (uint32_t trial = 0; trial < 24; ++trial) {
    const uint32_t n_sites = 1u + next32() % 300u;
    const uint32_t lo = trial % 3 == 0 ? 0u : 8u, hi = trial % 2 ? 32u : 28u;
    std::vector<gnm_prefix> p = random_prefixes(50u + next32() % 400u, n_sites, lo, hi);
    gnm_registry_opts o{};
    o.flags = opt_flags[trial % 4];
    o.root_bits = 8u + trial % 7u;
    o.list_max = 2u + trial % 7u;
    o.node_bits = trial % 5 == 0 ? 0u : 4u + trial % 13u;
    char name[64];
    std::snprintf(name, sizeof name, "random %u", trial);
    check_registry(name, p, n_sites, local, o);
  }
  // sites beyond 16 bits (wide site codes)
  {
    std::vector<gnm_prefix> p = random_prefixes(300, 70000, 8, 30);
    for (size_t i = 0; i < p.size(); ++i) p[i].site = 65000u + (uint32_t)(i * 13u % 5000u);
    for (size_t i = 0; i < p.size(); ++i)
      for (size_t j = 0; j < i; ++j)
        if (p[j].addr == p[i].addr && p[j].len == p[i].len) p[i].site = p[j].site;
    check_registry("70000 sites", p, 70000, local, dflt);
  }

  // invalid inputs are rejected without touching memory they should not
  gnm_registry *reg = nullptr;
  const gnm_prefix bad_len = {0x0A000000u, 33, 0};
  gnm_registry_opts ho{};
  ho.flags = GNM_REG_HOST_ONLY;
  EXPECT(gnm_registry_build(&bad_len, 1, 1, nullptr, 0, &ho, nullptr, &reg) == GNM_E_INVAL && !reg);
  const gnm_prefix bad_site = {0x0A000000u, 8, 5};
  EXPECT(gnm_registry_build(&bad_site, 1, 5, nullptr, 0, &ho, nullptr, &reg) == GNM_E_INVAL && !reg);
  const gnm_prefix conflict[2] = {{0x0B000000u, 8, 0}, {0x0B0000FFu, 8, 1}};
  EXPECT(gnm_registry_build(conflict, 2, 2, nullptr, 0, &ho, nullptr, &reg) == GNM_E_CONFLICT && !reg);
  EXPECT(gnm_registry_build(nullptr, 1, 1, nullptr, 0, &ho, nullptr, &reg) == GNM_E_INVAL);
  EXPECT(gnm_registry_build(&bad_site, 1, 0, nullptr, 0, &ho, nullptr, &reg) == GNM_E_INVAL);
  EXPECT(gnm_registry_build(nullptr, 0, 1, nullptr, 0, &ho, nullptr, nullptr) == GNM_E_INVAL);
  gnm_registry_opts bad_root = ho;
  bad_root.root_bits = 15;
  EXPECT(gnm_registry_build(nullptr, 0, 1, nullptr, 0, &bad_root, nullptr, &reg) == GNM_E_INVAL);
  gnm_registry_opts bad_list = ho;
  bad_list.list_max = 9;
  EXPECT(gnm_registry_build(nullptr, 0, 1, nullptr, 0, &bad_list, nullptr, &reg) == GNM_E_INVAL);
  std::vector<gnm_prefix> many_local;
  for (uint32_t j = 0; j < 40; ++j) many_local.push_back({(j * 2u) << 24, 8, 0});
  EXPECT(gnm_registry_build(nullptr, 0, 1, many_local.data(), 40, &ho, nullptr, &reg) == GNM_E_UNSUPPORTED);
  EXPECT(gnm_registry_free(nullptr) == GNM_OK);
  for (int code = 1; code >= -8; --code) EXPECT(gnm_strerror(code) != nullptr);
  EXPECT(gnm_version() != nullptr);

  std::printf(failures ? "registry_san: %d failure(s)\n" : "registry_san: ok\n", failures);
  return failures ? 1 : 0;
}
