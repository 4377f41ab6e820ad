/*
 * The C oracle under AddressSanitizer and UndefinedBehaviorSanitizer (built
 * with gcc by tests/test_sanitize_host.py).  The oracle's source is compiled
 * into this driver so that its static helpers are checked too.
 *
 * Edge cases: a /0 prefix (a mask from a shift by 32 would be undefined) and
 * /32 prefixes, lookups at both ends of the address space, rates at the
 * largest byte counts and durations, a duration that wraps modulo 2^32, sums
 * that wrap modulo 2^64, empty windows and invalid inputs.
 */
#include <stdio.h>

#include "../../oracle/gnm_oracle.c"

static int failures = 0;
#define EXPECT(c)                                                   \
  do {                                                              \
    if (!(c)) {                                                     \
      printf("FAILED %s:%d: %s\n", __FILE__, __LINE__, #c);         \
      ++failures;                                                   \
    }                                                               \
  } while (0)

int main(void) {
  /* registry: /0 -> site 0, 10.0.0.0/8 -> 1, 10.1.2.3/32 -> 2,
     255.255.255.255/32 -> 3, with host bits and a duplicate */
  const uint32_t addr[] = {0x12345678u, 0x0A0B0C0Du, 0x0A010203u, 0xFFFFFFFFu, 0x0A000000u};
  const uint32_t len[] = {0u, 8u, 32u, 32u, 8u};
  const uint32_t site[] = {0u, 1u, 2u, 3u, 1u};
  orc_registry *r = NULL;
  EXPECT(orc_registry_build(addr, len, site, 5, 4, &r) == ORC_OK && r);
  EXPECT(orc_lookup(r, 0u) == 0u);
  EXPECT(orc_lookup(r, 0xFFFFFFFFu) == 3u);
  EXPECT(orc_lookup(r, 0xFFFFFFFEu) == 0u);
  EXPECT(orc_lookup(r, 0x0A010203u) == 2u);
  EXPECT(orc_lookup(r, 0x0A010204u) == 1u);
  EXPECT(orc_lookup(r, 0x0AFFFFFFu) == 1u);
  EXPECT(orc_lookup(r, 0x0B000000u) == 0u);

  /* invalid registries */
  orc_registry *bad = NULL;
  const uint32_t len33[] = {33u};
  EXPECT(orc_registry_build(addr, len33, site, 1, 4, &bad) == ORC_E_INVAL && !bad);
  const uint32_t site9[] = {9u};
  EXPECT(orc_registry_build(addr, len, site9, 1, 4, &bad) == ORC_E_INVAL && !bad);
  const uint32_t caddr[] = {0x0B000000u, 0x0B0000FFu}, clen[] = {8u, 8u}, csite[] = {0u, 1u};
  EXPECT(orc_registry_build(caddr, clen, csite, 2, 2, &bad) == ORC_E_CONFLICT && !bad);
  orc_registry *empty = NULL;
  EXPECT(orc_registry_build(NULL, NULL, NULL, 0, 1, &empty) == ORC_OK && empty);
  EXPECT(orc_lookup(empty, 0x01020304u) == 1u);
  orc_registry_free(empty);
  orc_registry_free(NULL);

  /* rates */
  EXPECT(orc_rate_bps(1ull << 40, 1u) == 8796093022208000ull);
  EXPECT(orc_rate_bps(1000003ull, 3u) == 2666674666ull);
  EXPECT(orc_rate_bps(1ull << 63, 1u) == ~0ull);
  EXPECT(orc_rate_bps(~0ull, 1u) == ~0ull);
  EXPECT(orc_rate_bps(~0ull, 0xFFFFFFFFu) == 34359738376000ull);
  EXPECT(orc_rate_bps(1ull, 0xFFFFFFFFu) == 0ull);

  /* bulk rule: thresholds at their extremes */
  orc_bulk_rule rule = {1000000ull, 0u, 0u, 0u, 0u};
  EXPECT(!orc_is_bulk(&rule, 1000000ull, 1u, 5u));
  EXPECT(orc_is_bulk(&rule, 1000001ull, 1u, 5u));
  EXPECT(!orc_is_bulk(&rule, ~0ull, 1u, 0u));
  orc_bulk_rule strict = {0ull, 0xFFFFFFFFu, 0xFFFFFFFFu, 0xFFFFFFFFu, 0u};
  EXPECT(!orc_is_bulk(&strict, ~0ull, 0xFFFFFFFFu, 5u));
  EXPECT(orc_is_bulk(&strict, ~0ull, 0u, 0xFFFFFFFFu) == 0);

  /* records: local 198.18.0.0/16; sums that wrap, a duration that wraps */
  const uint32_t laddr[] = {0xC6120000u}, llen[] = {16u};
  enum { N = 6 };
  const uint32_t src[N] = {0xC6120101u, 0x0A010203u, 0xC6120101u, 0xFFFFFFFFu, 0xC6120101u, 0x01010101u};
  const uint32_t dst[N] = {0x0A010203u, 0xC6120202u, 0x0A010203u, 0xC6120303u, 0xC6120202u, 0x02020202u};
  const uint64_t bytes[N] = {1ull << 63, 1ull << 63, ~0ull, 5000000ull, 7ull, 9ull};
  const uint32_t packets[N] = {0xFFFFFFFFu, 0xFFFFFFFFu, 1u, 10u, 1u, 1u};
  const uint32_t first[N] = {0xFFFFFF00u, 0u, 10u, 100u, 0u, 0u};
  const uint32_t last[N] = {0x00000100u, 1u, 10u, 1100u, 0xFFFFFFFFu, 3u};
  const uint64_t rows = 2ull * 4u + 3ull;
  orc_row out[11];
  EXPECT(orc_classify_aggregate(r, laddr, llen, 1, src, dst, bytes, packets, first, last, N, &rule, 2, out) == ORC_OK);
  /* row 5 = site 2 outbound: records 0 and 2 (bytes wrap to 2^63 - 1) */
  EXPECT(out[5].flows == 2u && out[5].bytes == (1ull << 63) - 1ull && out[5].duration_ms == 0x200u);
  EXPECT(out[5].bulk_flows == 1u && out[5].rate_min == ~0ull && out[5].rate_max == ~0ull);
  /* row 4 = site 2 inbound: record 1 */
  EXPECT(out[4].flows == 1u && out[4].bulk_flows == 1u && out[4].rate_sum == ~0ull);
  /* row 6 = site 3 inbound: record 3, rate 40,000,000 */
  EXPECT(out[6].flows == 1u && out[6].rate_min == 40000000ull && out[6].rate_max == 40000000ull);
  /* row 10 = NODIR: records 4 (both local) and 5 (neither) */
  EXPECT(out[10].flows == 2u && out[10].bytes == 16u && out[10].duration_ms == 0xFFFFFFFFull + 3ull);
  uint64_t total = 0;
  for (uint64_t k = 0; k < rows; ++k) total += out[k].flows;
  EXPECT(total == N);

  /* empty window and several windows */
  EXPECT(orc_classify_aggregate(r, laddr, llen, 1, src, dst, bytes, packets, first, last, 0, &rule, 1, out) == ORC_OK);
  EXPECT(out[0].flows == 0u && out[0].rate_min == ~0ull);
  const uint64_t off[4] = {0u, 0u, 3u, N};
  orc_row outw[33];
  EXPECT(orc_classify_aggregate_windows(r, laddr, llen, 1, src, dst, bytes, packets, first, last, off, 3, &rule,
                                        1, outw) == ORC_OK);
  EXPECT(outw[0].flows == 0u && outw[rows + 5].flows == 2u && outw[2 * rows + 10].flows == 2u);
  const uint64_t off_bad[3] = {0u, 4u, 2u};
  EXPECT(orc_classify_aggregate_windows(r, laddr, llen, 1, src, dst, bytes, packets, first, last, off_bad, 2,
                                        &rule, 1, outw) == ORC_E_INVAL);
  const uint32_t llen_bad[] = {40u};
  EXPECT(orc_classify_aggregate(r, laddr, llen_bad, 1, src, dst, bytes, packets, first, last, N, &rule, 1, out) ==
         ORC_E_INVAL);

  /* per-record rows, bulk bits and rates */
  uint32_t row_out[N];
  uint8_t bulk_out[N];
  uint64_t rate_out[N];
  EXPECT(orc_classify_rows(r, laddr, llen, 1, src, dst, bytes, packets, first, last, N, &rule, row_out, bulk_out,
                           rate_out) == ORC_OK);
  EXPECT(row_out[0] == 5u && row_out[1] == 4u && row_out[3] == 6u && row_out[4] == 10u && row_out[5] == 10u);
  EXPECT(bulk_out[2] == 0u && rate_out[2] == 0u && rate_out[3] == 40000000ull);

  uint32_t ips[3] = {0u, 0xFFFFFFFFu, 0x0A010203u}, so[3];
  orc_lookup_many(r, ips, 3, so);
  EXPECT(so[0] == 0u && so[1] == 3u && so[2] == 2u);
  const uint64_t rb[2] = {1ull << 40, 1000003ull};
  const uint32_t rd[2] = {1u, 3u};
  uint64_t ro[2];
  orc_rate_many(rb, rd, 2, ro);
  EXPECT(ro[0] == 8796093022208000ull && ro[1] == 2666674666ull);

  orc_registry_free(r);
  printf(failures ? "oracle_san: %d failure(s)\n" : "oracle_san: ok\n", failures);
  return failures ? 1 : 0;
}
