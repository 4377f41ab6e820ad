/*
 * CPU oracle for flow-record classification and per-site aggregation.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, loads or
 * calls this file; only the test suite, the smoke check and the benchmark's
 * CPU-baseline leg do.  It shares no code, header, table or helper with the
 * GPU library.
 *
 * It evaluates the plain definition record by record, with no blocking or
 * reordering beyond an OpenMP split over records into thread-private tables
 * that are merged exactly (sums mod 2^64, min, max).
 *
 * Paper passages followed (G-NetMon, arXiv 1108.1785):
 *   - registered collaboration subnets identify science transfers between the
 *     local site and collaboration sites (§III.B.1, Site Registration Thread);
 *   - each record is assigned to a site from its source or destination
 *     address, and a transfer rate is computed from its byte count and the
 *     timestamps of its first and last packets (§III.B.2, TransRate Kernel);
 *   - per-site rate statistics maximum, minimum and average are accumulated
 *     with atomic updates (§III.B.2, TransRate Kernel; §IV.B);
 *   - the registry is read-only and rebuilt from scratch on change
 *     (§III.B.2, Catalog Kernel).
 * Readings where the paper is silent (longest-prefix match over /0../32, the
 * direction from the local endpoint, the NODIR and unmatched rows, the integer
 * rate floor(bytes*8000/duration_ms) with decimal units, bulk eligibility
 * bytes > threshold and duration > 0) are fixed readings; each function
 * below names the one it implements.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <omp.h>

#define ORC_OK 0
#define ORC_E_INVAL (-1)
#define ORC_E_CONFLICT (-2)
#define ORC_E_NOMEM (-3)

typedef struct {
  uint64_t flows, bytes, packets, duration_ms;
  uint64_t bulk_flows, rate_sum, rate_min, rate_max;
} orc_row;

/* Network mask of a prefix length; length 0 matches every address. */
static uint32_t orc_mask(uint32_t len) {
  return len == 0 ? 0u : (uint32_t)(0xFFFFFFFFu << (32u - len));
}

/* One sorted table of (network, site) per prefix length 0..32. */
typedef struct {
  uint32_t *net[33];
  uint32_t *site[33];
  uint64_t n[33];
  uint32_t n_sites;
} orc_registry;

typedef struct {
  uint64_t bulk_bytes;
  uint32_t min_avg_packet_bytes;
  uint32_t min_packets;
  uint32_t min_duration_ms;
  uint32_t reserved;
} orc_bulk_rule;

typedef struct { uint32_t net, site; } orc_pair;

static int orc_pair_cmp(const void *a, const void *b) {
  const orc_pair *x = (const orc_pair *)a, *y = (const orc_pair *)b;
  if (x->net != y->net) return x->net < y->net ? -1 : 1;
  if (x->site != y->site) return x->site < y->site ? -1 : 1;
  return 0;
}

void orc_registry_free(orc_registry *r) {
  if (!r) return;
  for (int L = 0; L <= 32; ++L) { free(r->net[L]); free(r->site[L]); }
  free(r);
}

/*
 * Build the registry.  Host bits of each prefix are cleared (normalisation);
 * the same (network, length) registered twice for one site counts once; the
 * same (network, length) registered to two different sites is a conflict.
 * A length above 32 or a site id >= n_sites is invalid.
 */
int orc_registry_build(const uint32_t *addr, const uint32_t *len, const uint32_t *site,
                       uint64_t n, uint32_t n_sites, orc_registry **out) {
  *out = NULL;
  if (n > 0 && (!addr || !len || !site)) return ORC_E_INVAL;
  for (uint64_t i = 0; i < n; ++i)
    if (len[i] > 32 || site[i] >= n_sites) return ORC_E_INVAL;
  orc_registry *r = (orc_registry *)calloc(1, sizeof(orc_registry));
  if (!r) return ORC_E_NOMEM;
  r->n_sites = n_sites;
  uint64_t cnt[33] = {0};
  for (uint64_t i = 0; i < n; ++i) cnt[len[i]]++;
  for (int L = 0; L <= 32; ++L) {
    if (!cnt[L]) continue;
    orc_pair *p = (orc_pair *)malloc(cnt[L] * sizeof(orc_pair));
    if (!p) { orc_registry_free(r); return ORC_E_NOMEM; }
    uint64_t k = 0;
    for (uint64_t i = 0; i < n; ++i)
      if (len[i] == (uint32_t)L) { p[k].net = addr[i] & orc_mask((uint32_t)L); p[k].site = site[i]; ++k; }
    qsort(p, cnt[L], sizeof(orc_pair), orc_pair_cmp);
    r->net[L] = (uint32_t *)malloc(cnt[L] * sizeof(uint32_t));
    r->site[L] = (uint32_t *)malloc(cnt[L] * sizeof(uint32_t));
    if (!r->net[L] || !r->site[L]) { free(p); orc_registry_free(r); return ORC_E_NOMEM; }
    uint64_t m = 0;
    for (uint64_t i = 0; i < cnt[L]; ++i) {
      if (m > 0 && r->net[L][m - 1] == p[i].net) {
        if (r->site[L][m - 1] != p[i].site) { free(p); orc_registry_free(r); return ORC_E_CONFLICT; }
        continue; /* exact duplicate for the same site */
      }
      r->net[L][m] = p[i].net; r->site[L][m] = p[i].site; ++m;
    }
    r->n[L] = m;
    free(p);
  }
  *out = r;
  return ORC_OK;
}

/*
 * Longest-prefix match: the site of the longest registered prefix that
 * contains ip, or n_sites when no prefix does.  Probing lengths from 32 down
 * to 0 and stopping at the first registered network equal to ip under that
 * length's mask is the definition "longest containing prefix" written out.
 */
uint32_t orc_lookup(const orc_registry *r, uint32_t ip) {
  for (int L = 32; L >= 0; --L) {
    uint64_t n = r->n[L];
    if (!n) continue;
    uint32_t key = ip & orc_mask((uint32_t)L);
    const uint32_t *a = r->net[L];
    uint64_t lo = 0, hi = n;
    while (lo < hi) {
      uint64_t mid = lo + (hi - lo) / 2;
      if (a[mid] < key) lo = mid + 1; else hi = mid;
    }
    if (lo < n && a[lo] == key) return r->site[L][lo];
  }
  return r->n_sites;
}

/* Membership in any local prefix (independent of the site registry). */
static int orc_is_local(const uint32_t *laddr, const uint32_t *llen, uint32_t n_local, uint32_t ip) {
  for (uint32_t j = 0; j < n_local; ++j) {
    uint32_t m = orc_mask(llen[j]);
    if ((ip & m) == (laddr[j] & m)) return 1;
  }
  return 0;
}

/*
 * Integer transfer rate in bits/s: floor(bytes * 8000 / duration_ms) in exact
 * 128-bit arithmetic, saturated to 2^64-1 (§III.B.2: rate from the byte count
 * and the first/last packet timestamps; decimal units as in §IV.A.3).
 * Requires dur_ms > 0.
 */
uint64_t orc_rate_bps(uint64_t bytes, uint32_t dur_ms) {
  unsigned __int128 q = ((unsigned __int128)bytes * 8000u) / dur_ms;
  return q > (unsigned __int128)UINT64_MAX ? UINT64_MAX : (uint64_t)q;
}

/*
 * Which records are rate-eligible ("bulk flows"; §III.B.2, TransRate Kernel).
 * The paper leaves out of the rate statistics the reverse-direction flows of
 * pure ACKs, recognised by their small average packet size, and the short
 * administrative exchanges with few packets and a short duration; it gives no
 * thresholds.  Read here as: more than bulk_bytes bytes, a non-zero duration,
 * an average packet size of at least min_avg_packet_bytes (bytes >=
 * min_avg_packet_bytes * packets, so a flow of 0 packets passes), at least
 * min_packets packets and a duration of at least min_duration_ms.  Zero
 * thresholds switch a filter off.
 */
int orc_is_bulk(const orc_bulk_rule *b, uint64_t bytes, uint32_t packets, uint32_t dur) {
  return bytes > b->bulk_bytes && dur > 0u && bytes >= (uint64_t)b->min_avg_packet_bytes * packets &&
         packets >= b->min_packets && dur >= b->min_duration_ms;
}

static void orc_row_init(orc_row *t, uint64_t rows) {
  memset(t, 0, rows * sizeof(orc_row));
  for (uint64_t i = 0; i < rows; ++i) t[i].rate_min = UINT64_MAX;
}

/*
 * Classify and aggregate one window of records into rows:
 *   row 2*site+dir for site in [0, n_sites] (n_sites = unmatched remote),
 *   dir 0 = inbound (remote source -> local destination),
 *   dir 1 = outbound (local source -> remote destination),
 *   row 2*n_sites+2 = NODIR (both endpoints local, or neither).
 * out must hold 2*n_sites+3 rows; it is initialised here.
 */
int orc_classify_aggregate(const orc_registry *r, const uint32_t *laddr, const uint32_t *llen,
                           uint32_t n_local, const uint32_t *src, const uint32_t *dst,
                           const uint64_t *bytes, const uint32_t *packets,
                           const uint32_t *first_ms, const uint32_t *last_ms, uint64_t n,
                           const orc_bulk_rule *rule, int n_threads, orc_row *out) {
  const uint32_t S = r->n_sites;
  const uint64_t rows = 2ull * S + 3ull;
  const uint64_t nodir = 2ull * S + 2ull;
  for (uint32_t j = 0; j < n_local; ++j)
    if (llen[j] > 32) return ORC_E_INVAL;
  orc_row_init(out, rows);
  if (n_threads <= 0) n_threads = omp_get_max_threads();
  int failed = 0;
#pragma omp parallel num_threads(n_threads)
  {
    orc_row *t = (orc_row *)malloc(rows * sizeof(orc_row));
    if (!t) {
#pragma omp atomic write
      failed = 1;
    } else {
      orc_row_init(t, rows);
#pragma omp for schedule(static)
      for (uint64_t i = 0; i < n; ++i) {
        int ls = orc_is_local(laddr, llen, n_local, src[i]);
        int ld = orc_is_local(laddr, llen, n_local, dst[i]);
        uint64_t row;
        if (ls == ld) {
          row = nodir;
        } else {
          uint32_t remote = ld ? src[i] : dst[i];
          uint64_t dir = ld ? 0u : 1u;
          row = 2ull * orc_lookup(r, remote) + dir;
        }
        uint32_t dur = last_ms[i] - first_ms[i]; /* modulo 2^32 */
        orc_row *o = &t[row];
        o->flows += 1u;
        o->bytes += bytes[i];
        o->packets += packets[i];
        o->duration_ms += dur;
        if (orc_is_bulk(rule, bytes[i], packets[i], dur)) {
          uint64_t rate = orc_rate_bps(bytes[i], dur);
          o->bulk_flows += 1u;
          o->rate_sum += rate;
          if (rate < o->rate_min) o->rate_min = rate;
          if (rate > o->rate_max) o->rate_max = rate;
        }
      }
#pragma omp critical
      {
        for (uint64_t k = 0; k < rows; ++k) {
          out[k].flows += t[k].flows;
          out[k].bytes += t[k].bytes;
          out[k].packets += t[k].packets;
          out[k].duration_ms += t[k].duration_ms;
          out[k].bulk_flows += t[k].bulk_flows;
          out[k].rate_sum += t[k].rate_sum;
          if (t[k].rate_min < out[k].rate_min) out[k].rate_min = t[k].rate_min;
          if (t[k].rate_max > out[k].rate_max) out[k].rate_max = t[k].rate_max;
        }
      }
      free(t);
    }
  }
  return failed ? ORC_E_NOMEM : ORC_OK;
}

/* Batch form of the above: each window [off[w], off[w+1]) into its own table. */
int orc_classify_aggregate_windows(const orc_registry *r, const uint32_t *laddr, const uint32_t *llen,
                                   uint32_t n_local, const uint32_t *src, const uint32_t *dst,
                                   const uint64_t *bytes, const uint32_t *packets,
                                   const uint32_t *first_ms, const uint32_t *last_ms,
                                   const uint64_t *off, uint32_t n_windows,
                                   const orc_bulk_rule *rule, int n_threads, orc_row *out) {
  const uint64_t rows = 2ull * r->n_sites + 3ull;
  for (uint32_t w = 0; w < n_windows; ++w) {
    uint64_t lo = off[w], hi = off[w + 1];
    if (hi < lo) return ORC_E_INVAL;
    int rc = orc_classify_aggregate(r, laddr, llen, n_local, src + lo, dst + lo, bytes + lo,
                                    packets + lo, first_ms + lo, last_ms + lo, hi - lo,
                                    rule, n_threads, out + (uint64_t)w * rows);
    if (rc) return rc;
  }
  return ORC_OK;
}

/*
 * Per record: its row (the same classification as orc_classify_aggregate),
 * whether it is a bulk flow (orc_is_bulk) and, if so, its
 * rate (0 otherwise).  Input of the median statistic: the paper counts each host's
 * and site's rates in 10 kbps buckets and takes the median of the counts
 * (§III.B.2, TransRate Kernel; §III.B.1, NetPerf Monitoring Thread).
 */
int orc_classify_rows(const orc_registry *r, const uint32_t *laddr, const uint32_t *llen, uint32_t n_local,
                      const uint32_t *src, const uint32_t *dst, const uint64_t *bytes, const uint32_t *packets,
                      const uint32_t *first_ms, const uint32_t *last_ms, uint64_t n, const orc_bulk_rule *rule,
                      uint32_t *row_out, uint8_t *bulk_out, uint64_t *rate_out) {
  const uint32_t S = r->n_sites;
  for (uint32_t j = 0; j < n_local; ++j)
    if (llen[j] > 32) return ORC_E_INVAL;
#pragma omp parallel for schedule(static)
  for (uint64_t i = 0; i < n; ++i) {
    int ls = orc_is_local(laddr, llen, n_local, src[i]);
    int ld = orc_is_local(laddr, llen, n_local, dst[i]);
    uint32_t row;
    if (ls == ld) {
      row = 2u * S + 2u;
    } else {
      uint32_t remote = ld ? src[i] : dst[i];
      row = 2u * orc_lookup(r, remote) + (ld ? 0u : 1u);
    }
    uint32_t dur = last_ms[i] - first_ms[i];
    row_out[i] = row;
    int bulk = orc_is_bulk(rule, bytes[i], packets[i], dur);
    bulk_out[i] = (uint8_t)bulk;
    rate_out[i] = bulk ? orc_rate_bps(bytes[i], dur) : 0u;
  }
  return ORC_OK;
}

/* Vectorised lookups for tests: site of the longest containing prefix. */
void orc_lookup_many(const orc_registry *r, const uint32_t *ip, uint64_t n, uint32_t *site_out) {
#pragma omp parallel for schedule(static)
  for (uint64_t i = 0; i < n; ++i) site_out[i] = orc_lookup(r, ip[i]);
}

void orc_rate_many(const uint64_t *bytes, const uint32_t *dur, uint64_t n, uint64_t *out) {
  for (uint64_t i = 0; i < n; ++i) out[i] = dur[i] ? orc_rate_bps(bytes[i], dur[i]) : 0u;
}

int orc_max_threads(void) { return omp_get_max_threads(); }
