/*
 * gnm.h — C ABI of libgnm: classification of NetFlow-style flow records by
 * longest-prefix match against a registry of collaboration-site subnets, and
 * reduction of the classified records into per-site, per-direction integer
 * totals and bulk-transfer rate statistics, on an AMD Instinct MI355X (gfx950).
 *
 * Method: G-NetMon (Wu, DeMar, Holmgren, Singh, Pordes; arXiv 1108.1785).
 *   - registered scientific subnets identify transfers between the local site
 *     and collaboration sites (§III.B.1, Site Registration Thread);
 *   - a read-only lookup structure is built from the registry and rebuilt
 *     from scratch on any change (§III.B.2, Catalog Kernel);
 *   - one pass over the flow records assigns each record to a site from its
 *     source or destination address and derives a transfer rate from its
 *     bytes and first/last packet timestamps; per-site statistics are
 *     accumulated with atomic updates (§III.B.2, TransRate Kernel);
 *   - sites whose rate statistic falls below a standard are warned about
 *     (§III.B.1, NetPerf Monitoring Thread; §IV.B): the mean rate per window
 *     (gnm_flag_suboptimal), or the paper's criterion, the median rate read
 *     from 10 kbps bucket counts, low in two consecutive windows
 *     (gnm_params.rate_hist, then gnm_median_flags).
 *
 * Definition computed (bit-exact, integer only).  For each record in a window:
 *   mask(L)      = 0 for L = 0, else the top L bits set.
 *   local(ip)    = ip lies in any local prefix.
 *   direction    : exactly one endpoint local; inbound (0) when the destination
 *                  is local (remote = source), outbound (1) when the source is
 *                  local (remote = destination).  Otherwise the record goes to
 *                  the NODIR row.
 *   site         = site of the longest registered prefix containing the remote
 *                  address, or n_sites ("no registered site") when none does.
 *   row          = 2*site + direction, or NODIR = 2*n_sites + 2.
 *   dur          = (last_ms - first_ms) mod 2^32.
 *   bulk         = bytes > bulk_bytes and dur > 0 (and the optional
 *                  exclusion filters of gnm_params).
 *   rate         = min(floor(bytes * 8000 / dur), 2^64 - 1)   [bit/s, decimal]
 *   row.flows += 1; row.bytes += bytes; row.packets += packets;
 *   row.duration_ms += dur; if bulk: row.bulk_flows += 1,
 *   row.rate_sum_bps += rate, row.rate_min_bps = min(.., rate),
 *   row.rate_max_bps = max(.., rate).
 * Every sum is modulo 2^64; an untouched row is all zero except
 * rate_min_bps = 2^64-1.  The result is a unique integer table: it does not
 * depend on record order, launch shape or thread timing.
 *
 * Conventions for every entry point:
 *   - Return GNM_OK (0) or a negative GNM_E_* code; nothing is thrown across
 *     the ABI.  After GNM_E_HIP, gnm_last_error() names the HIP error.
 *   - Device pointers are caller-owned device memory (hipMalloc or any
 *     allocator of the same device); the library never frees them.
 *   - Work is enqueued on the caller's stream (NULL = the null stream) and the
 *     call returns; results are valid once that stream has synchronised, and
 *     inputs must stay alive and unmodified until then.
 *   - Addresses are host-order uint32 with the first octet in the most
 *     significant byte (10.0.0.1 = 0x0A000001).
 */
#ifndef GNM_H
#define GNM_H

#include <stddef.h>
#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

#define GNM_OK 0
#define GNM_E_INVAL (-1)       /* null pointer, length > 32, site >= n_sites, bad sizes */
#define GNM_E_CONFLICT (-2)    /* one (network, length) registered to two sites */
#define GNM_E_NOMEM (-3)       /* host or device allocation failed */
#define GNM_E_HIP (-4)         /* a HIP runtime call failed; see gnm_last_error() */
#define GNM_E_UNSUPPORTED (-5) /* e.g. a host-only registry passed to a device call */

/* One CIDR prefix.  For the site registry, `site` is the collaboration-site id
 * in [0, n_sites); for the local set it is ignored.  Host bits of `addr`
 * below the prefix length are ignored (the prefix is normalised). */
typedef struct {
  uint32_t addr;
  uint32_t len; /* 0..32 */
  uint32_t site;
} gnm_prefix;

/* A run of flow records in structure-of-arrays form, all device pointers of
 * n elements.  Ports and protocol belong to the record format but are not
 * read by this path and may be NULL. */
typedef struct {
  const uint32_t *src_ip;
  const uint32_t *dst_ip;
  const uint16_t *src_port; /* may be NULL (not read) */
  const uint16_t *dst_port; /* may be NULL (not read) */
  const uint8_t *proto;     /* may be NULL (not read) */
  const uint64_t *bytes;
  const uint32_t *packets;
  const uint32_t *first_ms; /* router uptime at the first packet, ms */
  const uint32_t *last_ms;  /* router uptime at the last packet, ms */
  uint64_t n;
} gnm_records;

/* One accumulator row (64 bytes).  The table of one window holds
 * gnm_acc_rows(reg) rows: 2*site+dir for site in [0, n_sites] (site n_sites
 * = no registered site), then NODIR. */
typedef struct {
  uint64_t flows;
  uint64_t bytes;
  uint64_t packets;
  uint64_t duration_ms;
  uint64_t bulk_flows;
  uint64_t rate_sum_bps;
  uint64_t rate_min_bps; /* 2^64-1 while the row has no bulk flow */
  uint64_t rate_max_bps;
} gnm_acc;

#define GNM_ACCUMULATE 0x1u /* gnm_params.flags: add into acc (and rate_hist) instead of initialising them */

/* Rate histograms (§III.B.2, TransRate Kernel: per-rate frequency counts in
 * 10 kbps buckets, everything above 100 Mbps in the last of 10,001 buckets,
 * from which the median is read).  One histogram per registered (site,
 * direction) row 2*site+dir, site < n_sites, per window: uint32
 * rate_hist[n_windows][2*n_sites][GNM_RATE_BUCKETS], window-major.  A bulk
 * flow of rate r counts in bucket min(floor(r / 10,000), 10,000).  Counts
 * wrap modulo 2^32 (medians are exact while every row of a window has fewer
 * than 2^32 bulk flows).  The "no site" and NODIR rows have no histogram. */
#define GNM_RATE_BUCKETS 10001u
#define GNM_RATE_BUCKET_BPS 10000u
#define GNM_NO_MEDIAN 0xFFFFFFFFu /* median bucket of a row without bulk flows */

/* Per-host statistics (§III.B.2, TransRate Kernel: maximum, minimum,
 * average and median transfer rates for each host in a registered site, the
 * median read from the host's 10 kbps bucket array).  Filled by the classify
 * call for every (remote host, direction) of a registered site with at least
 * one bulk flow in the call's records (all windows of the call together),
 * keyed by ((uint64_t)remote_address << 32) | (2*site + dir), where the
 * remote address is the source of an inbound flow and the destination of an
 * outbound one.  Host i of the call has key keys[i], statistics
 * stats[5*i + f] (bulk flows, their bytes, rate sum (modulo 2^64), rate
 * minimum, rate maximum) and median[i], the lower-median bucket of its N bulk
 * flows' rates: the bucket of the ceil(N/2)-th smallest rate, buckets as for
 * rate_hist (exact while a host has fewer than 2^32 bulk flows in a call).
 * Hosts come in an order that depends on timing; the set of (key,
 * statistics, median) does not.  The call never accumulates into the table
 * (GNM_ACCUMULATE with hosts is GNM_E_INVAL), and needs fewer than 2^32
 * records. */
typedef struct {
  uint64_t *keys;      /* DEVICE [capacity], 8-byte aligned */
  uint64_t *stats;     /* DEVICE [capacity * 5], 8-byte aligned */
  uint32_t *median;    /* DEVICE [capacity], 4-byte aligned, or NULL (no medians written) */
  uint64_t capacity;   /* hosts the arrays hold; more hosts than that: counters[0] still counts them all,
                          and `capacity` of them (which ones depends on timing) are written */
  uint64_t *counters;  /* DEVICE [2], 8-byte aligned, written by the call: [0] hosts found, [1] bulk flows
                          of registered sites in the call */
  void *work;          /* DEVICE scratch, 256-byte aligned, caller-owned: contents before and after a call
                          do not matter; calls in flight must not share one */
  uint64_t work_bytes; /* its size: at least gnm_host_work_bytes(reg, rec->n, grid_blocks) */
} gnm_host_table;

/* Per-call parameters.  Zero-initialise and set what you need;
 * gnm_params_default() gives bulk_bytes = 1,000,000 and automatic tuning. */
typedef struct {
  uint64_t bulk_bytes;         /* bulk iff bytes > bulk_bytes and dur > 0 */
  uint32_t flags;              /* GNM_ACCUMULATE */
  uint32_t records_per_thread; /* 0 = automatic (4); else 1, 2 or 4 */
  uint32_t grid_blocks;        /* 0 = automatic; else workgroups of the launch */
  uint32_t flush_records;      /* records a workgroup aggregates in LDS before it flushes its table to the
                                  window table (device-scope atomics) and starts again: 0 = 2^31, the
                                  maximum (larger values are clamped to it, since a table row counts
                                  flows and bulk flows in 32 bits each).  Only tests lower it, to
                                  exercise the mid-launch flush; results do not depend on it */
  void *workspace;             /* optional DEVICE scratch, 16-byte aligned (256-byte for spilled tables and
                                  staged histograms); see below */
  uint64_t workspace_bytes;    /* its size: gnm_workspace_bytes, _n or _hist (below) say what each part needs */
  uint32_t *rate_hist;         /* optional DEVICE rate histograms (layout above), 16-byte aligned: NULL = none;
                                  else filled by the same pass (overwritten unless GNM_ACCUMULATE) */
  /* Exclusion filters (§III.B.2, TransRate Kernel: reverse-direction flows of
   * pure ACKs, recognised by a small average packet size, and administrative
   * exchanges of few packets over a short time are left out of the rate
   * statistics; the paper gives no thresholds).  Each narrows which records
   * count as bulk flows (bulk_flows, rate fields, histograms); flows, bytes,
   * packets and duration still count every record.  0 = off. */
  uint32_t min_avg_packet_bytes; /* bulk only if bytes >= min_avg_packet_bytes * packets (0 packets pass) */
  uint32_t min_packets;          /* bulk only with packets >= min_packets */
  uint32_t min_duration_ms;      /* bulk only with dur >= min_duration_ms (dur > 0 is always required) */
  uint32_t reserved2;
  const gnm_host_table *hosts;   /* optional per-host statistics and medians (host pointer to a table
                                    description): NULL = none; else filled by the call */
} gnm_params;

#define GNM_REG_HOST_ONLY 0x1u   /* gnm_registry_opts.flags: build host structure only */
#define GNM_REG_FORCE_WIDE 0x2u  /* every multi-interval root cell gets a wide node */
#define GNM_REG_FORCE_LINES 0x4u /* root cells of <= list_max intervals stay leaf lines */
#define GNM_REG_SHALLOW 0x8u     /* below the root, cells of 5..list_max intervals are leaf lines, not deeper
                                    nodes (chosen automatically when deeper nodes would pass 64 MiB) */

/* Registry build options (NULL = defaults). */
typedef struct {
  uint32_t flags;          /* GNM_REG_HOST_ONLY: no device upload (inspection only) */
  uint32_t root_bits;      /* 0 = automatic (12); else 8..14 bits indexed by the LDS-resident top level */
  uint32_t list_max;       /* 0 = automatic (8); else 2..8 intervals per 64-byte leaf line */
  uint32_t lds_bytes;      /* 0 = automatic (163840); else the LDS budget, at most 163840 bytes, of the
                              root table, accumulator table and leaf lines: what does not fit stays in
                              device memory */
  uint32_t node_bits;      /* 0 = automatic (12, or 8 when 12-bit first-level nodes would pass 256 MiB);
                              else 4..16 index bits of the wide nodes just below the root (deeper nodes
                              use 8) */
} gnm_registry_opts;

/* Facts about a built registry. */
typedef struct {
  uint64_t n_prefixes_in;   /* prefixes passed in */
  uint64_t n_prefixes;      /* distinct normalised prefixes */
  uint64_t n_host_bits;     /* prefixes that had host bits set (cleared) */
  uint64_t n_duplicates;    /* exact duplicates for the same site (dropped) */
  uint64_t n_intervals;     /* maximal address intervals with one answer */
  uint64_t n_nodes;         /* wide inner nodes below the root */
  uint64_t n_leaf_lines;    /* 64-byte leaf lines (up to 8 intervals each) */
  uint64_t device_bytes;    /* device memory held by the registry */
  uint32_t n_sites;
  uint32_t n_local_ranges;  /* disjoint address ranges of the local set */
  uint32_t root_bits;
  uint32_t list_max;
  uint32_t lines_in_lds;    /* 1 if leaf lines are staged into LDS */
  uint32_t acc_in_lds;      /* 1 if the whole per-block accumulator table fits LDS */
  uint32_t lds_bytes;       /* LDS a classify workgroup uses */
  uint32_t cache_slots;     /* acc_in_lds == 0: rows a workgroup caches in LDS (first claim wins; the other
                               rows update the device table directly) */
  uint32_t node_bits;       /* index bits of first-level wide nodes */
  uint32_t reserved;
} gnm_registry_info;

typedef struct gnm_registry gnm_registry; /* opaque, immutable after build */

/*
 * gnm_registry_build — §III.B.1 (Site Registration Thread) and §III.B.2
 * (Catalog Kernel: a read-only lookup structure, rebuilt from scratch).
 *   sites[n_prefixes]  host array of site prefixes (site < n_sites).
 *   n_sites            number of collaboration sites (1 .. 2^28).
 *   local[n_local]     host array of local-site prefixes (site ignored);
 *                      n_local may be 0 (then every record is NODIR).
 *   opts               NULL or build options.
 *   stream             stream for the device upload; the call synchronises it
 *                      before returning (registry builds are not on the hot path).
 *   out                receives the handle; free it with gnm_registry_free.
 * Host bits are cleared; duplicates for one site are merged; the same
 * (network, length) for two sites is GNM_E_CONFLICT.  The handle is immutable
 * and may be shared by concurrent calls on any streams of its device.
 */
int gnm_registry_build(const gnm_prefix *sites, uint64_t n_prefixes, uint32_t n_sites,
                       const gnm_prefix *local, uint32_t n_local,
                       const gnm_registry_opts *opts, hipStream_t stream,
                       gnm_registry **out);

/* Free a registry (NULL is a no-op).  The caller must ensure no enqueued work
 * still uses it (synchronise the streams that used it first). */
int gnm_registry_free(gnm_registry *reg);

/* Describe a registry.  Host only. */
int gnm_registry_info_get(const gnm_registry *reg, gnm_registry_info *info);

/* Rows per window table: 2*(n_sites+1) + 1.  0 for a NULL registry. */
uint64_t gnm_acc_rows(const gnm_registry *reg);

/*
 * gnm_registry_lookup_host — walk the registry's lookup structure on the host
 * for n host addresses: site_out[i] = longest-match site (n_sites if none),
 * local_out[i] = 1 if the address is local (either output may be NULL).
 * For validating a built structure; the classify path never calls it.
 */
int gnm_registry_lookup_host(const gnm_registry *reg, const uint32_t *ip, uint64_t n,
                             uint32_t *site_out, uint8_t *local_out);

/* Defaults: bulk_bytes 1,000,000, no flags, automatic launch shape, no workspace. */
gnm_params gnm_params_default(void);

/*
 * gnm_workspace_bytes — size of the optional classify workspace for a launch
 * of grid_blocks workgroups (0 = the automatic maximum on the registry's
 * device).  With a workspace, each workgroup writes its final LDS table there
 * with plain stores and one small reduce kernel combines the tables; without
 * one, the tables are merged with device-scope 64-bit atomics, which give the
 * same result more slowly.  The workspace is caller-owned scratch: its
 * contents before and after a call do not matter, and two calls in flight at
 * the same time must not share one.  0 for a NULL registry.
 */
uint64_t gnm_workspace_bytes(const gnm_registry *reg, uint32_t grid_blocks);

/*
 * gnm_workspace_bytes_n — size of the classify workspace for a call over
 * n_records records in n_windows windows on grid_blocks workgroups (0 = the
 * automatic launch; the size fits every automatic launch of up to n_records
 * records).  For a registry whose table fits LDS it is gnm_workspace_bytes.
 * For one whose table does not (gnm_registry_info.acc_in_lds == 0), the
 * workspace holds the spilled rows instead: the rows that miss a workgroup's
 * LDS row cache and the cached rows flushed at window changes are staged as
 * 64-byte partial rows (at most one per record, and twice: staged, then in
 * partition order) and merged by one workgroup per (window, 256 table rows),
 * which writes its rows of the table and their flag bytes without
 * device-scope atomics: about 128 bytes per record.  Without that workspace
 * the rows go to the table with device-scope atomics, with the same results.
 * 0 for a NULL registry, n_windows = 0, or more than 16,384 (window, 256-row)
 * ranges (such calls always use the atomics).
 */
uint64_t gnm_workspace_bytes_n(const gnm_registry *reg, uint64_t n_records, uint32_t n_windows,
                               uint32_t grid_blocks);

/*
 * gnm_workspace_bytes_hist — size of the classify workspace for a call with
 * rate histograms (gnm_params.rate_hist) over n_records records in n_windows
 * windows on grid_blocks workgroups (0 = the automatic launch; the size fits
 * every automatic launch of up to n_records records): the tables' part,
 * gnm_workspace_bytes_n rounded up to 256 bytes, then the histograms' part.
 * With it (and a 256-byte aligned workspace) the classify kernel stages one
 * 4-byte key (the flow's row over all windows, its rate bucket) per bulk
 * flow of a registered site instead of counting it; the keys are ordered by
 * ranges of rows (twice 4 bytes per record, plus a partition count per
 * workgroup) and one workgroup per range (or per slice of 16,384 keys of a
 * range) counts them in LDS and writes the range's rows of rate_hist whole,
 * so no zeroing pass and no device-scope atomics are needed except for the
 * rows of ranges holding several slices.  Results are the same bit for bit.
 * Calls whose n_windows * 2 * n_sites rows pass 65,536, calls of 2^32 records
 * or more, and calls whose workspace is smaller keep the LDS cache and
 * device-scope atomics; for the first two this returns the tables' part
 * alone.  0 for a NULL registry or n_windows = 0.
 */
uint64_t gnm_workspace_bytes_hist(const gnm_registry *reg, uint64_t n_records, uint32_t n_windows,
                                  uint32_t grid_blocks);

/*
 * gnm_host_work_bytes — size of the work buffer of a gnm_host_table for a
 * classify call over n_records records on grid_blocks workgroups (0 = the
 * automatic launch; it fits every automatic launch of up to n_records
 * records).  The buffer holds one 32-byte entry per bulk flow of a
 * registered site (room for every record) twice, to stage the flows and to
 * order them by host partition, plus a partition count per workgroup: about
 * 64 bytes per record.  0 for a NULL registry.
 */
uint64_t gnm_host_work_bytes(const gnm_registry *reg, uint64_t n_records, uint32_t grid_blocks);

/*
 * gnm_classify_aggregate — §III.B.2 (TransRate Kernel) with the definition
 * above, for one or many windows in one launch.
 *   reg             registry built with a device upload.
 *   rec             device SoA records; rec->n records.
 *   window_offsets  NULL: one window [0, rec->n).  Otherwise a DEVICE array of
 *                   n_windows+1 uint64 with offsets[0] = 0, non-decreasing,
 *                   offsets[n_windows] = rec->n; window w is
 *                   [offsets[w], offsets[w+1]) (empty windows allowed).
 *                   Offsets outside [0, rec->n] are clamped; records are never
 *                   read out of bounds, but inconsistent offsets give
 *                   unspecified (not undefined) table contents.
 *   n_windows       >= 1 (must be 1 when window_offsets is NULL).
 *   p               NULL = gnm_params_default().
 *   acc             DEVICE array of n_windows * gnm_acc_rows(reg) rows,
 *                   window-major.  Initialised by the call unless
 *                   p->flags has GNM_ACCUMULATE (then added into).
 *   stream          the caller's stream.
 * Enqueues table initialisation (skipped when accumulating, or when a single
 * window is rebuilt entirely by the reduce step), histogram zeroing
 * (p->rate_hist set, not accumulating, and no workspace for the histograms),
 * the classify kernel, and (with a usable p->workspace) the reduce kernel.
 * With p->rate_hist, each bulk flow of a registered site also adds one to
 * its row's histogram: through an LDS cache and device-scope 32-bit atomics,
 * or, with a workspace of gnm_workspace_bytes_hist, as a staged key, which
 * four more kernels order by row and count (see gnm_workspace_bytes_hist);
 * the caller owns the histogram memory (n_windows * 2 * n_sites *
 * GNM_RATE_BUCKETS * 4 bytes).
 * With p->hosts, the classify kernel also stages each such flow (host key,
 * bytes, rate) in p->hosts->work, and four kernels follow: partition counts
 * by a hash of the key, their scan, the scatter into partition order, and one
 * workgroup per partition that gathers the hosts' statistics and medians in
 * LDS and writes them to the table.  Each classify workgroup walks a balanced contiguous slice of all
 * records, flushing its LDS table at window changes.  Errors: GNM_E_INVAL
 * (null pointers, n_windows = 0, offsets NULL with n_windows > 1,
 * records_per_thread not 0/1/2/4, n_windows tables beyond 2^39 words,
 * rate_hist not 16-byte aligned, a malformed host table or one with too
 * small a work buffer, hosts with GNM_ACCUMULATE or with 2^32 records or
 * more), GNM_E_UNSUPPORTED (host-only registry), GNM_E_HIP (launch failed).
 */
int gnm_classify_aggregate(const gnm_registry *reg, const gnm_records *rec,
                           const uint64_t *window_offsets, uint32_t n_windows,
                           const gnm_params *p, gnm_acc *acc, hipStream_t stream);

/*
 * gnm_flag_suboptimal — §III.B.1 (NetPerf Monitoring Thread) and §IV.B:
 * warn about sites whose transfer rate falls below a standard.
 *   acc             DEVICE tables of n_windows windows (as produced above).
 *   threshold_bps   e.g. 1,000,000 (1 Mbps, the paper's standard).
 *   min_bulk_flows  a (site, direction) needs at least max(1, min_bulk_flows)
 *                   bulk flows to be judged.
 *   flags           DEVICE array of n_windows * n_sites bytes, window-major:
 *                   bit 0 = inbound flagged, bit 1 = outbound flagged, where
 *                   flagged means floor(rate_sum_bps / bulk_flows) <
 *                   threshold_bps (strict).  The "no site" and NODIR rows are
 *                   never flagged.
 * Errors: GNM_E_INVAL (null pointers, n_windows = 0, a registry of another
 * device), GNM_E_UNSUPPORTED (host-only registry), GNM_E_HIP.
 */
int gnm_flag_suboptimal(const gnm_registry *reg, const gnm_acc *acc, uint32_t n_windows,
                        uint64_t threshold_bps, uint64_t min_bulk_flows, uint8_t *flags,
                        hipStream_t stream);

/*
 * gnm_classify_flag — one window step of §III.B.1 (NetPerf Monitoring
 * Thread) over §III.B.2 (TransRate Kernel): gnm_classify_aggregate(reg, rec,
 * window_offsets, n_windows, p, acc) followed by gnm_flag_suboptimal(reg,
 * acc, n_windows, threshold_bps, min_bulk_flows, flags), in one call with the
 * same results bit for bit.  With a usable p->workspace the mean-rate test
 * runs inside the reduce kernel on the rows it has just combined (no flag
 * launch); otherwise the flag kernel follows the classify kernel.  Arguments,
 * layouts and ownership are those of the two calls; flags is a DEVICE array
 * of n_windows * n_sites bytes.  Errors: those of gnm_classify_aggregate, and
 * GNM_E_INVAL for a NULL flags.
 */
int gnm_classify_flag(const gnm_registry *reg, const gnm_records *rec, const uint64_t *window_offsets,
                      uint32_t n_windows, const gnm_params *p, gnm_acc *acc, uint64_t threshold_bps,
                      uint64_t min_bulk_flows, uint8_t *flags, hipStream_t stream);

/*
 * gnm_classify_flag_static — gnm_classify_flag for callers that cannot
 * allocate device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc).  Same arguments, results and errors,
 * except that the workspace is not the caller's: the per-workgroup partial
 * tables (and, when they fit after them, the spilled rows of a table beyond
 * LDS or the staged keys of rate histograms; otherwise those use device-scope
 * atomics, with the same results) live in a static device array of
 * gnm_static_scratch_bytes() bytes (32 MiB) that the library holds on each
 * GPU it runs on until the process ends.  The call itself allocates nothing (no hipMalloc, hipFree or
 * allocating library routine); the array's device address is looked up once
 * per device, on the first call made with that device current.
 *   p->workspace    must be NULL (GNM_E_INVAL otherwise).
 * A launch whose partial tables (gnm_workspace_bytes(reg, grid)) would pass
 * the array's size is rejected with GNM_E_INVAL before anything is enqueued:
 * lower p->grid_blocks.  Registries whose table does not fit LDS need no
 * partial tables and are never rejected for size.  Every call on one GPU
 * shares that GPU's array, which keeps the last call's contents: calls whose
 * work overlaps on one GPU (concurrent streams, or graphs replayed
 * concurrently) race on it and give unspecified tables.  Serialise them.
 */
int gnm_classify_flag_static(const gnm_registry *reg, const gnm_records *rec, const uint64_t *window_offsets,
                             uint32_t n_windows, const gnm_params *p, gnm_acc *acc, uint64_t threshold_bps,
                             uint64_t min_bulk_flows, uint8_t *flags, hipStream_t stream);

/* Size in bytes of the static scratch array of gnm_classify_flag_static. */
uint64_t gnm_static_scratch_bytes(void);

/*
 * gnm_median_flags — the paper's warning criterion (§III.B.1, NetPerf
 * Monitoring Thread; §IV.B): a site is warned about when the median of its
 * transfer rates stays below a standard (1 Mbps) for two consecutive windows
 * (the paper's hours).
 *   rate_hist       DEVICE histograms of n_windows windows, as filled by
 *                   gnm_classify_aggregate with p->rate_hist.
 *   threshold_bps   e.g. 1,000,000.
 *   min_bulk_flows  a (site, direction) needs at least max(1, min_bulk_flows)
 *                   bulk flows (its histogram's total) to be judged.
 *   prev_flags      NULL, or a DEVICE array of n_sites flag bytes of the
 *                   window just before the first one (bits 0/1 are read), so
 *                   that consecutive calls chain across their boundary.
 *   median_bucket   NULL, or a DEVICE array of n_windows * 2 * n_sites uint32,
 *                   window-major by row 2*site+dir: the lower median bucket,
 *                   i.e. the smallest bucket m whose cumulative count reaches
 *                   ceil(N/2) of the row's N bulk flows; GNM_NO_MEDIAN when
 *                   N = 0.  The median rate lies in [m * 10 kbps, (m+1) *
 *                   10 kbps), or above 100 Mbps for the last bucket.
 *   flags           DEVICE array of n_windows * n_sites bytes, window-major:
 *                   bit d (0 inbound, 1 outbound) = the row is judged and
 *                   m * 10,000 < threshold_bps (exactly "median below the
 *                   threshold" when the threshold is a multiple of 10 kbps);
 *                   bit 2 + d = bit d is set in this window and in the one
 *                   before it (the warning).
 * Enqueues two kernels: the medians and low bits (one workgroup per
 * (window, site), reading each histogram once), then the two-window rule
 * (one lane per site).  Errors: GNM_E_INVAL (null pointers, n_windows = 0,
 * a registry of another device), GNM_E_UNSUPPORTED (host-only registry),
 * GNM_E_HIP.
 */
int gnm_median_flags(const gnm_registry *reg, const uint32_t *rate_hist, uint32_t n_windows,
                     uint64_t threshold_bps, uint64_t min_bulk_flows, const uint8_t *prev_flags,
                     uint32_t *median_bucket, uint8_t *flags, hipStream_t stream);

/* ------------------------------------------------------------------ batched form
 * Many windows of uneven size go through one persistent classify launch (see
 * gnm_classify_aggregate with window offsets); the paper instead launches once
 * per hourly window (§III.B.1, NetPerf Monitoring Thread).  For a step that
 * repeats over the same buffers, the launch sequence can be captured once into
 * a HIP graph and replayed.
 */
typedef struct gnm_graph gnm_graph; /* opaque */

/*
 * gnm_graph_create — capture one step: gnm_classify_aggregate(reg, rec,
 * window_offsets, n_windows, p, acc), or, when flags is not NULL,
 * gnm_classify_flag(reg, rec, window_offsets, n_windows, p, acc,
 * threshold_bps, min_bulk_flows, flags).  All pointers (records, offsets, acc, flags, p->workspace,
 * p->rate_hist) are
 * baked into the graph: every replay reads and writes those same buffers,
 * whose contents the caller may change between replays.  The call validates
 * the arguments and sets up the kernels without running the step (so a step
 * with GNM_ACCUMULATE adds once per replay, and only then); the first replay
 * computes the results.  Errors: those of the two captured calls, GNM_E_HIP.
 */
int gnm_graph_create(const gnm_registry *reg, const gnm_records *rec, const uint64_t *window_offsets,
                     uint32_t n_windows, const gnm_params *p, gnm_acc *acc, uint64_t threshold_bps,
                     uint64_t min_bulk_flows, uint8_t *flags, gnm_graph **out);

/* Replay a captured step on `stream`.  Replays on one graph must not overlap
 * (they share buffers). */
int gnm_graph_launch(gnm_graph *g, hipStream_t stream);

/* Free a graph (NULL is a no-op); its replays must have completed. */
int gnm_graph_free(gnm_graph *g);

#define GNM_TUNE_MAX 16
/* Result of gnm_autotune: the fastest parameters and every timing taken. */
typedef struct {
  gnm_params best;                         /* base parameters with the best launch shape */
  float best_ms;                           /* median classify-call time of `best` */
  uint32_t n_tried;
  float ms[GNM_TUNE_MAX];                  /* median time of candidate i */
  uint32_t records_per_thread[GNM_TUNE_MAX];
  uint32_t grid_blocks[GNM_TUNE_MAX];      /* 0 = automatic */
} gnm_tune_result;

/*
 * gnm_autotune — time gnm_classify_aggregate on the caller's own records for
 * candidate launch shapes (records per lane 4, 2, 1 x automatic, half, double
 * and quadruple workgroup counts), each as a warm-up plus the median of `reps`
 * (0 = 3) timed calls on `stream`, and return the fastest.  acc is
 * overwritten (initialised per call unless base->flags has GNM_ACCUMULATE,
 * in which case it accumulates every timed call).  Without a workspace
 * every candidate merges with atomics; with base->workspace set, candidates
 * whose workgroup count needs more workspace than base->workspace_bytes are
 * skipped, so every shape timed merges the way the tuned launch with that
 * workspace will.
 * Synchronous.  Errors: those of gnm_classify_aggregate, GNM_E_HIP.
 */
int gnm_autotune(const gnm_registry *reg, const gnm_records *rec, const uint64_t *window_offsets,
                 uint32_t n_windows, const gnm_params *base, gnm_acc *acc, uint32_t reps,
                 hipStream_t stream, gnm_tune_result *out);

/* ------------------------------------------------------------------ NetFlow v5 ingest
 * The step before the path: router export datagrams (§III.B.1, FlowData
 * Receiver Thread; §IV.A.3: NetFlow V5, 48-byte records, at most 30 per
 * datagram) decoded on the device into the structure-of-arrays records that
 * gnm_classify_aggregate reads.  Field layout: the public NetFlow version 5
 * export format, every field big-endian; a 24-byte header (version u16,
 * count u16, sys_uptime, unix_secs, unix_nsecs, flow_sequence u32,
 * engine_type u8, engine_id u8, sampling_interval u16) and 48-byte records
 * (srcaddr, dstaddr, nexthop u32, input, output u16, dPkts, dOctets, First,
 * Last u32, srcport, dstport u16, pad1, tcp_flags, prot, tos u8, src_as,
 * dst_as u16, src_mask, dst_mask u8, pad2 u16).  Decoded: src_ip = srcaddr,
 * dst_ip = dstaddr, packets = dPkts, bytes = dOctets (zero-extended),
 * first_ms = First, last_ms = Last, ports, proto = prot.
 */

/* Writable SoA record arrays (DEVICE pointers) of `capacity` records. */
typedef struct {
  uint32_t *src_ip;
  uint32_t *dst_ip;
  uint16_t *src_port; /* may be NULL (not written) */
  uint16_t *dst_port; /* may be NULL (not written) */
  uint8_t *proto;     /* may be NULL (not written) */
  uint64_t *bytes;
  uint32_t *packets;
  uint32_t *first_ms;
  uint32_t *last_ms;
  uint64_t capacity;
} gnm_records_out;

/* Scratch bytes gnm_netflow_v5_decode needs for n_datagrams datagrams. */
uint64_t gnm_netflow_v5_workspace_bytes(uint64_t n_datagrams);

/*
 * gnm_netflow_v5_decode — decode datagrams stored back to back.
 *   datagrams       DEVICE buffer of buf_bytes bytes, 4-byte aligned.
 *   offsets         DEVICE array of n_datagrams+1 uint64 (8-byte aligned):
 *                   datagram d spans [offsets[d], offsets[d+1]).
 *   workspace       DEVICE scratch of gnm_netflow_v5_workspace_bytes(n)
 *                   bytes, 256-byte aligned, caller-owned (contents do not
 *                   matter; calls in flight must not share one).
 *   out             output arrays; record j of the accepted datagrams, in
 *                   datagram order, goes to index j if j < out->capacity
 *                   (later records are dropped).
 *   n_records       DEVICE uint64 (8-byte aligned): records the accepted
 *                   datagrams carry (may exceed out->capacity).
 *   n_rejected      DEVICE uint64 (8-byte aligned): datagrams rejected.
 * A datagram is accepted when its span lies in the buffer, starts at a
 * multiple of 4, holds the header, carries version 5 and a count of 1..30,
 * and holds count records (bytes after them are ignored).  Enqueues five
 * kernels on `stream` (count, three scan passes, decode).  Errors:
 * GNM_E_INVAL (null pointers, misaligned buffer, offsets, counters or
 * workspace, workspace too small, more than 2^31 datagrams), GNM_E_HIP.
 */
int gnm_netflow_v5_decode(const uint8_t *datagrams, uint64_t buf_bytes, const uint64_t *offsets,
                          uint64_t n_datagrams, void *workspace, uint64_t workspace_bytes,
                          const gnm_records_out *out, uint64_t *n_records, uint64_t *n_rejected,
                          hipStream_t stream);

/* Static description of an error code. */
const char *gnm_strerror(int code);

/* Text of the last HIP error seen by this thread ("" if none). */
const char *gnm_last_error(void);

/* Library version string. */
const char *gnm_version(void);

#ifdef __cplusplus
}
#endif

#endif /* GNM_H */
