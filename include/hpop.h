/*
 * hpop: heterogeneous POP efficiency metrics on an AMD Instinct MI355X (gfx950).
 *
 * C ABI of the engine that reduces timestamped traces of host states and
 * device activity to the two metric trees of Rahimi et al., "Hardware-
 * Agnostic and Insightful Efficiency Metrics for Accelerated Systems"
 * (arXiv 2603.26576):
 *
 *   host tree (Section 4.1, eqs. 6-8)
 *     Parallel Efficiency            = sum_i U_i / (n E)                 (eq. 6)
 *     +- MPI Parallel Efficiency     = sum_i (U_i + W_i) / (n E)         (eq. 7)
 *     |  +- Communication Efficiency = max_i (U_i + W_i) / E             (eq. 5, U+W useful)
 *     |  +- Load Balance             = sum_i (U_i + W_i) / (n max(U+W))  (eq. 4, U+W useful)
 *     +- Device Offload Efficiency   = sum_i U_i / sum_i (U_i + W_i)     (eq. 8)
 *   device tree (Section 4.1, eqs. 9-12)
 *     Parallel Efficiency            = sum_g K_g / (m E)                 (eq. 9)
 *     +- Load Balance                = sum_g K_g / (m max K)             (eq. 10)
 *     +- Communication Efficiency    = max K / max (K + M)               (eq. 11)
 *     +- Orchestration Efficiency    = max (K + M) / E                   (eq. 12)
 *
 * U, W and MPI are the host states Useful, Device Offloading and MPI; K and M
 * are device Kernel and Memory-operation time. Device records are flattened
 * as in Section 4.2: overlapping kernels of any streams count once, memory
 * operations under kernels are removed, uncovered time is idle. Host records
 * overlap with the priority Useful > Offloading > MPI; host time covered by
 * no record is "Other". E is the region length t1 - t0.
 *
 * Every interval is half-open [start, end) in int64 nanoseconds, with
 * 0 <= start <= end < 2^62. A ratio whose denominator is 0 is defined as 1.0
 * and its bit is set in hpop_metric_tree.undefined_mask (bit j = j-th ratio
 * in the order of the struct fields).
 *
 * Errors: every call returns an hpop_status (0 = OK, negative = error); no
 * exception crosses the ABI; a failed call leaves the session unchanged
 * except where a function says otherwise. hpop_last_error() gives a message.
 * Sessions are not thread-safe (one thread at a time per session); the
 * server is thread-safe.
 */
#ifndef HPOP_H
#define HPOP_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t hpop_status;
#define HPOP_OK 0
#define HPOP_E_ARG (-1)          /* null pointer, negative count, bad flag */
#define HPOP_E_KIND (-2)         /* unknown kind, or host kind on a device resource and vice versa */
#define HPOP_E_RESOURCE (-3)     /* resource id outside 0 .. n_hosts+n_devices-1 */
#define HPOP_E_BAD_INTERVAL (-4) /* start > end, start < 0 or end >= 2^62 */
#define HPOP_E_REGION (-5)       /* t0 >= t1, or an unknown region id */
#define HPOP_E_OVERFLOW (-6)     /* (t1 - t0) * max(n, m) >= 2^53: ratios would not be exact */
#define HPOP_E_OOM (-7)          /* device or host allocation failed */
#define HPOP_E_BUSY (-8)         /* server queue full (back-pressure); retry later */
#define HPOP_E_HIP (-9)          /* a HIP runtime call failed; the message names it */
#define HPOP_E_TIMEOUT (-10)     /* hpop_server_wait timed out; the ticket stays valid */
#define HPOP_E_STATE (-11)       /* call not valid in the current state */

/* record kinds (Section 4.1 host states and device states) */
#define HPOP_HOST_USEFUL 0   /* host computing */
#define HPOP_HOST_OFFLOAD 1  /* host blocked in a device runtime call: launch, copy, synchronisation */
#define HPOP_HOST_MPI 2      /* host inside MPI */
#define HPOP_DEV_KERNEL 3    /* device executing a kernel (any stream) */
#define HPOP_DEV_MEMOP 4     /* device memory operation: memcpy H2D/D2H/D2D, memset */

/* where the caller's arrays live */
#define HPOP_MEM_HOST 0
#define HPOP_MEM_DEVICE 1

/* flags of hpop_metrics_compute_all and hpop_batch_compute */
#define HPOP_FORCE_REBUILD 1u /* rebuild the merged interval lists even if no record was added */
#define HPOP_NO_GRAPH 2u      /* launch the kernels one by one instead of replaying the captured HIP graph */

typedef struct hpop_session hpop_session;
typedef struct hpop_server hpop_server;

/* Optional device allocator. `stream` is the hipStream_t the memory is used on.
 * alloc returns NULL when it cannot serve the request: the call that needed the
 * memory then fails with HPOP_E_OOM and leaves the session as it was. free may
 * be handed a block that work already queued on `stream` still uses: it must
 * not reuse the block before that stream passes this point (a stream-ordered
 * free, or a synchronisation of `stream` first). */
typedef void* (*hpop_alloc_fn)(void* ctx, size_t bytes, void* stream);
typedef void (*hpop_free_fn)(void* ctx, void* ptr, void* stream);

typedef struct {
    int32_t n_hosts;       /* n: host processes, resource ids 0 .. n-1 */
    int32_t n_devices;     /* m: devices, resource ids n .. n+m-1 */
    void* stream;          /* hipStream_t for all work; NULL: the session creates one */
    hpop_alloc_fn alloc;   /* NULL: hipMallocAsync on the session stream */
    hpop_free_fn free;
    void* alloc_ctx;
} hpop_session_config;

/* One region's metric trees with the exact integer aggregates they come from. */
typedef struct {
    int64_t E;                    /* region length t1 - t0 */
    int32_t n, m;                 /* host processes and devices counted */
    int64_t sumU, sumW, sumMPI, sumOther;
    int64_t sumUW, maxUW;         /* sum and max over hosts of U + W */
    int64_t sumK, sumM, maxK, maxKM;
    double host_pe, host_mpi_pe, host_mpi_lb, host_mpi_ce, host_oe;  /* bits 0-4 */
    double dev_pe, dev_lb, dev_ce, dev_oe;                            /* bits 5-8 */
    uint32_t undefined_mask;
    uint32_t reserved;
} hpop_metric_tree;

/* Tuning of the reduction kernels (see hpop_autotune). Zero fields keep defaults. */
typedef struct {
    int32_t bucket_target;  /* records per time bucket of a resource, before rounding the bucket
                               count up to a power of two (16 .. 4096) */
    int32_t bucket_cap;     /* records a bucket may hold for the on-chip sort: 2048 or 4096 */
    int32_t tile_elems;     /* records per workgroup in the streaming passes: 512, 2048, 4096 or 8192 */
    int32_t scatter_slots;  /* records reserved per bucket by the single-pass scatter: 0 = 4 x
                               bucket_target (at most bucket_cap), -1 = always count first
                               (exact two-pass). A bucket that outgrows its slots makes the
                               build rerun with exact counts. */
} hpop_tuning;

/* Counters of one session (sizes of the last build). */
typedef struct {
    int64_t n_events;       /* records added */
    int64_t n_chunks;       /* add_events calls kept */
    int64_t n_buckets;      /* time buckets of the last build */
    int64_t n_oversized;    /* buckets of the last build too large for the on-chip sort */
    int64_t n_components;   /* merged intervals written by the last build, all levels */
    int32_t n_regions;
    int32_t graph_replays;  /* builds served by replaying a captured HIP graph */
    int64_t n_wide_components; /* of n_components, those stored in the 16 B form (resources
                                  whose time buckets are wider than 2^30 ns); the rest take 8 B */
    int64_t n_wide_records; /* records of the last build regrouped in the 16 B form (wide
                               buckets, or an end 2^32 - 1 ns or more past the bucket start);
                               the rest take 8 B */
} hpop_session_info;

/* One batch of records of one kind on one resource (hpop_add_events_multi,
 * hpop_server_submit). */
typedef struct {
    int32_t resource;
    int32_t kind;
    const int64_t* start;
    const int64_t* end;
    int64_t count;
} hpop_event_chunk;

/* Renderings of a metric tree (host code, no device work): the two trees of
 * the paper's metric tables (Sec. 4.1; host PE -> {MPI PE -> {LB, CE},
 * Device Offload Eff.}, device PE -> {LB, CE, Orchestration Eff.}) as
 * indented text, or as one JSON object with the ratios, the integer times and
 * the list of 0/0 ratios. Writes at most cap bytes including the terminating
 * NUL (cap = 0: nothing written); *needed (optional) receives the full size
 * including the NUL. HPOP_E_ARG for a null tree, an unknown format, or a
 * null buffer with cap > 0. */
#define HPOP_FORMAT_TEXT 0
#define HPOP_FORMAT_JSON 1
hpop_status hpop_tree_format(const hpop_metric_tree* tree, int32_t format, char* buf, int64_t cap,
                             int64_t* needed);

/* Status text; never NULL. */
const char* hpop_status_string(hpop_status status);
/* Last error message of a session (owned by the session, valid until its next call);
 * with s == NULL the calling thread's last error of a session-less call. */
const char* hpop_last_error(const hpop_session* s);

/* Create a session for n hosts and m devices (both fixed; resources without
 * records still count in n and m). The HIP device current on the calling
 * thread is used. */
hpop_status hpop_session_create(const hpop_session_config* cfg, hpop_session** out);
hpop_status hpop_session_destroy(hpop_session* s);

/* Append `count` records of one kind on one resource (Section 4.2: records
 * arrive in batches, in any order). start/end are HPOP_MEM_HOST or
 * HPOP_MEM_DEVICE pointers to int64 arrays; they are copied before the call
 * returns (host) or in stream order on the session stream (device: the
 * caller must not overwrite them until that stream passes this call).
 * Host input is validated here (HPOP_E_BAD_INTERVAL names the index);
 * device input is validated by the next build, which then fails with
 * HPOP_E_BAD_INTERVAL naming the call and index, and drops that call's records. */
hpop_status hpop_add_events(hpop_session* s, int32_t resource, int32_t kind,
                            const int64_t* start, const int64_t* end, int64_t count,
                            int32_t mem_space);
/* Several hpop_add_events calls at once (one staging copy for host input).
 * Either every chunk is added or, on error, none is. */
hpop_status hpop_add_events_multi(hpop_session* s, const hpop_event_chunk* chunks, int32_t n_chunks,
                                  int32_t mem_space);
/* Wait until the session stream has passed every call made so far (after
 * which device arrays given to hpop_add_events may be reused). */
hpop_status hpop_session_synchronize(hpop_session* s);
/* Drop every record (regions are kept). */
hpop_status hpop_clear_events(hpop_session* s);

/* A user region [t0, t1) (Section 3.2: regions of interest annotated by the
 * user). Returns its id (0, 1, ...). */
hpop_status hpop_region_define(hpop_session* s, int64_t t0, int64_t t1, int32_t* out_region);
hpop_status hpop_num_regions(const hpop_session* s, int32_t* out);
/* A region entered repeatedly, each resource on its own clock (regions that
 * processes enter and leave through TALP's user-level API, Sec. 3.2):
 * `count` intervals [t0[i], t1[i]) of resource[i] (0 .. n+m-1; intervals of one
 * resource must not overlap; resources without intervals are outside the
 * region). A resource's state times are measured over its own intervals and
 * its remainder (Other / Idle) completes its own time in the region. E is
 * eq. 1 read literally: the largest in-region time of a host process (of a
 * device when no host process has an interval). Errors: HPOP_E_ARG (null
 * pointer, count < 1), HPOP_E_RESOURCE, HPOP_E_REGION (t0 >= t1, overlap,
 * bounds outside [-2^62, 2^62]), HPOP_E_OVERFLOW (E * max(n, m) >= 2^53). */
hpop_status hpop_region_define_multi(hpop_session* s, const int32_t* resource, const int64_t* t0,
                                     const int64_t* t1, int64_t count, int32_t* out_region);

/* Metric trees of one region / of every region (out: hpop_num_regions entries).
 * Builds the merged interval lists first if records were added since the
 * last build (or with HPOP_FORCE_REBUILD), then clips every resource to the
 * region(s) and reduces. Blocks until the trees are in host memory. */
hpop_status hpop_metrics_compute(hpop_session* s, int32_t region, hpop_metric_tree* out);
hpop_status hpop_metrics_compute_all(hpop_session* s, uint32_t flags, hpop_metric_tree* out);

/* State times of one resource in one region after a compute:
 * host -> {Useful, Offloading, MPI, Other}, device -> {Kernel, Memory, Idle, 0}. */
hpop_status hpop_resource_times(hpop_session* s, int32_t region, int32_t resource, int64_t out[4]);

/* One region's report for a user (the run-time report of Sec. 3.2: the
 * metric trees with the raw times they come from): the rendering of
 * hpop_tree_format followed by every resource's state times in the region
 * (hosts: useful, offload, MPI, other; devices: kernels, memory operations,
 * idle), as text lines or as a "resources" array inside the JSON object.
 * Computes the region first, as hpop_metrics_compute does. Buffer rules as
 * hpop_tree_format. Errors: HPOP_E_ARG, HPOP_E_REGION, and those of
 * hpop_metrics_compute. */
hpop_status hpop_region_format(hpop_session* s, int32_t region, int32_t format, char* buf, int64_t cap,
                               int64_t* needed);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): one-shot
 * evaluation with no session and no allocation. The results are those of a
 * session with n_hosts hosts and n_devices devices, the chunks added with
 * HPOP_MEM_DEVICE, the regions [region_t0[g], region_t1[g]) defined in
 * order, then hpop_metrics_compute_all (trees into out[0..n_regions)) and
 * hpop_resource_times (into times_out, optional: [n_regions][n + m][4]).
 * Chunk arrays must be device memory and are read in place. Every
 * intermediate lives in a library-owned device array of
 * HPOP_STATIC_SCRATCH_BYTES per GPU, taken when the first call on that GPU
 * loads it and held until the process ends; each call overwrites it. A call
 * whose build needs more than that fails with HPOP_E_ARG (message in
 * hpop_last_error(NULL) with the size needed). Calls on one GPU share that
 * array: within a process they are serialised by the library; work of one
 * call overlapping another's on the same GPU by other means would race.
 * The call runs on `stream` (a hipStream_t, NULL for the null stream) and
 * synchronises it before returning. Errors: HPOP_E_ARG, HPOP_E_RESOURCE,
 * HPOP_E_KIND, HPOP_E_REGION, HPOP_E_OVERFLOW as for the session calls;
 * HPOP_E_BAD_INTERVAL naming the chunk and index of an invalid record (no
 * tree is written); HPOP_E_HIP. */
#define HPOP_STATIC_SCRATCH_BYTES ((size_t)256 << 20)
hpop_status hpop_metrics_compute_static(int32_t n_hosts, int32_t n_devices, const hpop_event_chunk* chunks,
                                        int32_t n_chunks, const int64_t* region_t0, const int64_t* region_t1,
                                        int32_t n_regions, void* stream, hpop_metric_tree* out,
                                        int64_t* times_out);

/* Batched evaluation: the records and regions of k sessions reduced together
 * in one launch sequence (captured once in a HIP graph and replayed while no
 * session changes). out receives every region of every session, session by
 * session, regions in id order. All sessions must use the same HIP device;
 * the work runs on the first session's stream. */
hpop_status hpop_batch_compute(hpop_session* const* sessions, int32_t k, uint32_t flags,
                               hpop_metric_tree* out);

hpop_status hpop_session_get_info(const hpop_session* s, hpop_session_info* out);
hpop_status hpop_session_set_tuning(hpop_session* s, const hpop_tuning* t);
hpop_status hpop_session_get_tuning(const hpop_session* s, hpop_tuning* out);

/* Per-kernel device time of the last build and clip, measured with HIP
 * events on the session stream when enabled (off by default).
 * names/ms receive up to `cap` entries; *n_out the number written. */
hpop_status hpop_session_enable_timing(hpop_session* s, int32_t on);
hpop_status hpop_session_stage_times(const hpop_session* s, int32_t cap, const char** names,
                                     float* ms, int32_t* n_out);
/* Time only one stage while timing is enabled (names as stage_times reports
 * them: "reset", "stats", "hist", "scan", "scatter", "carry", "merge_wave",
 * "merge_block", "base", "region"; with fixed scatter slots "scan" also
 * holds the carry pass, and "hist" and "carry" do not run): one event right
 * before its launches and one right after, instead of one after every stage,
 * so timing perturbs the build less. NULL or "" times every stage again. A
 * stage the build does not run yields no entry. HPOP_E_ARG for an unknown
 * name. Applies to the
 * session's own builds and to batched builds it leads. */
hpop_status hpop_session_time_stage(hpop_session* s, const char* stage);

/* Autotuner: times candidate tunings on the given sessions (batched when
 * k > 1), keeps the fastest, applies it to every session and returns it.
 * With cache_path != NULL the choice is read from / appended to that JSON
 * file ({"<size class>": [bucket_target, bucket_cap, tile_elems], ...}),
 * keyed by the workload's size class (log2 of records, resources and
 * sessions, rounded), so later calls skip the search. A cache file that
 * cannot be read, does not parse or holds a value outside the ranges of
 * hpop_tuning fails with HPOP_E_ARG (message in hpop_last_error(NULL)); so
 * does a failed trial build or a cache that cannot be written, and in every
 * failing case the sessions keep the tunings they had. */
hpop_status hpop_autotune(hpop_session* const* sessions, int32_t k, const char* cache_path,
                          hpop_tuning* out);

/* ----------------------------------------------------------------------------
 * Stream concurrency. The paper counts each device as one resource and leaves
 * its streams to a future Device Computational Efficiency branch (Sec. 4.1),
 * so this measure is the library's own definition. For device g with S_g
 * declared streams and a region [t0, t1):
 *   B_g  = time during which at least one of its streams runs a kernel
 *   ST_g = sum over its streams of the time that stream runs a kernel
 *          (the integral of the number of active streams)
 * and over the devices:
 *   stream_eff  = sum ST_g / sum S_g B_g   (1: every declared stream runs
 *                 whenever its device runs a kernel; 1/S: one at a time)
 *   mean_active = sum ST_g / sum B_g        (mean active streams while busy)
 * Each ratio is one IEEE division of exact integers; 0/0 is 1 with its bit
 * (0, 1) set. Records of one stream that overlap count once.
 * -------------------------------------------------------------------------- */

typedef struct {
    int64_t busy;          /* sum over devices of B_g */
    int64_t stream_time;   /* sum over devices of ST_g */
    int64_t capacity;      /* sum over devices of S_g * B_g */
    int32_t m;             /* devices */
    int32_t n_streams;     /* sum over devices of S_g */
    double stream_eff;     /* bit 0 */
    double mean_active;    /* bit 1 */
    uint32_t undefined_mask;
    uint32_t reserved;
} hpop_stream_tree;

/* Declares S_g = n_streams[g] >= 0 streams on each of the session's devices
 * (array of n_devices; stream ids 0 .. S_g - 1; sum of S_g + 1 at most 2^24).
 * May be called again only while no stream record was added (HPOP_E_STATE).
 * Errors: HPOP_E_ARG (null, negative or too many streams). */
hpop_status hpop_session_set_streams(hpop_session* s, const int32_t* n_streams);

/* Kernel records of one stream of one device: like hpop_add_events with kind
 * HPOP_DEV_KERNEL (they count in the device tree too), and kept by stream for
 * hpop_stream_metrics. Same memory rules and validation as hpop_add_events.
 * Errors: HPOP_E_STATE (no hpop_session_set_streams), HPOP_E_RESOURCE (not a
 * device, or stream outside 0 .. S_g - 1), HPOP_E_ARG, HPOP_E_BAD_INTERVAL;
 * a failed call adds nothing. */
hpop_status hpop_add_stream_events(hpop_session* s, int32_t resource, int32_t stream, const int64_t* start,
                                   const int64_t* end, int64_t count, int32_t mem_space);

/* Stream concurrency of every region (out[n_regions]) and, if per_device is
 * not NULL, per region and device the triple (B_g, ST_g, S_g)
 * (int64[n_regions][n_devices][3]). flags as hpop_metrics_compute_all.
 * Errors: HPOP_E_STATE (no hpop_session_set_streams), HPOP_E_REGION (a region
 * of hpop_region_define_multi: stream measures need one span per region),
 * HPOP_E_OVERFLOW ((t1 - t0) * sum S_g >= 2^53), HPOP_E_BAD_INTERVAL (an
 * invalid device-memory record), HPOP_E_OOM, HPOP_E_HIP. */
hpop_status hpop_stream_metrics(hpop_session* s, uint32_t flags, hpop_stream_tree* out, int64_t* per_device);

/* ----------------------------------------------------------------------------
 * Serving runtime (online analysis: Section 3.2 describes TALP's run-time
 * queries; Section 4.2 its batched, asynchronously delivered device records).
 *
 * The server keeps each session's merged interval lists resident in device
 * memory. A submitted query carries new records of one session and closes a
 * region [t0, t1); the server merges the records into the session state
 * incrementally and returns the metric trees of that region and of the
 * session's whole span so far. Queries of different sessions are admitted
 * while others run (continuous batching) and reduced together; queries of one
 * session are applied in submission order. The result of a query depends only
 * on the records submitted to its session up to and including it.
 * -------------------------------------------------------------------------- */

typedef struct {
    int32_t max_sessions;       /* sessions the server may open */
    int32_t max_inflight;       /* queries admitted per device step (1 .. 4096) */
    int32_t queue_capacity;     /* queued queries before hpop_server_submit returns HPOP_E_BUSY */
    int32_t host_staging_mib;   /* page-locked MiB holding host payloads of queued queries: > 0 taken at
                                   hpop_server_create; 0: 1024 MiB taken at the first host payload */
    int64_t mem_budget_bytes;   /* device bytes for staged records of admitted queries */
    int64_t list_heap_bytes;    /* device bytes taken at creation for the session lists (0: grown on
                                   demand); lists move within it as they grow and are compacted into
                                   a new heap only when it is full */
} hpop_server_config;

typedef struct {
    int64_t completed;          /* queries finished */
    int64_t events;             /* records merged */
    int64_t device_steps;       /* batched device steps run */
    double mean_batch;          /* mean queries per device step */
    double p50_us, p99_us, max_us;  /* submit -> result latency of finished queries */
    double max_submit_us;       /* longest hpop_server_submit (host payloads: includes their copy) */
    double max_step_us;         /* longest device step of the worker, admission to results */
    int64_t host_staging_bytes; /* page-locked staging area of host payloads (0 before it is taken) */
    double max_pinned_alloc_us; /* its allocation */
    int64_t max_host_staging_used; /* most of it held by queued payloads at once */
    /* Longest time of each phase of one device step. Host clocks: prep =
     * admission to the first enqueue (planning, growth of device buffers),
     * grow = the device allocations within prep, wait = the worker blocked on
     * the step's end. Device times (HIP events on the server stream): h2d =
     * host payload copies, build = bucketed build of the new records, move =
     * list moves, splice = the merge into the session lists, region = the
     * region trees and the copies of the results. */
    double max_prep_us, max_grow_us, max_wait_us;
    double max_h2d_us, max_build_us, max_move_us, max_splice_us, max_region_us;
    /* the same phases' mean per step */
    double mean_prep_us, mean_grow_us, mean_wait_us;
    double mean_h2d_us, mean_build_us, mean_move_us, mean_splice_us, mean_region_us;
    /* Longest single runtime call the worker made while enqueueing a step
     * (copies, kernel launches, event records; not the step's
     * synchronisation), in host time, and where: one of HPOP_CALL_*
     * (-1: none yet). */
    double max_call_us;
    int32_t max_call_site;
    int32_t reserved;
} hpop_server_stats;

/* Sites of hpop_server_stats.max_call_site. */
#define HPOP_CALL_EVENT 0    /* a phase's HIP event record */
#define HPOP_CALL_PAYLOAD 1  /* a host payload's copy to the device */
#define HPOP_CALL_MOVE 2     /* the list moves: table copy and kernel */
#define HPOP_CALL_BUILD 3    /* the build of the step's records: descriptor copies and kernels */
#define HPOP_CALL_TABLES 4   /* list, item and request table copies */
#define HPOP_CALL_CONTROL 5  /* the scratch control word's copy */
#define HPOP_CALL_SPLICE 6   /* the prep and splice kernels */
#define HPOP_CALL_REGION 7   /* the region kernel */
#define HPOP_CALL_RESULTS 8  /* the copies of trees, lists and error flags to the host */

hpop_status hpop_server_create(const hpop_server_config* cfg, hpop_server** out);
hpop_status hpop_server_destroy(hpop_server* srv);
/* Open a session of n hosts and m devices; t_origin is the start of its
 * global region. */
hpop_status hpop_server_open_session(hpop_server* srv, int32_t n_hosts, int32_t n_devices,
                                     int64_t t_origin, int32_t* out_sid);
/* Non-blocking. Records in `chunks` are HPOP_MEM_HOST (copied into the
 * server's page-locked staging area before return) or HPOP_MEM_DEVICE (read
 * by the server's stream; keep them unchanged until the ticket completes).
 * Records are validated on the device in both cases: a query holding an
 * invalid one (start < 0, start > end or end >= 2^62) is not applied and its
 * hpop_server_wait returns HPOP_E_BAD_INTERVAL. Returns HPOP_E_BUSY when the
 * queue, the memory budget or the staging area is full (nothing is copied
 * then); HPOP_E_ARG for a host payload larger than the whole staging area.
 * No call on this path allocates page-locked memory except the first host
 * payload's, when the staging area is taken then. */
hpop_status hpop_server_submit(hpop_server* srv, int32_t sid, const hpop_event_chunk* chunks,
                               int32_t n_chunks, int32_t mem_space, int64_t t0, int64_t t1,
                               uint64_t* out_ticket);
/* Wait for a ticket (timeout_ns < 0: forever). Writes the trees of the
 * query's region and of [t_origin, max end so far) of its session. */
hpop_status hpop_server_wait(hpop_server* srv, uint64_t ticket, int64_t timeout_ns,
                             hpop_metric_tree* out_region, hpop_metric_tree* out_global);
hpop_status hpop_server_get_stats(hpop_server* srv, hpop_server_stats* out);
/* Restart the statistics (counts, latencies, maxima, means) from now, e.g.
 * after a warm-up; the staging area's figures are kept. */
hpop_status hpop_server_reset_stats(hpop_server* srv);

/* One query of an arrival schedule replayed by hpop_server_replay. */
typedef struct {
    int32_t sid;
    int32_t n_chunks;
    const hpop_event_chunk* chunks;
    int64_t t0, t1;             /* the query's region, as for hpop_server_submit */
    int64_t arrival_ns;         /* arrival after the start of the replay; non-decreasing */
} hpop_replay_query;

/* Load generator without a host language in the loop: submits qs[0..n) from
 * the calling thread, each at its arrival time (retrying while the server
 * answers HPOP_E_BUSY), then waits for all of them. Per query (arrays of n
 * entries, each optional): the two trees as hpop_server_wait writes them,
 * and latency_ns = time from the scheduled arrival until the worker had the
 * trees on the host. out_wall_ns: start of the replay to the last completion;
 * out_busy: submissions refused with HPOP_E_BUSY. All queries are waited for
 * even when one fails; the first failing status is returned (its message in
 * hpop_server_last_error) and the trees of failed queries are left unchanged.
 * Record buffers follow the rules of hpop_server_submit for `mem_space`. */
hpop_status hpop_server_replay(hpop_server* srv, const hpop_replay_query* qs, int32_t n,
                               int32_t mem_space, hpop_metric_tree* out_region,
                               hpop_metric_tree* out_global, int64_t* latency_ns,
                               int64_t* out_wall_ns, int64_t* out_busy);
const char* hpop_server_last_error(const hpop_server* srv);

#ifdef __cplusplus
}
#endif
#endif /* HPOP_H */
