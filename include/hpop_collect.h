/*
 * hpop_collect: a rocprofiler-sdk tool that records, inside a running HIP
 * application, the host and device states of the heterogeneous POP metrics
 * (Rahimi et al., arXiv 2603.26576), in the form hpop.h takes as input.
 *
 * What is recorded follows the paper's description of its tracing backends
 * (Section 4.2, its AMD backend): host runtime calls are seen synchronously, device
 * activity arrives asynchronously in buffers.
 *
 *   resource 0 (this process, a host):
 *     HPOP_HOST_OFFLOAD  every HIP runtime API call, from entry to return.
 *                        Only the outermost call of a thread counts, and
 *                        calls of different threads may overlap.
 *     HPOP_HOST_USEFUL   the rest of the process's time since the collector
 *                        started: the gaps between the offload calls of all
 *                        threads (Section 4.1: a host is Useful when it is
 *                        neither offloading nor in MPI).
 *     HPOP_HOST_MPI      none. No MPI layer is intercepted.
 *   resource 1 + g (GPU agent g, in the HIP device order):
 *     HPOP_DEV_KERNEL    kernel dispatches, from start to end timestamp.
 *     HPOP_DEV_MEMOP     memory copies that read or write that GPU (host to
 *                        device, device to host, and device to device, which
 *                        counts on both GPUs when they differ).
 *
 * Every time is an int64 nanosecond on rocprofiler's clock, which host and
 * device records share. Records are half-open [start, end) with
 * start <= end; a device record whose end precedes its start (never seen, but
 * not ruled out by the runtime) is kept with end = start.
 *
 * Loading. Either name the library in ROCP_TOOL_LIBRARIES when the process
 * starts (any HIP application, unchanged), or link it into the application.
 * rocprofiler-sdk then calls its configuration entry when the HIP runtime
 * starts. One configuration per process; later ones are declined.
 *
 * Output. At process exit (all records flushed), if HPOP_COLLECT_OUT names a path (a "%p" in it is
 * replaced by the process id), every record is written there in the format
 * below. An application can also take the records while it runs with
 * hpop_collect_poll / hpop_collect_count / hpop_collect_copy and hand them to
 * hpop_server_submit, region by region (self-profiling).
 *
 * Trace file (little-endian):
 *   char[8]  "HPOPTRC1"
 *   int32    n_hosts (1), n_devices
 *   int64    t_begin, t_end          the span the records cover
 *   int32    n_chunks
 *   n_chunks times:
 *     int32  resource, kind
 *     int64  count
 *     int64  start[count], end[count]
 *
 * Thread safety: every function may be called from any thread. The
 * functions make no HIP call, so they may be called while HIP work runs.
 */
#ifndef HPOP_COLLECT_H
#define HPOP_COLLECT_H

#include <stdint.h>

#include "hpop.h"

#ifdef __cplusplus
extern "C" {
#endif

/* 1 if rocprofiler-sdk configured this library in the current process (the
 * HIP runtime has started with the tool loaded), else 0. */
int32_t hpop_collect_active(void);

/* Device resources (GPU agents) of this process; 0 before configuration. */
int32_t hpop_collect_devices(void);

/* The collector's clock now, and the time it started recording (0 before
 * configuration). */
int64_t hpop_collect_now(void);
int64_t hpop_collect_begin(void);

/* Makes the host records up to a frontier final and returns the frontier:
 * the current time, or the start of the earliest offload call still running
 * in any thread if that is earlier. Every host record that starts before the
 * frontier is then known, so the Useful gaps up to it are appended. Takes
 * microseconds: device records are not flushed here. They arrive from
 * rocprofiler's buffers in completion order, delivered by the tool's own
 * thread every HPOP_COLLECT_FLUSH_MS milliseconds (environment, default 10;
 * 0 = only when a buffer fills), or at once by hpop_collect_flush; a kernel
 * that ends before the frontier may therefore be taken by a later poll.
 * Errors: HPOP_E_STATE before configuration, HPOP_E_ARG for a null pointer. */
hpop_status hpop_collect_poll(int64_t* out_frontier);

/* Delivers every device record the runtime has completed (blocks, typically
 * for milliseconds). Call it before a final poll to take everything.
 * HPOP_E_STATE before configuration. */
hpop_status hpop_collect_flush(void);

/* Records of (resource, kind) made final so far (0 for an unknown pair). */
int64_t hpop_collect_count(int32_t resource, int32_t kind);

/* Copies records [first, first + count) of (resource, kind), in the order they
 * were made final, into caller arrays start[count] and end[count] (host
 * memory). Errors: HPOP_E_ARG (null array with count > 0, first < 0,
 * count < 0), HPOP_E_RESOURCE / HPOP_E_KIND (unknown pair), HPOP_E_REGION
 * (first + count beyond hpop_collect_count). */
hpop_status hpop_collect_copy(int32_t resource, int32_t kind, int64_t first, int64_t count, int64_t* start,
                              int64_t* end);

/* Writes every final record to `path` in the trace file format, with
 * t_end = the last frontier. HPOP_E_ARG if the file cannot be written. */
hpop_status hpop_collect_write(const char* path);

/* Records dropped: device records rocprofiler reported lost, plus records that
 * could not be stored. */
int64_t hpop_collect_dropped(void);

#ifdef __cplusplus
}
#endif

#endif
