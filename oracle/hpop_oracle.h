/*
 * CPU oracle for the heterogeneous POP efficiency metrics.
 *
 * TEST INFRASTRUCTURE ONLY. Only the test-suite, the smoke check and the
 * benchmark's CPU-baseline leg may load this library. The GPU product path
 * never links, loads or calls it, and the two share no code.
 *
 * It computes, with a plain sort-and-sweep per resource, what the paper
 * defines:
 *   - host states Useful / Device Offloading / MPI (Section 4.1), device
 *     states Kernel / Memory operation / Idle (Section 4.1), with overlapping
 *     records of one resource flattened into one interval and memory
 *     operations hidden under kernels removed (Section 4.2, post-processing);
 *   - host metrics: Hybrid Parallel Efficiency (eq. 6), MPI Parallel
 *     Efficiency (eq. 7) with its Load Balance and Communication Efficiency
 *     children (eqs. 4 and 5 with Useful+Offloading as the useful state),
 *     Device Offload Efficiency (eq. 8);
 *   - device metrics: Parallel Efficiency (eq. 9), Load Balance (eq. 10),
 *     Communication Efficiency (eq. 11), Orchestration Efficiency (eq. 12).
 *
 * Every interval is half-open [start, end) in int64 nanoseconds.
 */
#ifndef HPOP_ORACLE_H
#define HPOP_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* kinds: host Useful, host Device Offloading, host MPI, device Kernel, device Memory op */
#define ORC_HOST_USEFUL 0
#define ORC_HOST_OFFLOAD 1
#define ORC_HOST_MPI 2
#define ORC_DEV_KERNEL 3
#define ORC_DEV_MEMOP 4

/* Error codes returned by oracle_compute. */
#define ORC_OK 0
#define ORC_E_ARG -1
#define ORC_E_KIND -2
#define ORC_E_INTERVAL -4
#define ORC_E_REGION -5
#define ORC_E_OOM -7

/*
 * Measure of the union of intervals [s[i], e[i]) clipped to each region
 * [t0[r], t1[r]). out[r] receives the measure for region r.
 */
int oracle_union_measure(const int64_t* s, const int64_t* e, int64_t n,
                         int32_t n_regions, const int64_t* t0, const int64_t* t1,
                         int64_t* out);

/*
 * Full evaluation of one trace.
 *   resources 0..n_hosts-1 are host processes, n_hosts..n_hosts+n_devices-1 devices;
 *   event i has resource[i], kind[i], start[i], end[i];
 *   times  : int64 [n_regions][n_hosts+n_devices][4]
 *            host   -> Useful, Offloading, MPI, Other (time covered by no host state)
 *            device -> Kernel, Memory, Idle, 0
 *   sums   : int64 [n_regions][10]
 *            sumU, sumW, sumMPI, sumOther, sumUW, maxUW, sumK, sumM, maxK, maxKM
 *   ratios : double [n_regions][9]
 *            host PE, MPI PE, MPI LB, MPI CE, Offload Eff,
 *            device PE, device LB, device CE, device Orchestration Eff
 *   mask   : uint32 [n_regions], bit j set when ratio j had a zero denominator
 *            (its value is then 1.0)
 *   n_threads > 1 spreads resources over POSIX threads (same arithmetic).
 */
int oracle_compute(int32_t n_hosts, int32_t n_devices, int64_t n_events,
                   const int32_t* resource, const int32_t* kind,
                   const int64_t* start, const int64_t* end,
                   int32_t n_regions, const int64_t* t0, const int64_t* t1,
                   int32_t n_threads,
                   int64_t* times, int64_t* sums, double* ratios, uint32_t* mask);

#ifdef __cplusplus
}
#endif
#endif
