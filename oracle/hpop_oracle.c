/*
 * CPU oracle for the heterogeneous POP efficiency metrics (plain C).
 *
 * TEST INFRASTRUCTURE ONLY: loaded by the tests, the smoke check and the
 * benchmark's CPU-baseline leg, never by the product path. It shares no code
 * with the GPU engine.
 *
 * Per resource and per nested state level it collects the level's records,
 * sorts them by (start, end), sweeps them into disjoint merged intervals and
 * sums the merged intervals' overlap with each region. This is the
 * flattening the paper describes for device records (Section 4.2: records of
 * overlapping launches across streams become one continuous interval; memory
 * records overlapping kernels are removed; what no record covers is idle),
 * applied with the same priority rule on the host.
 *
 * Levels (each a union of kinds, nested):
 *   device: L1 = {Kernel}, L2 = {Kernel, Memory}
 *           Kernel = |L1|, Memory = |L2| - |L1|, Idle = E - |L2|
 *   host:   L1 = {Useful}, L2 = {Useful, Offloading}, L3 = {all three}
 *           Useful = |L1|, Offloading = |L2| - |L1|, MPI = |L3| - |L2|,
 *           Other = E - |L3|
 * where |L| is the measure of the level's union inside the region and
 * E = t1 - t0 is the region length.
 */
#include "hpop_oracle.h"

#include <pthread.h>
#include <stdlib.h>
#include <string.h>

typedef struct {
    int64_t s, e;
} orc_ivl;

static int orc_cmp(const void* a, const void* b) {
    const orc_ivl* x = (const orc_ivl*)a;
    const orc_ivl* y = (const orc_ivl*)b;
    if (x->s != y->s) return x->s < y->s ? -1 : 1;
    if (x->e != y->e) return x->e < y->e ? -1 : 1;
    return 0;
}

static int64_t orc_max(int64_t a, int64_t b) { return a > b ? a : b; }
static int64_t orc_min(int64_t a, int64_t b) { return a < b ? a : b; }

/* Sort, merge overlapping or touching intervals, then clip-sum per region. */
static void orc_measure_sorted(orc_ivl* v, int64_t n, int32_t n_regions,
                               const int64_t* t0, const int64_t* t1, int64_t* out) {
    for (int32_t r = 0; r < n_regions; ++r) out[r] = 0;
    if (n == 0) return;
    qsort(v, (size_t)n, sizeof(orc_ivl), orc_cmp);
    /* sweep: v[0..k) becomes the list of disjoint merged intervals */
    int64_t k = 0;
    orc_ivl cur = v[0];
    for (int64_t i = 1; i < n; ++i) {
        if (v[i].s <= cur.e) {
            cur.e = orc_max(cur.e, v[i].e);
        } else {
            v[k++] = cur;
            cur = v[i];
        }
    }
    v[k++] = cur;
    /* measure of (union intersect [t0, t1)) */
    for (int32_t r = 0; r < n_regions; ++r) {
        int64_t acc = 0;
        for (int64_t j = 0; j < k; ++j) {
            int64_t a = orc_max(v[j].s, t0[r]);
            int64_t b = orc_min(v[j].e, t1[r]);
            if (b > a) acc += b - a;
        }
        out[r] = acc;
    }
}

int oracle_union_measure(const int64_t* s, const int64_t* e, int64_t n,
                         int32_t n_regions, const int64_t* t0, const int64_t* t1,
                         int64_t* out) {
    if (n < 0 || n_regions < 0) return ORC_E_ARG;
    orc_ivl* v = (orc_ivl*)malloc(sizeof(orc_ivl) * (size_t)(n > 0 ? n : 1));
    if (!v) return ORC_E_OOM;
    int64_t k = 0;
    for (int64_t i = 0; i < n; ++i) {
        if (s[i] > e[i]) {
            free(v);
            return ORC_E_INTERVAL;
        }
        if (s[i] < e[i]) { /* an empty interval covers nothing */
            v[k].s = s[i];
            v[k].e = e[i];
            ++k;
        }
    }
    orc_measure_sorted(v, k, n_regions, t0, t1, out);
    free(v);
    return ORC_OK;
}

/* ------------------------------------------------------------------------ */

typedef struct {
    int32_t n_hosts, n_devices, n_regions;
    const int64_t* t0;
    const int64_t* t1;
    /* events grouped by resource: ev_off[r] .. ev_off[r+1] */
    const int64_t* ev_off;
    const int32_t* g_kind;
    const int64_t* g_s;
    const int64_t* g_e;
    int64_t* times;
    int32_t tid, n_threads;
    int status;
} orc_job;

/* level membership: a kind belongs to level L if its rank in the priority
 * order (Useful < Offloading < MPI, Kernel < Memory) is <= L */
static int orc_rank(int32_t kind) {
    switch (kind) {
        case ORC_HOST_USEFUL: return 0;
        case ORC_HOST_OFFLOAD: return 1;
        case ORC_HOST_MPI: return 2;
        case ORC_DEV_KERNEL: return 0;
        case ORC_DEV_MEMOP: return 1;
        default: return 99;
    }
}

static void* orc_worker(void* arg) {
    orc_job* J = (orc_job*)arg;
    const int32_t R = J->n_hosts + J->n_devices;
    const int32_t NR = J->n_regions;
    int64_t* lev = (int64_t*)malloc(sizeof(int64_t) * 3 * (size_t)(NR > 0 ? NR : 1));
    if (!lev) {
        J->status = ORC_E_OOM;
        return NULL;
    }
    for (int32_t r = J->tid; r < R; r += J->n_threads) {
        const int is_host = r < J->n_hosts;
        const int n_levels = is_host ? 3 : 2;
        const int64_t lo = J->ev_off[r], hi = J->ev_off[r + 1];
        orc_ivl* v = (orc_ivl*)malloc(sizeof(orc_ivl) * (size_t)(hi - lo > 0 ? hi - lo : 1));
        if (!v) {
            J->status = ORC_E_OOM;
            break;
        }
        for (int L = 0; L < n_levels; ++L) {
            int64_t k = 0;
            for (int64_t i = lo; i < hi; ++i) {
                if (orc_rank(J->g_kind[i]) <= L && J->g_s[i] < J->g_e[i]) {
                    v[k].s = J->g_s[i];
                    v[k].e = J->g_e[i];
                    ++k;
                }
            }
            orc_measure_sorted(v, k, NR, J->t0, J->t1, lev + (size_t)L * NR);
        }
        free(v);
        for (int32_t g = 0; g < NR; ++g) {
            const int64_t E = J->t1[g] - J->t0[g];
            int64_t* out = J->times + ((size_t)g * R + r) * 4;
            const int64_t d1 = lev[g], d2 = lev[NR + g];
            if (is_host) {
                const int64_t d3 = lev[2 * NR + g];
                out[0] = d1;
                out[1] = d2 - d1;
                out[2] = d3 - d2;
                out[3] = E - d3;
            } else {
                out[0] = d1;
                out[1] = d2 - d1;
                out[2] = E - d2;
                out[3] = 0;
            }
        }
    }
    free(lev);
    return NULL;
}

/* one IEEE division of two exact integers; 0/0 is defined as 1 and flagged */
static double orc_ratio(int64_t num, int64_t den, int bit, uint32_t* mask) {
    if (den == 0) {
        *mask |= 1u << bit;
        return 1.0;
    }
    return (double)num / (double)den;
}

int oracle_compute(int32_t n_hosts, int32_t n_devices, int64_t n_events,
                   const int32_t* resource, const int32_t* kind,
                   const int64_t* start, const int64_t* end,
                   int32_t n_regions, const int64_t* t0, const int64_t* t1,
                   int32_t n_threads,
                   int64_t* times, int64_t* sums, double* ratios, uint32_t* mask) {
    if (n_hosts < 0 || n_devices < 0 || n_events < 0 || n_regions < 0) return ORC_E_ARG;
    const int32_t R = n_hosts + n_devices;
    for (int32_t g = 0; g < n_regions; ++g)
        if (!(t0[g] < t1[g])) return ORC_E_REGION;
    for (int64_t i = 0; i < n_events; ++i) {
        if (resource[i] < 0 || resource[i] >= R) return ORC_E_ARG;
        const int host_kind = kind[i] >= ORC_HOST_USEFUL && kind[i] <= ORC_HOST_MPI;
        const int dev_kind = kind[i] == ORC_DEV_KERNEL || kind[i] == ORC_DEV_MEMOP;
        if ((resource[i] < n_hosts && !host_kind) || (resource[i] >= n_hosts && !dev_kind))
            return ORC_E_KIND;
        if (start[i] > end[i]) return ORC_E_INTERVAL;
    }
    /* group events by resource (counting sort on the resource id) */
    int64_t* off = (int64_t*)calloc((size_t)R + 1, sizeof(int64_t));
    int32_t* gk = (int32_t*)malloc(sizeof(int32_t) * (size_t)(n_events > 0 ? n_events : 1));
    int64_t* gs = (int64_t*)malloc(sizeof(int64_t) * (size_t)(n_events > 0 ? n_events : 1));
    int64_t* ge = (int64_t*)malloc(sizeof(int64_t) * (size_t)(n_events > 0 ? n_events : 1));
    int64_t* cur = (int64_t*)malloc(sizeof(int64_t) * ((size_t)R + 1));
    if (!off || !gk || !gs || !ge || !cur) {
        free(off); free(gk); free(gs); free(ge); free(cur);
        return ORC_E_OOM;
    }
    for (int64_t i = 0; i < n_events; ++i) off[resource[i] + 1]++;
    for (int32_t r = 0; r < R; ++r) off[r + 1] += off[r];
    memcpy(cur, off, sizeof(int64_t) * ((size_t)R + 1));
    for (int64_t i = 0; i < n_events; ++i) {
        const int64_t p = cur[resource[i]]++;
        gk[p] = kind[i];
        gs[p] = start[i];
        ge[p] = end[i];
    }
    free(cur);

    if (n_threads < 1) n_threads = 1;
    if (n_threads > R && R > 0) n_threads = R;
    orc_job* jobs = (orc_job*)calloc((size_t)n_threads, sizeof(orc_job));
    pthread_t* th = (pthread_t*)calloc((size_t)n_threads, sizeof(pthread_t));
    int status = ORC_OK;
    if (!jobs || !th) status = ORC_E_OOM;
    for (int32_t t = 0; status == ORC_OK && t < n_threads; ++t) {
        orc_job J = {n_hosts, n_devices, n_regions, t0, t1, off, gk, gs, ge, times, t, n_threads, ORC_OK};
        jobs[t] = J;
    }
    if (status == ORC_OK) {
        if (n_threads == 1) {
            orc_worker(&jobs[0]);
        } else {
            for (int32_t t = 0; t < n_threads; ++t) pthread_create(&th[t], NULL, orc_worker, &jobs[t]);
            for (int32_t t = 0; t < n_threads; ++t) pthread_join(th[t], NULL);
        }
        for (int32_t t = 0; t < n_threads; ++t)
            if (jobs[t].status != ORC_OK) status = jobs[t].status;
    }
    free(jobs); free(th); free(off); free(gk); free(gs); free(ge);
    if (status != ORC_OK) return status;

    /* aggregates over resources and the metric tree of each region */
    for (int32_t g = 0; g < n_regions; ++g) {
        const int64_t E = t1[g] - t0[g];
        int64_t sU = 0, sW = 0, sMPI = 0, sO = 0, sUW = 0, mUW = 0;
        int64_t sK = 0, sM = 0, mK = 0, mKM = 0;
        for (int32_t r = 0; r < R; ++r) {
            const int64_t* x = times + ((size_t)g * R + r) * 4;
            if (r < n_hosts) {
                sU += x[0]; sW += x[1]; sMPI += x[2]; sO += x[3];
                sUW += x[0] + x[1];
                mUW = orc_max(mUW, x[0] + x[1]);
            } else {
                sK += x[0]; sM += x[1];
                mK = orc_max(mK, x[0]);
                mKM = orc_max(mKM, x[0] + x[1]);
            }
        }
        int64_t* S = sums + (size_t)g * 10;
        S[0] = sU; S[1] = sW; S[2] = sMPI; S[3] = sO; S[4] = sUW; S[5] = mUW;
        S[6] = sK; S[7] = sM; S[8] = mK; S[9] = mKM;
        uint32_t mk = 0;
        double* q = ratios + (size_t)g * 9;
        const int64_t n = n_hosts, m = n_devices;
        q[0] = orc_ratio(sU, n * E, 0, &mk);       /* eq. 6: host hybrid PE */
        q[1] = orc_ratio(sUW, n * E, 1, &mk);      /* eq. 7: MPI PE */
        q[2] = orc_ratio(sUW, n * mUW, 2, &mk);    /* eq. 4 with U+W useful: MPI LB */
        q[3] = orc_ratio(mUW, E, 3, &mk);          /* eq. 5 with U+W useful: MPI CE */
        q[4] = orc_ratio(sU, sUW, 4, &mk);         /* eq. 8: device offload eff. */
        q[5] = orc_ratio(sK, m * E, 5, &mk);       /* eq. 9: device PE */
        q[6] = orc_ratio(sK, m * mK, 6, &mk);      /* eq. 10: device LB */
        q[7] = orc_ratio(mK, mKM, 7, &mk);         /* eq. 11: device comm. eff. */
        q[8] = orc_ratio(mKM, E, 8, &mk);          /* eq. 12: orchestration eff. */
        mask[g] = mk;
    }
    return ORC_OK;
}
