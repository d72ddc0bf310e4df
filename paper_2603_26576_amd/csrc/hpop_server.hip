// Serving runtime: device-resident sessions updated incrementally by region-
// close queries, with continuous batching of queries from different sessions.
//
// State: for every (session, resource, level) a list of disjoint merged
// intervals in start order, stored as (start, measure before it) pairs plus
// the list's total measure, resident in device memory.
//
// One device step serves up to max_inflight queued queries (at most one per
// session, oldest first):
//   build  : the records of all queries of the step go through the same
//            bucketed build as a trace (validation, time buckets, LDS sort,
//            flattening), one segment per (query, resource)
//   prep   : per (query, resource, level): the first list entry whose end
//            reaches the earliest new start (k0; entries before it cannot
//            change), the list's largest end X and the last new bucket that
//            starts at or before X; scratch for the overlap is reserved
//   splice : the list entries from k0 on and the new records of buckets up to
//            X's bucket are sorted (LDS or global radix) and flattened again
//            from the running state of entry k0-1; the new merged intervals
//            of the later buckets cannot touch the old list and are appended
//            with their measures shifted
//   region : per query, every resource clipped to the closing region and to
//            [origin, frontier) by binary search, then reduced to two trees
// Queries that arrive while a step runs wait for the next step.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <climits>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <string>
#include <system_error>
#include <thread>
#include <vector>

#include "hpop.h"
#include "hpop_device.h"
#include "hpop_internal.h"
#include "hpop_runtime.h"

namespace hpop {

struct ListDev {
  Comp* base;
  long long len;
  long long total;
  long long cap;
};

struct ServItem {
  int32_t req;     // query index in the step
  int32_t seg;     // segment of the step's build
  int32_t list0;   // list index of level 0 (levels follow)
  int32_t nlev;
  int32_t sid;
  int32_t pad;
  long long k0[3];       // prep: first list entry that may change (-1: nothing to do)
  long long xb[3];       // prep: last new bucket (segment-relative) merged with the old entries, -1: none
  long long scr_off[3];  // prep: scratch offset per level
  long long scr_len[3];
};

struct ServReq {
  long long t0, t1, origin;
  int32_t sid;
  int32_t n_hosts;
  int32_t n_devices;
  int32_t list_begin;  // list index of (resource 0, level 0); 3 slots per resource
};

// a list that moves to a new place in the list heap
struct ListMove {
  const Comp* src;
  Comp* dst;
  long long len;
};

struct ServCtl {
  unsigned long long pool_used;  // scratch records reserved by prep
  unsigned long long pool_cap;
  unsigned long long pool_overflow;
  unsigned long long pad;
};

constexpr int kServThreads = 256;
constexpr int kServCap = 2048;

__device__ __forceinline__ long long list_ce(const ListDev& L, long long k) {
  const Comp c = L.base[k];
  const long long next = k + 1 < L.len ? L.base[k + 1].pl : L.total;
  return c.cs + (next - c.pl);
}

// measure of list L before time t
__device__ __forceinline__ long long list_measure(const ListDev& L, long long t) {
  long long lo = 0, hi = L.len;
  while (lo < hi) {
    const long long mid = (lo + hi) >> 1;
    if (L.base[mid].cs < t) lo = mid + 1; else hi = mid;
  }
  const long long k = lo - 1;
  if (k < 0) return 0;
  const long long ce = list_ce(L, k);
  return L.base[k].pl + (ce < t ? ce : t) - L.base[k].cs;
}

// one thread per (item, level)
__global__ __launch_bounds__(64) void k_serv_prep(ServItem* items, int n_items, Plan p, const ListDev* lists,
                                                  long long* frontier, ServCtl* ctl) {
  const int t = blockIdx.x * 64 + threadIdx.x;
  if (t >= n_items * 3) return;
  ServItem& it = items[t / 3];
  const int l = t % 3;
  it.k0[l] = -1;
  it.xb[l] = -1;
  it.scr_len[l] = 0;
  it.scr_off[l] = 0;
  // a query with an invalid record is not applied; a build whose buckets
  // outgrew their slots is redone before anything is applied
  if (l >= it.nlev || p.owner_err[it.req] || p.oversized[1]) return;
  const SegDesc sd = p.segs[it.seg];
  const SegStats stt = p.stats[it.seg];
  if (l == 0 && stt.max_e > stt.min_s) atomicMax((unsigned long long*)&frontier[it.sid], stt.max_e);
  const long long nb = sd.nb;
  // first bucket with a new merged interval of this level
  long long b0 = -1;
  for (long long b = 0; b < nb; ++b)
    if (p.ncomp[(sd.bucket_begin + b) * 3 + l]) {
      b0 = b;
      break;
    }
  if (b0 < 0) return;  // no new interval at this level
  const ListDev L = lists[it.list0 + l];
  const Geom g0 = seg_geom(p, it.seg);
  const long long x = comp_view(p, g0, sd.bucket_begin, sd.bucket_begin + b0, l).cs(0);
  long long lo = 0, hi = L.len;
  while (lo < hi) {
    const long long mid = (lo + hi) >> 1;
    if (list_ce(L, mid) < x) lo = mid + 1; else hi = mid;
  }
  const long long k0 = lo;
  // new buckets that may reach back into the old list: those starting at or before its largest end
  long long xb = -1;
  if (L.len > 0) {
    const long long X = list_ce(L, L.len - 1);
    if (X >= g0.min_s) xb = bucket_index(g0, (unsigned long long)(X - g0.min_s));
  }
  long long need = L.len - k0;
  for (long long b = 0; b <= xb; ++b) need += p.counts[sd.bucket_begin + b];
  const unsigned long long at = atomicAdd(&ctl->pool_used, (unsigned long long)(2 * need));
  if (at + 2 * need > ctl->pool_cap) {
    atomicAdd(&ctl->pool_overflow, (unsigned long long)(2 * need));
    return;
  }
  it.k0[l] = k0;
  it.xb[l] = xb;
  it.scr_off[l] = (long long)at;
  it.scr_len[l] = need;
}

// one workgroup per (item, level)
__global__ __launch_bounds__(kServThreads) void k_serv_splice(const ServItem* items, Plan p, ListDev* lists,
                                                              Elem* pool, const ServCtl* ctl) {
  __shared__ SortSmem<kServThreads, kServCap> sm;
  __shared__ unsigned int s_fill;
  __shared__ long long s_min[kServThreads / 64];
  __shared__ long long s_pref[kServThreads + 1];
  if (ctl->pool_overflow || p.oversized[1]) return;  // the host redoes the step
  const ServItem it = items[blockIdx.x / 3];
  const int l = blockIdx.x % 3;
  if (l >= it.nlev || it.k0[l] < 0) return;
  ListDev& Lr = lists[it.list0 + l];
  const ListDev L = Lr;
  const SegDesc sd = p.segs[it.seg];
  const long long nb = sd.nb;
  const long long k0 = it.k0[l], xb = it.xb[l];
  const long long nS = L.len - k0;
  const long long total = it.scr_len[l];
  Elem* A = pool + it.scr_off[l];
  Elem* B = A + total;
  FlatState st;
  for (int q = 0; q < 3; ++q) {
    st.M[q] = LLONG_MIN;
    st.P[q] = 0;
    st.R[q] = 0;
  }
  st.M[0] = k0 > 0 ? list_ce(L, k0 - 1) : LLONG_MIN;
  st.P[0] = k0 < L.len ? L.base[k0].pl : L.total;
  st.R[0] = k0;
  Comp* out[3] = {L.base, nullptr, nullptr};
  const Geom gs = seg_geom(p, it.seg);
  if (total > 0) {
    // old entries from k0 on, then the level's new records of buckets 0..xb
    for (long long i = threadIdx.x; i < nS; i += kServThreads) {
      Elem el;
      el.s = L.base[k0 + i].cs;
      el.e_slot = list_ce(L, k0 + i);
      A[i] = el;
    }
    if (threadIdx.x == 0) s_fill = 0;
    __syncthreads();
    for (long long b = 0; b <= xb; ++b) {
      const long long gb = sd.bucket_begin + b;
      const BucketRecs br = bucket_recs(p, gb);
      const long long blo = bucket_lo(gs, b);
      const long long n = (long long)br.n8 + br.n16;
      for (long long i = threadIdx.x; i < n; i += kServThreads) {
        const Elem el = i < br.n8 ? widen(br.narrow[i], blo, p.maxend + gb * 3) : br.wide[i - br.n8];
        const int slot = (int)((unsigned long long)el.e_slot >> kSlotShift);
        if (slot <= l) {
          const unsigned int q = atomicAdd(&s_fill, 1u);
          Elem o;
          o.s = el.s;
          o.e_slot = el.e_slot & ((1ll << kSlotShift) - 1);
          A[nS + q] = o;
        }
      }
    }
    __syncthreads();
    const long long cnt = nS + (long long)s_fill;
    long long m = LLONG_MAX;
    for (long long i = threadIdx.x; i < cnt; i += kServThreads) m = A[i].s < m ? A[i].s : m;
    m = wave_red_min(m);
    if ((threadIdx.x & 63) == 0) s_min[threadIdx.x >> 6] = m;
    __syncthreads();
    long long lo = LLONG_MAX;
    for (int w = 0; w < kServThreads / 64; ++w) lo = s_min[w] < lo ? s_min[w] : lo;
    __syncthreads();
    if (cnt <= kServCap) {
      const int ni = (int)cnt;
      for (int i = threadIdx.x; i < ni; i += kServThreads) sm.E[i] = A[i];
      __syncthreads();
      const unsigned short* ord = sort_lds<kServThreads, kServCap>(sm, ni, lo);
      flatten_tile<kServThreads>(sm.E, ord, ni, 1, 0, out, nullptr, 0, st, sm.lds_scan, nullptr);
    } else if (cnt > 0) {
      const Elem* src = sort_global<kServThreads, kServCap>(sm, A, B, cnt, lo);
      for (long long t0 = 0; t0 < cnt; t0 += kServCap) {
        const int c = (int)min((long long)kServCap, cnt - t0);
        for (int i = threadIdx.x; i < c; i += kServThreads) sm.E[i] = src[t0 + i];
        __syncthreads();
        flatten_tile<kServThreads>(sm.E, nullptr, c, 1, 0, out, nullptr, 0, st, sm.lds_scan, nullptr);
        __syncthreads();
      }
    }
  }
  // later buckets: their merged intervals start after the old list's end; append
  // them with measures rebased from the new buckets' own prefix to the list's
  long long R = st.R[0];
  long long P = st.P[0];
  const long long bt = xb + 1;
  if (bt < nb) {
    const long long shift = P - p.base[(sd.bucket_begin + bt) * 3 + l];
    for (long long b0 = bt; b0 < nb; b0 += kServThreads) {
      // component counts of a chunk of buckets -> prefix in LDS, then one
      // thread per component copies it (coalesced) with its measure rebased
      const long long b = b0 + threadIdx.x;
      const long long c = b < nb ? (long long)p.ncomp[(sd.bucket_begin + b) * 3 + l] : 0;
      long long v[1] = {c}, ex[1], tot[1];
      block_excl_scan<kServThreads, 1, OpSum>(v, ex, tot, 0, sm.lds_scan);
      s_pref[threadIdx.x] = ex[0];
      if (threadIdx.x == 0) s_pref[kServThreads] = tot[0];
      __syncthreads();
      for (long long j = threadIdx.x; j < tot[0]; j += kServThreads) {
        int a = 0, z = kServThreads - 1;  // last chunk bucket whose prefix is <= j
        while (a < z) {
          const int mid = (a + z + 1) >> 1;
          if (s_pref[mid] <= j) a = mid; else z = mid - 1;
        }
        const long long gb = sd.bucket_begin + b0 + a;
        const CompView src = comp_view(p, gs, sd.bucket_begin, gb, l);
        const long long k = j - s_pref[a];
        Comp o;
        o.cs = src.cs(k);
        o.pl = src.pl(k) + p.base[gb * 3 + l] + shift;
        L.base[R + j] = o;
      }
      R += tot[0];
      __syncthreads();
    }
    P = p.seg_total[it.seg * 3 + l] + shift;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    Lr.len = R;
    Lr.total = P;
  }
}

// grid (moves, k): workgroup y of a move copies every k-th run of 256 entries
__global__ __launch_bounds__(256) void k_list_move(const ListMove* mv) {
  const ListMove m = mv[blockIdx.x];
  for (long long i = (long long)blockIdx.y * 256 + threadIdx.x; i < m.len; i += 256ll * gridDim.y) m.dst[i] = m.src[i];
}

__global__ __launch_bounds__(256) void k_serv_region(const ServReq* reqs, const ListDev* lists,
                                                     const long long* frontier, Tree* trees) {
  __shared__ long long lds[4 * 10];
  const ServReq q = reqs[blockIdx.x >> 1];
  const bool global = blockIdx.x & 1;
  const long long t0 = global ? q.origin : q.t0;
  long long t1 = global ? frontier[q.sid] : q.t1;
  if (t1 <= t0) t1 = t0 + 1;  // an empty session: a one-ns global region
  const long long E = t1 - t0;
  const int R = q.n_hosts + q.n_devices;
  long long sU = 0, sW = 0, sMPI = 0, sO = 0, sK = 0, sM = 0, mUW = 0, mK = 0, mKM = 0;
  for (int r = threadIdx.x; r < R; r += 256) {
    const bool host = r < q.n_hosts;
    const int nl = host ? 3 : 2;
    long long D[3] = {0, 0, 0};
    for (int l = 0; l < nl; ++l) {
      const ListDev L = lists[q.list_begin + r * 3 + l];
      D[l] = list_measure(L, t1) - list_measure(L, t0);
    }
    if (host) {
      const long long u = D[0], w = D[1] - D[0];
      sU += u;
      sW += w;
      sMPI += D[2] - D[1];
      sO += E - D[2];
      mUW = u + w > mUW ? u + w : mUW;
    } else {
      const long long k = D[0], m = D[1] - D[0];
      sK += k;
      sM += m;
      mK = k > mK ? k : mK;
      mKM = k + m > mKM ? k + m : mKM;
    }
  }
  long long v[9] = {sU, sW, sMPI, sO, sK, sM, mUW, mK, mKM};
  block_tree<256>(v, lds);
  if (threadIdx.x == 0) trees[blockIdx.x] = make_tree(E, q.n_hosts, q.n_devices, v);
}

}  // namespace hpop

using namespace hpop;

namespace {

// Page-locked staging of host payloads: one area, taken once, cut first-fit
// into 256-byte-aligned ranges (freed ranges merge with their neighbours). A
// payload is copied into it once, at submission, and DMA-ed from there; a
// payload that does not fit while others hold the area waits (HPOP_E_BUSY),
// so the request path never allocates page-locked memory.
struct HostArena {
  std::mutex mu;
  char* base = nullptr;
  size_t bytes = 0;
  std::map<size_t, size_t> free_ranges;  // offset -> length
  size_t used = 0, max_used = 0;
  double alloc_us = 0.0;
  static size_t round_up(size_t n) { return (n + 255) & ~size_t(255); }
  // takes the area (called with mu held); false if the allocation failed
  bool take(size_t n) {
    const auto t = std::chrono::steady_clock::now();
    void* p = nullptr;
    if (hipHostMalloc(&p, n, hipHostMallocDefault) != hipSuccess) {
      (void)hipGetLastError();
      return false;
    }
    alloc_us = std::chrono::duration<double, std::micro>(std::chrono::steady_clock::now() - t).count();
    base = (char*)p;
    bytes = n;
    free_ranges.clear();
    free_ranges[0] = n;
    return true;
  }
  // a range of n bytes, or nullptr if none is free now
  char* get(size_t n) {
    std::lock_guard<std::mutex> g(mu);
    n = round_up(n);
    for (auto it = free_ranges.begin(); it != free_ranges.end(); ++it) {
      if (it->second < n) continue;
      const size_t off = it->first, len = it->second;
      free_ranges.erase(it);
      if (len > n) free_ranges[off + n] = len - n;
      used += n;
      max_used = std::max(max_used, used);
      return base + off;
    }
    return nullptr;
  }
  void put(char* p, size_t n) {
    if (!p) return;
    std::lock_guard<std::mutex> g(mu);
    n = round_up(n);
    used -= n;
    size_t off = (size_t)(p - base), len = n;
    auto next = free_ranges.lower_bound(off);
    if (next != free_ranges.end() && next->first == off + len) {
      len += next->second;
      next = free_ranges.erase(next);
    }
    if (next != free_ranges.begin()) {
      auto prev = std::prev(next);
      if (prev->first + prev->second == off) {
        off = prev->first;
        len += prev->second;
        free_ranges.erase(prev);
      }
    }
    free_ranges[off] = len;
  }
  void release() {
    if (base) (void)hipHostFree(base);
    base = nullptr;
    bytes = 0;
    free_ranges.clear();
  }
};

constexpr size_t kDefaultStagingBytes = size_t(1024) << 20;

// One contiguous copy of a host payload into its page-locked block.
struct CopySpan {
  char* dst;
  const char* src;
  size_t bytes;
};

// Copies the spans; payloads of kParallelCopyBytes and more are split in
// equal byte ranges over a few threads (one copying thread reaches only
// part of the host's memory bandwidth), the calling thread taking one.
constexpr size_t kParallelCopyBytes = size_t(1) << 20;
constexpr int kCopyThreads = 4;

void copy_range(const std::vector<CopySpan>& spans, size_t lo, size_t hi) {
  size_t base = 0;
  for (const CopySpan& c : spans) {
    const size_t a = std::max(lo, base), b = std::min(hi, base + c.bytes);
    if (a < b) memcpy(c.dst + (a - base), c.src + (a - base), b - a);
    base += c.bytes;
    if (base >= hi) break;
  }
}

void copy_spans(const std::vector<CopySpan>& spans, size_t total) {
  if (total < kParallelCopyBytes) {
    copy_range(spans, 0, total);
    return;
  }
  std::vector<std::thread> th;
  const size_t part = (total + kCopyThreads - 1) / kCopyThreads;
  try {
    for (int t = 1; t < kCopyThreads; ++t) {
      const size_t lo = std::min(total, t * part), hi = std::min(total, (t + 1) * part);
      th.emplace_back(copy_range, std::cref(spans), lo, hi);
    }
  } catch (const std::system_error&) {
    // no thread available: the calling thread copies what no thread took
    const size_t done_from = (th.size() + 1) * part;
    copy_range(spans, std::min(total, done_from), total);
  }
  copy_range(spans, 0, std::min(total, part));
  for (std::thread& x : th) x.join();
}

struct Query {
  uint64_t ticket = 0;
  int32_t sid = 0;
  int32_t mem_space = HPOP_MEM_HOST;
  int64_t t0 = 0, t1 = 0;
  std::vector<hpop_event_chunk> chunks;  // device pointers, or pointers into `host`
  int64_t* host = nullptr;               // copied host records (pinned): start arrays then end arrays
  size_t host_words = 0;
  long long n_records = 0;
  std::chrono::steady_clock::time_point submitted, finished;
  bool done = false;
  hpop_status status = HPOP_OK;
  std::string error;
  hpop_metric_tree region{}, global{};
};

struct SessionState {
  int32_t n_hosts = 0, n_devices = 0;
  int64_t origin = 0;
  int32_t list_begin = 0;
  bool busy = false;  // a query of this session is in the current step
};

// A session list: `cap` entries from `off` in the server's list heap.
struct ListHost {
  long long off = 0;
  long long cap = 0;
  long long len = 0;
  long long total = 0;
};

}  // namespace

struct hpop_server {
  hpop_server_config cfg{};
  int device = 0;
  hipStream_t stream = nullptr;
  Alloc alloc;
  std::mutex mu;        // queue, tickets, statistics, session table size
  std::mutex state_mu;  // held by the worker for a whole step and by session opening
  std::condition_variable cv_work, cv_done;
  std::deque<Query*> queue;
  std::map<uint64_t, Query*> tickets;
  std::vector<SessionState> sessions;
  std::vector<ListHost> lists;
  uint64_t next_ticket = 1;
  bool stop = false;
  std::thread worker;
  std::string last_error;
  long long inflight_bytes = 0;
  // device buffers of a step
  Engine engine;  // the bucketed build of each step's records
  DevBuf d_lists, d_items, d_reqs, d_pool, d_frontier, d_ctl, d_trees, d_stage, d_moves;
  DevBuf heap;  // every session list, Comp entries; bump-allocated, compacted when full
  long long heap_cap = 0, heap_used = 0;
  PinnedBuf h_out;
  HostArena staging;  // host payloads of queued queries
  long long pool_cap = 0;
  // statistics
  std::vector<double> lat_us;
  long long completed = 0, events = 0, steps = 0, batched = 0;
  double max_submit_us = 0.0, max_step_us = 0.0;
  // phases of a step: host clocks and HIP events on the server stream
  double max_prep_us = 0.0, max_grow_us = 0.0, max_wait_us = 0.0;
  double max_phase_us[5] = {0, 0, 0, 0, 0};  // h2d, move, build, splice, region
  double sum_phase_us[5] = {0, 0, 0, 0, 0};
  double sum_prep_us = 0.0, sum_grow_us = 0.0, sum_wait_us = 0.0;
  hipEvent_t ev[6] = {};
  bool have_events = false;
  double step_prep_us = 0.0, step_wait_us = 0.0;  // of the step just run (set by run_step)
  // longest single runtime call of the step's enqueueing, and its site (set by run_step)
  double step_call_us = 0.0;
  int step_call_site = -1;
  double max_call_us = 0.0;
  int max_call_site = -1;
};

namespace {

hpop_status srv_fail(hpop_server* s, hpop_status code, const std::string& msg) {
  if (s) {
    std::lock_guard<std::mutex> g(s->mu);
    s->last_error = msg;
  } else {
    g_thread_error = msg;
  }
  return code;
}

bool ensure(DevBuf& b, Alloc& a, size_t bytes) { return b.reserve(a, bytes, false); }

// Runs one device step over `batch` (queries of distinct sessions). Returns a
// status for the whole step; per-query failures are stored in the queries.
hpop_status run_step(hpop_server* S, std::vector<Query*>& batch, std::string& err) {
  Alloc& A = S->alloc;
  Engine& En = S->engine;
  const int nq = (int)batch.size();
  hipStream_t st = S->stream;
  // ---- host payloads go to the device straight from their pinned copies;
  // then every chunk is described to the build
  size_t host_bytes = 0;
  for (int q = 0; q < nq; ++q)
    if (batch[q]->mem_space == HPOP_MEM_HOST) host_bytes += batch[q]->host_words * 8;
  if (host_bytes && !ensure(S->d_stage, A, host_bytes)) {
    err = "staging allocation failed";
    return HPOP_E_OOM;
  }
  En.h_chunks.clear();
  En.h_regions.clear();
  En.h_ivls.clear();
  std::vector<long long> seg_count;
  std::vector<char> seg_host;
  std::vector<ServItem> items;
  std::vector<ServReq> reqs(nq);
  std::vector<long long> level_new(S->lists.size(), 0);
  size_t hoff = 0;
  const auto t_start = std::chrono::steady_clock::now();
  // host time of one runtime call (copies, launches, event records; not the
  // step's synchronisation), the longest of the step kept with its site
  auto timed = [&](int site, auto&& f) {
    const auto t0 = std::chrono::steady_clock::now();
    const hipError_t r = f();
    const double us = std::chrono::duration<double, std::micro>(std::chrono::steady_clock::now() - t0).count();
    if (us > S->step_call_us) {
      S->step_call_us = us;
      S->step_call_site = site;
    }
    return r;
  };
  auto mark = [&](int i) {
    if (S->have_events) (void)timed(HPOP_CALL_EVENT, [&] { return hipEventRecord(S->ev[i], st); });
  };
  mark(0);
  for (int q = 0; q < nq; ++q) {
    Query* Q = batch[q];
    const SessionState& ss = S->sessions[Q->sid];
    ServReq& r = reqs[q];
    r.t0 = Q->t0;
    r.t1 = Q->t1;
    r.origin = ss.origin;
    r.sid = Q->sid;
    r.n_hosts = ss.n_hosts;
    r.n_devices = ss.n_devices;
    r.list_begin = ss.list_begin;
    const int R = ss.n_hosts + ss.n_devices;
    const int64_t* dev_base = nullptr;
    if (Q->mem_space == HPOP_MEM_HOST && Q->host_words) {
      dev_base = (const int64_t*)((char*)S->d_stage.ptr + hoff);
      const hipError_t e = timed(HPOP_CALL_PAYLOAD, [&] {
        return hipMemcpyAsync((char*)S->d_stage.ptr + hoff, Q->host, Q->host_words * 8, hipMemcpyHostToDevice, st);
      });
      if (e != hipSuccess) return err = std::string("host payload copy: ") + hipGetErrorString(e), HPOP_E_HIP;
      hoff += Q->host_words * 8;
    }
    std::vector<int> seg_of_res(R, -1);
    for (const hpop_event_chunk& ch : Q->chunks) {
      if (ch.count == 0) continue;
      int& sg = seg_of_res[ch.resource];
      if (sg < 0) {
        sg = (int)seg_count.size();
        seg_count.push_back(0);
        seg_host.push_back(ch.resource < ss.n_hosts ? 1 : 0);
        ServItem it{};
        it.req = q;
        it.seg = sg;
        it.list0 = ss.list_begin + ch.resource * 3;
        it.nlev = ch.resource < ss.n_hosts ? 3 : 2;
        it.sid = Q->sid;
        items.push_back(it);
      }
      ChunkDesc d;
      if (Q->mem_space == HPOP_MEM_HOST) {
        d.s = dev_base + (ch.start - Q->host);
        d.e = dev_base + (ch.end - Q->host);
      } else {
        d.s = ch.start;
        d.e = ch.end;
      }
      d.count = ch.count;
      d.tile_begin = 0;
      d.seg = sg;
      d.slot = slot_of_kind(ch.kind);
      d.chunk_id = (int32_t)En.h_chunks.size();
      d.owner = q;
      En.h_chunks.push_back(d);
      seg_count[sg] += ch.count;
      const int nlev = ch.resource < ss.n_hosts ? 3 : 2;
      for (int l = d.slot; l < nlev; ++l) level_new[ss.list_begin + ch.resource * 3 + l] += ch.count;
    }
  }
  mark(1);  // payload copies
  hpop_tuning tun{};
  hpop_status rc = En.assemble_plan(tun, seg_count, seg_host, std::max(1, nq), 0, err);
  if (rc != HPOP_OK) return rc;
  // ---- list capacity: a list grows by at most its level's new records. A list
  // that outgrows its place moves to the end of the heap (at least doubling);
  // when the heap is full, every list moves into a new heap four times the live
  // size. All moves of a step are one kernel; the host tables change only
  // once it is enqueued.
  const size_t nl = S->lists.size();
  std::vector<long long> n_off(nl), n_cap(nl);
  long long grow = 0;
  for (size_t i = 0; i < nl; ++i) {
    const ListHost& L = S->lists[i];
    n_off[i] = L.off;
    n_cap[i] = L.cap;
    if (!level_new[i]) continue;
    const long long need = L.len + level_new[i] + 1;
    if (need <= L.cap) continue;
    n_cap[i] = (std::max({need, 2 * L.cap, 1024ll}) + 63) & ~63ll;
    n_off[i] = -1;  // placed below
    grow += n_cap[i];
  }
  std::vector<ListMove> moves;
  DevBuf new_heap;
  long long new_heap_cap = S->heap_cap, new_used = S->heap_used;
  if (grow) {
    Comp* old_base = (Comp*)S->heap.ptr;
    if (S->heap_used + grow <= S->heap_cap) {
      for (size_t i = 0; i < nl; ++i)
        if (n_off[i] < 0) {
          n_off[i] = new_used;
          new_used += n_cap[i];
          if (S->lists[i].len) moves.push_back({old_base + S->lists[i].off, old_base + n_off[i], S->lists[i].len});
        }
    } else {
      long long live = 0;
      for (size_t i = 0; i < nl; ++i) live += n_cap[i];
      new_heap_cap = std::max(4 * live, 1ll << 16);  // 4x: few compactions while sessions grow
      if (!new_heap.reserve(A, (size_t)new_heap_cap * sizeof(Comp), false)) {
        err = "device allocation for the session lists failed";
        return HPOP_E_OOM;
      }
      Comp* nb = (Comp*)new_heap.ptr;
      new_used = 0;
      for (size_t i = 0; i < nl; ++i) {
        if (S->lists[i].len) moves.push_back({old_base + S->lists[i].off, nb + new_used, S->lists[i].len});
        n_off[i] = new_used;
        new_used += n_cap[i];
      }
    }
  }
  if (!moves.empty() && !ensure(S->d_moves, A, moves.size() * sizeof(ListMove) + 64)) {
    new_heap.release(A);
    err = "device allocation for a serving step failed";
    return HPOP_E_OOM;
  }
  Comp* heap_base = (Comp*)(new_heap.ptr ? new_heap.ptr : S->heap.ptr);
  std::vector<ListDev> ld(nl);
  for (size_t i = 0; i < nl; ++i) {
    ld[i].base = heap_base + n_off[i];
    ld[i].len = S->lists[i].len;
    ld[i].total = S->lists[i].total;
    ld[i].cap = n_cap[i];
  }
  const int ni = (int)items.size();
  const size_t b_lists = ld.size() * sizeof(ListDev), b_items = items.size() * sizeof(ServItem),
               b_reqs = reqs.size() * sizeof(ServReq), b_trees = 2 * (size_t)nq * sizeof(Tree),
               b_moves = moves.size() * sizeof(ListMove);
  if (!ensure(S->d_lists, A, b_lists + 64) || !ensure(S->d_items, A, b_items + 64) ||
      !ensure(S->d_reqs, A, b_reqs + 64) || !ensure(S->d_ctl, A, sizeof(ServCtl)) ||
      !ensure(S->d_trees, A, b_trees + 64) ||
      // pinned layout: lists, items, requests, moves (uploads), then control, trees, lists, error flags
      !S->h_out.reserve(b_lists + b_items + b_reqs + b_moves + sizeof(ServCtl) + b_trees + b_lists + 4 * (size_t)nq +
                        256)) {
    new_heap.release(A);
    err = "device allocation for a serving step failed";
    return HPOP_E_OOM;
  }
  // ---- list moves, then the new placement becomes the server's
  if (!moves.empty()) {
    char* hm = (char*)S->h_out.ptr + b_lists + b_items + b_reqs;
    memcpy(hm, moves.data(), b_moves);
    hipError_t e = timed(HPOP_CALL_MOVE, [&] {
      hipError_t r = hipMemcpyAsync(S->d_moves.ptr, hm, b_moves, hipMemcpyHostToDevice, st);
      if (r == hipSuccess) {
        hipLaunchKernelGGL(k_list_move, dim3((unsigned)moves.size(), 8), dim3(256), 0, st,
                           (const ListMove*)S->d_moves.ptr);
        r = hipGetLastError();
      }
      return r;
    });
    if (e != hipSuccess) {
      (void)hipStreamSynchronize(st);
      new_heap.release(A);
      err = std::string("list move: ") + hipGetErrorString(e);
      return HPOP_E_HIP;
    }
  }
  mark(2);  // list moves
  if (new_heap.ptr) {
    S->heap.release(A);  // stream-ordered: after the moves out of it
    S->heap = new_heap;
    S->heap_cap = new_heap_cap;
  }
  S->heap_used = new_used;
  for (size_t i = 0; i < nl; ++i) {
    S->lists[i].off = n_off[i];
    S->lists[i].cap = n_cap[i];
  }
  long long total_rec = 0;
  for (long long c : seg_count) total_rec += c;
  const long long want_pool = std::max<long long>(1 << 20, 4 * total_rec + 4096);
  if (want_pool > S->pool_cap) {
    S->d_pool.release(A);
    if (!ensure(S->d_pool, A, (size_t)want_pool * sizeof(Elem))) {
      err = "scratch pool allocation failed";
      return HPOP_E_OOM;
    }
    S->pool_cap = (long long)(S->d_pool.bytes / sizeof(Elem));
  }
  // ---- the build of the step's records (no regions: the trees come from the lists)
  if (!En.ws.pinned.reserve(64)) {
    err = "pinned host allocation failed";
    return HPOP_E_OOM;
  }
  (void)timed(HPOP_CALL_BUILD, [&] {
    rc = En.upload(err);
    if (rc == HPOP_OK) rc = En.enqueue(true, false, err);
    return hipSuccess;
  });
  if (rc != HPOP_OK) return rc;
  mark(3);  // build of the new records
  char* h = (char*)S->h_out.ptr;
  memcpy(h, ld.data(), b_lists);
  memcpy(h + b_lists, items.data(), b_items);
  memcpy(h + b_lists + b_items, reqs.data(), b_reqs);
  char* hres = h + b_lists + b_items + b_reqs + b_moves;
  hipError_t e = timed(HPOP_CALL_TABLES, [&] {
    hipError_t r = hipSuccess;
    if (b_lists) r = hipMemcpyAsync(S->d_lists.ptr, h, b_lists, hipMemcpyHostToDevice, st);
    if (r == hipSuccess && b_items) r = hipMemcpyAsync(S->d_items.ptr, h + b_lists, b_items, hipMemcpyHostToDevice, st);
    if (r == hipSuccess) r = hipMemcpyAsync(S->d_reqs.ptr, h + b_lists + b_items, b_reqs, hipMemcpyHostToDevice, st);
    return r;
  });
  if (e != hipSuccess) return err = hipGetErrorString(e), HPOP_E_HIP;
  const Plan& P = En.ws.plan;
  char* o = hres + sizeof(ServCtl);  // results: trees, lists, error flags
  // one synchronisation per step: the scratch check travels back with the results
  for (int attempt = 0; attempt < 4; ++attempt) {
    ServCtl ctl{0, (unsigned long long)S->pool_cap, 0, 0};
    memcpy(hres, &ctl, sizeof ctl);
    e = timed(HPOP_CALL_CONTROL,
              [&] { return hipMemcpyAsync(S->d_ctl.ptr, hres, sizeof ctl, hipMemcpyHostToDevice, st); });
    if (e != hipSuccess) return err = hipGetErrorString(e), HPOP_E_HIP;
    if (ni > 0) {
      (void)timed(HPOP_CALL_SPLICE, [&] {
        hipLaunchKernelGGL(k_serv_prep, dim3((unsigned)((3 * ni + 63) / 64)), dim3(64), 0, st,
                           (ServItem*)S->d_items.ptr, ni, P, (const ListDev*)S->d_lists.ptr,
                           (long long*)S->d_frontier.ptr, (ServCtl*)S->d_ctl.ptr);
        hipLaunchKernelGGL(k_serv_splice, dim3((unsigned)(3 * ni)), dim3(kServThreads), 0, st,
                           (const ServItem*)S->d_items.ptr, P, (ListDev*)S->d_lists.ptr, (Elem*)S->d_pool.ptr,
                           (const ServCtl*)S->d_ctl.ptr);
        return hipSuccess;
      });
    }
    mark(4);  // prep and splice
    // on a scratch overflow no list was written and these trees are discarded
    e = timed(HPOP_CALL_REGION, [&] {
      hipLaunchKernelGGL(k_serv_region, dim3((unsigned)(2 * nq)), dim3(256), 0, st, (const ServReq*)S->d_reqs.ptr,
                         (const ListDev*)S->d_lists.ptr, (const long long*)S->d_frontier.ptr, (Tree*)S->d_trees.ptr);
      return hipGetLastError();
    });
    if (e == hipSuccess)
      e = timed(HPOP_CALL_RESULTS, [&] {
        hipError_t r = hipMemcpyAsync(hres, S->d_ctl.ptr, sizeof(ServCtl), hipMemcpyDeviceToHost, st);
        if (r == hipSuccess) r = hipMemcpyAsync(o, S->d_trees.ptr, b_trees, hipMemcpyDeviceToHost, st);
        if (r == hipSuccess && b_lists)
          r = hipMemcpyAsync(o + b_trees, S->d_lists.ptr, b_lists, hipMemcpyDeviceToHost, st);
        if (r == hipSuccess) r = hipMemcpyAsync(o + b_trees + b_lists, P.owner_err, nq * 4, hipMemcpyDeviceToHost, st);
        return r;
      });
    mark(5);  // region trees and result copies
    const auto t_sync = std::chrono::steady_clock::now();
    if (attempt == 0) S->step_prep_us = std::chrono::duration<double, std::micro>(t_sync - t_start).count();
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    S->step_wait_us +=
        std::chrono::duration<double, std::micro>(std::chrono::steady_clock::now() - t_sync).count();
    if (e != hipSuccess) return err = std::string("serving step: ") + hipGetErrorString(e), HPOP_E_HIP;
    ServCtl got;
    memcpy(&got, hres, sizeof got);
    if (!got.pool_overflow) break;
    // a long overlap needed more scratch: grow the pool and redo prep, splice and region
    const long long np = (long long)(got.pool_used + got.pool_overflow + 4096) * 2;
    S->d_pool.release(A);
    if (!ensure(S->d_pool, A, (size_t)np * sizeof(Elem))) {
      err = "scratch pool allocation failed";
      return HPOP_E_OOM;
    }
    S->pool_cap = (long long)(S->d_pool.bytes / sizeof(Elem));
    if (attempt == 3) {
      err = "scratch pool kept overflowing";
      return HPOP_E_OOM;
    }
  }
  if (S->have_events) {
    for (int i = 0; i < 5; ++i) {
      float ms = 0.f;
      if (hipEventElapsedTime(&ms, S->ev[i], S->ev[i + 1]) == hipSuccess) {
        S->max_phase_us[i] = std::max(S->max_phase_us[i], 1e3 * (double)ms);
        S->sum_phase_us[i] += 1e3 * (double)ms;
      }
    }
  }
  unsigned long long slot_over;
  memcpy(&slot_over, (const char*)En.ws.pinned.ptr + 16, 8);
  if (slot_over && !En.exact_forced) {
    // a bucket outgrew its scatter slots: no list was touched; redo with exact counts
    En.exact_forced = true;
    rc = run_step(S, batch, err);
    En.exact_forced = false;
    return rc;
  }
  const ListDev* lo = (const ListDev*)(o + b_trees);
  for (size_t i = 0; i < S->lists.size(); ++i) {
    S->lists[i].len = lo[i].len;
    S->lists[i].total = lo[i].total;
  }
  const unsigned int* re = (const unsigned int*)(o + b_trees + b_lists);
  for (int q = 0; q < nq; ++q) {
    Query* Q = batch[q];
    if (re[q]) {
      Q->status = HPOP_E_BAD_INTERVAL;
      Q->error = "a record of this query violates 0 <= start <= end < 2^62; the query was not applied";
    } else {
      memcpy(&Q->region, o + (2 * q) * sizeof(Tree), sizeof(Tree));
      memcpy(&Q->global, o + (2 * q + 1) * sizeof(Tree), sizeof(Tree));
    }
  }
  return HPOP_OK;
}

void worker_loop(hpop_server* S) {
  (void)hipSetDevice(S->device);
  std::unique_lock<std::mutex> lk(S->mu);
  while (true) {
    S->cv_work.wait(lk, [&] { return S->stop || !S->queue.empty(); });
    if (S->stop && S->queue.empty()) break;
    // admit: oldest query of each idle session, up to max_inflight
    std::vector<Query*> batch;
    std::vector<char> taken(S->sessions.size(), 0);
    for (auto it = S->queue.begin(); it != S->queue.end() && (int)batch.size() < S->cfg.max_inflight;) {
      Query* Q = *it;
      if (taken[Q->sid]) {
        ++it;
        continue;
      }
      taken[Q->sid] = 1;  // later queries of this session wait for the next step
      batch.push_back(Q);
      it = S->queue.erase(it);
    }
    lk.unlock();
    const auto t_admit = std::chrono::steady_clock::now();
    std::string err;
    hpop_status st;
    S->step_prep_us = S->step_wait_us = 0.0;
    S->step_call_us = 0.0;
    S->step_call_site = -1;
    const double alloc0 = g_alloc_us;
    {
      std::lock_guard<std::mutex> sg(S->state_mu);
      st = run_step(S, batch, err);
    }
    const double grow_us = g_alloc_us - alloc0;
    // every step ends synchronised: the host payloads have been copied
    for (Query* Q : batch) {
      S->staging.put((char*)Q->host, Q->host_words * 8);
      Q->host = nullptr;
    }
    const auto now = std::chrono::steady_clock::now();
    lk.lock();
    ++S->steps;
    S->max_prep_us = std::max(S->max_prep_us, S->step_prep_us);
    S->max_wait_us = std::max(S->max_wait_us, S->step_wait_us);
    S->max_grow_us = std::max(S->max_grow_us, grow_us);
    if (S->step_call_us > S->max_call_us) {
      S->max_call_us = S->step_call_us;
      S->max_call_site = S->step_call_site;
    }
    S->sum_prep_us += S->step_prep_us;
    S->sum_wait_us += S->step_wait_us;
    S->sum_grow_us += grow_us;
    S->batched += (long long)batch.size();
    S->max_step_us = std::max(S->max_step_us, std::chrono::duration<double, std::micro>(now - t_admit).count());
    for (Query* Q : batch) {
      if (st != HPOP_OK) {
        Q->status = st;
        Q->error = err;
      }
      Q->done = true;
      Q->finished = now;
      S->inflight_bytes -= Q->n_records * 16;
      if (Q->status == HPOP_OK) {
        ++S->completed;
        S->events += Q->n_records;
        S->lat_us.push_back(std::chrono::duration<double, std::micro>(now - Q->submitted).count());
      }
    }
    S->cv_done.notify_all();
  }
}

// Waits for a ticket and releases it; `finished` receives its completion time.
hpop_status wait_ticket(hpop_server* S, uint64_t ticket, int64_t timeout_ns, hpop_metric_tree* out_region,
                        hpop_metric_tree* out_global, std::chrono::steady_clock::time_point* finished) {
  std::unique_lock<std::mutex> lk(S->mu);
  auto it = S->tickets.find(ticket);
  if (it == S->tickets.end()) {
    S->last_error = "unknown ticket";
    return HPOP_E_ARG;
  }
  Query* Q = it->second;
  if (timeout_ns < 0) {
    S->cv_done.wait(lk, [&] { return Q->done; });
  } else if (!S->cv_done.wait_for(lk, std::chrono::nanoseconds(timeout_ns), [&] { return Q->done; })) {
    S->last_error = "timed out";
    return HPOP_E_TIMEOUT;
  }
  const hpop_status st = Q->status;
  if (st == HPOP_OK) {
    if (out_region) *out_region = Q->region;
    if (out_global) *out_global = Q->global;
  } else {
    S->last_error = Q->error;
  }
  if (finished) *finished = Q->finished;
  S->tickets.erase(it);
  delete Q;
  return st;
}

}  // namespace

extern "C" {

hpop_status hpop_server_create(const hpop_server_config* cfg, hpop_server** out) {
  try {
    if (!cfg || !out) return srv_fail(nullptr, HPOP_E_ARG, "null argument");
    *out = nullptr;
    if (cfg->max_sessions <= 0 || cfg->max_inflight <= 0 || cfg->max_inflight > 4096 || cfg->queue_capacity <= 0 ||
        cfg->mem_budget_bytes <= 0 || cfg->host_staging_mib < 0 || cfg->list_heap_bytes < 0)
      return srv_fail(nullptr, HPOP_E_ARG,
                      "server limits must be positive (max_inflight <= 4096, host_staging_mib >= 0)");
    hpop_server* S = new hpop_server();
    S->cfg = *cfg;
    if (hipGetDevice(&S->device) != hipSuccess ||
        hipStreamCreateWithFlags(&S->stream, hipStreamNonBlocking) != hipSuccess) {
      delete S;
      return srv_fail(nullptr, HPOP_E_HIP, "stream creation failed");
    }
    S->alloc.stream = S->stream;  // every device allocation of the server is ordered on its stream
    if (cfg->host_staging_mib > 0 && !S->staging.take((size_t)cfg->host_staging_mib << 20)) {
      (void)hipStreamDestroy(S->stream);
      delete S;
      return srv_fail(nullptr, HPOP_E_OOM, "page-locked staging allocation failed");
    }
    S->have_events = true;
    for (hipEvent_t& e : S->ev)
      if (hipEventCreate(&e) != hipSuccess) S->have_events = false;
    if (cfg->list_heap_bytes > 0) {
      const long long cap = cfg->list_heap_bytes / (long long)sizeof(Comp);
      if (!S->heap.reserve(S->alloc, (size_t)cap * sizeof(Comp), false) ||
          hipStreamSynchronize(S->stream) != hipSuccess) {
        S->heap.release(S->alloc);
        S->staging.release();
        for (hipEvent_t e : S->ev)
          if (e) (void)hipEventDestroy(e);
        (void)hipStreamDestroy(S->stream);
        delete S;
        return srv_fail(nullptr, HPOP_E_OOM, "device allocation of the list heap failed");
      }
      S->heap_cap = cap;
    }
    S->engine.alloc = S->alloc;
    S->engine.use_graphs = false;
    S->worker = std::thread(worker_loop, S);
    *out = S;
    return HPOP_OK;
  } catch (...) {
    return srv_fail(nullptr, HPOP_E_STATE, "server creation failed");
  }
}

hpop_status hpop_server_destroy(hpop_server* S) {
  if (!S) return srv_fail(nullptr, HPOP_E_ARG, "null server");
  {
    std::lock_guard<std::mutex> g(S->mu);
    S->stop = true;
  }
  S->cv_work.notify_all();
  if (S->worker.joinable()) S->worker.join();
  (void)hipStreamSynchronize(S->stream);
  S->heap.release(S->alloc);
  S->engine.release();
  for (DevBuf* b : {&S->d_lists, &S->d_items, &S->d_reqs, &S->d_pool, &S->d_frontier, &S->d_ctl, &S->d_trees,
                    &S->d_stage, &S->d_moves})
    b->release(S->alloc);
  S->staging.release();
  for (hipEvent_t e : S->ev)
    if (e) (void)hipEventDestroy(e);
  S->h_out.release();
  (void)hipStreamSynchronize(S->stream);
  (void)hipStreamDestroy(S->stream);
  for (auto& kv : S->tickets) delete kv.second;
  delete S;
  return HPOP_OK;
}

hpop_status hpop_server_open_session(hpop_server* S, int32_t n_hosts, int32_t n_devices, int64_t t_origin,
                                     int32_t* out_sid) {
  if (!S || !out_sid) return srv_fail(S, HPOP_E_ARG, "null argument");
  if (n_hosts < 0 || n_devices < 0 || n_hosts + n_devices == 0 || n_hosts + n_devices > (1 << 16))
    return srv_fail(S, HPOP_E_ARG, "need 1 <= n_hosts + n_devices <= 65536");
  if (t_origin < 0 || t_origin >= kTimeLimit) return srv_fail(S, HPOP_E_REGION, "origin out of range");
  std::lock_guard<std::mutex> sg(S->state_mu);  // no step runs while the tables change
  int sid;
  {
    std::lock_guard<std::mutex> g(S->mu);
    if ((int)S->sessions.size() >= S->cfg.max_sessions) {
      S->last_error = "max_sessions reached";
      return HPOP_E_STATE;
    }
    SessionState ss;
    ss.n_hosts = n_hosts;
    ss.n_devices = n_devices;
    ss.origin = t_origin;
    ss.list_begin = (int32_t)S->lists.size();
    S->lists.resize(S->lists.size() + (size_t)3 * (n_hosts + n_devices));
    sid = (int)S->sessions.size();
    S->sessions.push_back(ss);
  }
  // frontier table: existing sessions keep their device values, the new one starts at its origin
  std::vector<long long> fr((size_t)sid + 1);
  fr[sid] = t_origin;
  hpop_status rc = HPOP_OK;
  DevBuf& F = S->d_frontier;
  if (F.ptr && sid > 0) {
    if (hipMemcpyAsync(fr.data(), F.ptr, (size_t)sid * 8, hipMemcpyDeviceToHost, S->stream) != hipSuccess ||
        hipStreamSynchronize(S->stream) != hipSuccess)
      rc = HPOP_E_HIP;
  }
  if (rc == HPOP_OK && !F.reserve(S->alloc, fr.size() * 8 + 64, false)) rc = HPOP_E_OOM;
  if (rc == HPOP_OK && (hipMemcpyAsync(F.ptr, fr.data(), fr.size() * 8, hipMemcpyHostToDevice, S->stream) != hipSuccess ||
                        hipStreamSynchronize(S->stream) != hipSuccess))
    rc = HPOP_E_HIP;
  if (rc != HPOP_OK) {
    std::lock_guard<std::mutex> g(S->mu);
    S->last_error = "frontier table update failed";
  }
  if (rc != HPOP_OK) return rc;
  *out_sid = sid;
  return HPOP_OK;
}

hpop_status hpop_server_submit(hpop_server* S, int32_t sid, const hpop_event_chunk* chunks, int32_t n_chunks,
                               int32_t mem_space, int64_t t0, int64_t t1, uint64_t* out_ticket) {
  try {
    if (!S || !out_ticket || n_chunks < 0 || (n_chunks > 0 && !chunks)) return srv_fail(S, HPOP_E_ARG, "bad arguments");
    if (mem_space != HPOP_MEM_HOST && mem_space != HPOP_MEM_DEVICE) return srv_fail(S, HPOP_E_ARG, "bad mem_space");
    if (!(t0 < t1)) return srv_fail(S, HPOP_E_REGION, "region needs t0 < t1");
    const auto t_enter = std::chrono::steady_clock::now();
    int32_t nh, nd;
    {
      std::lock_guard<std::mutex> g(S->mu);
      if (sid < 0 || sid >= (int)S->sessions.size()) {
        S->last_error = "unknown session";
        return HPOP_E_ARG;
      }
      nh = S->sessions[sid].n_hosts;
      nd = S->sessions[sid].n_devices;
    }
    const unsigned long long w = (unsigned long long)std::max(1, std::max(nh, nd));
    if ((unsigned long long)(t1 - t0) >= (1ull << 53) / w)
      return srv_fail(S, HPOP_E_OVERFLOW, "(t1 - t0) * max(n, m) must be below 2^53");
    Query* Q = new Query();
    Q->sid = sid;
    Q->mem_space = mem_space;
    Q->t0 = t0;
    Q->t1 = t1;
    long long total = 0;
    for (int32_t i = 0; i < n_chunks; ++i) {
      const hpop_event_chunk& c = chunks[i];
      const int slot = slot_of_kind(c.kind);
      if (c.resource < 0 || c.resource >= nh + nd || slot < 0 || ((c.kind <= HPOP_HOST_MPI) != (c.resource < nh)) ||
          c.count < 0 || (c.count > 0 && (!c.start || !c.end))) {
        delete Q;
        return srv_fail(S, c.resource < 0 || c.resource >= nh + nd ? HPOP_E_RESOURCE : HPOP_E_KIND,
                        "bad chunk " + std::to_string(i));
      }
      total += c.count;
    }
    auto busy = [&] {
      return (int)S->queue.size() >= S->cfg.queue_capacity ||
             (S->inflight_bytes + total * 16 > S->cfg.mem_budget_bytes && S->inflight_bytes > 0);
    };
    if (mem_space == HPOP_MEM_HOST) {
      {
        std::lock_guard<std::mutex> g(S->mu);  // no copy for a query that would be refused anyway
        if (busy()) {
          S->last_error = "queue full";
          delete Q;
          return HPOP_E_BUSY;
        }
      }
      // one copy into the page-locked staging area; the records are validated
      // on the device like device payloads (an invalid one fails the query at
      // hpop_server_wait)
      if (total > 0) {
        size_t area;
        {
          std::lock_guard<std::mutex> g(S->staging.mu);
          if (!S->staging.base) {
            const size_t want = S->cfg.host_staging_mib > 0 ? (size_t)S->cfg.host_staging_mib << 20
                                                            : kDefaultStagingBytes;
            if (!S->staging.take(want)) {
              delete Q;
              return srv_fail(S, HPOP_E_OOM, "page-locked staging allocation failed");
            }
          }
          area = S->staging.bytes;
        }
        if ((size_t)total * 16 > area) {
          delete Q;
          return srv_fail(S, HPOP_E_ARG, "host payload larger than the page-locked staging area");
        }
        Q->host = (int64_t*)S->staging.get((size_t)total * 16);
        if (!Q->host) {  // the area is held by queued payloads: back-pressure
          delete Q;
          return srv_fail(S, HPOP_E_BUSY, "page-locked staging area full");
        }
      }
      Q->host_words = (size_t)2 * total;
      std::vector<CopySpan> spans;
      long long o = 0;
      for (int32_t i = 0; i < n_chunks; ++i) {
        const hpop_event_chunk& c = chunks[i];
        if (c.count == 0) continue;
        spans.push_back({(char*)(Q->host + o), (const char*)c.start, (size_t)c.count * 8});
        spans.push_back({(char*)(Q->host + o + c.count), (const char*)c.end, (size_t)c.count * 8});
        hpop_event_chunk cc = c;
        cc.start = Q->host + o;
        cc.end = Q->host + o + c.count;
        Q->chunks.push_back(cc);
        o += 2 * c.count;
      }
      copy_spans(spans, (size_t)total * 16);
    } else {
      Q->chunks.assign(chunks, chunks + n_chunks);
    }
    Q->n_records = total;
    Q->submitted = std::chrono::steady_clock::now();
    {
      std::lock_guard<std::mutex> g(S->mu);
      if (busy()) {
        S->last_error = "queue full";
        S->staging.put((char*)Q->host, (size_t)total * 16);
        delete Q;
        return HPOP_E_BUSY;
      }
      Q->ticket = S->next_ticket++;
      S->max_submit_us =
          std::max(S->max_submit_us, std::chrono::duration<double, std::micro>(Q->submitted - t_enter).count());
      S->inflight_bytes += total * 16;
      S->tickets[Q->ticket] = Q;
      S->queue.push_back(Q);
      *out_ticket = Q->ticket;
    }
    S->cv_work.notify_one();
    return HPOP_OK;
  } catch (const std::bad_alloc&) {
    return srv_fail(S, HPOP_E_OOM, "host allocation failed");
  } catch (...) {
    return srv_fail(S, HPOP_E_STATE, "internal error");
  }
}

hpop_status hpop_server_wait(hpop_server* S, uint64_t ticket, int64_t timeout_ns, hpop_metric_tree* out_region,
                             hpop_metric_tree* out_global) {
  if (!S) return srv_fail(nullptr, HPOP_E_ARG, "null server");
  return wait_ticket(S, ticket, timeout_ns, out_region, out_global, nullptr);
}

hpop_status hpop_server_get_stats(hpop_server* S, hpop_server_stats* out) {
  if (!S || !out) return srv_fail(S, HPOP_E_ARG, "null argument");
  std::lock_guard<std::mutex> g(S->mu);
  out->completed = S->completed;
  out->events = S->events;
  out->device_steps = S->steps;
  out->mean_batch = S->steps ? (double)S->batched / (double)S->steps : 0.0;
  std::vector<double> v = S->lat_us;
  std::sort(v.begin(), v.end());
  auto pct = [&](double p) { return v.empty() ? 0.0 : v[std::min(v.size() - 1, (size_t)(p * (v.size() - 1) + 0.5))]; };
  out->p50_us = pct(0.50);
  out->p99_us = pct(0.99);
  out->max_us = v.empty() ? 0.0 : v.back();
  out->max_submit_us = S->max_submit_us;
  out->max_step_us = S->max_step_us;
  out->max_prep_us = S->max_prep_us;
  out->max_grow_us = S->max_grow_us;
  out->max_wait_us = S->max_wait_us;
  out->max_h2d_us = S->max_phase_us[0];
  out->max_move_us = S->max_phase_us[1];
  out->max_build_us = S->max_phase_us[2];
  out->max_splice_us = S->max_phase_us[3];
  out->max_region_us = S->max_phase_us[4];
  const double ns = S->steps ? (double)S->steps : 1.0;
  out->mean_prep_us = S->sum_prep_us / ns;
  out->mean_grow_us = S->sum_grow_us / ns;
  out->mean_wait_us = S->sum_wait_us / ns;
  out->mean_h2d_us = S->sum_phase_us[0] / ns;
  out->mean_move_us = S->sum_phase_us[1] / ns;
  out->mean_build_us = S->sum_phase_us[2] / ns;
  out->mean_splice_us = S->sum_phase_us[3] / ns;
  out->mean_region_us = S->sum_phase_us[4] / ns;
  out->max_call_us = S->max_call_us;
  out->max_call_site = S->max_call_site;
  out->reserved = 0;
  {
    std::lock_guard<std::mutex> pg(S->staging.mu);
    out->host_staging_bytes = (int64_t)S->staging.bytes;
    out->max_pinned_alloc_us = S->staging.alloc_us;
    out->max_host_staging_used = (int64_t)S->staging.max_used;
  }
  return HPOP_OK;
}

hpop_status hpop_server_reset_stats(hpop_server* S) {
  if (!S) return srv_fail(nullptr, HPOP_E_ARG, "null server");
  std::lock_guard<std::mutex> g(S->mu);
  S->lat_us.clear();
  S->completed = S->events = S->steps = S->batched = 0;
  S->max_submit_us = S->max_step_us = 0.0;
  S->max_prep_us = S->max_grow_us = S->max_wait_us = 0.0;
  S->sum_prep_us = S->sum_grow_us = S->sum_wait_us = 0.0;
  for (int i = 0; i < 5; ++i) S->max_phase_us[i] = S->sum_phase_us[i] = 0.0;
  S->max_call_us = 0.0;
  S->max_call_site = -1;
  return HPOP_OK;
}

hpop_status hpop_server_replay(hpop_server* S, const hpop_replay_query* qs, int32_t n, int32_t mem_space,
                               hpop_metric_tree* out_region, hpop_metric_tree* out_global, int64_t* latency_ns,
                               int64_t* out_wall_ns, int64_t* out_busy) {
  using clk = std::chrono::steady_clock;
  if (!S || n < 0 || (n > 0 && !qs)) return srv_fail(S, HPOP_E_ARG, "bad arguments");
  for (int32_t i = 1; i < n; ++i)
    if (qs[i].arrival_ns < qs[i - 1].arrival_ns) return srv_fail(S, HPOP_E_ARG, "arrival times must not decrease");
  std::vector<uint64_t> tickets((size_t)n, 0);
  std::vector<char> submitted((size_t)n, 0);
  hpop_status first = HPOP_OK;
  std::string first_err;
  long long busy = 0;
  const clk::time_point t_start = clk::now();
  for (int32_t i = 0; i < n; ++i) {
    const clk::time_point due = t_start + std::chrono::nanoseconds(qs[i].arrival_ns);
    // sleep while the arrival is far, spin for the last stretch
    while (true) {
      const auto left = due - clk::now();
      if (left <= std::chrono::nanoseconds(0)) break;
      if (left > std::chrono::microseconds(200)) std::this_thread::sleep_for(left - std::chrono::microseconds(100));
    }
    hpop_status st;
    while ((st = hpop_server_submit(S, qs[i].sid, qs[i].chunks, qs[i].n_chunks, mem_space, qs[i].t0, qs[i].t1,
                                    &tickets[i])) == HPOP_E_BUSY) {
      ++busy;
      std::this_thread::sleep_for(std::chrono::microseconds(50));
    }
    if (st == HPOP_OK) {
      submitted[i] = 1;
    } else if (first == HPOP_OK) {
      first = st;
      first_err = hpop_server_last_error(S);
    }
  }
  clk::time_point last = t_start;
  for (int32_t i = 0; i < n; ++i) {
    if (!submitted[i]) continue;
    clk::time_point fin;
    const hpop_status st = wait_ticket(S, tickets[i], -1, out_region ? out_region + i : nullptr,
                                       out_global ? out_global + i : nullptr, &fin);
    if (st != HPOP_OK) {
      if (first == HPOP_OK) {
        first = st;
        first_err = hpop_server_last_error(S);
      }
      continue;
    }
    last = std::max(last, fin);
    if (latency_ns)
      latency_ns[i] = std::chrono::duration_cast<std::chrono::nanoseconds>(
                          fin - (t_start + std::chrono::nanoseconds(qs[i].arrival_ns))).count();
  }
  if (out_wall_ns) *out_wall_ns = std::chrono::duration_cast<std::chrono::nanoseconds>(last - t_start).count();
  if (out_busy) *out_busy = busy;
  if (first != HPOP_OK) {
    std::lock_guard<std::mutex> g(S->mu);
    S->last_error = first_err;
  }
  return first;
}

const char* hpop_server_last_error(const hpop_server* S) {
  return S ? S->last_error.c_str() : g_thread_error.c_str();
}

}  // extern "C"
