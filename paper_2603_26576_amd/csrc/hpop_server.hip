// Serving runtime: device-resident sessions updated incrementally by region-
// close queries, with continuous batching of queries from different sessions.
//
// State: for every (session, resource, level) a list of disjoint merged
// intervals in start order, stored as (start, measure before it) pairs plus
// the list's total measure, resident in device memory.
//
// One device step serves up to max_inflight queued queries (at most one per
// session, oldest first):
//   pack   : the queries' records -> 16 B records per (query, resource) item,
//            validated; the session's frontier (largest end) is advanced
//   prep   : per item and level, the smallest new start x and the first list
//            entry whose end reaches x (k0): entries before k0 cannot change;
//            scratch space for the rest is reserved from a pool
//   splice : per item and level, the list entries from k0 on plus the new
//            records are sorted by start (LDS or global radix) and flattened
//            again with the running state of entry k0-1, overwriting the
//            list from k0 on
//   region : per query, every resource clipped to the closing region and to
//            [origin, frontier) by binary search, then reduced to the two trees
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

struct ServChunk {
  const int64_t* s;
  const int64_t* e;
  long long count;
  long long dst;         // offset of the first packed record
  long long tile_begin;  // first tile of the chunk
  int32_t slot;
  int32_t req;
  int32_t sid;
  int32_t pad;
};

struct ServItem {
  long long rec_off;     // packed records [rec_off, rec_off + n)
  long long n;
  long long k0[3];       // prep output per level
  long long scr_off[3];  // prep output: scratch offset per level
  long long scr_len[3];
  int32_t req;
  int32_t list0;         // list index of level 0 (levels follow)
  int32_t nlev;
  int32_t pad;
};

struct ServReq {
  long long t0, t1, origin;
  int32_t sid;
  int32_t n_hosts;
  int32_t n_devices;
  int32_t list_begin;  // list index of (resource 0, level 0); 3 slots per resource
};

struct ServCtl {
  unsigned long long pool_used;  // scratch records reserved by prep
  unsigned long long pool_cap;
  unsigned long long pool_overflow;
  unsigned long long pad;
};

constexpr int kServThreads = 256;
constexpr int kServCap = 2048;
constexpr int kServTile = 4096;

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

__global__ __launch_bounds__(256) void k_serv_pack(const ServChunk* chunks, int n_chunks, Elem* raw,
                                                   long long* frontier, unsigned int* req_err) {
  __shared__ int s_c;
  const long long tile = blockIdx.x;
  if (threadIdx.x == 0) {
    int lo = 0, hi = n_chunks - 1;
    while (lo < hi) {
      int mid = (lo + hi + 1) >> 1;
      if (chunks[mid].tile_begin <= tile) lo = mid; else hi = mid - 1;
    }
    s_c = lo;
  }
  __syncthreads();
  const ServChunk c = chunks[s_c];
  const long long b = (tile - c.tile_begin) * kServTile;
  const long long end = min(c.count, b + kServTile);
  const unsigned long long slotbits = (unsigned long long)c.slot << kSlotShift;
  long long mx = LLONG_MIN;
  bool bad = false;
  for (long long i = b + threadIdx.x; i < end; i += 256) {
    const long long s = (long long)c.s[i], e = (long long)c.e[i];
    if (!rec_valid(s, e)) bad = true;
    Elem el;
    el.s = rec_valid(s, e) ? s : 0;
    el.e_slot = (long long)((unsigned long long)(rec_valid(s, e) ? e : 0) | slotbits);
    raw[c.dst + i] = el;
    if (rec_valid(s, e) && e > mx) mx = e;
  }
  mx = wave_red_max(mx);
  if ((threadIdx.x & 63) == 0 && mx != LLONG_MIN) atomicMax((unsigned long long*)&frontier[c.sid], (unsigned long long)mx);
  if (bad) atomicOr(&req_err[c.req], 1u);
}

__global__ __launch_bounds__(256) void k_serv_prep(ServItem* items, const Elem* raw, const ListDev* lists,
                                                   const unsigned int* req_err, ServCtl* ctl) {
  __shared__ long long red[3][4];
  ServItem& it = items[blockIdx.x];
  const bool skip = req_err[it.req] != 0;
  long long xm[3] = {LLONG_MAX, LLONG_MAX, LLONG_MAX};
  long long cnt[3] = {0, 0, 0};
  if (!skip) {
    for (long long i = threadIdx.x; i < it.n; i += 256) {
      const Elem el = raw[it.rec_off + i];
      const int slot = (int)((unsigned long long)el.e_slot >> kSlotShift);
      const long long e = el.e_slot & ((1ll << kSlotShift) - 1);
      if (el.s >= e) continue;  // empty records cover nothing
      for (int l = 0; l < 3; ++l)
        if (slot <= l) {
          xm[l] = el.s < xm[l] ? el.s : xm[l];
          cnt[l] += 1;
        }
    }
  }
  for (int l = 0; l < 3; ++l) {
    xm[l] = wave_red_min(xm[l]);
    cnt[l] = wave_red_sum(cnt[l]);
  }
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  __shared__ long long rc[3][4];
  if (lane == 0)
    for (int l = 0; l < 3; ++l) {
      red[l][wave] = xm[l];
      rc[l][wave] = cnt[l];
    }
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int l = 0; l < 3; ++l) {
      long long x = LLONG_MAX, c = 0;
      for (int w = 0; w < 4; ++w) {
        x = red[l][w] < x ? red[l][w] : x;
        c += rc[l][w];
      }
      it.k0[l] = -1;
      it.scr_len[l] = 0;
      if (l >= it.nlev || c == 0) continue;
      const ListDev L = lists[it.list0 + l];
      // first entry whose end reaches x: ends increase along the list
      long long lo = 0, hi = L.len;
      while (lo < hi) {
        const long long mid = (lo + hi) >> 1;
        if (list_ce(L, mid) < x) lo = mid + 1; else hi = mid;
      }
      it.k0[l] = lo;
      const long long need = (L.len - lo) + c;
      it.scr_len[l] = need;
      // two areas per level: the records and the sort's scratch
      const unsigned long long at = atomicAdd(&ctl->pool_used, (unsigned long long)(2 * need));
      if (at + 2 * need > ctl->pool_cap) {
        atomicAdd(&ctl->pool_overflow, (unsigned long long)(2 * need));
        it.k0[l] = -1;
      } else {
        it.scr_off[l] = (long long)at;
      }
    }
  }
}

__global__ __launch_bounds__(kServThreads) void k_serv_splice(const ServItem* items, const Elem* raw,
                                                              ListDev* lists, Elem* pool, const ServCtl* ctl) {
  __shared__ SortSmem<kServThreads, kServCap> sm;
  const ServItem it = items[blockIdx.x / 3];
  const int l = blockIdx.x % 3;
  if (ctl->pool_overflow) return;  // the host grows the pool and runs the step again
  if (l >= it.nlev || it.k0[l] < 0) return;
  ListDev& Lr = lists[it.list0 + l];
  const ListDev L = Lr;
  const long long k0 = it.k0[l];
  const long long nS = L.len - k0;
  const long long total = it.scr_len[l];
  Elem* A = pool + it.scr_off[l];
  Elem* B = A + total;
  // gather: list entries from k0 on, then the level's new records
  for (long long i = threadIdx.x; i < nS; i += kServThreads) {
    Elem el;
    el.s = L.base[k0 + i].cs;
    el.e_slot = list_ce(L, k0 + i);
    A[i] = el;
  }
  __shared__ unsigned int s_fill;
  if (threadIdx.x == 0) s_fill = 0;
  __syncthreads();
  for (long long i = threadIdx.x; i < it.n; i += kServThreads) {
    const Elem el = raw[it.rec_off + i];
    const int slot = (int)((unsigned long long)el.e_slot >> kSlotShift);
    const long long e = el.e_slot & ((1ll << kSlotShift) - 1);
    if (slot <= l && el.s < e) {
      const unsigned int p = atomicAdd(&s_fill, 1u);
      Elem o;
      o.s = el.s;
      o.e_slot = e;
      A[nS + p] = o;
    }
  }
  __syncthreads();
  // running state of the unchanged prefix
  FlatState st;
  for (int q = 0; q < 3; ++q) {
    st.M[q] = LLONG_MIN;
    st.P[q] = 0;
    st.R[q] = 0;
  }
  st.M[0] = k0 > 0 ? list_ce(L, k0 - 1) : LLONG_MIN;
  st.P[0] = k0 < L.len ? L.base[k0].pl : L.total;
  st.R[0] = k0;
  long long lo = LLONG_MAX;
  {
    long long m = LLONG_MAX;
    for (long long i = threadIdx.x; i < total; i += kServThreads) m = A[i].s < m ? A[i].s : m;
    m = wave_red_min(m);
    __shared__ long long r4[4];
    if ((threadIdx.x & 63) == 0) r4[threadIdx.x >> 6] = m;
    __syncthreads();
    for (int w = 0; w < 4; ++w) lo = r4[w] < lo ? r4[w] : lo;
    __syncthreads();
  }
  Comp* out[3] = {L.base, nullptr, nullptr};
  if (total <= kServCap) {
    const int ni = (int)total;
    for (int i = threadIdx.x; i < ni; i += kServThreads) sm.E[i] = A[i];
    __syncthreads();
    const unsigned short* ord = sort_lds<kServThreads, kServCap>(sm, ni, lo);
    flatten_tile<kServThreads>(sm.E, ord, ni, 1, 0, out, st, sm.lds_scan, nullptr);
  } else {
    const Elem* src = sort_global<kServThreads, kServCap>(sm, A, B, total, lo);
    for (long long t0 = 0; t0 < total; t0 += kServCap) {
      const int cnt = (int)min((long long)kServCap, total - t0);
      for (int i = threadIdx.x; i < cnt; i += kServThreads) sm.E[i] = src[t0 + i];
      __syncthreads();
      flatten_tile<kServThreads>(sm.E, nullptr, cnt, 1, 0, out, st, sm.lds_scan, nullptr);
      __syncthreads();
    }
  }
  if (threadIdx.x == 0) {
    Lr.len = st.R[0];
    Lr.total = st.P[0];
  }
}

__global__ __launch_bounds__(256) void k_serv_region(const ServReq* reqs, const ListDev* lists,
                                                     const long long* frontier, const unsigned int* req_err,
                                                     Tree* trees) {
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

struct Query {
  uint64_t ticket = 0;
  int32_t sid = 0;
  int32_t mem_space = HPOP_MEM_HOST;
  int64_t t0 = 0, t1 = 0;
  std::vector<hpop_event_chunk> chunks;  // device pointers, or pointers into `host`
  std::vector<int64_t> host;             // copied host records (start arrays then end arrays)
  long long n_records = 0;
  std::chrono::steady_clock::time_point submitted;
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

struct ListHost {
  DevBuf buf;
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
  DevBuf d_lists, d_chunks, d_items, d_reqs, d_raw, d_pool, d_frontier, d_err, d_ctl, d_trees, d_stage;
  PinnedBuf h_stage, h_out;
  long long pool_cap = 0;
  // statistics
  std::vector<double> lat_us;
  long long completed = 0, events = 0, steps = 0, batched = 0;
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
  const int nq = (int)batch.size();
  const int ns = (int)S->sessions.size();
  // ---- host plan: chunks, items, requests
  std::vector<ServChunk> chunks;
  std::vector<ServItem> items;
  std::vector<ServReq> reqs(nq);
  std::vector<long long> level_new(S->lists.size(), 0);
  long long tiles = 0, rec = 0;
  size_t host_bytes = 0;
  for (int q = 0; q < nq; ++q)
    if (batch[q]->mem_space == HPOP_MEM_HOST) host_bytes += batch[q]->host.size() * 8;
  if (host_bytes) {
    if (!S->h_stage.reserve(host_bytes) || !ensure(S->d_stage, A, host_bytes)) {
      err = "staging allocation failed";
      return HPOP_E_OOM;
    }
  }
  size_t hoff = 0;
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
    std::vector<long long> per_res(R, 0);
    std::vector<std::vector<int>> res_chunks(R);
    for (size_t c = 0; c < Q->chunks.size(); ++c) {
      per_res[Q->chunks[c].resource] += Q->chunks[c].count;
      res_chunks[Q->chunks[c].resource].push_back((int)c);
    }
    const int64_t* dev_base = nullptr;
    if (Q->mem_space == HPOP_MEM_HOST && !Q->host.empty()) {
      memcpy((char*)S->h_stage.ptr + hoff, Q->host.data(), Q->host.size() * 8);
      dev_base = (const int64_t*)((char*)S->d_stage.ptr + hoff);
    }
    for (int res = 0; res < R; ++res) {
      if (per_res[res] == 0) continue;
      ServItem it{};
      it.rec_off = rec;
      it.n = per_res[res];
      it.req = q;
      it.list0 = ss.list_begin + res * 3;
      it.nlev = res < ss.n_hosts ? 3 : 2;
      long long off = rec;
      for (int c : res_chunks[res]) {
        const hpop_event_chunk& ch = Q->chunks[c];
        if (ch.count == 0) continue;
        ServChunk sc{};
        if (Q->mem_space == HPOP_MEM_HOST) {
          // host chunks point into Q->host; rebase onto the device staging copy
          sc.s = dev_base + (ch.start - Q->host.data());
          sc.e = dev_base + (ch.end - Q->host.data());
        } else {
          sc.s = ch.start;
          sc.e = ch.end;
        }
        sc.count = ch.count;
        sc.dst = off;
        sc.tile_begin = tiles;
        sc.slot = slot_of_kind(ch.kind);
        sc.req = q;
        sc.sid = Q->sid;
        chunks.push_back(sc);
        tiles += (ch.count + kServTile - 1) / kServTile;
        off += ch.count;
        for (int l = sc.slot; l < it.nlev; ++l) level_new[it.list0 + l] += ch.count;
      }
      rec = off;
      items.push_back(it);
    }
    if (Q->mem_space == HPOP_MEM_HOST) hoff += Q->host.size() * 8;
  }
  hipStream_t st = S->stream;
  // ---- list capacity: a list grows by at most its level's new records
  for (size_t i = 0; i < S->lists.size(); ++i) {
    if (!level_new[i]) continue;
    ListHost& L = S->lists[i];
    const size_t need = (size_t)(L.len + level_new[i] + 1) * sizeof(Comp);
    L.buf.used = (size_t)L.len * sizeof(Comp);
    if (!L.buf.reserve(A, need, true)) {
      err = "device allocation for a session list failed";
      return HPOP_E_OOM;
    }
  }
  // ---- uploads
  std::vector<ListDev> ld(S->lists.size());
  for (size_t i = 0; i < S->lists.size(); ++i) {
    ld[i].base = (Comp*)S->lists[i].buf.ptr;
    ld[i].len = S->lists[i].len;
    ld[i].total = S->lists[i].total;
    ld[i].cap = (long long)(S->lists[i].buf.bytes / sizeof(Comp));
  }
  const size_t b_lists = ld.size() * sizeof(ListDev), b_chunks = chunks.size() * sizeof(ServChunk),
               b_items = items.size() * sizeof(ServItem), b_reqs = reqs.size() * sizeof(ServReq);
  const size_t b_out = 2 * nq * sizeof(Tree) + b_lists + nq * 4 + ns * 8 + sizeof(ServCtl) + 64;
  if (!ensure(S->d_lists, A, b_lists + 64) || !ensure(S->d_chunks, A, b_chunks + 64) ||
      !ensure(S->d_items, A, b_items + 64) || !ensure(S->d_reqs, A, b_reqs + 64) ||
      !ensure(S->d_raw, A, (size_t)(rec + 1) * sizeof(Elem)) || !ensure(S->d_err, A, nq * 4 + 64) ||
      !ensure(S->d_ctl, A, sizeof(ServCtl)) ||
      !ensure(S->d_trees, A, 2 * nq * sizeof(Tree) + 64) || !S->h_out.reserve(b_lists + b_chunks + b_items + b_reqs + b_out)) {
    err = "device allocation for a serving step failed";
    return HPOP_E_OOM;
  }
  const size_t want_pool = (size_t)std::max<long long>(1 << 20, 4 * rec + 4096);
  if ((long long)want_pool > S->pool_cap) {
    if (!ensure(S->d_pool, A, want_pool * sizeof(Elem))) {
      err = "scratch pool allocation failed";
      return HPOP_E_OOM;
    }
    S->pool_cap = (long long)(S->d_pool.bytes / sizeof(Elem));
  }
  if (host_bytes) {
    hipError_t e = hipMemcpyAsync(S->d_stage.ptr, S->h_stage.ptr, host_bytes, hipMemcpyHostToDevice, st);
    if (e != hipSuccess) return err = hipGetErrorString(e), HPOP_E_HIP;
  }
  char* h = (char*)S->h_out.ptr;
  memcpy(h, ld.data(), b_lists);
  memcpy(h + b_lists, chunks.data(), b_chunks);
  memcpy(h + b_lists + b_chunks, items.data(), b_items);
  memcpy(h + b_lists + b_chunks + b_items, reqs.data(), b_reqs);
  char* hres = h + b_lists + b_chunks + b_items + b_reqs;
  hipError_t e = hipSuccess;
  if (b_lists) e = hipMemcpyAsync(S->d_lists.ptr, h, b_lists, hipMemcpyHostToDevice, st);
  if (e == hipSuccess && b_chunks) e = hipMemcpyAsync(S->d_chunks.ptr, h + b_lists, b_chunks, hipMemcpyHostToDevice, st);
  if (e == hipSuccess && b_items)
    e = hipMemcpyAsync(S->d_items.ptr, h + b_lists + b_chunks, b_items, hipMemcpyHostToDevice, st);
  if (e == hipSuccess)
    e = hipMemcpyAsync(S->d_reqs.ptr, h + b_lists + b_chunks + b_items, b_reqs, hipMemcpyHostToDevice, st);
  if (e != hipSuccess) return err = hipGetErrorString(e), HPOP_E_HIP;
  for (int attempt = 0; attempt < 4; ++attempt) {
    // per-step control words
    ServCtl ctl{0, (unsigned long long)S->pool_cap, 0, 0};
    memcpy(hres, &ctl, sizeof ctl);
    e = hipMemcpyAsync(S->d_ctl.ptr, hres, sizeof ctl, hipMemcpyHostToDevice, st);
    if (e == hipSuccess) e = hipMemsetAsync(S->d_err.ptr, 0, nq * 4, st);
    if (e != hipSuccess) return err = hipGetErrorString(e), HPOP_E_HIP;
    if (tiles > 0)
      hipLaunchKernelGGL(k_serv_pack, dim3((unsigned)tiles), dim3(256), 0, st, (const ServChunk*)S->d_chunks.ptr,
                         (int)chunks.size(), (Elem*)S->d_raw.ptr, (long long*)S->d_frontier.ptr,
                         (unsigned int*)S->d_err.ptr);
    if (!items.empty()) {
      hipLaunchKernelGGL(k_serv_prep, dim3((unsigned)items.size()), dim3(256), 0, st, (ServItem*)S->d_items.ptr,
                         (const Elem*)S->d_raw.ptr, (const ListDev*)S->d_lists.ptr,
                         (const unsigned int*)S->d_err.ptr, (ServCtl*)S->d_ctl.ptr);
      hipLaunchKernelGGL(k_serv_splice, dim3((unsigned)items.size() * 3), dim3(kServThreads), 0, st,
                         (const ServItem*)S->d_items.ptr, (const Elem*)S->d_raw.ptr, (ListDev*)S->d_lists.ptr,
                         (Elem*)S->d_pool.ptr, (const ServCtl*)S->d_ctl.ptr);
    }
    e = hipGetLastError();
    if (e != hipSuccess) return err = std::string("serving kernels: ") + hipGetErrorString(e), HPOP_E_HIP;
    e = hipMemcpyAsync(hres, S->d_ctl.ptr, sizeof(ServCtl), hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) return err = hipGetErrorString(e), HPOP_E_HIP;
    ServCtl got;
    memcpy(&got, hres, sizeof got);
    if (!got.pool_overflow) break;
    // a long suffix needed more scratch: grow the pool and redo the step (no list was written)
    const size_t np = (size_t)(got.pool_used + got.pool_overflow + 4096) * 2;
    S->d_pool.release(A);
    if (!ensure(S->d_pool, A, np * sizeof(Elem))) {
      err = "scratch pool allocation failed";
      return HPOP_E_OOM;
    }
    S->pool_cap = (long long)(S->d_pool.bytes / sizeof(Elem));
    // the frontier advanced by pack is idempotent (a max); records are packed again
    if (attempt == 3) {
      err = "scratch pool kept overflowing";
      return HPOP_E_OOM;
    }
  }
  hipLaunchKernelGGL(k_serv_region, dim3((unsigned)(2 * nq)), dim3(256), 0, st, (const ServReq*)S->d_reqs.ptr,
                     (const ListDev*)S->d_lists.ptr, (const long long*)S->d_frontier.ptr,
                     (const unsigned int*)S->d_err.ptr, (Tree*)S->d_trees.ptr);
  e = hipGetLastError();
  char* o = hres;
  if (e == hipSuccess) e = hipMemcpyAsync(o, S->d_trees.ptr, 2 * nq * sizeof(Tree), hipMemcpyDeviceToHost, st);
  if (e == hipSuccess && b_lists)
    e = hipMemcpyAsync(o + 2 * nq * sizeof(Tree), S->d_lists.ptr, b_lists, hipMemcpyDeviceToHost, st);
  if (e == hipSuccess)
    e = hipMemcpyAsync(o + 2 * nq * sizeof(Tree) + b_lists, S->d_err.ptr, nq * 4, hipMemcpyDeviceToHost, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  if (e != hipSuccess) return err = std::string("serving step: ") + hipGetErrorString(e), HPOP_E_HIP;
  const ListDev* lo = (const ListDev*)(o + 2 * nq * sizeof(Tree));
  for (size_t i = 0; i < S->lists.size(); ++i) {
    S->lists[i].len = lo[i].len;
    S->lists[i].total = lo[i].total;
  }
  const unsigned int* re = (const unsigned int*)(o + 2 * nq * sizeof(Tree) + b_lists);
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
    std::string err;
    hpop_status st;
    {
      std::lock_guard<std::mutex> sg(S->state_mu);
      st = run_step(S, batch, err);
    }
    const auto now = std::chrono::steady_clock::now();
    lk.lock();
    ++S->steps;
    S->batched += (long long)batch.size();
    for (Query* Q : batch) {
      if (st != HPOP_OK) {
        Q->status = st;
        Q->error = err;
      }
      Q->done = true;
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

}  // namespace

extern "C" {

hpop_status hpop_server_create(const hpop_server_config* cfg, hpop_server** out) {
  try {
    if (!cfg || !out) return srv_fail(nullptr, HPOP_E_ARG, "null argument");
    *out = nullptr;
    if (cfg->max_sessions <= 0 || cfg->max_inflight <= 0 || cfg->max_inflight > 4096 || cfg->queue_capacity <= 0 ||
        cfg->mem_budget_bytes <= 0)
      return srv_fail(nullptr, HPOP_E_ARG, "server limits must be positive (max_inflight <= 4096)");
    hpop_server* S = new hpop_server();
    S->cfg = *cfg;
    if (hipGetDevice(&S->device) != hipSuccess ||
        hipStreamCreateWithFlags(&S->stream, hipStreamNonBlocking) != hipSuccess) {
      delete S;
      return srv_fail(nullptr, HPOP_E_HIP, "stream creation failed");
    }
    S->alloc.stream = S->stream;
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
  for (auto& L : S->lists) L.buf.release(S->alloc);
  for (DevBuf* b : {&S->d_lists, &S->d_chunks, &S->d_items, &S->d_reqs, &S->d_raw, &S->d_pool, &S->d_frontier,
                    &S->d_err, &S->d_ctl, &S->d_trees, &S->d_stage})
    b->release(S->alloc);
  S->h_stage.release();
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
    if (mem_space == HPOP_MEM_HOST) {
      Q->host.resize((size_t)2 * total);
      long long o = 0;
      for (int32_t i = 0; i < n_chunks; ++i) {
        const hpop_event_chunk& c = chunks[i];
        for (int64_t j = 0; j < c.count; ++j)
          if (c.start[j] < 0 || c.start[j] > c.end[j] || c.end[j] >= kTimeLimit) {
            delete Q;
            return srv_fail(S, HPOP_E_BAD_INTERVAL, "chunk " + std::to_string(i) + " record " + std::to_string(j));
          }
        memcpy(Q->host.data() + o, c.start, c.count * 8);
        memcpy(Q->host.data() + o + c.count, c.end, c.count * 8);
        hpop_event_chunk cc = c;
        cc.start = Q->host.data() + o;
        cc.end = Q->host.data() + o + c.count;
        Q->chunks.push_back(cc);
        o += 2 * c.count;
      }
    } else {
      Q->chunks.assign(chunks, chunks + n_chunks);
    }
    Q->n_records = total;
    Q->submitted = std::chrono::steady_clock::now();
    {
      std::lock_guard<std::mutex> g(S->mu);
      if ((int)S->queue.size() >= S->cfg.queue_capacity ||
          (S->inflight_bytes + total * 16 > S->cfg.mem_budget_bytes && S->inflight_bytes > 0)) {
        S->last_error = "queue full";
        delete Q;
        return HPOP_E_BUSY;
      }
      Q->ticket = S->next_ticket++;
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
  S->tickets.erase(it);
  delete Q;
  return st;
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
  return HPOP_OK;
}

const char* hpop_server_last_error(const hpop_server* S) {
  return S ? S->last_error.c_str() : g_thread_error.c_str();
}

}  // extern "C"
