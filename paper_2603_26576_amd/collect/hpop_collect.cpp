// rocprofiler-sdk tool that records the host and device states of the
// heterogeneous POP metrics inside a running HIP application (the interface
// and the recorded states are described in hpop_collect.h).
//
// Host side: a synchronous callback on every HIP runtime API call, as the
// paper's AMD backend does (Section 4.2); the outermost call of a thread is
// one Device Offloading record, and the Useful records are the gaps between
// offload calls, made final up to a frontier before which no call can still
// be missing. Device side: kernel dispatch and memory copy records delivered
// in rocprofiler buffers, one device resource per GPU agent, flushed
// periodically by a thread of the tool (a flush blocks for milliseconds, too
// long for the application's own threads). The library makes no HIP call.
#include <rocprofiler-sdk/registration.h>
#include <rocprofiler-sdk/rocprofiler.h>

#include <unistd.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <string>
#include <thread>
#include <unordered_map>
#include <unordered_set>
#include <vector>

#include "hpop_collect.h"

namespace {

constexpr int kKinds = 5;
constexpr int64_t kIdle = -1;      // thread not inside a runtime call
constexpr int64_t kEntering = -2;  // thread entering a call, start not yet read

struct Series {
  std::vector<int64_t> s, e;
};

// One per thread that ever made a runtime call; never freed (a thread that
// ends leaves its slot idle).
struct ThreadSlot {
  std::atomic<int64_t> inflight{kIdle};  // start of the thread's outermost running call
  int depth = 0;                         // touched by the owning thread only
};

struct Collector {
  std::atomic<int> configured{0};
  std::atomic<int> active{0};
  rocprofiler_context_id_t ctx{};
  rocprofiler_buffer_id_t buf{};
  int n_dev = 0;
  int64_t t_begin = 0;
  std::unordered_map<uint64_t, int> agent_dev;  // GPU agent handle -> device index (set once at start)

  std::mutex mu;                 // everything below
  std::vector<Series> series;    // [(1 + n_dev) * kKinds]
  std::vector<std::pair<int64_t, int64_t>> pending;  // offload calls that may reach past `sealed`
  int64_t sealed = 0;            // Useful gaps are final before this time
  std::unordered_set<uint64_t> runtime_kernels;  // the runtime's own copy and fill kernels

  std::mutex mu_threads;
  std::vector<ThreadSlot*> threads;
  std::atomic<int64_t> dropped{0};

  // periodic delivery of device records, off the application's threads
  std::thread flusher;
  std::mutex mu_flush;
  std::condition_variable cv_flush;
  bool stop_flush = false;
};

// Created on first use and never destroyed: rocprofiler may call the tool
// while the libraries of the process are still being initialised (before
// this library's static constructors) and while they are being torn down
// (after its static destructors), so no static object with a constructor or
// destructor may hold the state.
Collector& G() {
  static Collector* c = new Collector();
  return *c;
}
thread_local ThreadSlot* t_slot = nullptr;  // plain pointer: no constructor

int64_t clock_ns() {
  rocprofiler_timestamp_t t = 0;
  rocprofiler_get_timestamp(&t);
  return (int64_t)t;
}

ThreadSlot* my_slot() {
  if (!t_slot) {
    ThreadSlot* s = new ThreadSlot();
    std::lock_guard<std::mutex> lk(G().mu_threads);
    G().threads.push_back(s);
    t_slot = s;
  }
  return t_slot;
}

// caller holds G().mu
void push(int resource, int kind, int64_t s, int64_t e) {
  try {
    Series& q = G().series[(size_t)resource * kKinds + kind];
    q.s.push_back(s);
    q.e.push_back(e < s ? s : e);
  } catch (...) {
    G().dropped.fetch_add(1);
  }
}

void on_hip_api(rocprofiler_callback_tracing_record_t rec, rocprofiler_user_data_t* ud, void*) {
  ThreadSlot* ts = my_slot();
  if (rec.phase == ROCPROFILER_CALLBACK_PHASE_ENTER) {
    if (ts->depth++ == 0) {
      // announce the call before reading its start: a poll that misses the
      // announcement took its own time before this start (see hpop_collect_poll)
      ts->inflight.store(kEntering, std::memory_order_seq_cst);
      const int64_t t = clock_ns();
      ud->value = (uint64_t)t;
      ts->inflight.store(t, std::memory_order_seq_cst);
    }
  } else if (rec.phase == ROCPROFILER_CALLBACK_PHASE_EXIT) {
    if (ts->depth > 0 && --ts->depth == 0) {
      const int64_t s = (int64_t)ud->value, e = clock_ns();
      {
        std::lock_guard<std::mutex> lk(G().mu);
        push(0, HPOP_HOST_OFFLOAD, s, e);
        try {
          G().pending.emplace_back(s, e);
        } catch (...) {
          G().dropped.fetch_add(1);
        }
      }
      // after the record is visible: a poll that sees the thread idle also sees its record
      ts->inflight.store(kIdle, std::memory_order_seq_cst);
    }
  }
}

void on_code_object(rocprofiler_callback_tracing_record_t rec, rocprofiler_user_data_t*, void*) {
  if (rec.kind != ROCPROFILER_CALLBACK_TRACING_CODE_OBJECT ||
      rec.operation != ROCPROFILER_CODE_OBJECT_DEVICE_KERNEL_SYMBOL_REGISTER ||
      rec.phase != ROCPROFILER_CALLBACK_PHASE_LOAD)
    return;
  const auto* d = static_cast<const rocprofiler_callback_tracing_code_object_kernel_symbol_register_data_t*>(
      rec.payload);
  // the HIP runtime's blit kernels implement memcpy and memset: memory operations
  if (d->kernel_name && std::strncmp(d->kernel_name, "__amd_rocclr_", 13) == 0) {
    std::lock_guard<std::mutex> lk(G().mu);
    G().runtime_kernels.insert(d->kernel_id);
  }
}

int dev_of(rocprofiler_agent_id_t a) {
  auto it = G().agent_dev.find(a.handle);
  return it == G().agent_dev.end() ? -1 : it->second;
}

void on_buffer(rocprofiler_context_id_t, rocprofiler_buffer_id_t, rocprofiler_record_header_t** headers,
               size_t n, void*, uint64_t drop_count) {
  if (drop_count) G().dropped.fetch_add((int64_t)drop_count);
  std::lock_guard<std::mutex> lk(G().mu);
  for (size_t i = 0; i < n; ++i) {
    const rocprofiler_record_header_t* h = headers[i];
    if (h->category != ROCPROFILER_BUFFER_CATEGORY_TRACING) continue;
    if (h->kind == ROCPROFILER_BUFFER_TRACING_KERNEL_DISPATCH) {
      const auto* r = static_cast<const rocprofiler_buffer_tracing_kernel_dispatch_record_t*>(h->payload);
      const int d = dev_of(r->dispatch_info.agent_id);
      if (d < 0) continue;
      const int kind = G().runtime_kernels.count(r->dispatch_info.kernel_id) ? HPOP_DEV_MEMOP : HPOP_DEV_KERNEL;
      push(1 + d, kind, (int64_t)r->start_timestamp, (int64_t)r->end_timestamp);
    } else if (h->kind == ROCPROFILER_BUFFER_TRACING_MEMORY_COPY) {
      const auto* r = static_cast<const rocprofiler_buffer_tracing_memory_copy_record_t*>(h->payload);
      const int ds = dev_of(r->src_agent_id), dd = dev_of(r->dst_agent_id);
      if (dd >= 0) push(1 + dd, HPOP_DEV_MEMOP, (int64_t)r->start_timestamp, (int64_t)r->end_timestamp);
      if (ds >= 0 && ds != dd) push(1 + ds, HPOP_DEV_MEMOP, (int64_t)r->start_timestamp, (int64_t)r->end_timestamp);
    }
  }
}

rocprofiler_status_t on_agents(rocprofiler_agent_version_t, const void** agents, size_t n, void*) {
  std::vector<std::pair<int32_t, uint64_t>> gpus;  // (position among GPUs, handle)
  for (size_t i = 0; i < n; ++i) {
    const auto* a = static_cast<const rocprofiler_agent_v0_t*>(agents[i]);
    if (a->type == ROCPROFILER_AGENT_TYPE_GPU) gpus.emplace_back(a->logical_node_type_id, a->id.handle);
  }
  std::sort(gpus.begin(), gpus.end());
  for (size_t i = 0; i < gpus.size(); ++i) G().agent_dev[gpus[i].second] = (int)i;
  G().n_dev = (int)gpus.size();
  return ROCPROFILER_STATUS_SUCCESS;
}

// Useful gaps of [G().sealed, frontier) between the pending offload calls;
// caller holds G().mu.
void seal(int64_t frontier) {
  if (frontier <= G().sealed) return;
  auto& p = G().pending;
  std::sort(p.begin(), p.end());
  int64_t cur = G().sealed;  // covered (by a call) or emitted up to here
  for (const auto& iv : p) {
    if (iv.first >= frontier) break;
    if (iv.first > cur) push(0, HPOP_HOST_USEFUL, cur, iv.first);
    cur = std::max(cur, iv.second);
    if (cur >= frontier) break;
  }
  if (cur < frontier) push(0, HPOP_HOST_USEFUL, cur, frontier);
  // calls that end by the frontier can no longer cover later time
  p.erase(std::remove_if(p.begin(), p.end(), [&](const std::pair<int64_t, int64_t>& iv) { return iv.second <= frontier; }),
          p.end());
  G().sealed = frontier;
}

int64_t take_frontier() {
  // the time first, then the threads: a call announced after the scan reads
  // its start after the scan, so after this time
  int64_t f = clock_ns();
  std::vector<ThreadSlot*> ts;
  {
    std::lock_guard<std::mutex> lk(G().mu_threads);
    ts = G().threads;
  }
  for (ThreadSlot* s : ts) {
    int64_t v = s->inflight.load(std::memory_order_seq_cst);
    while (v == kEntering) {
      std::this_thread::yield();
      v = s->inflight.load(std::memory_order_seq_cst);
    }
    if (v >= 0 && v < f) f = v;
  }
  return f;
}

std::string out_path() {
  const char* p = std::getenv("HPOP_COLLECT_OUT");
  if (!p || !*p) return std::string();
  std::string s(p);
  const size_t i = s.find("%p");
  if (i != std::string::npos) s.replace(i, 2, std::to_string((long long)getpid()));
  return s;
}

void flush_loop(int period_ms) {
  std::unique_lock<std::mutex> lk(G().mu_flush);
  while (!G().cv_flush.wait_for(lk, std::chrono::milliseconds(period_ms), [] { return G().stop_flush; })) {
    lk.unlock();
    rocprofiler_flush_buffer(G().buf);
    lk.lock();
  }
}

int flush_period_ms() {
  const char* v = std::getenv("HPOP_COLLECT_FLUSH_MS");
  if (!v || !*v) return 10;
  const int ms = std::atoi(v);
  return ms < 0 ? 0 : ms;
}

int tool_init(rocprofiler_client_finalize_t, void*) {
  if (rocprofiler_query_available_agents(ROCPROFILER_AGENT_INFO_VERSION_0, on_agents, sizeof(rocprofiler_agent_v0_t),
                                         nullptr) != ROCPROFILER_STATUS_SUCCESS)
    return -1;
  G().series.assign((size_t)(1 + G().n_dev) * kKinds, Series());
  if (rocprofiler_create_context(&G().ctx) != ROCPROFILER_STATUS_SUCCESS) return -1;
  if (rocprofiler_configure_callback_tracing_service(G().ctx, ROCPROFILER_CALLBACK_TRACING_CODE_OBJECT, nullptr, 0,
                                                     on_code_object, nullptr) != ROCPROFILER_STATUS_SUCCESS)
    return -1;
  if (rocprofiler_configure_callback_tracing_service(G().ctx, ROCPROFILER_CALLBACK_TRACING_HIP_RUNTIME_API, nullptr, 0,
                                                     on_hip_api, nullptr) != ROCPROFILER_STATUS_SUCCESS)
    return -1;
  constexpr size_t kBufBytes = 8u << 20;
  if (rocprofiler_create_buffer(G().ctx, kBufBytes, kBufBytes / 2, ROCPROFILER_BUFFER_POLICY_LOSSLESS, on_buffer,
                                nullptr, &G().buf) != ROCPROFILER_STATUS_SUCCESS)
    return -1;
  if (rocprofiler_configure_buffer_tracing_service(G().ctx, ROCPROFILER_BUFFER_TRACING_KERNEL_DISPATCH, nullptr, 0,
                                                   G().buf) != ROCPROFILER_STATUS_SUCCESS)
    return -1;
  if (rocprofiler_configure_buffer_tracing_service(G().ctx, ROCPROFILER_BUFFER_TRACING_MEMORY_COPY, nullptr, 0,
                                                   G().buf) != ROCPROFILER_STATUS_SUCCESS)
    return -1;
  G().t_begin = clock_ns();
  G().sealed = G().t_begin;
  if (rocprofiler_start_context(G().ctx) != ROCPROFILER_STATUS_SUCCESS) return -1;
  G().active.store(1);
  const int period = flush_period_ms();
  if (period > 0) {
    try {
      G().flusher = std::thread(flush_loop, period);
    } catch (...) {
      // no thread: records still arrive when a buffer fills or on hpop_collect_flush
    }
  }
  return 0;
}

void tool_fini(void*) {
  if (!G().active.load()) return;
  if (G().flusher.joinable()) {
    {
      std::lock_guard<std::mutex> lk(G().mu_flush);
      G().stop_flush = true;
    }
    G().cv_flush.notify_all();
    G().flusher.join();
  }
  hpop_collect_flush();
  int64_t f = 0;
  hpop_collect_poll(&f);
  const std::string p = out_path();
  if (!p.empty() && hpop_collect_write(p.c_str()) != HPOP_OK)
    std::fprintf(stderr, "hpop_collect: cannot write %s\n", p.c_str());
  rocprofiler_stop_context(G().ctx);
  G().active.store(0);
}

bool pair_ok(int32_t resource, int32_t kind) {
  if (resource < 0 || resource > G().n_dev || kind < 0 || kind >= kKinds) return false;
  const bool host_kind = kind <= HPOP_HOST_MPI;
  return (resource == 0) == host_kind;
}

}  // namespace

extern "C" {

rocprofiler_tool_configure_result_t* rocprofiler_configure(uint32_t, const char*, uint32_t,
                                                           rocprofiler_client_id_t* id) {
  int expected = 0;
  if (!G().configured.compare_exchange_strong(expected, 1)) return nullptr;  // one configuration per process
  id->name = "hpop_collect";
  static rocprofiler_tool_configure_result_t cfg{sizeof(rocprofiler_tool_configure_result_t), &tool_init, &tool_fini,
                                                 nullptr};
  return &cfg;
}

int32_t hpop_collect_active(void) { return G().active.load(); }

int32_t hpop_collect_devices(void) { return G().active.load() ? G().n_dev : 0; }

int64_t hpop_collect_now(void) { return clock_ns(); }

int64_t hpop_collect_begin(void) { return G().active.load() ? G().t_begin : 0; }

hpop_status hpop_collect_poll(int64_t* out_frontier) {
  if (!out_frontier) return HPOP_E_ARG;
  if (!G().active.load()) return HPOP_E_STATE;
  const int64_t f = take_frontier();
  std::lock_guard<std::mutex> lk(G().mu);
  seal(std::max(f, G().sealed));
  *out_frontier = G().sealed;
  return HPOP_OK;
}

hpop_status hpop_collect_flush(void) {
  if (!G().active.load()) return HPOP_E_STATE;
  // no lock held: the buffer callback takes it
  return rocprofiler_flush_buffer(G().buf) == ROCPROFILER_STATUS_SUCCESS ? HPOP_OK : HPOP_E_STATE;
}

int64_t hpop_collect_count(int32_t resource, int32_t kind) {
  if (!G().active.load() || !pair_ok(resource, kind)) return 0;
  std::lock_guard<std::mutex> lk(G().mu);
  return (int64_t)G().series[(size_t)resource * kKinds + kind].s.size();
}

hpop_status hpop_collect_copy(int32_t resource, int32_t kind, int64_t first, int64_t count, int64_t* start,
                              int64_t* end) {
  if (first < 0 || count < 0 || (count > 0 && (!start || !end))) return HPOP_E_ARG;
  if (!G().active.load()) return HPOP_E_STATE;
  if (resource < 0 || resource > G().n_dev) return HPOP_E_RESOURCE;
  if (!pair_ok(resource, kind)) return HPOP_E_KIND;
  std::lock_guard<std::mutex> lk(G().mu);
  const Series& q = G().series[(size_t)resource * kKinds + kind];
  if (first + count > (int64_t)q.s.size()) return HPOP_E_REGION;
  if (count > 0) {
    std::memcpy(start, q.s.data() + first, (size_t)count * sizeof(int64_t));
    std::memcpy(end, q.e.data() + first, (size_t)count * sizeof(int64_t));
  }
  return HPOP_OK;
}

hpop_status hpop_collect_write(const char* path) {
  if (!path) return HPOP_E_ARG;
  if (!G().active.load()) return HPOP_E_STATE;
  std::lock_guard<std::mutex> lk(G().mu);
  FILE* f = std::fopen(path, "wb");
  if (!f) return HPOP_E_ARG;
  bool ok = std::fwrite("HPOPTRC1", 1, 8, f) == 8;
  const int32_t hdr[2] = {1, G().n_dev};
  const int64_t span[2] = {G().t_begin, G().sealed};
  int32_t n_chunks = 0;
  for (const Series& q : G().series) n_chunks += q.s.empty() ? 0 : 1;
  ok = ok && std::fwrite(hdr, sizeof hdr, 1, f) == 1 && std::fwrite(span, sizeof span, 1, f) == 1 &&
       std::fwrite(&n_chunks, sizeof n_chunks, 1, f) == 1;
  for (size_t i = 0; ok && i < G().series.size(); ++i) {
    const Series& q = G().series[i];
    if (q.s.empty()) continue;
    const int32_t rk[2] = {(int32_t)(i / kKinds), (int32_t)(i % kKinds)};
    const int64_t n = (int64_t)q.s.size();
    ok = std::fwrite(rk, sizeof rk, 1, f) == 1 && std::fwrite(&n, sizeof n, 1, f) == 1 &&
         std::fwrite(q.s.data(), sizeof(int64_t), q.s.size(), f) == q.s.size() &&
         std::fwrite(q.e.data(), sizeof(int64_t), q.e.size(), f) == q.e.size();
  }
  ok = (std::fclose(f) == 0) && ok;
  return ok ? HPOP_OK : HPOP_E_ARG;
}

int64_t hpop_collect_dropped(void) { return G().dropped.load(); }

}  // extern "C"
