// Stream concurrency (the C entry points declared under "Stream concurrency"
// in hpop.h): union measures per stream and per device from the engine's
// own build and clip, reduced per region on the GPU.
#include <hip/hip_runtime.h>

#include <cstring>
#include <string>
#include <vector>

#include "hpop.h"
#include "hpop_runtime.h"

using namespace hpop;

namespace {

constexpr int kThreads = 256;

// One workgroup per region. times: the inner session's per-resource state
// times ([row][4], K first); a device's busy time is the K of its first
// inner resource, its stream time the sum of the K of the S_g that follow.
__global__ __launch_bounds__(kThreads) void k_stream_tree(const long long* times, const long long* times_off,
                                                           const int* stream_n, const int* stream_off, int m,
                                                           hpop_stream_tree* trees, long long* per_dev) {
  __shared__ long long red[4][kThreads];
  const int r = blockIdx.x, tid = threadIdx.x;
  const long long base = times_off[r];
  long long busy = 0, st = 0, cap = 0, ns = 0;
  for (int g = tid; g < m; g += kThreads) {
    const long long o = base + stream_off[g];
    const long long S = stream_n[g];
    const long long B = times[o * 4];
    long long ST = 0;
    for (long long j = 0; j < S; ++j) ST += times[(o + 1 + j) * 4];
    if (per_dev) {
      long long* q = per_dev + ((long long)r * m + g) * 3;
      q[0] = B;
      q[1] = ST;
      q[2] = S;
    }
    busy += B;
    st += ST;
    cap += S * B;
    ns += S;
  }
  red[0][tid] = busy;
  red[1][tid] = st;
  red[2][tid] = cap;
  red[3][tid] = ns;
  __syncthreads();
  for (int w = kThreads / 2; w > 0; w >>= 1) {
    if (tid < w)
      for (int k = 0; k < 4; ++k) red[k][tid] += red[k][tid + w];
    __syncthreads();
  }
  if (tid == 0) {
    hpop_stream_tree t{};
    t.busy = red[0][0];
    t.stream_time = red[1][0];
    t.capacity = red[2][0];
    t.m = m;
    t.n_streams = (int32_t)red[3][0];
    unsigned int mask = 0;
    // one IEEE division of exact integers each; 0/0 := 1 and flagged
    if (t.capacity == 0) {
      t.stream_eff = 1.0;
      mask |= 1u;
    } else {
      t.stream_eff = (double)t.stream_time / (double)t.capacity;
    }
    if (t.busy == 0) {
      t.mean_active = 1.0;
      mask |= 2u;
    } else {
      t.mean_active = (double)t.stream_time / (double)t.busy;
    }
    t.undefined_mask = mask;
    trees[r] = t;
  }
}

hpop_status sfail(hpop_session* s, hpop_status code, const std::string& msg) {
  if (s) s->last_error = msg;
  else g_thread_error = msg;
  return code;
}

size_t align256(size_t b) { return (b + 255) & ~size_t(255); }

}  // namespace

#define HPOP_SGUARD_BEGIN try {
#define HPOP_SGUARD_END(sess)                                                     \
  }                                                                               \
  catch (const std::bad_alloc&) {                                                 \
    return sfail(sess, HPOP_E_OOM, "host allocation failed");                     \
  }                                                                               \
  catch (...) {                                                                   \
    return sfail(sess, HPOP_E_STATE, "internal error");                           \
  }

extern "C" {

hpop_status hpop_session_set_streams(hpop_session* s, const int32_t* n_streams) {
  HPOP_SGUARD_BEGIN
  if (!s) return sfail(nullptr, HPOP_E_ARG, "null session");
  if (s->n_devices > 0 && !n_streams) return sfail(s, HPOP_E_ARG, "null stream counts");
  if (s->streams && s->streams->n_events > 0)
    return sfail(s, HPOP_E_STATE, "streams are fixed once stream records were added");
  std::vector<int32_t> n((size_t)s->n_devices), off((size_t)s->n_devices);
  long long total = 0;
  for (int g = 0; g < s->n_devices; ++g) {
    if (n_streams[g] < 0) return sfail(s, HPOP_E_ARG, "negative stream count on device " + std::to_string(g));
    n[g] = n_streams[g];
    off[g] = (int32_t)total;
    total += (long long)n_streams[g] + 1;
    if (total > (1ll << 24)) return sfail(s, HPOP_E_ARG, "at most 2^24 streams plus devices");
  }
  hpop_session_config cfg{};
  cfg.n_hosts = 0;
  cfg.n_devices = (int32_t)total;
  cfg.stream = s->stream;
  cfg.alloc = s->alloc.fn_alloc;
  cfg.free = s->alloc.fn_free;
  cfg.alloc_ctx = s->alloc.ctx;
  hpop_session* inner = nullptr;
  const hpop_status st = hpop_session_create(&cfg, &inner);
  if (st != HPOP_OK) return sfail(s, st, hpop_last_error(nullptr));
  if (s->streams) hpop_session_destroy(s->streams);
  s->streams = inner;
  s->stream_n = std::move(n);
  s->stream_off = std::move(off);
  return HPOP_OK;
  HPOP_SGUARD_END(s)
}

hpop_status hpop_add_stream_events(hpop_session* s, int32_t resource, int32_t stream, const int64_t* start,
                                   const int64_t* end, int64_t count, int32_t mem_space) {
  HPOP_SGUARD_BEGIN
  if (!s) return sfail(nullptr, HPOP_E_ARG, "null session");
  if (!s->streams) return sfail(s, HPOP_E_STATE, "call hpop_session_set_streams first");
  if (resource < s->n_hosts || resource >= s->n_hosts + s->n_devices)
    return sfail(s, HPOP_E_RESOURCE, "resource " + std::to_string(resource) + " is not a device");
  const int g = resource - s->n_hosts;
  if (stream < 0 || stream >= s->stream_n[g])
    return sfail(s, HPOP_E_RESOURCE, "stream " + std::to_string(stream) + " not declared on device " + std::to_string(g));
  hpop_session* in = s->streams;
  // state of the inner session before the call, to undo it if the outer add fails
  const size_t n_chunks = in->chunks.size(), arena_used = in->arena_used;
  const int64_t n_events = in->n_events, n_calls = in->n_calls;
  hpop_event_chunk c[2];
  c[0].resource = s->stream_off[g];
  c[1].resource = s->stream_off[g] + 1 + stream;
  for (hpop_event_chunk& x : c) {
    x.kind = HPOP_DEV_KERNEL;
    x.start = start;
    x.end = end;
    x.count = count;
  }
  hpop_status st = hpop_add_events_multi(in, c, 2, mem_space);
  if (st != HPOP_OK) return sfail(s, st, in->last_error);
  st = hpop_add_events(s, resource, HPOP_DEV_KERNEL, start, end, count, mem_space);
  if (st != HPOP_OK) {
    in->chunks.resize(n_chunks);
    in->arena_used = arena_used;
    in->arena.used = arena_used;
    in->n_events = n_events;
    in->n_calls = n_calls;
    ++in->version;
    return st;  // the outer session holds the message
  }
  return HPOP_OK;
  HPOP_SGUARD_END(s)
}

hpop_status hpop_stream_metrics(hpop_session* s, uint32_t flags, hpop_stream_tree* out, int64_t* per_device) {
  HPOP_SGUARD_BEGIN
  if (!s) return sfail(nullptr, HPOP_E_ARG, "null session");
  if (!s->streams) return sfail(s, HPOP_E_STATE, "call hpop_session_set_streams first");
  const size_t nreg = s->regions.size();
  if (nreg && !out) return sfail(s, HPOP_E_ARG, "null output");
  long long n_total = 0;
  for (int32_t n : s->stream_n) n_total += n;
  for (size_t r = 0; r < nreg; ++r) {
    if (!s->region_ivls[r].empty())
      return sfail(s, HPOP_E_REGION, "region " + std::to_string(r) + " is given per resource; stream measures need one span");
    const unsigned long long E = (unsigned long long)(s->regions[r].second - s->regions[r].first);
    if (n_total > 0 && E >= (1ull << 53) / (unsigned long long)n_total)
      return sfail(s, HPOP_E_OVERFLOW, "(t1 - t0) * streams must be below 2^53 for exact FP64 ratios");
  }
  hpop_session* in = s->streams;
  // the inner session answers the same regions (regions are only ever appended)
  while (in->regions.size() < nreg) {
    in->regions.push_back(s->regions[in->regions.size()]);
    in->region_ivls.emplace_back();
  }
  in->tuning = s->tuning;
  std::vector<hpop_metric_tree> inner_trees(nreg ? nreg : 1);
  hpop_status st = hpop_metrics_compute_all(in, flags, inner_trees.data());
  if (st != HPOP_OK) return sfail(s, st, in->last_error);
  if (nreg == 0) return HPOP_OK;
  const int m = s->n_devices;
  // device tables and outputs in one buffer
  const size_t b_off = align256(nreg * sizeof(long long)), b_n = align256((size_t)m * sizeof(int32_t) + 4),
               b_so = b_n, b_tree = align256(nreg * sizeof(hpop_stream_tree)),
               b_per = align256(nreg * (size_t)m * 3 * sizeof(long long) + 8);
  const size_t in_bytes = b_off + b_n + b_so;
  if (!s->stream_buf.reserve(s->alloc, in_bytes + b_tree + b_per, false))
    return sfail(s, HPOP_E_OOM, "device allocation for stream measures failed");
  std::vector<char> h(in_bytes, 0);
  long long* h_off = (long long*)h.data();
  for (size_t r = 0; r < nreg; ++r) h_off[r] = in->engine.h_regions[r].times_off;
  std::memcpy(h.data() + b_off, s->stream_n.data(), (size_t)m * sizeof(int32_t));
  std::memcpy(h.data() + b_off + b_n, s->stream_off.data(), (size_t)m * sizeof(int32_t));
  char* d = (char*)s->stream_buf.ptr;
  hpop_stream_tree* d_tree = (hpop_stream_tree*)(d + in_bytes);
  long long* d_per = (long long*)(d + in_bytes + b_tree);
  hipError_t e = hipMemcpyAsync(d, h.data(), in_bytes, hipMemcpyHostToDevice, s->stream);
  if (e == hipSuccess) {
    hipLaunchKernelGGL(k_stream_tree, dim3((unsigned)nreg), dim3(kThreads), 0, s->stream, in->engine.ws.d_times,
                       (const long long*)d, (const int*)(d + b_off), (const int*)(d + b_off + b_n), m, d_tree,
                       per_device ? d_per : nullptr);
    e = hipGetLastError();
  }
  if (e == hipSuccess) e = hipMemcpyAsync(out, d_tree, nreg * sizeof(hpop_stream_tree), hipMemcpyDeviceToHost, s->stream);
  if (e == hipSuccess && per_device)
    e = hipMemcpyAsync(per_device, d_per, nreg * (size_t)m * 3 * sizeof(long long), hipMemcpyDeviceToHost, s->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(s->stream);
  if (e != hipSuccess) return sfail(s, HPOP_E_HIP, std::string("stream measures: ") + hipGetErrorString(e));
  return HPOP_OK;
  HPOP_SGUARD_END(s)
}

}  // extern "C"
