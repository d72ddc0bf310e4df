// hpop_metrics_compute_static: the session path's build and region kernels
// over records the caller already holds in device memory, with every
// intermediate buffer carved from one file-scope device array instead of
// allocated. For callers that cannot allocate device memory.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <climits>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "hpop.h"
#include "hpop_internal.h"
#include "hpop_runtime.h"

using namespace hpop;

// Every build intermediate of one call: bucketed records, merged intervals
// of each level, per-bucket and per-segment words, descriptors and results.
// One copy per GPU, loaded with this file's code object and held until the
// process ends. Host code never passes this name to a kernel or a copy: it
// is a host-side stand-in; the device address comes from hipGetSymbolAddress.
static __device__ __align__(256) unsigned char scratch[HPOP_STATIC_SCRATCH_BYTES];

namespace {

constexpr size_t kScratchBytes = HPOP_STATIC_SCRATCH_BYTES;

void* refuse_alloc(void*, size_t, void*) { return nullptr; }  // nothing here may allocate
void ignore_free(void*, void*, void*) {}

struct StaticDevice {
  std::mutex mu;          // one call at a time per GPU in this process
  char* ptr = nullptr;    // device address of `scratch` on this GPU
  Engine engine;
  std::vector<char> result;  // trees and status words copied back
  std::vector<int32_t> chunk_index;  // caller's chunk index of each descriptor
};

std::mutex g_devices_mu;
std::vector<StaticDevice*> g_devices;  // never freed: each GPU keeps its array until exit

hpop_status fail(hpop_status code, const std::string& msg) {
  g_thread_error = msg;
  return code;
}

// The state of GPU `dev` (current on this thread), resolving the array's
// address there on first use.
hpop_status device_state(int dev, StaticDevice** out) {
  std::lock_guard<std::mutex> g(g_devices_mu);
  if ((int)g_devices.size() <= dev) g_devices.resize((size_t)dev + 1, nullptr);
  if (!g_devices[dev]) {
    char* p = nullptr;
    const hipError_t e = hipGetSymbolAddress((void**)&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
      return fail(HPOP_E_HIP, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
    StaticDevice* d = new StaticDevice();
    d->ptr = p;
    d->engine.alloc.fn_alloc = refuse_alloc;
    d->engine.alloc.fn_free = ignore_free;
    d->engine.use_graphs = false;
    d->engine.ws.fixed = p;
    d->engine.ws.fixed_bytes = kScratchBytes;
    g_devices[dev] = d;
  }
  *out = g_devices[dev];
  return HPOP_OK;
}

bool is_device_memory(const void* p) {
  hipPointerAttribute_t a;
  if (hipPointerGetAttributes(&a, p) != hipSuccess) {
    (void)hipGetLastError();
    return false;
  }
  return a.type == hipMemoryTypeDevice || a.type == hipMemoryTypeManaged;
}

hpop_status check_args(int32_t n_hosts, int32_t n_devices, const hpop_event_chunk* chunks, int32_t n_chunks,
                       const int64_t* t0, const int64_t* t1, int32_t n_regions, const hpop_metric_tree* out) {
  if (n_hosts < 0 || n_devices < 0 || n_hosts + (long long)n_devices > (1 << 24))
    return fail(HPOP_E_ARG, "n_hosts and n_devices must be >= 0 with n + m <= 2^24");
  if (n_chunks < 0 || (n_chunks > 0 && !chunks)) return fail(HPOP_E_ARG, "bad chunk list");
  if (n_regions < 0 || (n_regions > 0 && (!t0 || !t1 || !out))) return fail(HPOP_E_ARG, "bad region list or output");
  const int R = n_hosts + n_devices;
  for (int32_t i = 0; i < n_chunks; ++i) {
    const hpop_event_chunk& c = chunks[i];
    if (c.resource < 0 || c.resource >= R) return fail(HPOP_E_RESOURCE, "chunk " + std::to_string(i) + ": bad resource");
    const bool host = c.resource < n_hosts;
    const bool host_kind = c.kind == HPOP_HOST_USEFUL || c.kind == HPOP_HOST_OFFLOAD || c.kind == HPOP_HOST_MPI;
    const bool dev_kind = c.kind == HPOP_DEV_KERNEL || c.kind == HPOP_DEV_MEMOP;
    if (host ? !host_kind : !dev_kind)
      return fail(HPOP_E_KIND, "chunk " + std::to_string(i) + ": kind does not fit the resource");
    if (c.count < 0 || c.count > (1ll << 40) || (c.count > 0 && (!c.start || !c.end)))
      return fail(HPOP_E_ARG, "chunk " + std::to_string(i) + ": bad count or null array");
    if (c.count > 0 && (!is_device_memory(c.start) || !is_device_memory(c.end)))
      return fail(HPOP_E_ARG, "chunk " + std::to_string(i) + ": start and end must be device memory");
  }
  const unsigned long long w = (unsigned long long)std::max(1, std::max(n_hosts, n_devices));
  for (int32_t g = 0; g < n_regions; ++g) {
    if (!(t0[g] < t1[g])) return fail(HPOP_E_REGION, "region " + std::to_string(g) + " needs t0 < t1");
    if (t0[g] < -kTimeLimit || t1[g] > kTimeLimit)
      return fail(HPOP_E_REGION, "region " + std::to_string(g) + " bounds out of range");
    const unsigned long long E = (unsigned long long)(t1[g] - t0[g]);
    if (E >= (1ull << 53) || E * w >= (1ull << 53))
      return fail(HPOP_E_OVERFLOW, "region " + std::to_string(g) +
                                       ": (t1 - t0) * max(n, m) must be below 2^53 for exact FP64 ratios");
  }
  return HPOP_OK;
}

// Descriptors of one call in the engine (one owner; segments are the
// resources, hosts first; regions in order) and its plan in the scratch array.
hpop_status plan(StaticDevice& d, int32_t n_hosts, int32_t n_devices, const hpop_event_chunk* chunks,
                 int32_t n_chunks, const int64_t* t0, const int64_t* t1, int32_t n_regions, std::string& err) {
  Engine& E = d.engine;
  const int R = n_hosts + n_devices;
  E.h_chunks.clear();
  E.h_regions.clear();
  E.h_ivls.clear();
  E.chunk_owner.clear();
  d.chunk_index.clear();
  std::vector<long long> seg_count((size_t)R, 0);
  std::vector<char> seg_host((size_t)R, 0);
  for (int r = 0; r < n_hosts; ++r) seg_host[r] = 1;
  for (int32_t i = 0; i < n_chunks; ++i) {
    const hpop_event_chunk& c = chunks[i];
    if (c.count == 0) continue;
    ChunkDesc cd;
    cd.s = c.start;
    cd.e = c.end;
    cd.count = c.count;
    cd.tile_begin = 0;
    cd.seg = c.resource;
    cd.slot = slot_of_kind(c.kind);
    cd.chunk_id = (int32_t)E.h_chunks.size();
    cd.owner = 0;
    E.h_chunks.push_back(cd);
    d.chunk_index.push_back(i);
    seg_count[c.resource] += c.count;
  }
  for (int32_t g = 0; g < n_regions; ++g) {
    RegionDesc rd;
    rd.t0 = t0[g];
    rd.t1 = t1[g];
    rd.seg_begin = 0;
    rd.n_hosts = n_hosts;
    rd.n_devices = n_devices;
    rd.n_ivl = 0;
    rd.times_off = (int64_t)g * R;
    rd.ivl_begin = 0;
    E.h_regions.push_back(rd);
  }
  const hpop_tuning defaults{};
  hpop_status st = E.assemble_plan(defaults, seg_count, seg_host, 1, (long long)n_regions * R, err);
  if (st == HPOP_E_ARG && E.ws.fixed_needed > E.ws.fixed_bytes && !E.exact_forced) {
    // fixed scatter slots do not fit: exact offsets need less room
    E.exact_forced = true;
    st = E.assemble_plan(defaults, seg_count, seg_host, 1, (long long)n_regions * R, err);
  }
  return st;
}

}  // namespace

extern "C" hpop_status hpop_metrics_compute_static(int32_t n_hosts, int32_t n_devices, const hpop_event_chunk* chunks,
                                                   int32_t n_chunks, const int64_t* region_t0,
                                                   const int64_t* region_t1, int32_t n_regions, void* stream,
                                                   hpop_metric_tree* out, int64_t* times_out) {
  try {
    hpop_status st = check_args(n_hosts, n_devices, chunks, n_chunks, region_t0, region_t1, n_regions, out);
    if (st != HPOP_OK) return st;
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return fail(HPOP_E_HIP, std::string("hipGetDevice: ") + hipGetErrorString(e));
    StaticDevice* d = nullptr;
    st = device_state(dev, &d);
    if (st != HPOP_OK) return st;
    std::lock_guard<std::mutex> g(d->mu);
    Engine& E = d->engine;
    E.alloc.stream = (hipStream_t)stream;
    E.exact_forced = false;
    const size_t bt = (size_t)n_regions * sizeof(Tree);
    std::string err;
    for (int attempt = 0; attempt < 2; ++attempt) {
      st = plan(*d, n_hosts, n_devices, chunks, n_chunks, region_t0, region_t1, n_regions, err);
      if (st != HPOP_OK) return fail(st, err);
      d->result.assign(bt + 24, 0);
      E.result_host = d->result.data();
      st = E.upload(err);
      if (st == HPOP_OK) st = E.enqueue(true, false, err);
      if (st != HPOP_OK) return fail(st, err);
      e = hipStreamSynchronize((hipStream_t)stream);
      if (e != hipSuccess) return fail(HPOP_E_HIP, std::string("hipStreamSynchronize: ") + hipGetErrorString(e));
      unsigned long long bad, slot_over;
      memcpy(&bad, d->result.data() + bt, 8);
      memcpy(&slot_over, d->result.data() + bt + 16, 8);
      if (bad != ULLONG_MAX) {
        const unsigned long long cid = bad >> 40, idx = bad & ((1ull << 40) - 1);
        const int ci = cid < d->chunk_index.size() ? d->chunk_index[cid] : -1;
        return fail(HPOP_E_BAD_INTERVAL, "invalid record: chunk " + std::to_string(ci) + ", index " +
                                             std::to_string(idx) + " (need 0 <= start <= end < 2^62)");
      }
      if (slot_over > 0 && E.ws.plan.slot_cap > 0) {
        // a bucket outgrew its fixed slots: the same call with exact offsets
        E.exact_forced = true;
        continue;
      }
      if (bt) memcpy(out, d->result.data(), bt);
      const size_t btimes = (size_t)n_regions * (size_t)(n_hosts + n_devices) * 32;
      if (times_out && btimes) {
        e = hipMemcpy(times_out, E.ws.d_times, btimes, hipMemcpyDeviceToHost);
        if (e != hipSuccess) return fail(HPOP_E_HIP, std::string("hipMemcpy: ") + hipGetErrorString(e));
      }
      return HPOP_OK;
    }
    return fail(HPOP_E_STATE, "slot overflow persisted with exact offsets");
  } catch (const std::bad_alloc&) {
    return fail(HPOP_E_OOM, "host allocation failed");
  } catch (...) {
    return fail(HPOP_E_STATE, "internal error");
  }
}
