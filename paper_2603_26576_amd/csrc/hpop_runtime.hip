// Host runtime of the engine: sessions, record storage, build plans, the
// batched path with HIP-graph replay, and the C ABI declared in hpop.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <climits>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "hpop.h"
#include "hpop_internal.h"
#include "hpop_kernels.h"
#include "hpop_runtime.h"

using namespace hpop;

static_assert(sizeof(Tree) == sizeof(hpop_metric_tree), "tree layout");

namespace hpop {

thread_local std::string g_thread_error;
thread_local double g_alloc_us = 0.0;

const char* status_name(hpop_status s) {
  switch (s) {
    case HPOP_OK: return "ok";
    case HPOP_E_ARG: return "invalid argument";
    case HPOP_E_KIND: return "invalid record kind for this resource";
    case HPOP_E_RESOURCE: return "resource id out of range";
    case HPOP_E_BAD_INTERVAL: return "invalid interval (need 0 <= start <= end < 2^62)";
    case HPOP_E_REGION: return "invalid region";
    case HPOP_E_OVERFLOW: return "region too long for exact FP64 ratios";
    case HPOP_E_OOM: return "out of memory";
    case HPOP_E_BUSY: return "server queue full";
    case HPOP_E_HIP: return "HIP runtime error";
    case HPOP_E_TIMEOUT: return "timed out";
    case HPOP_E_STATE: return "invalid state";
    default: return "unknown status";
  }
}

int slot_of_kind(int kind) {
  switch (kind) {
    case HPOP_HOST_USEFUL: return 0;
    case HPOP_HOST_OFFLOAD: return 1;
    case HPOP_HOST_MPI: return 2;
    case HPOP_DEV_KERNEL: return 0;
    case HPOP_DEV_MEMOP: return 1;
    default: return -1;
  }
}

// ----------------------------------------------------------------------------
// device memory
// ----------------------------------------------------------------------------

// The library's own stream-ordered pool per device. Memory freed back to it
// stays cached (release threshold = all), so the grow-and-copy of session
// lists and workspaces does not return memory to the driver and map it again.
static hipMemPool_t library_pool(int dev) {
  static std::mutex mu;
  static std::vector<hipMemPool_t> pools;
  std::lock_guard<std::mutex> g(mu);
  if ((int)pools.size() <= dev) pools.resize(dev + 1, nullptr);
  if (!pools[dev]) {
    hipMemPoolProps props{};
    props.allocType = hipMemAllocationTypePinned;
    props.handleTypes = hipMemHandleTypeNone;
    props.location.type = hipMemLocationTypeDevice;
    props.location.id = dev;
    hipMemPool_t pool = nullptr;
    if (hipMemPoolCreate(&pool, &props) != hipSuccess) {
      (void)hipGetLastError();
      return nullptr;
    }
    unsigned long long keep = ~0ull;
    (void)hipMemPoolSetAttribute(pool, hipMemPoolAttrReleaseThreshold, &keep);
    pools[dev] = pool;
  }
  return pools[dev];
}

void* Alloc::get(size_t bytes) {
  if (bytes == 0) bytes = 256;
  void* p = nullptr;
  if (fn_alloc) return fn_alloc(ctx, bytes, (void*)stream);
  const auto t0 = std::chrono::steady_clock::now();
  int dev = 0;
  hipMemPool_t pool = hipGetDevice(&dev) == hipSuccess ? library_pool(dev) : nullptr;
  const hipError_t e = pool ? hipMallocFromPoolAsync(&p, bytes, pool, stream) : hipMallocAsync(&p, bytes, stream);
  g_alloc_us += std::chrono::duration<double, std::micro>(std::chrono::steady_clock::now() - t0).count();
  if (e != hipSuccess) {
    (void)hipGetLastError();
    p = nullptr;
  }
  return p;
}

void Alloc::put(void* p) {
  if (!p) return;
  if (fn_free) fn_free(ctx, p, (void*)stream);
  else (void)hipFreeAsync(p, stream);
}

bool DevBuf::reserve(Alloc& a, size_t need, bool keep) {
  if (need <= bytes && ptr) return true;
  size_t nb = std::max(need, bytes + bytes / 2);
  nb = (nb + 255) & ~size_t(255);
  void* q = a.get(nb);
  if (!q) return false;
  if (keep && ptr && used) {
    if (hipMemcpyAsync(q, ptr, used, hipMemcpyDeviceToDevice, a.stream) != hipSuccess) {
      a.put(q);
      return false;
    }
  }
  a.put(ptr);
  ptr = q;
  bytes = nb;
  return true;
}

void DevBuf::release(Alloc& a) {
  a.put(ptr);
  ptr = nullptr;
  bytes = 0;
  used = 0;
}

bool PinnedBuf::reserve(size_t need) {
  if (need <= bytes && ptr) return true;
  size_t nb = std::max(need, bytes * 2);
  nb = std::max<size_t>(nb, 4096);
  void* q = nullptr;
  const auto t0 = std::chrono::steady_clock::now();
  const hipError_t e = hipHostMalloc(&q, nb, hipHostMallocDefault);
  g_alloc_us += std::chrono::duration<double, std::micro>(std::chrono::steady_clock::now() - t0).count();
  if (e != hipSuccess) {
    (void)hipGetLastError();
    return false;
  }
  if (ptr) (void)hipHostFree(ptr);
  ptr = q;
  bytes = nb;
  return true;
}

void PinnedBuf::release() {
  if (ptr) (void)hipHostFree(ptr);
  ptr = nullptr;
  bytes = 0;
}

// ----------------------------------------------------------------------------
// workspace of one build plan
// ----------------------------------------------------------------------------

template <class T>
static T* carve(char*& cur, size_t n) {
  T* p = reinterpret_cast<T*>(cur);
  cur += (n * sizeof(T) + 255) & ~size_t(255);
  return p;
}

static size_t carve_bytes(size_t n, size_t sz) { return (n * sz + 255) & ~size_t(255); }

hpop_status Workspace::prepare(Alloc& a, long long n_chunks, long long n_tiles, long long n_segs,
                               long long n_buckets, long long n_elems, long long n_slots, long long n_regions,
                               long long n_times, long long n_owners, long long n_ivls, std::string& err) {
  const size_t nscan = (size_t)((n_buckets + kScanTile - 1) / kScanTile + 1);
  size_t small = 0;
  small += carve_bytes(n_chunks, sizeof(ChunkDesc));
  small += carve_bytes(n_tiles, sizeof(int32_t));
  small += carve_bytes(n_segs, sizeof(SegDesc));
  small += carve_bytes(n_segs, sizeof(SegStats));
  small += carve_bytes(n_segs, sizeof(SegGeom));
  small += carve_bytes(n_buckets, sizeof(unsigned int)) * 2;
  small += carve_bytes(n_buckets + 1, sizeof(unsigned long long));
  small += carve_bytes(n_buckets, sizeof(unsigned long long));
  small += carve_bytes(3 * n_buckets, sizeof(unsigned long long));
  small += carve_bytes(3 * n_buckets, sizeof(long long)) * 3;
  small += carve_bytes(3 * n_buckets, sizeof(unsigned int));
  small += carve_bytes(3 * n_segs, sizeof(long long));
  small += carve_bytes(1, 8) + carve_bytes(nscan, 8) + carve_bytes(4, 4) + carve_bytes(2, 8);
  small += carve_bytes(n_buckets, sizeof(unsigned int));
  small += carve_bytes(n_owners, sizeof(unsigned int));
  small += carve_bytes(n_regions, sizeof(RegionDesc)) + carve_bytes(n_regions, sizeof(Tree));
  small += carve_bytes(9 * n_regions, sizeof(unsigned long long));
  small += carve_bytes(n_ivls, sizeof(IvlDesc)) + carve_bytes(n_ivls ? 4 * n_times : 0, sizeof(long long));
  small += carve_bytes(4 * n_times, sizeof(long long));
  // bucketed records: fixed slots per bucket (n_slots > 0) or exact offsets,
  // where oversized buckets also need a scratch copy for their global sort
  const size_t big_e = carve_bytes(n_slots > 0 ? n_slots : n_elems, sizeof(Elem));
  const size_t big_e2 = carve_bytes(n_slots > 0 ? 1 : n_elems, sizeof(Elem));
  const size_t big_c = carve_bytes(n_elems, sizeof(Comp)), big_n = carve_bytes(n_elems, sizeof(CompN));
  char* meta_p;
  char* elems_p;
  char* elems2_p;
  char* comp_p[3];
  char* compn_p[3];
  if (fixed) {
    // one caller-provided region holds everything, in this order
    fixed_needed = small + big_e + big_e2 + 3 * (big_c + big_n);
    if (fixed_needed > fixed_bytes) {
      err = "the build needs " + std::to_string(fixed_needed) + " bytes of scratch; " +
            std::to_string(fixed_bytes) + " are available";
      return HPOP_E_ARG;
    }
    char* c = fixed;
    meta_p = c;
    c += small;
    elems_p = c;
    c += big_e;
    elems2_p = c;
    c += big_e2;
    for (int l = 0; l < 3; ++l) {
      comp_p[l] = c;
      c += big_c;
      compn_p[l] = c;
      c += big_n;
    }
  } else {
    if (!meta.reserve(a, small, false)) {
      err = "device allocation of " + std::to_string(small) + " bytes (build metadata) failed";
      return HPOP_E_OOM;
    }
    if (!elems.reserve(a, big_e, false) || !elems2.reserve(a, big_e2, false) || !comp[0].reserve(a, big_c, false) ||
        !comp[1].reserve(a, big_c, false) || !comp[2].reserve(a, big_c, false) ||
        !compn[0].reserve(a, big_n, false) || !compn[1].reserve(a, big_n, false) ||
        !compn[2].reserve(a, big_n, false)) {
      err = "device allocation for " + std::to_string(n_elems) + " records failed";
      return HPOP_E_OOM;
    }
    meta_p = (char*)meta.ptr;
    elems_p = (char*)elems.ptr;
    elems2_p = (char*)elems2.ptr;
    for (int l = 0; l < 3; ++l) {
      comp_p[l] = (char*)comp[l].ptr;
      compn_p[l] = (char*)compn[l].ptr;
    }
  }
  char* cur = meta_p;
  Plan& p = plan;
  p.chunks = d_chunks = carve<ChunkDesc>(cur, n_chunks);
  p.tile_chunk = carve<int32_t>(cur, n_tiles);
  p.segs = d_segs = carve<SegDesc>(cur, n_segs);
  p.stats = carve<SegStats>(cur, n_segs);
  p.geom = carve<SegGeom>(cur, n_segs);
  p.counts = carve<unsigned int>(cur, n_buckets);
  p.bucket_seg = carve<int32_t>(cur, n_buckets);
  p.offsets = carve<unsigned long long>(cur, n_buckets + 1);
  p.cursor = carve<unsigned long long>(cur, n_buckets);
  p.maxend = carve<unsigned long long>(cur, 3 * n_buckets);
  p.carry = carve<long long>(cur, 3 * n_buckets);
  p.bsum = carve<long long>(cur, 3 * n_buckets);
  p.base = carve<long long>(cur, 3 * n_buckets);
  p.ncomp = carve<unsigned int>(cur, 3 * n_buckets);
  p.seg_total = carve<long long>(cur, 3 * n_segs);
  p.err = carve<unsigned long long>(cur, 1);
  p.scan_state = carve<unsigned long long>(cur, nscan);
  p.ticket = carve<unsigned int>(cur, 4);
  p.oversized = carve<unsigned long long>(cur, 2);
  p.queue = carve<unsigned int>(cur, n_buckets);
  p.owner_err = carve<unsigned int>(cur, n_owners);
  p.n_owners = (int32_t)n_owners;
  p.seg_group = 1;
  d_regions = carve<RegionDesc>(cur, n_regions);
  d_trees = carve<Tree>(cur, n_regions);
  p.racc = carve<unsigned long long>(cur, 9 * n_regions);
  p.n_racc = n_regions;
  d_times = carve<long long>(cur, 4 * n_times);
  d_ivls = carve<IvlDesc>(cur, n_ivls);
  d_macc = carve<long long>(cur, n_ivls ? 4 * n_times : 0);
  p.elems = (Elem*)elems_p;
  p.elems2 = (Elem*)elems2_p;
  for (int l = 0; l < 3; ++l) {
    p.comp[l] = (Comp*)comp_p[l];
    p.compn[l] = (CompN*)compn_p[l];
  }
  p.n_chunks = (int32_t)n_chunks;
  p.n_segs = (int32_t)n_segs;
  p.n_buckets = n_buckets;
  p.n_elems = n_elems;
  ++layout_gen;
  return HPOP_OK;
}

void Workspace::release(Alloc& a) {
  meta.release(a);
  elems.release(a);
  elems2.release(a);
  for (auto& c : comp) c.release(a);
  for (auto& c : compn) c.release(a);
  if (graph_exec) (void)hipGraphExecDestroy(graph_exec);
  graph_exec = nullptr;
  if (desc_done) {
    (void)hipEventSynchronize(desc_done);
    (void)hipEventDestroy(desc_done);
  }
  desc_done = nullptr;
  pinned.release();
  pinned_desc.release();
}

// ----------------------------------------------------------------------------
// plan assembly and the launch sequence
// ----------------------------------------------------------------------------

static hpop_status hip_fail(std::string& err, const char* what, hipError_t e) {
  err = std::string(what) + ": " + hipGetErrorString(e);
  return HPOP_E_HIP;
}

#define HPOP_HIP(call, what)                                 \
  do {                                                       \
    hipError_t e_ = (call);                                  \
    if (e_ != hipSuccess) return hip_fail(err, what, e_);    \
  } while (0)

static int pow2ceil(int x) {
  int v = 1;
  while (v < x) v <<= 1;
  return v;
}

static void tuned(const hpop_tuning& t, int& target, int& cap, int& tile, int& slots) {
  target = t.bucket_target > 0 ? std::min(4096, std::max(16, t.bucket_target)) : 352;
  cap = t.bucket_cap == 4096 ? 4096 : 2048;
  tile = t.tile_elems == 512 || t.tile_elems == 2048 || t.tile_elems == 8192 ? t.tile_elems : 4096;
  // single-pass scatter slots: 4x the mean bucket, within the on-chip capacity
  if (t.scatter_slots < 0) slots = 0;
  else if (t.scatter_slots > 0) slots = std::min(cap, pow2ceil(std::max(64, t.scatter_slots)));
  else slots = std::min(cap, pow2ceil(4 * target));
}

// The k sessions of `ss` become one plan: segments are session by session,
// hosts before devices; regions likewise.
hpop_status Engine::assemble(hpop_session* const* ss, int k, std::string& err) {
  h_chunks.clear();
  h_regions.clear();
  h_ivls.clear();
  chunk_owner.clear();
  seg_of_session.assign(k, 0);
  reg_of_session.assign(k, 0);
  std::vector<long long> seg_count;
  std::vector<char> seg_host;
  long long times = 0;
  int seg_base = 0;
  for (int i = 0; i < k; ++i) {
    hpop_session* s = ss[i];
    const int R = s->n_hosts + s->n_devices;
    seg_of_session[i] = seg_base;
    for (int r = 0; r < R; ++r) {
      seg_count.push_back(0);
      seg_host.push_back(r < s->n_hosts ? 1 : 0);
    }
    for (size_t c = 0; c < s->chunks.size(); ++c) {
      const RecChunk& rc = s->chunks[c];
      if (rc.count == 0) continue;
      ChunkDesc d;
      d.s = (const int64_t*)((char*)s->arena.ptr + rc.off_s);
      d.e = (const int64_t*)((char*)s->arena.ptr + rc.off_e);
      d.count = rc.count;
      d.tile_begin = 0;
      d.seg = seg_base + rc.resource;
      d.slot = slot_of_kind(rc.kind);
      d.chunk_id = (int32_t)h_chunks.size();
      d.owner = i;
      h_chunks.push_back(d);
      chunk_owner.push_back(std::make_pair(i, (int)c));
      seg_count[seg_base + rc.resource] += rc.count;
    }
    reg_of_session[i] = (int)h_regions.size();
    for (size_t g = 0; g < s->regions.size(); ++g) {
      RegionDesc rd;
      rd.t0 = s->regions[g].first;
      rd.t1 = s->regions[g].second;
      rd.seg_begin = seg_base;
      rd.n_hosts = s->n_hosts;
      rd.n_devices = s->n_devices;
      rd.times_off = times;
      rd.n_ivl = (int32_t)s->region_ivls[g].size();
      rd.ivl_begin = (int64_t)h_ivls.size();
      for (IvlDesc iv : s->region_ivls[g]) {
        iv.region = (int32_t)h_regions.size();
        h_ivls.push_back(iv);
      }
      times += R;
      h_regions.push_back(rd);
    }
    seg_base += R;
  }
  return assemble_plan(ss[0]->tuning, seg_count, seg_host, k, times, err);
}

// Segments, tiles, buckets and the workspace for the chunks in h_chunks (their
// seg and owner set) and the regions in h_regions.
hpop_status Engine::assemble_plan(const hpop_tuning& tun, const std::vector<long long>& seg_count,
                                  const std::vector<char>& seg_host, int n_owners, long long times, std::string& err) {
  int target, cap, tile, slots;
  tuned(tun, target, cap, tile, slots);
  if (exact_forced) slots = 0;
  const long long n_segs = (long long)seg_count.size();
  if (n_segs > INT_MAX / 2 || h_chunks.size() > (size_t)INT_MAX / 2) {
    err = "too many resources or record batches in one build";
    return HPOP_E_ARG;
  }
  long long buckets = 0, elems = 0;
  h_segs.clear();
  for (long long r = 0; r < n_segs; ++r) {
    SegDesc sd;
    sd.bucket_begin = buckets;
    const long long want = (seg_count[r] + target - 1) / target;
    sd.nb = (int32_t)std::min(1ll << 24, std::max(1ll, want));
    sd.n_levels = seg_host[r] ? 3 : 2;
    buckets += sd.nb;
    h_segs.push_back(sd);
  }
  // Streaming tiles. A chunk of fewer than half a tile of records would leave
  // its own tile mostly empty (traces of many small record batches), so such
  // chunks share tiles: the chunks with tiles of their own come first in the
  // table, then the small ones, packed in order up to a tile of records and
  // kTileChunks chunks per tile. Shared tiles are numbered after the others,
  // so tile_begin never decreases along the table. Tile sizes without a
  // shared-tile kernel, and builds of 2^31 buckets or more (their kernels
  // index buckets in 32 bits), keep one chunk per tile.
  const bool share = (tile == 512 || tile == 2048) && buckets < INT_MAX;
  const long long small_below = share ? tile / 2 : 0;
  std::stable_partition(h_chunks.begin(), h_chunks.end(),
                        [&](const ChunkDesc& d) { return d.count >= small_below; });
  long long tiles = 0;
  for (auto& d : h_chunks) {
    elems += d.count;
    if (d.count < small_below) continue;
    d.tile_begin = tiles;
    d.tile_pos = -1;
    d.tile_off = 0;
    tiles += (d.count + tile - 1) / tile;
  }
  const long long own_tiles = tiles;
  int pos = 0;
  long long fill = 0;
  for (auto& d : h_chunks) {
    if (d.count >= small_below) continue;
    if (pos > 0 && (fill + d.count > tile || pos == kTileChunks)) {
      ++tiles;  // this tile is full
      pos = 0;
      fill = 0;
    }
    d.tile_begin = tiles;
    d.tile_pos = pos++;
    d.tile_off = (int32_t)fill;
    fill += d.count;
  }
  if (pos > 0) ++tiles;
  // tile -> chunk map of the streaming passes: the last chunk whose first
  // tile is at or before the tile (for a shared tile, its last chunk), so
  // their workgroups start with one load instead of a search
  h_tile_chunk.resize((size_t)tiles);
  for (long long t = 0, c = 0, nc = (long long)h_chunks.size(); t < tiles; ++t) {
    while (c + 1 < nc && h_chunks[(size_t)c + 1].tile_begin <= t) ++c;
    h_tile_chunk[(size_t)t] = (int32_t)c;
  }
  hpop_status st = ws.prepare(alloc, (long long)h_chunks.size(), tiles, n_segs, buckets, elems,
                              slots > 0 ? buckets * (long long)slots : 0, (long long)h_regions.size(), times,
                              std::max(1, n_owners), (long long)h_ivls.size(), err);
  if (st != HPOP_OK) return st;
  ws.plan.n_tiles = tiles;
  ws.plan.n_own_tiles = own_tiles;
  // many segments of a few buckets each (batches of small traces): the
  // per-segment passes take them eight to a wave
  ws.plan.seg_group = n_segs >= 4096 && buckets <= 8 * n_segs ? 8 : 1;
  ws.plan.tile_elems = tile;
  ws.plan.cap = cap;
  ws.plan.slot_cap = slots;
  ws.plan.pad1 = 0;
  n_times = times;
  return HPOP_OK;
}

hpop_status Engine::upload(std::string& err) {
  const size_t bc = h_chunks.size() * sizeof(ChunkDesc), bs = h_segs.size() * sizeof(SegDesc),
               br = h_regions.size() * sizeof(RegionDesc), bi = h_ivls.size() * sizeof(IvlDesc),
               bt = h_tile_chunk.size() * sizeof(int32_t);
  if (ws.fixed) {
    // no page-locked staging (it would be an allocation): copies straight from
    // the host vectors, which stay untouched until the caller synchronises
    if (bc) HPOP_HIP(hipMemcpyAsync(ws.d_chunks, h_chunks.data(), bc, hipMemcpyHostToDevice, alloc.stream), "upload chunks");
    if (bt)
      HPOP_HIP(hipMemcpyAsync(ws.plan.tile_chunk, h_tile_chunk.data(), bt, hipMemcpyHostToDevice, alloc.stream),
               "upload tile map");
    if (bs) HPOP_HIP(hipMemcpyAsync(ws.d_segs, h_segs.data(), bs, hipMemcpyHostToDevice, alloc.stream), "upload segments");
    if (br)
      HPOP_HIP(hipMemcpyAsync(ws.d_regions, h_regions.data(), br, hipMemcpyHostToDevice, alloc.stream),
               "upload regions");
    if (bi)
      HPOP_HIP(hipMemcpyAsync(ws.d_ivls, h_ivls.data(), bi, hipMemcpyHostToDevice, alloc.stream),
               "upload region intervals");
    return HPOP_OK;
  }
  // descriptors go through pinned memory so the copies are stream-ordered;
  // the previous upload from this buffer must have left it (an event, not a
  // wait for everything else queued on the stream)
  if (ws.desc_done) HPOP_HIP(hipEventSynchronize(ws.desc_done), "hipEventSynchronize");
  else HPOP_HIP(hipEventCreateWithFlags(&ws.desc_done, hipEventDisableTiming), "hipEventCreate");
  if (!ws.pinned_desc.reserve(bc + bs + br + bi + bt + 64)) {
    err = "pinned host allocation failed";
    return HPOP_E_OOM;
  }
  char* h = (char*)ws.pinned_desc.ptr;
  if (bc) memcpy(h, h_chunks.data(), bc);
  if (bs) memcpy(h + bc, h_segs.data(), bs);
  if (br) memcpy(h + bc + bs, h_regions.data(), br);
  if (bi) memcpy(h + bc + bs + br, h_ivls.data(), bi);
  if (bt) memcpy(h + bc + bs + br + bi, h_tile_chunk.data(), bt);
  if (bc) HPOP_HIP(hipMemcpyAsync(ws.d_chunks, h, bc, hipMemcpyHostToDevice, alloc.stream), "upload chunks");
  if (bs) HPOP_HIP(hipMemcpyAsync(ws.d_segs, h + bc, bs, hipMemcpyHostToDevice, alloc.stream), "upload segments");
  if (br)
    HPOP_HIP(hipMemcpyAsync(ws.d_regions, h + bc + bs, br, hipMemcpyHostToDevice, alloc.stream), "upload regions");
  if (bi)
    HPOP_HIP(hipMemcpyAsync(ws.d_ivls, h + bc + bs + br, bi, hipMemcpyHostToDevice, alloc.stream),
             "upload region intervals");
  if (bt)
    HPOP_HIP(hipMemcpyAsync(ws.plan.tile_chunk, h + bc + bs + br + bi, bt, hipMemcpyHostToDevice, alloc.stream),
             "upload tile map");
  HPOP_HIP(hipEventRecord(ws.desc_done, alloc.stream), "hipEventRecord");
  return HPOP_OK;
}

// All kernels of a build plus the region kernel and the copy of the results.
hpop_status Engine::enqueue(bool build, bool with_timing, std::string& err) {
  const Plan& p = ws.plan;
  hipStream_t st = alloc.stream;
  const int nreg = (int)h_regions.size();
  if (with_timing && events.empty()) {
    events.resize(12);
    for (auto& e : events) HPOP_HIP(hipEventCreate(&e), "hipEventCreate");
  }
  mark_names.clear();
  int ev = 0;
  // every stage: one event before the first and one after each; one named
  // stage (timing_stage): an event right before it and one right after it
  const bool one = with_timing && !timing_stage.empty();
  auto pre = [&](const char* name) -> hipError_t {
    if (!one || timing_stage != name) return hipSuccess;
    return hipEventRecord(events[ev++], st);
  };
  auto mark = [&](const char* name) -> hipError_t {
    if (!with_timing || (one && (!name || timing_stage != name))) return hipSuccess;
    if (name) mark_names.push_back(name);
    return hipEventRecord(events[ev++], st);
  };
  HPOP_HIP(mark(nullptr), "hipEventRecord");
  if (build) {
    HPOP_HIP(pre("reset"), "hipEventRecord");
    HPOP_HIP(launch_reset(p, st), "k_reset");
    HPOP_HIP(mark("reset"), "hipEventRecord");
    HPOP_HIP(pre("stats"), "hipEventRecord");
    HPOP_HIP(launch_stats(p, st), "k_stats");
    HPOP_HIP(mark("stats"), "hipEventRecord");
    if (p.slot_cap == 0) {  // exact offsets: count, then scan, then scatter, then carry
      HPOP_HIP(pre("hist"), "hipEventRecord");
      HPOP_HIP(launch_hist(p, st), "k_hist");
      HPOP_HIP(mark("hist"), "hipEventRecord");
      HPOP_HIP(pre("scan"), "hipEventRecord");
      HPOP_HIP(launch_scan(p, st), "k_scan");
      HPOP_HIP(mark("scan"), "hipEventRecord");
      HPOP_HIP(pre("scatter"), "hipEventRecord");
      HPOP_HIP(launch_scatter(p, st), "k_scatter");
      HPOP_HIP(mark("scatter"), "hipEventRecord");
      HPOP_HIP(pre("carry"), "hipEventRecord");
      HPOP_HIP(launch_carry(p, st), "k_carry");
      HPOP_HIP(mark("carry"), "hipEventRecord");
    } else {  // fixed slots: scatter in one pass, then offsets of the merged intervals and the carry pass together
      HPOP_HIP(pre("scatter"), "hipEventRecord");
      HPOP_HIP(launch_scatter(p, st), "k_scatter");
      HPOP_HIP(mark("scatter"), "hipEventRecord");
      HPOP_HIP(pre("scan"), "hipEventRecord");
      HPOP_HIP(launch_scan_carry(p, st), "k_scan_carry");
      HPOP_HIP(mark("scan"), "hipEventRecord");
    }
    HPOP_HIP(pre("merge_wave"), "hipEventRecord");
    HPOP_HIP(launch_merge_wave(p, st), "k_merge_wave");
    HPOP_HIP(mark("merge_wave"), "hipEventRecord");
    HPOP_HIP(pre("merge_block"), "hipEventRecord");
    HPOP_HIP(launch_merge_block(p, p.cap, st), "k_merge_block");
    HPOP_HIP(mark("merge_block"), "hipEventRecord");
    HPOP_HIP(pre("base"), "hipEventRecord");
    HPOP_HIP(launch_base(p, st), "k_base");
    HPOP_HIP(mark("base"), "hipEventRecord");
  }
  int max_res = 0;
  for (const RegionDesc& rd : h_regions) max_res = std::max(max_res, rd.n_hosts + rd.n_devices);
  HPOP_HIP(pre("region"), "hipEventRecord");
  HPOP_HIP(launch_region(p, ws.d_regions, nreg, max_res, ws.d_trees, ws.d_times, ws.d_ivls, (long long)h_ivls.size(),
                         ws.d_macc, st),
           "k_region");
  HPOP_HIP(mark("region"), "hipEventRecord");
  n_marks = ev;
  // results: trees, first bad record, oversized buckets, slot overflow
  const size_t bt = (size_t)nreg * sizeof(Tree);
  char* h = result_host ? result_host : (char*)ws.pinned.ptr;
  if (bt) HPOP_HIP(hipMemcpyAsync(h, ws.d_trees, bt, hipMemcpyDeviceToHost, st), "copy trees");
  HPOP_HIP(hipMemcpyAsync(h + bt, p.err, 8, hipMemcpyDeviceToHost, st), "copy error word");
  HPOP_HIP(hipMemcpyAsync(h + bt + 8, p.oversized, 16, hipMemcpyDeviceToHost, st), "copy counters");
  return HPOP_OK;
}

hpop_status Engine::collect_timing(std::string& err) {
  stage_ms.clear();
  for (int i = 1; i < n_marks; ++i) {
    float ms = 0.f;
    HPOP_HIP(hipEventElapsedTime(&ms, events[i - 1], events[i]), "hipEventElapsedTime");
    stage_ms.push_back(std::make_pair(mark_names[i - 1], ms));
  }
  return HPOP_OK;
}

// Build (if needed) and reduce the regions of sessions ss[0..k). Trees land in
// `out` (all regions, session by session).
hpop_status Engine::run(hpop_session* const* ss, int k, uint32_t flags, hpop_metric_tree* out, bool timing,
                        std::string& err) {
  // does the current plan still describe these sessions?
  bool same = (int)key_sessions.size() == k && built;
  if (same) {
    for (int i = 0; i < k; ++i)
      if (key_sessions[i] != ss[i] || key_versions[i] != ss[i]->version || key_arena[i] != ss[i]->arena.ptr ||
          key_regions[i] != ss[i]->regions.size() || key_tuning[i] != tuning_key(ss[i]->tuning))
        same = false;
  }
  const bool build = !same || (flags & HPOP_FORCE_REBUILD);
  if (!same && exact_forced) {
    // new records, another session set or another tuning (slots follow the
    // bucket size): try the single-pass scatter again
    bool changed = (int)forced_versions.size() != k || forced_tuning != tuning_key(ss[0]->tuning);
    for (int i = 0; !changed && i < k; ++i) changed = forced_versions[i] != ss[i]->version;
    if (changed) {
      exact_forced = false;
      forced_versions.clear();
    }
  }
  const size_t nreg_total = [&] {
    size_t t = 0;
    for (int i = 0; i < k; ++i) t += ss[i]->regions.size();
    return t;
  }();
  if (!same) {
    hpop_status st = assemble(ss, k, err);
    if (st != HPOP_OK) {
      built = false;
      return st;
    }
    if (!ws.pinned.reserve(nreg_total * sizeof(Tree) + 64)) {
      err = "pinned host allocation failed";
      return HPOP_E_OOM;
    }
    st = upload(err);
    if (st != HPOP_OK) {
      built = false;
      return st;
    }
    if (ws.graph_exec) {
      (void)hipGraphExecDestroy(ws.graph_exec);
      ws.graph_exec = nullptr;
    }
  } else if (nreg_total != h_regions.size()) {
    built = false;
    return run(ss, k, flags, out, timing, err);
  }
  built = false;
  if (build && use_graphs && !timing && !(flags & HPOP_NO_GRAPH)) {
    // capture the whole launch sequence once per plan and replay it
    if (!ws.graph_exec) {
      // capture starts on an idle stream: the descriptor upload has landed
      HPOP_HIP(hipStreamSynchronize(alloc.stream), "hipStreamSynchronize");
      hipGraph_t g = nullptr;
      HPOP_HIP(hipStreamBeginCapture(alloc.stream, hipStreamCaptureModeThreadLocal), "hipStreamBeginCapture");
      hpop_status st = enqueue(true, false, err);
      hipError_t ce = hipStreamEndCapture(alloc.stream, &g);
      if (st != HPOP_OK) {
        if (g) (void)hipGraphDestroy(g);
        return st;
      }
      if (ce != hipSuccess) return hip_fail(err, "hipStreamEndCapture", ce);
      hipError_t ie = hipGraphInstantiate(&ws.graph_exec, g, nullptr, nullptr, 0);
      (void)hipGraphDestroy(g);
      if (ie != hipSuccess) {
        ws.graph_exec = nullptr;
        return hip_fail(err, "hipGraphInstantiate", ie);
      }
    }
    HPOP_HIP(hipGraphLaunch(ws.graph_exec, alloc.stream), "hipGraphLaunch");
    ++graph_replays;
  } else {
    hpop_status st = enqueue(build, timing, err);
    if (st != HPOP_OK) return st;
  }
  HPOP_HIP(hipStreamSynchronize(alloc.stream), "hipStreamSynchronize");
  if (timing) {
    hpop_status st = collect_timing(err);
    if (st != HPOP_OK) return st;
  }
  const size_t bt = h_regions.size() * sizeof(Tree);
  const char* h = (const char*)ws.pinned.ptr;
  unsigned long long bad, over, slot_over;
  memcpy(&bad, h + bt, 8);
  memcpy(&over, h + bt + 8, 8);
  memcpy(&slot_over, h + bt + 16, 8);
  if (build) last_oversized = (long long)over;
  if (build && bad == ULLONG_MAX && ws.plan.slot_cap > 0 && slot_over > 0) {
    // a bucket outgrew its fixed slots: redo this plan with exact offsets
    exact_forced = true;
    forced_versions.clear();
    for (int i = 0; i < k; ++i) forced_versions.push_back(ss[i]->version);
    forced_tuning = tuning_key(ss[0]->tuning);
    key_sessions.clear();
    return run(ss, k, flags | HPOP_FORCE_REBUILD, out, timing, err);
  }
  if (bad != ULLONG_MAX) {
    const unsigned long long cid = bad >> 40, idx = bad & ((1ull << 40) - 1);
    if (cid < chunk_owner.size()) {
      const int si = chunk_owner[cid].first, ci = chunk_owner[cid].second;
      hpop_session* s = ss[si];
      const RecChunk rc = s->chunks[ci];
      char buf[256];
      snprintf(buf, sizeof buf,
               "invalid record: resource %d kind %d, add_events call %lld, index %llu (need 0 <= start <= end < 2^62); "
               "that call's records were dropped",
               rc.resource, rc.kind, (long long)rc.call, idx);
      err = buf;
      s->last_error = buf;
      s->n_events -= rc.count;
      s->chunks.erase(s->chunks.begin() + ci);
      ++s->version;
    } else {
      err = "invalid record";
    }
    return HPOP_E_BAD_INTERVAL;
  }
  if (out && bt) memcpy(out, h, bt);
  key_sessions.assign(ss, ss + k);
  key_versions.resize(k);
  key_arena.resize(k);
  key_regions.resize(k);
  key_tuning.resize(k);
  for (int i = 0; i < k; ++i) {
    key_versions[i] = ss[i]->version;
    key_arena[i] = ss[i]->arena.ptr;
    key_regions[i] = ss[i]->regions.size();
    key_tuning[i] = tuning_key(ss[i]->tuning);
  }
  built = true;
  return HPOP_OK;
}

void Engine::release() {
  for (auto& e : events) (void)hipEventDestroy(e);
  events.clear();
  ws.release(alloc);
  built = false;
}

long long tuning_key(const hpop_tuning& t) {
  return ((long long)t.bucket_target << 40) ^ ((long long)t.bucket_cap << 24) ^ ((long long)t.tile_elems << 8) ^
         (long long)(t.scatter_slots + 1);
}

}  // namespace hpop

// ----------------------------------------------------------------------------
// C ABI
// ----------------------------------------------------------------------------

#define HPOP_GUARD_BEGIN try {
#define HPOP_GUARD_END(sess)                                   \
  }                                                            \
  catch (const std::bad_alloc&) {                              \
    if (sess) (sess)->last_error = "host allocation failed";   \
    else g_thread_error = "host allocation failed";            \
    return HPOP_E_OOM;                                         \
  }                                                            \
  catch (...) {                                                \
    if (sess) (sess)->last_error = "internal error";           \
    else g_thread_error = "internal error";                    \
    return HPOP_E_STATE;                                       \
  }

static hpop_status fail(hpop_session* s, hpop_status code, const std::string& msg) {
  if (s) s->last_error = msg;
  else g_thread_error = msg;
  return code;
}

extern "C" {

const char* hpop_status_string(hpop_status status) { return status_name(status); }

const char* hpop_last_error(const hpop_session* s) { return s ? s->last_error.c_str() : g_thread_error.c_str(); }

hpop_status hpop_session_create(const hpop_session_config* cfg, hpop_session** out) {
  HPOP_GUARD_BEGIN
  if (!cfg || !out) return fail(nullptr, HPOP_E_ARG, "null argument");
  *out = nullptr;
  if (cfg->n_hosts < 0 || cfg->n_devices < 0 || cfg->n_hosts + (long long)cfg->n_devices > (1 << 24))
    return fail(nullptr, HPOP_E_ARG, "n_hosts and n_devices must be >= 0 with n + m <= 2^24");
  if ((cfg->alloc == nullptr) != (cfg->free == nullptr))
    return fail(nullptr, HPOP_E_ARG, "alloc and free callbacks must be given together");
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return fail(nullptr, HPOP_E_HIP, std::string("hipGetDevice: ") + hipGetErrorString(e));
  hpop_session* s = new hpop_session();
  s->n_hosts = cfg->n_hosts;
  s->n_devices = cfg->n_devices;
  s->device = dev;
  if (cfg->stream) {
    s->stream = (hipStream_t)cfg->stream;
    s->own_stream = false;
  } else {
    e = hipStreamCreateWithFlags(&s->stream, hipStreamNonBlocking);
    if (e != hipSuccess) {
      delete s;
      return fail(nullptr, HPOP_E_HIP, std::string("hipStreamCreate: ") + hipGetErrorString(e));
    }
    s->own_stream = true;
  }
  s->alloc.stream = s->stream;
  s->alloc.fn_alloc = cfg->alloc;
  s->alloc.fn_free = cfg->free;
  s->alloc.ctx = cfg->alloc_ctx;
  s->engine.alloc = s->alloc;
  s->batch_engine.alloc = s->alloc;
  *out = s;
  return HPOP_OK;
  HPOP_GUARD_END((hpop_session*)nullptr)
}

hpop_status hpop_session_destroy(hpop_session* s) {
  HPOP_GUARD_BEGIN
  if (!s) return fail(nullptr, HPOP_E_ARG, "null session");
  (void)hipStreamSynchronize(s->stream);
  if (s->streams) hpop_session_destroy(s->streams);
  s->stream_buf.release(s->alloc);
  s->engine.release();
  s->batch_engine.release();
  s->arena.release(s->alloc);
  s->staging.release();
  (void)hipStreamSynchronize(s->stream);
  if (s->own_stream) (void)hipStreamDestroy(s->stream);
  delete s;
  return HPOP_OK;
  HPOP_GUARD_END((hpop_session*)nullptr)
}

static hpop_status check_kind(hpop_session* s, int32_t resource, int32_t kind) {
  if (resource < 0 || resource >= s->n_hosts + s->n_devices)
    return fail(s, HPOP_E_RESOURCE, "resource " + std::to_string(resource) + " out of range");
  const int slot = slot_of_kind(kind);
  if (slot < 0) return fail(s, HPOP_E_KIND, "unknown kind " + std::to_string(kind));
  const bool host_kind = kind <= HPOP_HOST_MPI;
  if (host_kind != (resource < s->n_hosts))
    return fail(s, HPOP_E_KIND, std::string(host_kind ? "host" : "device") + " kind on a " +
                                    (resource < s->n_hosts ? "host" : "device") + " resource");
  return HPOP_OK;
}

hpop_status hpop_add_events(hpop_session* s, int32_t resource, int32_t kind, const int64_t* start,
                            const int64_t* end, int64_t count, int32_t mem_space) {
  hpop_event_chunk c;
  c.resource = resource;
  c.kind = kind;
  c.start = start;
  c.end = end;
  c.count = count;
  return hpop_add_events_multi(s, &c, 1, mem_space);
}

hpop_status hpop_add_events_multi(hpop_session* s, const hpop_event_chunk* chunks, int32_t n_chunks,
                                  int32_t mem_space) {
  HPOP_GUARD_BEGIN
  if (!s) return fail(nullptr, HPOP_E_ARG, "null session");
  if (n_chunks < 0 || (n_chunks > 0 && !chunks)) return fail(s, HPOP_E_ARG, "bad chunk list");
  if (mem_space != HPOP_MEM_HOST && mem_space != HPOP_MEM_DEVICE) return fail(s, HPOP_E_ARG, "bad mem_space");
  size_t need = 0;
  for (int32_t i = 0; i < n_chunks; ++i) {
    const hpop_event_chunk& c = chunks[i];
    hpop_status st = check_kind(s, c.resource, c.kind);
    if (st != HPOP_OK) return st;
    if (c.count < 0 || (c.count > 0 && (!c.start || !c.end))) return fail(s, HPOP_E_ARG, "bad count or null array");
    if (c.count > (1ll << 40)) return fail(s, HPOP_E_ARG, "too many records in one call");
    need += 2 * ((size_t(c.count) * 8 + 255) & ~size_t(255));
  }
  if (mem_space == HPOP_MEM_HOST) {
    // validate eagerly (Section 4.1 states need 0 <= start <= end)
    for (int32_t i = 0; i < n_chunks; ++i) {
      const hpop_event_chunk& c = chunks[i];
      for (int64_t j = 0; j < c.count; ++j) {
        const int64_t a = c.start[j], b = c.end[j];
        if (a < 0 || a > b || b >= kTimeLimit)
          return fail(s, HPOP_E_BAD_INTERVAL, "chunk " + std::to_string(i) + " record " + std::to_string(j) +
                                                   ": need 0 <= start <= end < 2^62");
      }
    }
  }
  if (need == 0) return HPOP_OK;
  s->arena.used = s->arena_used;
  if (!s->arena.reserve(s->alloc, s->arena_used + need, true))
    return fail(s, HPOP_E_OOM, "device allocation for " + std::to_string(need) + " bytes of records failed");
  s->copies_pending = true;  // the arena's growth and the records' copies go on the session stream
  char* base = (char*)s->arena.ptr;
  size_t off = s->arena_used;
  std::vector<RecChunk> added;
  if (mem_space == HPOP_MEM_HOST) {
    if (!s->staging.reserve(need)) return fail(s, HPOP_E_OOM, "pinned staging allocation failed");
    // the staging buffer's previous copy must have left it
    hipError_t e = hipStreamSynchronize(s->stream);
    if (e != hipSuccess) return fail(s, HPOP_E_HIP, std::string("hipStreamSynchronize: ") + hipGetErrorString(e));
    char* h = (char*)s->staging.ptr;
    size_t o = 0;
    for (int32_t i = 0; i < n_chunks; ++i) {
      const hpop_event_chunk& c = chunks[i];
      if (c.count == 0) continue;
      const size_t b = size_t(c.count) * 8, bp = (b + 255) & ~size_t(255);
      memcpy(h + o, c.start, b);
      memcpy(h + o + bp, c.end, b);
      RecChunk rc;
      rc.resource = c.resource;
      rc.kind = c.kind;
      rc.count = c.count;
      rc.off_s = off + o;
      rc.off_e = off + o + bp;
      rc.call = s->n_calls + i;
      added.push_back(rc);
      o += 2 * bp;
    }
    e = hipMemcpyAsync(base + off, h, o, hipMemcpyHostToDevice, s->stream);
    if (e != hipSuccess) return fail(s, HPOP_E_HIP, std::string("hipMemcpyAsync: ") + hipGetErrorString(e));
    off += o;
  } else {
    for (int32_t i = 0; i < n_chunks; ++i) {
      const hpop_event_chunk& c = chunks[i];
      if (c.count == 0) continue;
      const size_t b = size_t(c.count) * 8, bp = (b + 255) & ~size_t(255);
      hipError_t e = hipMemcpyAsync(base + off, c.start, b, hipMemcpyDeviceToDevice, s->stream);
      if (e == hipSuccess) e = hipMemcpyAsync(base + off + bp, c.end, b, hipMemcpyDeviceToDevice, s->stream);
      if (e != hipSuccess) return fail(s, HPOP_E_HIP, std::string("hipMemcpyAsync: ") + hipGetErrorString(e));
      RecChunk rc;
      rc.resource = c.resource;
      rc.kind = c.kind;
      rc.count = c.count;
      rc.off_s = off;
      rc.off_e = off + bp;
      rc.call = s->n_calls + i;
      added.push_back(rc);
      off += 2 * bp;
    }
  }
  s->arena_used = off;
  s->arena.used = off;
  for (auto& rc : added) {
    s->chunks.push_back(rc);
    s->n_events += rc.count;
  }
  s->n_calls += n_chunks;
  ++s->version;
  return HPOP_OK;
  HPOP_GUARD_END(s)
}

hpop_status hpop_session_synchronize(hpop_session* s) {
  if (!s) return fail(nullptr, HPOP_E_ARG, "null session");
  hipError_t e = hipStreamSynchronize(s->stream);
  if (e != hipSuccess) return fail(s, HPOP_E_HIP, std::string("hipStreamSynchronize: ") + hipGetErrorString(e));
  s->copies_pending = false;
  return HPOP_OK;
}

hpop_status hpop_clear_events(hpop_session* s) {
  HPOP_GUARD_BEGIN
  if (!s) return fail(nullptr, HPOP_E_ARG, "null session");
  if (s->streams) hpop_clear_events(s->streams);
  s->chunks.clear();
  s->arena_used = 0;
  s->arena.used = 0;
  s->n_events = 0;
  ++s->version;
  return HPOP_OK;
  HPOP_GUARD_END(s)
}

hpop_status hpop_region_define(hpop_session* s, int64_t t0, int64_t t1, int32_t* out_region) {
  HPOP_GUARD_BEGIN
  if (!s || !out_region) return fail(s, HPOP_E_ARG, "null argument");
  if (!(t0 < t1)) return fail(s, HPOP_E_REGION, "region needs t0 < t1");
  if (t0 < -kTimeLimit || t1 > kTimeLimit) return fail(s, HPOP_E_REGION, "region bounds out of range");
  const unsigned long long E = (unsigned long long)(t1 - t0);
  const unsigned long long w = (unsigned long long)std::max(1, std::max(s->n_hosts, s->n_devices));
  if (E >= (1ull << 53) || E * w >= (1ull << 53))
    return fail(s, HPOP_E_OVERFLOW, "(t1 - t0) * max(n, m) must be below 2^53 for exact FP64 ratios");
  s->regions.push_back(std::make_pair(t0, t1));
  s->region_ivls.emplace_back();
  *out_region = (int32_t)s->regions.size() - 1;
  return HPOP_OK;
  HPOP_GUARD_END(s)
}

hpop_status hpop_region_define_multi(hpop_session* s, const int32_t* resource, const int64_t* t0,
                                     const int64_t* t1, int64_t count, int32_t* out_region) {
  HPOP_GUARD_BEGIN
  if (!s || !resource || !t0 || !t1 || !out_region || count < 1) return fail(s, HPOP_E_ARG, "bad arguments");
  const int R = s->n_hosts + s->n_devices;
  std::vector<IvlDesc> iv((size_t)count);
  for (int64_t i = 0; i < count; ++i) {
    if (resource[i] < 0 || resource[i] >= R) return fail(s, HPOP_E_RESOURCE, "interval " + std::to_string(i));
    if (!(t0[i] < t1[i]) || t0[i] < -kTimeLimit || t1[i] > kTimeLimit)
      return fail(s, HPOP_E_REGION, "interval " + std::to_string(i) + " needs t0 < t1 within [-2^62, 2^62]");
    iv[i].region = 0;
    iv[i].resource = resource[i];
    iv[i].a = t0[i];
    iv[i].b = t1[i];
  }
  std::sort(iv.begin(), iv.end(), [](const IvlDesc& x, const IvlDesc& y) {
    return x.resource != y.resource ? x.resource < y.resource : x.a < y.a;
  });
  // no overlap within a resource; E as eq. 1: the largest host total (device total without hosts)
  std::vector<unsigned long long> tot((size_t)R, 0);
  for (size_t i = 0; i < iv.size(); ++i) {
    if (i > 0 && iv[i].resource == iv[i - 1].resource && iv[i].a < iv[i - 1].b)
      return fail(s, HPOP_E_REGION, "overlapping intervals on resource " + std::to_string(iv[i].resource));
    tot[iv[i].resource] += (unsigned long long)(iv[i].b - iv[i].a);
  }
  unsigned long long eh = 0, ed = 0;
  for (int r = 0; r < R; ++r) (r < s->n_hosts ? eh : ed) = std::max(r < s->n_hosts ? eh : ed, tot[r]);
  const unsigned long long E = eh ? eh : ed;
  unsigned long long maxdur = 0;
  for (unsigned long long t : tot) maxdur = std::max(maxdur, t);
  const unsigned long long w = (unsigned long long)std::max(1, std::max(s->n_hosts, s->n_devices));
  (void)E;
  if (maxdur >= (1ull << 53) / w)
    return fail(s, HPOP_E_OVERFLOW, "E * max(n, m) must be below 2^53 for exact FP64 ratios");
  int64_t lo = iv[0].a, hi = iv[0].b;
  for (const IvlDesc& x : iv) {
    lo = std::min(lo, x.a);
    hi = std::max(hi, x.b);
  }
  s->regions.push_back(std::make_pair(lo, hi));
  s->region_ivls.push_back(std::move(iv));
  *out_region = (int32_t)s->regions.size() - 1;
  return HPOP_OK;
  HPOP_GUARD_END(s)
}

hpop_status hpop_num_regions(const hpop_session* s, int32_t* out) {
  if (!s || !out) return HPOP_E_ARG;
  *out = (int32_t)s->regions.size();
  return HPOP_OK;
}

hpop_status hpop_metrics_compute_all(hpop_session* s, uint32_t flags, hpop_metric_tree* out) {
  HPOP_GUARD_BEGIN
  if (!s) return fail(nullptr, HPOP_E_ARG, "null session");
  if (flags & ~(HPOP_FORCE_REBUILD | HPOP_NO_GRAPH)) return fail(s, HPOP_E_ARG, "unknown flags");
  if (!s->regions.empty() && !out) return fail(s, HPOP_E_ARG, "null output");
  std::string err;
  hpop_session* one[1] = {s};
  s->last_timed_batch = false;
  hpop_status st = s->engine.run(one, 1, flags, out, s->timing, err);
  if (st != HPOP_OK) return fail(s, st, err);
  return HPOP_OK;
  HPOP_GUARD_END(s)
}

hpop_status hpop_metrics_compute(hpop_session* s, int32_t region, hpop_metric_tree* out) {
  HPOP_GUARD_BEGIN
  if (!s || !out) return fail(s, HPOP_E_ARG, "null argument");
  if (region < 0 || region >= (int32_t)s->regions.size())
    return fail(s, HPOP_E_REGION, "unknown region " + std::to_string(region));
  std::vector<hpop_metric_tree> all(s->regions.size());
  hpop_status st = hpop_metrics_compute_all(s, 0, all.data());
  if (st != HPOP_OK) return st;
  *out = all[region];
  return HPOP_OK;
  HPOP_GUARD_END(s)
}

hpop_status hpop_resource_times(hpop_session* s, int32_t region, int32_t resource, int64_t out[4]) {
  HPOP_GUARD_BEGIN
  if (!s || !out) return fail(s, HPOP_E_ARG, "null argument");
  if (region < 0 || region >= (int32_t)s->regions.size()) return fail(s, HPOP_E_REGION, "unknown region");
  if (resource < 0 || resource >= s->n_hosts + s->n_devices) return fail(s, HPOP_E_RESOURCE, "bad resource");
  if (!s->engine.built || s->engine.key_versions.empty() || s->engine.key_versions[0] != s->version ||
      s->engine.key_regions[0] != s->regions.size())
    return fail(s, HPOP_E_STATE, "call hpop_metrics_compute_all after the last change first");
  const long long row = s->engine.h_regions[region].times_off + resource;
  hipError_t e = hipMemcpy(out, s->engine.ws.d_times + row * 4, 32, hipMemcpyDeviceToHost);
  if (e != hipSuccess) return fail(s, HPOP_E_HIP, std::string("hipMemcpy: ") + hipGetErrorString(e));
  return HPOP_OK;
  HPOP_GUARD_END(s)
}

hpop_status hpop_region_format(hpop_session* s, int32_t region, int32_t format, char* buf, int64_t cap,
                               int64_t* needed) {
  HPOP_GUARD_BEGIN
  if (!s) return fail(s, HPOP_E_ARG, "null session");
  if ((format != HPOP_FORMAT_TEXT && format != HPOP_FORMAT_JSON) || cap < 0 || (cap > 0 && !buf))
    return fail(s, HPOP_E_ARG, "bad format or buffer");
  hpop_metric_tree tree;
  hpop_status st = hpop_metrics_compute(s, region, &tree);
  if (st != HPOP_OK) return st;
  // the region's state times are one contiguous row block (4 int64 per resource)
  const int R = s->n_hosts + s->n_devices;
  std::vector<int64_t> times(4 * (size_t)R + 1);
  if (R > 0) {
    const long long row = s->engine.h_regions[region].times_off;
    hipError_t e = hipMemcpy(times.data(), s->engine.ws.d_times + row * 4, 32 * (size_t)R, hipMemcpyDeviceToHost);
    if (e != hipSuccess) return fail(s, HPOP_E_HIP, std::string("hipMemcpy: ") + hipGetErrorString(e));
  }
  return hpop::emit_string(hpop::render_region(tree, format, s->n_hosts, s->n_devices, times.data()), buf, cap,
                           needed);
  HPOP_GUARD_END(s)
}

hpop_status hpop_batch_compute(hpop_session* const* sessions, int32_t k, uint32_t flags, hpop_metric_tree* out) {
  HPOP_GUARD_BEGIN
  if (!sessions || k <= 0) return fail(nullptr, HPOP_E_ARG, "empty session list");
  if (flags & ~(HPOP_FORCE_REBUILD | HPOP_NO_GRAPH)) return fail(nullptr, HPOP_E_ARG, "unknown flags");
  for (int i = 0; i < k; ++i) {
    if (!sessions[i]) return fail(nullptr, HPOP_E_ARG, "null session in list");
    if (sessions[i]->device != sessions[0]->device) return fail(nullptr, HPOP_E_ARG, "sessions on different devices");
  }
  hpop_session* s0 = sessions[0];
  // records of the other sessions were copied on their own streams: wait for
  // those with copies since their last wait (a wait on each idle stream of a
  // thousand sessions would cost more than the build)
  for (int i = 1; i < k; ++i)
    if (sessions[i]->copies_pending && sessions[i]->stream != s0->stream) {
      hipError_t e = hipStreamSynchronize(sessions[i]->stream);
      if (e != hipSuccess) return fail(nullptr, HPOP_E_HIP, std::string("hipStreamSynchronize: ") + hipGetErrorString(e));
      sessions[i]->copies_pending = false;
    }
  std::string err;
  s0->last_timed_batch = true;
  hpop_status st = s0->batch_engine.run(sessions, k, flags, out, s0->timing, err);
  if (st != HPOP_OK) return fail(nullptr, st, err);
  return HPOP_OK;
  HPOP_GUARD_END((hpop_session*)nullptr)
}

hpop_status hpop_session_get_info(const hpop_session* s, hpop_session_info* out) {
  if (!s || !out) return HPOP_E_ARG;
  out->n_events = s->n_events;
  out->n_chunks = (int64_t)s->chunks.size();
  out->n_buckets = s->engine.ws.plan.n_buckets;
  out->n_oversized = s->engine.last_oversized;
  out->n_components = 0;
  out->n_wide_components = 0;
  out->n_wide_records = 0;
  const Engine& En = s->engine;
  if (En.built && En.ws.plan.n_buckets > 0) {
    // read back the per-bucket component counts and the segment ranges
    // (diagnostics, not on the hot path)
    const long long nb = En.ws.plan.n_buckets;
    const size_t ns = En.h_segs.size();
    std::vector<unsigned int> nc((size_t)(3 * nb));
    std::vector<SegGeom> geo(ns);
    std::vector<unsigned long long> cur((size_t)nb);
    if (hipStreamSynchronize(s->stream) == hipSuccess &&
        hipMemcpy(cur.data(), En.ws.plan.cursor, cur.size() * 8, hipMemcpyDeviceToHost) == hipSuccess &&
        hipMemcpy(nc.data(), En.ws.plan.ncomp, nc.size() * 4, hipMemcpyDeviceToHost) == hipSuccess &&
        (ns == 0 || hipMemcpy(geo.data(), En.ws.plan.geom, ns * sizeof(SegGeom), hipMemcpyDeviceToHost) == hipSuccess)) {
      long long t = 0, w = 0;
      for (unsigned int v : nc) t += v;
      for (size_t g = 0; g < ns; ++g) {
        // buckets wider than 2^kNarrowShift ns keep their components in the 16 B form
        if (geo[g].empty || ((unsigned long long)geo[g].wx << geo[g].s0) <= (1ull << kNarrowShift)) continue;
        const long long b0 = En.h_segs[g].bucket_begin, b1 = b0 + En.h_segs[g].nb;
        for (long long b = b0; b < b1; ++b) w += (long long)nc[3 * b] + nc[3 * b + 1] + nc[3 * b + 2];
      }
      out->n_components = t;
      out->n_wide_components = w;
      for (unsigned long long c : cur) out->n_wide_records += (long long)(c >> 32);
    }
  }
  out->n_regions = (int32_t)s->regions.size();
  out->graph_replays = s->engine.graph_replays + s->batch_engine.graph_replays;
  return HPOP_OK;
}

hpop_status hpop_session_set_tuning(hpop_session* s, const hpop_tuning* t) {
  if (!s || !t) return HPOP_E_ARG;
  if (t->bucket_target < 0 || t->bucket_cap < 0 || t->tile_elems < 0 || t->scatter_slots < -1)
    return fail(s, HPOP_E_ARG, "negative tuning");
  s->tuning = *t;
  return HPOP_OK;
}

hpop_status hpop_session_get_tuning(const hpop_session* s, hpop_tuning* out) {
  if (!s || !out) return HPOP_E_ARG;
  int target, cap, tile, slots;
  tuned(s->tuning, target, cap, tile, slots);
  out->bucket_target = target;
  out->bucket_cap = cap;
  out->tile_elems = tile;
  out->scatter_slots = slots > 0 ? slots : -1;
  return HPOP_OK;
}

hpop_status hpop_session_enable_timing(hpop_session* s, int32_t on) {
  if (!s) return HPOP_E_ARG;
  s->timing = on != 0;
  return HPOP_OK;
}

hpop_status hpop_session_time_stage(hpop_session* s, const char* stage) {
  if (!s) return HPOP_E_ARG;
  static const char* const known[] = {"reset", "stats", "hist", "scan", "scatter", "carry",
                                      "merge_wave", "merge_block", "base", "region"};
  std::string name = stage ? stage : "";
  if (!name.empty() && std::find(std::begin(known), std::end(known), name) == std::end(known))
    return fail(s, HPOP_E_ARG, "unknown stage name: " + name);
  s->timing_stage = name;
  s->engine.timing_stage = name;
  s->batch_engine.timing_stage = name;
  return HPOP_OK;
}

hpop_status hpop_session_stage_times(const hpop_session* s, int32_t cap, const char** names, float* ms,
                                     int32_t* n_out) {
  if (!s || !n_out || cap < 0) return HPOP_E_ARG;
  const Engine& en = s->last_timed_batch ? s->batch_engine : s->engine;
  int n = std::min<int>(cap, (int)en.stage_ms.size());
  for (int i = 0; i < n; ++i) {
    if (names) names[i] = en.stage_ms[i].first.c_str();
    if (ms) ms[i] = en.stage_ms[i].second;
  }
  *n_out = n;
  return HPOP_OK;
}

}  // extern "C"
