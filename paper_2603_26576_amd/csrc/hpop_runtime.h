// Host-side structures of the runtime (sessions, device buffers, build plans).
#pragma once
#include <hip/hip_runtime.h>

#include <string>
#include <utility>
#include <vector>

#include "hpop.h"
#include "hpop_internal.h"

namespace hpop {

extern thread_local std::string g_thread_error;
// microseconds this thread has spent in device and page-locked allocations (statistics)
extern thread_local double g_alloc_us;
const char* status_name(hpop_status s);
int slot_of_kind(int kind);
long long tuning_key(const hpop_tuning& t);

// Renderings (hpop_format.hip): a region's report with per-resource times
// (4 int64 per resource, hosts then devices), and the buffer rule of the
// formatting calls.
std::string render_region(const hpop_metric_tree& t, int32_t format, int n, int m, const int64_t* times);
hpop_status emit_string(const std::string& s, char* buf, int64_t cap, int64_t* needed);

// Stream-ordered device allocator: the caller's callbacks or hipMallocAsync.
struct Alloc {
  hipStream_t stream = nullptr;
  hpop_alloc_fn fn_alloc = nullptr;
  hpop_free_fn fn_free = nullptr;
  void* ctx = nullptr;
  void* get(size_t bytes);
  void put(void* p);
};

// Grow-only device buffer; `used` bytes are preserved on growth when asked.
struct DevBuf {
  void* ptr = nullptr;
  size_t bytes = 0;
  size_t used = 0;
  bool reserve(Alloc& a, size_t need, bool keep);
  void release(Alloc& a);
};

struct PinnedBuf {
  void* ptr = nullptr;
  size_t bytes = 0;
  bool reserve(size_t need);
  void release();
};

// One add_events call kept in the session's record arena.
struct RecChunk {
  int32_t resource = 0;
  int32_t kind = 0;
  int64_t count = 0;
  size_t off_s = 0;  // byte offsets of the start and end arrays in the arena
  size_t off_e = 0;
  int64_t call = 0;  // index of the add_events call (error reports)
};

// Device buffers of one build plan.
struct Workspace {
  DevBuf meta, elems, elems2, comp[3], compn[3];
  PinnedBuf pinned;       // trees and status words copied back
  PinnedBuf pinned_desc;  // descriptor uploads
  hipEvent_t desc_done = nullptr;  // recorded after the last upload from pinned_desc
  Plan plan{};
  ChunkDesc* d_chunks = nullptr;
  SegDesc* d_segs = nullptr;
  RegionDesc* d_regions = nullptr;
  Tree* d_trees = nullptr;
  long long* d_times = nullptr;
  IvlDesc* d_ivls = nullptr;     // intervals of regions given per resource
  long long* d_macc = nullptr;   // [n_times][4] their per-resource accumulators
  hipGraphExec_t graph_exec = nullptr;
  long long layout_gen = 0;
  // set: everything is carved from this one device region of fixed_bytes
  // (no allocation, no page-locked staging); fixed_needed is the last plan's size
  char* fixed = nullptr;
  size_t fixed_bytes = 0;
  size_t fixed_needed = 0;
  hpop_status prepare(Alloc& a, long long n_chunks, long long n_tiles, long long n_segs, long long n_buckets,
                      long long n_elems,
                      long long n_slots, long long n_regions, long long n_times, long long n_owners,
                      long long n_ivls, std::string& err);
  void release(Alloc& a);
};

// Builds and reduces the records of one or more sessions.
struct Engine {
  Alloc alloc;
  Workspace ws;
  std::vector<ChunkDesc> h_chunks;
  std::vector<int32_t> h_tile_chunk;  // [n_tiles] chunk of each streaming tile (see Plan::tile_chunk)
  std::vector<SegDesc> h_segs;
  std::vector<RegionDesc> h_regions;
  std::vector<IvlDesc> h_ivls;
  std::vector<std::pair<int, int>> chunk_owner;  // (session index, chunk index) per chunk desc
  std::vector<int> seg_of_session, reg_of_session;
  long long n_times = 0;
  // what the current plan was built from
  bool built = false;
  std::vector<hpop_session*> key_sessions;
  std::vector<unsigned long long> key_versions;
  std::vector<void*> key_arena;
  std::vector<size_t> key_regions;
  std::vector<long long> key_tuning;
  bool use_graphs = true;
  int graph_replays = 0;
  long long last_oversized = 0;
  char* result_host = nullptr;  // set: enqueue copies the results here instead of the page-locked buffer
  // timing
  bool exact_forced = false;  // a bucket outgrew its scatter slots: use exact offsets
  std::vector<unsigned long long> forced_versions;
  long long forced_tuning = 0;  // tuning_key of the plan whose slots overflowed
  std::vector<hipEvent_t> events;
  std::vector<const char*> mark_names;
  int n_marks = 0;
  std::vector<std::pair<std::string, float>> stage_ms;

  hpop_status assemble(hpop_session* const* ss, int k, std::string& err);
  hpop_status assemble_plan(const hpop_tuning& tun, const std::vector<long long>& seg_count,
                            const std::vector<char>& seg_host, int n_owners, long long times, std::string& err);
  hpop_status upload(std::string& err);
  std::string timing_stage;  // non-empty: time only this stage (see hpop_session_time_stage)
  hpop_status enqueue(bool build, bool with_timing, std::string& err);
  hpop_status collect_timing(std::string& err);
  hpop_status run(hpop_session* const* ss, int k, uint32_t flags, hpop_metric_tree* out, bool timing,
                  std::string& err);
  void release();
};

}  // namespace hpop

struct hpop_session {
  int32_t n_hosts = 0;
  int32_t n_devices = 0;
  int device = 0;
  hipStream_t stream = nullptr;
  bool own_stream = false;
  hpop::Alloc alloc;
  std::vector<hpop::RecChunk> chunks;
  hpop::DevBuf arena;
  size_t arena_used = 0;
  int64_t n_events = 0;
  int64_t n_calls = 0;
  std::vector<std::pair<int64_t, int64_t>> regions;  // [t0, t1), or the span of a per-resource region
  std::vector<std::vector<hpop::IvlDesc>> region_ivls;  // per region: its intervals (empty: [t0, t1))
  unsigned long long version = 0;
  bool copies_pending = false;  // record copies enqueued on `stream` since a batch last waited for it
  hpop::PinnedBuf staging;
  hpop_tuning tuning{};
  bool timing = false;
  std::string timing_stage;
  bool last_timed_batch = false;
  hpop::Engine engine;
  hpop::Engine batch_engine;
  std::string last_error;
  // stream concurrency (hpop_session_set_streams): an inner session whose
  // resources are, per device g, one holding all its stream records followed
  // by one per stream (resource stream_off[g] + 1 + stream)
  hpop_session* streams = nullptr;
  std::vector<int32_t> stream_n, stream_off;
  hpop::DevBuf stream_buf;
};
