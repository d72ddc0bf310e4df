// Internal layout shared by the runtime and the kernels of the engine.
//
// The build turns the records of every resource (a "segment") into, per
// nested state level, a list of disjoint merged intervals with prefix
// measures, stored per time bucket:
//
//   level 0: device {Kernel}            host {Useful}
//   level 1: device {Kernel, Memory}    host {Useful, Offloading}
//   level 2: -                          host {Useful, Offloading, MPI}
//
// Kernel time of a device in a region is the measure of level 0 inside it,
// memory time the measure of level 1 minus that, idle the rest; host states
// follow the same nesting (Section 4.2 post-processing and the host-state
// priority Useful > Offloading > MPI).
//
// Pipeline (one pass over the records per arrow):
//   records --stats--> per-segment min / max start
//           --scatter-> validated records regrouped by bucket (16 B each, bucket
//                       = (start - min) >> shift) + per-bucket max end; by default
//                       into fixed slots per bucket, else after an exact
//                       --hist--> count and --scan--> offset pass
//           --scan---> bucket offsets of the merged intervals
//   carry  : per-bucket running max end of all earlier buckets (per level)
//   merge  : per bucket, sort by start in LDS, then a block-wide max-scan of
//            ends with the carry finds merge breaks; each break starts a
//            component written as (start, prefix measure within bucket)
//   base   : per-bucket prefix of the buckets' measures
//   region : M(t) = measure of the level before t, by binary search; a
//            region's state time is M(t1) - M(t0); per-region reductions and
//            the FP64 ratios.
#pragma once
#include <stdint.h>

namespace hpop {

constexpr int kLevels = 3;
constexpr int64_t kTimeLimit = int64_t(1) << 62;
constexpr int kSlotShift = 62;  // element end word: end | slot << 62

struct ChunkDesc {
  const int64_t* s;
  const int64_t* e;
  int64_t count;
  int64_t tile_begin;  // first tile of this chunk in the streaming passes
  int32_t seg;         // global segment (resource) index
  int32_t slot;        // level rank of the kind: 0, 1 or 2
  int32_t chunk_id;    // index in the chunk table (error reports)
  int32_t owner;       // session (or serving query) the records belong to
  int32_t tile_pos;    // -1: the chunk has tiles of its own; else its place among a shared tile's chunks
  int32_t tile_off;    // in a shared tile: the tile's record index of the chunk's first record
};

// Chunks smaller than half a tile share tiles: consecutive ones (in the
// chunk table) fill a tile with at most this many chunks and tile_elems records.
constexpr int kTileChunks = 32;

struct SegDesc {
  int64_t bucket_begin;  // first global bucket of the segment
  int32_t nb;            // the segment has nb buckets (any count: records / target)
  int32_t n_levels;      // 2 for devices, 3 for hosts
};

// Time buckets of one segment, fixed per build from its start range: bucket b
// holds the records starting in [lo_b, lo_b + W) with lo_b = min_s + b * W and
// W = wx * 2^s0 ns, s0 chosen so that (max_s - min_s) >> s0 < 2^31 and
// wx = ((max_s - min_s) >> s0) / nb + 1, so nb buckets of equal width cover
// the range. The bucket of x = (start - min_s) >> s0 is x / wx, computed as
// the high half of x * minv (minv = floor(2^32 / wx)) plus one correction.
struct SegGeom {
  int64_t min_s;
  uint32_t wx;
  uint32_t minv;  // floor(2^32 / wx) for wx >= 2, else 0
  int32_t s0;
  int32_t nb;
  int32_t empty;  // no valid record with a start
  int32_t pad;
};

struct SegStats {
  unsigned long long min_s;  // over valid non-empty records; ULLONG_MAX if none
  unsigned long long max_s;
  unsigned long long max_e;
  unsigned long long pad;
};

struct RegionDesc {
  int64_t t0, t1;
  int32_t seg_begin;   // first segment of the region's session (hosts first, then devices)
  int32_t n_hosts;
  int32_t n_devices;
  int32_t n_ivl;       // > 0: a region given as per-resource intervals (IvlDesc), not [t0, t1)
  int64_t times_off;   // offset (in resources) of the region's rows in the times array
  int64_t ivl_begin;   // first IvlDesc of the region
};

// One interval of a region given per resource.
struct IvlDesc {
  int32_t region;
  int32_t resource;  // within the region's session
  int64_t a, b;
};

struct Tree {  // identical layout to hpop_metric_tree
  int64_t E;
  int32_t n, m;
  int64_t sum[10];
  double ratio[9];
  uint32_t undefined_mask;
  uint32_t reserved;
};

struct Comp {  // one merged component inside a bucket
  int64_t cs;  // start
  int64_t pl;  // measure of the level before cs, counted from the bucket's start (with carry)
};

// A component of a segment whose buckets are at most 2^kNarrowShift ns wide:
// its start and its measure before it are both below the bucket width, so
// both fit 32 bits relative to the bucket's first time (8 B instead of 16).
struct CompN {
  uint32_t cs;  // start - first time of the bucket
  uint32_t pl;  // as Comp::pl
};
constexpr int kNarrowShift = 30;

struct Elem {  // one record regrouped by bucket (the 16 B form)
  int64_t s;
  int64_t e_slot;  // end | slot << 62
};

// Records regrouped by bucket. A bucket owns a region of 2 x capacity 8 B
// units (capacity = slot_cap with fixed slots, else its record count) at
// unit 2 x (gb x slot_cap, or offsets[gb]). A record of a narrow segment
// takes one unit from the front, in the 8 B form
//   x = (start - lo) << 2 | slot,  y = min(end - lo + 1, 0xFFFFFFFF)
// where lo is the bucket's first time (a clamped end stands for the largest
// end of the bucket's records of that slot, maxend); a record of a wide
// segment takes two units from the back in the 16 B form. cursor[gb] counts
// both: 8 B records in the low 32 bits, 16 B records in the high 32.
// Device pointers of one build plan.
struct Plan {
  const ChunkDesc* chunks;
  int32_t n_chunks;
  int32_t n_segs;
  int64_t n_tiles;                   // tiles of single chunks [0, n_own_tiles), then shared tiles
  int64_t n_own_tiles;
  int32_t* tile_chunk;               // [n_tiles] chunk of each streaming tile, the last one of a shared
                                     // tile (computed with the plan on the host, uploaded with the chunks)
  int32_t tile_elems;
  int32_t cap;                       // records a bucket may hold for the LDS sort
  int32_t slot_cap;                  // >0: single-pass scatter into fixed slots of this many records per bucket
  int32_t pad1;
  const SegDesc* segs;
  SegStats* stats;
  SegGeom* geom;                     // [n_segs] bucket geometry (filled by the geometry kernel)
  int64_t n_buckets;
  unsigned int* counts;              // [n_buckets]
  int32_t* bucket_seg;               // [n_buckets] segment of each bucket (filled by the carry kernel)
  unsigned long long* offsets;       // [n_buckets + 1]
  unsigned long long* cursor;        // [n_buckets] records placed: 8 B form | 16 B form << 32
  unsigned long long* maxend;        // [n_buckets][3] per slot, 0 = none
  long long* carry;                  // [n_buckets][3] per level
  long long* bsum;                    // [n_buckets][3] measure contributed by the bucket
  unsigned int* ncomp;               // [n_buckets][3]
  long long* base;                    // [n_buckets][3] measure of all earlier buckets
  long long* seg_total;              // [n_segs][3]
  Elem* elems;                       // bucket regions, 16 B per record slot (see above)
  Elem* elems2;                      // [n_elems] scratch for oversized buckets
  Comp* comp[kLevels];               // [n_elems] each: components of wide segments
  CompN* compn[kLevels];             // [n_elems] each: components of narrow segments
  int64_t n_elems;
  unsigned long long* err;           // [0] first bad record: chunk << 40 | index
  unsigned long long* scan_state;    // decoupled look-back words of the bucket scan
  unsigned int* ticket;              // [4]: scan ticket, block-path take counter, block-path queue length
  unsigned int* queue;               // [n_buckets] buckets handed to the block path
  unsigned long long* oversized;     // [0] buckets above the on-chip capacity, [1] buckets above slot_cap
  unsigned int* owner_err;           // [n_owners] set when an owner has an invalid record
  unsigned long long* racc;          // [n_racc][9] per-region partial sums and maxima, zero between launches
  int64_t n_racc;
  int32_t n_owners;
  int32_t seg_group;                 // > 1: the per-segment passes take segments in groups (many small segments)
};

}  // namespace hpop
