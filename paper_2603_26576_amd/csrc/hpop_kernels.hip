// HIP kernels of the trace reduction, written for CDNA4 (gfx950, wave64).
//
// All passes are memory-bound integer work: no MFMA (there is no dense
// contraction), loads and stores are coalesced, the fine-grained sort runs in
// LDS (160 KB per workgroup on gfx950), and cross-workgroup communication is
// limited to atomics on per-bucket counters plus one decoupled look-back scan
// over bucket counts.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <climits>

#include "hpop_device.h"
#include "hpop_internal.h"
#include "hpop_kernels.h"

namespace hpop {

// ----------------------------------------------------------------------------
// reset: per-build counters to their identities
// ----------------------------------------------------------------------------

__global__ void k_reset(Plan p) {
  const long long tid = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const long long stride = (long long)gridDim.x * blockDim.x;
  for (long long i = tid; i < p.n_segs; i += stride) {
    p.stats[i].min_s = ULLONG_MAX;
    p.stats[i].max_s = 0;
    p.stats[i].max_e = 0;
    p.stats[i].pad = 0;
  }
  for (long long i = tid; i < p.n_buckets; i += stride) {
    p.counts[i] = 0;
    p.cursor[i] = 0;
  }
  for (long long i = tid; i < 3 * p.n_buckets; i += stride) p.maxend[i] = 0;
  const long long nscan = (p.n_buckets + kScanTile - 1) / kScanTile + 1;
  for (long long i = tid; i < nscan; i += stride) p.scan_state[i] = 0;
  if (tid == 0) {
    p.err[0] = ULLONG_MAX;
    p.oversized[0] = 0;
    p.oversized[1] = 0;
  }
  if (tid < 4) p.ticket[tid] = 0;
  for (long long i = tid; i < p.n_owners; i += stride) p.owner_err[i] = 0;
  for (long long i = tid; i < 9 * p.n_racc; i += stride) p.racc[i] = 0;
}

// ----------------------------------------------------------------------------
// shared tiles: chunks of fewer than half a tile of records, several per tile.
// The same passes as for a tile of one chunk, with the chunk (and so the
// segment, kind and bucket geometry) looked up per record and buckets indexed
// globally. They run in the same launches as the other tiles (the blocks past
// n_own_tiles), reusing those kernels' LDS arrays where the layouts agree.
// ----------------------------------------------------------------------------

// One 8 B word stored past the caches: a record in the bucketed form (the
// regrouped records, 1 GB for 1.25e8, are read back only by the merge, after
// the scatter has finished), or a merged interval of the wave merge.
__device__ __forceinline__ void put_rec8(uint2* dst, unsigned int key, unsigned int end) {
  __builtin_nontemporal_store((unsigned long long)key | ((unsigned long long)end << 32), (unsigned long long*)dst);
}

// Two 8 B words loaded past the caches: the start-range pass reads every
// start once, and the scatter after it reads them again from HBM anyway.
__device__ __forceinline__ ulonglong2 get_pair_nt(const ulonglong2* src) {
  typedef unsigned long long u64x2 __attribute__((ext_vector_type(2)));
  const u64x2 t = __builtin_nontemporal_load((const u64x2*)src);
  return make_ulonglong2(t.x, t.y);
}

// The chunks of one shared tile, staged in LDS.
struct ShTile {
  const int64_t* s[kTileChunks];
  const int64_t* e[kTileChunks];
  long long bucket_begin[kTileChunks];
  Geom g[kTileChunks];
  int off[kTileChunks + 1];  // off[j]: the tile's index of chunk j's first record; off[n]: records in the tile
  int seg[kTileChunks];
  int slot[kTileChunks];
  int n;                     // chunks in the tile
  int first;                 // index of the first one in the chunk table
};

// Stages the chunks of shared tile `tile` (every thread calls; ends with a
// barrier). They are the chunks up to the tile's last one whose first tile is
// `tile`: thread j takes the j-th from the end and files it at its place. The
// geometry exists only after the start-range pass.
template <bool kGeom>
__device__ __forceinline__ void sh_load(const Plan& p, long long tile, ShTile& T) {
  const int last = p.tile_chunk[tile];
  for (int j = threadIdx.x; j < kTileChunks && j <= last; j += blockDim.x) {
    const ChunkDesc cd = p.chunks[last - j];
    if (cd.tile_begin != tile) continue;
    const int q = cd.tile_pos;
    T.s[q] = cd.s;
    T.e[q] = cd.e;
    T.off[q] = cd.tile_off;
    T.seg[q] = cd.seg;
    T.slot[q] = cd.slot;
    if (kGeom) {
      T.bucket_begin[q] = p.segs[cd.seg].bucket_begin;
      T.g[q] = p.geom[cd.seg];
    }
    if (j == 0) {
      T.off[q + 1] = cd.tile_off + (int)cd.count;
      T.n = q + 1;
      T.first = last - q;
    }
  }
  __syncthreads();
}

// The chunk of tile record x < off[n]: the largest j < n with off[j] <= x.
__device__ __forceinline__ int sh_find(const ShTile& T, int x) {
  int j = 0;
#pragma unroll
  for (int step = kTileChunks / 2; step > 0; step >>= 1) {
    const int m = j + step;
    if (m < T.n && T.off[m] <= x) j = m;
  }
  return j;
}

struct ShStatsSmem {
  ShTile T;
  unsigned long long mn[kTileChunks], mx[kTileChunks];  // start range per chunk of the tile
};

// Start range of the records of shared tile `tile`, per chunk, into the segment statistics.
template <int THREADS>
__device__ __forceinline__ void stats_shared(const Plan& p, long long tile, ShStatsSmem& S) {
  for (int j = threadIdx.x; j < kTileChunks; j += THREADS) {
    S.mn[j] = ULLONG_MAX;
    S.mx[j] = 0;
  }
  sh_load<false>(p, tile, S.T);
  const int n = S.T.off[S.T.n];
  for (int x = threadIdx.x; x < n; x += THREADS) {
    const int j = sh_find(S.T, x);
    const unsigned long long v = (unsigned long long)S.T.s[j][x - S.T.off[j]];
    if (v < (unsigned long long)kTimeLimit) {  // invalid starts stay out of the range
      atomicMin(&S.mn[j], v);
      atomicMax(&S.mx[j], v);
    }
  }
  __syncthreads();
  for (int j = threadIdx.x; j < S.T.n; j += THREADS) {
    if (S.mn[j] != ULLONG_MAX) {
      atomicMin(&p.stats[S.T.seg[j]].min_s, S.mn[j]);
      atomicMax(&p.stats[S.T.seg[j]].max_s, S.mx[j]);
    }
  }
}

// Per record of a shared tile: its chunk, and its start and end, loaded for
// all rounds first from positions clamped into the tile (n >= 1).
template <int THREADS, int IPT>
__device__ __forceinline__ void sh_records(const ShTile& T, int n, int (&jj)[IPT], long long (&svs)[IPT],
                                           long long (&evs)[IPT]) {
#pragma unroll
  for (int k = 0; k < IPT; ++k) {
    const int x = threadIdx.x + k * THREADS;
    const int xc = x < n ? x : n - 1;
    jj[k] = sh_find(T, xc);
  }
#pragma unroll
  for (int k = 0; k < IPT; ++k) {
    const int x = threadIdx.x + k * THREADS;
    const int i = (x < n ? x : n - 1) - T.off[jj[k]];
    svs[k] = T.s[jj[k]][i];
    evs[k] = T.e[jj[k]][i];
  }
}

// Bucket counts of shared tile `tile` (s_rng and hist: the count kernel's LDS arrays).
template <int THREADS, int IPT>
__device__ __forceinline__ void hist_shared(const Plan& p, long long tile, ShTile& T, int (*s_rng)[THREADS / 64],
                                            unsigned int* hist) {
  constexpr int NW = THREADS / 64;
  constexpr int HW = THREADS * IPT <= kHistWin ? THREADS * IPT / 4 : kHistWin;
  for (int i = threadIdx.x; i < HW; i += THREADS) hist[i] = 0;
  sh_load<true>(p, tile, T);
  const int n = T.off[T.n];
  int jj[IPT], gbk[IPT];
  long long svs[IPT], evs[IPT];
  sh_records<THREADS, IPT>(T, n, jj, svs, evs);
  int bmin = INT_MAX, bmax = -1;
#pragma unroll
  for (int k = 0; k < IPT; ++k) {
    gbk[k] = -1;
    if ((int)threadIdx.x + k * THREADS < n && rec_valid(svs[k], evs[k]) && svs[k] < evs[k]) {
      const int j = jj[k];
      gbk[k] = (int)(T.bucket_begin[j] + bucket_of(svs[k], T.g[j]));
      bmin = min(bmin, gbk[k]);
      bmax = max(bmax, gbk[k]);
    }
  }
  bmin = wave_reduce_i32<OpMinI>(bmin, INT_MAX);
  bmax = wave_reduce_i32<OpMaxI>(bmax, -1);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (lane == 0) { s_rng[0][wave] = bmin; s_rng[1][wave] = bmax; }
  __syncthreads();
  bmin = INT_MAX; bmax = -1;
  for (int w = 0; w < NW; ++w) { bmin = min(bmin, s_rng[0][w]); bmax = max(bmax, s_rng[1][w]); }
  if (bmax < 0) return;  // uniform: no valid record in this tile
  if (bmax - bmin < HW) {
#pragma unroll
    for (int k = 0; k < IPT; ++k) {
      unsigned long long todo = __ballot(gbk[k] >= 0);
      while (todo) {
        const int leader = __ffsll((long long)todo) - 1;
        const int lb = __builtin_amdgcn_readlane(gbk[k], leader);
        const unsigned long long m = __ballot(gbk[k] == lb);
        if (lane == leader) atomicAdd(&hist[lb - bmin], (unsigned int)__popcll(m));
        todo &= ~m;
      }
    }
    __syncthreads();
    for (int i = threadIdx.x; i <= bmax - bmin; i += THREADS)
      if (hist[i]) atomicAdd(&p.counts[bmin + i], hist[i]);
  } else {
#pragma unroll
    for (int k = 0; k < IPT; ++k)
      if (gbk[k] >= 0) atomicAdd(&p.counts[gbk[k]], 1u);
  }
}

// Scatter of shared tile `tile`. s_rng, hist, bbase and bunit are the
// scatter kernel's LDS arrays; the largest ends are kept per bucket and kind
// slot: slot 0 in the kernel's bmaxe, slots 1 and 2 in bmaxe12 (2 x HW).
template <int THREADS, int IPT>
__device__ __forceinline__ void scatter_shared(const Plan& p, long long tile, ShTile& T, int (*s_rng)[THREADS / 64],
                                               unsigned long long* hist, unsigned long long* bbase,
                                               unsigned long long* bmaxe0, unsigned long long* bmaxe12,
                                               long long* bunit) {
  constexpr int NW = THREADS / 64;
  constexpr int HW = THREADS * IPT <= kHistWin ? THREADS * IPT / 4 : kHistWin;
  auto bmaxe = [&](int w, int sl) -> unsigned long long& { return sl == 0 ? bmaxe0[w] : bmaxe12[(sl - 1) * HW + w]; };
  for (int i = threadIdx.x; i < HW; i += THREADS) {
    hist[i] = 0;
    bmaxe0[i] = 0;
    bmaxe12[i] = 0;
    bmaxe12[HW + i] = 0;
  }
  sh_load<true>(p, tile, T);
  const int n = T.off[T.n];
  int jj[IPT], gbk[IPT];
  bool nr[IPT];
  unsigned int kx[IPT], ex[IPT];
  {
    long long svs[IPT], evs[IPT];
    sh_records<THREADS, IPT>(T, n, jj, svs, evs);
#pragma unroll
    for (int k = 0; k < IPT; ++k) {
      const int x = threadIdx.x + k * THREADS;
      gbk[k] = -1;
      nr[k] = false;
      kx[k] = 0;
      ex[k] = 0;
      if (x < n) {
        const int j = jj[k];
        const long long sv = svs[k], ev = evs[k];
        if (!rec_valid(sv, ev)) {
          // first bad record of the build: chunk << 40 | index (rare path)
          const ChunkDesc& cd = p.chunks[T.first + j];
          atomicMin(p.err, ((unsigned long long)cd.chunk_id << 40) | (unsigned long long)(x - T.off[j]));
          p.owner_err[cd.owner] = 1u;
        } else if (sv < ev) {
          const Geom& g = T.g[j];
          const int b = bucket_of(sv, g);
          const long long lo = bucket_lo(g, b);
          gbk[k] = (int)(T.bucket_begin[j] + b);
          nr[k] = seg_narrow(g);
          kx[k] = ((unsigned int)(sv - lo) << 2) | (unsigned int)T.slot[j];
          ex[k] = ev - lo < 0xFFFFFFFFll ? (unsigned int)(ev - lo + 1) : 0xFFFFFFFFu;  // far ends clamped
        }
      }
    }
  }
  int bmin = INT_MAX, bmax = -1;
#pragma unroll
  for (int k = 0; k < IPT; ++k) {
    if (gbk[k] >= 0) {
      bmin = min(bmin, gbk[k]);
      bmax = max(bmax, gbk[k]);
    }
  }
  bmin = wave_reduce_i32<OpMinI>(bmin, INT_MAX);
  bmax = wave_reduce_i32<OpMaxI>(bmax, -1);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (lane == 0) { s_rng[0][wave] = bmin; s_rng[1][wave] = bmax; }
  __syncthreads();
  bmin = INT_MAX; bmax = -1;
  for (int w = 0; w < NW; ++w) { bmin = min(bmin, s_rng[0][w]); bmax = max(bmax, s_rng[1][w]); }
  if (bmax < 0) return;  // uniform: no valid record in this tile
  const long long scap = p.slot_cap;
  unsigned long long* gmax = p.maxend;
  uint2* units = (uint2*)p.elems;
  auto region = [&](long long gb, long long& ub, long long& ucap) {
    if (scap) {
      ub = 2 * gb * scap;
      ucap = 2 * scap;
    } else {
      ub = 2 * (long long)p.offsets[gb];
      ucap = 2 * (long long)p.counts[gb];
    }
  };
  // a record in the 16 B form, read again from its chunk (rare)
  auto put_wide = [&](int k, long long ub, long long ucap, unsigned long long rank) {
    if (2 * ((long long)rank + 1) <= ucap) {
      const int j = jj[k];
      const int i = (int)threadIdx.x + k * THREADS - T.off[j];
      Elem el;
      el.s = T.s[j][i];
      el.e_slot = (long long)((unsigned long long)T.e[j][i] | ((unsigned long long)T.slot[j] << kSlotShift));
      *(Elem*)(units + ub + ucap - 2 * ((long long)rank + 1)) = el;
    }
  };
  auto end_of = [&](int k) { return T.e[jj[k]][(int)threadIdx.x + k * THREADS - T.off[jj[k]]]; };
  if (bmax - bmin < HW) {
    unsigned int rk[IPT];
    const unsigned long long lt = (1ull << lane) - 1ull;
#pragma unroll
    for (int k = 0; k < IPT; ++k) {
      // lanes of one bucket and kind share one LDS atomic: the leader reserves
      // their ranks (per form) and folds their largest end in
      rk[k] = 0;
      const int sl = gbk[k] >= 0 ? T.slot[jj[k]] : 0;
      unsigned long long todo = __ballot(gbk[k] >= 0);
      while (todo) {
        const int leader = __ffsll((long long)todo) - 1;
        const int lb = __builtin_amdgcn_readlane(gbk[k], leader);
        const int ls = __builtin_amdgcn_readlane(sl, leader);
        const bool in = gbk[k] == lb && sl == ls;
        const unsigned long long m = __ballot(in);
        const unsigned long long mn = __ballot(in && nr[k]);
        long long emax;
        unsigned int e32 = 0;
        if (mn == m) e32 = (unsigned int)wave_reduce_i32<OpMaxU32>((int)(in ? ex[k] : 0u), 0);
        if (mn == m && e32 != 0xFFFFFFFFu) {
          // all 8 B records, none clamped: the largest end in 32 bits, relative to the bucket
          const int jl = __builtin_amdgcn_readlane(jj[k], leader);
          emax = bucket_lo(T.g[jl], lb - T.bucket_begin[jl]) + (long long)e32 - 1;
        } else {
          emax = wave_reduce_i64<OpMax>(in ? end_of(k) : 0ll, 0ll);
        }
        unsigned long long b = 0;
        if (lane == leader) {
          const unsigned long long c8 = (unsigned long long)__popcll(mn), c16 = (unsigned long long)__popcll(m & ~mn);
          b = atomicAdd(&hist[lb - bmin], c8 | (c16 << 32));
          atomicMax(&bmaxe(lb - bmin, ls), (unsigned long long)emax);
        }
        b = (unsigned long long)readlane64((long long)b, leader);
        if (in) rk[k] = nr[k] ? (unsigned int)b + (unsigned int)__popcll(mn & lt)
                              : (unsigned int)(b >> 32) + (unsigned int)__popcll(m & ~mn & lt);
        todo &= ~m;
      }
    }
    __syncthreads();
    for (int i = threadIdx.x; i <= bmax - bmin; i += THREADS) {
      const unsigned long long h = hist[i];
      if (h) {
        const long long gb = (long long)bmin + i;
        const unsigned long long old = atomicAdd(&p.cursor[gb], h);
        bbase[i] = old;
        long long ub, ucap;
        region(gb, ub, ucap);
        bunit[i] = ub;
        for (int sl = 0; sl < 3; ++sl)
          if (bmaxe(i, sl)) atomicMax(&gmax[gb * 3 + sl], bmaxe(i, sl));
        const unsigned long long tot = (old & 0xFFFFFFFFull) + (old >> 32) + (h & 0xFFFFFFFFull) + (h >> 32);
        if (scap && tot > (unsigned long long)scap && tot - (h & 0xFFFFFFFFull) - (h >> 32) <= (unsigned long long)scap)
          atomicAdd(&p.oversized[1], 1ull);  // slot overflow: the build is redone with exact offsets
      }
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < IPT; ++k) {
      if (gbk[k] >= 0) {
        const int w = gbk[k] - bmin;
        const unsigned long long bb = bbase[w];
        const long long ub = bunit[w];
        long long ub2, ucap;
        region(gbk[k], ub2, ucap);
        if (nr[k]) {
          const unsigned long long rank = (bb & 0xFFFFFFFFull) + rk[k];
          // non-temporal: written once here and read once by the merge, never cached in between
          if ((long long)rank < ucap) put_rec8(units + ub + (long long)rank, kx[k], ex[k]);
        } else {
          put_wide(k, ub, ucap, (bb >> 32) + rk[k]);
        }
      }
    }
  } else {
#pragma unroll
    for (int k = 0; k < IPT; ++k) {
      if (gbk[k] >= 0) {
        const long long gb = gbk[k];
        const unsigned long long old = atomicAdd(&p.cursor[gb], nr[k] ? 1ull : (1ull << 32));
        atomicMax(&gmax[gb * 3 + T.slot[jj[k]]], (unsigned long long)end_of(k));
        if (scap && (old & 0xFFFFFFFFull) + (old >> 32) == (unsigned long long)scap)
          atomicAdd(&p.oversized[1], 1ull);
        long long ub, ucap;
        region(gb, ub, ucap);
        if (nr[k]) {
          if ((long long)(old & 0xFFFFFFFFull) < ucap) units[ub + (long long)(old & 0xFFFFFFFFull)] = make_uint2(kx[k], ex[k]);
        } else {
          put_wide(k, ub, ucap, old >> 32);
        }
      }
    }
  }
}

// ----------------------------------------------------------------------------
// stats: validate records, per-segment min/max start and max end
// ----------------------------------------------------------------------------

template <int THREADS, bool kShared>
__global__ __launch_bounds__(THREADS) void k_stats(Plan p) {
  // The bucket grid needs only the range of starts; validation happens in the
  // scatter, which reads both ends anyway. Starts outside [0, 2^62) belong to
  // invalid records and are left out of the range.
  constexpr int NW = THREADS / 64;
  __shared__ unsigned long long red[2][NW];
  if constexpr (kShared) {
    if (blockIdx.x >= p.n_own_tiles) {
      __shared__ ShStatsSmem sh;
      stats_shared<THREADS>(p, blockIdx.x, sh);
      return;
    }
  }
  const long long tile = blockIdx.x;
  const ChunkDesc cd = p.chunks[p.tile_chunk[tile]];
  const long long base = (tile - cd.tile_begin) * (long long)p.tile_elems;
  const long long end = min((long long)cd.count, base + p.tile_elems);
  unsigned long long mn = ULLONG_MAX, mxs = 0;
  auto take = [&](unsigned long long s) {
    if (s < (unsigned long long)kTimeLimit) {
      mn = s < mn ? s : mn;
      mxs = s > mxs ? s : mxs;
    }
  };
  if ((((uintptr_t)cd.s) & 15) == 0 && end - base == p.tile_elems && (p.tile_elems & (2 * THREADS - 1)) == 0) {
    // a full tile from a 16 B aligned array: pairs of starts, all loads issued first
    const ulonglong2* v = (const ulonglong2*)(cd.s + base);
    const int npairs = p.tile_elems / 2;
    constexpr int U = 4;
    for (int j0 = threadIdx.x; j0 < npairs; j0 += U * THREADS) {
      ulonglong2 x[U];
#pragma unroll
      for (int u = 0; u < U; ++u) x[u] = j0 + u * THREADS < npairs ? get_pair_nt(v + j0 + u * THREADS) : make_ulonglong2(ULLONG_MAX, ULLONG_MAX);
#pragma unroll
      for (int u = 0; u < U; ++u) {
        take(x[u].x);
        take(x[u].y);
      }
    }
  } else {
    for (long long i = base + threadIdx.x; i < end; i += THREADS) take((unsigned long long)cd.s[i]);
  }
  mn = wave_red_minu(mn);
  mxs = wave_red_maxu(mxs);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (lane == 0) {
    red[0][wave] = mn;
    red[1][wave] = mxs;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int w = 1; w < NW; ++w) {
      mn = red[0][w] < mn ? red[0][w] : mn;
      mxs = red[1][w] > mxs ? red[1][w] : mxs;
    }
    if (mn != ULLONG_MAX) {
      atomicMin(&p.stats[cd.seg].min_s, mn);
      atomicMax(&p.stats[cd.seg].max_s, mxs);
    }
  }
}

// Small tiles (at most 512 records): one wave per tile, four tiles per
// workgroup, so a lane reduces 8 records instead of a workgroup reducing 2 per
// thread (traces of many small record batches have mostly partial tiles).
template <bool kShared>
__global__ __launch_bounds__(256) void k_stats_small(Plan p) {
  if constexpr (kShared) {
    // blocks past those of the other tiles: one shared tile each
    const long long own_blocks = (p.n_own_tiles + 3) / 4;
    if (blockIdx.x >= own_blocks) {
      __shared__ ShStatsSmem sh;
      stats_shared<256>(p, p.n_own_tiles + (blockIdx.x - own_blocks), sh);
      return;
    }
  }
  const int lane = threadIdx.x & 63;
  const long long tile = (long long)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (tile >= p.n_own_tiles) return;
  const ChunkDesc cd = p.chunks[p.tile_chunk[tile]];
  const long long base = (tile - cd.tile_begin) * (long long)p.tile_elems;
  const long long end = min((long long)cd.count, base + p.tile_elems);
  unsigned long long mn = ULLONG_MAX, mxs = 0;
  long long v[8];
#pragma unroll
  for (int k = 0; k < 8; ++k) {  // all loads first, from positions clamped into the tile (base < end)
    const long long i = base + lane + 64 * k;
    v[k] = __builtin_nontemporal_load(cd.s + (i < end ? i : end - 1));
  }
#pragma unroll
  for (int k = 0; k < 8; ++k) {
    const unsigned long long s = (unsigned long long)v[k];
    if (base + lane + 64 * k < end && s < (unsigned long long)kTimeLimit) {
      mn = s < mn ? s : mn;
      mxs = s > mxs ? s : mxs;
    }
  }
  mn = wave_red_minu(mn);
  mxs = wave_red_maxu(mxs);
  if (lane == 0 && mn != ULLONG_MAX) {
    atomicMin(&p.stats[cd.seg].min_s, mn);
    atomicMax(&p.stats[cd.seg].max_s, mxs);
  }
}

// The bucket geometry of every segment from its start range (one thread per
// segment, after the start-range pass).
__global__ void k_geom(Plan p) {
  const long long seg = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (seg < p.n_segs) p.geom[seg] = make_geom(p.stats[seg], p.segs[seg]);
}

// ----------------------------------------------------------------------------
// hist / scatter: regroup records by time bucket
// ----------------------------------------------------------------------------

// Buckets of one tile usually span a narrow window (records arrive roughly in
// time order), so per-tile counting uses an LDS window [bmin, bmin + HW): kHistWin
// buckets, or a quarter of the tile's records for tiles of at most kHistWin records.
// Wider tiles fall back to global atomics per record.

template <int THREADS, int IPT, bool kShared>
__global__ __launch_bounds__(THREADS) void k_hist(Plan p) {
  constexpr int NW = THREADS / 64;
  constexpr int HW = THREADS * IPT <= kHistWin ? THREADS * IPT / 4 : kHistWin;  // LDS bucket window
  __shared__ int s_rng[2][NW];
  __shared__ unsigned int hist[HW];
  if constexpr (kShared) {
    if (blockIdx.x >= p.n_own_tiles) {
      __shared__ ShTile T;
      hist_shared<THREADS, IPT>(p, blockIdx.x, T, s_rng, hist);
      return;
    }
  }
  const long long tile = blockIdx.x;
  const ChunkDesc cd = p.chunks[p.tile_chunk[tile]];
  const SegDesc sd = p.segs[cd.seg];
  const Geom g = seg_geom(p, cd.seg);
  const long long base = (tile - cd.tile_begin) * (long long)p.tile_elems;
  const long long end = min((long long)cd.count, base + p.tile_elems);
  int bk[IPT];
  int bmin = INT_MAX, bmax = -1;
  // the loads of all rounds first, from positions clamped into the tile
  long long svs[IPT], evs[IPT];
#pragma unroll
  for (int k = 0; k < IPT; ++k) {
    const long long i = base + threadIdx.x + (long long)k * THREADS;
    const long long ic = i < end ? i : end - 1;
    svs[k] = cd.s[ic];
    evs[k] = cd.e[ic];
  }
#pragma unroll
  for (int k = 0; k < IPT; ++k) {
    const long long i = base + threadIdx.x + (long long)k * THREADS;
    bk[k] = -1;
    if (i < end) {
      const long long s = svs[k], e = evs[k];
      if (rec_valid(s, e) && s < e) {
        bk[k] = bucket_of(s, g);
        bmin = min(bmin, bk[k]);
        bmax = max(bmax, bk[k]);
      }
    }
  }
  bmin = wave_reduce_i32<OpMinI>(bmin, INT_MAX);
  bmax = wave_reduce_i32<OpMaxI>(bmax, -1);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (lane == 0) { s_rng[0][wave] = bmin; s_rng[1][wave] = bmax; }
  for (int i = threadIdx.x; i < HW; i += THREADS) hist[i] = 0;
  __syncthreads();
  bmin = INT_MAX; bmax = -1;
  for (int w = 0; w < NW; ++w) { bmin = min(bmin, s_rng[0][w]); bmax = max(bmax, s_rng[1][w]); }
  if (bmax < 0) return;  // uniform: no valid record in this tile
  const bool windowed = bmax - bmin < HW;
  if (windowed) {
#pragma unroll
    for (int k = 0; k < IPT; ++k) {
      // one LDS atomic per distinct bucket of the wave, not one per record
      unsigned long long todo = __ballot(bk[k] >= 0);
      while (todo) {
        const int leader = __ffsll((long long)todo) - 1;
        const int lb = __builtin_amdgcn_readlane(bk[k], leader);
        const unsigned long long m = __ballot(bk[k] == lb);
        if (lane == leader) atomicAdd(&hist[lb - bmin], (unsigned int)__popcll(m));
        todo &= ~m;
      }
    }
    __syncthreads();
    for (int i = threadIdx.x; i <= bmax - bmin; i += THREADS)
      if (hist[i]) atomicAdd(&p.counts[sd.bucket_begin + bmin + i], hist[i]);
  } else {
#pragma unroll
    for (int k = 0; k < IPT; ++k)
      if (bk[k] >= 0) atomicAdd(&p.counts[sd.bucket_begin + bk[k]], 1u);
  }
}

// exclusive scan of bucket counts -> offsets (decoupled look-back), one tile
// of kScanTile buckets per workgroup in the order of a ticket
template <int THREADS>
__device__ __forceinline__ void scan_tile(const Plan& p) {
  constexpr int IPT = kScanTile / THREADS;
  __shared__ unsigned int s_bid;
  __shared__ long long lds[THREADS / 64];
  __shared__ unsigned long long s_excl;
  if (threadIdx.x == 0) s_bid = atomicAdd(&p.ticket[0], 1u);
  __syncthreads();
  const long long bid = s_bid;
  const long long b0 = bid * kScanTile + (long long)threadIdx.x * IPT;
  unsigned int c[IPT];
  long long tsum = 0;
  const bool slots = p.slot_cap > 0;
#pragma unroll
  for (int k = 0; k < IPT; ++k) {
    c[k] = 0u;
    if (b0 + k < p.n_buckets) {
      if (slots) {
        // counts of the single-pass scatter (capped: an overflow is redone exactly)
        const unsigned long long cu = p.cursor[b0 + k];
        const unsigned long long n = (cu & 0xFFFFFFFFull) + (cu >> 32);
        c[k] = (unsigned int)(n < (unsigned long long)p.slot_cap ? n : (unsigned long long)p.slot_cap);
        p.counts[b0 + k] = c[k];
      } else {
        c[k] = p.counts[b0 + k];
      }
    }
    tsum += c[k];
  }
  long long v[1] = {tsum}, ex[1], tot[1];
  block_excl_scan<THREADS, 1, OpSum>(v, ex, tot, 0, lds);
  constexpr unsigned long long FLAG_AGG = 1ull << 62, FLAG_INC = 2ull << 62, VMASK = (1ull << 62) - 1;
  if (threadIdx.x == 0) {
    unsigned long long* st = p.scan_state;
    if (bid == 0) {
      __hip_atomic_store(&st[0], FLAG_INC | (unsigned long long)tot[0], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      s_excl = 0;
    } else {
      __hip_atomic_store(&st[bid], FLAG_AGG | (unsigned long long)tot[0], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      unsigned long long acc = 0;
      long long j = bid - 1;
      while (j >= 0) {
        unsigned long long w = __hip_atomic_load(&st[j], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        const unsigned long long f = w & ~VMASK;
        if (f == 0) { __builtin_amdgcn_s_sleep(1); continue; }
        acc += w & VMASK;
        if (f == FLAG_INC) break;
        --j;
      }
      __hip_atomic_store(&st[bid], FLAG_INC | (acc + (unsigned long long)tot[0]), __ATOMIC_RELAXED,
                         __HIP_MEMORY_SCOPE_AGENT);
      s_excl = acc;
    }
  }
  __syncthreads();
  unsigned long long run = s_excl + (unsigned long long)ex[0];
#pragma unroll
  for (int k = 0; k < IPT; ++k) {
    if (b0 + k < p.n_buckets) {
      p.offsets[b0 + k] = run;  // cursors stay relative: the scatter adds the bucket's base
      if (c[k] > (unsigned)p.cap) atomicAdd(p.oversized, 1ull);
    }
    run += c[k];
  }
  // the thread holding the last bucket also writes the grand total
  if (b0 < p.n_buckets && p.n_buckets <= b0 + IPT) p.offsets[p.n_buckets] = run;
}

template <int THREADS>
__global__ __launch_bounds__(THREADS) void k_scan(Plan p) {
  scan_tile<THREADS>(p);
}

template <int THREADS, int IPT, bool kShared>
__global__ __launch_bounds__(THREADS) void k_scatter(Plan p) {
  constexpr int NW = THREADS / 64;
  // LDS bucket window: a quarter of the tile's records for tiles of at most kHistWin records
  constexpr int HW = THREADS * IPT <= kHistWin ? THREADS * IPT / 4 : kHistWin;
  __shared__ int s_rng[2][NW];
  __shared__ unsigned long long hist[HW];   // per window bucket: 8 B records | 16 B records << 32
  __shared__ unsigned long long bbase[HW];  // the same counts placed before this tile
  __shared__ unsigned long long bmaxe[HW];  // largest end of the tile's records
  __shared__ long long bunit[HW];           // first unit of the bucket's region
  if constexpr (kShared) {
    if (blockIdx.x >= p.n_own_tiles) {
      __shared__ ShTile T;
      __shared__ unsigned long long bmaxe12[2 * HW];
      scatter_shared<THREADS, IPT>(p, blockIdx.x, T, s_rng, hist, bbase, bmaxe, bmaxe12, bunit);
      return;
    }
  }
  const long long tile = blockIdx.x;
  const ChunkDesc cd = p.chunks[p.tile_chunk[tile]];
  const SegDesc sd = p.segs[cd.seg];
  const Geom g = seg_geom(p, cd.seg);
  const bool seg_n = seg_narrow(g);
  const long long base = (tile - cd.tile_begin) * (long long)p.tile_elems;
  const long long end = min((long long)cd.count, base + p.tile_elems);
  // per record: bucket (-1: none), form, and the 8 B form itself; a record in
  // the 16 B form is read again where it is needed (rare)
  int bk[IPT];
  bool nr[IPT];
  unsigned int kx[IPT], ex[IPT];
  int bmin = INT_MAX, bmax = -1;
  // the loads of all rounds first, from positions clamped into the tile
  // (base < end): they issue back to back instead of one masked block (and
  // one wait) per round; non-temporal, as this pass reads each record once
  long long svs[IPT], evs[IPT];
#pragma unroll
  for (int k = 0; k < IPT; ++k) {
    const long long i = base + threadIdx.x + (long long)k * THREADS;
    const long long ic = i < end ? i : end - 1;
    svs[k] = __builtin_nontemporal_load(cd.s + ic);
    evs[k] = __builtin_nontemporal_load(cd.e + ic);
  }
#pragma unroll
  for (int k = 0; k < IPT; ++k) {
    const long long i = base + threadIdx.x + (long long)k * THREADS;
    bk[k] = -1;
    nr[k] = false;
    kx[k] = 0;
    ex[k] = 0;
    if (i < end) {
      const long long sv = svs[k], ev = evs[k];
      if (!rec_valid(sv, ev)) {
        // first bad record of the build: chunk << 40 | index (rare path)
        atomicMin(p.err, ((unsigned long long)cd.chunk_id << 40) | (unsigned long long)i);
        p.owner_err[cd.owner] = 1u;
      } else if (sv < ev) {
        bk[k] = bucket_of(sv, g);
        const long long lo = bucket_lo(g, bk[k]);
        nr[k] = seg_n;
        kx[k] = ((unsigned int)(sv - lo) << 2) | (unsigned int)cd.slot;
        ex[k] = ev - lo < 0xFFFFFFFFll ? (unsigned int)(ev - lo + 1) : 0xFFFFFFFFu;  // far ends clamped
        bmin = min(bmin, bk[k]);
        bmax = max(bmax, bk[k]);
      }
    }
  }
  bmin = wave_reduce_i32<OpMinI>(bmin, INT_MAX);
  bmax = wave_reduce_i32<OpMaxI>(bmax, -1);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const long long scap = p.slot_cap;
  if (lane == 0) { s_rng[0][wave] = bmin; s_rng[1][wave] = bmax; }
  for (int i = threadIdx.x; i < HW; i += THREADS) { hist[i] = 0; bmaxe[i] = 0; }
  __syncthreads();
  bmin = INT_MAX; bmax = -1;
  for (int w = 0; w < NW; ++w) { bmin = min(bmin, s_rng[0][w]); bmax = max(bmax, s_rng[1][w]); }
  if (bmax < 0) return;
  const unsigned long long slotbits = (unsigned long long)cd.slot << kSlotShift;
  unsigned long long* gmax = p.maxend;
  uint2* units = (uint2*)p.elems;
  auto region = [&](long long gb, long long& ub, long long& ucap) {
    if (scap) {
      ub = 2 * gb * scap;
      ucap = 2 * scap;
    } else {
      ub = 2 * (long long)p.offsets[gb];
      ucap = 2 * (long long)p.counts[gb];
    }
  };
  auto put_wide = [&](int k, long long ub, long long ucap, unsigned long long rank) {
    if (2 * ((long long)rank + 1) <= ucap) {
      const long long i = base + threadIdx.x + (long long)k * THREADS;
      Elem el;
      el.s = cd.s[i];
      el.e_slot = (long long)((unsigned long long)cd.e[i] | slotbits);
      *(Elem*)(units + ub + ucap - 2 * ((long long)rank + 1)) = el;
    }
  };
  if (bmax - bmin < HW) {
    unsigned int rk[IPT];
    const unsigned long long lt = (1ull << lane) - 1ull;
#pragma unroll
    for (int k = 0; k < IPT; ++k) {
      // lanes of one bucket share one LDS atomic: the leader reserves their
      // ranks (per form) and folds their largest end in
      rk[k] = 0;
      unsigned long long todo = __ballot(bk[k] >= 0);
      while (todo) {
        const int leader = __ffsll((long long)todo) - 1;
        const int lb = __builtin_amdgcn_readlane(bk[k], leader);
        const bool in = bk[k] == lb;
        const unsigned long long m = __ballot(in);
        const unsigned long long mn = __ballot(in && nr[k]);
        long long emax;
        unsigned int e32 = 0;
        if (mn == m) e32 = (unsigned int)wave_reduce_i32<OpMaxU32>((int)(in ? ex[k] : 0u), 0);
        if (mn == m && e32 != 0xFFFFFFFFu) {
          // all 8 B records, none clamped: the largest end in 32 bits, relative to the bucket
          emax = bucket_lo(g, lb) + (long long)e32 - 1;
        } else {
          long long ev = 0;
          if (in) ev = cd.e[base + threadIdx.x + (long long)k * THREADS];
          emax = wave_reduce_i64<OpMax>(ev, 0ll);
        }
        unsigned long long b = 0;
        if (lane == leader) {
          const unsigned long long c8 = (unsigned long long)__popcll(mn), c16 = (unsigned long long)__popcll(m & ~mn);
          b = atomicAdd(&hist[lb - bmin], c8 | (c16 << 32));
          atomicMax(&bmaxe[lb - bmin], (unsigned long long)emax);
        }
        b = (unsigned long long)readlane64((long long)b, leader);
        if (in) rk[k] = nr[k] ? (unsigned int)b + (unsigned int)__popcll(mn & lt)
                              : (unsigned int)(b >> 32) + (unsigned int)__popcll(m & ~mn & lt);
        todo &= ~m;
      }
    }
    __syncthreads();
    for (int i = threadIdx.x; i <= bmax - bmin; i += THREADS) {
      const unsigned long long h = hist[i];
      if (h) {
        const long long gb = sd.bucket_begin + bmin + i;
        const unsigned long long old = atomicAdd(&p.cursor[gb], h);
        bbase[i] = old;
        long long ub, ucap;
        region(gb, ub, ucap);
        bunit[i] = ub;
        atomicMax(&gmax[gb * 3 + cd.slot], bmaxe[i]);
        const unsigned long long tot = (old & 0xFFFFFFFFull) + (old >> 32) + (h & 0xFFFFFFFFull) + (h >> 32);
        if (scap && tot > (unsigned long long)scap && tot - (h & 0xFFFFFFFFull) - (h >> 32) <= (unsigned long long)scap)
          atomicAdd(&p.oversized[1], 1ull);  // slot overflow: the build is redone with exact offsets
      }
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < IPT; ++k) {
      if (bk[k] >= 0) {
        const int w = bk[k] - bmin;
        const unsigned long long bb = bbase[w];
        const long long ub = bunit[w];
        if (nr[k]) {
          const unsigned long long rank = (bb & 0xFFFFFFFFull) + rk[k];
          const long long ucap = scap ? 2 * scap : 2 * (long long)p.counts[sd.bucket_begin + bk[k]];
          // non-temporal: written once here and read once by the merge, never cached in between
          if ((long long)rank < ucap) put_rec8(units + ub + (long long)rank, kx[k], ex[k]);
        } else {
          long long ub2, ucap;
          region(sd.bucket_begin + bk[k], ub2, ucap);
          put_wide(k, ub, ucap, (bb >> 32) + rk[k]);
        }
      }
    }
  } else {
#pragma unroll
    for (int k = 0; k < IPT; ++k) {
      if (bk[k] >= 0) {
        const long long gb = sd.bucket_begin + bk[k];
        const unsigned long long old = atomicAdd(&p.cursor[gb], nr[k] ? 1ull : (1ull << 32));
        const long long ev = cd.e[base + threadIdx.x + (long long)k * THREADS];
        atomicMax(&gmax[gb * 3 + cd.slot], (unsigned long long)ev);
        if (scap && (old & 0xFFFFFFFFull) + (old >> 32) == (unsigned long long)scap)
          atomicAdd(&p.oversized[1], 1ull);
        long long ub, ucap;
        region(gb, ub, ucap);
        if (nr[k]) {
          if ((long long)(old & 0xFFFFFFFFull) < ucap) units[ub + (long long)(old & 0xFFFFFFFFull)] = make_uint2(kx[k], ex[k]);
        } else {
          put_wide(k, ub, ucap, old >> 32);
        }
      }
    }
  }
}

// ----------------------------------------------------------------------------
// carry / base: per-segment scans over buckets, one wave per segment. A round
// covers kSegRows x 64 buckets: all of its loads are issued first (row j,
// lane i: bucket c0 + 64 j + i, coalesced), then one DPP scan per row in
// bucket order, then the stores; so a round costs one memory round trip
// ----------------------------------------------------------------------------

constexpr int kSegRows = 8;

// The carry pass of segment `seg` by one whole wave (every lane calls).
__device__ __forceinline__ void carry_segment(const Plan& p, long long seg, int lane) {
  const SegDesc sd = p.segs[seg];
  const SegStats st = p.stats[seg];
  const long long nb = sd.nb;
  // the running max end before any record: just below the first start
  const long long init = st.min_s > st.max_s ? -1 : (long long)st.min_s - 1;
  long long run[3] = {init, init, init};
  for (long long c0 = 0; c0 < nb; c0 += 64 * kSegRows) {
    unsigned long long m[kSegRows][3];
#pragma unroll
    for (int j = 0; j < kSegRows; ++j) {
      const long long b = c0 + 64 * j + lane;
      m[j][0] = m[j][1] = m[j][2] = 0;
      if (b < nb) {
        p.bucket_seg[sd.bucket_begin + b] = (int32_t)seg;
        const unsigned long long* q = p.maxend + (sd.bucket_begin + b) * 3;
        m[j][0] = q[0];
        m[j][1] = q[1];
        m[j][2] = q[2];
      }
    }
#pragma unroll
    for (int j = 0; j < kSegRows; ++j) {
      if (c0 + 64 * j >= nb) break;  // wave-uniform: rows past the segment change nothing
      const long long b = c0 + 64 * j + lane;
      long long v[3];
      v[0] = m[j][0] ? (long long)m[j][0] : LLONG_MIN;
      const long long m1 = m[j][1] ? (long long)m[j][1] : LLONG_MIN;
      const long long m2 = m[j][2] ? (long long)m[j][2] : LLONG_MIN;
      v[1] = m1 > v[0] ? m1 : v[0];
      v[2] = m2 > v[1] ? m2 : v[1];
#pragma unroll
      for (int l = 0; l < 3; ++l) {
        long long all;
        const long long ex = wave_excl_scan_dpp<OpMax>(v[l], LLONG_MIN, all);
        if (b < nb) p.carry[(sd.bucket_begin + b) * 3 + l] = ex > run[l] ? ex : run[l];
        run[l] = all > run[l] ? all : run[l];
      }
    }
  }
  // largest end of the segment (level 2 holds every kind); no record: the min start
  if (lane == 0) p.stats[seg].max_e = (unsigned long long)(run[2] > init ? run[2] : (init + 1 > 0 ? init + 1 : 0));
}

template <int THREADS>
__global__ __launch_bounds__(THREADS) void k_carry(Plan p) {
  const int lane = threadIdx.x & 63;
  const long long seg = (long long)blockIdx.x * (THREADS / 64) + (threadIdx.x >> 6);
  if (seg >= p.n_segs) return;
  carry_segment(p, seg, lane);
}

// The base pass of segment `seg` by one whole wave (every lane calls).
__device__ __forceinline__ void base_segment(const Plan& p, long long seg, int lane) {
  const SegDesc sd = p.segs[seg];
  const long long nb = sd.nb;
  long long run[3] = {0, 0, 0};
  for (long long c0 = 0; c0 < nb; c0 += 64 * kSegRows) {
    long long v[kSegRows][3];
#pragma unroll
    for (int j = 0; j < kSegRows; ++j) {
      const long long b = c0 + 64 * j + lane;
#pragma unroll
      for (int l = 0; l < 3; ++l) v[j][l] = b < nb ? p.bsum[(sd.bucket_begin + b) * 3 + l] : 0;
    }
#pragma unroll
    for (int j = 0; j < kSegRows; ++j) {
      if (c0 + 64 * j >= nb) break;  // wave-uniform: rows past the segment add nothing
      const long long b = c0 + 64 * j + lane;
#pragma unroll
      for (int l = 0; l < 3; ++l) {
        long long all;
        const long long ex = wave_excl_scan_dpp<OpSum>(v[j][l], 0, all);
        if (b < nb) p.base[(sd.bucket_begin + b) * 3 + l] = run[l] + ex;
        run[l] += all;
      }
    }
  }
  if (lane == 0) {
    for (int l = 0; l < 3; ++l) p.seg_total[seg * 3 + l] = run[l];
  }
}

template <int THREADS>
__global__ __launch_bounds__(THREADS) void k_base(Plan p) {
  const int lane = threadIdx.x & 63;
  const long long seg = (long long)blockIdx.x * (THREADS / 64) + (threadIdx.x >> 6);
  if (seg >= p.n_segs) return;
  base_segment(p, seg, lane);
}

// Plans of many small segments (a batch of small traces): a wave takes
// kSegGroup consecutive segments. A segment of at most kSegGroup buckets is
// scanned by its own group of kSegGroup lanes (a lane per bucket, scans by
// lane shuffles within the group); the larger ones of the wave follow, one
// after another, with the whole wave as above.
constexpr int kSegGroup = 8;

// inclusive scan over the kSegGroup lanes of a group (identity in lanes past
// the segment's buckets)
template <class Op>
__device__ __forceinline__ long long group_incl_scan(long long v, int k) {
#pragma unroll
  for (int d = 1; d < kSegGroup; d <<= 1) {
    const long long o = __shfl_up(v, (unsigned)d, kSegGroup);
    if (k >= d) v = Op::apply(v, o);
  }
  return v;
}

// The carry pass of segments [w kSegGroup, (w + 1) kSegGroup) by one wave.
__device__ __forceinline__ void carry_group(const Plan& p, long long w, int lane) {
  const int k = lane & (kSegGroup - 1);
  const long long seg0 = w * kSegGroup;
  if (seg0 >= p.n_segs) return;
  const long long seg = seg0 + (lane / kSegGroup);
  const bool have = seg < p.n_segs;
  const SegDesc sd = have ? p.segs[seg] : SegDesc{0, 0, 0};
  const bool small = have && sd.nb <= kSegGroup;
  if (small) {  // uniform within each group
    const SegStats st = p.stats[seg];
    const long long init = st.min_s > st.max_s ? -1 : (long long)st.min_s - 1;
    long long v[3] = {LLONG_MIN, LLONG_MIN, LLONG_MIN};
    if (k < sd.nb) {
      const long long gb = sd.bucket_begin + k;
      p.bucket_seg[gb] = (int32_t)seg;
      const unsigned long long* q = p.maxend + gb * 3;
      const unsigned long long m0 = q[0], m1 = q[1], m2 = q[2];
      v[0] = m0 ? (long long)m0 : LLONG_MIN;
      v[1] = m1 && (long long)m1 > v[0] ? (long long)m1 : v[0];
      v[2] = m2 && (long long)m2 > v[1] ? (long long)m2 : v[1];
    }
    long long last2 = init;
#pragma unroll
    for (int l = 0; l < 3; ++l) {
      const long long inc = group_incl_scan<OpMax>(v[l], k);
      long long ex = __shfl_up(inc, 1u, kSegGroup);
      if (k == 0) ex = LLONG_MIN;
      if (k < sd.nb) p.carry[(sd.bucket_begin + k) * 3 + l] = ex > init ? ex : init;
      if (l == 2) last2 = __shfl(inc, kSegGroup - 1, kSegGroup);
    }
    const long long r2 = last2 > init ? last2 : init;
    if (k == 0) p.stats[seg].max_e = (unsigned long long)(r2 > init ? r2 : (init + 1 > 0 ? init + 1 : 0));
  }
  unsigned long long big = __ballot(k == 0 && have && !small);
  while (big) {
    const int g = __ffsll((long long)big) - 1;
    big &= big - 1;
    carry_segment(p, seg0 + g / kSegGroup, lane);
  }
}

template <int THREADS>
__global__ __launch_bounds__(THREADS) void k_carry_grouped(Plan p) {
  carry_group(p, (long long)blockIdx.x * (THREADS / 64) + (threadIdx.x >> 6), threadIdx.x & 63);
}

// Fixed slots: the bucket scan and the carry pass read only what the scatter
// wrote, so one launch does both: workgroups [0, scan_blocks) scan (tiles in
// ticket order), the ones after give each wave a segment (or a group of
// kSegGroup segments).
template <bool kGrouped>
__global__ __launch_bounds__(256) void k_scan_carry(Plan p, int scan_blocks) {
  if ((int)blockIdx.x < scan_blocks) {
    scan_tile<256>(p);
    return;
  }
  const int lane = threadIdx.x & 63;
  const long long w = (long long)(blockIdx.x - scan_blocks) * 4 + (threadIdx.x >> 6);
  if constexpr (kGrouped) {
    carry_group(p, w, lane);
  } else {
    if (w < p.n_segs) carry_segment(p, w, lane);
  }
}

template <int THREADS>
__global__ __launch_bounds__(THREADS) void k_base_grouped(Plan p) {
  const int lane = threadIdx.x & 63, k = lane & (kSegGroup - 1);
  const long long seg0 = ((long long)blockIdx.x * (THREADS / 64) + (threadIdx.x >> 6)) * kSegGroup;
  if (seg0 >= p.n_segs) return;
  const long long seg = seg0 + (lane / kSegGroup);
  const bool have = seg < p.n_segs;
  const SegDesc sd = have ? p.segs[seg] : SegDesc{0, 0, 0};
  const bool small = have && sd.nb <= kSegGroup;
  if (small) {  // uniform within each group
#pragma unroll
    for (int l = 0; l < 3; ++l) {
      const long long v = k < sd.nb ? p.bsum[(sd.bucket_begin + k) * 3 + l] : 0;
      const long long inc = group_incl_scan<OpSum>(v, k);
      if (k < sd.nb) p.base[(sd.bucket_begin + k) * 3 + l] = inc - v;
      const long long tot = __shfl(inc, kSegGroup - 1, kSegGroup);
      if (k == 0) p.seg_total[seg * 3 + l] = tot;
    }
  }
  unsigned long long big = __ballot(k == 0 && have && !small);
  while (big) {
    const int g = __ffsll((long long)big) - 1;
    big &= big - 1;
    base_segment(p, seg0 + g / kSegGroup, lane);
  }
}

// ----------------------------------------------------------------------------
// merge: per bucket, sort by start in LDS and flatten each level
// ----------------------------------------------------------------------------

// Block path: one workgroup flattens bucket gb (LDS radix sort up to CAP
// records, global-memory radix sort beyond).
template <int THREADS, int CAP>
__device__ void merge_bucket_block(const Plan& p, long long gb, SortSmem<THREADS, CAP>& sm, int* s_seg) {
  if (threadIdx.x == 0) *s_seg = p.bucket_seg[gb];
  __syncthreads();
  const int seg = *s_seg;
  const SegDesc sd = p.segs[seg];
  const Geom g = seg_geom(p, seg);
  const long long bl = gb - sd.bucket_begin;
  const BucketRecs br = bucket_recs(p, gb);
  // a slot overflow makes the host redo the build: write an empty bucket
  const long long n = br.overflow ? 0 : (long long)br.n8 + br.n16;
  const long long off = (long long)p.offsets[gb];
  const int nlev = sd.n_levels;
  FlatState st;
#pragma unroll
  for (int l = 0; l < 3; ++l) {
    st.M[l] = p.carry[gb * 3 + l];
    st.P[l] = 0;
    st.R[l] = 0;
  }
  Comp* comp[3] = {p.comp[0] + off, p.comp[1] + off, p.comp[2] + off};
  CompN* compn_b[3] = {p.compn[0] + off, p.compn[1] + off, p.compn[2] + off};
  CompN* const* compn = seg_narrow(g) ? compn_b : nullptr;
  if (n > 0) {
    const long long lo = bucket_lo(g, bl);
    if (n <= CAP) {
      const int ni = (int)n;
      const unsigned long long* mx = p.maxend + gb * 3;
      for (int i = threadIdx.x; i < br.n8; i += THREADS) sm.E[i] = widen(br.narrow[i], lo, mx);
      for (int i = threadIdx.x; i < br.n16; i += THREADS) sm.E[br.n8 + i] = br.wide[i];
      __syncthreads();
      const unsigned short* ord = sort_lds<THREADS, CAP>(sm, ni, lo);
      flatten_tile<THREADS>(sm.E, ord, ni, nlev, 0, comp, compn, lo, st, sm.lds_scan, nullptr);
    } else {
      // oversized bucket (exact offsets only): every record in the 16 B form
      // into the scratch copy, a stable LSD sort between it and the bucket's
      // own region (16 B per record), then flatten CAP records at a time,
      // carrying the running state across tiles
      Elem* a = p.elems2 + off;
      const unsigned long long* mx = p.maxend + gb * 3;
      for (long long i = threadIdx.x; i < br.n8; i += THREADS) a[i] = widen(br.narrow[i], lo, mx);
      for (long long i = threadIdx.x; i < br.n16; i += THREADS) a[br.n8 + i] = br.wide[i];
      __threadfence_block();
      __syncthreads();
      const Elem* src = sort_global<THREADS, CAP>(sm, a, p.elems + off, n, lo);
      for (long long t0 = 0; t0 < n; t0 += CAP) {
        const int cnt = (int)min((long long)CAP, n - t0);
        for (int i = threadIdx.x; i < cnt; i += THREADS) sm.E[i] = src[t0 + i];
        __syncthreads();
        flatten_tile<THREADS>(sm.E, nullptr, cnt, nlev, 0, comp, compn, lo, st, sm.lds_scan, nullptr);
        __syncthreads();
      }
    }
  }
  if (threadIdx.x == 0) {
#pragma unroll
    for (int l = 0; l < 3; ++l) {
      p.bsum[gb * 3 + l] = st.P[l];
      p.ncomp[gb * 3 + l] = (unsigned int)st.R[l];
    }
  }
  __syncthreads();
}

// Buckets the wave path handed over (ticket[2] of them in p.queue): one per
// workgroup by index when they are at most as many as the workgroups, else
// taken by persistent workgroups from a shared counter (ticket[1]), every
// workgroup leaving once the counter passes the queue length.
template <int THREADS, int CAP>
__global__ __launch_bounds__(THREADS) void k_merge_block(Plan p) {
  __shared__ SortSmem<THREADS, CAP> sm;
  __shared__ int s_seg;
  __shared__ unsigned int s_idx;
  const unsigned int qlen = __hip_atomic_load(&p.ticket[2], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  if (qlen <= gridDim.x) {
    // at most one bucket per workgroup: taken by index, so the workgroups
    // without one leave at once instead of queueing on the shared counter
    if (blockIdx.x < qlen) merge_bucket_block<THREADS, CAP>(p, (long long)p.queue[blockIdx.x], sm, &s_seg);
    return;
  }
  while (true) {
    if (threadIdx.x == 0) s_idx = atomicAdd(&p.ticket[1], 1u);
    __syncthreads();
    const unsigned int idx = s_idx;
    __syncthreads();
    if (idx >= qlen) break;
    merge_bucket_block<THREADS, CAP>(p, (long long)p.queue[idx], sm, &s_seg);
  }
}

// Wave path: each wave sorts and flattens one bucket of at most kWaveCap
// records with no workgroup barrier, in 32-bit arithmetic relative to the
// bucket's first time `lo`. It takes the buckets whose records are all in the
// scatter's 8 B form:
//   key = (start - lo) << 2 | slot    (start - lo < 2^30: bucket width <= 2^30)
//   end = end - lo + 1                (< 2^32; 0 stands for "before the bucket")
// Comparisons, maxima and measure differences are unchanged by the common
// shift, and the union measure of one bucket's records stays below 2^32, so
// every quantity of the flatten fits 32 bits. The sort is a counting sort on
// the top bits of the start into 128-512 sub-bins (about one per record), writing keys and ends to
// their sorted places in LDS, then an insertion sort inside each sub-bin that
// received two or more records (equal starts may end in any order: the merged
// result does not depend on it). Other buckets (more records, any record in
// the 16 B form, a crowded sub-bin) go to the block path's queue.
struct alignas(16) WaveSmem {
  unsigned int key[kWaveCap];        // sorted keys (then, with end[], the components of one level)
  unsigned int end[kWaveCap];        // ends of the sorted records
  unsigned int bins[kWaveBins / 2];  // two 16-bit counters (then sub-bin starts) per word
};

__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// N consecutive LDS words from a position that is a multiple of N: 16-byte
// reads when N is a multiple of 4, 8-byte reads when it is even, else words
template <int N>
__device__ __forceinline__ void lds_load(const unsigned int* src, unsigned int (&dst)[N]) {
  if constexpr (N % 2 == 1) {
#pragma unroll
    for (int j = 0; j < N; ++j) dst[j] = src[j];
  } else if constexpr (N % 4 == 2) {
#pragma unroll
    for (int j = 0; j < N; j += 2) {
      const uint2 v = *(const uint2*)(src + j);
      dst[j] = v.x;
      dst[j + 1] = v.y;
    }
  } else {
#pragma unroll
    for (int j = 0; j < N; j += 4) {
      const uint4 v = *(const uint4*)(src + j);
      dst[j] = v.x;
      dst[j + 1] = v.y;
      dst[j + 2] = v.z;
      dst[j + 3] = v.w;
    }
  }
}

template <int N>
__device__ __forceinline__ void lds_store(unsigned int* dst, const unsigned int (&src)[N]) {
  if constexpr (N == 4) {
    *(uint4*)dst = make_uint4(src[0], src[1], src[2], src[3]);
  } else if constexpr (N == 2) {
    *(uint2*)dst = make_uint2(src[0], src[1]);
  } else {
#pragma unroll
    for (int j = 0; j < N; ++j) dst[j] = src[j];
  }
}

// Flatten of one sorted bucket by one wave: lane owns sorted positions
// [lane*IPL, lane*IPL + IPL), kept in registers through the three phases
// (running max of ends, measures and break counts, component writes). A
// record outside level l takes part as the empty pair (0, 0), which changes
// no maximum, measure or break, so the phases need no branches; only the
// component stores are conditional. A position past the bucket holds the key
// 2 (rank 2, start lo) with end 0: outside every lower level, and in the top
// level the pair (1, 0), which also changes nothing there, because position 0
// holds a record whose end is at least 1 and comes first in the sweep.
template <int IPL, int NLEV>
__device__ __forceinline__ void wave_flatten(const Plan& p, WaveSmem& W, long long gb, long long off, int ni,
                                             long long lo, const long long (&carry)[3],
                                             const long long (&maxe)[3]) {
  const int lane = threadIdx.x & 63;
  const int q0 = lane * IPL;
  // positions past the bucket already hold the padding pair (key 2, end 0)
  unsigned int kv[IPL], ev[IPL];
  lds_load<IPL>(W.key + q0, kv);
  lds_load<IPL>(W.end + q0, ev);
  // start - lo + 1, the same shift as the ends (recomputed at each use: fewer
  // live registers than keeping it)
  auto sv = [&](int j) { return (kv[j] >> 2) + 1u; };
  // the top level holds every record; the ones below only ranks <= l (ranks
  // are 0..2, so rank <= 1 is rank != 2: both tests share one mask of the key)
  auto in_level = [&](int j, int l) {
    return l == NLEV - 1 || (l == 0 ? (kv[j] & 3u) == 0u : (kv[j] & 3u) != 2u);
  };
  auto s_in = [&](int j, int l) { return in_level(j, l) ? sv(j) : 0u; };
  auto e_in = [&](int j, int l) { return in_level(j, l) ? ev[j] : 0u; };
  // the largest end before each lane: earlier lanes, else the earlier buckets
  unsigned int M[NLEV];
#pragma unroll
  for (int l = 0; l < NLEV; ++l) {
    unsigned int tmax = 0;
#pragma unroll
    for (int j = 0; j < IPL; ++j) tmax = max(tmax, e_in(j, l));
    unsigned int tot;
    const unsigned int ex = wave_excl_scan_u32<OpMaxU>(tmax, 0u, tot);
    // carry - lo + 1 clamped to [0, 2^32 - 1], in wave-uniform 32-bit halves
    const long long d = carry[l] - lo;
    const int dh = (int)(d >> 32);
    const unsigned int dl = (unsigned int)d;
    const unsigned int cr = dh < 0 ? 0u : (dh > 0 || dl == 0xFFFFFFFFu ? 0xFFFFFFFFu : dl + 1u);
    M[l] = max(ex, cr);
  }
  // per-lane measure per level; break counts packed in 10-bit fields (<= 512 each)
  unsigned int acc[NLEV];
  unsigned int nbrk = 0;
#pragma unroll
  for (int l = 0; l < NLEV; ++l) {
    unsigned int Mb = M[l], a = 0, c = 0;
#pragma unroll
    for (int j = 0; j < IPL; ++j) {
      const unsigned int s = s_in(j, l), e = e_in(j, l);
      const unsigned int b = max(s, Mb);
      a += max(e, b) - b;
      c += s > Mb ? 1u : 0u;
      Mb = max(Mb, e);
    }
    acc[l] = a;
    nbrk |= c << (10 * l);
  }
  if constexpr (IPL == 8) {
    // opaque to the compiler: it recomputes the per-level selections of each
    // phase instead of keeping them all live (which spills at 64 VGPRs)
#pragma unroll
    for (int j = 0; j < IPL; ++j) asm volatile("" : "+v"(kv[j]), "+v"(ev[j]));
  }
  unsigned int P[NLEV], totp[NLEV];
#pragma unroll
  for (int l = 0; l < NLEV; ++l) P[l] = wave_excl_scan_u32<OpSumU>(acc[l], 0u, totp[l]);
  unsigned int totr;
  const unsigned int Rp = wave_excl_scan_u32<OpSumU>(nbrk, 0u, totr);
  // components of one level at a time are staged in LDS (the sorted keys and
  // ends are in registers by now) and then written out in full 64-lane rows
  if constexpr (IPL == 8) {
    // opaque to the compiler: it recomputes the per-level selections of each
    // phase instead of keeping them all live (which spills at 64 VGPRs)
#pragma unroll
    for (int j = 0; j < IPL; ++j) asm volatile("" : "+v"(kv[j]), "+v"(ev[j]));
  }
  uint2* stage = (uint2*)W.key;  // key[] and end[]: kWaveCap entries of 8 B
  wave_sync();
#pragma unroll
  for (int l = 0; l < NLEV; ++l) {
    unsigned int r = (Rp >> (10 * l)) & 0x3FFu;
    unsigned int Ml = M[l], Pl = P[l];
#pragma unroll
    for (int j = 0; j < IPL; ++j) {
      const unsigned int s = s_in(j, l), e = e_in(j, l);
      const bool brk = s > Ml;
      if (brk) stage[r] = make_uint2(kv[j] >> 2, Pl);  // CompN {start - lo, measure before}
      r += brk ? 1u : 0u;
      const unsigned int b = max(s, Ml);
      Pl += max(e, b) - b;
      Ml = max(Ml, e);
    }
    wave_sync();
    const int nl = (int)((totr >> (10 * l)) & 0x3FFu);
    uint2* out = (uint2*)(p.compn[l] + off);
    // non-temporal, like the bucketed records: the components (1.2 GB on the
    // large trace) would otherwise sit dirty in L2 and be written back while
    // the next kernels stream their own data
    for (int i = lane; i < nl; i += 64) {
      const uint2 c = stage[i];
      put_rec8(out + i, c.x, c.y);
    }
    wave_sync();
  }
  if (lane < 3) {
    long long bs = 0;
#pragma unroll
    for (int l = 0; l < NLEV; ++l) {
      if (lane == l) {
        bs = (long long)totp[l];
        // ends clamped to lo + 2^32 - 2: the level's union also covers up to
        // its largest true end, beyond what earlier buckets already covered
        const long long from = max(carry[l], lo + 0xFFFFFFFEll);
        if (maxe[l] > from) bs += maxe[l] - from;
      }
    }
    p.bsum[gb * 3 + lane] = bs;
    p.ncomp[gb * 3 + lane] = (totr >> (10 * lane)) & 0x3FFu;
  }
}

// Records of the first rounds that the wave path loads before it knows the
// bucket's count (fixed slots only).
constexpr int kWavePre = 4;

// Sort of one bucket of 64*(IPL-1) < ni <= 64*IPL records into W, then its
// flatten: every round but the last is full, so only the last one tests for
// positions past the bucket. With fixed slots (kSlots) the first kWavePre
// rounds come loaded in `pre` (read before the count was known, so past the
// end of a bucket of fewer records: places its slots hold). Returns false
// (nothing written) when the bucket must take the block path.
template <int IPL, bool kSlots>
__device__ __forceinline__ bool wave_bucket(const Plan& p, WaveSmem& W, long long gb, long long off, int ni,
                                            const uint2* rec, const uint2 (&pre)[kWavePre], long long lo, int nlev,
                                            const long long (&carry)[3], const long long (&maxe)[3]) {
  const int lane = threadIdx.x & 63;
  // round r holds position lane + 64 r; rounds before the last are inside the bucket
  auto in_bucket = [&](int r) { return r < IPL - 1 || lane + 64 * r < ni; };
  unsigned int kr[IPL], er[IPL], rk[IPL];
  // every lane loads every round, from a position clamped into the bucket
  // (ni >= 1): the loads issue back to back instead of one masked block (and
  // one wait) each
  uint2 x[IPL];
#pragma unroll
  for (int r = 0; r < IPL; ++r) {
    if (kSlots && r < kWavePre) {
      x[r] = pre[r];
      continue;
    }
    // a 32-bit byte offset from the wave-uniform base (ni <= kWaveCap); the
    // last round clamps into the bucket, so it reads no lines past its end
    const unsigned int i = (unsigned int)(r < IPL - 1 ? lane + 64 * r : min(lane + 64 * r, ni - 1));
    x[r] = *(const uint2*)((const char*)rec + 8u * i);  // relative to lo: (start - lo) << 2 | slot, end - lo + 1
  }
  // a position past the bucket keeps the padding pair of the flatten: key 2
  // (rank 2, start lo), end 0; it is stored at its own index below
  unsigned int kor = 0;
#pragma unroll
  for (int r = 0; r < IPL; ++r) {
    const bool in = in_bucket(r);
    kr[r] = in ? x[r].x : 2u;
    er[r] = in ? x[r].y : 0u;
    kor |= kr[r];
  }
  kor >>= 2;
  kor = (unsigned int)wave_reduce_i32<OpOrI>((int)kor, 0);
  // sub-bins: about one per record (128 up to 128 records, 256 up to 256,
  // else 512: the round count fixes the range of ni); a lane owns 2*wpl of
  // them, two per LDS word
  constexpr int dbits = IPL <= 2 ? 7 : (IPL <= 4 ? 8 : 9);
  constexpr int nbins = 1 << dbits, wpl = nbins >> 7;
  unsigned int bw[wpl];
#pragma unroll
  for (int j = 0; j < wpl; ++j) bw[j] = 0;
  lds_store<wpl>(W.bins + lane * wpl, bw);
  wave_sync();
  const int hb = kor ? 32 - __clz((int)kor) : 0;
  const int ksh = 2 + (hb > dbits ? hb - dbits : 0);  // sub-bin = key >> ksh (ksh <= 25)
  // the atomics of all rounds are issued with no branch, so they overlap
  // instead of waiting one by one; a position past the bucket adds 0 to a
  // word of its own (word `lane`: there are at least 64), so lanes past the
  // bucket never pile onto one address
  // (sub-bin d = key >> ksh counts in half d & 1 of word d >> 1)
#pragma unroll
  for (int r = 0; r < IPL; ++r) {
    const bool in = in_bucket(r);
    const unsigned int w = in ? kr[r] >> (ksh + 1) : (unsigned int)lane;
    const unsigned int sh = in ? ((kr[r] >> ksh) & 1u) << 4 : 0u;
    rk[r] = __builtin_amdgcn_ubfe(atomicAdd(&W.bins[w], in ? 1u << sh : 0u), sh, 16);
  }
  wave_sync();
  // exclusive scan of the sub-bin counters (lane order = sub-bin order)
  lds_load<wpl>(W.bins + lane * wpl, bw);
  unsigned int tot = 0;
#pragma unroll
  for (int j = 0; j < wpl; ++j) tot += (bw[j] & 0xFFFFu) + (bw[j] >> 16);
  unsigned int all;
  unsigned int run = wave_excl_scan_u32<OpSumU>(tot, 0u, all);
#pragma unroll
  for (int j = 0; j < wpl; ++j) {
    const unsigned int a = run, b = run + (bw[j] & 0xFFFFu);
    run = b + (bw[j] >> 16);
    bw[j] = a | (b << 16);
  }
  lds_store<wpl>(W.bins + lane * wpl, bw);
  wave_sync();
  unsigned int fix = 0;  // bit r: the record of round r is the second one of its sub-bin
  constexpr int G = IPL < 4 ? IPL : 4;  // rounds placed together (bounds the live registers)
#pragma unroll
  for (int r0 = 0; r0 < IPL; r0 += G) {
    unsigned int pos[G];
#pragma unroll
    for (int u = 0; u < G; ++u) {  // the reads of a group first (past the bucket: word `lane`)
      if (r0 + u >= IPL) break;  // a last group shorter than G
      const bool in = in_bucket(r0 + u);
      const unsigned int w = in ? kr[r0 + u] >> (ksh + 1) : (unsigned int)lane;
      const unsigned int sh = in ? ((kr[r0 + u] >> ksh) & 1u) << 4 : 0u;
      pos[u] = __builtin_amdgcn_ubfe(W.bins[w], sh, 16) + rk[r0 + u];
    }
#pragma unroll
    for (int u = 0; u < G; ++u) {
      // a position past the bucket stores to its own index (>= ni): never
      // read as a record, and no branch around the stores (distinct addresses)
      const int r = r0 + u;
      if (r >= IPL) break;
      const bool in = in_bucket(r);
      const unsigned int q = in ? pos[u] : (unsigned int)(lane + 64 * r);
      W.key[q] = kr[r];
      W.end[q] = er[r];
      fix |= (in && rk[r] == 1) ? 1u << r : 0u;
    }
  }
  wave_sync();
  // order inside each sub-bin by the full key, where it holds two or more
  // records: an insertion sort per such sub-bin (c > 32 records: block path)
  bool crowded = false;
  auto fix_sub_bin = [&](unsigned int d) {
    const int st0 = (int)((W.bins[d >> 1] >> (16u * (d & 1u))) & 0xFFFFu);
    const int st1 = (int)d + 1 < nbins ? (int)((W.bins[(d + 1) >> 1] >> (16u * ((d + 1) & 1u))) & 0xFFFFu) : ni;
    const int c = st1 - st0;
    if (c > 32) {
      crowded = true;
      return;
    }
    unsigned int* ko = W.key + st0;
    unsigned int* eo = W.end + st0;
    for (int a = 1; a < c; ++a) {
      const unsigned int kx = ko[a], ex = eo[a];
      int b = a - 1;
      while (b >= 0 && ko[b] > kx) {
        ko[b + 1] = ko[b];
        eo[b + 1] = eo[b];
        --b;
      }
      ko[b + 1] = kx;
      eo[b + 1] = ex;
    }
  };
  if (ksh > 2) {
    // the sub-bins to fix (each named by the lane that placed its second
    // record) are listed in the key array past the bucket's records, so the
    // work spreads evenly over the lanes: ceil(fixes / 64) rounds instead of
    // the largest number of fixes of one lane
    unsigned int nfix;
    const unsigned int fb = wave_excl_scan_u32<OpSumU>((unsigned int)__popc(fix), 0u, nfix);
    if (nfix <= 2u * (unsigned int)(kWaveCap - ni)) {  // 16-bit entries in the free words
      unsigned short* list = (unsigned short*)(W.key + ni);
      unsigned int q = fb;
#pragma unroll
      for (int r = 0; r < IPL; ++r) {
        if (fix & (1u << r)) list[q++] = (unsigned short)(kr[r] >> ksh);
      }
      wave_sync();
      for (unsigned int i = (unsigned int)lane; i < nfix; i += 64) fix_sub_bin(list[i]);
      wave_sync();
      // the list's words back to the padding key
      for (unsigned int i = (unsigned int)lane; 2 * i < nfix; i += 64) W.key[ni + i] = 2u;
    } else {
      // no room: each lane walks its own such records
      unsigned int todo = fix;
      while (todo) {
        const int rr = __builtin_ctz(todo);
        todo &= todo - 1u;
        unsigned int kk = kr[0];
#pragma unroll
        for (int j = 1; j < IPL; ++j) kk = rr == j ? kr[j] : kk;  // kr[rr] without indexing registers
        fix_sub_bin(kk >> ksh);
      }
    }
  }
  if (__ballot(crowded)) return false;
  wave_sync();
  if (nlev == 2) wave_flatten<IPL, 2>(p, W, gb, off, ni, lo, carry, maxe);
  else wave_flatten<IPL, 3>(p, W, gb, off, ni, lo, carry, maxe);
  return true;
}

// One wave per bucket, 8 waves per SIMD (64 VGPRs). Buckets that need the
// block path go to its queue. kSlots: fixed slots of at least 128 records
// (2 slot_cap record places per bucket, whatever its count).
template <bool kSlots>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(8, 8))) void k_merge_wave(Plan p) {
  __shared__ WaveSmem wsm[4];
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);  // everything per bucket is wave-uniform
  const long long gb = (long long)blockIdx.x * 4 + wave;
  if (gb >= p.n_buckets) return;
  WaveSmem& W = wsm[wave];
  uint2 pre[kWavePre];
  if constexpr (kSlots) {
    // the first rounds load while the bucket's count is still on its way:
    // its slots start at a known place and hold 2 slot_cap >= 256 records
    const uint2* base = (const uint2*)p.elems + 2 * gb * (long long)p.slot_cap;
#pragma unroll
    for (int r = 0; r < kWavePre; ++r) pre[r] = base[lane + 64 * r];
  }
  // every per-bucket word is read here, before any of them is used, so the
  // reads travel together (only the segment's words wait for its index)
  BucketRecs br;
  if constexpr (kSlots) {
    // fixed slots (slot_cap > 0): the places need no other word
    const unsigned long long cu = p.cursor[gb];
    br.n8 = (int)(unsigned int)cu;
    br.n16 = (int)(cu >> 32);
    br.overflow = (long long)br.n8 + br.n16 > (long long)p.slot_cap;
    br.narrow = (const uint2*)p.elems + 2 * gb * (long long)p.slot_cap;
    br.wide = nullptr;  // never read here: such buckets take the block path
  } else {
    br = bucket_recs(p, gb);
  }
  const long long off = (long long)p.offsets[gb];
  const long long carry[3] = {p.carry[gb * 3], p.carry[gb * 3 + 1], p.carry[gb * 3 + 2]};
  const unsigned long long mx[3] = {p.maxend[gb * 3], p.maxend[gb * 3 + 1], p.maxend[gb * 3 + 2]};
  const int seg = p.bucket_seg[gb];
  const SegDesc sd = p.segs[seg];
  const Geom g = seg_geom(p, seg);
  const long long n = (long long)br.n8 + br.n16;
  // largest end per level of the bucket's own records (0: none)
  long long maxe[3];
  maxe[0] = (long long)mx[0];
  maxe[1] = max(maxe[0], (long long)mx[1]);
  maxe[2] = max(maxe[1], (long long)mx[2]);
  if (n == 0 || br.overflow) {
    // empty, or a slot overflow that makes the host redo the build
    // a use of the early loads on this path too, so that the compiler issues
    // them before the count's test instead of moving them below it
    if constexpr (kSlots) asm volatile("" ::"v"(pre[0].x), "v"(pre[1].x), "v"(pre[2].x), "v"(pre[3].x));
    asm volatile("" ::"s"(off), "s"(carry[0]), "s"(carry[1]), "s"(carry[2]), "s"(mx[0]), "s"(mx[1]), "s"(mx[2]),
                 "s"(sd.bucket_begin), "s"(sd.n_levels), "s"(g.min_s), "s"(g.wx), "s"(g.s0));
    if (lane < 3) {
      p.bsum[gb * 3 + lane] = 0;
      p.ncomp[gb * 3 + lane] = 0;
    }
    return;
  }
  bool done = false;
  if (br.n16 == 0 && n <= kWaveCap) {
    // only 8 B records (so the segment is narrow: buckets at most 2^30 ns wide)
    const int ni = (int)n;
    const uint2* rec = br.narrow;
    const long long lo = bucket_lo(g, gb - sd.bucket_begin);
    const int nlev = sd.n_levels;
    // as many records per lane as the bucket needs: every slot costs the
    // same instructions, filled or not
    if (ni <= 64) done = wave_bucket<1, kSlots>(p, W, gb, off, ni, rec, pre, lo, nlev, carry, maxe);
    else if (ni <= 128) done = wave_bucket<2, kSlots>(p, W, gb, off, ni, rec, pre, lo, nlev, carry, maxe);
    else if (ni <= 192) done = wave_bucket<3, kSlots>(p, W, gb, off, ni, rec, pre, lo, nlev, carry, maxe);
    else if (ni <= 256) done = wave_bucket<4, kSlots>(p, W, gb, off, ni, rec, pre, lo, nlev, carry, maxe);
    else if (ni <= 320) done = wave_bucket<5, kSlots>(p, W, gb, off, ni, rec, pre, lo, nlev, carry, maxe);
    else if (ni <= 384) done = wave_bucket<6, kSlots>(p, W, gb, off, ni, rec, pre, lo, nlev, carry, maxe);
    else if (ni <= 448) done = wave_bucket<7, kSlots>(p, W, gb, off, ni, rec, pre, lo, nlev, carry, maxe);
    else done = wave_bucket<8, kSlots>(p, W, gb, off, ni, rec, pre, lo, nlev, carry, maxe);
  }
  if (!done && lane == 0) p.queue[atomicAdd(&p.ticket[2], 1u)] = (unsigned int)gb;
}

// ----------------------------------------------------------------------------
// region: clip every resource by binary search, reduce, finalize in FP64
// ----------------------------------------------------------------------------

// Measure of level l of segment seg before time t.
__device__ long long measure_before(const Plan& p, int seg, int l, long long t) {
  const SegDesc sd = p.segs[seg];
  const Geom g = seg_geom(p, seg);
  if (g.empty || t <= g.min_s) return 0;
  if (t >= (long long)p.stats[seg].max_e) return p.seg_total[seg * 3 + l];
  const long long gb = sd.bucket_begin + bucket_index(g, (unsigned long long)(t - g.min_s));
  const long long carry = p.carry[gb * 3 + l];
  const long long base = p.base[gb * 3 + l];
  const long long bs = p.bsum[gb * 3 + l];
  const long long cnt = p.ncomp[gb * 3 + l];
  const CompView c = comp_view(p, g, sd.bucket_begin, gb, l);
  // first component with start >= t
  long long lo = 0, hi = cnt;
  while (lo < hi) {
    const long long mid = (lo + hi) >> 1;
    if (c.cs(mid) < t) lo = mid + 1; else hi = mid;
  }
  const long long k = lo - 1;
  if (k < 0) {
    // only the component carried in from earlier buckets lies before t
    const long long ext = carry + (cnt > 0 ? c.pl(0) : bs);
    return base + (ext < t ? ext : t) - carry;
  }
  const long long cs = c.cs(k), pl = c.pl(k);
  const long long next_pl = k + 1 < cnt ? c.pl(k + 1) : bs;
  const long long ce = cs + (next_pl - pl);
  return base + pl + (ce < t ? ce : t) - cs;
}

// Region, part 1: one thread per (resource, level, end of the region) clips by
// binary search; a slice of kRegionSlice resources of one region per
// workgroup writes their state times and adds its sums and maxima to the
// region's accumulator (exact integer atomics: the order does not matter).
constexpr int kRegionSlice = 32;

template <int THREADS>
__global__ __launch_bounds__(THREADS) void k_region_part(Plan p, const RegionDesc* regions, long long* times) {
  static_assert(THREADS == 8 * kRegionSlice, "8 threads per resource");
  __shared__ long long sM[kRegionSlice][4][2];
  __shared__ long long lds[THREADS / 64 * 10];
  const RegionDesc rd = regions[blockIdx.x];
  const int R = rd.n_hosts + rd.n_devices;
  const int r0 = blockIdx.y * kRegionSlice;
  if (r0 >= R || rd.n_ivl) return;  // uniform: past the region's resources, or a per-resource region
  const int rl = threadIdx.x >> 3, l = (threadIdx.x >> 1) & 3, ep = threadIdx.x & 1;
  const int r = r0 + rl;
  const bool host = r < rd.n_hosts;
  if (r < R && l < (host ? 3 : 2)) sM[rl][l][ep] = measure_before(p, rd.seg_begin + r, l, ep ? rd.t1 : rd.t0);
  __syncthreads();
  const long long E = rd.t1 - rd.t0;
  // sums: U, W, MPI, Other, K, M ; maxes: U+W, K, K+M
  long long v[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
  if ((threadIdx.x & 7) == 0 && r < R) {
    long long D[3] = {0, 0, 0};
    for (int k = 0; k < (host ? 3 : 2); ++k) D[k] = sM[rl][k][1] - sM[rl][k][0];
    long long* out = times + (rd.times_off + r) * 4;
    if (host) {
      const long long u = D[0], w = D[1] - D[0], mpi = D[2] - D[1], o = E - D[2];
      out[0] = u; out[1] = w; out[2] = mpi; out[3] = o;
      v[0] = u; v[1] = w; v[2] = mpi; v[3] = o;
      v[6] = u + w;
    } else {
      const long long k = D[0], mm = D[1] - D[0], idle = E - D[1];
      out[0] = k; out[1] = mm; out[2] = idle; out[3] = 0;
      v[4] = k; v[5] = mm;
      v[7] = k;
      v[8] = k + mm;
    }
  }
  block_tree<THREADS>(v, lds);
  if (threadIdx.x == 0) {
    unsigned long long* acc = p.racc + (long long)blockIdx.x * 9;
#pragma unroll
    for (int i = 0; i < 6; ++i)
      if (v[i]) atomicAdd(acc + i, (unsigned long long)v[i]);
#pragma unroll
    for (int i = 6; i < 9; ++i)
      if (v[i]) atomicMax(acc + i, (unsigned long long)v[i]);
  }
}

// Region, part 2: one thread per region turns the accumulator into the tree
// (FP64 ratios) and clears it for the next launch.
__global__ __launch_bounds__(64) void k_region_final(Plan p, const RegionDesc* regions, int n_regions, Tree* trees) {
  const int g = blockIdx.x * 64 + threadIdx.x;
  if (g >= n_regions) return;
  const RegionDesc rd = regions[g];
  if (rd.n_ivl) return;  // a per-resource region: k_region_multi
  unsigned long long* acc = p.racc + (long long)g * 9;
  long long v[9];
#pragma unroll
  for (int i = 0; i < 9; ++i) {
    v[i] = (long long)acc[i];
    acc[i] = 0;
  }
  trees[g] = make_tree(rd.t1 - rd.t0, rd.n_hosts, rd.n_devices, v);
}

// Regions given as per-resource interval lists (a region entered repeatedly,
// each resource on its own clock). Part 1 clears the accumulators of their
// resources; part 2 adds, per (interval, level, end of the interval), the
// level's measure before that end (the start with a minus sign) and each
// interval's length; part 3 turns them into state times (the remainder
// completes the resource's own time in the region) and the tree, with E the
// largest host in-region time (eq. 1), or the largest device one when no host
// process is in the region.
__global__ __launch_bounds__(256) void k_ivl_zero(const RegionDesc* regions, long long* macc) {
  const RegionDesc rd = regions[blockIdx.x];
  if (rd.n_ivl == 0) return;
  const int R = rd.n_hosts + rd.n_devices;
  for (int i = threadIdx.x; i < 4 * R; i += 256) macc[rd.times_off * 4 + i] = 0;
}

__global__ __launch_bounds__(256) void k_ivl_acc(Plan p, const RegionDesc* regions, const IvlDesc* ivls,
                                                 long long n_ivls, long long* macc) {
  const long long t = (long long)blockIdx.x * 256 + threadIdx.x;
  const long long i = t >> 3;
  if (i >= n_ivls) return;
  const int l = (int)((t >> 1) & 3), ep = (int)(t & 1);
  const IvlDesc iv = ivls[i];
  const RegionDesc rd = regions[iv.region];
  unsigned long long* acc = (unsigned long long*)(macc + (rd.times_off + iv.resource) * 4);
  if (l == 3) {
    if (ep) atomicAdd(acc + 3, (unsigned long long)(iv.b - iv.a));
    return;
  }
  if (l >= (iv.resource < rd.n_hosts ? 3 : 2)) return;
  const long long v = measure_before(p, rd.seg_begin + iv.resource, l, ep ? iv.b : iv.a);
  atomicAdd(acc + l, (unsigned long long)(ep ? v : -v));  // two's complement: the sum is exact
}

template <int THREADS>
__global__ __launch_bounds__(THREADS) void k_region_multi(const RegionDesc* regions, const long long* macc, Tree* trees,
                                                          long long* times) {
  __shared__ long long lds[THREADS / 64 * 10];
  __shared__ long long semax[2][THREADS / 64];
  const RegionDesc rd = regions[blockIdx.x];
  if (rd.n_ivl == 0) return;
  const int R = rd.n_hosts + rd.n_devices;
  // sums: U, W, MPI, Other, K, M ; maxes: U+W, K, K+M
  long long v[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
  long long eh = 0, ed = 0;
  for (int r = threadIdx.x; r < R; r += THREADS) {
    const long long* a = macc + (rd.times_off + r) * 4;
    const long long D0 = a[0], D1 = a[1], D2 = a[2], Er = a[3];
    long long* out = times + (rd.times_off + r) * 4;
    if (r < rd.n_hosts) {
      const long long u = D0, w = D1 - D0, mpi = D2 - D1, o = Er - D2;
      out[0] = u; out[1] = w; out[2] = mpi; out[3] = o;
      v[0] += u; v[1] += w; v[2] += mpi; v[3] += o;
      v[6] = u + w > v[6] ? u + w : v[6];
      eh = Er > eh ? Er : eh;
    } else {
      const long long k = D0, mm = D1 - D0, idle = Er - D1;
      out[0] = k; out[1] = mm; out[2] = idle; out[3] = 0;
      v[4] += k; v[5] += mm;
      v[7] = k > v[7] ? k : v[7];
      v[8] = k + mm > v[8] ? k + mm : v[8];
      ed = Er > ed ? Er : ed;
    }
  }
  eh = wave_reduce_i64<OpMax>(eh, 0);
  ed = wave_reduce_i64<OpMax>(ed, 0);
  if ((threadIdx.x & 63) == 0) {
    semax[0][threadIdx.x >> 6] = eh;
    semax[1][threadIdx.x >> 6] = ed;
  }
  block_tree<THREADS>(v, lds);  // its barriers also publish semax
  if (threadIdx.x == 0) {
    for (int w = 0; w < THREADS / 64; ++w) {
      eh = semax[0][w] > eh ? semax[0][w] : eh;
      ed = semax[1][w] > ed ? semax[1][w] : ed;
    }
    trees[blockIdx.x] = make_tree(eh ? eh : ed, rd.n_hosts, rd.n_devices, v);
  }
}

// ----------------------------------------------------------------------------
// launchers
// ----------------------------------------------------------------------------

hipError_t launch_reset(const Plan& p, hipStream_t st) {
  const long long work = max(3 * p.n_buckets + p.n_segs, p.n_tiles) + 64;
  int blocks = (int)min(2048ll, (work + 255) / 256);
  hipLaunchKernelGGL(k_reset, dim3(blocks), dim3(256), 0, st, p);
  return hipGetLastError();
}

hipError_t launch_stats(const Plan& p, hipStream_t st) {
  // the tiles of single chunks, then (in the same launch) the shared tiles
  const long long own = p.n_own_tiles, sh = p.n_tiles - p.n_own_tiles;
  if (p.tile_elems <= 512) {
    const unsigned blocks = (unsigned)((own + 3) / 4 + sh);
    if (sh > 0) hipLaunchKernelGGL(k_stats_small<true>, dim3(blocks), dim3(256), 0, st, p);
    else if (own > 0) hipLaunchKernelGGL(k_stats_small<false>, dim3(blocks), dim3(256), 0, st, p);
  } else if (sh > 0) {
    hipLaunchKernelGGL((k_stats<256, true>), dim3((unsigned)p.n_tiles), dim3(256), 0, st, p);
  } else if (own > 0) {
    hipLaunchKernelGGL((k_stats<256, false>), dim3((unsigned)p.n_tiles), dim3(256), 0, st, p);
  }
  if (p.n_segs > 0) hipLaunchKernelGGL(k_geom, dim3((unsigned)((p.n_segs + 255) / 256)), dim3(256), 0, st, p);
  return hipGetLastError();
}

// Count and scatter launches: one block per tile, the shared tiles (if any)
// after the others; plans share tiles only at 512 and 2048 records per tile.
hipError_t launch_hist(const Plan& p, hipStream_t st) {
  if (p.n_tiles == 0) return hipSuccess;
  const dim3 grid((unsigned)p.n_tiles);
  if (p.n_tiles > p.n_own_tiles) {
    switch (p.tile_elems) {
      case 512: hipLaunchKernelGGL((k_hist<128, 4, true>), grid, dim3(128), 0, st, p); break;
      case 2048: hipLaunchKernelGGL((k_hist<512, 4, true>), grid, dim3(512), 0, st, p); break;
      default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
  }
  switch (p.tile_elems) {
    case 512: hipLaunchKernelGGL((k_hist<128, 4, false>), grid, dim3(128), 0, st, p); break;
    case 2048: hipLaunchKernelGGL((k_hist<512, 4, false>), grid, dim3(512), 0, st, p); break;
    case 8192: hipLaunchKernelGGL((k_hist<1024, 8, false>), grid, dim3(1024), 0, st, p); break;
    default: hipLaunchKernelGGL((k_hist<512, 8, false>), grid, dim3(512), 0, st, p); break;
  }
  return hipGetLastError();
}

hipError_t launch_scan(const Plan& p, hipStream_t st) {
  const long long blocks = (p.n_buckets + kScanTile - 1) / kScanTile;
  if (blocks == 0) return hipSuccess;
  hipLaunchKernelGGL(k_scan<256>, dim3((unsigned)blocks), dim3(256), 0, st, p);
  return hipGetLastError();
}

hipError_t launch_scatter(const Plan& p, hipStream_t st) {
  if (p.n_tiles == 0) return hipSuccess;
  const dim3 grid((unsigned)p.n_tiles);
  if (p.n_tiles > p.n_own_tiles) {
    switch (p.tile_elems) {
      case 512: hipLaunchKernelGGL((k_scatter<128, 4, true>), grid, dim3(128), 0, st, p); break;
      case 2048: hipLaunchKernelGGL((k_scatter<512, 4, true>), grid, dim3(512), 0, st, p); break;
      default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
  }
  switch (p.tile_elems) {
    case 512: hipLaunchKernelGGL((k_scatter<128, 4, false>), grid, dim3(128), 0, st, p); break;
    case 2048: hipLaunchKernelGGL((k_scatter<512, 4, false>), grid, dim3(512), 0, st, p); break;
    case 8192: hipLaunchKernelGGL((k_scatter<1024, 8, false>), grid, dim3(1024), 0, st, p); break;
    default: hipLaunchKernelGGL((k_scatter<512, 8, false>), grid, dim3(512), 0, st, p); break;
  }
  return hipGetLastError();
}

hipError_t launch_carry(const Plan& p, hipStream_t st) {
  if (p.n_segs == 0) return hipSuccess;
  if (p.seg_group > 1)
    hipLaunchKernelGGL(k_carry_grouped<64>, dim3((unsigned)((p.n_segs + kSegGroup - 1) / kSegGroup)), dim3(64), 0, st, p);
  else
    hipLaunchKernelGGL(k_carry<64>, dim3((unsigned)p.n_segs), dim3(64), 0, st, p);  // a wave per segment, spread over the CUs
  return hipGetLastError();
}

hipError_t launch_scan_carry(const Plan& p, hipStream_t st) {
  const long long scan_blocks = (p.n_buckets + kScanTile - 1) / kScanTile;
  const long long waves = p.seg_group > 1 ? (p.n_segs + kSegGroup - 1) / kSegGroup : p.n_segs;
  const long long blocks = scan_blocks + (waves + 3) / 4;
  if (blocks == 0) return hipSuccess;
  if (p.seg_group > 1)
    hipLaunchKernelGGL(k_scan_carry<true>, dim3((unsigned)blocks), dim3(256), 0, st, p, (int)scan_blocks);
  else
    hipLaunchKernelGGL(k_scan_carry<false>, dim3((unsigned)blocks), dim3(256), 0, st, p, (int)scan_blocks);
  return hipGetLastError();
}

hipError_t launch_merge_wave(const Plan& p, hipStream_t st) {
  if (p.n_buckets == 0) return hipSuccess;
  const dim3 grid((unsigned)((p.n_buckets + 3) / 4));
  if (p.slot_cap >= 128)
    hipLaunchKernelGGL(k_merge_wave<true>, grid, dim3(256), 0, st, p);
  else
    hipLaunchKernelGGL(k_merge_wave<false>, grid, dim3(256), 0, st, p);
  return hipGetLastError();
}

hipError_t launch_merge_block(const Plan& p, int cap, hipStream_t st) {
  if (p.n_buckets == 0) return hipSuccess;
  // persistent workgroups for the buckets the wave path handed over
  const unsigned grid = (unsigned)std::min<long long>(p.n_buckets, 1024);
  if (cap == 2048)
    hipLaunchKernelGGL((k_merge_block<256, 2048>), dim3(grid), dim3(256), 0, st, p);
  else
    hipLaunchKernelGGL((k_merge_block<256, 4096>), dim3(grid), dim3(256), 0, st, p);
  return hipGetLastError();
}

hipError_t launch_base(const Plan& p, hipStream_t st) {
  if (p.n_segs == 0) return hipSuccess;
  if (p.seg_group > 1)
    hipLaunchKernelGGL(k_base_grouped<64>, dim3((unsigned)((p.n_segs + kSegGroup - 1) / kSegGroup)), dim3(64), 0, st, p);
  else
    hipLaunchKernelGGL(k_base<64>, dim3((unsigned)p.n_segs), dim3(64), 0, st, p);  // a wave per segment, spread over the CUs
  return hipGetLastError();
}

hipError_t launch_region(const Plan& p, const RegionDesc* regions, int n_regions, int max_res, Tree* trees,
                         long long* times, const IvlDesc* ivls, long long n_ivls, long long* macc, hipStream_t st) {
  if (n_regions == 0) return hipSuccess;
  const unsigned slices = (unsigned)std::max(1, (max_res + kRegionSlice - 1) / kRegionSlice);
  hipLaunchKernelGGL(k_region_part<8 * kRegionSlice>, dim3((unsigned)n_regions, slices), dim3(8 * kRegionSlice), 0, st,
                     p, regions, times);
  hipLaunchKernelGGL(k_region_final, dim3((unsigned)((n_regions + 63) / 64)), dim3(64), 0, st, p, regions, n_regions,
                     trees);
  if (n_ivls > 0) {
    hipLaunchKernelGGL(k_ivl_zero, dim3((unsigned)n_regions), dim3(256), 0, st, regions, macc);
    hipLaunchKernelGGL(k_ivl_acc, dim3((unsigned)((8 * n_ivls + 255) / 256)), dim3(256), 0, st, p, regions, ivls,
                       n_ivls, macc);
    hipLaunchKernelGGL(k_region_multi<256>, dim3((unsigned)n_regions), dim3(256), 0, st, regions,
                       (const long long*)macc, trees, times);
  }
  return hipGetLastError();
}

}  // namespace hpop
