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
}

// ----------------------------------------------------------------------------
// stats: validate records, per-segment min/max start and max end
// ----------------------------------------------------------------------------

template <int THREADS>
__global__ __launch_bounds__(THREADS) void k_stats(Plan p) {
  // The bucket grid needs only the range of starts; validation happens in the
  // scatter, which reads both ends anyway. Starts outside [0, 2^62) belong to
  // invalid records and are left out of the range.
  constexpr int NW = THREADS / 64;
  __shared__ int s_chunk;
  __shared__ unsigned long long red[2][NW];
  const long long tile = blockIdx.x;
  if (threadIdx.x == 0) s_chunk = upper_index_chunk(p.chunks, p.n_chunks, tile);
  __syncthreads();
  const ChunkDesc cd = p.chunks[s_chunk];
  const long long base = (tile - cd.tile_begin) * (long long)p.tile_elems;
  const long long end = min((long long)cd.count, base + p.tile_elems);
  unsigned long long mn = ULLONG_MAX, mxs = 0;
  for (long long i = base + threadIdx.x; i < end; i += THREADS) {
    const unsigned long long s = (unsigned long long)cd.s[i];
    if (s < (unsigned long long)kTimeLimit) {
      mn = s < mn ? s : mn;
      mxs = s > mxs ? s : mxs;
    }
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

// ----------------------------------------------------------------------------
// hist / scatter: regroup records by time bucket
// ----------------------------------------------------------------------------

// Buckets of one tile usually span a narrow window (records arrive roughly in
// time order), so per-tile counting uses an LDS window [bmin, bmin + kHistWin).
// Wider tiles fall back to global atomics per record.

template <int THREADS, int IPT>
__global__ __launch_bounds__(THREADS) void k_hist(Plan p) {
  constexpr int NW = THREADS / 64;
  __shared__ int s_chunk;
  __shared__ int s_rng[2][NW];
  __shared__ unsigned int hist[kHistWin];
  const long long tile = blockIdx.x;
  if (threadIdx.x == 0) s_chunk = upper_index_chunk(p.chunks, p.n_chunks, tile);
  __syncthreads();
  const ChunkDesc cd = p.chunks[s_chunk];
  const SegDesc sd = p.segs[cd.seg];
  const Geom g = seg_geom(p.stats[cd.seg], sd);
  const long long base = (tile - cd.tile_begin) * (long long)p.tile_elems;
  const long long end = min((long long)cd.count, base + p.tile_elems);
  int bk[IPT];
  int bmin = INT_MAX, bmax = -1;
#pragma unroll
  for (int k = 0; k < IPT; ++k) {
    const long long i = base + threadIdx.x + (long long)k * THREADS;
    bk[k] = -1;
    if (i < end) {
      const long long s = cd.s[i], e = cd.e[i];
      if (rec_valid(s, e) && s < e) {
        bk[k] = bucket_of(s, g);
        bmin = min(bmin, bk[k]);
        bmax = max(bmax, bk[k]);
      }
    }
  }
  for (int d = 32; d >= 1; d >>= 1) {
    bmin = min(bmin, __shfl_xor(bmin, d, 64));
    bmax = max(bmax, __shfl_xor(bmax, d, 64));
  }
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (lane == 0) { s_rng[0][wave] = bmin; s_rng[1][wave] = bmax; }
  for (int i = threadIdx.x; i < kHistWin; i += THREADS) hist[i] = 0;
  __syncthreads();
  bmin = INT_MAX; bmax = -1;
  for (int w = 0; w < NW; ++w) { bmin = min(bmin, s_rng[0][w]); bmax = max(bmax, s_rng[1][w]); }
  if (bmax < 0) return;  // uniform: no valid record in this tile
  const bool windowed = bmax - bmin < kHistWin;
  if (windowed) {
#pragma unroll
    for (int k = 0; k < IPT; ++k) {
      // one LDS atomic per distinct bucket of the wave, not one per record
      unsigned long long todo = __ballot(bk[k] >= 0);
      while (todo) {
        const int leader = __ffsll((long long)todo) - 1;
        const int lb = __shfl(bk[k], leader, 64);
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

// exclusive scan of bucket counts -> offsets and cursors (decoupled look-back)
template <int THREADS>
__global__ __launch_bounds__(THREADS) void k_scan(Plan p) {
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
        c[k] = (unsigned int)(cu < (unsigned long long)p.slot_cap ? cu : (unsigned long long)p.slot_cap);
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
      p.offsets[b0 + k] = run;
      if (!slots) p.cursor[b0 + k] = run;
      if (c[k] > (unsigned)p.cap) atomicAdd(p.oversized, 1ull);
    }
    run += c[k];
  }
  // the thread holding the last bucket also writes the grand total
  if (b0 < p.n_buckets && p.n_buckets <= b0 + IPT) p.offsets[p.n_buckets] = run;
}

template <int THREADS, int IPT>
__global__ __launch_bounds__(THREADS) void k_scatter(Plan p) {
  constexpr int NW = THREADS / 64;
  __shared__ int s_chunk;
  __shared__ int s_rng[2][NW];
  __shared__ unsigned int hist[kHistWin];
  __shared__ unsigned long long bbase[kHistWin];
  __shared__ unsigned long long bmaxe[kHistWin];
  const long long tile = blockIdx.x;
  if (threadIdx.x == 0) s_chunk = upper_index_chunk(p.chunks, p.n_chunks, tile);
  __syncthreads();
  const ChunkDesc cd = p.chunks[s_chunk];
  const SegDesc sd = p.segs[cd.seg];
  const Geom g = seg_geom(p.stats[cd.seg], sd);
  const long long base = (tile - cd.tile_begin) * (long long)p.tile_elems;
  const long long end = min((long long)cd.count, base + p.tile_elems);
  int bk[IPT];
  long long sv[IPT], ev[IPT];
  int bmin = INT_MAX, bmax = -1;
#pragma unroll
  for (int k = 0; k < IPT; ++k) {
    const long long i = base + threadIdx.x + (long long)k * THREADS;
    bk[k] = -1;
    sv[k] = 0;
    ev[k] = 0;
    if (i < end) {
      sv[k] = cd.s[i];
      ev[k] = cd.e[i];
      if (!rec_valid(sv[k], ev[k])) {
        // first bad record of the build: chunk << 40 | index (rare path)
        atomicMin(p.err, ((unsigned long long)cd.chunk_id << 40) | (unsigned long long)i);
        p.owner_err[cd.owner] = 1u;
      } else if (sv[k] < ev[k]) {
        bk[k] = bucket_of(sv[k], g);
        bmin = min(bmin, bk[k]);
        bmax = max(bmax, bk[k]);
      }
    }
  }
  for (int d = 32; d >= 1; d >>= 1) {
    bmin = min(bmin, __shfl_xor(bmin, d, 64));
    bmax = max(bmax, __shfl_xor(bmax, d, 64));
  }
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const long long scap = p.slot_cap;
  if (lane == 0) { s_rng[0][wave] = bmin; s_rng[1][wave] = bmax; }
  for (int i = threadIdx.x; i < kHistWin; i += THREADS) { hist[i] = 0; bmaxe[i] = 0; }
  __syncthreads();
  bmin = INT_MAX; bmax = -1;
  for (int w = 0; w < NW; ++w) { bmin = min(bmin, s_rng[0][w]); bmax = max(bmax, s_rng[1][w]); }
  if (bmax < 0) return;
  const unsigned long long slotbits = (unsigned long long)cd.slot << kSlotShift;
  unsigned long long* gmax = p.maxend;
  if (bmax - bmin < kHistWin) {
    unsigned int rk[IPT];
    const unsigned long long lt = (1ull << lane) - 1ull;
#pragma unroll
    for (int k = 0; k < IPT; ++k) {
      // lanes of one bucket share one LDS atomic: the leader reserves their
      // ranks and folds their largest end in
      rk[k] = 0;
      unsigned long long todo = __ballot(bk[k] >= 0);
      while (todo) {
        const int leader = __ffsll((long long)todo) - 1;
        const int lb = __shfl(bk[k], leader, 64);
        const bool in = bk[k] == lb;
        const unsigned long long m = __ballot(in);
        const unsigned long long emax = wave_red_maxu(in ? (unsigned long long)ev[k] : 0ull);
        unsigned int b = 0;
        if (lane == leader) {
          b = atomicAdd(&hist[lb - bmin], (unsigned int)__popcll(m));
          atomicMax(&bmaxe[lb - bmin], emax);
        }
        b = __shfl(b, leader, 64);
        if (in) rk[k] = b + (unsigned int)__popcll(m & lt);
        todo &= ~m;
      }
    }
    __syncthreads();
    for (int i = threadIdx.x; i <= bmax - bmin; i += THREADS) {
      if (hist[i]) {
        const long long gb = sd.bucket_begin + bmin + i;
        bbase[i] = atomicAdd(&p.cursor[gb], (unsigned long long)hist[i]);
        atomicMax(&gmax[gb * 3 + cd.slot], bmaxe[i]);
      }
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < IPT; ++k) {
      if (bk[k] >= 0) {
        const long long pos = (long long)(bbase[bk[k] - bmin] + rk[k]);
        Elem el;
        el.s = sv[k];
        el.e_slot = (long long)((unsigned long long)ev[k] | slotbits);
        if (scap == 0) {
          p.elems[pos] = el;  // cursors started at the exact offsets
        } else if (pos < scap) {
          p.elems[(sd.bucket_begin + bk[k]) * scap + pos] = el;
        } else {
          atomicAdd(&p.oversized[1], 1ull);  // slot overflow: the build is redone with exact offsets
        }
      }
    }
  } else {
#pragma unroll
    for (int k = 0; k < IPT; ++k) {
      if (bk[k] >= 0) {
        const long long gb = sd.bucket_begin + bk[k];
        const long long pos = (long long)atomicAdd(&p.cursor[gb], 1ull);
        atomicMax(&gmax[gb * 3 + cd.slot], (unsigned long long)ev[k]);
        Elem el;
        el.s = sv[k];
        el.e_slot = (long long)((unsigned long long)ev[k] | slotbits);
        if (scap == 0) {
          p.elems[pos] = el;
        } else if (pos < scap) {
          p.elems[gb * scap + pos] = el;
        } else {
          atomicAdd(&p.oversized[1], 1ull);
        }
      }
    }
  }
}

// ----------------------------------------------------------------------------
// carry / base: per-segment scans over buckets, one wave per segment
// ----------------------------------------------------------------------------

template <int THREADS>
__global__ __launch_bounds__(THREADS) void k_carry(Plan p) {
  const int lane = threadIdx.x & 63;
  const long long seg = (long long)blockIdx.x * (THREADS / 64) + (threadIdx.x >> 6);
  if (seg >= p.n_segs) return;
  const SegDesc sd = p.segs[seg];
  const SegStats st = p.stats[seg];
  const long long nb = 1ll << sd.log_nb;
  // the running max end before any record: just below the first start
  const long long init = st.min_s > st.max_s ? -1 : (long long)st.min_s - 1;
  long long run[3] = {init, init, init};
  for (long long b0 = 0; b0 < nb; b0 += 64) {
    const long long b = b0 + lane;
    const bool ok = b < nb;
    long long v[3] = {LLONG_MIN, LLONG_MIN, LLONG_MIN};
    if (ok) {
      const unsigned long long* m = p.maxend + (sd.bucket_begin + b) * 3;
      const long long m0 = m[0] ? (long long)m[0] : LLONG_MIN;
      const long long m1 = m[1] ? (long long)m[1] : LLONG_MIN;
      const long long m2 = m[2] ? (long long)m[2] : LLONG_MIN;
      v[0] = m0;
      v[1] = m1 > m0 ? m1 : m0;
      v[2] = m2 > v[1] ? m2 : v[1];
    }
#pragma unroll
    for (int l = 0; l < 3; ++l) {
      long long all;
      const long long ex = wave_excl_scan_dpp<OpMax>(v[l], LLONG_MIN, all);
      if (ok) p.carry[(sd.bucket_begin + b) * 3 + l] = ex > run[l] ? ex : run[l];
      run[l] = all > run[l] ? all : run[l];
    }
  }
  // largest end of the segment (level 2 holds every kind); no record: the min start
  if (lane == 0) p.stats[seg].max_e = (unsigned long long)(run[2] > init ? run[2] : (init + 1 > 0 ? init + 1 : 0));
}

template <int THREADS>
__global__ __launch_bounds__(THREADS) void k_base(Plan p) {
  const int lane = threadIdx.x & 63;
  const long long seg = (long long)blockIdx.x * (THREADS / 64) + (threadIdx.x >> 6);
  if (seg >= p.n_segs) return;
  const SegDesc sd = p.segs[seg];
  const long long nb = 1ll << sd.log_nb;
  long long run[3] = {0, 0, 0};
  for (long long b0 = 0; b0 < nb; b0 += 64) {
    const long long b = b0 + lane;
    const bool ok = b < nb;
#pragma unroll
    for (int l = 0; l < 3; ++l) {
      long long all;
      const long long ex = wave_excl_scan_dpp<OpSum>(ok ? p.bsum[(sd.bucket_begin + b) * 3 + l] : 0, 0, all);
      if (ok) p.base[(sd.bucket_begin + b) * 3 + l] = run[l] + ex;
      run[l] += all;
    }
  }
  if (lane == 0) {
    for (int l = 0; l < 3; ++l) p.seg_total[seg * 3 + l] = run[l];
  }
}

// ----------------------------------------------------------------------------
// merge: per bucket, sort by start in LDS and flatten each level
// ----------------------------------------------------------------------------

// Block path: one workgroup flattens bucket gb (LDS radix sort up to CAP
// records, global-memory radix sort beyond).
template <int THREADS, int CAP>
__device__ void merge_bucket_block(const Plan& p, long long gb, SortSmem<THREADS, CAP>& sm, int* s_seg) {
  if (threadIdx.x == 0) *s_seg = upper_index_seg(p.segs, p.n_segs, gb);
  __syncthreads();
  const int seg = *s_seg;
  const SegDesc sd = p.segs[seg];
  const Geom g = seg_geom(p.stats[seg], sd);
  const long long bl = gb - sd.bucket_begin;
  const long long n = p.counts[gb];
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
  if (n > 0) {
    const long long lo = g.min_s + (bl << g.shift);
    if (n <= CAP) {
      const int ni = (int)n;
      const Elem* rec = p.slot_cap ? p.elems + gb * p.slot_cap : p.elems + off;
      for (int i = threadIdx.x; i < ni; i += THREADS) sm.E[i] = rec[i];  // coalesced 16 B per lane
      __syncthreads();
      const unsigned short* ord = sort_lds<THREADS, CAP>(sm, ni, lo);
      flatten_tile<THREADS>(sm.E, ord, ni, nlev, 0, comp, st, sm.lds_scan, nullptr);
    } else {
      // oversized bucket: stable LSD sort through global scratch, then flatten
      // CAP records at a time, carrying the running state across tiles
      const Elem* src = sort_global<THREADS, CAP>(sm, p.elems + off, p.elems2 + off, n, lo);
      for (long long t0 = 0; t0 < n; t0 += CAP) {
        const int cnt = (int)min((long long)CAP, n - t0);
        for (int i = threadIdx.x; i < cnt; i += THREADS) sm.E[i] = src[t0 + i];
        __syncthreads();
        flatten_tile<THREADS>(sm.E, nullptr, cnt, nlev, 0, comp, st, sm.lds_scan, nullptr);
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

// Buckets the wave path handed over (ticket[2] of them in p.queue), taken by
// persistent workgroups from a shared counter (ticket[1]). Every workgroup
// exits once the counter passes the queue length.
template <int THREADS, int CAP>
__global__ __launch_bounds__(THREADS) void k_merge_block(Plan p) {
  __shared__ SortSmem<THREADS, CAP> sm;
  __shared__ int s_seg;
  __shared__ unsigned int s_idx;
  const unsigned int qlen = __hip_atomic_load(&p.ticket[2], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  while (true) {
    if (threadIdx.x == 0) s_idx = atomicAdd(&p.ticket[1], 1u);
    __syncthreads();
    const unsigned int idx = s_idx;
    __syncthreads();
    if (idx >= qlen) break;
    merge_bucket_block<THREADS, CAP>(p, (long long)p.queue[idx], sm, &s_seg);
  }
}

// Wave path: each wave flattens one bucket of at most kWaveCap records whose
// time width fits 32 bits, with no workgroup barrier. The sort is a counting
// sort on the top bits of the start offset into 1024 sub-bins followed by an
// insertion sort inside each sub-bin (records with equal starts may end in
// any order: the flattened result does not depend on it). Buckets that do not
// fit, or whose sub-bins are too crowded, go to the block path's queue.
struct WaveSmem {
  unsigned int key[kWaveCap];
  long long eslot[kWaveCap];
  unsigned short ord[kWaveCap];
  unsigned short rank[kWaveCap];     // rank of a record inside its sub-bin
  unsigned int bins[kWaveBins / 2];  // two 16-bit counters per word
};

__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

template <int K, class Op>
__device__ __forceinline__ void wave_excl_scan(const long long (&v)[K], long long (&ex)[K], long long (&tot)[K],
                                               long long ident) {
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int k = 0; k < K; ++k) {
    long long x = v[k];
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
      const long long y = __shfl_up(x, d, 64);
      if (lane >= d) x = Op::apply(x, y);
    }
    long long e = __shfl_up(x, 1, 64);
    if (lane == 0) e = ident;
    ex[k] = e;
    tot[k] = __shfl(x, 63, 64);
  }
}

// Flatten of one sorted bucket by one wave: lane owns sorted positions
// [lane*IPL, lane*IPL + cnt), kept in registers through the three phases
// (running max of ends, measures and break counts, component writes).
template <int IPL, int NLEV>
__device__ __forceinline__ void wave_flatten(const Plan& p, const WaveSmem& W, long long gb, long long off, int ni,
                                             long long lo) {
  const int lane = threadIdx.x & 63;
  const int ipl = (ni + 63) >> 6;
  const int q0 = lane * ipl;
  const int cnt = min(max(ni - q0, 0), ipl);
  constexpr long long EMASK = (1ll << kSlotShift) - 1;
  long long sv[IPL], ev[IPL];
  int sl[IPL];
  long long tmax[NLEV];
#pragma unroll
  for (int l = 0; l < NLEV; ++l) tmax[l] = LLONG_MIN;
#pragma unroll
  for (int j = 0; j < IPL; ++j) {
    sv[j] = 0;
    ev[j] = 0;
    sl[j] = 3;
    if (j < cnt) {
      const int i = W.ord[q0 + j];
      const long long es = W.eslot[i];
      sv[j] = lo + (long long)W.key[i];
      ev[j] = es & EMASK;
      sl[j] = (int)((unsigned long long)es >> kSlotShift);
#pragma unroll
      for (int l = 0; l < NLEV; ++l)
        if (sl[j] <= l && ev[j] > tmax[l]) tmax[l] = ev[j];
    }
  }
  long long M[NLEV];
#pragma unroll
  for (int l = 0; l < NLEV; ++l) {
    long long tot;
    const long long ex = wave_excl_scan_dpp<OpMax>(tmax[l], LLONG_MIN, tot);
    const long long c = p.carry[gb * 3 + l];
    M[l] = ex > c ? ex : c;
  }
  // per-lane measure per level; the break counts packed in 16-bit fields
  long long acc[NLEV];
  long long nbrk = 0;
  {
    long long Mb[NLEV];
#pragma unroll
    for (int l = 0; l < NLEV; ++l) {
      Mb[l] = M[l];
      acc[l] = 0;
    }
#pragma unroll
    for (int j = 0; j < IPL; ++j) {
#pragma unroll
      for (int l = 0; l < NLEV; ++l) {
        if (j < cnt && sl[j] <= l) {
          const long long b = sv[j] > Mb[l] ? sv[j] : Mb[l];
          if (ev[j] > b) acc[l] += ev[j] - b;
          if (sv[j] > Mb[l]) nbrk += 1ll << (16 * l);
          if (ev[j] > Mb[l]) Mb[l] = ev[j];
        }
      }
    }
  }
  long long P[NLEV], totp[NLEV];
#pragma unroll
  for (int l = 0; l < NLEV; ++l) P[l] = wave_excl_scan_dpp<OpSum>(acc[l], 0, totp[l]);
  long long totr;
  const long long Rp = wave_excl_scan_dpp<OpSum>(nbrk, 0, totr);
  long long R[NLEV];
#pragma unroll
  for (int l = 0; l < NLEV; ++l) R[l] = (Rp >> (16 * l)) & 0xFFFF;
#pragma unroll
  for (int j = 0; j < IPL; ++j) {
#pragma unroll
    for (int l = 0; l < NLEV; ++l) {
      if (j < cnt && sl[j] <= l) {
        if (sv[j] > M[l]) {
          Comp c;
          c.cs = sv[j];
          c.pl = P[l];
          p.comp[l][off + R[l]] = c;
          R[l] += 1;
        }
        const long long b = sv[j] > M[l] ? sv[j] : M[l];
        if (ev[j] > b) P[l] += ev[j] - b;
        if (ev[j] > M[l]) M[l] = ev[j];
      }
    }
  }
  if (lane < 3) {
    long long bs = 0;
#pragma unroll
    for (int l = 0; l < NLEV; ++l)
      if (lane == l) bs = totp[l];
    p.bsum[gb * 3 + lane] = bs;
    p.ncomp[gb * 3 + lane] = (unsigned int)((totr >> (16 * lane)) & 0xFFFF);
  }
}

__global__ __launch_bounds__(256) void k_merge_wave(Plan p) {
  __shared__ WaveSmem wsm[4];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const long long gb = (long long)blockIdx.x * 4 + wave;
  if (gb >= p.n_buckets) return;
  WaveSmem& W = wsm[wave];
  const int seg = upper_index_seg(p.segs, p.n_segs, gb);
  const SegDesc sd = p.segs[seg];
  const Geom g = seg_geom(p.stats[seg], sd);
  const long long n = p.counts[gb];
  const long long off = (long long)p.offsets[gb];
  const int nlev = sd.n_levels;
  if (n == 0) {
    if (lane < 3) {
      p.bsum[gb * 3 + lane] = 0;
      p.ncomp[gb * 3 + lane] = 0;
    }
    return;
  }
  if (n > kWaveCap || g.shift > 32) {
    if (lane == 0) p.queue[atomicAdd(&p.ticket[2], 1u)] = (unsigned int)gb;
    return;
  }
  const int ni = (int)n;
  const long long lo = g.min_s + ((gb - sd.bucket_begin) << g.shift);
  const Elem* rec = p.slot_cap ? p.elems + gb * p.slot_cap : p.elems + off;
  // load; find the highest varying key bit
  unsigned int kor = 0;
  for (int i = lane; i < ni; i += 64) {
    const Elem el = rec[i];
    const unsigned int k = (unsigned int)(el.s - lo);
    W.key[i] = k;
    W.eslot[i] = el.e_slot;
    kor |= k;
  }
  for (int d = 32; d >= 1; d >>= 1) kor |= __shfl_xor(kor, d, 64);
  // sub-bins: about two per record, 128 .. 1024; a lane owns bpl of them (two per LDS word)
  int dbits = 7;
  while ((1 << dbits) < 2 * ni && dbits < 10) ++dbits;
  const int nbins = 1 << dbits, bpl = nbins >> 6, wpl = bpl >> 1;
  for (int j = 0; j < wpl; ++j) W.bins[lane * wpl + j] = 0;
  wave_sync();
  const int hb = kor ? 32 - __clz((int)kor) : 0;
  const int dsh = hb > dbits ? hb - dbits : 0;  // sub-bin = key >> dsh
  for (int i = lane; i < ni; i += 64) {
    const unsigned int d = W.key[i] >> dsh;
    const unsigned int sh = 16u * (d & 1u);
    W.rank[i] = (unsigned short)((atomicAdd(&W.bins[d >> 1], 1u << sh) >> sh) & 0xFFFFu);
  }
  wave_sync();
  // exclusive scan of the sub-bin counters (lane order = sub-bin order)
  long long tot = 0;
  for (int j = 0; j < wpl; ++j) {
    const unsigned int w = W.bins[lane * wpl + j];
    tot += (w & 0xFFFFu) + (w >> 16);
  }
  long long all;
  unsigned int run = (unsigned int)wave_excl_scan_dpp<OpSum>(tot, 0, all);
  wave_sync();
  for (int j = 0; j < wpl; ++j) {
    const unsigned int w = W.bins[lane * wpl + j];
    const unsigned int a = run, b = run + (w & 0xFFFFu);
    run = b + (w >> 16);
    W.bins[lane * wpl + j] = a | (b << 16);
  }
  wave_sync();
  unsigned int fix = 0;  // bit r: the record of round r is the second one of its sub-bin
  for (int i = lane, r = 0; i < ni; i += 64, ++r) {
    const unsigned int d = W.key[i] >> dsh;
    const unsigned int st0 = (W.bins[d >> 1] >> (16u * (d & 1u))) & 0xFFFFu;
    const unsigned int rk = W.rank[i];
    W.ord[st0 + rk] = (unsigned short)i;
    if (rk == 1) fix |= 1u << r;
  }
  wave_sync();
  // order inside each sub-bin by the full key: one lane per sub-bin holding
  // two or more records (the lane that placed its second record)
  bool crowded = false;
  if (dsh > 0) {
    while (fix) {
      const int r = __ffs((int)fix) - 1;
      fix &= fix - 1;
      const unsigned int d = W.key[r * 64 + lane] >> dsh;
      const int st0 = (int)((W.bins[d >> 1] >> (16u * (d & 1u))) & 0xFFFFu);
      const int st1 = (int)d + 1 < nbins ? (int)((W.bins[(d + 1) >> 1] >> (16u * ((d + 1) & 1u))) & 0xFFFFu) : ni;
      const int c = st1 - st0;
      if (c > 32) {
        crowded = true;
        continue;
      }
      unsigned short* o = W.ord + st0;
      for (int a = 1; a < c; ++a) {
        const unsigned short x = o[a];
        const unsigned int kx = W.key[x];
        int b = a - 1;
        while (b >= 0 && W.key[o[b]] > kx) {
          o[b + 1] = o[b];
          --b;
        }
        o[b + 1] = x;
      }
    }
  }
  if (__ballot(crowded)) {
    if (lane == 0) p.queue[atomicAdd(&p.ticket[2], 1u)] = (unsigned int)gb;
    return;
  }
  wave_sync();
  // flatten: lane owns sorted positions [q0, q0 + cnt); specialised by records per lane and levels
  const int ipl = (ni + 63) >> 6;
  if (nlev == 2) {
    if (ipl <= 1) wave_flatten<1, 2>(p, W, gb, off, ni, lo);
    else if (ipl <= 2) wave_flatten<2, 2>(p, W, gb, off, ni, lo);
    else if (ipl <= 4) wave_flatten<4, 2>(p, W, gb, off, ni, lo);
    else wave_flatten<8, 2>(p, W, gb, off, ni, lo);
  } else {
    if (ipl <= 1) wave_flatten<1, 3>(p, W, gb, off, ni, lo);
    else if (ipl <= 2) wave_flatten<2, 3>(p, W, gb, off, ni, lo);
    else if (ipl <= 4) wave_flatten<4, 3>(p, W, gb, off, ni, lo);
    else wave_flatten<8, 3>(p, W, gb, off, ni, lo);
  }
}

// ----------------------------------------------------------------------------
// region: clip every resource by binary search, reduce, finalize in FP64
// ----------------------------------------------------------------------------

// Measure of level l of segment seg before time t.
__device__ long long measure_before(const Plan& p, int seg, int l, long long t) {
  const SegDesc sd = p.segs[seg];
  const Geom g = seg_geom(p.stats[seg], sd);
  if (g.empty || t <= g.min_s) return 0;
  if (t >= g.max_e) return p.seg_total[seg * 3 + l];
  const unsigned long long rel = (unsigned long long)(t - g.min_s);
  unsigned long long b = rel >> g.shift;
  const unsigned long long nb = 1ull << g.log_nb;
  if (b >= nb) b = nb - 1;
  const long long gb = sd.bucket_begin + (long long)b;
  const long long carry = p.carry[gb * 3 + l];
  const long long base = p.base[gb * 3 + l];
  const long long bs = p.bsum[gb * 3 + l];
  const long long cnt = p.ncomp[gb * 3 + l];
  const Comp* c = p.comp[l] + p.offsets[gb];
  // first component with start >= t
  long long lo = 0, hi = cnt;
  while (lo < hi) {
    const long long mid = (lo + hi) >> 1;
    if (c[mid].cs < t) lo = mid + 1; else hi = mid;
  }
  const long long k = lo - 1;
  if (k < 0) {
    // only the component carried in from earlier buckets lies before t
    const long long ext = carry + (cnt > 0 ? c[0].pl : bs);
    return base + (ext < t ? ext : t) - carry;
  }
  const Comp ck = c[k];
  const long long next_pl = k + 1 < cnt ? c[k + 1].pl : bs;
  const long long ce = ck.cs + (next_pl - ck.pl);
  return base + ck.pl + (ce < t ? ce : t) - ck.cs;
}

template <int THREADS>
__global__ __launch_bounds__(THREADS) void k_region(Plan p, const RegionDesc* regions, Tree* trees,
                                                    long long* times) {
  __shared__ long long lds[THREADS / 64 * 10];
  const RegionDesc rd = regions[blockIdx.x];
  const long long E = rd.t1 - rd.t0;
  const int R = rd.n_hosts + rd.n_devices;
  // sums: U, W, MPI, Other, UW, K, M ; maxes: UW, K, KM
  long long sU = 0, sW = 0, sMPI = 0, sO = 0, sK = 0, sM = 0;
  long long mUW = 0, mK = 0, mKM = 0;
  for (int r = threadIdx.x; r < R; r += THREADS) {
    const int seg = rd.seg_begin + r;
    const bool host = r < rd.n_hosts;
    const int nl = host ? 3 : 2;
    long long D[3] = {0, 0, 0};
    for (int l = 0; l < nl; ++l) D[l] = measure_before(p, seg, l, rd.t1) - measure_before(p, seg, l, rd.t0);
    long long* out = times + (rd.times_off + r) * 4;
    if (host) {
      const long long u = D[0], w = D[1] - D[0], mpi = D[2] - D[1], o = E - D[2];
      out[0] = u; out[1] = w; out[2] = mpi; out[3] = o;
      sU += u; sW += w; sMPI += mpi; sO += o;
      mUW = u + w > mUW ? u + w : mUW;
    } else {
      const long long k = D[0], mm = D[1] - D[0], idle = E - D[1];
      out[0] = k; out[1] = mm; out[2] = idle; out[3] = 0;
      sK += k; sM += mm;
      mK = k > mK ? k : mK;
      mKM = k + mm > mKM ? k + mm : mKM;
    }
  }
  long long v[9] = {sU, sW, sMPI, sO, sK, sM, mUW, mK, mKM};
  block_tree<THREADS>(v, lds);
  if (threadIdx.x == 0) trees[blockIdx.x] = make_tree(E, rd.n_hosts, rd.n_devices, v);
}

// ----------------------------------------------------------------------------
// launchers
// ----------------------------------------------------------------------------

hipError_t launch_reset(const Plan& p, hipStream_t st) {
  const long long work = 3 * p.n_buckets + p.n_segs + 64;
  int blocks = (int)min(2048ll, (work + 255) / 256);
  hipLaunchKernelGGL(k_reset, dim3(blocks), dim3(256), 0, st, p);
  return hipGetLastError();
}

hipError_t launch_stats(const Plan& p, hipStream_t st) {
  if (p.n_tiles == 0) return hipSuccess;
  hipLaunchKernelGGL(k_stats<256>, dim3((unsigned)p.n_tiles), dim3(256), 0, st, p);
  return hipGetLastError();
}

hipError_t launch_hist(const Plan& p, hipStream_t st) {
  if (p.n_tiles == 0) return hipSuccess;
  switch (p.tile_elems) {
    case 2048: hipLaunchKernelGGL((k_hist<256, 8>), dim3((unsigned)p.n_tiles), dim3(256), 0, st, p); break;
    case 8192: hipLaunchKernelGGL((k_hist<512, 16>), dim3((unsigned)p.n_tiles), dim3(512), 0, st, p); break;
    default: hipLaunchKernelGGL((k_hist<256, 16>), dim3((unsigned)p.n_tiles), dim3(256), 0, st, p); break;
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
  switch (p.tile_elems) {
    case 2048: hipLaunchKernelGGL((k_scatter<256, 8>), dim3((unsigned)p.n_tiles), dim3(256), 0, st, p); break;
    case 8192: hipLaunchKernelGGL((k_scatter<512, 16>), dim3((unsigned)p.n_tiles), dim3(512), 0, st, p); break;
    default: hipLaunchKernelGGL((k_scatter<256, 16>), dim3((unsigned)p.n_tiles), dim3(256), 0, st, p); break;
  }
  return hipGetLastError();
}

hipError_t launch_carry(const Plan& p, hipStream_t st) {
  if (p.n_segs == 0) return hipSuccess;
  hipLaunchKernelGGL(k_carry<256>, dim3((unsigned)((p.n_segs + 3) / 4)), dim3(256), 0, st, p);
  return hipGetLastError();
}

hipError_t launch_merge_wave(const Plan& p, hipStream_t st) {
  if (p.n_buckets == 0) return hipSuccess;
  hipLaunchKernelGGL(k_merge_wave, dim3((unsigned)((p.n_buckets + 3) / 4)), dim3(256), 0, st, p);
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
  hipLaunchKernelGGL(k_base<256>, dim3((unsigned)((p.n_segs + 3) / 4)), dim3(256), 0, st, p);
  return hipGetLastError();
}

hipError_t launch_region(const Plan& p, const RegionDesc* regions, int n_regions, Tree* trees, long long* times,
                         hipStream_t st) {
  if (n_regions == 0) return hipSuccess;
  hipLaunchKernelGGL(k_region<256>, dim3((unsigned)n_regions), dim3(256), 0, st, p, regions, trees, times);
  return hipGetLastError();
}

}  // namespace hpop
