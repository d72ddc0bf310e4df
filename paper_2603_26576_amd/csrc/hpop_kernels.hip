// HIP kernels of the trace reduction, written for CDNA4 (gfx950, wave64).
//
// All passes are memory-bound integer work: no MFMA (there is no dense
// contraction), loads and stores are coalesced, the fine-grained sort runs in
// LDS (160 KB per workgroup on gfx950), and cross-workgroup communication is
// limited to atomics on per-bucket counters plus one decoupled look-back scan
// over bucket counts.
#include <hip/hip_runtime.h>

#include <climits>

#include "hpop_internal.h"
#include "hpop_kernels.h"

namespace hpop {

// ----------------------------------------------------------------------------
// small device helpers
// ----------------------------------------------------------------------------

__device__ __forceinline__ int bitlen64(unsigned long long x) { return x ? 64 - __clzll((long long)x) : 0; }

__device__ __forceinline__ bool rec_valid(long long s, long long e) {
  return s >= 0 && s <= e && e < kTimeLimit;
}

struct Geom {
  long long min_s;
  long long max_e;
  int shift;
  int log_nb;
  bool empty;
};

__device__ __forceinline__ Geom seg_geom(const SegStats& st, const SegDesc& sd) {
  Geom g;
  g.empty = st.min_s > st.max_s;
  g.min_s = (long long)st.min_s;
  g.max_e = (long long)st.max_e;
  g.log_nb = sd.log_nb;
  const int bl = g.empty ? 0 : bitlen64(st.max_s - st.min_s);
  g.shift = bl > sd.log_nb ? bl - sd.log_nb : 0;
  return g;
}

// bucket of a record start inside its segment (clamped; start >= min_s for valid records)
__device__ __forceinline__ int bucket_of(long long s, const Geom& g) {
  unsigned long long rel = (unsigned long long)(s - g.min_s);
  unsigned long long b = rel >> g.shift;
  const unsigned long long nb = 1ull << g.log_nb;
  return (int)(b < nb ? b : nb - 1);
}

// index of the last entry with key <= x in a sorted array of n int64 (n >= 1, a[0] <= x)
__device__ __forceinline__ int upper_index_chunk(const ChunkDesc* c, int n, long long x) {
  int lo = 0, hi = n - 1;
  while (lo < hi) {
    int mid = (lo + hi + 1) >> 1;
    if (c[mid].tile_begin <= x) lo = mid; else hi = mid - 1;
  }
  return lo;
}

__device__ __forceinline__ int upper_index_seg(const SegDesc* s, int n, long long x) {
  int lo = 0, hi = n - 1;
  while (lo < hi) {
    int mid = (lo + hi + 1) >> 1;
    if (s[mid].bucket_begin <= x) lo = mid; else hi = mid - 1;
  }
  return lo;
}

__device__ __forceinline__ long long wave_red_min(long long v) {
  for (int d = 32; d >= 1; d >>= 1) { long long o = __shfl_xor(v, d, 64); v = o < v ? o : v; }
  return v;
}
__device__ __forceinline__ unsigned long long wave_red_minu(unsigned long long v) {
  for (int d = 32; d >= 1; d >>= 1) { unsigned long long o = __shfl_xor(v, d, 64); v = o < v ? o : v; }
  return v;
}
__device__ __forceinline__ unsigned long long wave_red_maxu(unsigned long long v) {
  for (int d = 32; d >= 1; d >>= 1) { unsigned long long o = __shfl_xor(v, d, 64); v = o > v ? o : v; }
  return v;
}
__device__ __forceinline__ long long wave_red_sum(long long v) {
  for (int d = 32; d >= 1; d >>= 1) v += __shfl_xor(v, d, 64);
  return v;
}
__device__ __forceinline__ long long wave_red_max(long long v) {
  for (int d = 32; d >= 1; d >>= 1) { long long o = __shfl_xor(v, d, 64); v = o > v ? o : v; }
  return v;
}

struct OpMax {
  __device__ static long long apply(long long a, long long b) { return a > b ? a : b; }
};
struct OpSum {
  __device__ static long long apply(long long a, long long b) { return a + b; }
};

// Block-wide exclusive scan of K int64 lanes per thread (thread order), with totals.
// `lds` holds NW*K int64. Contains barriers: call from uniform control flow.
template <int THREADS, int K, class Op>
__device__ __forceinline__ void block_excl_scan(const long long (&v)[K], long long (&excl)[K],
                                                long long (&total)[K], long long ident, long long* lds) {
  constexpr int NW = THREADS / 64;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  long long inc[K];
#pragma unroll
  for (int k = 0; k < K; ++k) {
    long long x = v[k];
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
      long long y = __shfl_up(x, d, 64);
      if (lane >= d) x = Op::apply(x, y);
    }
    inc[k] = x;
  }
  if (lane == 63) {
#pragma unroll
    for (int k = 0; k < K; ++k) lds[wave * K + k] = inc[k];
  }
  __syncthreads();
#pragma unroll
  for (int k = 0; k < K; ++k) {
    long long pre = ident, tot = ident;
    for (int w = 0; w < NW; ++w) {
      const long long t = lds[w * K + k];
      if (w < wave) pre = Op::apply(pre, t);
      tot = Op::apply(tot, t);
    }
    long long ex = __shfl_up(inc[k], 1, 64);
    if (lane == 0) ex = ident;
    excl[k] = Op::apply(pre, ex);
    total[k] = tot;
  }
  __syncthreads();
}

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
  for (long long i = tid; i < p.n_buckets; i += stride) p.counts[i] = 0;
  for (long long i = tid; i < 3 * p.n_buckets; i += stride) p.maxend[i] = 0;
  const long long nscan = (p.n_buckets + kScanTile - 1) / kScanTile + 1;
  for (long long i = tid; i < nscan; i += stride) p.scan_state[i] = 0;
  if (tid == 0) {
    p.err[0] = ULLONG_MAX;
    p.oversized[0] = 0;
  }
  if (tid < 4) p.ticket[tid] = 0;
}

// ----------------------------------------------------------------------------
// stats: validate records, per-segment min/max start and max end
// ----------------------------------------------------------------------------

template <int THREADS>
__global__ __launch_bounds__(THREADS) void k_stats(Plan p) {
  constexpr int NW = THREADS / 64;
  __shared__ int s_chunk;
  __shared__ unsigned long long red[4][NW];
  const long long tile = blockIdx.x;
  if (threadIdx.x == 0) s_chunk = upper_index_chunk(p.chunks, p.n_chunks, tile);
  __syncthreads();
  const ChunkDesc cd = p.chunks[s_chunk];
  const long long base = (tile - cd.tile_begin) * (long long)p.tile_elems;
  const long long end = min((long long)cd.count, base + p.tile_elems);
  unsigned long long mn = ULLONG_MAX, mxs = 0, mxe = 0, bad = ULLONG_MAX;
  for (long long i = base + threadIdx.x; i < end; i += THREADS) {
    const long long s = cd.s[i], e = cd.e[i];
    if (!rec_valid(s, e)) {
      bad = (unsigned long long)i < bad ? (unsigned long long)i : bad;
    } else if (s < e) {
      mn = (unsigned long long)s < mn ? (unsigned long long)s : mn;
      mxs = (unsigned long long)s > mxs ? (unsigned long long)s : mxs;
      mxe = (unsigned long long)e > mxe ? (unsigned long long)e : mxe;
    }
  }
  mn = wave_red_minu(mn);
  mxs = wave_red_maxu(mxs);
  mxe = wave_red_maxu(mxe);
  bad = wave_red_minu(bad);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (lane == 0) {
    red[0][wave] = mn;
    red[1][wave] = mxs;
    red[2][wave] = mxe;
    red[3][wave] = bad;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int w = 1; w < NW; ++w) {
      mn = red[0][w] < mn ? red[0][w] : mn;
      mxs = red[1][w] > mxs ? red[1][w] : mxs;
      mxe = red[2][w] > mxe ? red[2][w] : mxe;
      bad = red[3][w] < bad ? red[3][w] : bad;
    }
    if (mn != ULLONG_MAX) {
      atomicMin(&p.stats[cd.seg].min_s, mn);
      atomicMax(&p.stats[cd.seg].max_s, mxs);
      atomicMax(&p.stats[cd.seg].max_e, mxe);
    }
    if (bad != ULLONG_MAX) atomicMin(p.err, ((unsigned long long)cd.chunk_id << 40) | bad);
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
    for (int k = 0; k < IPT; ++k)
      if (bk[k] >= 0) atomicAdd(&hist[bk[k] - bmin], 1u);
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
#pragma unroll
  for (int k = 0; k < IPT; ++k) {
    c[k] = (b0 + k < p.n_buckets) ? p.counts[b0 + k] : 0u;
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
      p.cursor[b0 + k] = run;
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
      if (rec_valid(sv[k], ev[k]) && sv[k] < ev[k]) {
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
#pragma unroll
    for (int k = 0; k < IPT; ++k) {
      rk[k] = 0;
      if (bk[k] >= 0) {
        rk[k] = atomicAdd(&hist[bk[k] - bmin], 1u);
        atomicMax(&bmaxe[bk[k] - bmin], (unsigned long long)ev[k]);
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
        const unsigned long long pos = bbase[bk[k] - bmin] + rk[k];
        Elem el;
        el.s = sv[k];
        el.e_slot = (long long)((unsigned long long)ev[k] | slotbits);
        p.elems[pos] = el;
      }
    }
  } else {
#pragma unroll
    for (int k = 0; k < IPT; ++k) {
      if (bk[k] >= 0) {
        const long long gb = sd.bucket_begin + bk[k];
        const unsigned long long pos = atomicAdd(&p.cursor[gb], 1ull);
        atomicMax(&gmax[gb * 3 + cd.slot], (unsigned long long)ev[k]);
        Elem el;
        el.s = sv[k];
        el.e_slot = (long long)((unsigned long long)ev[k] | slotbits);
        p.elems[pos] = el;
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
      long long x = v[l];
#pragma unroll
      for (int d = 1; d < 64; d <<= 1) {
        long long y = __shfl_up(x, d, 64);
        if (lane >= d) x = x > y ? x : y;
      }
      long long ex = __shfl_up(x, 1, 64);
      if (lane == 0) ex = LLONG_MIN;
      if (ok) p.carry[(sd.bucket_begin + b) * 3 + l] = ex > run[l] ? ex : run[l];
      const long long all = __shfl(x, 63, 64);
      run[l] = all > run[l] ? all : run[l];
    }
  }
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
      long long x = ok ? p.bsum[(sd.bucket_begin + b) * 3 + l] : 0;
#pragma unroll
      for (int d = 1; d < 64; d <<= 1) {
        long long y = __shfl_up(x, d, 64);
        if (lane >= d) x += y;
      }
      long long ex = __shfl_up(x, 1, 64);
      if (lane == 0) ex = 0;
      if (ok) p.base[(sd.bucket_begin + b) * 3 + l] = run[l] + ex;
      run[l] += __shfl(x, 63, 64);
    }
  }
  if (lane == 0) {
    for (int l = 0; l < 3; ++l) p.seg_total[seg * 3 + l] = run[l];
  }
}

// ----------------------------------------------------------------------------
// merge: per bucket, sort by start in LDS and flatten each level
// ----------------------------------------------------------------------------

// One stable LSD pass on 8 bits of (start - lo) >> sh over the positions
// in[0..n): out[] receives the element indices in the new order, dstart[d] the
// first output position of digit d. Waves own contiguous position ranges;
// lanes with equal digits are matched with ballots, so the pass is stable.
template <int THREADS, int MAXR>
__device__ __forceinline__ void radix_pass(const Elem* E, const unsigned short* in, unsigned short* out, int n,
                                           long long lo, int sh, unsigned int* whist, unsigned int* dstart,
                                           long long* lds_scan) {
  constexpr int NW = THREADS / 64;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int span = (((n + NW - 1) / NW) + 63) & ~63;
  const unsigned long long lt = (1ull << lane) - 1ull;
  for (int i = threadIdx.x; i < NW * 256; i += THREADS) whist[i] = 0;
  __syncthreads();
  unsigned int loc[MAXR];
  unsigned char dig[MAXR];
  unsigned short idx[MAXR];
#pragma unroll
  for (int r = 0; r < MAXR; ++r) {
    loc[r] = 0;
    dig[r] = 0;
    idx[r] = 0;
    if (r * 64 < span) {  // wave-uniform
      const int pos = wave * span + r * 64 + lane;
      const bool act = pos < n;
      const unsigned short i = act ? (in ? in[pos] : (unsigned short)pos) : (unsigned short)0;
      const unsigned int d = act ? (unsigned int)(((unsigned long long)(E[i].s - lo) >> sh) & 255ull) : 0u;
      unsigned long long peers = __ballot(act);
#pragma unroll
      for (int bit = 0; bit < 8; ++bit) {
        const bool b = (d >> bit) & 1u;
        const unsigned long long m = __ballot(b);
        peers &= b ? m : ~m;
      }
      if (act) {
        unsigned int* h = &whist[wave * 256 + d];
        const unsigned int before = *h;
        loc[r] = before + (unsigned int)__popcll(peers & lt);
        dig[r] = (unsigned char)d;
        idx[r] = i;
        if ((peers & lt) == 0) *h = before + (unsigned int)__popcll(peers);
      }
    }
  }
  __syncthreads();
  // digit-major exclusive prefix over (digit, wave)
  {
    long long tot = 0;
    unsigned int h[NW];
    if (threadIdx.x < 256) {
#pragma unroll
      for (int w = 0; w < NW; ++w) { h[w] = whist[w * 256 + threadIdx.x]; tot += h[w]; }
    }
    long long v[1] = {threadIdx.x < 256 ? tot : 0}, ex[1], all[1];
    block_excl_scan<THREADS, 1, OpSum>(v, ex, all, 0, lds_scan);
    if (threadIdx.x < 256) {
      unsigned int run = (unsigned int)ex[0];
      dstart[threadIdx.x] = run;
#pragma unroll
      for (int w = 0; w < NW; ++w) { whist[w * 256 + threadIdx.x] = run; run += h[w]; }
    }
  }
  __syncthreads();
#pragma unroll
  for (int r = 0; r < MAXR; ++r) {
    if (r * 64 < span) {
      const int pos = wave * span + r * 64 + lane;
      if (pos < n) out[whist[wave * 256 + dig[r]] + loc[r]] = idx[r];
    }
  }
  __syncthreads();
}

struct FlatState {
  long long M[3];  // running max end (with the carry)
  long long P[3];  // measure accumulated in this bucket
  long long R[3];  // components written in this bucket
};

// Flatten one sorted tile: positions 0..n-1 in order ord (or identity).
// Writes components of each level at comp[l][off + R], advances `st`.
template <int THREADS>
__device__ __forceinline__ void flatten_tile(const Elem* E, const unsigned short* ord, int n, int nlev,
                                             long long off, Comp* const* comp, FlatState& st, long long* lds_scan,
                                             long long* lds_bc) {
  const int ipt = (n + THREADS - 1) / THREADS;
  const int p0 = threadIdx.x * ipt;
  const int p1 = min(n, p0 + ipt);
  const long long EMASK = (1ll << kSlotShift) - 1;
  // phase A: exclusive max-scan of ends per level
  long long tmax[3] = {LLONG_MIN, LLONG_MIN, LLONG_MIN};
  for (int q = p0; q < p1; ++q) {
    const Elem el = E[ord ? ord[q] : q];
    const int slot = (int)((unsigned long long)el.e_slot >> kSlotShift);
    const long long e = el.e_slot & EMASK;
#pragma unroll
    for (int l = 0; l < 3; ++l)
      if (slot <= l && e > tmax[l]) tmax[l] = e;
  }
  long long exm[3], totm[3];
  block_excl_scan<THREADS, 3, OpMax>(tmax, exm, totm, LLONG_MIN, lds_scan);
  long long M[3];
#pragma unroll
  for (int l = 0; l < 3; ++l) M[l] = exm[l] > st.M[l] ? exm[l] : st.M[l];
  // phase B: per-thread measure and break counts
  long long acc[6] = {0, 0, 0, 0, 0, 0};
  {
    long long Mb[3] = {M[0], M[1], M[2]};
    for (int q = p0; q < p1; ++q) {
      const Elem el = E[ord ? ord[q] : q];
      const int slot = (int)((unsigned long long)el.e_slot >> kSlotShift);
      const long long e = el.e_slot & EMASK;
      const long long s = el.s;
#pragma unroll
      for (int l = 0; l < 3; ++l) {
        if (l < nlev && slot <= l) {
          const long long lo = s > Mb[l] ? s : Mb[l];
          if (e > lo) acc[l] += e - lo;
          if (s > Mb[l]) acc[3 + l] += 1;
          if (e > Mb[l]) Mb[l] = e;
        }
      }
    }
  }
  long long exa[6], tota[6];
  block_excl_scan<THREADS, 6, OpSum>(acc, exa, tota, 0, lds_scan);
  // phase C: write components
  {
    long long P[3], R[3];
#pragma unroll
    for (int l = 0; l < 3; ++l) {
      P[l] = st.P[l] + exa[l];
      R[l] = st.R[l] + exa[3 + l];
    }
    for (int q = p0; q < p1; ++q) {
      const Elem el = E[ord ? ord[q] : q];
      const int slot = (int)((unsigned long long)el.e_slot >> kSlotShift);
      const long long e = el.e_slot & EMASK;
      const long long s = el.s;
#pragma unroll
      for (int l = 0; l < 3; ++l) {
        if (l < nlev && slot <= l) {
          if (s > M[l]) {
            Comp c;
            c.cs = s;
            c.pl = P[l];
            comp[l][off + R[l]] = c;
            R[l] += 1;
          }
          const long long lo = s > M[l] ? s : M[l];
          if (e > lo) P[l] += e - lo;
          if (e > M[l]) M[l] = e;
        }
      }
    }
  }
#pragma unroll
  for (int l = 0; l < 3; ++l) {
    st.M[l] = totm[l] > st.M[l] ? totm[l] : st.M[l];
    st.P[l] += tota[l];
    st.R[l] += tota[3 + l];
  }
  (void)lds_bc;
}

template <int THREADS, int CAP>
__global__ __launch_bounds__(THREADS) void k_merge(Plan p) {
  constexpr int NW = THREADS / 64;
  constexpr int MAXR = CAP / THREADS;  // rounds per wave in a radix pass
  __shared__ Elem E[CAP];
  __shared__ unsigned short ordA[CAP];
  __shared__ unsigned short ordB[CAP];
  __shared__ unsigned int whist[NW * 256];
  __shared__ unsigned int dstart[256];
  __shared__ unsigned int dcount[256];
  __shared__ long long lds_scan[NW * 6];
  __shared__ unsigned long long red[2][NW];
  __shared__ int s_seg;

  const long long gb = blockIdx.x;
  if (threadIdx.x == 0) s_seg = upper_index_seg(p.segs, p.n_segs, gb);
  __syncthreads();
  const int seg = s_seg;
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
  Comp* comp[3] = {p.comp[0], p.comp[1], p.comp[2]};
  if (n > 0) {
    const long long lo = g.min_s + (bl << g.shift);
    if (n <= CAP) {
      const int ni = (int)n;
      // load the bucket (coalesced 16 B per lane) and find the bits that vary
      unsigned long long kor = 0, kand = ~0ull;
      for (int i = threadIdx.x; i < ni; i += THREADS) {
        const Elem el = p.elems[off + i];
        E[i] = el;
        const unsigned long long k = (unsigned long long)(el.s - lo);
        kor |= k;
        kand &= k;
      }
      for (int d = 32; d >= 1; d >>= 1) {
        kor |= __shfl_xor(kor, d, 64);
        kand &= __shfl_xor(kand, d, 64);
      }
      const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
      if (lane == 0) { red[0][wave] = kor; red[1][wave] = kand; }
      __syncthreads();
      kor = 0; kand = ~0ull;
      for (int w = 0; w < NW; ++w) { kor |= red[0][w]; kand &= red[1][w]; }
      const unsigned long long vary = kor ^ kand;
      const unsigned short* ord = nullptr;
      if (vary) {
        const int lb = __ffsll((long long)vary) - 1;
        const int hb = bitlen64(vary);
        const int passes = (hb - lb + 7) >> 3;
        unsigned short* in = nullptr;  // identity for the first pass
        for (int ps = 0; ps < passes; ++ps) {
          unsigned short* out = (ps & 1) ? ordB : ordA;
          radix_pass<THREADS, MAXR>(E, in, out, ni, lo, lb + 8 * ps, whist, dstart, lds_scan);
          in = out;
        }
        ord = in;
      }
      flatten_tile<THREADS>(E, ord, ni, nlev, off, comp, st, lds_scan, nullptr);
    } else {
      // oversized bucket: stable LSD sort through global scratch, then flatten
      // CAP records at a time, carrying the running state across tiles
      Elem* src = p.elems + off;
      Elem* dst = p.elems2 + off;
      unsigned long long kor = 0, kand = ~0ull;
      for (long long i = threadIdx.x; i < n; i += THREADS) {
        const unsigned long long k = (unsigned long long)(src[i].s - lo);
        kor |= k;
        kand &= k;
      }
      for (int d = 32; d >= 1; d >>= 1) {
        kor |= __shfl_xor(kor, d, 64);
        kand &= __shfl_xor(kand, d, 64);
      }
      const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
      if (lane == 0) { red[0][wave] = kor; red[1][wave] = kand; }
      __syncthreads();
      kor = 0; kand = ~0ull;
      for (int w = 0; w < NW; ++w) { kor |= red[0][w]; kand &= red[1][w]; }
      __syncthreads();
      const unsigned long long vary = kor ^ kand;
      if (vary) {
        const int lb = __ffsll((long long)vary) - 1;
        const int hb = bitlen64(vary);
        const int passes = (hb - lb + 7) >> 3;
        for (int ps = 0; ps < passes; ++ps) {
          const int sh = lb + 8 * ps;
          // global digit histogram -> running bin bases (dcount)
          for (int i = threadIdx.x; i < 256; i += THREADS) dcount[i] = 0;
          __syncthreads();
          for (long long i = threadIdx.x; i < n; i += THREADS)
            atomicAdd(&dcount[((unsigned long long)(src[i].s - lo) >> sh) & 255ull], 1u);
          __syncthreads();
          {
            long long v[1] = {threadIdx.x < 256 ? (long long)dcount[threadIdx.x] : 0}, ex[1], all[1];
            block_excl_scan<THREADS, 1, OpSum>(v, ex, all, 0, lds_scan);
            if (threadIdx.x < 256) dcount[threadIdx.x] = (unsigned int)ex[0];
          }
          __syncthreads();
          for (long long t0 = 0; t0 < n; t0 += CAP) {
            const int cnt = (int)min((long long)CAP, n - t0);
            for (int i = threadIdx.x; i < cnt; i += THREADS) E[i] = src[t0 + i];
            __syncthreads();
            radix_pass<THREADS, MAXR>(E, nullptr, ordA, cnt, lo, sh, whist, dstart, lds_scan);
            for (int q = threadIdx.x; q < cnt; q += THREADS) {
              const unsigned short i = ordA[q];
              const unsigned int d = (unsigned int)(((unsigned long long)(E[i].s - lo) >> sh) & 255ull);
              dst[dcount[d] + (q - dstart[d])] = E[i];
            }
            __syncthreads();
            // advance the bin bases by this tile's digit counts
            if (threadIdx.x < 256) {
              const unsigned int d = threadIdx.x;
              const unsigned int next = d < 255 ? dstart[d + 1] : (unsigned int)cnt;
              dcount[d] += next - dstart[d];
            }
            __syncthreads();
          }
          Elem* t = src;
          src = dst;
          dst = t;
        }
      }
      for (long long t0 = 0; t0 < n; t0 += CAP) {
        const int cnt = (int)min((long long)CAP, n - t0);
        for (int i = threadIdx.x; i < cnt; i += THREADS) E[i] = src[t0 + i];
        __syncthreads();
        flatten_tile<THREADS>(E, nullptr, cnt, nlev, off, comp, st, lds_scan, nullptr);
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

__device__ __forceinline__ double ratio(long long num, long long den, int bit, unsigned int& mask) {
  if (den == 0) {
    mask |= 1u << bit;
    return 1.0;
  }
  return (double)num / (double)den;
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
#pragma unroll
  for (int i = 0; i < 6; ++i) v[i] = wave_red_sum(v[i]);
#pragma unroll
  for (int i = 6; i < 9; ++i) v[i] = wave_red_max(v[i]);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (lane == 0)
    for (int i = 0; i < 9; ++i) lds[wave * 10 + i] = v[i];
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int w = 1; w < THREADS / 64; ++w) {
      for (int i = 0; i < 6; ++i) v[i] += lds[w * 10 + i];
      for (int i = 6; i < 9; ++i) v[i] = lds[w * 10 + i] > v[i] ? lds[w * 10 + i] : v[i];
    }
    Tree t;
    t.E = E;
    t.n = rd.n_hosts;
    t.m = rd.n_devices;
    const long long U = v[0], W = v[1], UW = v[0] + v[1];
    t.sum[0] = U; t.sum[1] = W; t.sum[2] = v[2]; t.sum[3] = v[3];
    t.sum[4] = UW; t.sum[5] = v[6];
    t.sum[6] = v[4]; t.sum[7] = v[5]; t.sum[8] = v[7]; t.sum[9] = v[8];
    unsigned int mask = 0;
    const long long n = rd.n_hosts, m = rd.n_devices;
    t.ratio[0] = ratio(U, n * E, 0, mask);          // eq. 6
    t.ratio[1] = ratio(UW, n * E, 1, mask);         // eq. 7
    t.ratio[2] = ratio(UW, n * v[6], 2, mask);      // eq. 4, U+W useful
    t.ratio[3] = ratio(v[6], E, 3, mask);           // eq. 5, U+W useful
    t.ratio[4] = ratio(U, UW, 4, mask);             // eq. 8
    t.ratio[5] = ratio(v[4], m * E, 5, mask);       // eq. 9
    t.ratio[6] = ratio(v[4], m * v[7], 6, mask);    // eq. 10
    t.ratio[7] = ratio(v[7], v[8], 7, mask);        // eq. 11
    t.ratio[8] = ratio(v[8], E, 8, mask);           // eq. 12
    t.undefined_mask = mask;
    t.reserved = 0;
    trees[blockIdx.x] = t;
  }
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

hipError_t launch_merge(const Plan& p, int cap, hipStream_t st) {
  if (p.n_buckets == 0) return hipSuccess;
  if (cap == 2048)
    hipLaunchKernelGGL((k_merge<256, 2048>), dim3((unsigned)p.n_buckets), dim3(256), 0, st, p);
  else
    hipLaunchKernelGGL((k_merge<256, 4096>), dim3((unsigned)p.n_buckets), dim3(256), 0, st, p);
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
