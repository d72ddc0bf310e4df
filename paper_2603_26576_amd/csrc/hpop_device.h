// Device building blocks shared by the trace-reduction and serving kernels.
#pragma once
#include <hip/hip_runtime.h>

#include <climits>

#include "hpop_geom.h"
#include "hpop_internal.h"

namespace hpop {

// ----------------------------------------------------------------------------
// small device helpers
// ----------------------------------------------------------------------------

__device__ __forceinline__ int bitlen64(unsigned long long x) { return x ? 64 - __clzll((long long)x) : 0; }

__device__ __forceinline__ bool rec_valid(long long s, long long e) {
  return s >= 0 && s <= e && e < kTimeLimit;
}

__device__ __forceinline__ Geom seg_geom(const Plan& p, long long seg) { return p.geom[seg]; }

// The components of one bucket at one level, in either storage form.
struct CompView {
  const Comp* wide;     // wide segments
  const CompN* narrow;  // narrow segments: relative to lo
  long long lo;
  __device__ __forceinline__ long long cs(long long k) const {
    return narrow ? lo + (long long)narrow[k].cs : wide[k].cs;
  }
  __device__ __forceinline__ long long pl(long long k) const {
    return narrow ? (long long)narrow[k].pl : wide[k].pl;
  }
};

__device__ __forceinline__ CompView comp_view(const Plan& p, const Geom& g, long long bucket_begin, long long gb,
                                              int l) {
  CompView v;
  const long long off = (long long)p.offsets[gb];
  if (seg_narrow(g)) {
    v.wide = nullptr;
    v.narrow = p.compn[l] + off;
    v.lo = bucket_lo(g, gb - bucket_begin);
  } else {
    v.wide = p.comp[l] + off;
    v.narrow = nullptr;
    v.lo = 0;
  }
  return v;
}

// The records of one bucket: n8 in the 8 B form, n16 in the 16 B form.
struct BucketRecs {
  const uint2* narrow;
  const Elem* wide;
  int n8, n16;
  bool overflow;  // more records than fixed slots: the build is redone with exact offsets
};

__device__ __forceinline__ BucketRecs bucket_recs(const Plan& p, long long gb) {
  BucketRecs r;
  const unsigned long long cu = p.cursor[gb];
  r.n8 = (int)(unsigned int)cu;
  r.n16 = (int)(cu >> 32);
  long long ub, ucap;
  if (p.slot_cap) {
    ub = 2 * gb * (long long)p.slot_cap;
    ucap = 2 * (long long)p.slot_cap;
    r.overflow = (long long)r.n8 + r.n16 > (long long)p.slot_cap;
  } else {
    ub = 2 * (long long)p.offsets[gb];
    ucap = 2 * ((long long)r.n8 + r.n16);
    r.overflow = false;
  }
  const uint2* u = (const uint2*)p.elems;
  r.narrow = u + ub;
  r.wide = (const Elem*)(u + ub + ucap) - r.n16;
  return r;
}

// The 16 B form of an 8 B record of the bucket starting at lo. A clamped end
// (field 0xFFFFFFFF) becomes the largest end of the bucket's records of the
// same rank (maxend: per rank): every clamped record of a rank reaches past
// lo + 2^32 - 2 and starts before lo + 2^30, so they all overlap, and giving
// each the largest of their ends leaves the union of every level unchanged.
__device__ __forceinline__ Elem widen(uint2 x, long long lo, const unsigned long long* maxend) {
  Elem el;
  const unsigned int slot = x.x & 3u;
  el.s = lo + (long long)(x.x >> 2);
  const long long e = x.y == 0xFFFFFFFFu ? (long long)maxend[slot] : lo + (long long)x.y - 1;
  el.e_slot = (long long)((unsigned long long)e | ((unsigned long long)slot << kSlotShift));
  return el;
}

// bucket of a valid record start inside its segment (min_s <= start <= max_s)
__device__ __forceinline__ int bucket_of(long long s, const Geom& g) { return bucket_of_start(g, s); }

// index of the last entry with key <= x in a sorted array of n int64 (n >= 1, a[0] <= x)
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

// ----------------------------------------------------------------------------
// wave-level scans with DPP lane shifts (no LDS round trips)
// ----------------------------------------------------------------------------

// DPP controls of the gfx9 family: row_shr:n, row_bcast:15 / :31, wave_shr:1
constexpr int kDppRowShr1 = 0x111, kDppRowShr2 = 0x112, kDppRowShr4 = 0x114, kDppRowShr8 = 0x118;
constexpr int kDppRowBcast15 = 0x142, kDppRowBcast31 = 0x143, kDppWaveShr1 = 0x138;

// v from the lane selected by CTRL, or `old` where that lane is outside the
// row/bank masks or has no source lane
template <int CTRL, int ROW_MASK, int BANK_MASK>
__device__ __forceinline__ long long dpp64(long long old, long long v) {
  const int lo = __builtin_amdgcn_update_dpp((int)old, (int)v, CTRL, ROW_MASK, BANK_MASK, false);
  const int hi = __builtin_amdgcn_update_dpp((int)(old >> 32), (int)(v >> 32), CTRL, ROW_MASK, BANK_MASK, false);
  return (long long)(((unsigned long long)(unsigned int)hi << 32) | (unsigned long long)(unsigned int)lo);
}

__device__ __forceinline__ long long readlane64(long long v, int lane) {
  const int lo = __builtin_amdgcn_readlane((int)v, lane);
  const int hi = __builtin_amdgcn_readlane((int)(v >> 32), lane);
  return (long long)(((unsigned long long)(unsigned int)hi << 32) | (unsigned long long)(unsigned int)lo);
}

// Exclusive scan over the 64 lanes (lane order) with identity `id`, and the total.
template <class Op>
__device__ __forceinline__ long long wave_excl_scan_dpp(long long x, long long id, long long& total) {
  x = Op::apply(x, dpp64<kDppRowShr1, 0xf, 0xf>(id, x));
  x = Op::apply(x, dpp64<kDppRowShr2, 0xf, 0xf>(id, x));
  x = Op::apply(x, dpp64<kDppRowShr4, 0xf, 0xf>(id, x));
  x = Op::apply(x, dpp64<kDppRowShr8, 0xf, 0xf>(id, x));
  x = Op::apply(x, dpp64<kDppRowBcast15, 0xa, 0xf>(id, x));
  x = Op::apply(x, dpp64<kDppRowBcast31, 0xc, 0xf>(id, x));
  total = readlane64(x, 63);
  return dpp64<kDppWaveShr1, 0xf, 0xf>(id, x);
}

struct OpMaxU {
  __device__ static unsigned int apply(unsigned int a, unsigned int b) { return a > b ? a : b; }
};
struct OpSumU {
  __device__ static unsigned int apply(unsigned int a, unsigned int b) { return a + b; }
};

template <int CTRL, int ROW_MASK, int BANK_MASK>
__device__ __forceinline__ unsigned int dpp32(unsigned int old, unsigned int v) {
  return (unsigned int)__builtin_amdgcn_update_dpp((int)old, (int)v, CTRL, ROW_MASK, BANK_MASK, false);
}

// Exclusive scan over the 64 lanes (lane order) with identity `id`, and the total.
template <class Op>
__device__ __forceinline__ unsigned int wave_excl_scan_u32(unsigned int x, unsigned int id, unsigned int& total) {
  x = Op::apply(x, dpp32<kDppRowShr1, 0xf, 0xf>(id, x));
  x = Op::apply(x, dpp32<kDppRowShr2, 0xf, 0xf>(id, x));
  x = Op::apply(x, dpp32<kDppRowShr4, 0xf, 0xf>(id, x));
  x = Op::apply(x, dpp32<kDppRowShr8, 0xf, 0xf>(id, x));
  x = Op::apply(x, dpp32<kDppRowBcast15, 0xa, 0xf>(id, x));
  x = Op::apply(x, dpp32<kDppRowBcast31, 0xc, 0xf>(id, x));
  total = (unsigned int)__builtin_amdgcn_readlane((int)x, 63);
  return dpp32<kDppWaveShr1, 0xf, 0xf>(id, x);
}

struct OpMinI {
  __device__ static int apply(int a, int b) { return a < b ? a : b; }
};
struct OpMaxI {
  __device__ static int apply(int a, int b) { return a > b ? a : b; }
};
struct OpMaxU32 {  // unsigned maximum on int lanes
  __device__ static int apply(int a, int b) { return (unsigned int)a > (unsigned int)b ? a : b; }
};
struct OpOrI {
  __device__ static int apply(int a, int b) { return a | b; }
};

// Reduction over the 64 lanes with DPP row shifts (no LDS round trips); every
// lane receives the result.
template <class Op>
__device__ __forceinline__ int wave_reduce_i32(int x, int id) {
  x = Op::apply(x, __builtin_amdgcn_update_dpp(id, x, kDppRowShr1, 0xf, 0xf, false));
  x = Op::apply(x, __builtin_amdgcn_update_dpp(id, x, kDppRowShr2, 0xf, 0xf, false));
  x = Op::apply(x, __builtin_amdgcn_update_dpp(id, x, kDppRowShr4, 0xf, 0xf, false));
  x = Op::apply(x, __builtin_amdgcn_update_dpp(id, x, kDppRowShr8, 0xf, 0xf, false));
  x = Op::apply(x, __builtin_amdgcn_update_dpp(id, x, kDppRowBcast15, 0xa, 0xf, false));
  x = Op::apply(x, __builtin_amdgcn_update_dpp(id, x, kDppRowBcast31, 0xc, 0xf, false));
  return __builtin_amdgcn_readlane(x, 63);
}

template <class Op>
__device__ __forceinline__ long long wave_reduce_i64(long long x, long long id) {
  long long total;
  (void)wave_excl_scan_dpp<Op>(x, id, total);
  return total;
}

// Block-wide exclusive scan of K int64 lanes per thread (thread order), with totals.
// `lds` holds NW*K int64. Contains barriers: call from uniform control flow.
template <int THREADS, int K, class Op>
__device__ __forceinline__ void block_excl_scan(const long long (&v)[K], long long (&excl)[K],
                                                long long (&total)[K], long long ident, long long* lds) {
  constexpr int NW = THREADS / 64;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  long long ex[K];
#pragma unroll
  for (int k = 0; k < K; ++k) {
    long long tot;
    ex[k] = wave_excl_scan_dpp<Op>(v[k], ident, tot);
    if (lane == 0) lds[wave * K + k] = tot;
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
    excl[k] = Op::apply(pre, ex[k]);
    total[k] = tot;
  }
  __syncthreads();
}

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
// Writes components of each level at comp[l][off + R], or in the narrow form
// relative to `nlo` at compn[l][off + R] when compn is given; advances `st`.
template <int THREADS>
__device__ __forceinline__ void flatten_tile(const Elem* E, const unsigned short* ord, int n, int nlev,
                                             long long off, Comp* const* comp, CompN* const* compn, long long nlo,
                                             FlatState& st, long long* lds_scan, long long* lds_bc) {
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
            if (compn) {
              CompN c;
              c.cs = (uint32_t)(s - nlo);
              c.pl = (uint32_t)P[l];
              compn[l][off + R[l]] = c;
            } else {
              Comp c;
              c.cs = s;
              c.pl = P[l];
              comp[l][off + R[l]] = c;
            }
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

__device__ __forceinline__ double ratio(long long num, long long den, int bit, unsigned int& mask) {
  if (den == 0) {
    mask |= 1u << bit;
    return 1.0;
  }
  return (double)num / (double)den;
}


// LDS of the sorting workgroups (one bucket or one list tile at a time).
template <int THREADS, int CAP>
struct SortSmem {
  static constexpr int NW = THREADS / 64;
  Elem E[CAP];
  unsigned short ordA[CAP];
  unsigned short ordB[CAP];
  unsigned int whist[NW * 256];
  unsigned int dstart[256];
  unsigned int dcount[256];
  long long lds_scan[NW * 6];
  unsigned long long red[2][NW];
};

// Block-wide OR and AND of per-thread key accumulators: the bits in which keys differ.
template <int THREADS>
__device__ __forceinline__ unsigned long long block_vary(unsigned long long kor, unsigned long long kand,
                                                         unsigned long long (*red)[THREADS / 64]) {
  constexpr int NW = THREADS / 64;
  for (int d = 32; d >= 1; d >>= 1) {
    kor |= __shfl_xor(kor, d, 64);
    kand &= __shfl_xor(kand, d, 64);
  }
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) {
    red[0][wave] = kor;
    red[1][wave] = kand;
  }
  __syncthreads();
  kor = 0;
  kand = ~0ull;
  for (int w = 0; w < NW; ++w) {
    kor |= red[0][w];
    kand &= red[1][w];
  }
  __syncthreads();
  return kor ^ kand;
}

// Sort sm.E[0..n) (n <= CAP, already in LDS and visible to the block) by
// start - lo. Returns the sorted order, or nullptr when E is already in an
// acceptable order (all starts equal). Only the bits that vary are sorted.
template <int THREADS, int CAP>
__device__ const unsigned short* sort_lds(SortSmem<THREADS, CAP>& sm, int n, long long lo) {
  constexpr int MAXR = CAP / THREADS;
  unsigned long long kor = 0, kand = ~0ull;
  for (int i = threadIdx.x; i < n; i += THREADS) {
    const unsigned long long k = (unsigned long long)(sm.E[i].s - lo);
    kor |= k;
    kand &= k;
  }
  const unsigned long long vary = block_vary<THREADS>(kor, kand, sm.red);
  if (!vary) return nullptr;
  const int lb = __ffsll((long long)vary) - 1;
  const int hb = bitlen64(vary);
  const int passes = (hb - lb + 7) >> 3;
  const unsigned short* in = nullptr;  // identity for the first pass
  for (int ps = 0; ps < passes; ++ps) {
    unsigned short* out = (ps & 1) ? sm.ordB : sm.ordA;
    radix_pass<THREADS, MAXR>(sm.E, in, out, n, lo, lb + 8 * ps, sm.whist, sm.dstart, sm.lds_scan);
    in = out;
  }
  return in;
}

// Stable LSD sort of n records in global memory by start - lo, CAP records of
// LDS at a time; dst is scratch of the same size. Returns the buffer that
// holds the sorted records (src or dst).
template <int THREADS, int CAP>
__device__ Elem* sort_global(SortSmem<THREADS, CAP>& sm, Elem* src, Elem* dst, long long n, long long lo) {
  constexpr int MAXR = CAP / THREADS;
  unsigned long long kor = 0, kand = ~0ull;
  for (long long i = threadIdx.x; i < n; i += THREADS) {
    const unsigned long long k = (unsigned long long)(src[i].s - lo);
    kor |= k;
    kand &= k;
  }
  const unsigned long long vary = block_vary<THREADS>(kor, kand, sm.red);
  if (!vary) return src;
  const int lb = __ffsll((long long)vary) - 1;
  const int hb = bitlen64(vary);
  const int passes = (hb - lb + 7) >> 3;
  for (int ps = 0; ps < passes; ++ps) {
    const int sh = lb + 8 * ps;
    // digit histogram of all records -> running output base per digit
    for (int i = threadIdx.x; i < 256; i += THREADS) sm.dcount[i] = 0;
    __syncthreads();
    for (long long i = threadIdx.x; i < n; i += THREADS)
      atomicAdd(&sm.dcount[((unsigned long long)(src[i].s - lo) >> sh) & 255ull], 1u);
    __syncthreads();
    {
      long long v[1] = {threadIdx.x < 256 ? (long long)sm.dcount[threadIdx.x] : 0}, ex[1], all[1];
      block_excl_scan<THREADS, 1, OpSum>(v, ex, all, 0, sm.lds_scan);
      if (threadIdx.x < 256) sm.dcount[threadIdx.x] = (unsigned int)ex[0];
    }
    __syncthreads();
    for (long long t0 = 0; t0 < n; t0 += CAP) {
      const int cnt = (int)min((long long)CAP, n - t0);
      for (int i = threadIdx.x; i < cnt; i += THREADS) sm.E[i] = src[t0 + i];
      __syncthreads();
      radix_pass<THREADS, MAXR>(sm.E, nullptr, sm.ordA, cnt, lo, sh, sm.whist, sm.dstart, sm.lds_scan);
      for (int q = threadIdx.x; q < cnt; q += THREADS) {
        const unsigned short i = sm.ordA[q];
        const unsigned int d = (unsigned int)(((unsigned long long)(sm.E[i].s - lo) >> sh) & 255ull);
        dst[sm.dcount[d] + (q - sm.dstart[d])] = sm.E[i];
      }
      __syncthreads();
      if (threadIdx.x < 256) {
        const unsigned int d = threadIdx.x;
        const unsigned int next = d < 255 ? sm.dstart[d + 1] : (unsigned int)cnt;
        sm.dcount[d] += next - sm.dstart[d];
      }
      __syncthreads();
    }
    Elem* t = src;
    src = dst;
    dst = t;
  }
  return src;
}

// Ratios of one region's metric trees from exact integer aggregates.
// v: sumU, sumW, sumMPI, sumOther, sumK, sumM, maxUW, maxK, maxKM
__device__ __forceinline__ Tree make_tree(long long E, int n_hosts, int n_devices, const long long (&v)[9]) {
  Tree t;
  t.E = E;
  t.n = n_hosts;
  t.m = n_devices;
  const long long U = v[0], W = v[1], UW = v[0] + v[1];
  t.sum[0] = U;
  t.sum[1] = W;
  t.sum[2] = v[2];
  t.sum[3] = v[3];
  t.sum[4] = UW;
  t.sum[5] = v[6];
  t.sum[6] = v[4];
  t.sum[7] = v[5];
  t.sum[8] = v[7];
  t.sum[9] = v[8];
  unsigned int mask = 0;
  const long long n = n_hosts, m = n_devices;
  t.ratio[0] = ratio(U, n * E, 0, mask);        // eq. 6
  t.ratio[1] = ratio(UW, n * E, 1, mask);       // eq. 7
  t.ratio[2] = ratio(UW, n * v[6], 2, mask);    // eq. 4, U+W useful
  t.ratio[3] = ratio(v[6], E, 3, mask);         // eq. 5, U+W useful
  t.ratio[4] = ratio(U, UW, 4, mask);           // eq. 8
  t.ratio[5] = ratio(v[4], m * E, 5, mask);     // eq. 9
  t.ratio[6] = ratio(v[4], m * v[7], 6, mask);  // eq. 10
  t.ratio[7] = ratio(v[7], v[8], 7, mask);      // eq. 11
  t.ratio[8] = ratio(v[8], E, 8, mask);         // eq. 12
  t.undefined_mask = mask;
  t.reserved = 0;
  return t;
}

// Block reduction of per-thread resource state times into a tree (thread 0
// returns it). Per thread: host rows add U, W, MPI, Other; device rows K, M.
template <int THREADS>
__device__ __forceinline__ void block_tree(long long (&v)[9], long long* lds) {
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
  }
  __syncthreads();
}

}  // namespace hpop
