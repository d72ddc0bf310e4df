// Time-bucket geometry of a segment (see SegGeom): the same arithmetic on
// the device (kernels) and the host (diagnostics, CPU tests).
#pragma once
#include <stdint.h>

#include "hpop_internal.h"

namespace hpop {

typedef SegGeom Geom;

__host__ __device__ inline int geom_bitlen64(unsigned long long x) {
  int n = 0;
  while (x) {
    ++n;
    x >>= 1;
  }
  return n;
}

// The bucket geometry of a segment from its start range and bucket count
// (the geometry kernel computes it once per build; kernels read p.geom).
__host__ __device__ inline Geom make_geom(const SegStats& st, const SegDesc& sd) {
  Geom g;
  g.empty = st.min_s > st.max_s ? 1 : 0;
  g.min_s = (long long)st.min_s;
  g.nb = sd.nb;
  const unsigned long long span = g.empty ? 0ull : st.max_s - st.min_s;
  const int bl = geom_bitlen64(span);
  g.s0 = bl > 31 ? bl - 31 : 0;  // xmax < 2^31, so wx = xmax / nb + 1 <= 2^31
  const unsigned int xmax = (unsigned int)(span >> g.s0);
  g.wx = xmax / (unsigned int)sd.nb + 1u;
  // floor(2^32 / wx), at most 2^32 - 1 (wx = 1): the high half of x * minv is
  // then x / wx or one less
  const unsigned long long mv = (1ull << 32) / g.wx;
  g.minv = mv > 0xFFFFFFFFull ? 0xFFFFFFFFu : (unsigned int)mv;
  g.pad = 0;
  return g;
}

// first time of bucket b (segment-relative) of a segment
__host__ __device__ inline long long bucket_lo(const Geom& g, long long b) {
  // b * wx <= (nb - 1) * wx < 2^31 + nb: 32 bits
  return g.min_s + (long long)((unsigned long long)((unsigned int)b * g.wx) << g.s0);
}

// floor(x / wx) for x < 2^31: the high half of x * minv is the quotient or
// one less; the remainder decides (it stays below 2 wx <= 2^32)
__host__ __device__ inline unsigned int geom_div(const Geom& g, unsigned int x) {
  unsigned int q = (unsigned int)(((unsigned long long)x * g.minv) >> 32);
  return q + (x - q * g.wx >= g.wx ? 1u : 0u);
}

// bucket of a time rel = t - min_s >= 0 ns after the segment's first start,
// clamped to the last bucket
__host__ __device__ inline long long bucket_index(const Geom& g, unsigned long long rel) {
  const unsigned long long x64 = rel >> g.s0;
  if (x64 >= (1ull << 31)) return g.nb - 1;
  const unsigned int q = geom_div(g, (unsigned int)x64);
  return q < (unsigned int)g.nb ? (long long)q : (long long)g.nb - 1;
}

// bucket of a record start in [min_s, max_s] (no clamping needed there)
__host__ __device__ inline int bucket_of_start(const Geom& g, long long s) {
  return (int)geom_div(g, (unsigned int)((unsigned long long)(s - g.min_s) >> g.s0));
}

// buckets at most 2^kNarrowShift ns wide: records and components fit the 8 B forms
__host__ __device__ inline bool seg_narrow(const Geom& g) {
  return ((unsigned long long)g.wx << g.s0) <= (1ull << kNarrowShift);
}

}  // namespace hpop
