// Checks the time-bucket geometry (hpop_geom.h) on the host: for segment
// ranges from empty to 2^62 ns and bucket counts from 1 to 2^24, the bucket
// of every probed start is floor(((start - min) >> s0) / wx), lies in
// [0, nb), never decreases with the start, and the start lies inside its
// bucket's [lo, lo + width); times past the range clamp to the last bucket.
#define __host__
#define __device__
#include <cstdio>
#include <cstdlib>
#include <random>

#include "hpop_geom.h"

using namespace hpop;

static int fail(const char* what, unsigned long long span, int nb, unsigned long long rel) {
  std::printf("FAIL %s span=%llu nb=%d rel=%llu\n", what, span, nb, rel);
  return 1;
}

static int check(unsigned long long min_s, unsigned long long span, int nb, std::mt19937_64& rng) {
  SegStats st{min_s, min_s + span, 0, 0};
  SegDesc sd{0, nb, 2};
  const Geom g = make_geom(st, sd);
  if (g.empty || g.nb != nb || g.wx < 1 || (span >> g.s0) >= (1ull << 31)) return fail("geometry", span, nb, 0);
  const unsigned long long width = (unsigned long long)g.wx << g.s0;
  if (seg_narrow(g) != (width <= (1ull << kNarrowShift))) return fail("narrow", span, nb, 0);
  // probes: both ends, bucket edges, and random starts
  unsigned long long probes[64];
  int k = 0;
  probes[k++] = 0;
  probes[k++] = span;
  for (int i = 0; i < 20; ++i) {
    const unsigned long long b = rng() % (unsigned long long)nb;
    const unsigned long long edge = (b * g.wx) << g.s0;
    if (edge <= span) probes[k++] = edge;
    if (edge >= 1 && edge - 1 <= span) probes[k++] = edge - 1;
  }
  while (k < 64) probes[k++] = span ? rng() % (span + 1) : 0;
  long long prev_b = -1;
  unsigned long long prev_r = 0;
  for (int i = 0; i < 64; ++i) {
    const unsigned long long rel = probes[i];
    const long long b = bucket_index(g, rel);
    const unsigned long long want = (rel >> g.s0) / g.wx;
    if (b < 0 || b >= nb || (unsigned long long)b != want) return fail("index", span, nb, rel);
    if (bucket_of_start(g, (long long)(min_s + rel)) != b) return fail("start index", span, nb, rel);
    const long long lo = bucket_lo(g, b);
    const long long t = (long long)(min_s + rel);
    if (lo > t || t - lo >= (long long)width) return fail("inside", span, nb, rel);
    if (i > 0 && rel >= prev_r && b < prev_b) return fail("monotone", span, nb, rel);
    prev_b = b;
    prev_r = rel;
  }
  // past the range: the last bucket
  if (bucket_index(g, span + 1 + (rng() % (1ull << 40))) > nb - 1) return fail("clamp", span, nb, span + 1);
  if (bucket_index(g, ~0ull >> 2) != nb - 1 && (((~0ull >> 2) >> g.s0) / g.wx) >= (unsigned long long)nb)
    return fail("clamp far", span, nb, ~0ull >> 2);
  return 0;
}

int main() {
  std::mt19937_64 rng(12345);
  int cases = 0;
  const int nbs[] = {1, 2, 3, 7, 100, 255, 256, 257, 1000, 1526, 4096, 65535, 1 << 20, (1 << 24) - 1, 1 << 24};
  for (int nb : nbs) {
    for (int bits = 0; bits <= 62; ++bits) {
      for (int rep = 0; rep < 4; ++rep) {
        unsigned long long span = bits == 0 ? 0 : (1ull << (bits - 1)) + (rng() % (1ull << (bits - 1)));
        if (rep == 3 && bits > 0) span = (bits == 62) ? (1ull << 62) - 1 : (1ull << bits) - 1;
        const unsigned long long min_s = rng() % ((1ull << 62) - span);
        if (check(min_s, span, nb, rng)) return 1;
        ++cases;
      }
    }
    // spans below the bucket count, where every bucket is 1 ns
    for (unsigned long long span = 0; span < 300; span += 7) {
      if (check(1700000000000000000ull, span, nb, rng)) return 1;
      ++cases;
    }
  }
  // the division itself, for every width class and numerators at the edges
  for (int i = 0; i < 200000; ++i) {
    Geom g{};
    g.wx = (unsigned int)(1 + (rng() % ((i % 3 == 0) ? 4u : (1u << (1 + rng() % 31)))));
    if (g.wx > (1u << 31)) g.wx = 1u << 31;
    const unsigned long long mv = (1ull << 32) / g.wx;
    g.minv = mv > 0xFFFFFFFFull ? 0xFFFFFFFFu : (unsigned int)mv;
    unsigned int x = (unsigned int)(rng() % (1ull << 31));
    if (i % 4 == 1) x = (unsigned int)(((unsigned long long)(x / g.wx) * g.wx) & 0x7FFFFFFFu);
    if (i % 4 == 2 && x) x = x - 1;
    if (i % 4 == 3) x = (1u << 31) - 1;
    if (geom_div(g, x) != x / g.wx) return fail("div", g.wx, 0, x);
  }
  // an empty segment
  SegStats st{~0ull, 0, 0, 0};
  SegDesc sd{0, 5, 3};
  if (!make_geom(st, sd).empty) return fail("empty", 0, 5, 0);
  std::printf("ok %d\n", cases);
  return 0;
}
