/* Runs the C oracle on one trace read from a binary file, for a build with
 * AddressSanitizer and UndefinedBehaviorSanitizer (test infrastructure).
 *
 * input  (little endian): int32 n_hosts, n_devices; int64 n_events;
 *        int32 resource[n], kind[n]; int64 start[n], end[n];
 *        int32 n_regions; int64 t0[n_regions], t1[n_regions]; int32 threads
 * output: int32 status, then (status 0 only) times, sums, ratios, mask in the
 *        layout of oracle_compute. */
#include <stdio.h>
#include <stdlib.h>

#include "hpop_oracle.h"

static void* take(FILE* f, size_t n, size_t sz) {
  void* p = malloc(n * sz + 1);
  if (!p || fread(p, sz, n, f) != n) {
    fprintf(stderr, "short input\n");
    exit(2);
  }
  return p;
}

int main(int argc, char** argv) {
  if (argc != 3) return 2;
  FILE* f = fopen(argv[1], "rb");
  if (!f) return 2;
  int32_t* hdr = take(f, 2, 4);
  int64_t* np = take(f, 1, 8);
  const int64_t n = *np;
  int32_t* res = take(f, (size_t)n, 4);
  int32_t* kind = take(f, (size_t)n, 4);
  int64_t* st = take(f, (size_t)n, 8);
  int64_t* en = take(f, (size_t)n, 8);
  int32_t* nrp = take(f, 1, 4);
  const int32_t nreg = *nrp;
  int64_t* t0 = take(f, (size_t)nreg, 8);
  int64_t* t1 = take(f, (size_t)nreg, 8);
  int32_t* thr = take(f, 1, 4);
  fclose(f);
  const size_t R = (size_t)hdr[0] + (size_t)hdr[1];
  int64_t* times = calloc((size_t)nreg * R * 4 + 1, 8);
  int64_t* sums = calloc((size_t)nreg * 10 + 1, 8);
  double* ratios = calloc((size_t)nreg * 9 + 1, 8);
  uint32_t* mask = calloc((size_t)nreg + 1, 4);
  const int32_t rc = oracle_compute(hdr[0], hdr[1], n, res, kind, st, en, nreg, t0, t1, *thr, times, sums, ratios,
                                    mask);
  FILE* o = fopen(argv[2], "wb");
  if (!o) return 2;
  fwrite(&rc, 4, 1, o);
  if (rc == 0) {
    fwrite(times, 8, (size_t)nreg * R * 4, o);
    fwrite(sums, 8, (size_t)nreg * 10, o);
    fwrite(ratios, 8, (size_t)nreg * 9, o);
    fwrite(mask, 4, (size_t)nreg, o);
  }
  fclose(o);
  free(hdr); free(np); free(res); free(kind); free(st); free(en); free(nrp); free(t0); free(t1); free(thr);
  free(times); free(sums); free(ratios); free(mask);
  return 0;
}
