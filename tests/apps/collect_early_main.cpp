// Host program for the start-up regression case of libhpop_collect.so (see
// collect_early_lib.cpp): makes HIP runtime calls, polls, and checks that
// every call was recorded and that the process ends cleanly.
#include <hip/hip_runtime.h>

#include <cstdio>

#include "hpop_collect.h"

int main() {
  int n = -1;
  for (int i = 0; i < 1000; ++i) (void)hipGetDeviceCount(&n);
  int64_t f = 0;
  const hpop_status st = hpop_collect_poll(&f);
  const long long calls = (long long)hpop_collect_count(0, HPOP_HOST_OFFLOAD);
  std::printf("active=%d poll=%d offload_calls=%lld\n", hpop_collect_active(), (int)st, calls);
  return (hpop_collect_active() == 1 && st == HPOP_OK && calls >= 1000) ? 0 : 1;
}
