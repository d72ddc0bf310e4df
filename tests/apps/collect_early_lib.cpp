// Starts the HIP runtime from a library constructor. Linked ahead of
// libhpop_collect.so, it makes rocprofiler-sdk configure the tool before the
// tool library's own constructors have run (a regression case: the tool's
// state must not depend on them).
#include <hip/hip_runtime.h>

#include <cstdio>

__attribute__((constructor)) static void start_hip_early() {
  int n = -1;
  (void)hipGetDeviceCount(&n);
  std::fprintf(stderr, "collect_early: HIP started from a constructor\n");
}
