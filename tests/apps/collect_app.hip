// Test application for the hpop_collect tool: a fixed pattern per iteration
// (host work, a host-to-device copy, one kernel on each of two streams, a
// fill, a device-to-host copy, a device synchronisation), so the collected
// records can be checked against what the program did. With LIVE_EVERY > 0
// it also feeds the records to an hpop server while it runs, one region per
// LIVE_EVERY iterations, and keeps every answer.
//
//   collect_app ITERS LIVE_EVERY OUT_PREFIX
//
// Writes OUT_PREFIX.trace (hpop_collect_write), OUT_PREFIX.kern (float32 ms
// per kernel, from HIP events, two per iteration: stream 0 then stream 1),
// and with LIVE_EVERY > 0 OUT_PREFIX.live: per region, int64 t0, t1, the
// cumulative record count of every (resource, kind) pair (resource-major,
// 5 kinds each), then the region's and the session's hpop_metric_tree.
// Prints one summary line; exits non-zero on any error. The line also holds
// what the tool costs the program: call_ns, the mean time of a cheap runtime
// call (hipGetDevice, each one traced when the tool is active), iter_us, the
// mean time of one iteration, and in live mode the latency of each region
// (poll, copy, submit and wait). With HPOP_APP_ALLOW_INACTIVE=1 in the
// environment the program also runs without the tool (LIVE_EVERY must be 0;
// no trace is written), for the same timings without tracing.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cstdio>
#include <cstdlib>
#include <string>
#include <vector>

#include "hpop.h"
#include "hpop_collect.h"

#define CK(x)                                                                        \
  do {                                                                               \
    hipError_t e_ = (x);                                                             \
    if (e_ != hipSuccess) {                                                          \
      std::fprintf(stderr, "%s failed: %s\n", #x, hipGetErrorString(e_));            \
      std::exit(2);                                                                  \
    }                                                                                \
  } while (0)

#define CKH(x)                                                                       \
  do {                                                                               \
    hpop_status s_ = (x);                                                            \
    if (s_ != HPOP_OK) {                                                             \
      std::fprintf(stderr, "%s failed: %s\n", #x, hpop_status_string(s_));              \
      std::exit(3);                                                                  \
    }                                                                                \
  } while (0)

// about `rounds` x 100 x 64 cycles of sleeping, then one word written by no lane in practice
__global__ void spin(unsigned int* out, int rounds) {
  unsigned int x = threadIdx.x + 1u;
  for (int i = 0; i < rounds; ++i) {
    __builtin_amdgcn_s_sleep(100);
    x = x * 1664525u + 1013904223u;
  }
  if (x == 0u) out[threadIdx.x] = x;
}

struct Feed {
  hpop_server* srv = nullptr;
  int32_t sid = -1;
  int n_res = 0;
  std::vector<int64_t> taken;  // per (resource, kind) pair
  int64_t prev = 0;            // end of the last region
  FILE* out = nullptr;
  int regions = 0;
  std::vector<double> lat_us;   // per region: poll to answer
  std::vector<double> poll_us;  // per region: the poll alone
  double records = 0;           // submitted in all regions

  void step() {
    const auto c0 = std::chrono::steady_clock::now();
    int64_t f = 0;
    CKH(hpop_collect_poll(&f));
    poll_us.push_back(std::chrono::duration<double, std::micro>(std::chrono::steady_clock::now() - c0).count());
    if (f <= prev) return;
    std::vector<std::vector<int64_t>> keep;
    std::vector<hpop_event_chunk> chunks;
    for (int r = 0; r < n_res; ++r)
      for (int k = 0; k < 5; ++k) {
        if ((r == 0) != (k <= HPOP_HOST_MPI)) continue;
        const size_t i = (size_t)r * 5 + k;
        const int64_t c = hpop_collect_count(r, k);
        const int64_t n = c - taken[i];
        if (n <= 0) continue;
        keep.emplace_back(2 * n);
        int64_t* s = keep.back().data();
        CKH(hpop_collect_copy(r, k, taken[i], n, s, s + n));
        chunks.push_back(hpop_event_chunk{r, k, s, s + n, n});
        taken[i] = c;
        records += (double)n;
      }
    uint64_t ticket = 0;
    CKH(hpop_server_submit(srv, sid, chunks.data(), (int32_t)chunks.size(), HPOP_MEM_HOST, prev, f, &ticket));
    hpop_metric_tree reg{}, glob{};
    CKH(hpop_server_wait(srv, ticket, -1, &reg, &glob));
    lat_us.push_back(std::chrono::duration<double, std::micro>(std::chrono::steady_clock::now() - c0).count());
    const int64_t span[2] = {prev, f};
    std::fwrite(span, sizeof span, 1, out);
    std::fwrite(taken.data(), sizeof(int64_t), taken.size(), out);
    std::fwrite(&reg, sizeof reg, 1, out);
    std::fwrite(&glob, sizeof glob, 1, out);
    prev = f;
    ++regions;
  }
};

int main(int argc, char** argv) {
  if (argc != 4) {
    std::fprintf(stderr, "usage: collect_app ITERS LIVE_EVERY OUT_PREFIX\n");
    return 1;
  }
  const int iters = std::atoi(argv[1]);
  const int live_every = std::atoi(argv[2]);
  const std::string prefix = argv[3];
  std::setvbuf(stdout, nullptr, _IOLBF, 0);  // a failure later on keeps what was printed
  CK(hipSetDevice(0));
  const char* allow = std::getenv("HPOP_APP_ALLOW_INACTIVE");
  const bool active = hpop_collect_active() != 0;
  if (!active && !(allow && allow[0] == '1' && live_every == 0)) {
    std::fprintf(stderr, "the hpop_collect tool is not active in this process\n");
    return 4;
  }
  std::printf("collect_app: tool %s, %d device(s)\n", active ? "active" : "not loaded", hpop_collect_devices());
  // a cheap runtime call, traced like any other when the tool is active
  const int n_calls = 20000;
  int dev = -1;
  const auto q0 = std::chrono::steady_clock::now();
  for (int i = 0; i < n_calls; ++i) CK(hipGetDevice(&dev));
  const double call_ns =
      std::chrono::duration<double, std::nano>(std::chrono::steady_clock::now() - q0).count() / n_calls;
  const size_t bytes = 4u << 20;
  void *d0 = nullptr, *d1 = nullptr, *h0 = nullptr, *h1 = nullptr;
  CK(hipMalloc(&d0, bytes));
  CK(hipMalloc(&d1, bytes));
  CK(hipHostMalloc(&h0, bytes, hipHostMallocDefault));
  CK(hipHostMalloc(&h1, bytes, hipHostMallocDefault));
  hipStream_t s0, s1;
  CK(hipStreamCreate(&s0));
  CK(hipStreamCreate(&s1));
  std::vector<hipEvent_t> ev((size_t)4 * iters);
  for (auto& e : ev) CK(hipEventCreate(&e));

  Feed feed;
  if (live_every > 0) {
    hpop_server_config cfg{};
    cfg.max_sessions = 2;
    cfg.max_inflight = 4;
    cfg.queue_capacity = 16;
    cfg.mem_budget_bytes = 256ll << 20;
    CKH(hpop_server_create(&cfg, &feed.srv));
    feed.n_res = 1 + hpop_collect_devices();
    CKH(hpop_server_open_session(feed.srv, 1, feed.n_res - 1, hpop_collect_begin(), &feed.sid));
    feed.taken.assign((size_t)feed.n_res * 5, 0);
    feed.prev = hpop_collect_begin();
    feed.out = std::fopen((prefix + ".live").c_str(), "wb");
    if (!feed.out) return 5;
  }

  double busy_ns = 0;
  const auto l0 = std::chrono::steady_clock::now();
  for (int it = 0; it < iters; ++it) {
    const auto b0 = std::chrono::steady_clock::now();
    while (std::chrono::steady_clock::now() - b0 < std::chrono::microseconds(150)) {
    }
    busy_ns += std::chrono::duration<double, std::nano>(std::chrono::steady_clock::now() - b0).count();
    CK(hipMemcpyAsync(d0, h0, bytes, hipMemcpyHostToDevice, s0));
    CK(hipEventRecord(ev[4 * it], s0));
    spin<<<1, 64, 0, s0>>>((unsigned int*)d1, 40);
    CK(hipGetLastError());
    CK(hipEventRecord(ev[4 * it + 1], s0));
    CK(hipEventRecord(ev[4 * it + 2], s1));
    spin<<<1, 64, 0, s1>>>((unsigned int*)d1 + 64, 25);
    CK(hipGetLastError());
    CK(hipEventRecord(ev[4 * it + 3], s1));
    CK(hipMemsetAsync((char*)d1 + (1u << 20), 0, 1u << 20, s1));
    CK(hipMemcpyAsync(h1, d0, bytes, hipMemcpyDeviceToHost, s1));
    CK(hipDeviceSynchronize());
    if (live_every > 0 && (it + 1) % live_every == 0) feed.step();
  }
  const double iter_us =
      std::chrono::duration<double, std::micro>(std::chrono::steady_clock::now() - l0).count() / std::max(1, iters);
  if (live_every > 0) {
    CKH(hpop_collect_flush());  // the last region takes every record
    feed.step();
    std::fclose(feed.out);
    CKH(hpop_server_destroy(feed.srv));
  }

  std::printf("collect_app: %d iterations done\n", iters);
  std::vector<float> ms((size_t)2 * iters);
  for (int k = 0; k < 2 * iters; ++k) CK(hipEventElapsedTime(&ms[k], ev[2 * k], ev[2 * k + 1]));
  FILE* fk = std::fopen((prefix + ".kern").c_str(), "wb");
  if (!fk) return 5;
  std::fwrite(ms.data(), sizeof(float), ms.size(), fk);
  std::fclose(fk);
  for (auto& e : ev) CK(hipEventDestroy(e));
  CK(hipStreamDestroy(s0));
  CK(hipStreamDestroy(s1));
  CK(hipFree(d0));
  CK(hipFree(d1));
  CK(hipHostFree(h0));
  CK(hipHostFree(h1));
  CK(hipDeviceSynchronize());
  if (active) {
    CKH(hpop_collect_flush());
    int64_t f = 0;
    CKH(hpop_collect_poll(&f));
    CKH(hpop_collect_write((prefix + ".trace").c_str()));
  }
  std::vector<double> lat = feed.lat_us;
  std::sort(lat.begin(), lat.end());
  const double p50 = lat.empty() ? 0.0 : lat[lat.size() / 2], mx = lat.empty() ? 0.0 : lat.back();
  std::vector<double> pl = feed.poll_us;
  std::sort(pl.begin(), pl.end());
  const double poll_p50 = pl.empty() ? 0.0 : pl[pl.size() / 2];
  std::printf(
      "collect_app iters=%d kernels=%d fills=%d copies=%d busy_ns=%.0f regions=%d dropped=%lld call_ns=%.1f "
      "iter_us=%.1f live_p50_us=%.1f live_max_us=%.1f live_poll_p50_us=%.1f live_records=%.0f\n",
      iters, 2 * iters, iters, 2 * iters, busy_ns, feed.regions, (long long)hpop_collect_dropped(), call_ns, iter_us,
      p50, mx, poll_p50, feed.records);
  return 0;
}
