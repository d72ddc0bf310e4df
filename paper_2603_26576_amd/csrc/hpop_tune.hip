// Autotuner: picks the bucket size, on-chip bucket capacity and streaming tile
// of the reduction kernels by timing full builds on the caller's workload, and
// remembers the choice per workload size class in a small JSON file.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <map>
#include <string>
#include <vector>

#include "hpop.h"
#include "hpop_runtime.h"
#include "hpop_tune_cache.h"

using namespace hpop;

namespace {

// size class: log2 of records and of resources, rounded
std::string size_key(hpop_session* const* ss, int k) {
  long long ev = 0, res = 0;
  for (int i = 0; i < k; ++i) {
    ev += ss[i]->n_events;
    res += ss[i]->n_hosts + ss[i]->n_devices;
  }
  char buf[96];
  snprintf(buf, sizeof buf, "ev2^%d_res2^%d_k2^%d", (int)std::lround(std::log2((double)std::max(1ll, ev))),
           (int)std::lround(std::log2((double)std::max(1ll, res))), (int)std::lround(std::log2((double)k)));
  return buf;
}

hpop_status run_once(hpop_session* const* ss, int k, std::vector<hpop_metric_tree>& out) {
  if (k == 1) return hpop_metrics_compute_all(ss[0], HPOP_FORCE_REBUILD, out.data());
  return hpop_batch_compute(ss, k, HPOP_FORCE_REBUILD, out.data());
}

}  // namespace

extern "C" hpop_status hpop_autotune(hpop_session* const* ss, int32_t k, const char* cache_path, hpop_tuning* out) {
  try {
    if (!ss || k <= 0 || !out) {
      g_thread_error = "bad arguments";
      return HPOP_E_ARG;
    }
    for (int i = 0; i < k; ++i)
      if (!ss[i]) {
        g_thread_error = "null session";
        return HPOP_E_ARG;
      }
    const std::string key = size_key(ss, k);
    TuneCache cache;
    std::string cerr;
    if (cache_path && !read_tune_cache(cache_path, cache, cerr)) {
      g_thread_error = cerr;
      return HPOP_E_ARG;
    }
    hpop_tuning best{};
    auto it = cache.find(key);
    if (it != cache.end()) {
      best.bucket_target = it->second[0];
      best.bucket_cap = it->second[1];
      best.tile_elems = it->second[2];
    } else {
      std::vector<hpop_tuning> saved(k);
      for (int i = 0; i < k; ++i) saved[i] = ss[i]->tuning;
      auto restore = [&](hpop_status st) {
        for (int i = 0; i < k; ++i) ss[i]->tuning = saved[i];
        return st;
      };
      size_t nreg = 0;
      for (int i = 0; i < k; ++i) nreg += ss[i]->regions.size();
      std::vector<hpop_metric_tree> trees(std::max<size_t>(1, nreg));
      double best_t = 1e30;
      const int targets[] = {256, 320, 352, 384};  // mean records per time bucket
      const int caps[] = {2048, 4096};
      const int tiles[] = {512, 2048, 4096, 8192};  // 512: traces of many small record batches
      for (int tg : targets)
        for (int cp : caps)
          for (int tl : tiles) {
            if (cp == 4096 && tg < 512) continue;  // small buckets never need the large capacity
            hpop_tuning t{tg, cp, tl, 0};
            for (int i = 0; i < k; ++i) ss[i]->tuning = t;
            hpop_status st = run_once(ss, k, trees);  // warm-up: plan, allocations, graph
            if (st != HPOP_OK) return restore(st);
            std::vector<double> v;
            for (int r = 0; r < 5; ++r) {
              auto t0 = std::chrono::steady_clock::now();
              st = run_once(ss, k, trees);
              auto t1 = std::chrono::steady_clock::now();
              if (st != HPOP_OK) return restore(st);
              v.push_back(std::chrono::duration<double>(t1 - t0).count());
            }
            std::sort(v.begin(), v.end());
            if (v[2] < best_t) {  // the median of five
              best_t = v[2];
              best = t;
            }
          }
      if (cache_path) {
        cache[key] = {best.bucket_target, best.bucket_cap, best.tile_elems};
        if (!write_tune_cache(cache_path, cache)) {
          g_thread_error = std::string("cannot write tuning cache ") + cache_path;
          return restore(HPOP_E_ARG);
        }
      }
    }
    for (int i = 0; i < k; ++i) ss[i]->tuning = best;
    *out = best;
    return HPOP_OK;
  } catch (...) {
    g_thread_error = "internal error in autotune";
    return HPOP_E_STATE;
  }
}
