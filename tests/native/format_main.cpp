// Drives hpop_tree_format and the region renderer over trees with extreme
// values and every buffer size up to the full rendering (host code only;
// built with AddressSanitizer and UndefinedBehaviorSanitizer by the tests).
#include <cinttypes>
#include <climits>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <limits>
#include <string>
#include <vector>

#include "hpop.h"

namespace hpop {
std::string render_region(const hpop_metric_tree& t, int32_t format, int n, int m, const int64_t* times);
hpop_status emit_string(const std::string& s, char* buf, int64_t cap, int64_t* needed);
}

static int check(const hpop_metric_tree& t) {
  for (int fmt = 0; fmt < 2; ++fmt) {
    int64_t need = 0;
    if (hpop_tree_format(&t, fmt, nullptr, 0, &need) != HPOP_OK || need < 2) return 1;
    for (int64_t cap = 1; cap <= need; ++cap) {
      std::vector<char> buf((size_t)cap + 8, '#');
      int64_t again = 0;
      if (hpop_tree_format(&t, fmt, buf.data(), cap, &again) != HPOP_OK || again != need) return 2;
      if ((int64_t)std::strlen(buf.data()) != cap - 1) return 3;
      for (size_t j = (size_t)cap; j < buf.size(); ++j)
        if (buf[j] != '#') return 4;  // nothing written past cap
    }
  }
  return 0;
}

int main() {
  const double inf = std::numeric_limits<double>::infinity();
  const double vals[] = {0.0, 1.0, 0.125, 1e300, -1e300, inf, -inf, std::nan(""), 5e-324, -0.0};
  const int64_t ints[] = {0, 1, INT64_MAX, INT64_MIN, -1, (int64_t)1 << 62};
  int cases = 0;
  for (double v : vals)
    for (int64_t x : ints) {
      hpop_metric_tree t{};
      t.E = x;
      t.n = INT32_MAX;
      t.m = INT32_MIN;
      t.sumU = t.sumW = t.sumMPI = t.sumOther = t.sumUW = t.maxUW = x;
      t.sumK = t.sumM = t.maxK = t.maxKM = x;
      t.host_pe = t.host_mpi_pe = t.host_mpi_lb = t.host_mpi_ce = t.host_oe = v;
      t.dev_pe = t.dev_lb = t.dev_ce = t.dev_oe = v;
      t.undefined_mask = (uint32_t)(x & 0x1ff) | 0xfffffe00u;
      if (int rc = check(t)) {
        std::printf("tree check failed %d\n", rc);
        return 1;
      }
      // region reports over 0..5 resources with the same extreme times
      for (int n = 0; n <= 3; ++n)
        for (int m = 0; m <= 2; ++m) {
          std::vector<int64_t> times(4 * (size_t)(n + m) + 1, x);
          for (int fmt = 0; fmt < 2; ++fmt) {
            const std::string s = hpop::render_region(t, fmt, n, m, times.data());
            int64_t need = 0;
            std::vector<char> buf(s.size() / 2 + 1);
            if (hpop::emit_string(s, buf.data(), (int64_t)buf.size(), &need) != HPOP_OK ||
                need != (int64_t)s.size() + 1 || std::strlen(buf.data()) != buf.size() - 1)
              return 1;
          }
        }
      ++cases;
    }
  hpop_metric_tree t{};
  if (hpop_tree_format(nullptr, 0, nullptr, 0, nullptr) != HPOP_E_ARG) return 1;
  if (hpop_tree_format(&t, 2, nullptr, 0, nullptr) != HPOP_E_ARG) return 1;
  if (hpop_tree_format(&t, 0, nullptr, 5, nullptr) != HPOP_E_ARG) return 1;
  if (hpop_tree_format(&t, 0, nullptr, -1, nullptr) != HPOP_E_ARG) return 1;
  std::printf("ok %d\n", cases);
  return 0;
}
