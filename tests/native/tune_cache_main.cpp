// Reads an autotuner cache file with the library's reader and prints what it
// found ("ok <entries>" and one line per entry) or "error <message>"; built
// with AddressSanitizer and UndefinedBehaviorSanitizer by the tests.
#include <cstdio>

#include "hpop_tune_cache.h"

int main(int argc, char** argv) {
  if (argc != 2) return 2;
  hpop::TuneCache m;
  std::string err;
  if (!hpop::read_tune_cache(argv[1], m, err)) {
    std::printf("error %s\n", err.c_str());
    return 0;
  }
  std::printf("ok %zu\n", m.size());
  for (auto& kv : m) std::printf("%s %d %d %d\n", kv.first.c_str(), kv.second[0], kv.second[1], kv.second[2]);
  return 0;
}
