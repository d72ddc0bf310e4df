// The autotuner's cache file (host code only, no HIP): a JSON object that
// maps a workload size class to the chosen tuning,
//   {"ev2^27_res2^9_k2^0": [256, 2048, 2048], ...}
// i.e. [bucket_target, bucket_cap, tile_elems]. The reader accepts exactly
// that shape (keys without escapes, three integers each, every value in the
// range hpop_tuning documents) and reports anything else as an error with
// the byte offset, so a truncated or garbled file is never half-applied.
#pragma once

#include <cerrno>
#include <climits>
#include <cstdio>
#include <cstdlib>
#include <fstream>
#include <map>
#include <string>
#include <vector>

namespace hpop {

using TuneCache = std::map<std::string, std::vector<int>>;

inline bool tune_entry_valid(const std::vector<int>& v) {
  return v.size() == 3 && v[0] >= 16 && v[0] <= 4096 && (v[1] == 2048 || v[1] == 4096) &&
         (v[2] == 512 || v[2] == 2048 || v[2] == 4096 || v[2] == 8192);
}

// Parses `s` into `out`. Returns false with a message in `err` on any
// deviation from the format above.
inline bool parse_tune_cache(const std::string& s, TuneCache& out, std::string& err) {
  size_t i = 0;
  const size_t n = s.size();
  auto ws = [&]() {
    while (i < n && (s[i] == ' ' || s[i] == '\n' || s[i] == '\r' || s[i] == '\t')) ++i;
  };
  auto bad = [&](const char* what) {
    err = std::string(what) + " at byte " + std::to_string(i);
    return false;
  };
  auto expect = [&](char c) {
    ws();
    if (i >= n || s[i] != c) return false;
    ++i;
    return true;
  };
  TuneCache m;
  if (!expect('{')) return bad("expected '{'");
  ws();
  if (i < n && s[i] == '}') {
    ++i;
  } else {
    while (true) {
      if (!expect('"')) return bad("expected a quoted key");
      const size_t k0 = i;
      while (i < n && s[i] != '"' && s[i] != '\\' && (unsigned char)s[i] >= 0x20) ++i;
      if (i >= n || s[i] != '"') return bad("unterminated or escaped key");
      std::string key = s.substr(k0, i - k0);
      ++i;
      if (key.empty()) return bad("empty key");
      if (!expect(':')) return bad("expected ':'");
      if (!expect('[')) return bad("expected '['");
      std::vector<int> v;
      for (int j = 0; j < 3; ++j) {
        if (j && !expect(',')) return bad("expected ','");
        ws();
        const size_t d0 = i;
        if (i < n && s[i] == '-') ++i;
        while (i < n && s[i] >= '0' && s[i] <= '9' && i - d0 < 12) ++i;
        if (i == d0 || (i == d0 + 1 && s[d0] == '-')) return bad("expected an integer");
        if (i < n && s[i] >= '0' && s[i] <= '9') return bad("integer too long");
        const long long x = std::strtoll(s.substr(d0, i - d0).c_str(), nullptr, 10);
        if (x < INT_MIN || x > INT_MAX) return bad("integer out of range");
        v.push_back((int)x);
      }
      if (!expect(']')) return bad("expected ']' after three integers");
      if (!tune_entry_valid(v)) return bad("tuning outside the documented ranges");
      if (m.count(key)) return bad("duplicate key");
      m[key] = v;
      ws();
      if (i < n && s[i] == ',') {
        ++i;
        continue;
      }
      if (!expect('}')) return bad("expected ',' or '}'");
      break;
    }
  }
  ws();
  if (i != n) return bad("trailing data");
  out.swap(m);
  return true;
}

// Reads the cache at `path`. A missing file is an empty cache; a file that
// cannot be opened or read, or does not parse, is an error.
inline bool read_tune_cache(const char* path, TuneCache& out, std::string& err) {
  out.clear();
  errno = 0;
  std::FILE* f = std::fopen(path, "rb");
  if (!f) {
    if (errno == ENOENT) return true;
    err = std::string("cannot open tuning cache ") + path;
    return false;
  }
  std::string text;
  char buf[4096];
  size_t k;
  while ((k = std::fread(buf, 1, sizeof buf, f)) > 0) text.append(buf, k);
  const bool failed = std::ferror(f) != 0;
  std::fclose(f);
  if (failed) {
    err = std::string("cannot read tuning cache ") + path;
    return false;
  }
  std::string perr;
  if (!parse_tune_cache(text, out, perr)) {
    err = std::string("malformed tuning cache ") + path + ": " + perr;
    return false;
  }
  return true;
}

// Writes the whole cache through a temporary file renamed over `path`.
inline bool write_tune_cache(const char* path, const TuneCache& m) {
  const std::string tmp = std::string(path) + ".tmp";
  {
    std::ofstream f(tmp, std::ios::binary);
    if (!f) return false;
    f << "{\n";
    size_t k = 0;
    for (auto& kv : m) {
      f << "  \"" << kv.first << "\": [" << kv.second[0] << ", " << kv.second[1] << ", " << kv.second[2] << "]"
        << (++k < m.size() ? "," : "") << "\n";
    }
    f << "}\n";
    if (!f) return false;
  }
  return std::rename(tmp.c_str(), path) == 0;
}

}  // namespace hpop
