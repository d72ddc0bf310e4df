// Text and JSON renderings of a metric tree (host code only). The tree shape
// follows the paper's metric tables (Sec. 4.1, Sec. 5.1): the host Parallel
// Efficiency splits into MPI Parallel Efficiency (itself Load Balance and
// Communication Efficiency) and Device Offload Efficiency; the device Parallel
// Efficiency into Load Balance, Communication Efficiency and Orchestration
// Efficiency.
#include <cinttypes>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <string>

#include "hpop.h"

namespace {

struct Node {
  const char* label;
  const char* key;
  int depth;
  int bit;  // bit of undefined_mask
};

// Depth-first order of the two trees; ratio i of the tree is bit i.
const Node kNodes[9] = {
    {"Host Parallel Efficiency", "parallel_efficiency", 0, 0},
    {"MPI Parallel Efficiency", "mpi_parallel_efficiency", 1, 1},
    {"MPI Load Balance", "mpi_load_balance", 2, 2},
    {"MPI Communication Efficiency", "mpi_communication_efficiency", 2, 3},
    {"Device Offload Efficiency", "device_offload_efficiency", 1, 4},
    {"Device Parallel Efficiency", "parallel_efficiency", 0, 5},
    {"Load Balance", "load_balance", 1, 6},
    {"Communication Efficiency", "communication_efficiency", 1, 7},
    {"Orchestration Efficiency", "orchestration_efficiency", 1, 8},
};

double value(const hpop_metric_tree& t, int bit) {
  switch (bit) {
    case 0: return t.host_pe;
    case 1: return t.host_mpi_pe;
    case 2: return t.host_mpi_lb;
    case 3: return t.host_mpi_ce;
    case 4: return t.host_oe;
    case 5: return t.dev_pe;
    case 6: return t.dev_lb;
    case 7: return t.dev_ce;
    default: return t.dev_oe;
  }
}

void appendf(std::string& s, const char* fmt, ...) __attribute__((format(printf, 2, 3)));
void appendf(std::string& s, const char* fmt, ...) {
  va_list ap, ap2;
  va_start(ap, fmt);
  va_copy(ap2, ap);
  const int k = vsnprintf(nullptr, 0, fmt, ap);  // the full length, however long
  va_end(ap);
  if (k > 0) {
    const size_t at = s.size();
    s.resize(at + (size_t)k + 1);
    vsnprintf(&s[at], (size_t)k + 1, fmt, ap2);
    s.resize(at + (size_t)k);
  }
  va_end(ap2);
}

std::string text(const hpop_metric_tree& t) {
  std::string s;
  appendf(s, "Region length E = %" PRId64 " ns, %d host processes, %d devices\n", t.E, t.n, t.m);
  bool any = false;
  for (const Node& n : kNodes) {
    const bool undef = (t.undefined_mask >> n.bit) & 1u;
    any |= undef;
    const int pad = 2 * n.depth;
    appendf(s, "%*s%-*s %6.2f%s\n", pad, "", 34 - pad, n.label, value(t, n.bit), undef ? " *" : "");
  }
  appendf(s, "Host times (ns):   useful %" PRId64 ", offload %" PRId64 ", MPI %" PRId64 ", other %" PRId64 "\n",
          t.sumU, t.sumW, t.sumMPI, t.sumOther);
  appendf(s, "Device times (ns): kernels %" PRId64 ", memory operations %" PRId64 "\n", t.sumK, t.sumM);
  if (any) appendf(s, "* 0/0: no time of that kind in the region; the ratio is set to 1\n");
  return s;
}

std::string json(const hpop_metric_tree& t) {
  std::string s;
  appendf(s, "{\"E\": %" PRId64 ", \"n\": %d, \"m\": %d, ", t.E, t.n, t.m);
  for (int tree = 0; tree < 2; ++tree) {
    appendf(s, "\"%s\": {", tree == 0 ? "host" : "device");
    bool first = true;
    for (const Node& n : kNodes) {
      if ((n.bit < 5) != (tree == 0)) continue;
      appendf(s, "%s\"%s\": %.17g", first ? "" : ", ", n.key, value(t, n.bit));
      first = false;
    }
    s += "}, ";
  }
  appendf(s,
          "\"times\": {\"useful\": %" PRId64 ", \"offload\": %" PRId64 ", \"mpi\": %" PRId64 ", \"other\": %" PRId64
          ", \"useful_plus_offload\": %" PRId64 ", \"max_useful_plus_offload\": %" PRId64 ", \"kernel\": %" PRId64
          ", \"memory_operations\": %" PRId64 ", \"max_kernel\": %" PRId64 ", \"max_kernel_plus_memory\": %" PRId64
          "}, \"undefined\": [",
          t.sumU, t.sumW, t.sumMPI, t.sumOther, t.sumUW, t.maxUW, t.sumK, t.sumM, t.maxK, t.maxKM);
  bool first = true;
  for (const Node& n : kNodes) {
    if (!((t.undefined_mask >> n.bit) & 1u)) continue;
    appendf(s, "%s\"%s.%s\"", first ? "" : ", ", n.bit < 5 ? "host" : "device", n.key);
    first = false;
  }
  s += "]}";
  return s;
}

// One line (text) or object (JSON) per resource: hosts 0..n-1 with their
// useful, offload, MPI and other times, devices n..n+m-1 with kernel,
// memory-operation and idle times (times: 4 int64 per resource, in that order).
std::string resources_text(int n, int m, const int64_t* times) {
  std::string s = "Resource times in the region (ns):\n";
  for (int r = 0; r < n + m; ++r) {
    const int64_t* x = times + 4 * (size_t)r;
    if (r < n)
      appendf(s, "  host %d: useful %" PRId64 ", offload %" PRId64 ", MPI %" PRId64 ", other %" PRId64 "\n", r, x[0],
              x[1], x[2], x[3]);
    else
      appendf(s, "  device %d: kernels %" PRId64 ", memory operations %" PRId64 ", idle %" PRId64 "\n", r - n, x[0],
              x[1], x[2]);
  }
  return s;
}

std::string resources_json(int n, int m, const int64_t* times) {
  std::string s = "\"resources\": [";
  for (int r = 0; r < n + m; ++r) {
    const int64_t* x = times + 4 * (size_t)r;
    if (r < n)
      appendf(s, "%s{\"host\": %d, \"useful\": %" PRId64 ", \"offload\": %" PRId64 ", \"mpi\": %" PRId64
              ", \"other\": %" PRId64 "}", r ? ", " : "", r, x[0], x[1], x[2], x[3]);
    else
      appendf(s, "%s{\"device\": %d, \"kernel\": %" PRId64 ", \"memory_operations\": %" PRId64 ", \"idle\": %" PRId64
              "}", r ? ", " : "", r - n, x[0], x[1], x[2]);
  }
  s += "]";
  return s;
}

}  // namespace

namespace hpop {

// The string, NUL-terminated and cut to cap - 1 characters, into buf; the
// full size with the terminator into *needed.
hpop_status emit_string(const std::string& s, char* buf, int64_t cap, int64_t* needed) {
  if (cap < 0 || (cap > 0 && !buf)) return HPOP_E_ARG;
  if (needed) *needed = (int64_t)s.size() + 1;
  if (cap > 0) {
    const size_t k = s.size() < (size_t)cap - 1 ? s.size() : (size_t)cap - 1;
    memcpy(buf, s.data(), k);
    buf[k] = '\0';
  }
  return HPOP_OK;
}

// A region's report: the tree rendering followed by every resource's state
// times (the run-time report with raw metrics, Sec. 3.2).
std::string render_region(const hpop_metric_tree& t, int32_t format, int n, int m, const int64_t* times) {
  if (format == HPOP_FORMAT_TEXT) return text(t) + resources_text(n, m, times);
  std::string s = json(t);
  s.pop_back();  // the closing brace of the tree object
  return s + ", " + resources_json(n, m, times) + "}";
}

}  // namespace hpop

extern "C" hpop_status hpop_tree_format(const hpop_metric_tree* tree, int32_t format, char* buf, int64_t cap,
                                        int64_t* needed) {
  if (!tree || (format != HPOP_FORMAT_TEXT && format != HPOP_FORMAT_JSON) || cap < 0 || (cap > 0 && !buf))
    return HPOP_E_ARG;
  return hpop::emit_string(format == HPOP_FORMAT_TEXT ? text(*tree) : json(*tree), buf, cap, needed);
}
