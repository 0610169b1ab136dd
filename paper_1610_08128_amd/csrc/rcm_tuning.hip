// Tuning tables written by the autotuner (paper_1610_08128_amd/tune.py): per
// size class of a call, the launch options that measured fastest.  Host code
// only.
//
// Format (text, one entry per line; '#' starts a comment):
//   <kind>:n2^<lg>:d<deg> <option>=<integer> ...
// kind is "single" or "batch"; lg = floor(log2(vertices)); deg = entries per
// vertex rounded half to even (the tuner's own size class).  Only launch
// options are taken from a table (they change the time of a call, never its
// result); any other key makes the table invalid.

#include <cerrno>
#include <cfenv>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "rcm_common.hpp"

namespace rcm {

namespace {

struct Entry {
  bool batch = false;
  int lg = 0;
  int deg = 0;
  std::vector<std::pair<int32_t rcm_options::*, int32_t>> set;
};

struct Table {
  bool ok = false;
  std::vector<Entry> entries;
};

struct Field {
  const char* name;
  int32_t rcm_options::*member;
};

const Field kFields[] = {
    {"team_size", &rcm_options::team_size},
    {"block_threads", &rcm_options::block_threads},
    {"small_cutoff", &rcm_options::small_cutoff},
    {"narrow_cutoff", &rcm_options::narrow_cutoff},
    {"small_threads", &rcm_options::small_threads},
    {"max_teams", &rcm_options::max_teams},
    {"rebalance_levels", &rcm_options::rebalance_levels},
    {"async_search", &rcm_options::async_search},
    {"label_team", &rcm_options::label_team},
    {"search_round", &rcm_options::search_round},
    {"mode", &rcm_options::mode},
    {"relabel_levels", &rcm_options::relabel_levels},
};

bool parse_class(const char* s, Entry* e) {
  char kind[16] = {};
  int lg = 0, deg = 0;
  if (std::sscanf(s, "%15[a-z]:n2^%d:d%d", kind, &lg, &deg) != 3) return false;
  if (std::strcmp(kind, "single") == 0) e->batch = false;
  else if (std::strcmp(kind, "batch") == 0) e->batch = true;
  else return false;
  e->lg = lg;
  e->deg = deg;
  return true;
}

Table read_table(const char* path) {
  Table t;
  FILE* f = std::fopen(path, "r");
  if (!f) return t;
  char line[4096];
  bool ok = true;
  while (ok && std::fgets(line, sizeof(line), f)) {
    char* hash = std::strchr(line, '#');
    if (hash) *hash = '\0';
    char* save = nullptr;
    char* tok = strtok_r(line, " \t\r\n", &save);
    if (!tok) continue;
    Entry e;
    if (!parse_class(tok, &e)) {
      ok = false;
      break;
    }
    while ((tok = strtok_r(nullptr, " \t\r\n", &save)) != nullptr) {
      char* eq = std::strchr(tok, '=');
      if (!eq) {
        ok = false;
        break;
      }
      *eq = '\0';
      errno = 0;
      char* end = nullptr;
      const long v = std::strtol(eq + 1, &end, 10);
      if (errno != 0 || end == eq + 1 || *end != '\0' || v < -1 || v > (1l << 30)) {
        ok = false;
        break;
      }
      const Field* fld = nullptr;
      for (const Field& c : kFields)
        if (std::strcmp(c.name, tok) == 0) fld = &c;
      if (!fld) {
        ok = false;
        break;
      }
      e.set.emplace_back(fld->member, static_cast<int32_t>(v));
    }
    if (ok) t.entries.push_back(e);
  }
  std::fclose(f);
  t.ok = ok;
  return t;
}

std::mutex g_mutex;
std::map<std::string, Table> g_tables;  // parsed once per path for the process

const Table& table_for(const char* path) {
  std::lock_guard<std::mutex> lk(g_mutex);
  auto it = g_tables.find(path);
  if (it == g_tables.end()) it = g_tables.emplace(path, read_table(path)).first;
  return it->second;
}

}  // namespace

bool tuning_apply(const char* path, int64_t n, int64_t nnz, int32_t graphs, rcm_options* opts) {
  const Table& t = table_for(path);
  if (!t.ok) return false;
  const bool batch = graphs > 1;
  int lg = 0;
  for (int64_t x = n > 1 ? n : 1; x > 1; x >>= 1) ++lg;
  // rounded half to even, as the tuner's round() does
  const int prev = std::fegetround();
  std::fesetround(FE_TONEAREST);
  const int deg = static_cast<int>(std::nearbyint(static_cast<double>(nnz) /
                                                  static_cast<double>(n > 1 ? n : 1)));
  std::fesetround(prev);
  // the exact class, else the nearest of the same kind (log2 distance plus
  // four times the row-length distance)
  const Entry* best = nullptr;
  long best_d = -1;
  for (const Entry& e : t.entries) {
    if (e.batch != batch) continue;
    const long d = std::labs(static_cast<long>(e.lg - lg)) + 4 * std::labs(static_cast<long>(e.deg - deg));
    if (best_d < 0 || d < best_d) {
      best = &e;
      best_d = d;
    }
  }
  if (best) {
    for (const auto& kv : best->set) {
      // the engine is taken only from the entry of the call's own class; a
      // table's mode 2 asks for the one-work-group engine where the graph
      // fits, as auto does (a caller's own mode 2 requires it)
      if (kv.first == &rcm_options::mode && (best_d != 0 || kv.second == 2)) continue;
      if (opts->*(kv.first) == 0) opts->*(kv.first) = kv.second;
    }
  }
  return true;
}

const char* tuning_path(const rcm_options* opts) {
  if (opts && opts->tuning_file && opts->tuning_file[0]) return opts->tuning_file;
  const char* e = std::getenv("RCM_TUNING_FILE");
  return e && e[0] ? e : nullptr;
}

}  // namespace rcm

extern "C" rcm_status rcm_tuning_options(const char* path, int32_t num_graphs, int64_t n,
                                         int64_t nnz, rcm_options* out) {
  if (!path || !out || n < 0 || nnz < 0 || num_graphs < 1) return RCM_ERR_INVALID_ARGUMENT;
  return rcm::tuning_apply(path, n, nnz, num_graphs, out) ? RCM_OK : RCM_ERR_INVALID_ARGUMENT;
}
