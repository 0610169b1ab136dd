// Host-side checks of the ordering library, built with AddressSanitizer and
// UndefinedBehaviorSanitizer on the host code only (tests/test_sanitizers.py
// compiles every library source with the sanitizers behind -Xarch_host and
// links this driver against them).  Everything here runs without a GPU: argument and
// option validation, the tuning-table parser (also on malformed tables),
// the workspace arithmetic, the abort-flag registry, the server's
// configuration checks and the seeded shuffle bijection.
//
// usage: host_checks <scratch directory>
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>
#include <vector>

#include "rcm.h"
#include "rcm_common.hpp"
#include "rcm_server.h"

static int g_checks = 0, g_failed = 0;

#define CHECK(cond)                                                          \
  do {                                                                       \
    ++g_checks;                                                              \
    if (!(cond)) {                                                           \
      ++g_failed;                                                            \
      std::fprintf(stderr, "%s:%d: check failed: %s\n", __FILE__, __LINE__, #cond); \
    }                                                                        \
  } while (0)

static std::string write_file(const std::string& dir, const char* name, const std::string& text) {
  const std::string path = dir + "/" + name;
  FILE* f = std::fopen(path.c_str(), "w");
  if (!f) {
    std::perror(path.c_str());
    std::exit(2);
  }
  std::fwrite(text.data(), 1, text.size(), f);
  std::fclose(f);
  return path;
}

static void check_status_strings() {
  for (int s = 0; s <= 7; ++s) {
    const char* m = rcm_status_string(static_cast<rcm_status>(s));
    CHECK(m != nullptr && std::strlen(m) > 0);
  }
  CHECK(std::strcmp(rcm_status_string(static_cast<rcm_status>(99)), "unknown status") == 0);
}

static void check_option_validation() {
  rcm_options o;
  rcm_default_options(&o);
  const unsigned char* b = reinterpret_cast<const unsigned char*>(&o);
  bool zero = true;
  for (size_t i = 0; i < sizeof(o); ++i) zero = zero && b[i] == 0;
  CHECK(zero);
  rcm_default_options(nullptr);  // ignored
  int32_t perm[4];
  const int32_t rowptr[2] = {0, 0};
  // argument checks before any device work
  CHECK(rcm_order_ex(-1, rowptr, nullptr, perm, nullptr, nullptr, nullptr, nullptr, 0, nullptr) ==
        RCM_ERR_INVALID_ARGUMENT);
  CHECK(rcm_order_ex(3, nullptr, nullptr, perm, nullptr, nullptr, nullptr, nullptr, 0, nullptr) ==
        RCM_ERR_INVALID_ARGUMENT);
  CHECK(rcm_order_ex(3, rowptr, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, 0,
                     nullptr) == RCM_ERR_INVALID_ARGUMENT);
  rcm_stats st;
  std::memset(&st, 0x5a, sizeof(st));
  CHECK(rcm_order_ex(0, nullptr, nullptr, nullptr, nullptr, &st, nullptr, nullptr, 0, nullptr) ==
        RCM_OK);
  CHECK(st.num_components == 0 && st.edges_traversed == 0);
  CHECK(rcm_order(0, nullptr, nullptr, nullptr, nullptr, nullptr) == RCM_OK);
  // every out-of-range option field is rejected
  struct Bad {
    int32_t rcm_options::*field;
    int32_t value;
  };
  const Bad bad[] = {
      {&rcm_options::pp_variant, 2},      {&rcm_options::pp_variant, -1},
      {&rcm_options::reverse_mode, 2},    {&rcm_options::check_full, 3},
      {&rcm_options::team_size, -1},      {&rcm_options::team_size, 257},
      {&rcm_options::block_threads, 128}, {&rcm_options::block_threads, 1024},
      {&rcm_options::small_cutoff, -5},   {&rcm_options::narrow_cutoff, -2},
      {&rcm_options::small_threads, 64},  {&rcm_options::max_teams, 65},
      {&rcm_options::max_teams, -1},      {&rcm_options::rebalance_levels, -1},
      {&rcm_options::label_mode, 3},      {&rcm_options::async_search, 2},
      {&rcm_options::label_team, 300},    {&rcm_options::search_round, -1},
      {&rcm_options::mode, 3},            {&rcm_options::mode, -1},
  };
  for (const Bad& x : bad) {
    rcm_default_options(&o);
    o.*(x.field) = x.value;
    CHECK(rcm_order_ex(3, rowptr, nullptr, perm, nullptr, nullptr, &o, nullptr, 0, nullptr) ==
          RCM_ERR_INVALID_ARGUMENT);
    CHECK(rcm_order_noalloc(3, rowptr, nullptr, perm, nullptr, nullptr, &o, nullptr) ==
          RCM_ERR_INVALID_ARGUMENT);
  }
  // an abort flag the library did not create
  int32_t not_a_flag = 0;
  rcm_default_options(&o);
  o.abort_flag = &not_a_flag;
  CHECK(rcm_order_ex(3, rowptr, nullptr, perm, nullptr, nullptr, &o, nullptr, 0, nullptr) ==
        RCM_ERR_INVALID_ARGUMENT);
  // batched argument checks
  const int64_t vo_bad[3] = {0, 5, 3}, no_ok[3] = {0, 0, 0};
  CHECK(rcm_order_batched(-1, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr,
                          nullptr, 0, nullptr) == RCM_ERR_INVALID_ARGUMENT);
  CHECK(rcm_order_batched(0, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr,
                          nullptr, 0, nullptr) == RCM_OK);
  CHECK(rcm_order_batched(2, vo_bad, no_ok, rowptr, nullptr, perm, nullptr, nullptr, nullptr, 0,
                          nullptr) == RCM_ERR_INVALID_ARGUMENT);
  const int64_t vo_big[2] = {0, int64_t(1) << 31}, no_big[2] = {0, 0};
  CHECK(rcm_order_batched(1, vo_big, no_big, rowptr, nullptr, perm, nullptr, nullptr, nullptr, 0,
                          nullptr) == RCM_ERR_INVALID_ARGUMENT);
  const int64_t vo_nz[2] = {1, 3};
  CHECK(rcm_order_batched(1, vo_nz, no_ok, rowptr, nullptr, perm, nullptr, nullptr, nullptr, 0,
                          nullptr) == RCM_ERR_INVALID_ARGUMENT);
}

static void check_workspace_sizes() {
  CHECK(rcm_workspace_bytes(0, 0, nullptr) == 0);
  CHECK(rcm_workspace_bytes(-3, 0, nullptr) == 0);
  size_t prev = 0;
  for (int32_t n : {1, 2, 100, 4096, 1 << 20, 1 << 24, 2147483646}) {
    const size_t b = rcm_workspace_bytes(n, 7ll * n, nullptr);
    CHECK(b >= static_cast<size_t>(n) * 16 && b >= prev && b % 256 == 0);
    prev = b;
  }
  CHECK(rcm_batched_workspace_bytes(0, 10, 10, nullptr) == 0);
  CHECK(rcm_batched_workspace_bytes(3, 0, 0, nullptr) == 0);
  const size_t one = rcm_workspace_bytes(1000, 5000, nullptr);
  const size_t three = rcm_batched_workspace_bytes(3, 1000, 5000, nullptr);
  // the batch also holds the union's CSR; a single graph holds a 32-byte
  // copy of each row instead
  CHECK(three + 32 * 1000 >= one + 4 * 5000);
  CHECK(three < rcm_batched_workspace_bytes(3, 1000, 50000, nullptr));
  // a single graph's workspace does not depend on its entry count
  CHECK(rcm_workspace_bytes(1000, 50000, nullptr) == one);
  CHECK(rcm_server_request_bytes(1000, 5000) >= one);
}

static void check_tuning_tables(const std::string& dir) {
  rcm_options o;
  const std::string good = write_file(
      dir, "good.txt",
      "# comment line\n"
      "\n"
      "single:n2^12:d5 team_size=8 mode=1   # trailing comment\n"
      "single:n2^21:d7 team_size=256 label_team=96 search_round=12\n"
      "batch:n2^24:d8 small_threads=512 max_teams=32\n");
  rcm_default_options(&o);
  CHECK(rcm_tuning_options(good.c_str(), 1, 4096, 20224, &o) == RCM_OK);
  CHECK(o.team_size == 8 && o.mode == 1);
  rcm_default_options(&o);
  CHECK(rcm_tuning_options(good.c_str(), 1, 1 << 20, 7 << 20, &o) == RCM_OK);  // nearest class
  CHECK(o.team_size == 256 && o.label_team == 96 && o.search_round == 12 && o.mode == 0);
  rcm_default_options(&o);
  CHECK(rcm_tuning_options(good.c_str(), 5, 100, 300, &o) == RCM_OK);
  CHECK(o.small_threads == 512 && o.max_teams == 32);
  rcm_default_options(&o);
  o.team_size = 4;  // the caller's value wins
  CHECK(rcm_tuning_options(good.c_str(), 1, 4096, 20224, &o) == RCM_OK && o.team_size == 4);
  CHECK(rcm_tuning_options(good.c_str(), 1, 0, 0, &o) == RCM_OK);  // n = 0 is a class too
  CHECK(rcm_tuning_options(nullptr, 1, 10, 10, &o) == RCM_ERR_INVALID_ARGUMENT);
  CHECK(rcm_tuning_options(good.c_str(), 1, 10, 10, nullptr) == RCM_ERR_INVALID_ARGUMENT);
  CHECK(rcm_tuning_options(good.c_str(), 0, 10, 10, &o) == RCM_ERR_INVALID_ARGUMENT);
  CHECK(rcm_tuning_options(good.c_str(), 1, -1, 10, &o) == RCM_ERR_INVALID_ARGUMENT);
  CHECK(rcm_tuning_options((dir + "/missing.txt").c_str(), 1, 10, 10, &o) ==
        RCM_ERR_INVALID_ARGUMENT);
  // malformed tables: each is rejected as a whole
  const char* bad_tables[] = {
      "single:n2^12:d5 pp_variant=1\n",          // not a launch option
      "single:n2^12:d5 team_size\n",             // no value
      "single:n2^12:d5 team_size=\n",            // empty value
      "single:n2^12:d5 team_size=8x\n",          // trailing junk
      "single:n2^12:d5 team_size=99999999999\n", // out of range
      "single:n2^12:d5 team_size=-7\n",          // below -1
      "double:n2^12:d5 team_size=8\n",           // unknown kind
      "single:n12:d5 team_size=8\n",             // malformed class
      "single team_size=8\n",
      "=\n",
  };
  int i = 0;
  for (const char* t : bad_tables) {
    const std::string name = "bad" + std::to_string(i++) + ".txt";
    const std::string p = write_file(dir, name.c_str(), t);
    rcm_default_options(&o);
    CHECK(rcm_tuning_options(p.c_str(), 1, 4096, 20224, &o) == RCM_ERR_INVALID_ARGUMENT);
  }
  // a line longer than the parser's buffer, and an empty table
  std::string longline = "single:n2^12:d5";
  while (longline.size() < 10000) longline += " team_size=8";
  const std::string lp = write_file(dir, "long.txt", longline + "\n");
  rcm_default_options(&o);
  (void)rcm_tuning_options(lp.c_str(), 1, 4096, 20224, &o);  // either status; no overrun
  const std::string empty = write_file(dir, "empty.txt", "");
  rcm_default_options(&o);
  CHECK(rcm_tuning_options(empty.c_str(), 1, 4096, 20224, &o) == RCM_OK && o.team_size == 0);
  // a bad table fails the ordering call before any device work
  rcm_default_options(&o);
  const std::string bad0 = dir + "/bad0.txt";
  o.tuning_file = bad0.c_str();
  const int32_t rowptr[2] = {0, 0};
  int32_t perm[1];
  CHECK(rcm_order_ex(1, rowptr, nullptr, perm, nullptr, nullptr, &o, nullptr, 0, nullptr) !=
        RCM_OK);
}

static void check_abort_flags() {
  CHECK(rcm_abort_flag_create(nullptr) == RCM_ERR_INVALID_ARGUMENT);
  int32_t* f = reinterpret_cast<int32_t*>(0x1);
  const rcm_status s = rcm_abort_flag_create(&f);
  if (s == RCM_OK) {
    CHECK(f != nullptr && *f == 0);
    rcm_abort_flag_destroy(f);
  } else {
    CHECK(s == RCM_ERR_HIP && f == nullptr);  // no GPU here
  }
  rcm_abort_flag_destroy(nullptr);
  int32_t local = 0;
  rcm_abort_flag_destroy(&local);  // not the library's: ignored
}

static void check_server_config() {
  rcm_server_config cfg;
  rcm_server_default_config(&cfg);
  CHECK(cfg.max_batch == 0 && cfg.executors == 0 && cfg.mem_budget_bytes == 0);
  rcm_server* srv = reinterpret_cast<rcm_server*>(0x1);
  CHECK(rcm_server_create(&cfg, nullptr) == RCM_ERR_INVALID_ARGUMENT);
  cfg.executors = 9;
  CHECK(rcm_server_create(&cfg, &srv) == RCM_ERR_INVALID_ARGUMENT);
  rcm_server_default_config(&cfg);
  cfg.order_options.mode = 7;
  CHECK(rcm_server_create(&cfg, &srv) == RCM_ERR_INVALID_ARGUMENT);
}

static void check_shuffle_bijection() {
  for (uint32_t seed : {0u, 1u, 2u, 7u, 12345u, 0xdeadbeefu}) {
    for (int32_t count : {0, 1, 2, 3, 5, 8, 63, 64, 65, 100, 255, 256, 257, 1000, 4097}) {
      std::vector<int> seen(static_cast<size_t>(count), 0);
      bool in_range = true;
      int moved = 0;
      for (int32_t i = 0; i < count; ++i) {
        const int32_t j = rcm::shuffle_index(i, count, seed);
        if (j < 0 || j >= count) {
          in_range = false;
          continue;
        }
        seen[static_cast<size_t>(j)] += 1;
        moved += j != i;
      }
      bool bij = in_range;
      for (int c : seen) bij = bij && c == 1;
      CHECK(bij);
      if (seed == 0) CHECK(moved == 0);
    }
  }
  // larger counts, and indexes outside [0, count) pass through
  const int32_t big = 1000003;
  std::vector<uint8_t> seen(big, 0);
  bool bij = true;
  for (int32_t i = 0; i < big; ++i) {
    const int32_t j = rcm::shuffle_index(i, big, 99u);
    if (j < 0 || j >= big || seen[static_cast<size_t>(j)]) bij = false;
    else seen[static_cast<size_t>(j)] = 1;
  }
  CHECK(bij);
  CHECK(rcm::shuffle_index(-1, 10, 5u) == -1 && rcm::shuffle_index(10, 10, 5u) == 10);
  CHECK(rcm::mix32(0) == 0 && rcm::mix32(1) != 1);
}

int main(int argc, char** argv) {
  if (argc < 2) {
    std::fprintf(stderr, "usage: %s <scratch dir>\n", argv[0]);
    return 2;
  }
  check_status_strings();
  check_option_validation();
  check_workspace_sizes();
  check_tuning_tables(argv[1]);
  check_abort_flags();
  check_server_config();
  check_shuffle_bijection();
  std::printf("%d checks, %d failed\n", g_checks, g_failed);
  return g_failed == 0 ? 0 : 1;
}
