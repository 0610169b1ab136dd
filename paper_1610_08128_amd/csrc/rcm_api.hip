// C ABI of the ordering library and its host-side orchestration.
//
// Call flow (one graph, or a batch treated as the disjoint union of its
// graphs, which the per-component ordering makes equivalent):
//   1. argument checks; rowptr[0] and rowptr[n] read back;
//   2. CSR checks + degrees + bandwidth/profile of the input order;
//   3. (optional) duplicate / symmetry check;
//   4. connected components -> seeds (lowest ids) -> sizes and label offsets
//      -> three task lists: isolated vertices, small components (one
//      work-group each) and large components (one team of work-groups);
//   5. the ordering kernels;
//   6. bandwidth/profile of the result and per-graph statistics.
// Small readbacks (status flags, component counts, statistics) synchronise
// the stream a handful of times per call; everything else stays on device.

#include <algorithm>
#include <cstdlib>
#include <cstring>
#include <cstdio>
#include <map>
#include <mutex>
#include <vector>

#include "rcm_common.hpp"

using namespace rcm;

namespace {

thread_local rcm_timings g_timings;
// the launch settings of the current call, copied into g_timings at its end
thread_local int32_t g_used[6];

inline size_t align_up(size_t x, size_t a = 256) { return (x + a - 1) / a * a; }

struct Opts {
  int pp_variant = 0;
  int reverse_mode = 0;
  int check_full = 0;
  int team_size = 0;  // 0: by size, see team_for
  int threads = 256;
  int small_threads = 256;
  int small_cutoff = 1 << 18;
  int narrow_cutoff = 256;
  int max_teams = 16;
  // batched call with team_size and max_teams left to auto: a batch of many
  // large components, none of them very large, gets many small teams
  bool batch_auto = false;
  int rebalance = 8;
  int label_mode = 0;
  int async_search = 1;
  int label_team = 64;
  int search_round = 16;
  int mode = 0;  // 0 auto, 1 team kernel only, 2 one-work-group LDS engine only
  int relabel_levels = 4096;  // renumber a long whole-graph component (0 = never)
  uint32_t shuffle = 0;                 // seed of the work-group / task shuffle
  const int32_t* abort_flag = nullptr;  // the caller's abort flag (host address) ...
  const int32_t* abort_dev = nullptr;   // ... and the address the kernels read
};

// Abort flags made by rcm_abort_flag_create, host address -> device
// address; an option naming any other pointer is rejected, since the
// kernels read the flag as coherent host memory.
std::mutex g_flag_mutex;
std::map<const int32_t*, const int32_t*> g_flags;

bool known_flag(const int32_t* f, const int32_t** dev) {
  *dev = nullptr;
  if (!f) return true;
  std::lock_guard<std::mutex> lk(g_flag_mutex);
  auto it = g_flags.find(f);
  if (it == g_flags.end()) return false;
  *dev = it->second;
  return true;
}

// The caller's flag as the host sees it now.
inline bool abort_set(const Opts& o) {
  return o.abort_flag && __atomic_load_n(o.abort_flag, __ATOMIC_ACQUIRE) != 0;
}

// RCM_ELL=0 keeps the team kernel on the CSR for graphs whose rows would
// fit the fixed-stride copy, for tests of both paths.
inline bool ell_enabled() {
  const char* e = std::getenv("RCM_ELL");
  return !(e && e[0] == '0');
}

// RCM_WINDOW=0 keeps the window engine out (renumbered components then go
// to the team kernel), for tests of that path.
inline bool window_enabled() {
  const char* e = std::getenv("RCM_WINDOW");
  return !(e && e[0] == '0');
}

// Auto team size of a single graph: all compute units for a large graph
// (its asynchronous search passes speed up up to one work-group per CU),
// 64 for a smaller one, whose narrow levels only pay for more barrier slots.
inline int team_for(const Opts& o, int64_t n) {
  if (o.team_size > 0) return o.team_size;
  return n >= (1 << 18) ? 256 : 64;
}

// Auto values differ for batched calls: many components of many graphs share
// one launch, so more, smaller teams take the larger ones (measured on the
// 512-graph batch and on the request pool of the serving benchmark); see
// also batch_auto.
bool parse_options(const rcm_options* o, Opts* out, bool batched = false) {
  Opts r;
  if (batched) {
    r.small_cutoff = 1 << 16;
    r.team_size = 8;
    r.max_teams = 32;
    r.batch_auto = !o || (o->team_size == 0 && o->max_teams == 0);
  }
  if (o) {
    if (o->pp_variant != 0 && o->pp_variant != 1) return false;
    if (o->reverse_mode != 0 && o->reverse_mode != 1) return false;
    if (o->check_full != 0 && o->check_full != 1) return false;
    if (o->team_size < 0 || o->team_size > kMaxTeam) return false;
    if (o->block_threads != 0 && o->block_threads != 256 && o->block_threads != 512)
      return false;
    if (o->small_cutoff < 0) return false;
    if (o->narrow_cutoff < -1) return false;
    if (o->small_threads != 0 && o->small_threads != 256 && o->small_threads != 512)
      return false;
    if (o->max_teams < 0 || o->max_teams > kMaxConcurrentTeams) return false;
    if (o->rebalance_levels < 0) return false;
    if (o->label_mode < 0 || o->label_mode > 2) return false;
    if (o->async_search < -1 || o->async_search > 1) return false;
    if (o->label_team < 0 || o->label_team > kMaxTeam) return false;
    if (o->search_round < 0) return false;
    if (o->mode < 0 || o->mode > 2) return false;
    if (o->relabel_levels < -1) return false;
    if (!known_flag(o->abort_flag, &r.abort_dev)) return false;
    r.pp_variant = o->pp_variant;
    r.reverse_mode = o->reverse_mode;
    r.check_full = o->check_full;
    if (o->team_size) r.team_size = o->team_size;
    if (o->block_threads) r.threads = o->block_threads;
    if (o->small_cutoff) r.small_cutoff = o->small_cutoff;
    if (o->narrow_cutoff) r.narrow_cutoff = o->narrow_cutoff;
    if (o->small_threads) r.small_threads = o->small_threads;
    if (o->max_teams) r.max_teams = o->max_teams;
    if (o->rebalance_levels) r.rebalance = o->rebalance_levels;
    r.label_mode = o->label_mode;
    if (o->async_search) r.async_search = o->async_search > 0 ? 1 : 0;
    if (o->label_team) r.label_team = o->label_team;
    if (o->search_round) r.search_round = o->search_round;
    r.mode = o->mode;
    r.shuffle = static_cast<uint32_t>(o->shuffle_seed);
    if (o->relabel_levels) r.relabel_levels = o->relabel_levels > 0 ? o->relabel_levels : 0;
    r.abort_flag = o->abort_flag;
  }
  *out = r;
  return true;
}

// Workspace layout (every region 256-byte aligned).
struct Layout {
  size_t vinfo, beta, parent, flags, pos, csize, seeds, visit, claim, qi, tmp, iperm, dkey;
  size_t sizes, offs, results, t_single, t_small, t_big, scan_blk;
  size_t seg_off, comp_seg_off, segstats, gctl, teams, slots, sub_slots, small_ctl, misc, sched;
  size_t rowptr_g, colidx_g;
  size_t ell;  // single graphs: the fixed-stride copy of bounded rows (0 = none)
  size_t total;
};

Layout make_layout(int64_t n, int64_t nnz, int64_t nseg, bool batched, int teams_small) {
  Layout L;
  size_t off = 0;
  auto take = [&](size_t bytes) {
    size_t at = off;
    off += align_up(bytes);
    return at;
  };
  const size_t N = static_cast<size_t>(n);
  L.vinfo = take(16 * N);
  L.beta = take(4 * N);
  L.parent = take(4 * N);
  L.flags = take(4 * N);
  L.pos = take(4 * N + 4 * (N / 4096 + 2));
  L.csize = take(4 * N);
  L.seeds = take(4 * N);
  L.visit = take(4 * N);
  L.claim = take(4 * N);
  L.qi = take(16 * N);
  L.tmp = take(4 * N);
  L.iperm = take(4 * N);
  L.dkey = take(8 * N);
  L.sizes = take(4 * N);
  L.offs = take(4 * N);
  L.results = take(sizeof(CompResult) * N);
  L.t_single = take(sizeof(CompTask) * N);
  L.t_small = take(sizeof(CompTask) * N);
  // (at least 4 KB: the level orders' sort uses the task lists as scratch,
  // with a fixed part of about 2 KB however small the graph)
  L.t_big = take(std::max<size_t>(sizeof(CompTask) * N, 4096));
  L.scan_blk = take(4 * (N / 4096 + 2));
  L.seg_off = take(4 * static_cast<size_t>(nseg + 1));
  L.comp_seg_off = take(4 * static_cast<size_t>(nseg + 1));
  L.segstats = take(sizeof(SegStats) * static_cast<size_t>(nseg));
  L.gctl = take(sizeof(GlobalCtl));
  L.teams = take(sizeof(TeamCtl) * kMaxConcurrentTeams);
  L.slots = take(sizeof(TeamSlots) * kMaxConcurrentTeams);
  L.sub_slots = take(sizeof(TeamSlots) * kMaxConcurrentTeams);
  L.small_ctl = take(sizeof(TeamCtl) * static_cast<size_t>(teams_small));
  L.misc = take(256);
  L.sched = take(128 * sizeof(int32_t));
  if (batched) {
    L.rowptr_g = take(4 * (N + 1));
    L.colidx_g = take(4 * static_cast<size_t>(nnz));
    L.ell = 0;
  } else {
    L.rowptr_g = L.colidx_g = 0;
    L.ell = take(4 * kEllWidth * N);
  }
  L.total = off;
  return L;
}

constexpr int kSmallTeams = 1024;
constexpr int kWideBatchTeam = 4;  // team size of a batch's many-teams layout

// The calling thread's timing events on the current device, created on its
// first timed call there and kept (creating ten events costs more than a
// small graph's whole ordering).
bool thread_events(hipEvent_t** out) {
  thread_local std::map<int, std::vector<hipEvent_t>> pool;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return false;
  auto it = pool.find(dev);
  if (it == pool.end()) {
    std::vector<hipEvent_t> ev(10);
    for (auto& x : ev)
      if (hipEventCreate(&x) != hipSuccess) return false;
    it = pool.emplace(dev, std::move(ev)).first;
  }
  *out = it->second.data();
  return true;
}

// Phase timing with HIP events on the call's stream (RCM_TIMING=1).
// Event slots: 0 start, 1 checks done, 2/3 around the component search,
// 4 ordering done, 5 statistics done; kernel slots around the launches.
struct Timer {
  bool on;
  hipStream_t s;
  hipEvent_t* ev = nullptr;   // 6 phase events, then kev
  hipEvent_t* kev = nullptr;  // 4 kernel events
  bool used[6] = {false, false, false, false, false, false};
  bool kused[2] = {false, false};
  long long clk[32] = {};
  // allow = false: never (the allocation-free entry point creates no events)
  Timer(hipStream_t st, bool allow) : s(st) {
    const char* e = std::getenv("RCM_TIMING");
    on = allow && e && e[0] == '1';
    if (on) {
      on = thread_events(&ev);
      kev = on ? ev + 6 : nullptr;
    }
  }
  void mark(int slot) {
    if (!on) return;
    (void)hipEventRecord(ev[slot], s);
    used[slot] = true;
  }
  void kmark(int which, bool start) {
    if (!on) return;
    (void)hipEventRecord(kev[2 * which + (start ? 0 : 1)], s);
    kused[which] = true;
  }
  float span(int a, int b) {
    float ms = 0.f;
    if (used[a] && used[b]) (void)hipEventElapsedTime(&ms, ev[a], ev[b]);
    return ms;
  }
  void finish() {
    rcm_timings t{};
    std::memcpy(&t.used_mode, g_used, sizeof(g_used));
    if (on && used[0]) {
      int last = 0;
      for (int i = 0; i < 6; ++i)
        if (used[i]) last = i;
      (void)hipEventSynchronize(ev[last]);
      t.validate_ms = span(0, 1);
      t.components_ms = span(2, 3);
      t.order_ms = span(1, 4);
      t.after_ms = span(4, 5);
      t.total_ms = span(0, last);
      if (kused[0]) (void)hipEventElapsedTime(&t.small_kernel_ms, kev[0], kev[1]);
      if (kused[1]) (void)hipEventElapsedTime(&t.team_kernel_ms, kev[2], kev[3]);
      t.team_pp_ms = static_cast<float>(clk[0] * 1e-5);
      t.team_label_ms = static_cast<float>(clk[1] * 1e-5);
      t.team_pp_levels = static_cast<int32_t>(clk[2]);
      t.team_label_levels = static_cast<int32_t>(clk[3]);
      for (int i = 0; i < 28; ++i) t.phase_ticks[i] = clk[4 + i];
    }
    g_timings = t;
  }
};

#define HIP_TRY(expr)                      \
  do {                                     \
    hipError_t _he = (expr);               \
    if (_he != hipSuccess) return RCM_ERR_HIP; \
  } while (0)

// With RCM_DEBUG=1 the library reports on stderr where a device-side check
// failed (site, component, pass, level, frontier bounds, block end).
void report_device_error(const GlobalCtl* gctl, hipStream_t s) {
  const char* e = std::getenv("RCM_DEBUG");
  if (!(e && e[0] == '1')) return;
  int32_t d[9] = {};
  if (hipMemcpyAsync(d, &gctl->error, sizeof(d), hipMemcpyDeviceToHost, s) != hipSuccess) return;
  if (hipStreamSynchronize(s) != hipSuccess) return;
  std::fprintf(stderr,
               "rcm: device error %d at site %d component %d pass %d level %d frontier [%d, %d) "
               "block end %d\n", d[0], d[1], d[2], d[3], d[4], d[5], d[6], d[7]);
}

// Read a few device ints synchronously.
rcm_status read_ints(int32_t* host, const int32_t* dev, int count, hipStream_t s) {
  HIP_TRY(hipMemcpyAsync(host, dev, sizeof(int32_t) * count, hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  return RCM_OK;
}

// The ordering of a (possibly segmented) graph whose CSR is global.
rcm_status run(const Graph& gin, const int32_t* seg_off_host, const Opts& opt, char* ws,
               const Layout& L, int32_t* perm_out, int32_t* iperm_out, rcm_stats* stats_host,
               hipStream_t s, Timer& timer) {
  Graph g = gin;
  const size_t N = static_cast<size_t>(g.n);
  int4* vinfo = reinterpret_cast<int4*>(ws + L.vinfo);
  int32_t* beta = reinterpret_cast<int32_t*>(ws + L.beta);
  int32_t* parent = reinterpret_cast<int32_t*>(ws + L.parent);
  int32_t* flags = reinterpret_cast<int32_t*>(ws + L.flags);
  int32_t* pos = reinterpret_cast<int32_t*>(ws + L.pos);
  int32_t* csize = reinterpret_cast<int32_t*>(ws + L.csize);
  int32_t* seeds = reinterpret_cast<int32_t*>(ws + L.seeds);
  int32_t* visit = reinterpret_cast<int32_t*>(ws + L.visit);
  uint32_t* claim = reinterpret_cast<uint32_t*>(ws + L.claim);
  int4* qi = reinterpret_cast<int4*>(ws + L.qi);
  int32_t* tmp = reinterpret_cast<int32_t*>(ws + L.tmp);
  int32_t* iperm = iperm_out ? iperm_out : reinterpret_cast<int32_t*>(ws + L.iperm);
  int32_t* sizes = reinterpret_cast<int32_t*>(ws + L.sizes);
  int32_t* offs = reinterpret_cast<int32_t*>(ws + L.offs);
  CompResult* results = reinterpret_cast<CompResult*>(ws + L.results);
  CompTask* t_single = reinterpret_cast<CompTask*>(ws + L.t_single);
  CompTask* t_small = reinterpret_cast<CompTask*>(ws + L.t_small);
  CompTask* t_big = reinterpret_cast<CompTask*>(ws + L.t_big);
  int32_t* scan_blk = reinterpret_cast<int32_t*>(ws + L.scan_blk);
  int32_t* seg_off = reinterpret_cast<int32_t*>(ws + L.seg_off);
  int32_t* comp_seg_off = reinterpret_cast<int32_t*>(ws + L.comp_seg_off);
  SegStats* segstats = reinterpret_cast<SegStats*>(ws + L.segstats);
  GlobalCtl* gctl = reinterpret_cast<GlobalCtl*>(ws + L.gctl);
  TeamCtl* teams = reinterpret_cast<TeamCtl*>(ws + L.teams);
  TeamSlots* slots = reinterpret_cast<TeamSlots*>(ws + L.slots);
  TeamCtl* small_ctl = reinterpret_cast<TeamCtl*>(ws + L.small_ctl);
  int32_t* misc = reinterpret_cast<int32_t*>(ws + L.misc);  // [0..2] errors, [4] ncomp, [8..10] counts
  int32_t* sched = reinterpret_cast<int32_t*>(ws + L.sched);

  if (abort_set(opt)) return RCM_ERR_ABORTED;
  HIP_TRY(hipMemcpyAsync(seg_off, seg_off_host, sizeof(int32_t) * (g.nseg + 1),
                         hipMemcpyHostToDevice, s));
  g.seg_off = seg_off;
  HIP_TRY(hipMemsetAsync(misc, 0, 256, s));
  HIP_TRY(hipMemsetAsync(segstats, 0, sizeof(SegStats) * g.nseg, s));

  timer.mark(0);
  // 2. checks, degrees, input bandwidth/profile
  int4* ell = L.ell != 0 && N > 0 ? reinterpret_cast<int4*>(ws + L.ell) : nullptr;
  HIP_TRY(launch_validate_scan(g, vinfo, beta, segstats, misc + 0, misc + 3, ell, misc + 6, s));
  int32_t h[7];
  rcm_status st = read_ints(h, misc, 7, s);
  if (st != RCM_OK) return st;
  if (h[0]) return RCM_ERR_BAD_CSR;
  // a row longer than the copy's width: the traversal reads the CSR
  if (h[6] || !ell_enabled()) ell = nullptr;
  if (h[3]) {
    // rows too long for the scan's own duplicate check
    HIP_TRY(launch_dup_long(g, misc + 0, s));
    st = read_ints(h, misc, 1, s);
    if (st != RCM_OK) return st;
    if (h[0]) return RCM_ERR_BAD_CSR;
  }
  // 3. optional full check
  if (opt.check_full) {
    HIP_TRY(launch_full_check(g, misc + 1, misc + 2, s));
    st = read_ints(h, misc, 3, s);
    if (st != RCM_OK) return st;
    if (h[1]) return RCM_ERR_BAD_CSR;
    if (h[2]) return RCM_ERR_NOT_SYMMETRIC;
  }
  timer.mark(1);
  // 4-5. components and ordering
  HIP_TRY(hipMemsetAsync(visit, 0, 4 * N, s));
  HIP_TRY(hipMemsetAsync(claim, 0xFF, 4 * N, s));
  HIP_TRY(hipMemsetAsync(gctl, 0, sizeof(GlobalCtl), s));
  BfsParams P;
  P.rowptr = g.rowptr;
  P.colidx = g.colidx;
  P.vinfo = vinfo;
  P.visit = visit;
  P.claim = claim;
  P.qi = qi;
  P.tmp = tmp;
  P.perm = perm_out;
  P.iperm = iperm;
  P.results = results;
  P.gctl = gctl;
  P.n = g.n;
  P.nnz = g.nnz;
  P.pp_variant = opt.pp_variant;
  P.reverse_mode = opt.reverse_mode;
  P.narrow_cutoff = opt.narrow_cutoff;
  P.rebalance = opt.rebalance;
  P.label_mode = opt.label_mode;
  P.async_search = opt.async_search;
  P.seg_off = g.seg_off;
  P.nseg = g.nseg;
  P.dkey = reinterpret_cast<unsigned long long*>(ws + L.dkey);
  P.abort_flag = opt.abort_dev;
  P.shuffle = opt.shuffle;
  P.relabel_levels = 0;
  P.resume = 0;
  P.relabelled = 0;
  P.new_of_old = nullptr;
  P.ell = ell;
  // distance words of the asynchronous passes start below every pass tag
  if (opt.async_search) HIP_TRY(hipMemsetAsync(P.dkey, 0, 8 * static_cast<size_t>(g.n), s));
  P.teams = teams;
  P.slots = slots;
  P.sub_slots = reinterpret_cast<TeamSlots*>(ws + L.sub_slots);
  P.label_team = opt.label_team;
  P.search_round = opt.search_round;
  P.small_teams = small_ctl;
  P.queues = misc + 16;
  const int team_auto = team_for(opt, g.n);
  P.team_size = team_auto;
  // One launch of the ordering kernel: teams of team_size work-groups take
  // the large components, largest first, and single-work-group blocks the
  // small ones; team work-groups join the small list once the large one is
  // empty.  With large components the launch is cooperative, so it is sized
  // to what is resident at once, half of it left to single-work-group blocks
  // when there are small components too.
  //
  // A batch's large components differ in time far more than in size (a 2D
  // grid has many more levels than a 3D grid of the same size).  With more
  // of them than teams, a largest-first queue sometimes hands a long one to
  // a team late, and the call runs a whole task longer (two modes, 55 and
  // 90 ms, on the 512-graph batch).  So when an auto-configured batch has
  // more large components than that layout starts at once and no graph of
  // 2^18 vertices or more (those want large teams), it runs teams of 4 over
  // every resident work-group instead: all large components start at once,
  // and the small ones follow when the team work-groups turn to them.
  int32_t largest_graph = 0;
  for (int i = 0; i < g.nseg; ++i)
    largest_graph = std::max(largest_graph, seg_off_host[i + 1] - seg_off_host[i]);
  auto launch = [&](const CompTask* big, int32_t n_big, const CompTask* small, int32_t n_small,
                    int kslot, bool copy_clk) -> rcm_status {
    P.big_tasks = big;
    P.n_big = n_big;
    P.tasks = small;
    P.ntasks = n_small;
    int blocks = 0, threads = 0, nteams = 0;
    if (n_big > 0) {
      threads = opt.threads;
      const int resident = max_team_blocks(threads);
      if (resident < 1) return RCM_ERR_HIP;
      // a team never exceeds what is resident at once (the launch is
      // cooperative)
      int team = std::min(team_auto, resident);
      int room = n_small > 0 ? std::max(resident / 2, team) : resident;
      int cap = opt.max_teams;
      if (opt.batch_auto && largest_graph < (1 << 18) && n_big > room / team) {
        team = std::min(kWideBatchTeam, resident);
        room = resident;
        cap = kMaxConcurrentTeams;
      }
      P.team_size = team;
      nteams = std::max(1, std::min({n_big, cap, room / team}));
      P.big_blocks = nteams * team;
      const int extra = n_small > 0 ? std::min(n_small, resident - P.big_blocks) : 0;
      blocks = std::min(P.big_blocks + std::max(extra, 0), kSmallTeams);
    } else {
      threads = opt.small_threads;
      P.big_blocks = 0;
      blocks = std::min(n_small, kSmallTeams);
    }
    if (blocks <= 0) return RCM_OK;
    HIP_TRY(hipMemsetAsync(P.queues, 0, 2 * sizeof(int32_t), s));
    if (nteams > 0) {
      HIP_TRY(hipMemsetAsync(teams, 0, sizeof(TeamCtl) * nteams, s));
      HIP_TRY(hipMemsetAsync(slots, 0, sizeof(TeamSlots) * nteams, s));
      HIP_TRY(hipMemsetAsync(P.sub_slots, 0, sizeof(TeamSlots) * nteams, s));
    }
    if (n_small > 0) HIP_TRY(hipMemsetAsync(small_ctl, 0, sizeof(TeamCtl) * blocks, s));
    if (n_big > 0) {
      g_used[1] = P.team_size;
      g_used[2] = threads;
      g_used[3] = opt.label_team;
      g_used[4] = opt.search_round;
    }
    g_used[5] = opt.small_cutoff;
    if (abort_set(opt)) return RCM_ERR_ABORTED;
    timer.kmark(kslot, true);
    HIP_TRY(launch_order(P, blocks, threads, s));
    timer.kmark(kslot, false);
    if (copy_clk && timer.on) {
      HIP_TRY(hipMemcpyAsync(timer.clk, teams[0].clk, sizeof(timer.clk), hipMemcpyDeviceToHost,
                             s));
      HIP_TRY(hipStreamSynchronize(s));
    }
    return RCM_OK;
  };
  // The component of vertex 0 has the lowest seed of all, so its label block
  // starts at 0 whatever the other components are: it is ordered first by
  // the team, its size found by its first level structure, and the
  // component search below only has to cover the vertices it did not reach.
  // (Single graphs only; a batch runs the search over every graph.)
  const bool head = g.nseg == 1;
  int32_t head_size = 0;
  if (head) {
    const CompTask ht{0, -1, 0, 0, opt.reverse_mode == 1 ? g.n - 1 : -1};
    const CompResult hr{0, 0, 0, 0, 0, 0, 0};
    HIP_TRY(hipMemcpyAsync(t_big, &ht, sizeof(ht), hipMemcpyHostToDevice, s));
    HIP_TRY(hipMemcpyAsync(results, &hr, sizeof(hr), hipMemcpyHostToDevice, s));
    HIP_TRY(hipMemsetAsync(seeds, 0, sizeof(int32_t), s));
    // a long component stops after its first level structure (asynchronous
    // passes and labelled orders only) when its renumbered columns fit the
    // component results' region (see below): at most 8 entries per vertex
    const size_t ci_room = L.t_single - L.results - 256;
    P.relabel_levels = opt.label_mode == 0 && opt.async_search &&
                               4 * static_cast<size_t>(g.nnz) <= ci_room
                           ? opt.relabel_levels
                           : 0;
    st = launch(t_big, 1, nullptr, 0, 1, true);
    P.relabel_levels = 0;
    if (st != RCM_OK) return st;
    int32_t hres[8];
    HIP_TRY(hipMemcpyAsync(hres, results, sizeof(CompResult), hipMemcpyDeviceToHost, s));
    // error, diag[8], p1_stop, p1_ecc, p1_tag, p1_size, p1_lastkey (two words)
    int32_t gc[15];
    st = read_ints(gc, &gctl->error, 15, s);
    if (st != RCM_OK) return st;
    if (gc[0]) report_device_error(gctl, s);
    if (gc[0] == RCM_ERR_NOT_SYMMETRIC) return RCM_ERR_NOT_SYMMETRIC;
    if (gc[0]) return RCM_ERR_ABORTED;
    if (gc[9]) {
      // Renumber the component in that structure's level order and order it
      // from there in a second launch.  Until that launch ends, only the
      // regions of the component search (which runs afterwards, on the
      // caller's numbering) and of the other components' tasks and results
      // are free: they hold the maps, the new rows and the new records.  The
      // second launch gets a visited array of its own, so that the stamps
      // of the first structure, which the component search reads, stay.
      const int32_t ecc1 = gc[10];
      const uint32_t tag1 = static_cast<uint32_t>(gc[11]);
      const int32_t size1 = gc[12];
      if (ecc1 < 0 || ecc1 >= size1 || size1 < 1 || size1 > g.n) return RCM_ERR_HIP;
      int32_t* err = misc + 12;
      int32_t* counted = misc + 13;
      int32_t* rowptr_new = pos;
      int32_t* colidx_new = reinterpret_cast<int32_t*>(ws + L.results + 256);
      int4* vinfo_new = reinterpret_cast<int4*>(ws + L.t_single);
      static_assert(sizeof(CompTask) >= sizeof(int4), "a task list holds the records");
      HIP_TRY(hipMemsetAsync(err, 0, 2 * sizeof(int32_t), s));
      HIP_TRY(launch_relabel(g, vinfo, P.dkey, tag1, ecc1, size1, csize, flags, parent, scan_blk,
                             sizes, offs, rowptr_new, colidx_new,
                             static_cast<int64_t>(ci_room / 4), vinfo_new, err, counted, s));
      st = read_ints(h, err, 2, s);
      if (st != RCM_OK) return st;
      if (h[0] || h[1] != size1) {
        if (std::getenv("RCM_DEBUG"))
          std::fprintf(stderr, "rcm: the first level structure counts %d of %d vertices\n",
                       h[1], size1);
        return RCM_ERR_NOT_SYMMETRIC;
      }
      // First the window engine: one work-group walks the remaining
      // passes from LDS along the renumbered ids.  It declines a component
      // whose rows or levels do not fit it, and the team kernel then
      // resumes the ordering on the renumbered copy.
      bool windowed = false;
      if (window_enabled()) {
        unsigned long long lastkey1 = 0;
        std::memcpy(&lastkey1, &gc[13], sizeof(lastkey1));
        WinParams W{};
        W.n = g.n;
        W.size = size1;
        W.colidx = colidx_new;
        W.vinfo = vinfo_new;
        W.new_of_old = sizes;
        // (the team kernel's records, 16 bytes a vertex, are free here: the
        // row records take 8, the order 4; the first structure's distance
        // words, read by the renumbering, hold the claims)
        W.ell = reinterpret_cast<uint2*>(ws + L.qi);
        W.order = reinterpret_cast<int32_t*>(ws + L.qi + 8 * static_cast<size_t>(size1));
        W.ell_flag = misc + 14;
        W.claim = reinterpret_cast<uint32_t*>(P.dkey);
        W.ecc1 = ecc1;
        W.lastkey1 = lastkey1;
        W.pp_variant = opt.pp_variant;
        W.anchor = ht.anchor >= 0 ? ht.anchor : size1 - 1;
        W.perm = perm_out;
        W.iperm = iperm;
        W.result = results;
        W.status = misc + 15;
        W.abort_flag = opt.abort_dev;
        if (abort_set(opt)) return RCM_ERR_ABORTED;
        HIP_TRY(launch_window_order(W, s));
        int32_t wst = 0;
        st = read_ints(&wst, misc + 15, 1, s);
        if (st != RCM_OK) return st;
        if (wst == RCM_ERR_NOT_SYMMETRIC) return RCM_ERR_NOT_SYMMETRIC;
        if (wst == RCM_ERR_ABORTED) return RCM_ERR_ABORTED;
        windowed = wst == 0;
        // declined: the team kernel's distance words start below every pass
        // tag again
        if (!windowed) HIP_TRY(hipMemsetAsync(P.dkey, 0, 8 * static_cast<size_t>(g.n), s));
      }
      if (!windowed) {
        long long clk_first[32];
        std::memcpy(clk_first, timer.clk, sizeof(clk_first));
        const CompTask rt{0, size1, 0, 0, ht.anchor};
        HIP_TRY(hipMemcpyAsync(t_big, &rt, sizeof(rt), hipMemcpyHostToDevice, s));
        int32_t* visit2 = csize;  // free again once the renumbering is built
        HIP_TRY(hipMemsetAsync(visit2, 0, 4 * N, s));
        const BfsParams saved = P;
        P.colidx = colidx_new;
        P.rowptr = rowptr_new;
        P.vinfo = vinfo_new;
        P.visit = visit2;
        P.new_of_old = sizes;
        P.relabelled = 1;
        P.resume = 1;
        P.ell = nullptr;  // the copy holds the caller's numbering
        st = launch(t_big, 1, nullptr, 0, 1, true);
        P = saved;
        if (st != RCM_OK) return st;
        if (timer.on)
          for (int i = 0; i < 32; ++i) timer.clk[i] += clk_first[i];
      }
      HIP_TRY(hipMemcpyAsync(hres, results, sizeof(CompResult), hipMemcpyDeviceToHost, s));
      st = read_ints(gc, &gctl->error, 1, s);
      if (st != RCM_OK) return st;
      if (gc[0]) report_device_error(gctl, s);
      if (gc[0] == RCM_ERR_NOT_SYMMETRIC) return RCM_ERR_NOT_SYMMETRIC;
      if (gc[0]) return RCM_ERR_ABORTED;
      // the other components claim in the caller's numbering from scratch
      if (size1 < g.n) HIP_TRY(hipMemsetAsync(claim, 0xFF, 4 * N, s));
      g_used[0] = windowed ? 4 : 3;  // the window engine / the team kernel, renumbered
    }
    head_size = hres[4];
    if (head_size < 1 || head_size > g.n) return RCM_ERR_HIP;
  }
  int32_t ncomp = head ? 1 : 0;
  if (head_size < g.n) {
    int32_t* seeds_rest = head ? seeds + 1 : seeds;
    timer.mark(2);
    HIP_TRY(launch_components(g, head ? visit : nullptr, parent, csize, flags, pos, seeds_rest,
                              misc + 4, misc + 5, s));
    st = read_ints(h, misc + 4, 2, s);
    if (st != RCM_OK) return st;
    if (h[1]) {
      if (std::getenv("RCM_DEBUG")) std::fprintf(stderr, "rcm: edge into the ordered head\n");
      return RCM_ERR_NOT_SYMMETRIC;
    }
    const int32_t nrest = h[0];
    ncomp += nrest;
    HIP_TRY(launch_tasks(g, nrest, seeds_rest, csize, opt.small_cutoff, opt.reverse_mode,
                         head_size, head ? 1 : 0, t_single, t_small, t_big, misc + 8, sizes, offs,
                         scan_blk, results, sched, s));
    st = read_ints(h, misc + 8, 4, s);
    if (st != RCM_OK) return st;
    // every vertex must belong to exactly one component (only an asymmetric
    // pattern can break this)
    if (head_size + h[3] != g.n) {
      if (std::getenv("RCM_DEBUG"))
        std::fprintf(stderr, "rcm: components cover %d + %d of %d vertices\n", head_size, h[3],
                     g.n);
      return RCM_ERR_NOT_SYMMETRIC;
    }
    timer.mark(3);
    const int32_t n_single = h[0], n_small = h[1], n_big = h[2];
    HIP_TRY(launch_singletons(t_single, n_single, perm_out, iperm,
                              opt.label_mode ? reinterpret_cast<int32_t*>(claim) : nullptr,
                              results, s));
    st = launch(t_big, n_big, t_small, n_small, 0, false);
    if (st != RCM_OK) return st;
  }
  timer.mark(4);
  st = read_ints(h, &gctl->error, 1, s);
  if (st != RCM_OK) return st;
  if (h[0]) report_device_error(gctl, s);
  if (h[0] == RCM_ERR_NOT_SYMMETRIC) return RCM_ERR_NOT_SYMMETRIC;
  if (h[0]) return RCM_ERR_ABORTED;
  if (opt.label_mode != 0) {
    // level orders: sort by the keys the ordering kernel left in claim
    // (the task lists and qi are free by now and serve as scratch)
    const size_t temp_need = level_order_temp_bytes(g.n);
    const size_t temp_have = L.scan_blk - L.t_single;
    if (temp_need == 0 || temp_need > temp_have) return RCM_ERR_WORKSPACE_TOO_SMALL;
    int32_t deg_bits = 1;
    while (deg_bits < 31 && (1ll << deg_bits) <= g.nnz) ++deg_bits;
    HIP_TRY(launch_level_order(g.n, deg_bits, opt.label_mode == 2, vinfo,
                               reinterpret_cast<const int32_t*>(claim), perm_out, iperm,
                               ws + L.qi, ws + L.t_single, temp_have, s));
  }
  // 6. result statistics
  HIP_TRY(launch_bw_after(g, perm_out, iperm, beta, segstats, s));
  HIP_TRY(launch_comp_stats(g, ncomp, seeds, results, comp_seg_off, segstats,
                            opt.label_mode == 0 || opt.pp_variant == 1 ? 1 : 0, s));
  if (stats_host) {
    std::vector<SegStats> hs(g.nseg);
    HIP_TRY(hipMemcpyAsync(hs.data(), segstats, sizeof(SegStats) * g.nseg,
                           hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    for (int i = 0; i < g.nseg; ++i) {
      rcm_stats& o = stats_host[i];
      o.bandwidth_before = static_cast<int64_t>(hs[i].bw_before);
      o.profile_before = static_cast<int64_t>(hs[i].prof_before);
      o.bandwidth_after = static_cast<int64_t>(hs[i].bw_after);
      o.profile_after = static_cast<int64_t>(hs[i].prof_after);
      o.edges_traversed = static_cast<int64_t>(hs[i].edges);
      o.num_components = hs[i].ncomp;
      o.pseudo_diameter = hs[i].diameter;
      o.num_bfs = hs[i].nbfs;
      o.num_levels = hs[i].nlevels;
    }
  } else {
    HIP_TRY(hipStreamSynchronize(s));
  }
  timer.mark(5);
  return RCM_OK;
}

// Turns the graphs' local CSR into the union's.  Each block takes tiles of
// kGlobTile consecutive vertices or entries; a tile finds the graph of its
// first element by binary search once, and its threads step forward over the
// (rare) graph boundaries inside it, so the loads and stores stay coalesced.
constexpr int kGlobThreads = 256;
constexpr int kGlobPer = 8;
constexpr int32_t kGlobTile = kGlobThreads * kGlobPer;

__global__ void __launch_bounds__(kGlobThreads)
k_globalize(int32_t G, const int32_t* __restrict__ vo, const int32_t* __restrict__ no,
            const int32_t* __restrict__ rowptr_cat, const int32_t* __restrict__ colidx_cat,
            int32_t N, int32_t NNZ, int32_t* __restrict__ rowptr_g,
            int32_t* __restrict__ colidx_g, int32_t* __restrict__ err) {
  const int64_t v_tiles = (static_cast<int64_t>(N) + kGlobTile - 1) / kGlobTile;
  const int64_t k_tiles = (static_cast<int64_t>(NNZ) + kGlobTile - 1) / kGlobTile;
  for (int64_t t = blockIdx.x; t < v_tiles + k_tiles; t += gridDim.x) {
    const bool rows = t < v_tiles;
    const int64_t base = (rows ? t : t - v_tiles) * kGlobTile;
    const int32_t end = rows ? N : NNZ;
    const int32_t* off = rows ? vo : no;
    int g = find_segment(off, G, static_cast<int32_t>(base));
    for (int j = 0; j < kGlobPer; ++j) {
      const int64_t x = base + static_cast<int64_t>(j) * kGlobThreads + threadIdx.x;
      if (x >= end) break;
      const int32_t i = static_cast<int32_t>(x);
      while (g + 1 < G && i >= off[g + 1]) ++g;
      if (rows) {
        rowptr_g[i] = no[g] + rowptr_cat[vo[g] + g + (i - vo[g])];
      } else {
        colidx_g[i] = colidx_cat[i] + vo[g];
      }
    }
  }
  const int32_t t0 = blockIdx.x * blockDim.x + threadIdx.x;
  const int32_t stride = gridDim.x * blockDim.x;
  if (t0 == 0) rowptr_g[N] = NNZ;
  for (int32_t g = t0; g < G; g += stride) {
    const int32_t n_g = vo[g + 1] - vo[g];
    const int32_t first = rowptr_cat[vo[g] + g];
    const int32_t last = rowptr_cat[vo[g] + g + n_g];
    if (first != 0 || last != no[g + 1] - no[g]) atomicOr(err, 1);
  }
}

__global__ void k_localize(int32_t N, const int32_t* __restrict__ vo, int32_t G,
                           int32_t* __restrict__ perm) {
  for (int32_t k = blockIdx.x * blockDim.x + threadIdx.x; k < N; k += gridDim.x * blockDim.x)
    perm[k] -= vo[find_segment(vo, G, k)];
}

rcm_status check_common(int32_t n, const rcm_options* opts, Opts* o) {
  if (n < 0) return RCM_ERR_INVALID_ARGUMENT;
  if (!parse_options(opts, o)) return RCM_ERR_INVALID_ARGUMENT;
  return RCM_OK;
}

}  // namespace

extern "C" {

const char* rcm_status_string(rcm_status s) {
  // a C caller may pass any int; reading it as the enum type would be
  // undefined for values outside the enumerators' range
  static_assert(sizeof(rcm_status) == sizeof(int32_t), "rcm_status is a 32-bit int");
  int32_t v = 0;
  std::memcpy(&v, &s, sizeof(v));
  switch (v) {
    case RCM_OK: return "ok";
    case RCM_ERR_INVALID_ARGUMENT: return "invalid argument";
    case RCM_ERR_BAD_CSR: return "malformed CSR pattern";
    case RCM_ERR_NOT_SYMMETRIC: return "pattern is not symmetric";
    case RCM_ERR_WORKSPACE_TOO_SMALL: return "workspace too small";
    case RCM_ERR_OUT_OF_MEMORY: return "out of device memory";
    case RCM_ERR_ABORTED: return "aborted: the abort flag was set or a device-side wait timed out";
    case RCM_ERR_HIP: return "HIP runtime error";
  }
  return "unknown status";
}

void rcm_default_options(rcm_options* opts) {
  if (opts) std::memset(opts, 0, sizeof(*opts));
}

size_t rcm_workspace_bytes(int32_t n, int64_t nnz, const rcm_options* opts) {
  (void)opts;
  if (n <= 0) return 0;
  return make_layout(n, nnz, 1, false, kSmallTeams).total;
}

size_t rcm_batched_workspace_bytes(int32_t num_graphs, int64_t total_vertices, int64_t total_nnz,
                                   const rcm_options* opts) {
  (void)opts;
  if (num_graphs <= 0 || total_vertices <= 0) return 0;
  return make_layout(total_vertices, total_nnz, num_graphs, true, kSmallTeams).total;
}

void rcm_last_timings(rcm_timings* out) {
  if (out) *out = g_timings;
}

rcm_status rcm_abort_flag_create(int32_t** flag_out) {
  if (!flag_out) return RCM_ERR_INVALID_ARGUMENT;
  *flag_out = nullptr;
  void* h = nullptr;
  if (hipHostMalloc(&h, sizeof(int32_t), hipHostMallocMapped | hipHostMallocCoherent) !=
      hipSuccess)
    return RCM_ERR_HIP;
  void* d = nullptr;
  if (hipHostGetDevicePointer(&d, h, 0) != hipSuccess || d == nullptr) {
    (void)hipHostFree(h);
    return RCM_ERR_HIP;
  }
  int32_t* f = static_cast<int32_t*>(h);
  __atomic_store_n(f, 0, __ATOMIC_RELEASE);
  {
    std::lock_guard<std::mutex> lk(g_flag_mutex);
    g_flags[f] = static_cast<const int32_t*>(d);
  }
  *flag_out = f;
  return RCM_OK;
}

void rcm_abort_flag_destroy(int32_t* flag) {
  if (!flag) return;
  {
    std::lock_guard<std::mutex> lk(g_flag_mutex);
    if (g_flags.erase(flag) == 0) return;
  }
  (void)hipHostFree(flag);
}

}  // extern "C"

namespace rcm {

namespace {

// A single graph through the one-work-group LDS engine (rcm_small.hip): one
// launch that reads the entry count itself and declines when the graph does
// not fit, then one readback of its result.  Returns false when the engine
// does not apply (level orders, too many vertices, or it declined), having
// written no output; else true with the call's status in *out.
// The calling thread's pinned, device-mapped result record: the engine's
// kernel writes it where the host reads it, so a call needs no copy back.
// Returns the host view (and the device view in *dev), null if it cannot be
// allocated.
SmallResult* thread_result(SmallResult** dev) {
  thread_local SmallResult* host_view = nullptr;
  thread_local SmallResult* dev_view = nullptr;
  if (host_view == nullptr) {
    void* h = nullptr;
    if (hipHostMalloc(&h, sizeof(SmallResult),
                      hipHostMallocMapped | hipHostMallocCoherent | hipHostMallocPortable) !=
        hipSuccess)
      return nullptr;
    void* d = nullptr;
    if (hipHostGetDevicePointer(&d, h, 0) != hipSuccess || d == nullptr) {
      (void)hipHostFree(h);
      return nullptr;
    }
    host_view = static_cast<SmallResult*>(h);
    dev_view = static_cast<SmallResult*>(d);
  }
  *dev = dev_view;
  return host_view;
}

// RCM_SMALL_ELL=0 keeps the bounded-row engine out (every small graph then
// takes the general one), for tests of the general engine on meshes.
bool small_ell_enabled() {
  const char* e = std::getenv("RCM_SMALL_ELL");
  return !(e && e[0] == '0');
}

bool order_small(int32_t n, const int32_t* rowptr, const int32_t* colidx, int32_t* perm_out,
                 int32_t* iperm_out, rcm_stats* stats, const Opts& o, void* workspace,
                 size_t workspace_bytes, hipStream_t s, bool timing, rcm_status* out,
                 int32_t* nnz_seen) {
  *nnz_seen = -1;
  if (o.label_mode != 0) return false;
  const size_t limit = small_lds_limit();
  if (limit == 0 || small_lds_bytes(n, 0) > limit) return false;
  *out = RCM_OK;
  if (colidx == nullptr) {
    // allowed only without entries
    int32_t nnz = 0;
    if (hipMemcpyAsync(&nnz, rowptr + n, 4, hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess) {
      *out = RCM_ERR_HIP;
      return true;
    }
    if (nnz != 0) {
      *out = RCM_ERR_INVALID_ARGUMENT;
      return true;
    }
    colidx = rowptr;  // never read
  }
  // the single-graph workspace does not depend on the entry count
  const size_t need = make_layout(n, 0, 1, false, kSmallTeams).total;
  // The result record: the thread's pinned one for a regular call; for the
  // allocation-free entry point (timing == false) the workspace's first bytes
  // (a caller's workspace must hold what the call documents whatever part
  // of it the call uses)
  if (workspace && workspace_bytes < need) {
    *out = RCM_ERR_WORKSPACE_TOO_SMALL;
    return true;
  }
  SmallResult* res = nullptr;
  SmallResult* host = timing ? thread_result(&res) : nullptr;
  bool owned = false;
  if (host == nullptr) {
    if (workspace) {
      res = static_cast<SmallResult*>(workspace);
    } else {
      if (hipMallocAsync(reinterpret_cast<void**>(&res), sizeof(SmallResult), s) != hipSuccess) {
        *out = RCM_ERR_OUT_OF_MEMORY;
        return true;
      }
      owned = true;
    }
  }
  Timer timer(s, timing);
  SmallJob job{n, -1, rowptr, colidx, perm_out, iperm_out, 0, 0, res};
  SmallOpts so{o.pp_variant, o.reverse_mode, o.check_full, static_cast<int32_t>(limit),
               o.shuffle, o.abort_dev};
  if (abort_set(o)) {
    *out = RCM_ERR_ABORTED;
    if (owned) {
      (void)hipFreeAsync(res, s);
      (void)hipStreamSynchronize(s);
    }
    return true;
  }
  SmallResult h{};
  auto run_kernel = [&](bool ell) -> bool {
    const hipError_t e =
        ell ? launch_small_ell(job, so, s) : launch_small_order(job, nullptr, 1, so, s);
    if (e != hipSuccess) return false;
    if (host == nullptr && hipMemcpyAsync(&h, res, sizeof(h), hipMemcpyDeviceToHost, s) !=
                               hipSuccess)
      return false;
    if (hipStreamSynchronize(s) != hipSuccess) return false;
    if (host != nullptr) std::memcpy(&h, host, sizeof(h));
    return true;
  };
  timer.mark(0);
  timer.kmark(0, true);
  // the bounded-row engine first where the graph can fit it; it declines
  // graphs with longer rows, which the general engine then takes
  const bool try_ell = small_ell_enabled() && small_ell_lds_bytes(n) <= limit;
  bool ok = true;
  if (try_ell) {
    ok = run_kernel(true);
    g_used[2] = 512;
  }
  if (ok && (!try_ell || h.status == kSmallDeclined)) {
    ok = run_kernel(false);
    g_used[2] = 64;
  }
  if (!ok) *out = RCM_ERR_HIP;
  timer.kmark(0, false);
  timer.mark(5);
  if (owned) {
    (void)hipFreeAsync(res, s);
    (void)hipStreamSynchronize(s);
  }
  timer.finish();
  if (timer.on)
    for (int i = 0; i < 6; ++i) g_timings.phase_ticks[20 + i] = h.ticks[i];
  if (*out != RCM_OK) return true;
  *nnz_seen = h.nnz;
  if (h.status == kSmallDeclined) return false;
  *out = static_cast<rcm_status>(h.status);
  if (*out == RCM_OK && stats) {
    stats->bandwidth_before = static_cast<int64_t>(h.bw_before);
    stats->profile_before = static_cast<int64_t>(h.prof_before);
    stats->bandwidth_after = static_cast<int64_t>(h.bw_after);
    stats->profile_after = static_cast<int64_t>(h.prof_after);
    stats->edges_traversed = static_cast<int64_t>(h.edges);
    stats->num_components = h.ncomp;
    stats->pseudo_diameter = h.diameter;
    stats->num_bfs = h.nbfs;
    stats->num_levels = h.nlevels;
  }
  return true;
}

}  // namespace

rcm_status check_call(int32_t n, const rcm_options* opts) {
  Opts o;
  return check_common(n, opts, &o);
}

rcm_status order_single(int32_t n, const int32_t* rowptr, const int32_t* colidx,
                        int32_t* perm_out, int32_t* iperm_out, rcm_stats* stats,
                        const rcm_options* opts, void* workspace, size_t workspace_bytes,
                        void* stream, bool timing) {
  Opts o;
  rcm_status st = check_common(n, opts, &o);
  if (st != RCM_OK) return st;
  std::memset(g_used, 0, sizeof(g_used));
  if (stats) std::memset(stats, 0, sizeof(*stats));
  if (n == 0) return RCM_OK;
  if (!rowptr || !perm_out) return RCM_ERR_INVALID_ARGUMENT;
  hipStream_t s = static_cast<hipStream_t>(stream);
  // A tuning table: its entry for this graph's size class supplies every
  // launch option left at 0.  The class needs the entry count, which the
  // engine reads itself and the team path reads back anyway, so the table
  // is applied once that count is known; only the engine choice (an exact
  // class's mode 1) can undo an engine result.
  const char* tf = tuning_path(opts);
  auto tuned = [&](int32_t nnz, rcm_options* eff) -> bool {
    *eff = opts ? *opts : rcm_options{};
    return tuning_apply(tf, n, nnz < 0 ? 0 : nnz, 1, eff);
  };
  if (tf) {
    rcm_options probe{};
    if (!tuned(0, &probe)) return RCM_ERR_INVALID_ARGUMENT;  // unreadable or malformed
  }
  if (o.mode != 1) {
    g_used[0] = 2;
    int32_t seen = -1;
    if (order_small(n, rowptr, colidx, perm_out, iperm_out, stats, o, workspace,
                    workspace_bytes, s, timing, &st, &seen)) {
      rcm_options eff{};
      const bool team = tf && o.mode == 0 && st == RCM_OK && seen >= 0 && tuned(seen, &eff) &&
                        eff.mode == 1;
      if (!team) return st;
    } else if (o.mode == 2) {
      return RCM_ERR_INVALID_ARGUMENT;
    }
  }
  g_used[0] = 1;
  int32_t ends[2];
  HIP_TRY(hipMemcpyAsync(&ends[0], rowptr, 4, hipMemcpyDeviceToHost, s));
  HIP_TRY(hipMemcpyAsync(&ends[1], rowptr + n, 4, hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  if (tf) {
    rcm_options eff{};
    if (!tuned(ends[1], &eff) || !parse_options(&eff, &o)) return RCM_ERR_INVALID_ARGUMENT;
  }
  if (ends[0] != 0 || ends[1] < 0) return RCM_ERR_BAD_CSR;
  if (ends[1] > 0 && !colidx) return RCM_ERR_INVALID_ARGUMENT;
  const Layout L = make_layout(n, ends[1], 1, false, kSmallTeams);
  char* ws = static_cast<char*>(workspace);
  bool owned = false;
  if (ws) {
    if (workspace_bytes < L.total) return RCM_ERR_WORKSPACE_TOO_SMALL;
  } else {
    if (hipMallocAsync(reinterpret_cast<void**>(&ws), L.total, s) != hipSuccess)
      return RCM_ERR_OUT_OF_MEMORY;
    owned = true;
  }
  Timer timer(s, timing);
  Graph g{n, ends[1], rowptr, colidx, 1, nullptr};
  const int32_t seg_host[2] = {0, n};
  st = run(g, seg_host, o, ws, L, perm_out, iperm_out, stats, s, timer);
  if (owned) {
    (void)hipFreeAsync(ws, s);
    (void)hipStreamSynchronize(s);
  }
  timer.finish();
  return st;
}

}  // namespace rcm

extern "C" {

rcm_status rcm_order_ex(int32_t n, const int32_t* rowptr, const int32_t* colidx,
                        int32_t* perm_out, int32_t* iperm_out, rcm_stats* stats,
                        const rcm_options* opts, void* workspace, size_t workspace_bytes,
                        void* stream) {
  return order_single(n, rowptr, colidx, perm_out, iperm_out, stats, opts, workspace,
                      workspace_bytes, stream, true);
}

rcm_status rcm_order(int32_t n, const int32_t* rowptr, const int32_t* colidx, int32_t* perm_out,
                     rcm_stats* stats, void* stream) {
  return rcm_order_ex(n, rowptr, colidx, perm_out, nullptr, stats, nullptr, nullptr, 0, stream);
}

rcm_status rcm_order_batched(int32_t num_graphs, const int64_t* vtx_offsets,
                             const int64_t* nnz_offsets, const int32_t* rowptr_cat,
                             const int32_t* colidx_cat, int32_t* perm_cat, rcm_stats* stats,
                             const rcm_options* opts, void* workspace, size_t workspace_bytes,
                             void* stream) {
  if (num_graphs < 0) return RCM_ERR_INVALID_ARGUMENT;
  if (num_graphs == 0) return RCM_OK;
  if (!vtx_offsets || !nnz_offsets) return RCM_ERR_INVALID_ARGUMENT;
  Opts o;
  if (!parse_options(opts, &o, true)) return RCM_ERR_INVALID_ARGUMENT;
  std::memset(g_used, 0, sizeof(g_used));
  g_used[0] = 1;
  if (vtx_offsets[0] != 0 || nnz_offsets[0] != 0) return RCM_ERR_INVALID_ARGUMENT;
  for (int g = 0; g < num_graphs; ++g)
    if (vtx_offsets[g + 1] < vtx_offsets[g] || nnz_offsets[g + 1] < nnz_offsets[g])
      return RCM_ERR_INVALID_ARGUMENT;
  const int64_t N64 = vtx_offsets[num_graphs];
  const int64_t NNZ64 = nnz_offsets[num_graphs];
  if (N64 >= (1ll << 31) - 1 || NNZ64 >= (1ll << 31) - 1) return RCM_ERR_INVALID_ARGUMENT;
  if (const char* tf = tuning_path(opts)) {
    rcm_options eff{};
    if (opts) eff = *opts;
    if (!tuning_apply(tf, N64, NNZ64, num_graphs > 1 ? num_graphs : 2, &eff))
      return RCM_ERR_INVALID_ARGUMENT;
    if (!parse_options(&eff, &o, true)) return RCM_ERR_INVALID_ARGUMENT;
  }
  if (stats) std::memset(stats, 0, sizeof(rcm_stats) * num_graphs);
  if (N64 == 0) return RCM_OK;
  if (!rowptr_cat || !perm_cat || (NNZ64 > 0 && !colidx_cat)) return RCM_ERR_INVALID_ARGUMENT;
  const int32_t N = static_cast<int32_t>(N64), NNZ = static_cast<int32_t>(NNZ64);
  hipStream_t s = static_cast<hipStream_t>(stream);
  const Layout L = make_layout(N, NNZ, num_graphs, true, kSmallTeams);
  char* ws = static_cast<char*>(workspace);
  bool owned = false;
  if (ws) {
    if (workspace_bytes < L.total) return RCM_ERR_WORKSPACE_TOO_SMALL;
  } else {
    if (hipMallocAsync(reinterpret_cast<void**>(&ws), L.total, s) != hipSuccess)
      return RCM_ERR_OUT_OF_MEMORY;
    owned = true;
  }
  std::vector<int32_t> vo(num_graphs + 1), no(num_graphs + 1);
  for (int g = 0; g <= num_graphs; ++g) {
    vo[g] = static_cast<int32_t>(vtx_offsets[g]);
    no[g] = static_cast<int32_t>(nnz_offsets[g]);
  }
  rcm_status st = RCM_OK;
  Timer timer(s, true);
  do {
    int32_t* rowptr_g = reinterpret_cast<int32_t*>(ws + L.rowptr_g);
    int32_t* colidx_g = reinterpret_cast<int32_t*>(ws + L.colidx_g);
    // the graph offsets live in the seg_off / comp_seg_off regions for the
    // duration of the globalisation (run() rewrites seg_off itself)
    int32_t* d_vo = reinterpret_cast<int32_t*>(ws + L.seg_off);
    int32_t* d_no = reinterpret_cast<int32_t*>(ws + L.comp_seg_off);
    int32_t* err = reinterpret_cast<int32_t*>(ws + L.misc);
    if (hipMemcpyAsync(d_vo, vo.data(), 4 * vo.size(), hipMemcpyHostToDevice, s) != hipSuccess ||
        hipMemcpyAsync(d_no, no.data(), 4 * no.size(), hipMemcpyHostToDevice, s) != hipSuccess ||
        hipMemsetAsync(err, 0, 4, s) != hipSuccess) {
      st = RCM_ERR_HIP;
      break;
    }
    const int64_t tiles = (static_cast<int64_t>(N) + kGlobTile - 1) / kGlobTile +
                          (static_cast<int64_t>(NNZ) + kGlobTile - 1) / kGlobTile;
    const int blocks = static_cast<int>(std::max<int64_t>(1, std::min<int64_t>(tiles, 8192)));
    k_globalize<<<blocks, kGlobThreads, 0, s>>>(num_graphs, d_vo, d_no, rowptr_cat, colidx_cat, N,
                                                NNZ, rowptr_g, colidx_g, err);
    int32_t herr = 0;
    if (hipGetLastError() != hipSuccess || read_ints(&herr, err, 1, s) != RCM_OK) {
      st = RCM_ERR_HIP;
      break;
    }
    if (herr) {
      st = RCM_ERR_BAD_CSR;
      break;
    }
    Graph g{N, NNZ, rowptr_g, colidx_g, num_graphs, nullptr};
    st = run(g, vo.data(), o, ws, L, perm_cat, nullptr, stats, s, timer);
    if (st != RCM_OK) break;
    // perm_cat holds union-wide ids; each graph's block lies in its own
    // vertex range, so subtracting the graph's offset gives local ids
    // (run() left the graph offsets in its segment table)
    const int32_t* seg = reinterpret_cast<const int32_t*>(ws + L.seg_off);
    k_localize<<<std::min((N + 255) / 256, 8192), 256, 0, s>>>(N, seg, num_graphs, perm_cat);
    if (hipGetLastError() != hipSuccess || hipStreamSynchronize(s) != hipSuccess) st = RCM_ERR_HIP;
  } while (false);
  if (owned) {
    (void)hipFreeAsync(ws, s);
    (void)hipStreamSynchronize(s);
  }
  timer.finish();
  return st;
}

}  // extern "C"
