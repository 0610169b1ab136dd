// Internal declarations shared by the library's translation units: device
// helpers, the workspace layout, control blocks and kernel launchers.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "rcm.h"

namespace rcm {

constexpr uint32_t kUnclaimed = 0xFFFFFFFFu;
constexpr uint64_t kMaxKey = ~0ull;
constexpr int kMaxTeam = 256;            // work-groups per team
static_assert(kMaxTeam % 64 == 0, "barrier slots are polled by the 64 lanes of one wave");
constexpr int kMaxConcurrentTeams = 64;  // large-component teams per launch
// A device-side wait gives up (and flags RCM_ERR_ABORTED) after 30 s of the
// 100 MHz constant-rate clock read by wall_clock64(): far beyond any
// legitimate wait, short enough to end a broken run cleanly.
constexpr long long kWaitLimitTicks = 30ll * 100000000ll;

// ---------------------------------------------------------------------------
// Per-component task and result.
// ---------------------------------------------------------------------------
struct CompTask {
  int32_t seed;    // lowest vertex id of the component = start vertex
  int32_t size;    // number of vertices; -1 = unknown, found by the first BFS
  int32_t offset;  // first position of the component's label block
  int32_t index;   // component index (ascending seed order)
  int32_t anchor;  // Cuthill-McKee label t of the component lands at position
                   // anchor - t; -1 = offset + size - 1 (size found by the BFS)
};

struct CompResult {
  int32_t root;    // pseudo-peripheral root used for the labelled BFS
  int32_t nbfs;    // level structures computed by the search
  int32_t levels;  // levels of the labelled BFS
  int32_t seg;     // graph (segment) the component belongs to
  int32_t size;    // number of vertices
  int32_t pad;
  int64_t m;       // sum of degrees over the component
};

// Control block of one team (zeroed before each launch).  Fields written by
// different agents sit on separate 128-byte lines.
struct alignas(128) TeamCtl {
  int32_t tail[6];               // append counters, [pass parity][level mod 3]
  int32_t pad1[26];
  unsigned long long minkey[6];  // min (deg << 32 | id) per level, same indexing
  unsigned long long pad2[10];
  unsigned long long wake;       // narrow-mode release generation
  unsigned long long pad3[15];
  int32_t narrow_state[8];       // frontier bounds handed back after narrow levels
  int32_t pad4[24];
  long long msum;                // sum of degrees of the current component
  long long pass_m[2];           // level orders: sum of degrees reached by the
                                 // current unlabelled pass, [pass parity]
  unsigned long long ldone;      // labelled passes finished by the labelling sub-team
  int32_t llevels;               // levels of the last labelled pass
  int32_t a_ecc[2];              // asynchronous passes, [pass parity]: largest
  int32_t a_cnt[2];              // distance, vertices reached, and the minimum
  unsigned long long a_key[2];   // (deg << 32 | id) at the largest distance
  unsigned long long lastkey;    // min (deg << 32 | id) over the last level of a
                                 // labelled pass that also serves the search
  int32_t task;                  // large-component task handed to the team
  long long clk[32];             // work-group 0's clock (diagnostics): [0] pp ticks,
                                 // [1] labelled ticks, [2] pp levels, [3] labelled
                                 // levels, [4..31] per-phase ticks and counts

};

// Barrier slots of one team (zeroed before each launch): work-group w
// arrives at barrier number q by storing (q << 32 | payload) into
// s[q & 1][w][0]; each slot has a 128-byte line of its own.  Two sets, so a
// work-group that has passed barrier q can arrive at q + 1 while others
// still read q's payloads.
struct alignas(128) TeamSlots {
  unsigned long long s[2][kMaxTeam][16];
};

// Global control shared by all teams of one launch.
struct alignas(128) GlobalCtl {
  int32_t queue;                 // next task for single-WG teams
  int32_t error;                 // first error of the launch (rcm_status)
  int32_t diag[8];               // where it was detected: site, component index,
                                 // pass (0 = labelled), level, cur_b, cur_e, end
  // a launch that stopped after the first level structure of vertex 0's
  // component so that the library can renumber the graph (BfsParams::
  // relabel_levels): the structure's eccentricity, its pass tag, and the
  // minimum (degree, id) key of its last level
  int32_t p1_stop;
  int32_t p1_ecc;
  uint32_t p1_tag;
  int32_t p1_size;
  unsigned long long p1_lastkey;
  int32_t pad[14];
};
static_assert(sizeof(GlobalCtl) == 128, "one line");

// Per-segment (per-graph) accumulators filled by the device.
struct SegStats {
  unsigned long long bw_before;
  unsigned long long prof_before;
  unsigned long long bw_after;
  unsigned long long prof_after;
  unsigned long long edges;
  int32_t ncomp;
  int32_t diameter;
  int32_t nbfs;
  int32_t nlevels;
};

// ---------------------------------------------------------------------------
// Device helpers.
// ---------------------------------------------------------------------------

// 32-bit mixing function (the finaliser of MurmurHash3).
__host__ __device__ __forceinline__ uint32_t mix32(uint32_t x) {
  x ^= x >> 16;
  x *= 0x85ebca6bu;
  x ^= x >> 13;
  x *= 0xc2b2ae35u;
  x ^= x >> 16;
  return x;
}

// A seeded bijection of [0, count) (seed 0: the identity): an affine map
// x -> a x + c with a odd is a bijection modulo the next power of two P >=
// count; applying it until the value falls below count (cycle walking)
// restricts it to a bijection of [0, count), in at most P - count + 1 steps.
__host__ __device__ __forceinline__ int32_t shuffle_index(int32_t i, int32_t count,
                                                          uint32_t seed) {
  if (seed == 0 || count <= 1 || i < 0 || i >= count) return i;
  uint32_t mask = 1;
  while (mask < static_cast<uint32_t>(count)) mask <<= 1;
  mask -= 1;
  const uint32_t a = mix32(seed) | 1u;
  const uint32_t c = mix32(seed ^ 0x9e3779b9u);
  uint32_t x = static_cast<uint32_t>(i);
  do {
    x = (a * x + c) & mask;
  } while (x >= static_cast<uint32_t>(count));
  return static_cast<int32_t>(x);
}

// The caller's abort flag, read at system scope so that the load reaches
// the host's copy (one PCIe round trip; callers poll it sparingly).
__device__ __forceinline__ bool abort_requested(const int32_t* flag) {
  return flag != nullptr &&
         __hip_atomic_load(flag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM) != 0;
}

// Shuffle mode's perturbation: a seeded wait of 0 to 7 times ~0.4 us
// (s_sleep 16 = 1024 clocks), the same for every thread of a work-group.
__device__ __forceinline__ void shuffle_delay(uint32_t seed, uint32_t a, uint32_t b) {
  if (seed == 0) return;
  const uint32_t k = mix32(seed ^ mix32(a * 0x9e3779b9u ^ b)) & 7u;
  for (uint32_t i = 0; i < k; ++i) __builtin_amdgcn_s_sleep(16);
}
__device__ __forceinline__ int32_t ld_relaxed(const int32_t* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ uint32_t ld_relaxed(const uint32_t* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ unsigned long long ld_relaxed(const unsigned long long* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_relaxed(int32_t* p, int32_t v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ uint64_t pack_key(int32_t deg, int32_t v) {
  return (static_cast<uint64_t>(static_cast<uint32_t>(deg)) << 32) | static_cast<uint32_t>(v);
}

// Wave (64-lane) reductions.
__device__ __forceinline__ uint64_t wave_min_u64(uint64_t x) {
  for (int o = 32; o > 0; o >>= 1) {
    uint64_t y = __shfl_xor(x, o, 64);
    x = y < x ? y : x;
  }
  return x;
}
__device__ __forceinline__ long long wave_sum_i64(long long x) {
  for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o, 64);
  return x;
}
__device__ __forceinline__ long long wave_max_i64(long long x) {
  for (int o = 32; o > 0; o >>= 1) {
    long long y = __shfl_xor(x, o, 64);
    x = y > x ? y : x;
  }
  return x;
}
__device__ __forceinline__ int wave_sum_i32(int x) {
  for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o, 64);
  return x;
}

// Inclusive prefix sum within a wave.
__device__ __forceinline__ int wave_incl_scan(int x) {
  const int lane = threadIdx.x & 63;
  for (int o = 1; o < 64; o <<= 1) {
    int y = __shfl_up(x, o, 64);
    if (lane >= o) x += y;
  }
  return x;
}

// Exclusive block scan of one int per thread; returns the exclusive prefix and
// the block total through *total.  scratch: >= 17 ints of LDS.  All threads
// of the block must call it.
__device__ __forceinline__ int block_excl_scan(int x, int* scratch, int* total) {
  const int lane = threadIdx.x & 63;
  const int wid = threadIdx.x >> 6;
  const int nw = (blockDim.x + 63) >> 6;
  int incl = wave_incl_scan(x);
  if (lane == 63) scratch[wid] = incl;
  __syncthreads();
  if (threadIdx.x == 0) {
    int run = 0;
    for (int w = 0; w < nw; ++w) {
      int t = scratch[w];
      scratch[w] = run;
      run += t;
    }
    scratch[16] = run;
  }
  __syncthreads();
  int res = scratch[wid] + incl - x;
  *total = scratch[16];
  __syncthreads();
  return res;
}

// Block reductions (result valid in every thread).  scratch: >= 16 entries.
__device__ __forceinline__ long long block_sum_i64(long long x, long long* scratch) {
  const int lane = threadIdx.x & 63;
  const int wid = threadIdx.x >> 6;
  const int nw = (blockDim.x + 63) >> 6;
  x = wave_sum_i64(x);
  if (lane == 0) scratch[wid] = x;
  __syncthreads();
  long long s = 0;
  for (int w = 0; w < nw; ++w) s += scratch[w];
  __syncthreads();
  return s;
}
__device__ __forceinline__ long long block_max_i64(long long x, long long* scratch) {
  const int lane = threadIdx.x & 63;
  const int wid = threadIdx.x >> 6;
  const int nw = (blockDim.x + 63) >> 6;
  x = wave_max_i64(x);
  if (lane == 0) scratch[wid] = x;
  __syncthreads();
  long long s = scratch[0];
  for (int w = 1; w < nw; ++w) s = scratch[w] > s ? scratch[w] : s;
  __syncthreads();
  return s;
}

// Segment (graph) of a vertex: largest g with seg_off[g] <= v.  nseg >= 1.
__device__ __forceinline__ int find_segment(const int32_t* seg_off, int nseg, int32_t v) {
  int lo = 0, hi = nseg - 1;
  while (lo < hi) {
    int mid = (lo + hi + 1) >> 1;
    if (seg_off[mid] <= v) lo = mid; else hi = mid - 1;
  }
  return lo;
}

// ---------------------------------------------------------------------------
// Host-side launchers (defined in the .hip files).
// ---------------------------------------------------------------------------
struct Graph {
  int32_t n;
  int32_t nnz;
  const int32_t* rowptr;  // device, global (segment offsets already applied)
  const int32_t* colidx;
  int32_t nseg;
  const int32_t* seg_off; // device int32[nseg+1] vertex offsets of segments
};

// err: malformed rows (bounds, columns out of range, repeated columns in
// rows of up to 64 entries); long_rows: set when a row is longer, whose
// repeated columns launch_dup_long then checks (into err).
// ell (may be null): the rows' copy of BfsParams::ell, written for every row
// of at most kEllWidth entries; *wide_rows is raised by any longer row.
hipError_t launch_validate_scan(const Graph& g, int4* vinfo, int32_t* beta, SegStats* seg,
                                int32_t* err, int32_t* long_rows, int4* ell,
                                int32_t* wide_rows, hipStream_t s);
hipError_t launch_dup_long(const Graph& g, int32_t* err, hipStream_t s);
hipError_t launch_full_check(const Graph& g, int32_t* err_dup, int32_t* err_sym, hipStream_t s);
// Components of the vertices with skip[v] == 0 (skip may be null: all).
hipError_t launch_components(const Graph& g, const int32_t* skip, int32_t* parent, int32_t* csize,
                             int32_t* flags, int32_t* scan_tmp, int32_t* seeds,
                             int32_t* num_comps, int32_t* err_asym, hipStream_t s);
// Tasks for ncomp components whose seeds are seeds[0..ncomp); their label
// blocks start at offset_base and their indices at index_base.  counts[0..2]
// receive the numbers of isolated / small / large tasks, counts[3] the
// total number of vertices covered.
hipError_t launch_tasks(const Graph& g, int32_t ncomp, const int32_t* seeds, const int32_t* csize,
                        int32_t small_cutoff, int32_t reverse_mode, int32_t offset_base,
                        int32_t index_base, CompTask* tasks_single, CompTask* tasks_small,
                        CompTask* tasks_big, int32_t* counts, int32_t* sizes, int32_t* offs,
                        int32_t* scan_blk, CompResult* results, int32_t* sched,
                        hipStream_t s);
// key (nullable): the level orders' key of an isolated vertex, its position
hipError_t launch_singletons(const CompTask* tasks, int32_t count, int32_t* perm, int32_t* iperm,
                             int32_t* key, CompResult* results, hipStream_t s);
hipError_t launch_bw_after(const Graph& g, const int32_t* perm, const int32_t* iperm,
                           int32_t* beta, SegStats* seg, hipStream_t s);
hipError_t launch_comp_stats(const Graph& g, int32_t ncomp, const int32_t* seeds,
                             const CompResult* results, int32_t* comp_seg_off, SegStats* seg,
                             int32_t labelled_bfs, hipStream_t s);

// Level orders (label_mode 1 and 2): the ordering kernel leaves in key[v]
// anchor - level, anchor being the final position of the component's
// Cuthill-McKee label 0 and level the vertex's level in the root's level
// structure (an isolated vertex: its position).  perm[k] = the vertices
// sorted by key ascending, then by degree (when by_degree) and id
// descending -- the reversed order -- and iperm its inverse.
// scratch: 16 n bytes (four int32 arrays of n); temp:
// level_order_temp_bytes(n).
size_t level_order_temp_bytes(int32_t n);
hipError_t launch_level_order(int32_t n, int32_t max_degree_bits, bool by_degree,
                              const int4* vinfo, const int32_t* key, int32_t* perm,
                              int32_t* iperm, void* scratch, void* temp, size_t temp_bytes,
                              hipStream_t s);
hipError_t launch_exclusive_scan(const int32_t* in, int32_t* out, int32_t count, int32_t* tmp,
                                 int32_t* total_out, hipStream_t s);

// Locality renumbering (rcm_relabel.hip) of the component whose `size`
// vertices carry the pass tag `tag` and their distance in dkey (an
// asynchronous level structure with eccentricity ecc): its vertices are
// renumbered 0 .. size - 1 level by level (in any order within a level),
// and the component is rebuilt in the new numbering -- rowptr_new
// (size + 1), colidx_new (its entries), vinfo_new (row begin, row end,
// degree, caller id) -- with new_of_old (for its vertices; 0 for the
// others) and old_of_new the two maps; colidx_new holds cap entries.  Scratch: hist and first (ecc + 1
// int32 each), scan_tmp (n / 4096 + 2 int32); cursor holds n int32.  err is
// set for a distance outside [0, ecc]; *counted receives the number of
// tagged vertices (which must equal size).
hipError_t launch_relabel(const Graph& g, const int4* vinfo, const unsigned long long* dkey,
                          uint32_t tag, int32_t ecc, int32_t size, int32_t* hist, int32_t* first,
                          int32_t* cursor, int32_t* scan_tmp, int32_t* new_of_old,
                          int32_t* old_of_new, int32_t* rowptr_new, int32_t* colidx_new,
                          int64_t cap, int4* vinfo_new, int32_t* err, int32_t* counted,
                          hipStream_t s);

struct BfsParams {
  const int32_t* rowptr;
  const int32_t* colidx;
  const int4* vinfo;  // per vertex: row begin, row end, degree, the vertex's id in
                      // the caller's graph (its own number unless relabelled)
  int32_t* visit;
  uint32_t* claim;
  int4* qi;           // per position: vertex, row begin, row end, degree
  int32_t* tmp;
  int32_t* perm;
  int32_t* iperm;
  const CompTask* big_tasks;  // components for multi-work-group teams, largest first
  int32_t n_big;
  int32_t big_blocks;         // blocks [0, big_blocks) form teams of team_size
  const CompTask* tasks;      // components for single-work-group teams, largest first
  int32_t ntasks;
  CompResult* results;
  TeamCtl* teams;             // one per multi-work-group team
  TeamSlots* slots;           // one per multi-work-group team
  TeamCtl* small_teams;       // one per block in single-work-group mode
  int32_t* queues;            // [0] next large task, [1] next small task (zeroed per launch)
  GlobalCtl* gctl;
  int32_t n;
  int32_t nnz;
  int32_t team_size;
  int32_t pp_variant;
  int32_t reverse_mode;
  int32_t narrow_cutoff;
  int32_t rebalance;          // wide unlabelled levels between redistributions
  int32_t label_mode;         // 0: labelled BFS; 1, 2: level order (keys left in claim)
  int32_t async_search;       // 1: large components' searches run asynchronous passes
  TeamSlots* sub_slots;       // barrier slots of the labelling sub-teams
  int32_t label_team;         // work-groups of a team that run the labelled BFS
  int32_t search_round;       // steps per round of the asynchronous passes
  const int32_t* seg_off;     // vertex offsets of the graphs (segments), nseg + 1
  int32_t nseg;
  unsigned long long* dkey;   // per vertex: pass tag << 32 | ~distance (asynchronous passes)
  const int32_t* abort_flag;  // the caller's abort flag (coherent host memory), or null
  uint32_t shuffle;           // 0, or the seed of the work-group / task shuffle
  // Locality renumbering of long components (single graphs): with
  // relabel_levels > 0, the task of vertex 0's component stops after its
  // first level structure when that has at least relabel_levels levels and
  // was asynchronous, leaving its results in GlobalCtl (p1_*).  resume = 1 continues that task from there, and a
  // relabelled launch runs on the graph renumbered in the structure's order:
  // new_of_old maps a caller id to its number, vinfo.w back; every
  // (degree, id) key and every output uses the caller's ids.
  int32_t relabel_levels;
  int32_t resume;
  int32_t relabelled;
  const int32_t* new_of_old;  // null unless relabelled
  // Null, or a copy of the rows of a graph whose rows all have at most
  // kEllWidth entries: row v is ell[2v], ell[2v + 1], its entries in order
  // and then v itself.  A neighbour's row is then at an address known from
  // its number alone, so the asynchronous passes load it in the same round
  // trip as the atomic on the neighbour's distance word.
  const int4* ell;
};
constexpr int kEllWidth = 8;

// The one-work-group engine for a whole small graph in LDS (rcm_small.hip).
struct SmallResult {
  int32_t status;  // rcm_status, or kSmallDeclined
  int32_t ncomp, diameter, nbfs, nlevels;
  int32_t nnz;     // the entry count the kernel read (-1 before it did)
  int32_t pad[2];
  unsigned long long bw_before, prof_before, bw_after, prof_after, edges;
  long long ticks[6];  // 100 MHz clock: load, row checks, searches, labelled
                       // BFS, reversal, result statistics (diagnostics)
};
constexpr int32_t kSmallDeclined = -1;  // the graph does not fit the LDS given
struct SmallJob {
  int32_t n;
  int32_t nnz;              // < 0: read rowptr[n] on the device
  const int32_t* rowptr;    // device, rowptr[0] = 0
  const int32_t* colidx;
  int32_t* perm;            // perm[k] = vertex + id_off
  int32_t* iperm;           // nullable: iperm[vertex] = k + pos_off
  int32_t id_off;
  int32_t pos_off;
  SmallResult* res;         // device
};
struct SmallOpts {
  int32_t pp_variant;
  int32_t reverse_mode;
  int32_t check_full;
  int32_t lds_bytes;        // dynamic LDS of each work-group
  uint32_t shuffle;         // 0, or the seed of the work-group -> job shuffle
  const int32_t* abort_flag;  // the caller's abort flag (coherent host memory), or null
};
// LDS bytes the engine needs for a graph (0 for n <= 0), and the most one
// work-group may have on the current device (0 if unknown).
size_t small_lds_bytes(int64_t n, int64_t nnz);
size_t small_lds_limit();
// jobs_dev == nullptr: one job, `single`.
hipError_t launch_small_order(const SmallJob& single, const SmallJob* jobs_dev, int32_t njobs,
                              const SmallOpts& opts, hipStream_t s);
// The window engine (rcm_window.hip): the remaining passes of a long
// component after its renumbering, by one work-group.  ids are the
// renumbered ones (0 .. size - 1).
constexpr int32_t kWindowDeclined = 1;  // *status when the team kernel must take over
struct WinParams {
  int32_t n;                      // vertices of the caller's graph
  int32_t size;                   // vertices of the renumbered component
  const int32_t* colidx;          // renumbered rows (entries of vinfo[x].x .. .y)
  const int4* vinfo;              // (row begin, row end, degree, caller id)
  const int32_t* new_of_old;      // caller id -> renumbered id
  uint2* ell;                     // [size] row records the launch builds (workspace)
  int32_t* ell_flag;              // set when a row does not fit its record
  uint32_t* claim;                // [size] claim words (workspace), the window's store
  int32_t* order;                 // [size] the labelled order (workspace)
  int32_t ecc1;                   // the first level structure: eccentricity ...
  unsigned long long lastkey1;    // ... and its last level's minimum (degree, caller id)
  int32_t pp_variant;
  int32_t anchor;                 // Cuthill-McKee label t goes to position anchor - t
  int32_t* perm;                  // caller-id space
  int32_t* iperm;                 // nullable
  CompResult* result;             // the component's result record
  int32_t* status;                // 0, kWindowDeclined, RCM_ERR_NOT_SYMMETRIC or RCM_ERR_ABORTED
  const int32_t* abort_flag;      // device view of the caller's abort flag, or null
};
hipError_t launch_window_order(const WinParams& P, hipStream_t s);

// The bounded-row variant (rcm_small_ell.hip) for one graph: LDS bytes it
// needs (0 for n <= 0, SIZE_MAX past its 16-bit ids) and its launch; it
// declines graphs with a row of more than 8 off-diagonal entries.
size_t small_ell_lds_bytes(int64_t n);
hipError_t launch_small_ell(const SmallJob& job, const SmallOpts& opts, hipStream_t s);

// Tuning tables (rcm_tuning.hip): the file named by opts->tuning_file, else
// by RCM_TUNING_FILE, else none (nullptr).  tuning_apply sets every launch
// option of *opts still at 0 from the table's entry for the call's size
// class; false when the table cannot be read or is malformed.
const char* tuning_path(const rcm_options* opts);
bool tuning_apply(const char* path, int64_t n, int64_t nnz, int32_t graphs, rcm_options* opts);

// rcm_order_ex without its extern "C" wrapper; timing = false never creates
// HIP events (the allocation-free entry point).
rcm_status order_single(int32_t n, const int32_t* rowptr, const int32_t* colidx,
                        int32_t* perm_out, int32_t* iperm_out, rcm_stats* stats,
                        const rcm_options* opts, void* workspace, size_t workspace_bytes,
                        void* stream, bool timing);
// The checks order_single makes before any HIP call: n >= 0, valid options
// (RCM_ERR_INVALID_ARGUMENT otherwise).
rcm_status check_call(int32_t n, const rcm_options* opts);

// One launch of the ordering kernel over the task lists in p; cooperative
// (all blocks co-resident) whenever p has multi-work-group teams.
hipError_t launch_order(const BfsParams& p, int32_t blocks, int32_t threads, hipStream_t s);
int max_team_blocks(int32_t threads);

}  // namespace rcm
