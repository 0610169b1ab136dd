// The ordering itself: for each connected component, the pseudo-peripheral
// search (Algorithm 2: repeated breadth-first searches, each returning its
// eccentricity and the minimum-(degree, id) vertex of its last level) and
// the labelled level-synchronous BFS of Algorithm 3, then the reversal.
//
// One persistent kernel does all of it.  A "team" of W work-groups owns one
// component at a time.  Its work-groups meet at team barriers: every
// work-group stores (barrier number, payload) into a slot of its own and
// polls the others' slots, so a barrier also exchanges one count per
// work-group (for W = 1 it is just __syncthreads).  In one launch:
//   - large components: teams of W co-resident work-groups (cooperative
//     launch; by default one work-group per CU for a large graph) take them
//     from a queue, largest first;
//   - small components: single-work-group teams take them from a second
//     queue, largest first; team work-groups join them once the large
//     queue is empty.
// The search's level structures of a large component are asynchronous: a
// label-correcting BFS with one team barrier per round of steps instead of
// one per level (async_bfs_pass).  The labelled BFS is level-synchronous and
// runs on the team's first label_team work-groups.  Narrow levels (fewer
// vertices than the narrow cutoff) of the level-synchronous passes are
// expanded by the team's first work-group alone, level after level with only
// __syncthreads, while the others sleep until the frontier widens again or
// the pass ends.
//
// Frontier entries are (vertex, row begin, row end): the row bounds of a
// vertex are fetched when it is discovered, in the shadow of the append, so
// expanding the next level starts with one coalesced read.  Rows are read in
// register batches of kRB entries so that all loads of a batch (columns,
// then visited/claim words, then atomics) are in flight together.
//
// Level step of the labelled BFS (Algorithm 3), for the frontier
// L_cur = q[cur_b, cur_e) whose labels are exactly the positions p:
//   A. SpMSpV over (select2nd, min): for every edge (u, v) with u = q[p] and
//      v unlabelled, claim[v] = min(claim[v], p) (an atomic min; claim[] of
//      already labelled vertices holds labels < cur_b <= p, so the min leaves
//      them alone -- this is the Select(R == -1) step).
//   B. The children of p are the neighbours v != u with claim[v] == p.  Each
//      parent counts them.
//   C. An exclusive scan of the counts over the level (in label order) gives
//      each parent's first child label; a child's rank among its siblings is
//      its rank by (degree, id).  Parent label first, then degree, then id:
//      exactly SortPerm's lexicographic (parent label, degree, id) order
//      (Table I), without sorting the whole level.
// Unlabelled BFS (Algorithm 2's level structures): vertices are stamped with
// the pass number (no reset between passes) and appended to the next level
// through an LDS stage and one global atomic per work-group.

#include <mutex>

#include "rcm_common.hpp"

namespace rcm {

namespace {

constexpr int kStageCap = 2048;
constexpr int kRB = 8;  // row batch: entries of a row loaded together

struct Team {
  TeamCtl* ctl;
  TeamSlots* slots;
  GlobalCtl* g;
  int W;
  int wid;
  int comp;                 // index of the component being ordered (diagnostics)
  uint32_t seq;             // team barriers passed (every thread, in step)
  TeamSlots* sub_slots;     // the labelling sub-team's barrier slots
  uint32_t sub_seq;         // barriers the labelling sub-team has passed
  unsigned long long ldone; // labelled passes seen finished
  int32_t anchor;           // level orders: final position of the component's
                            // Cuthill-McKee label 0
  long long pm;             // level orders: degrees of the vertices this thread
                            // reached in the current pass
  unsigned long long woke;  // narrow episodes seen (thread 0 only)
  const int32_t* abort_flag;  // the caller's abort flag, or null
  uint32_t shuffle;         // 0, or the seed of the shuffle mode
  uint32_t polls;           // single-work-group barriers passed (abort polling)
  bool aborted;
};

// LDS state of the single-work-group level engine (narrow levels).
constexpr int kNarrowCap = 1024;        // frontier records held in LDS
constexpr int kHashBits = 11;
constexpr int kHash = 1 << kHashBits;   // slots per next-level table
constexpr int32_t kEmpty = -1;

struct NarrowLds {
  int32_t lev[2][kNarrowCap][4];   // frontier records (vertex, row begin, row end, degree)
  int32_t key[2][kHash];           // next-level tables: vertex ...
  uint32_t val[2][kHash];          // ... and its smallest claiming label
  int32_t cnt[3];                  // size of the level being discovered (mod 3)
  int32_t rows[3];                 // its total row length (mod 3)
  int32_t maxrow[3];               // its longest row (mod 3)
  unsigned long long kmin[3];      // its minimum (degree << 32 | id) (mod 3)
};

constexpr int kOwnCap = 2048;  // own-frontier records per work-group and buffer

union SharedBuf {
  int32_t srec[kStageCap][4];      // append stage of the team levels
  int32_t own[2][kOwnCap][4];      // own frontier, current and next level
  NarrowLds nw;
};

// Labelled levels keep, behind a work-group's child list in srec, the rows
// (one register batch) its first kRowCap children loaded for their claims;
// at the next level those children are the work-group's parents and count
// their own children from there instead of reloading the rows.
constexpr int kRowCap = 1024;
static_assert(sizeof(SharedBuf) >= sizeof(int32_t) * (4 * kStageCap + kRB * kRowCap),
              "no room for the kept rows");
__device__ __forceinline__ int32_t* kept_row(SharedBuf& u, int32_t i) {
  return reinterpret_cast<int32_t*>(&u) + 4 * kStageCap + kRB * i;
}

// Asynchronous passes over a graph with a fixed-stride row copy: the rows of
// the first kORowCap records of each own-frontier buffer, loaded by whoever
// reached the vertex, alongside its atomic.
constexpr int kORowCap = 1024;

// Labelled levels: a parent on a row longer than a register batch ranks up
// to kLongKids children in registers itself; one with many more on a long
// row is placed by the whole work-group (kHeavyCap: such parents per chunk
// of the level, at most one per thread).
constexpr int kLongKids = 4;
constexpr int kHeavyCap = 512;
// A parent's own ranking of c > kLongKids children scans its row once per
// child: c * (row batches) dependent round trips.  Past this many, the
// work-group places them instead (one parent at a time, so not for the
// many parents of moderate rows that rank well in parallel).
constexpr int64_t kHeavyWork = 512;
// Asynchronous passes on the CSR: a record whose row is longer than this is
// expanded by its whole work-group, a batch per thread, instead of by one
// thread batch after batch.
constexpr int32_t kHeavyRow = 2048;

typedef int4 OwnRowStore[2][kORowCap][2];

struct Shared {
  SharedBuf u;
  OwnRowStore orow;
  int scan[17];
  long long red[16];
  int32_t cnt;
  int32_t base;
  unsigned long long key;
  int flag;
  int task;
  int32_t spill;                   // own-frontier level: records went to qi
  int32_t total;                   // own-frontier level: next level size
  int32_t nspill;                  // own-frontier level: records in qi
  int32_t appended;                // asynchronous passes: records this work-group
                                   // put in the ring this round

  int32_t wsum[kMaxTeam];          // slot_exchange: every work-group's count
  int32_t wpre;                    // slot_exchange: this work-group's prefix
  int32_t wtot;                    // slot_exchange: the team's total
  int32_t wmax;                    // slot_exchange: the largest count
  int32_t wspill;                  // slot_exchange: work-groups that flagged a spill
  int32_t ovf;                     // asynchronous passes: a record found no ring slot
  int32_t lown_base;               // wide labelled level: the label range of the
  int32_t lown_len;                // children this work-group placed (its list
  int32_t lown_ok;                 // in srec), valid when it holds them all
  int4 heavy[kHeavyCap];           // labelled levels: parents whose many children on a
  int32_t nheavy;                  // long row the whole work-group places (label, first
  int32_t mcnt;                    // label, children); children found so far
  int32_t stop;                    // abort polls: the flag or an error was seen
  int32_t state[8];
};

// Record the first error of the launch (RCM_ERR_ABORTED for a wait that timed
// out, RCM_ERR_NOT_SYMMETRIC when a traversal leaves its component's block,
// which only an asymmetric pattern can cause).
__device__ __forceinline__ void flag_error(GlobalCtl* g, int code, int site = 0, int comp = 0,
                                           int pass = 0, int level = 0, int cur_b = 0,
                                           int cur_e = 0, int end = 0) {
  int32_t expected = 0;
  if (__hip_atomic_compare_exchange_strong(&g->error, &expected, static_cast<int32_t>(code),
                                           __ATOMIC_RELAXED, __ATOMIC_RELAXED,
                                           __HIP_MEMORY_SCOPE_AGENT)) {
    const int32_t d[7] = {site, comp, pass, level, cur_b, cur_e, end};
    for (int i = 0; i < 7; ++i) st_relaxed(&g->diag[i], d[i]);
  }
}

// Abort poll by every thread of a work-group: thread 0 reads the launch's
// error word and the caller's abort flag (flagging RCM_ERR_ABORTED for the
// latter); t.aborted when either is set.
__device__ __forceinline__ void poll_stop(Team& t, Shared& S) {
  __syncthreads();
  if (threadIdx.x == 0) {
    int32_t stop = ld_relaxed(&t.g->error) != 0 ? 1 : 0;
    if (!stop && abort_requested(t.abort_flag)) {
      flag_error(t.g, RCM_ERR_ABORTED, 21, t.comp);
      stop = 1;
    }
    S.stop = stop;
  }
  __syncthreads();
  t.aborted = S.stop != 0;
}

// Wait (thread 0) until *ctr >= target, giving up after the wall-clock limit
// or when another work-group has flagged an error.  Returns false on give-up.
__device__ __forceinline__ bool wait_at_least(Team& t, unsigned long long* ctr,
                                              unsigned long long target, bool sleepy) {
  long spins = 0;
  const long long t0 = wall_clock64();
  while (ld_relaxed(ctr) < target) {
    if (sleepy) __builtin_amdgcn_s_sleep(2);
    if ((++spins & 255) == 0) {
      if (ld_relaxed(&t.g->error) != 0) return false;
      if (wall_clock64() - t0 > kWaitLimitTicks) {
        flag_error(t.g, RCM_ERR_ABORTED);
        return false;
      }
    }
  }
  return true;
}

// Every wave of the work-group waits until its own memory operations (loads,
// stores, atomics, also fire-and-forget ones) have completed.
__device__ __forceinline__ void drain_memory_ops() {
  __atomic_signal_fence(__ATOMIC_SEQ_CST);
  __builtin_amdgcn_s_waitcnt(0);
  __atomic_signal_fence(__ATOMIC_SEQ_CST);
}

// Team barrier that also exchanges one 32-bit payload per work-group (bit 31
// a flag, bits 0..30 a count): every work-group stores (barrier number,
// payload) into its own slot, and the lanes of wave 0 wait for the W slots
// (lane l for work-groups l, l + 64, ...).  Afterwards S.wsum[w] holds work-group w's count,
// S.wpre the sum over work-groups before this one, S.wtot the total, S.wmax
// the largest, S.wspill the number of flags.  drain: every wave first
// completes its own memory operations (whatever another work-group reads
// after the barrier was written with atomics or device-scope stores, so no
// L2 write-back is needed).
//
// No acquire fence follows: every load of data that other work-groups write
// during the launch (records, claims, visited stamps, distance words,
// control words) is a device-scope load, which on this GPU is served
// coherently by the L2 and sees every store or atomic another work-group
// completed before arriving (a probe saw no stale value in 20,000
// cross-XCD hand-overs, where plain loads saw one every time, from the
// CU's L1).  An agent-scope acquire would invalidate the CU's caches: it
// costs 0.4 us alone and its cost grows with the number of CUs doing it at
// once (1.7 us more per barrier for 256 work-groups), and afterwards even
// read-only data (rows, vertex records) must come back from memory.  The
// compiler barrier keeps the loads after the wait.
//
// The barrier has two halves: slot_arrive stores this work-group's slot and
// slot_wait collects the others'.  Between them a work-group may do work
// that needs nothing from the other work-groups (using LDS but not the
// fields slot_wait fills); slot_exchange is the two back to back.
__device__ __forceinline__ void slot_arrive(Team& t, Shared& S, uint32_t payload, bool drain) {
  shuffle_delay(t.shuffle, static_cast<uint32_t>(t.wid), t.seq);
  if (drain) drain_memory_ops();
  __syncthreads();
  t.seq += 1;
  const uint32_t seq = t.seq;
  if (threadIdx.x == 0)
    __hip_atomic_store(&t.slots->s[seq & 1][t.wid][0],
                       (static_cast<unsigned long long>(seq) << 32) | payload, __ATOMIC_RELAXED,
                       __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ void slot_wait(Team& t, Shared& S) {
  const uint32_t seq = t.seq;
  if (threadIdx.x < 64) {
    const int lane = threadIdx.x;
    unsigned long long* base = &t.slots->s[seq & 1][0][0];
    // lane l waits for work-groups l, l + 64, ... (kMaxTeam / 64 at most),
    // polling all of them in each round trip
    constexpr int kPer = kMaxTeam / 64;
    unsigned long long v[kPer];
    bool ok = true;
    {
      unsigned pending = 0;
#pragma unroll
      for (int j = 0; j < kPer; ++j)
        if (lane + 64 * j < t.W) pending |= 1u << j;
      long spins = 0;
      const long long t0 = wall_clock64();
      while (pending != 0) {
#pragma unroll
        for (int j = 0; j < kPer; ++j) {
          if (!(pending >> j & 1u)) continue;
          v[j] = __hip_atomic_load(base + (lane + 64 * j) * 16, __ATOMIC_RELAXED,
                                   __HIP_MEMORY_SCOPE_AGENT);
          if (static_cast<uint32_t>(v[j] >> 32) == seq) pending &= ~(1u << j);
        }
        if (pending == 0) break;
        // long waits back off, so that waiting lanes leave memory to the work
        if (spins > 64) __builtin_amdgcn_s_sleep(1);
        if ((++spins & 255) == 0) {
          if (ld_relaxed(&t.g->error) != 0) { ok = false; break; }
          if (wall_clock64() - t0 > kWaitLimitTicks) {
            flag_error(t.g, RCM_ERR_ABORTED);
            ok = false;
            break;
          }
        }
      }
    }
    // every 64th barrier the team's first work-group polls the caller's
    // abort flag; the others stop when it no longer arrives (their waits
    // check the error word)
    if (lane == 0 && t.wid == 0 && (seq & 63) == 0 && abort_requested(t.abort_flag)) {
      flag_error(t.g, RCM_ERR_ABORTED, 20, t.comp);
      ok = false;
    }
    int32_t below = 0, all = 0, mx = 0, fl = 0;
#pragma unroll
    for (int j = 0; j < kPer; ++j) {
      const int w = lane + 64 * j;
      if (w >= t.W) continue;
      const uint32_t p = static_cast<uint32_t>(v[j]);
      const int32_t c = ok ? static_cast<int32_t>(p & 0x7FFFFFFFu) : 0;
      S.wsum[w] = c;
      below += w < t.wid ? c : 0;
      all += c;
      mx = c > mx ? c : mx;
      fl += ok ? static_cast<int32_t>(p >> 31) : 0;
    }
    const bool all_ok = __all(ok);
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
      below += __shfl_xor(below, o, 64);
      all += __shfl_xor(all, o, 64);
      const int32_t y = __shfl_xor(mx, o, 64);
      mx = y > mx ? y : mx;
      fl += __shfl_xor(fl, o, 64);
    }
    if (lane == 0) {
      S.wpre = below;
      S.wtot = all;
      S.wmax = mx;
      S.wspill = fl;
      S.flag = all_ok ? 0 : 1;
    }
  }
  __syncthreads();
  __atomic_signal_fence(__ATOMIC_SEQ_CST);
  t.aborted = S.flag != 0;
}

__device__ __forceinline__ void slot_exchange(Team& t, Shared& S, uint32_t payload, bool drain) {
  slot_arrive(t, S, payload, drain);
  slot_wait(t, S);
}

// The same counts for a work-group alone.
__device__ __forceinline__ void local_counts(Shared& S, int32_t c) {
  if (threadIdx.x == 0) {
    S.wsum[0] = c;
    S.wpre = 0;
    S.wtot = c;
    S.wmax = c;
    S.wspill = 0;
  }
  __syncthreads();
}

// Team barrier; `solo` = only this work-group is active (narrow mode or W=1).
__device__ __forceinline__ void team_barrier(Team& t, Shared& S, bool solo) {
  if (solo || t.W == 1) {
    // a work-group alone polls for an abort every 64th barrier
    if (t.abort_flag != nullptr && ((++t.polls) & 63u) == 0)
      poll_stop(t, S);
    else
      __syncthreads();
    return;
  }
  slot_exchange(t, S, 0u, true);
}

// Narrow mode hand-over.  Work-group 0 publishes the pass state and wakes
// the others; they read it back.
__device__ __forceinline__ void narrow_publish(Team& t, int32_t cur_b, int32_t cur_e,
                                               int32_t level, bool done) {
  // work-group 0 wrote the stretch's records and stamps with plain stores:
  // every wave completes them, then one release writes them back
  drain_memory_ops();
  __syncthreads();
  if (threadIdx.x == 0) {
    st_relaxed(&t.ctl->narrow_state[0], cur_b);
    st_relaxed(&t.ctl->narrow_state[1], cur_e);
    st_relaxed(&t.ctl->narrow_state[2], level);
    st_relaxed(&t.ctl->narrow_state[3], done ? 1 : 0);
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    __hip_atomic_fetch_add(&t.ctl->wake, 1ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
}

__device__ __forceinline__ void narrow_wait(Team& t, Shared& S) {
  __syncthreads();
  if (threadIdx.x == 0) {
    t.woke += 1;
    const bool ok = wait_at_least(t, &t.ctl->wake, t.woke, true);
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
#pragma unroll
    for (int i = 0; i < 4; ++i) S.state[i] = ld_relaxed(&t.ctl->narrow_state[i]);
    S.flag = ok ? 0 : 1;
  }
  __syncthreads();
  t.aborted = S.flag != 0;
}

// Split [b, e) into W contiguous chunks; chunk of work-group wid.
__device__ __forceinline__ void my_chunk(int32_t b, int32_t e, int W, int wid, int32_t& lo,
                                         int32_t& hi) {
  const int32_t len = e - b;
  const int32_t c = (len + W - 1) / W;
  lo = b + c * wid;
  hi = lo + c < e ? lo + c : e;
  if (lo > e) lo = e;
}

// Load entries [k0, k0 + kRB) of the row [k0, b) (b > k0) into registers with
// unconditional loads (indices clamped into the row), so that the whole batch
// is in flight at once.  Lanes past the row end get the row's own vertex u,
// which every caller treats as "not a neighbour".
__device__ __forceinline__ void load_batch(const int32_t* __restrict__ colidx, int32_t k0,
                                           int32_t b, int32_t u, int32_t* nb) {
#pragma unroll
  for (int j = 0; j < kRB; ++j) {
    const int32_t k = k0 + j < b ? k0 + j : b - 1;
    const int32_t c = colidx[k];
    nb[j] = k0 + j < b ? c : u;
  }
}

__device__ __forceinline__ int4 record(int32_t v, int4 info) {
  return make_int4(v, info.x, info.y, info.z);
}

// Store a frontier record that other work-groups read after a team barrier.
// The two halves are device-scope stores, which reach the point of
// coherence of all XCDs by themselves, so the team barrier needs no L2
// write-back (every wave waits for its stores before arriving).
__device__ __forceinline__ void st_rec(int4* p, int4 r) {
  unsigned long long* q = reinterpret_cast<unsigned long long*>(p);
  const unsigned long long lo =
      static_cast<uint32_t>(r.x) | (static_cast<unsigned long long>(static_cast<uint32_t>(r.y)) << 32);
  const unsigned long long hi =
      static_cast<uint32_t>(r.z) | (static_cast<unsigned long long>(static_cast<uint32_t>(r.w)) << 32);
  __hip_atomic_store(q, lo, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  __hip_atomic_store(q + 1, hi, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// A compiler-only barrier: loads before it are issued before it (their
// results are still waited for only where they are used).  No instruction.
__device__ __forceinline__ void issue_fence() { asm volatile("" ::: "memory"); }

// Row v of the fixed-stride copy (the entries, then v): what load_batch
// returns for a row of at most kRB entries, in two 16-byte loads whose
// address needs no row pointer.
static_assert(kEllWidth == kRB, "a copied row is one register batch");
__device__ __forceinline__ void ell_row(const int4* __restrict__ ell, int32_t v, int32_t* nb) {
  const int4 a = ell[2 * static_cast<size_t>(v)];
  const int4 b = ell[2 * static_cast<size_t>(v) + 1];
  nb[0] = a.x; nb[1] = a.y; nb[2] = a.z; nb[3] = a.w;
  nb[4] = b.x; nb[5] = b.y; nb[6] = b.z; nb[7] = b.w;
}

// A frontier record as read back, clamped into the graph (vertex in [0, n),
// 0 <= row begin <= row end <= nnz), so that no read can leave the arrays
// whatever a position held.  The halves are read with device-scope loads,
// which see another work-group's completed stores without a cache
// invalidation (see slot_exchange).
__device__ __forceinline__ int4 ld_rec(const BfsParams& P, int32_t pos) {
  const unsigned long long* q = reinterpret_cast<const unsigned long long*>(P.qi + pos);
  const unsigned long long lo = ld_relaxed(q);
  const unsigned long long hi = ld_relaxed(q + 1);
  int4 r = make_int4(static_cast<int32_t>(lo), static_cast<int32_t>(lo >> 32),
                     static_cast<int32_t>(hi), static_cast<int32_t>(hi >> 32));
  r.x = min(max(r.x, 0), P.n - 1);
  r.z = min(max(r.z, 0), P.nnz);
  r.y = min(max(r.y, 0), r.z);
  return r;
}

// ---------------------------------------------------------------------------
// Unlabelled BFS (one level structure).
// ---------------------------------------------------------------------------

// Level orders keep, for every vertex the current pass expands (each once),
// the key anchor - level in claim[] (claims belong to the labelled BFS,
// which those orders never run; anchor = the final position of the
// component's Cuthill-McKee label 0, so the keys of a component stay inside
// its block and a deeper level gets a smaller key), and sum the degrees
// expanded.  The last pass of the search leaves the keys of the root's level
// structure.  The store is issued after the vertex's row load, so that its
// completion overlaps that load instead of delaying the next one.
__device__ __forceinline__ void note_level(const BfsParams& P, Team& t, int32_t v, int32_t level,
                                           int32_t deg) {
  if (P.label_mode != 0) {
    __hip_atomic_store(&P.claim[v], static_cast<uint32_t>(t.anchor - level), __ATOMIC_RELAXED,
                       __HIP_MEMORY_SCOPE_AGENT);
    t.pm += deg;
  }
}

// Expand qi[lo, hi) (this work-group's share of the level).  A neighbour is
// new when atomicMax(visit, epoch) returns an older stamp; past-the-row lanes
// hit the parent's own stamp, which already equals epoch.  New vertices go
// to the LDS stage or, when it is full, straight to qi[cur_e + ...] (at a
// slot reserved on the team's tail counter, or, for a work-group alone, at
// its own index in the level).
__device__ __forceinline__ void bfs_expand(const BfsParams& P, Team& t, Shared& S, int32_t lo,
                                           int32_t hi, int32_t cur_e, int32_t end, int32_t epoch,
                                           int32_t new_level, int32_t* tail_slot, bool solo,
                                           uint64_t& mykey) {
  const int B = blockDim.x;
  for (int32_t p = lo + threadIdx.x; p < hi; p += B) {
    const int4 e = ld_rec(P, p);
    const int32_t u = e.x;
    if (e.y >= e.z) note_level(P, t, u, new_level - 1, e.w);
    for (int32_t k0 = e.y; k0 < e.z; k0 += kRB) {
      int32_t nb[kRB];
      load_batch(P.colidx, k0, e.z, u, nb);
      if (k0 == e.y) note_level(P, t, u, new_level - 1, e.w);
      int32_t old[kRB];
      int4 inf[kRB];
      // the records are loaded alongside the atomics (both need only nb)
#pragma unroll
      for (int j = 0; j < kRB; ++j) inf[j] = P.vinfo[nb[j]];
#pragma unroll
      for (int j = 0; j < kRB; ++j) old[j] = atomicMax(&P.visit[nb[j]], epoch);
      unsigned mask = 0;
#pragma unroll
      for (int j = 0; j < kRB; ++j) mask |= (old[j] < epoch ? 1u : 0u) << j;
      if (mask == 0) continue;
#pragma unroll
      for (int j = 0; j < kRB; ++j) {
        if (mask >> j & 1u) {
          const uint64_t kv = pack_key(inf[j].z, inf[j].w);
          mykey = kv < mykey ? kv : mykey;
        }
      }
      int32_t idx = atomicAdd(&S.cnt, __popc(mask));
#pragma unroll
      for (int j = 0; j < kRB; ++j) {
        if (!(mask >> j & 1u)) continue;
        const int4 r = record(nb[j], inf[j]);
        if (idx < kStageCap) {
          reinterpret_cast<int4*>(S.u.srec)[idx] = r;
        } else {
          const int32_t at = solo ? idx : atomicAdd(tail_slot, 1);
          if (cur_e + at < end) st_rec(&P.qi[cur_e + at], r);
        }
        ++idx;
      }
    }
  }
}

__device__ __forceinline__ uint32_t hslot(int32_t v) {
  return (static_cast<uint32_t>(v) * 2654435761u) >> (32 - kHashBits);
}

// Insert v into an LDS table (open addressing); returns its slot and sets
// *fresh when this call inserted it.  The engine keeps every table at most
// half full, so a free slot is always found.
__device__ __forceinline__ int h_insert(int32_t* key, int32_t v, bool* fresh) {
  uint32_t h = hslot(v);
  for (int i = 0; i < kHash; ++i) {
    int32_t k = key[h];
    if (k == kEmpty) {
      k = atomicCAS(&key[h], kEmpty, v);
      if (k == kEmpty) {
        *fresh = true;
        return static_cast<int>(h);
      }
    }
    if (k == v) {
      *fresh = false;
      return static_cast<int>(h);
    }
    h = (h + 1) & (kHash - 1);
  }
  *fresh = false;
  return -1;
}

__device__ __forceinline__ int4 lds_rec(const NarrowLds& N, int buf, int i) {
  return make_int4(N.lev[buf][i][0], N.lev[buf][i][1], N.lev[buf][i][2], N.lev[buf][i][3]);
}
__device__ __forceinline__ void lds_put(NarrowLds& N, int buf, int i, int4 r) {
  N.lev[buf][i][0] = r.x;
  N.lev[buf][i][1] = r.y;
  N.lev[buf][i][2] = r.z;
  N.lev[buf][i][3] = r.w;
}

// Unlabelled levels in one work-group with the frontier in LDS.  A neighbour
// is new when its visited stamp is older than this pass and this work-group
// is the first to insert it into the next level's LDS table (no global
// atomics).  Runs from the frontier qi[cur_b, cur_e) at `level` until the
// pass ends, the next level no longer fits (more than kNarrowCap vertices or
// more than kHash / 2 row entries), or it reaches stop_width vertices.
// (Telling visited neighbours from LDS tables of the previous two levels
// instead of the global stamps measured slower: 5.5 against 3.4 us per level
// on a 32-wide strip, the table probes being dependent LDS round trips per
// lane where the stamp loads of a row batch are in flight together.)
// Returns false, having done nothing, when the current frontier does not fit.
// On return the global key / tail slots are as the team levels expect them.
__device__ __forceinline__ bool lds_bfs_levels(const BfsParams& P, Team& t, Shared& S, int32_t end, int32_t epoch,
                               int32_t* tail, unsigned long long* minkey, int32_t& cur_b,
                               int32_t& cur_e, int32_t& level, bool& done, int32_t stop_width) {
  NarrowLds& N = S.u.nw;
  const int B = blockDim.x;
  int32_t len = cur_e - cur_b;
  if (len > kNarrowCap) return false;
  const long long c0 = wall_clock64();
  long long rs = 0;
  for (int32_t i = threadIdx.x; i < len; i += B) {
    const int4 r = ld_rec(P, cur_b + i);
    lds_put(N, level & 1, i, r);
    rs += r.z - r.y;
  }
  rs = block_sum_i64(rs, S.red);
  if (rs > kHash / 2) return false;
  for (int i = threadIdx.x; i < 2 * kHash; i += B) (&N.key[0][0])[i] = kEmpty;
  if (threadIdx.x == 0) {
    for (int i = 0; i < 3; ++i) {
      N.cnt[i] = 0;
      N.rows[i] = 0;
      N.kmin[i] = kMaxKey;
    }
    N.kmin[level % 3] = ld_relaxed(minkey + level % 3);
  }
  __syncthreads();
  int32_t nlev = 0;
  long long e_clear = 0, e_expand = 0, e_reduce = 0, e_book = 0;
  while (true) {
    const long long q0 = wall_clock64();
    const int nx = (level + 1) % 3;
    int32_t* key_ins = N.key[(level + 1) & 1];
    int32_t* key_clr = N.key[level & 1];
    for (int i = threadIdx.x; i < kHash; i += B) key_clr[i] = kEmpty;  // used again at level + 2
    if (threadIdx.x == 0) {
      N.cnt[(level + 2) % 3] = 0;
      N.rows[(level + 2) % 3] = 0;
      N.kmin[(level + 2) % 3] = kMaxKey;
    }
    const long long q1 = wall_clock64();
    uint64_t mykey = kMaxKey;
    for (int32_t i = threadIdx.x; i < len; i += B) {
      const int4 e = lds_rec(N, level & 1, i);
      const int32_t u = e.x;
      if (e.y >= e.z) note_level(P, t, u, level, e.w);
      for (int32_t k0 = e.y; k0 < e.z; k0 += kRB) {
        int32_t nb[kRB];
        load_batch(P.colidx, k0, e.z, u, nb);
        if (k0 == e.y) note_level(P, t, u, level, e.w);
        int32_t vs[kRB];
        int4 inf[kRB];
#pragma unroll
        for (int j = 0; j < kRB; ++j) vs[j] = ld_relaxed(&P.visit[nb[j]]);
#pragma unroll
        for (int j = 0; j < kRB; ++j) inf[j] = P.vinfo[nb[j]];
#pragma unroll
        for (int j = 0; j < kRB; ++j) {
          if (nb[j] == u || vs[j] == epoch) continue;
          bool fresh = false;
          if (h_insert(key_ins, nb[j], &fresh) < 0) continue;  // cannot happen (half full)
          if (!fresh) continue;
          const int32_t idx = atomicAdd(&N.cnt[nx], 1);
          atomicAdd(&N.rows[nx], inf[j].y - inf[j].x);
          const int4 r = record(nb[j], inf[j]);
          if (cur_e + idx < end) P.qi[cur_e + idx] = r;
          if (idx < kNarrowCap) lds_put(N, (level + 1) & 1, idx, r);
          P.visit[nb[j]] = epoch;
          const uint64_t kv = pack_key(inf[j].z, inf[j].w);
          mykey = kv < mykey ? kv : mykey;
        }
      }
    }
    const long long q2 = wall_clock64();
    mykey = wave_min_u64(mykey);
    if ((threadIdx.x & 63) == 0 && mykey != kMaxKey) atomicMin(&N.kmin[nx], mykey);
    // every 64th level: abort poll
    const bool poll = t.abort_flag != nullptr && (nlev & 63) == 63;
    if (poll && threadIdx.x == 0) {
      S.stop = ld_relaxed(&t.g->error) != 0 ? 1 : 0;
      if (!S.stop && abort_requested(t.abort_flag)) {
        flag_error(t.g, RCM_ERR_ABORTED, 22, t.comp, epoch, level);
        S.stop = 1;
      }
    }
    __syncthreads();
    const long long q3 = wall_clock64();
    const int32_t cnt = N.cnt[nx];
    const int32_t rows = N.rows[nx];
    ++nlev;
    if (poll && S.stop) {
      t.aborted = true;
      done = true;
      break;
    }
    e_clear += q1 - q0;
    e_expand += q2 - q1;
    e_reduce += q3 - q2;
    e_book += wall_clock64() - q3;
    if (cnt == 0) {
      done = true;
      break;
    }
    cur_b = cur_e;
    cur_e += cnt;
    ++level;
    len = cnt;
    if (cur_e > end) {
      if (threadIdx.x == 0)
        flag_error(t.g, RCM_ERR_NOT_SYMMETRIC, 6, t.comp, epoch, level, cur_b, cur_e, end);
      done = true;
      break;
    }
    if (cnt > kNarrowCap || rows > kHash / 2 || cnt >= stop_width) break;
  }
  if (threadIdx.x == 0) {
    // as the team levels leave them: the frontier's minimum key, an empty
    // slot for the next level, a zero append counter
    __hip_atomic_store(minkey + level % 3, N.kmin[level % 3], __ATOMIC_RELAXED,
                       __HIP_MEMORY_SCOPE_AGENT);
    __hip_atomic_store(minkey + (level + 1) % 3, kMaxKey, __ATOMIC_RELAXED,
                       __HIP_MEMORY_SCOPE_AGENT);
    st_relaxed(tail + level % 3, 0);
    st_relaxed(tail + (level + 1) % 3, 0);
    t.ctl->clk[8] += wall_clock64() - c0;
    t.ctl->clk[9] += nlev;
    t.ctl->clk[20] += e_clear;
    t.ctl->clk[21] += e_expand;
    t.ctl->clk[22] += e_reduce;
    t.ctl->clk[23] += e_book;
  }
  __syncthreads();
  return true;
}

// One unlabelled level with the global frontier: the whole team (solo =
// false) or one work-group (solo = true).  Advances cur_b / cur_e / level;
// sets done when the level was the last one.
__device__ __forceinline__ void global_bfs_level(const BfsParams& P, Team& t, Shared& S, int32_t end,
                                 int32_t epoch, int32_t* tail, unsigned long long* minkey,
                                 bool solo, int32_t& cur_b, int32_t& cur_e, int32_t& level,
                                 bool& done) {
  const int B = blockDim.x;
  const int W = solo ? 1 : t.W;
  const int wid = solo ? 0 : t.wid;
  const int l3 = level % 3;
  if (threadIdx.x == 0) {
    S.cnt = 0;
    S.key = kMaxKey;
  }
  __syncthreads();
  int32_t lo, hi;
  my_chunk(cur_b, cur_e, W, wid, lo, hi);
  uint64_t mykey = kMaxKey;
  const long long ta = wall_clock64();
  bfs_expand(P, t, S, lo, hi, cur_e, end, epoch, level + 1, tail + l3, solo, mykey);
  mykey = wave_min_u64(mykey);
  if ((threadIdx.x & 63) == 0 && mykey != kMaxKey) atomicMin(&S.key, mykey);
  __syncthreads();
  const long long tb = wall_clock64();
  // final here; read now, since the next level resets it after fewer
  // barriers than separate this read from the end of the level
  const int32_t own_cnt = S.cnt;
  if (threadIdx.x == 0) {
    const int32_t ns = own_cnt < kStageCap ? own_cnt : kStageCap;
    if (solo) {
      // alone: the level is this work-group's own count, nothing to reserve
      S.base = 0;
      __hip_atomic_store(minkey + (level + 1) % 3, S.key, __ATOMIC_RELAXED,
                         __HIP_MEMORY_SCOPE_AGENT);
    } else {
      S.base = ns > 0 ? atomicAdd(tail + l3, ns) : 0;
      if (S.key != kMaxKey) atomicMin(minkey + (level + 1) % 3, S.key);
    }
    if (wid == 0) {
      // slots of the level after next; nobody reads them any more
      st_relaxed(tail + (level + 1) % 3, 0);
      __hip_atomic_store(minkey + (level + 2) % 3, kMaxKey, __ATOMIC_RELAXED,
                         __HIP_MEMORY_SCOPE_AGENT);
    }
  }
  __syncthreads();
  const long long tc = wall_clock64();
  {
    const int32_t ns = S.cnt < kStageCap ? S.cnt : kStageCap;
    const int4* stage = reinterpret_cast<const int4*>(S.u.srec);
    for (int32_t i = threadIdx.x; i < ns; i += B) {
      const int32_t at = cur_e + S.base + i;
      if (at < end) st_rec(&P.qi[at], stage[i]);
    }
  }
  team_barrier(t, S, solo);
  if (t.aborted) return;
  const int32_t cnt = solo ? own_cnt : ld_relaxed(tail + l3);
  if (t.wid == 0 && threadIdx.x == 0) {
    const long long td = wall_clock64();
    if (solo) {
      t.ctl->clk[10] += td - ta;
      t.ctl->clk[11] += 1;
    } else {
      t.ctl->clk[4] += tb - ta;
      t.ctl->clk[5] += tc - tb;
      t.ctl->clk[6] += td - tc;
      t.ctl->clk[7] += 1;
    }
  }
  if (cnt == 0) {
    done = true;
    return;
  }
  cur_b = cur_e;
  cur_e += cnt;
  ++level;
  if (cur_e > end) {  // left the component: the pattern is not symmetric
    if (threadIdx.x == 0)
      flag_error(t.g, RCM_ERR_NOT_SYMMETRIC, 1, t.comp, epoch, level, cur_b, cur_e, end);
    done = true;
  }
}

// Wide unlabelled levels with each work-group's share of the frontier in LDS:
// a work-group expands the vertices it found itself at the previous level
// (plus, at the first level and after a spill, its chunk of records in qi),
// so records neither go to nor come back from qi.  The level's size and a
// spill flag travel in the team barrier's slot payload, and the next
// level's minimum key is issued just before arriving (it is only read once
// the pass ends, behind a full barrier).  Enters with the
// frontier in qi[cur_b, cur_e); returns when the pass has ended (done) or
// the frontier is narrower than the narrow cutoff, which is then written to
// qi[cur_b, cur_e) for the narrow levels.
__device__ __forceinline__ void own_bfs_levels(const BfsParams& P, Team& t, Shared& S,
                                               int32_t end, int32_t epoch, int32_t* tail,
                                               unsigned long long* minkey, int32_t& cur_b,
                                               int32_t& cur_e, int32_t& level, bool& done) {
  const int B = blockDim.x;
  int cb = 0;                          // LDS buffer holding this work-group's frontier
  int32_t own_n = 0;                   // records in it
  int32_t g_b = cur_b, g_e = cur_e;    // records in qi expanded chunk-wise
  int since = 0;                       // levels since the frontier was spread evenly
  while (true) {
    const int l3 = level % 3;
    // Each work-group keeps what it found, so the shares drift apart from
    // level to level; every `rebalance` levels the whole next level goes to
    // qi (one reservation per work-group) and is chunked evenly again.
    const bool spread = ++since >= P.rebalance;
    if (spread) since = 0;
    if (threadIdx.x == 0) {
      S.cnt = 0;
      S.key = kMaxKey;
      S.spill = 0;
    }
    __syncthreads();
    const long long ta = wall_clock64();
    int32_t lo, hi;
    my_chunk(g_b, g_e, t.W, t.wid, lo, hi);
    const int32_t n_glob = hi - lo;
    uint64_t mykey = kMaxKey;
    for (int32_t i = threadIdx.x; i < n_glob + own_n; i += B) {
      int4 e;
      if (i < n_glob) {
        e = ld_rec(P, lo + i);
      } else {
        const int32_t j = i - n_glob;
        e = make_int4(S.u.own[cb][j][0], S.u.own[cb][j][1], S.u.own[cb][j][2],
                      S.u.own[cb][j][3]);
      }
      const int32_t u = e.x;
      if (e.y >= e.z) note_level(P, t, u, level, e.w);
      for (int32_t k0 = e.y; k0 < e.z; k0 += kRB) {
        int32_t nb[kRB];
        load_batch(P.colidx, k0, e.z, u, nb);
        if (k0 == e.y) note_level(P, t, u, level, e.w);
        int4 inf[kRB];
        int32_t old[kRB];
#pragma unroll
        for (int j = 0; j < kRB; ++j) inf[j] = P.vinfo[nb[j]];
#pragma unroll
        for (int j = 0; j < kRB; ++j) old[j] = atomicMax(&P.visit[nb[j]], epoch);
        unsigned mask = 0;
#pragma unroll
        for (int j = 0; j < kRB; ++j) mask |= (old[j] < epoch ? 1u : 0u) << j;
        if (mask == 0) continue;
        int32_t idx = atomicAdd(&S.cnt, __popc(mask));
#pragma unroll
        for (int j = 0; j < kRB; ++j) {
          if (!(mask >> j & 1u)) continue;
          const uint64_t kv = pack_key(inf[j].z, inf[j].w);
          mykey = kv < mykey ? kv : mykey;
          if (idx < kOwnCap) {
            S.u.own[cb ^ 1][idx][0] = nb[j];
            S.u.own[cb ^ 1][idx][1] = inf[j].x;
            S.u.own[cb ^ 1][idx][2] = inf[j].y;
            S.u.own[cb ^ 1][idx][3] = inf[j].z;
          } else {
            const int32_t at = atomicAdd(tail + l3, 1);
            if (cur_e + at < end) st_rec(&P.qi[cur_e + at], record(nb[j], inf[j]));
            S.spill = 1;
          }
          ++idx;
        }
      }
    }
    mykey = wave_min_u64(mykey);
    if ((threadIdx.x & 63) == 0 && mykey != kMaxKey) atomicMin(&S.key, mykey);
    __syncthreads();
    const long long tb = wall_clock64();
    const int32_t my_new = S.cnt;
    const int32_t kept = my_new < kOwnCap ? my_new : kOwnCap;
    if (spread) {
      if (threadIdx.x == 0) {
        S.base = kept > 0 ? atomicAdd(tail + l3, kept) : 0;
        if (kept > 0) S.spill = 1;
      }
      __syncthreads();
      for (int32_t i = threadIdx.x; i < kept; i += B) {
        const int32_t at = cur_e + S.base + i;
        if (at < end)
          st_rec(&P.qi[at], make_int4(S.u.own[cb ^ 1][i][0], S.u.own[cb ^ 1][i][1],
                                      S.u.own[cb ^ 1][i][2], S.u.own[cb ^ 1][i][3]));
      }
    }
    const bool spilled = S.spill != 0;
    if (spilled) {
      // records in qi must be complete before this work-group arrives
      drain_memory_ops();
      __syncthreads();
    }
    if (threadIdx.x == 0) {
      if (t.wid == 0) {
        // slots two levels ahead: free now, needed again after the next barrier
        st_relaxed(tail + (level + 1) % 3, 0);
        __hip_atomic_store(minkey + (level + 2) % 3, kMaxKey, __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_AGENT);
        drain_memory_ops();
      }
      // the next level's minimum key is only read once the pass has ended,
      // behind a full barrier
      if (S.key != kMaxKey) atomicMin(minkey + (level + 1) % 3, S.key);
    }
    // the level's size travels with the arrival; a flag marks a spill to qi
    slot_exchange(t, S, (spilled ? 0x80000000u : 0u) | static_cast<uint32_t>(my_new), false);
    if (t.aborted) return;
    if (threadIdx.x == 0) {
      S.total = S.wtot;
      S.nspill = 0;
      // some work-group spilled: its records are in qi
      if (S.wspill != 0) S.nspill = ld_relaxed(tail + l3);
    }
    __syncthreads();
    const int32_t total = S.total;
    const int32_t nspill = S.nspill;
    if (t.wid == 0 && threadIdx.x == 0) {
      t.ctl->clk[4] += tb - ta;
      t.ctl->clk[6] += wall_clock64() - tb;
      t.ctl->clk[7] += 1;
    }
    if (total == 0) {
      // the pass ended at this level: every minimum-key atomic is complete
      // before anyone reads the last level's key
      done = true;
      team_barrier(t, S, false);
      return;
    }
    cur_b = cur_e;
    cur_e += total;
    ++level;
    if (cur_e > end) {  // left the component: the pattern is not symmetric
      if (threadIdx.x == 0)
        flag_error(t.g, RCM_ERR_NOT_SYMMETRIC, 8, t.comp, epoch, level, cur_b, cur_e, end);
      done = true;
      t.aborted = true;
      return;
    }
    cb ^= 1;
    own_n = spread ? 0 : kept;
    g_b = cur_b;
    g_e = cur_b + nspill;
    if (total < P.narrow_cutoff) {
      // hand the frontier to the narrow levels: own records after the
      // spilled ones, in work-group order
      slot_exchange(t, S, static_cast<uint32_t>(own_n), true);
      if (t.aborted) return;
      const int32_t prefix = S.wpre;
      for (int32_t i = threadIdx.x; i < own_n; i += B) {
        const int32_t at = g_e + prefix + i;
        if (at < end)
          st_rec(&P.qi[at], make_int4(S.u.own[cb][i][0], S.u.own[cb][i][1], S.u.own[cb][i][2],
                                      S.u.own[cb][i][3]));
      }
      team_barrier(t, S, false);
      return;
    }
  }
}

// One level structure (Section II-A) of the component whose label block is
// [o, end), rooted at `root`.  Vertices are written level by level into qi.
// Returns the eccentricity of root and the minimum (degree << 32 | id) over
// the last level.  With find_end, the block end is unknown (end bounds it)
// and the pass reports where the component ended.
__device__ __forceinline__ void bfs_pass(const BfsParams& P, Team& t, Shared& S, int32_t o, int32_t end,
                         int32_t root, int32_t epoch, int parity, int32_t& ecc,
                         uint64_t& lastkey, bool find_end, int32_t& found_end) {
  const long long clk0 = wall_clock64();
  int32_t* tail = t.ctl->tail + parity * 3;
  unsigned long long* minkey = t.ctl->minkey + parity * 3;
  t.pm = 0;
  if (t.wid == 0 && threadIdx.x == 0) {
    const int4 ri = P.vinfo[root];
    st_rec(&P.qi[o], record(root, ri));
    __hip_atomic_store(&P.visit[root], epoch, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __hip_atomic_store(&t.ctl->pass_m[parity], 0ll, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    for (int i = 0; i < 3; ++i) st_relaxed(tail + i, 0);
    __hip_atomic_store(minkey + 0, pack_key(ri.z, ri.w), __ATOMIC_RELAXED,
                       __HIP_MEMORY_SCOPE_AGENT);
    __hip_atomic_store(minkey + 1, kMaxKey, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __hip_atomic_store(minkey + 2, kMaxKey, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
  team_barrier(t, S, false);
  if (t.aborted) return;
  int32_t cur_b = o, cur_e = o + 1, level = 0;
  bool done = false;
  while (!done) {
    const bool narrow = t.W > 1 && (cur_e - cur_b) < P.narrow_cutoff;
    if (narrow && t.wid != 0) {
      // sleep until work-group 0 has walked the narrow stretch
      narrow_wait(t, S);
      if (t.aborted) return;
      cur_b = S.state[0];
      cur_e = S.state[1];
      level = S.state[2];
      done = S.state[3] != 0;
      continue;
    }
    if (narrow || t.W == 1) {
      // one work-group: the LDS engine where the frontier fits, else one
      // global level at a time
      const int32_t stop = narrow ? P.narrow_cutoff : 0x7fffffff;
      int skip = 0;
      while (!done && (cur_e - cur_b) < stop) {
        bool ran = false;
        if (skip == 0) {
          ran = lds_bfs_levels(P, t, S, end, epoch, tail, minkey, cur_b, cur_e, level, done,
                               stop);
          if (!ran) skip = 8;
        } else {
          --skip;
        }
        if (!ran) global_bfs_level(P, t, S, end, epoch, tail, minkey, true, cur_b, cur_e, level,
                                   done);
        if (t.aborted) return;
      }
      if (narrow) {
        narrow_publish(t, cur_b, cur_e, level, done);
      }
      continue;
    }
    // wide levels: the whole team
    if (!done && (cur_e - cur_b) >= P.narrow_cutoff) {
      own_bfs_levels(P, t, S, end, epoch, tail, minkey, cur_b, cur_e, level, done);
      if (t.aborted) return;
    }
  }
  if (cur_e > end) {  // flagged inside already
    t.aborted = true;
    return;
  }
  if (find_end) {
    // size discovery: the component is whatever this pass reached
    found_end = cur_e;
  } else if (cur_e != end) {
    if (threadIdx.x == 0 && t.wid == 0)
      flag_error(t.g, RCM_ERR_NOT_SYMMETRIC, 2, t.comp, epoch, level, cur_b, cur_e, end);
    t.aborted = true;
    return;
  }
  if (P.label_mode != 0) {
    const long long tot = block_sum_i64(t.pm, S.red);
    if (threadIdx.x == 0 && tot != 0)
      __hip_atomic_fetch_add(&t.ctl->pass_m[parity], tot, __ATOMIC_RELAXED,
                             __HIP_MEMORY_SCOPE_AGENT);
  }
  __syncthreads();
  // the last level's slot is stable until the next pass of the same parity
  ecc = level;
  lastkey = ld_relaxed(minkey + level % 3);
  // every work-group has read the counters before the next pass reuses them
  team_barrier(t, S, false);
  if (P.label_mode != 0)
    t.pm = __hip_atomic_load(&t.ctl->pass_m[parity], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  if (t.wid == 0 && threadIdx.x == 0) {
    t.ctl->clk[0] += wall_clock64() - clk0;
    t.ctl->clk[2] += level + 1;
  }
}

// ---------------------------------------------------------------------------
// Asynchronous level structure: a label-correcting BFS without a barrier per
// level (the non-level-synchronous BFS that Section VI leaves as future
// work).  It yields the same eccentricity and the same minimum-(degree, id)
// vertex of the last level as bfs_pass, because the distances it settles on
// are the exact BFS distances whatever order the updates take.
// ---------------------------------------------------------------------------

// dkey[v] = tag << 32 | (2^32 - 1 - distance): in one pass a larger word is a
// shorter distance, and every word of the current pass (its tag) beats those
// of earlier passes, so atomicMax both visits and corrects.
__device__ __forceinline__ unsigned long long dist_key(uint32_t tag, int32_t d) {
  return (static_cast<unsigned long long>(tag) << 32) |
         (0xFFFFFFFFu - static_cast<uint32_t>(d));
}

// Position of virtual ring index v in qi[o, o + ring).
__device__ __forceinline__ int32_t ring_pos(int32_t o, int32_t ring, int32_t v) {
  return o + static_cast<int32_t>(static_cast<uint32_t>(v) % static_cast<uint32_t>(ring));
}

// One batch of entries [k0, min(k0 + kRB, kend)) of the row of a current
// record (vertex u at distance du) in an asynchronous pass on the CSR: the
// neighbours' records are gathered alongside the atomics on their distance
// words, and the neighbours this record reached are appended to the next
// own frontier (or, past its capacity, straight into the next round's ring).
// Reading the words first to spare the atomics of edges into vertices
// already as close adds a dependent round trip per step, which measured
// slower (3.5 -> 5.6 us per step on the 128^3 grid).
__device__ __forceinline__ void async_expand_batch(const BfsParams& P, Shared& S, int32_t u,
                                                   int32_t du, int32_t k0, int32_t kend,
                                                   unsigned long long want, int cb, int32_t o,
                                                   int32_t ring, int32_t room, int32_t g_e,
                                                   int32_t* tail) {
  int32_t nb[kRB];
  load_batch(P.colidx, k0, kend, u, nb);
  int4 inf[kRB];
  unsigned long long old[kRB];
#pragma unroll
  for (int j = 0; j < kRB; ++j) inf[j] = P.vinfo[nb[j]];
  // past-the-row lanes and self loops hit u, whose word beats want
#pragma unroll
  for (int j = 0; j < kRB; ++j) old[j] = atomicMax(&P.dkey[nb[j]], want);
  unsigned mask = 0;
#pragma unroll
  for (int j = 0; j < kRB; ++j) mask |= (old[j] < want ? 1u : 0u) << j;
  if (mask == 0) return;
  int32_t idx = atomicAdd(&S.cnt, __popc(mask));
#pragma unroll
  for (int j = 0; j < kRB; ++j) {
    if (!(mask >> j & 1u)) continue;
    if (idx < kOwnCap) {
      S.u.own[cb ^ 1][idx][0] = nb[j];
      S.u.own[cb ^ 1][idx][1] = inf[j].x;
      S.u.own[cb ^ 1][idx][2] = inf[j].y;
      S.u.own[cb ^ 1][idx][3] = du + 1;
    } else {
      // straight into the next round's frontier
      const int32_t at = atomicAdd(tail, 1);
      atomicAdd(&S.appended, 1);
      if (at < room) {
        st_rec(&P.qi[ring_pos(o, ring, g_e + at)], make_int4(nb[j], inf[j].x, inf[j].y, du + 1));
      } else {
        S.ovf = 1;
      }
      S.spill = 1;
    }
    ++idx;
  }
}

// One step of an asynchronous pass over a graph with a fixed-stride row
// copy.  A record's row is already in LDS (the first kORowCap records of the
// own buffer) or at a known address, so the supersede test of the record,
// the atomics on its neighbours' distance words and the loads of those
// neighbours' rows are all one round trip; the rows of the neighbours it
// reaches go into LDS with their records.  A record found superseded has
// made its atomics by then.  That is harmless: a neighbour w it won at
// distance du + 1 is adjacent to the record's vertex, whose distance is now
// below du, so the record that lowered it reaches w with a shorter distance
// later and expands it from there.  Only the records of a current vertex
// expand what they reached.
__device__ __forceinline__ void async_step_ell(const BfsParams& P, Shared& S, int32_t o,
                                               int32_t ring, int32_t lo, int32_t n_glob,
                                               int32_t own_n, int cb, uint32_t tag, int32_t room,
                                               int32_t g_e, int32_t* tail, long long& d_exp,
                                               long long& d_sup) {
  const int B = blockDim.x;
  for (int32_t i = threadIdx.x; i < n_glob + own_n; i += B) {
    int32_t u, du;
    int32_t nb[kRB];
    if (i < n_glob) {
      const int4 e = ld_rec(P, ring_pos(o, ring, lo + i));
      u = e.x;
      du = e.w;
      ell_row(P.ell, u, nb);
    } else {
      const int32_t j = i - n_glob;
      u = S.u.own[cb][j][0];
      du = S.u.own[cb][j][3];
      if (j < kORowCap) {
        const int4 a = S.orow[cb][j][0];
        const int4 b = S.orow[cb][j][1];
        nb[0] = a.x; nb[1] = a.y; nb[2] = a.z; nb[3] = a.w;
        nb[4] = b.x; nb[5] = b.y; nb[6] = b.z; nb[7] = b.w;
      } else {
        ell_row(P.ell, u, nb);
      }
    }
    const unsigned long long mine = dist_key(tag, du);
    const unsigned long long want = dist_key(tag, du + 1);
    const unsigned long long cur =
        __hip_atomic_load(&P.dkey[u], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    // Branch-free, so that every load and atomic is in flight before the
    // first result is waited for: the row's own vertex (its diagonal entry
    // and the padding) gets its atomic, which its own word always beats,
    // and loads vertex 0's row, one cache line for the whole wave, unused.
    // (rows in plain int arrays, which the compiler keeps in registers;
    // arrays of int4 it may leave in scratch memory)
    unsigned long long old[kRB];
    int32_t rw[kRB][kEllWidth];
#pragma unroll
    for (int j = 0; j < kRB; ++j) old[j] = atomicMax(&P.dkey[nb[j]], want);
#pragma unroll
    for (int j = 0; j < kRB; ++j) ell_row(P.ell, nb[j] != u ? nb[j] : 0, rw[j]);
    // a compiler barrier: the row loads are only used behind the
    // supersede test, and moved there they would start a round trip of
    // their own
    issue_fence();
    if (cur != mine) {
      ++d_sup;
      continue;
    }
    ++d_exp;
    unsigned mask = 0;
#pragma unroll
    for (int j = 0; j < kRB; ++j) mask |= (old[j] < want ? 1u : 0u) << j;
    if (mask == 0) continue;
    const int32_t base = atomicAdd(&S.cnt, __popc(mask));
    // each reached neighbour's place from the mask alone (no count carried
    // from one entry to the next, so the rows stay in registers)
#pragma unroll
    for (int j = 0; j < kRB; ++j) {
      if (!(mask >> j & 1u)) continue;
      const int32_t idx = base + __popc(mask & ((1u << j) - 1u));
      if (idx < kORowCap) {
        S.u.own[cb ^ 1][idx][0] = nb[j];
        S.u.own[cb ^ 1][idx][1] = 0;
        S.u.own[cb ^ 1][idx][2] = 0;
        S.u.own[cb ^ 1][idx][3] = du + 1;
        S.orow[cb ^ 1][idx][0] = make_int4(rw[j][0], rw[j][1], rw[j][2], rw[j][3]);
        S.orow[cb ^ 1][idx][1] = make_int4(rw[j][4], rw[j][5], rw[j][6], rw[j][7]);
      } else if (idx < kOwnCap) {
        S.u.own[cb ^ 1][idx][0] = nb[j];
        S.u.own[cb ^ 1][idx][1] = 0;
        S.u.own[cb ^ 1][idx][2] = 0;
        S.u.own[cb ^ 1][idx][3] = du + 1;
      } else {
        // straight into the next round's frontier (its row is reloaded)
        const int32_t at = atomicAdd(tail, 1);
        atomicAdd(&S.appended, 1);
        if (at < room) {
          st_rec(&P.qi[ring_pos(o, ring, g_e + at)], make_int4(nb[j], 0, 0, du + 1));
        } else {
          S.ovf = 1;
        }
        S.spill = 1;
      }
    }
  }
}

// One level structure of the component whose label block is [o, end), from
// `root`, for a team of several work-groups.  Rounds: every work-group
// expands its share of the frontier and then, for up to `search_round` steps,
// the vertices it reached itself (records carry their tentative distance;
// an improved vertex is expanded again by whoever improved it, a superseded
// record is skipped), with no team barrier between the steps.  One barrier
// per round then spreads all records evenly (qi[o, end) serves as a ring of
// frontier records) and detects the end.  Finally a sweep over the vertices
// of the component's graph [seg_b, seg_e) (a component never leaves its
// graph) carrying this pass's tag yields the eccentricity, the last level's minimum
// key, the number of vertices reached (the component's size when find_end
// is given) and, for level orders, the keys.  Returns false if the ring
// would overflow (a frontier and its successor above the block size), having
// computed nothing: the caller then runs bfs_pass.
__device__ __forceinline__ bool async_bfs_pass(const BfsParams& P, Team& t, Shared& S, int32_t o,
                                               int32_t end, int32_t root, uint32_t tag, int parity,
                                               int32_t seg_b, int32_t seg_e, int32_t& ecc,
                                               uint64_t& lastkey, bool find_end, int32_t& found_end) {
  const long long clk0 = wall_clock64();
  const int B = blockDim.x;
  int32_t* tail = t.ctl->tail + parity * 3;
  const int32_t ring = end - o;
  if (t.wid == 0 && threadIdx.x == 0) {
    const int4 ri = P.vinfo[root];
    __hip_atomic_store(&P.dkey[root], dist_key(tag, 0), __ATOMIC_RELAXED,
                       __HIP_MEMORY_SCOPE_AGENT);
    st_rec(&P.qi[o], make_int4(root, ri.x, ri.y, 0));
    for (int i = 0; i < 3; ++i) st_relaxed(tail + i, 0);
    st_relaxed(&t.ctl->a_ecc[parity], 0);
    st_relaxed(&t.ctl->a_cnt[parity], 0);
    __hip_atomic_store(&t.ctl->a_key[parity], kMaxKey, __ATOMIC_RELAXED,
                       __HIP_MEMORY_SCOPE_AGENT);
    __hip_atomic_store(&t.ctl->pass_m[parity], 0ll, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
  team_barrier(t, S, false);
  if (t.aborted) return true;
  int32_t g_b = 0, g_e = 1;  // the frontier: virtual ring indices [g_b, g_e)
  int32_t rounds = 0;
  bool overflow = false;
  // diagnostics (work-group 0): steps, records expanded / skipped, ticks
  long long d_steps = 0, d_exp = 0, d_sup = 0, d_tstep = 0, d_tbar = 0;
  while (true) {
    const int l3 = rounds % 3;
    int32_t lo, hi;
    my_chunk(g_b, g_e, t.W, t.wid, lo, hi);
    int32_t n_glob = hi - lo;
    const int32_t room = ring - (g_e - g_b);  // ring slots the next frontier may use
    int cb = 0;
    int32_t own_n = 0;
    if (threadIdx.x == 0) {
      S.spill = 0;
      S.ovf = 0;
      S.appended = 0;
    }
    const long long r0 = wall_clock64();
    for (int step = 0; step < P.search_round; ++step) {
      if (threadIdx.x == 0) {
        S.cnt = 0;
        S.nheavy = 0;
      }
      __syncthreads();
      ++d_steps;
      if (P.ell != nullptr) {
        async_step_ell(P, S, o, ring, lo, n_glob, own_n, cb, tag, room, g_e, tail + l3, d_exp,
                       d_sup);
      } else {
      for (int32_t i = threadIdx.x; i < n_glob + own_n; i += B) {
        int4 e;
        if (i < n_glob) {
          e = ld_rec(P, ring_pos(o, ring, lo + i));
        } else {
          const int32_t j = i - n_glob;
          e = make_int4(S.u.own[cb][j][0], S.u.own[cb][j][1], S.u.own[cb][j][2],
                        S.u.own[cb][j][3]);
        }
        const int32_t u = e.x;
        const int32_t du = e.w;
        // a record whose vertex has since been reached by a shorter path is
        // superseded (the vertex is expanded again from that path)
        const unsigned long long cur =
            __hip_atomic_load(&P.dkey[u], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        const unsigned long long want = dist_key(tag, du + 1);
        if (cur == dist_key(tag, du)) ++d_exp; else ++d_sup;
        if (cur != dist_key(tag, du)) continue;
        if (e.z - e.y > kHeavyRow) {
          // a long row: the whole work-group expands it below
          const int h = atomicAdd(&S.nheavy, 1);
          if (h < kHeavyCap) {
            S.heavy[h] = e;
            continue;
          }
        }
        for (int32_t k0 = e.y; k0 < e.z; k0 += kRB)
          async_expand_batch(P, S, u, du, k0, e.z, want, cb, o, ring, room, g_e, tail + l3);
      }
      __syncthreads();
      // the records on long rows, one at a time, a batch per thread
      const int nh = S.nheavy < kHeavyCap ? S.nheavy : kHeavyCap;
      for (int h = 0; h < nh; ++h) {
        const int4 e = S.heavy[h];
        const unsigned long long want = dist_key(tag, e.w + 1);
        for (int32_t k0 = e.y + static_cast<int32_t>(threadIdx.x) * kRB; k0 < e.z; k0 += B * kRB)
          async_expand_batch(P, S, e.x, e.w, k0, e.z, want, cb, o, ring, room, g_e, tail + l3);
      }
      }
      __syncthreads();
      const int32_t cnt = S.cnt;
      if (threadIdx.x == 0) S.nheavy = 0;  // (read by every thread before the barrier)
      own_n = cnt < kOwnCap ? cnt : kOwnCap;
      cb ^= 1;
      n_glob = 0;
      if (own_n == 0) break;
    }
    const long long r1 = wall_clock64();
    d_tstep += r1 - r0;
    // the rest of this work-group's records go to the next round's frontier
    if (threadIdx.x == 0) {
      S.base = own_n > 0 ? atomicAdd(tail + l3, own_n) : 0;
      if (own_n > 0) S.spill = 1;
      S.appended += own_n;
    }
    __syncthreads();
    for (int32_t i = threadIdx.x; i < own_n; i += B) {
      const int32_t at = S.base + i;
      if (at < room) {
        st_rec(&P.qi[ring_pos(o, ring, g_e + at)],
               make_int4(S.u.own[cb][i][0], S.u.own[cb][i][1], S.u.own[cb][i][2],
                         S.u.own[cb][i][3]));
      } else {
        S.ovf = 1;
      }
    }
    __syncthreads();
    const bool wrote = S.spill != 0;
    if (wrote) {
      // records in qi must be complete before this work-group arrives
      drain_memory_ops();
      __syncthreads();
    }
    if (t.wid == 0 && threadIdx.x == 0) {
      // the counter two rounds ahead: free now, needed after the next barrier
      st_relaxed(tail + (rounds + 1) % 3, 0);
      drain_memory_ops();
    }
    // payload: the records this work-group added to the ring (every add,
    // its own and its spills, went through the tail counter, so the team's
    // sum is the next frontier's size and the counter need not be read
    // back), and a flag for an overflow
    slot_exchange(t, S, (S.ovf ? 0x80000000u : 0u) | static_cast<uint32_t>(S.appended), false);
    if (t.aborted) return true;
    if (S.wspill != 0) {
      overflow = true;
      break;
    }
    const int32_t total = S.wtot;
    ++rounds;
    d_tbar += wall_clock64() - r1;
    if (total == 0) break;
    g_b = g_e;
    g_e += total;
    // bounds that a correct pass never reaches (index range, round count,
    // the device wait limit for the whole pass)
    if (g_e < 0 || rounds > 4 * ring + 16 || wall_clock64() - clk0 > kWaitLimitTicks) {
      if (threadIdx.x == 0) flag_error(t.g, RCM_ERR_ABORTED, 11, t.comp);
      t.aborted = true;
      return true;
    }
  }
  // every update of the pass is complete and visible before the sweep
  team_barrier(t, S, false);
  if (t.aborted || overflow) return !overflow;
  // sweep: this pass's distances are final
  int32_t my_max = -1, my_cnt = 0;
  uint64_t my_key = kMaxKey;
  long long my_m = 0;
  for (int32_t v = seg_b + t.wid * B + threadIdx.x; v < seg_e; v += t.W * B) {
    const unsigned long long kv = ld_relaxed(&P.dkey[v]);
    if (static_cast<uint32_t>(kv >> 32) != tag) continue;
    const int32_t d = static_cast<int32_t>(0xFFFFFFFFu - static_cast<uint32_t>(kv));
    ++my_cnt;
    // the visited stamp, as a level-synchronous pass leaves it (the search
    // for the other components skips the stamped vertices of vertex 0's)
    __hip_atomic_store(&P.visit[v], static_cast<int32_t>(tag & 63u), __ATOMIC_RELAXED,
                       __HIP_MEMORY_SCOPE_AGENT);
    if (P.label_mode != 0) {
      my_m += P.vinfo[v].z;
      __hip_atomic_store(&P.claim[v], static_cast<uint32_t>(t.anchor - d), __ATOMIC_RELAXED,
                         __HIP_MEMORY_SCOPE_AGENT);
    }
    if (d >= my_max) {
      const int4 vi = P.vinfo[v];
      const uint64_t kk = pack_key(vi.z, vi.w);
      if (d > my_max) {
        my_max = d;
        my_key = kk;
      } else if (kk < my_key) {
        my_key = kk;
      }
    }
  }
  // the largest distance first (with the counts), then the minimum key there
  if (threadIdx.x == 0) S.cnt = -1;
  __syncthreads();
  atomicMax(&S.cnt, my_max);
  const long long cnt_sum = block_sum_i64(my_cnt, S.red);
  const long long m_sum = block_sum_i64(my_m, S.red);
  const int32_t wg_max = S.cnt;
  if (threadIdx.x == 0) {
    if (wg_max >= 0) atomicMax(&t.ctl->a_ecc[parity], wg_max);
    if (cnt_sum != 0) atomicAdd(&t.ctl->a_cnt[parity], static_cast<int32_t>(cnt_sum));
    if (m_sum != 0)
      __hip_atomic_fetch_add(&t.ctl->pass_m[parity], m_sum, __ATOMIC_RELAXED,
                             __HIP_MEMORY_SCOPE_AGENT);
  }
  team_barrier(t, S, false);
  if (t.aborted) return true;
  const int32_t e_all = ld_relaxed(&t.ctl->a_ecc[parity]);
  if (my_max == e_all && my_key != kMaxKey) atomicMin(&t.ctl->a_key[parity], my_key);
  team_barrier(t, S, false);
  if (t.aborted) return true;
  ecc = e_all;
  lastkey = __hip_atomic_load(&t.ctl->a_key[parity], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  const int32_t count = ld_relaxed(&t.ctl->a_cnt[parity]);
  if (P.label_mode != 0)
    t.pm = __hip_atomic_load(&t.ctl->pass_m[parity], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  if (find_end) {
    found_end = o + count;
  } else if (count != end - o) {
    // the pass reached more or fewer vertices than the component holds
    if (threadIdx.x == 0 && t.wid == 0)
      flag_error(t.g, RCM_ERR_NOT_SYMMETRIC, 12, t.comp, 0, ecc, count, end - o, end);
    t.aborted = true;
    return true;
  }
  // records counted per thread: sum them over the work-group
  d_exp = block_sum_i64(d_exp, S.red);
  d_sup = block_sum_i64(d_sup, S.red);
  if (t.wid == 0 && threadIdx.x == 0) {
    t.ctl->clk[0] += wall_clock64() - clk0;
    t.ctl->clk[2] += ecc + 1;
    t.ctl->clk[24] += rounds;
    t.ctl->clk[25] += d_steps;
    t.ctl->clk[26] += d_exp;
    t.ctl->clk[27] += d_sup;
    t.ctl->clk[28] += d_tstep;
    t.ctl->clk[29] += d_tbar;
  }
  return true;
}

// ---------------------------------------------------------------------------
// Labelled BFS (Algorithm 3).
// ---------------------------------------------------------------------------

// (select2nd, min) SpMSpV contribution of one newly labelled vertex: its
// label becomes a claim on every neighbour.  Lanes past the row end and
// already labelled neighbours hold smaller claims, so the min leaves them
// alone (the Select(R == -1) step).  Fire-and-forget atomics.
__device__ __forceinline__ void claim_batch(const BfsParams& P, const int32_t* nb,
                                            uint32_t label) {
  // claims only decrease, so a neighbour whose claim is already at most
  // `label` (every labelled vertex, and every vertex a smaller label has
  // claimed) needs no atomic: reading the claims first trades random
  // atomics for random loads, which the chip does about twice as fast
  uint32_t cl[kRB];
#pragma unroll
  for (int j = 0; j < kRB; ++j) cl[j] = ld_relaxed(&P.claim[nb[j]]);
#pragma unroll
  for (int j = 0; j < kRB; ++j)
    if (cl[j] > label) atomicMin(&P.claim[nb[j]], label);
}

__device__ __forceinline__ void claim_row(const BfsParams& P, int32_t v, int4 info,
                                          uint32_t label) {
  for (int32_t k0 = info.x; k0 < info.y; k0 += kRB) {
    int32_t nb[kRB];
    load_batch(P.colidx, k0, info.y, v, nb);
    claim_batch(P, nb, label);
  }
}

// A placed child whose claims the work-group issues after placement: it goes
// to the work-group's LDS list (index = its label - list_base) when it fits,
// else it claims its neighbours at once.
__device__ __forceinline__ void defer_claims(const BfsParams& P, Shared& S, int32_t v, int4 inf,
                                             int32_t at, int32_t list_base) {
  const int32_t i = at - list_base;
  if (i >= 0 && i < kStageCap) {
    reinterpret_cast<int4*>(S.u.srec)[i] = make_int4(v, inf.x, inf.y, at);
  } else {
    claim_row(P, v, inf, static_cast<uint32_t>(at));
  }
}

// Children of parent p (vertex u, row [a, b)) ranked by (degree, id) among
// the siblings, for rows longer than a register batch.  One pass over the row
// collects the keys of up to four children in registers (placed by
// predicated selects, no indexed register access); they are ranked there and
// their records fetched together.  A parent with more children ranks each
// one against the whole row (place_many_children takes the parents for which
// that would be long).
__device__ __forceinline__ void place_long_row(const BfsParams& P, Shared& S, int32_t p, int32_t u,
                                               int32_t a, int32_t b, int32_t base, int32_t end,
                                               int32_t list_base, long long& my_m) {
  const uint32_t pl = static_cast<uint32_t>(p);
  constexpr int kKids = kLongKids;  // children ranked in registers
  uint64_t ck[kKids];  // their (degree, caller id) keys ...
  int32_t cv[kKids];   // ... and vertex numbers
#pragma unroll
  for (int i = 0; i < kKids; ++i) {
    ck[i] = kMaxKey;
    cv[i] = u;
  }
  int nc = 0;
  for (int32_t k0 = a; k0 < b; k0 += kRB) {
    int32_t nb[kRB];
    load_batch(P.colidx, k0, b, u, nb);
    uint32_t cl[kRB];
    int2 dw[kRB];  // (degree, caller id)
#pragma unroll
    for (int j = 0; j < kRB; ++j) cl[j] = ld_relaxed(&P.claim[nb[j]]);
#pragma unroll
    for (int j = 0; j < kRB; ++j) dw[j] = reinterpret_cast<const int2*>(P.vinfo + nb[j])[1];
#pragma unroll
    for (int j = 0; j < kRB; ++j) {
      const bool child = nb[j] != u && cl[j] == pl;
      const uint64_t kv = pack_key(dw[j].x, dw[j].y);
#pragma unroll
      for (int i = 0; i < kKids; ++i) {
        ck[i] = (child && i == nc) ? kv : ck[i];
        cv[i] = (child && i == nc) ? nb[j] : cv[i];
      }
      nc += child ? 1 : 0;
    }
  }
  if (nc <= kKids) {
    int4 inf[kKids];
#pragma unroll
    for (int i = 0; i < kKids; ++i) inf[i] = P.vinfo[cv[i]];
#pragma unroll
    for (int i = 0; i < kKids; ++i) {
      if (i >= nc) continue;
      int rank = 0;
#pragma unroll
      for (int x = 0; x < kKids; ++x) rank += ck[x] < ck[i] ? 1 : 0;
      const int32_t v = cv[i];
      const int32_t at = base + rank;
      if (at < end) st_rec(&P.qi[at], record(v, inf[i]));
      my_m += inf[i].z;
      defer_claims(P, S, v, inf[i], at, list_base);
    }
    return;
  }
  for (int32_t k0 = a; k0 < b; k0 += kRB) {
    int32_t nb[kRB];
    load_batch(P.colidx, k0, b, u, nb);
    uint32_t cl[kRB];
#pragma unroll
    for (int j = 0; j < kRB; ++j) cl[j] = ld_relaxed(&P.claim[nb[j]]);
#pragma unroll
    for (int j = 0; j < kRB; ++j) {
      if (!(nb[j] != u && cl[j] == pl)) continue;
      const int4 inf = P.vinfo[nb[j]];
      const uint64_t kv = pack_key(inf.z, inf.w);
      int rank = 0;
      for (int32_t k1 = a; k1 < b; k1 += kRB) {
        int32_t w[kRB];
        load_batch(P.colidx, k1, b, u, w);
        uint32_t cw[kRB];
        int2 dw[kRB];
#pragma unroll
        for (int i = 0; i < kRB; ++i) cw[i] = ld_relaxed(&P.claim[w[i]]);
#pragma unroll
        for (int i = 0; i < kRB; ++i) dw[i] = reinterpret_cast<const int2*>(P.vinfo + w[i])[1];
#pragma unroll
        for (int i = 0; i < kRB; ++i)
          rank += (w[i] != u && cw[i] == pl && pack_key(dw[i].x, dw[i].y) < kv) ? 1 : 0;
      }
      const int32_t at = base + rank;
      if (at < end) st_rec(&P.qi[at], record(nb[j], inf));
      my_m += inf.z;
      defer_claims(P, S, nb[j], inf, at, list_base);
    }
  }
}

// The children of parent p (label p, first child label `base`, c children)
// when there are more than kLongKids of them, placed by the whole
// work-group: the row is scanned in parallel for the neighbours that p
// claimed, their (degree, caller id) keys (distinct: the id is) are sorted
// ascending, and child i gets label base + i (SortPerm's order among
// siblings, Table I).  The keys sort in LDS (the asynchronous passes' row
// store, unused while labelling) up to kManyLds of them; more sort in place
// in the children's own record slots qi[base, base + c), 16 bytes each, of
// which the keys take the first half.  A bitonic network whose comparators
// all put the smaller key first (each merge starts with mirrored pairs)
// lets positions past c stand for keys above every other without storage.
// All threads of the work-group call it with the same arguments.
constexpr int kManyLds = static_cast<int>(sizeof(OwnRowStore) / sizeof(unsigned long long));

__device__ __forceinline__ void sort_keys_ascending(unsigned long long* a, int32_t len) {
  const int B = blockDim.x;
  int32_t pow2 = 1;
  while (pow2 < len) pow2 <<= 1;
  for (int32_t k = 2; k <= pow2; k <<= 1) {
    for (int32_t j = k >> 1; j > 0; j >>= 1) {
      for (int32_t i = threadIdx.x; i < pow2; i += B) {
        const int32_t q = j == (k >> 1) ? (i ^ (k - 1)) : (i ^ j);
        if (q > i && q < len) {
          const unsigned long long x = a[i], y = a[q];
          if (y < x) {
            a[i] = y;
            a[q] = x;
          }
        }
      }
      __syncthreads();
    }
  }
}

__device__ __forceinline__ void place_many_children(const BfsParams& P, Shared& S, int32_t p,
                                                    int32_t base, int32_t c, int32_t end,
                                                    int32_t list_base, long long& my_m) {
  const int B = blockDim.x;
  const int4 e = ld_rec(P, p);
  const int32_t u = e.x;
  const uint32_t pl = static_cast<uint32_t>(p);
  const bool in_lds = c <= kManyLds;
  // (the record slots are 16-byte aligned; the keys use their first 8c bytes)
  unsigned long long* keys = in_lds ? reinterpret_cast<unsigned long long*>(&S.orow)
                                    : reinterpret_cast<unsigned long long*>(P.qi + base);
  if (threadIdx.x == 0) S.mcnt = 0;
  __syncthreads();
  for (int32_t k = e.y + threadIdx.x; k < e.z; k += B) {
    const int32_t w = P.colidx[k];
    if (w == u || ld_relaxed(&P.claim[w]) != pl) continue;
    const int4 inf = P.vinfo[w];
    const int32_t at = atomicAdd(&S.mcnt, 1);
    if (at < c) keys[at] = pack_key(inf.z, inf.w);
  }
  __syncthreads();
  // the count phase found c children, and their claims have not changed
  // since (this level's claims are issued after placement)
  const int32_t n = S.mcnt < c ? S.mcnt : c;
  sort_keys_ascending(keys, n);
  // child i's record goes to slot base + i.  In the scratch case that slot
  // holds keys 2i and 2i + 1, so the children go out from the last chunk
  // down, each chunk read before any of its slots is written: every key a
  // record covers then belongs to a chunk already read.
  const int32_t chunks = (n + B - 1) / B;
  for (int32_t ch = chunks - 1; ch >= 0; --ch) {
    const int32_t i = ch * B + threadIdx.x;
    unsigned long long kv = 0;
    if (i < n) kv = keys[i];
    __syncthreads();
    if (i < n) {
      const int32_t id = static_cast<int32_t>(kv & 0xffffffffu);
      const int32_t v = P.new_of_old != nullptr ? P.new_of_old[id] : id;
      const int4 inf = P.vinfo[v];
      const int32_t at = base + i;
      if (at < end) st_rec(&P.qi[at], record(v, inf));
      my_m += inf.z;
      defer_claims(P, S, v, inf, at, list_base);
    }
    __syncthreads();
  }
}

// Count the children of parent p over a long row (batch by batch).
__device__ __forceinline__ int count_long_row(const BfsParams& P, int32_t p, int32_t u, int32_t a,
                                              int32_t b) {
  const uint32_t pl = static_cast<uint32_t>(p);
  int c = 0;
  for (int32_t k0 = a; k0 < b; k0 += kRB) {
    int32_t nb[kRB];
    load_batch(P.colidx, k0, b, u, nb);
    uint32_t cl[kRB];
#pragma unroll
    for (int j = 0; j < kRB; ++j) cl[j] = ld_relaxed(&P.claim[nb[j]]);
#pragma unroll
    for (int j = 0; j < kRB; ++j) c += (nb[j] != u && cl[j] == pl) ? 1 : 0;
  }
  return c;
}

// Labelled levels in one work-group with the frontier in LDS (one parent per
// thread, rows of at most kRB entries).  (1) Every parent loads its row and
// the claim words and records of its neighbours; an unlabelled neighbour
// (claim word not below cur_b) is entered into the next level's LDS table
// and takes the smallest claiming label there (the (select2nd, min) product
// done with LDS atomics).  (2) The children of a parent are the neighbours
// whose table entry holds its label; they are ranked by (degree, id), placed
// after an LDS scan of the counts, and their claim words set to the parent's
// label (which marks them labelled).  On leaving, the new frontier issues its
// claims on global memory, as the team levels expect.  Returns false, having
// done nothing, when the frontier does not fit.
__device__ __forceinline__ bool lds_label_levels(const BfsParams& P, Team& t, Shared& S, int32_t end,
                                 int32_t& cur_b, int32_t& cur_e, int32_t& levels, bool& done,
                                 long long& my_m, int32_t stop_width) {
  NarrowLds& N = S.u.nw;
  const int B = blockDim.x;
  int32_t len = cur_e - cur_b;
  if (len > B || len > kNarrowCap) return false;
  const long long c0 = wall_clock64();
  long long mr = 0, rs = 0;
  for (int32_t i = threadIdx.x; i < len; i += B) {
    const int4 r = ld_rec(P, cur_b + i);
    lds_put(N, 0, i, r);
    mr = (r.z - r.y) > mr ? (r.z - r.y) : mr;
    rs += r.z - r.y;
  }
  mr = block_max_i64(mr, S.red);
  rs = block_sum_i64(rs, S.red);
  // one batch per row, and at most kHash / 2 row entries so that the next
  // level's table stays at most half full
  if (mr > kRB || rs > kHash / 2) return false;
  for (int i = threadIdx.x; i < 2 * kHash; i += B) {
    (&N.key[0][0])[i] = kEmpty;
    (&N.val[0][0])[i] = kUnclaimed;
  }
  if (threadIdx.x == 0)
    for (int i = 0; i < 3; ++i) {
      N.maxrow[i] = 0;
      N.rows[i] = 0;
    }
  __syncthreads();
  int lv = 0;
  int32_t nlev = 0;
  while (true) {
    int32_t* key_ins = N.key[lv & 1];
    uint32_t* val_ins = N.val[lv & 1];
    int32_t* key_clr = N.key[(lv + 1) & 1];
    uint32_t* val_clr = N.val[(lv + 1) & 1];
    const int mx = (lv + 1) % 3;
    if (threadIdx.x == 0) {
      N.maxrow[(lv + 2) % 3] = 0;
      N.rows[(lv + 2) % 3] = 0;
    }
    // (1) claims in LDS
    const bool active = static_cast<int32_t>(threadIdx.x) < len;
    const int32_t p = cur_b + static_cast<int32_t>(threadIdx.x);
    const uint32_t pl = static_cast<uint32_t>(p);
    int4 e = make_int4(0, 0, 0, 0);
    int32_t nb[kRB];
    int4 inf[kRB];
    int slot[kRB];
    unsigned unl = 0;
    if (active) {
      e = lds_rec(N, lv & 1, threadIdx.x);
      if (e.z > e.y) {
        load_batch(P.colidx, e.y, e.z, e.x, nb);
        uint32_t cl[kRB];
#pragma unroll
        for (int j = 0; j < kRB; ++j) cl[j] = ld_relaxed(&P.claim[nb[j]]);
#pragma unroll
        for (int j = 0; j < kRB; ++j) inf[j] = P.vinfo[nb[j]];
#pragma unroll
        for (int j = 0; j < kRB; ++j) {
          slot[j] = -1;
          if (nb[j] == e.x || cl[j] < static_cast<uint32_t>(cur_b)) continue;
          bool fresh = false;
          slot[j] = h_insert(key_ins, nb[j], &fresh);
          if (slot[j] < 0) continue;  // cannot happen: the table is at most half full
          atomicMin(&val_ins[slot[j]], pl);
          unl |= 1u << j;
        }
      }
    }
    // the other table was last used two levels ago
    for (int i = threadIdx.x; i < kHash; i += B) {
      key_clr[i] = kEmpty;
      val_clr[i] = kUnclaimed;
    }
    __syncthreads();
    // (2) children of p, their ranks and labels
    unsigned ch = 0;
#pragma unroll
    for (int j = 0; j < kRB; ++j)
      if ((unl >> j & 1u) && val_ins[slot[j]] == pl) ch |= 1u << j;
    const int c = __popc(ch);
    int total;
    const int ex = block_excl_scan(c, S.scan, &total);
    if (total == 0) {
      done = true;
      ++nlev;
      break;
    }
    if (c > 0) {
      uint64_t key[kRB];
#pragma unroll
      for (int j = 0; j < kRB; ++j) key[j] = (ch >> j & 1u) ? pack_key(inf[j].z, inf[j].w) : kMaxKey;
      const int32_t base = cur_e + ex;
#pragma unroll
      for (int j = 0; j < kRB; ++j) {
        if (!(ch >> j & 1u)) continue;
        int rank = 0;
#pragma unroll
        for (int i = 0; i < kRB; ++i) rank += key[i] < key[j] ? 1 : 0;
        const int32_t at = base + rank;
        const int4 r = record(nb[j], inf[j]);
        if (at < end) P.qi[at] = r;
        if (at - cur_e < kNarrowCap) lds_put(N, (lv + 1) & 1, at - cur_e, r);
        P.claim[nb[j]] = pl;
        my_m += inf[j].z;
        atomicMax(&N.maxrow[mx], inf[j].y - inf[j].x);
        atomicAdd(&N.rows[mx], inf[j].y - inf[j].x);
      }
    }
    // every 64th level: abort poll
    const bool poll = t.abort_flag != nullptr && (nlev & 63) == 63;
    if (poll && threadIdx.x == 0) {
      S.stop = ld_relaxed(&t.g->error) != 0 ? 1 : 0;
      if (!S.stop && abort_requested(t.abort_flag)) {
        flag_error(t.g, RCM_ERR_ABORTED, 23, t.comp, 0, levels);
        S.stop = 1;
      }
    }
    __syncthreads();
    if (poll && S.stop) {
      t.aborted = true;
      done = true;
      ++nlev;
      break;
    }
    ++nlev;
    cur_b = cur_e;
    cur_e += total;
    ++levels;
    ++lv;
    len = total;
    if (cur_e > end) {
      if (threadIdx.x == 0)
        flag_error(t.g, RCM_ERR_NOT_SYMMETRIC, 7, t.comp, 0, levels, cur_b, cur_e, end);
      done = true;
      break;
    }
    if (len > B || len > kNarrowCap || N.maxrow[mx] > kRB || N.rows[mx] > kHash / 2 ||
        len >= stop_width)
      break;
  }
  if (!done) {
    // the team levels expect the frontier's claims on the next level
    for (int32_t i = threadIdx.x; i < len; i += B) {
      const int4 r = ld_rec(P, cur_b + i);
      claim_row(P, r.x, make_int4(r.y, r.z, r.w, 0), static_cast<uint32_t>(cur_b + i));
    }
  }
  if (threadIdx.x == 0) {
    t.ctl->clk[14] += wall_clock64() - c0;
    t.ctl->clk[15] += nlev;
  }
  __syncthreads();
  return true;
}

// One labelled level with the global frontier, by the whole team (solo =
// false) or one work-group.  (B) each parent counts its children -- the
// neighbours whose claim equals its label -- keeping them in registers when
// its row fits one batch; barrier; (C) a scan of the counts in label order
// gives every parent its first child label, children are placed by their
// (degree, id) rank, and each placed child immediately claims its own
// neighbours for the next level; barrier.
__device__ __forceinline__ void global_label_level(const BfsParams& P, Team& t, Shared& S, int32_t end, bool solo,
                                   int32_t& cur_b, int32_t& cur_e, int32_t& levels, bool& done,
                                   long long& my_m, bool own = false) {
  const int B = blockDim.x;
  const int W = solo ? 1 : t.W;
  const int wid = solo ? 0 : t.wid;
  // own: this work-group's parents are the children it placed at the
  // previous level, a contiguous label range whose records are still in its
  // LDS list; else an even chunk of the level, read from qi
  const bool use_own = own && !solo && S.lown_ok != 0;
  int32_t lo, hi;
  if (use_own) {
    lo = S.lown_base;
    hi = lo + S.lown_len;
  } else {
    my_chunk(cur_b, cur_e, W, wid, lo, hi);
  }
  const long long ta = wall_clock64();
  const bool one_round = hi - lo <= B;
  bool captured = false;
  bool deferred = false;  // a parent on a row longer than kHeavyRow, counted below
  int c_mine = 0;
  int32_t cnb[kRB];
  int4 cinf[kRB];
  unsigned cmask = 0;
  int wg_total = 0;
  for (int32_t p = lo + threadIdx.x; p < hi; p += B) {
    int4 e;
    if (use_own) {
      const int4 c = reinterpret_cast<const int4*>(S.u.srec)[p - lo];
      e = make_int4(c.x, c.y, c.z, 0);
    } else {
      e = ld_rec(P, p);
    }
    const int32_t u = e.x;
    const uint32_t pl = static_cast<uint32_t>(p);
    int c;
    if (one_round && e.z - e.y <= kRB) {
      if (e.z > e.y) {
        if (use_own && p - lo < kRowCap) {
          // the row this parent loaded for its claims at the previous level
          const int32_t* kr = kept_row(S.u, p - lo);
#pragma unroll
          for (int j = 0; j < kRB; ++j) cnb[j] = kr[j] & 0x7fffffff;
        } else {
          load_batch(P.colidx, e.y, e.z, u, cnb);
        }
        uint32_t cl[kRB];
#pragma unroll
        for (int j = 0; j < kRB; ++j) cl[j] = ld_relaxed(&P.claim[cnb[j]]);
#pragma unroll
        for (int j = 0; j < kRB; ++j) cinf[j] = P.vinfo[cnb[j]];
#pragma unroll
        for (int j = 0; j < kRB; ++j) cmask |= (cnb[j] != u && cl[j] == pl ? 1u : 0u) << j;
      }
      captured = true;
      c = __popc(cmask);
    } else {
      int h = kHeavyCap;
      if (e.z - e.y > kHeavyRow) h = atomicAdd(&S.nheavy, 1);
      if (h < kHeavyCap) {
        // a long row: its children are counted by the whole work-group below
        S.heavy[h] = make_int4(p, u, e.y, e.z);
        deferred = true;
        c = 0;
      } else {
        c = count_long_row(P, p, u, e.y, e.z);
        P.tmp[p] = c;
      }
    }
    c_mine = c;
    wg_total += c;
  }
  // the count's block sum also says whether any parent was deferred, so that
  // a level without such a row pays no extra barrier
  long long tot = block_sum_i64(wg_total + (deferred ? (1ll << 40) : 0ll), S.red);
  if (tot >> 40) {
    tot &= (1ll << 40) - 1;
    const int nh = S.nheavy < kHeavyCap ? S.nheavy : kHeavyCap;
    for (int h = 0; h < nh; ++h) {
      const int4 hv = S.heavy[h];
      const uint32_t pl = static_cast<uint32_t>(hv.x);
      long long mine = 0;
      for (int32_t k = hv.z + static_cast<int32_t>(threadIdx.x); k < hv.w; k += B) {
        const int32_t w = P.colidx[k];
        mine += (w != hv.y && ld_relaxed(&P.claim[w]) == pl) ? 1 : 0;
      }
      const long long cnt = block_sum_i64(mine, S.red);
      tot += cnt;
      if (threadIdx.x == 0) P.tmp[hv.x] = static_cast<int32_t>(cnt);
      if (one_round && hv.x - lo == static_cast<int32_t>(threadIdx.x)) c_mine = static_cast<int>(cnt);
    }
    __syncthreads();
    if (threadIdx.x == 0) S.nheavy = 0;
  }
  const long long t1 = wall_clock64();
  // A work-group whose children all sit in registers (every parent's row is
  // one batch, one parent per thread) and fit its LDS list orders them
  // before the barrier has completed: their order within the work-group's
  // list, their records and the rows they claim from need nothing from the
  // other work-groups, only their labels (the level's base plus the counts
  // of the work-groups before) do.  So it arrives, ranks its children into
  // the list, loads their rows into LDS while the others arrive, and then
  // waits; afterwards it writes the records at their labels and claims.
  const bool early = !solo && one_round && tot <= kStageCap &&
                     __syncthreads_and(captured || c_mine == 0) != 0;
  if (early) {
    slot_arrive(t, S, static_cast<uint32_t>(tot), false);
    int rtot;
    const int c = captured ? c_mine : 0;
    const int ex = block_excl_scan(c, S.scan, &rtot);
    if (c > 0) {
      uint64_t key[kRB];
#pragma unroll
      for (int j = 0; j < kRB; ++j)
        key[j] = (cmask >> j & 1u) ? pack_key(cinf[j].z, cinf[j].w) : kMaxKey;
#pragma unroll
      for (int j = 0; j < kRB; ++j) {
        if (!(cmask >> j & 1u)) continue;
        int rank = 0;
#pragma unroll
        for (int i = 0; i < kRB; ++i) rank += key[i] < key[j] ? 1 : 0;
        reinterpret_cast<int4*>(S.u.srec)[ex + rank] = record(cnb[j], cinf[j]);
        my_m += cinf[j].z;
      }
    }
    __syncthreads();
    // waves 1.. load the rows and read their claims while wave 0 waits for
    // the other work-groups.  Claims below this level's first label (cur_e)
    // are final for the children, whose labels are all at least cur_e;
    // every other claim (unclaimed, or one a work-group that already passed
    // this barrier has just made) may still need the child's atomic.  So the
    // flag does not depend on the child's label; it goes into bit 31 of the
    // kept row entry (vertex ids are below 2^31).
    const int32_t len = static_cast<int32_t>(tot);
    if (threadIdx.x >= 64) {
      for (int32_t i = threadIdx.x - 64; i < len && i < kRowCap; i += B - 64) {
        const int4 r = reinterpret_cast<const int4*>(S.u.srec)[i];
        if (r.z - r.y > kRB) continue;
        int32_t nb[kRB];
        if (r.z > r.y) {
          load_batch(P.colidx, r.y, r.z, r.x, nb);
        } else {
#pragma unroll
          for (int j = 0; j < kRB; ++j) nb[j] = r.x;
        }
        uint32_t cl[kRB];
#pragma unroll
        for (int j = 0; j < kRB; ++j) cl[j] = ld_relaxed(&P.claim[nb[j]]);
        int32_t* kr = kept_row(S.u, i);
#pragma unroll
        for (int j = 0; j < kRB; ++j)
          kr[j] = nb[j] | (cl[j] >= static_cast<uint32_t>(cur_e) && nb[j] != r.x
                               ? int32_t(0x80000000u) : 0);
      }
    }
    slot_wait(t, S);
    if (t.aborted) return;
    const long long t2 = wall_clock64();
    const int32_t total = S.wtot;
    if (total == 0) {
      done = true;
      return;
    }
    // (A) every listed child gets its record at its label and claims the
    // neighbours found unclaimed (rows past the kept ones claim from memory)
    const int32_t list_base = cur_e + S.wpre;
    for (int32_t i = threadIdx.x; i < len; i += B) {
      const int4 r = reinterpret_cast<const int4*>(S.u.srec)[i];
      const int32_t at = list_base + i;
      if (at < end) st_rec(&P.qi[at], r);
      if (i < kRowCap && r.z - r.y <= kRB) {
        const int32_t* kr = kept_row(S.u, i);
#pragma unroll
        for (int j = 0; j < kRB; ++j)
          if (kr[j] < 0) atomicMin(&P.claim[kr[j] & 0x7fffffff], static_cast<uint32_t>(at));
      } else {
        claim_row(P, r.x, make_int4(r.y, r.z, 0, 0), static_cast<uint32_t>(at));
      }
    }
    const long long t3 = wall_clock64();
    if (threadIdx.x == 0) {
      S.lown_base = list_base;
      S.lown_len = S.wsum[wid];
      S.lown_ok = S.wmax <= kStageCap ? 1 : 0;
    }
    team_barrier(t, S, false);
    if (t.aborted) return;
    if (t.wid == 0 && threadIdx.x == 0) {
      const long long t4 = wall_clock64();
      t.ctl->clk[12] += t4 - ta;
      t.ctl->clk[13] += 1;
      t.ctl->clk[16] += t1 - ta;
      t.ctl->clk[17] += t2 - t1;
      t.ctl->clk[18] += t3 - t2;
      t.ctl->clk[19] += t4 - t3;
      t.ctl->clk[30] += 1;  // levels that took this path
    }
    cur_b = cur_e;
    cur_e += total;
    ++levels;
    if (cur_e > end) {
      if (threadIdx.x == 0)
        flag_error(t.g, RCM_ERR_NOT_SYMMETRIC, 3, t.comp, 0, levels, cur_b, cur_e, end);
      done = true;
    }
    return;
  }
  // the counts are all this barrier hands over: the count phase only read,
  // and placement touches other labels and claims than it read
  if (solo) {
    local_counts(S, static_cast<int32_t>(tot));
  } else {
    slot_exchange(t, S, static_cast<uint32_t>(tot), false);
  }
  if (t.aborted) return;
  const long long t2 = wall_clock64();
  const int32_t prefix = S.wpre;
  const int32_t total = S.wtot;
  if (total == 0) {
    done = true;
    return;
  }
  int32_t run = cur_e + prefix;
  // this work-group's children are the labels [run, run + S.wsum[wid]):
  // their records are collected in LDS and their claims issued after
  // placement, one child per thread
  const int32_t list_base = run;
  const int32_t list_len = S.wsum[wid] < kStageCap ? S.wsum[wid] : kStageCap;
  if (threadIdx.x == 0) S.nheavy = 0;
  for (int32_t r0 = lo; r0 < hi; r0 += B) {
    const int32_t p = r0 + threadIdx.x;
    const int c = p < hi ? (one_round ? c_mine : P.tmp[p]) : 0;
    int rtot;
    const int ex = block_excl_scan(c, S.scan, &rtot);
    if (c > 0) {
      const int32_t base = run + ex;
      if (captured) {
        uint64_t key[kRB];
#pragma unroll
        for (int j = 0; j < kRB; ++j)
          key[j] = (cmask >> j & 1u) ? pack_key(cinf[j].z, cinf[j].w) : kMaxKey;
        int32_t at[kRB];
#pragma unroll
        for (int j = 0; j < kRB; ++j) {
          int rank = 0;
#pragma unroll
          for (int i = 0; i < kRB; ++i) rank += key[i] < key[j] ? 1 : 0;
          at[j] = base + rank;
        }
#pragma unroll
        for (int j = 0; j < kRB; ++j) {
          if (!(cmask >> j & 1u)) continue;
          if (at[j] < end) st_rec(&P.qi[at[j]], record(cnb[j], cinf[j]));
          my_m += cinf[j].z;
        }
#pragma unroll
        for (int j = 0; j < kRB; ++j)
          if (cmask >> j & 1u) defer_claims(P, S, cnb[j], cinf[j], at[j], list_base);
      } else {
        const int4 e = ld_rec(P, p);
        const int64_t batches = (static_cast<int64_t>(e.z - e.y) + kRB - 1) / kRB;
        if (c > kLongKids && c * batches > kHeavyWork) {
          // many children on a long row: placed by the whole work-group below
          const int h = atomicAdd(&S.nheavy, 1);
          S.heavy[h] = make_int4(p, base, c, 0);
        } else {
          place_long_row(P, S, p, e.x, e.y, e.z, base, end, list_base, my_m);
        }
      }
    }
    __syncthreads();
    const int nh = S.nheavy;
    for (int h = 0; h < nh; ++h) {
      const int4 hv = S.heavy[h];
      place_many_children(P, S, hv.x, hv.y, hv.z, end, list_base, my_m);
    }
    __syncthreads();
    if (threadIdx.x == 0) S.nheavy = 0;
    run += rtot;
  }
  // (A) for the next level: every listed child claims its neighbours
  __syncthreads();
  const long long t3 = wall_clock64();
  for (int32_t i = threadIdx.x; i < list_len; i += B) {
    const int4 c = reinterpret_cast<const int4*>(S.u.srec)[i];
    if (i < kRowCap && c.z - c.y <= kRB) {
      // one batch: claim, and keep the row for the child's own count
      int32_t nb[kRB];
      if (c.z > c.y) {
        load_batch(P.colidx, c.y, c.z, c.x, nb);
        claim_batch(P, nb, static_cast<uint32_t>(c.w));
      } else {
#pragma unroll
        for (int j = 0; j < kRB; ++j) nb[j] = c.x;
      }
      int32_t* kr = kept_row(S.u, i);
#pragma unroll
      for (int j = 0; j < kRB; ++j) kr[j] = nb[j];
    } else {
      claim_row(P, c.x, make_int4(c.y, c.z, 0, 0), static_cast<uint32_t>(c.w));
    }
  }
  if (threadIdx.x == 0) {
    // the lists serve as the next level's parents when every work-group's
    // list holds all its children (the same decision in every work-group:
    // each has all the counts)
    S.lown_base = list_base;
    S.lown_len = S.wsum[wid];
    S.lown_ok = (!solo && S.wmax <= kStageCap) ? 1 : 0;
  }
  team_barrier(t, S, solo);
  if (t.aborted) return;
  if (t.wid == 0 && threadIdx.x == 0 && !solo) {
    const long long t4 = wall_clock64();
    t.ctl->clk[12] += t4 - ta;
    t.ctl->clk[13] += 1;
    t.ctl->clk[16] += t1 - ta;
    t.ctl->clk[17] += t2 - t1;
    t.ctl->clk[18] += t3 - t2;
    t.ctl->clk[19] += t4 - t3;
  }
  cur_b = cur_e;
  cur_e += total;
  ++levels;
  if (cur_e > end) {
    if (threadIdx.x == 0)
      flag_error(t.g, RCM_ERR_NOT_SYMMETRIC, 3, t.comp, 0, levels, cur_b, cur_e, end);
    done = true;
  }
}

// The labelled BFS of Algorithm 3 from `root`; labels are the positions in
// qi[o, end).  Returns the number of levels; msum = sum of degrees.  With
// want_lastkey, it also reports (in lastkey) the minimum (degree << 32 | id) over its last
// level, so that it can stand in for a level structure of the search.
__device__ __forceinline__ int32_t label_pass(const BfsParams& P, Team& t, Shared& S, int32_t o, int32_t end,
                              int32_t root, long long& msum, bool want_lastkey,
                              uint64_t& lastkey) {
  const long long clk0 = wall_clock64();
  const int B = blockDim.x;
  const int4 rinf = P.vinfo[root];
  if (t.wid == 0 && threadIdx.x == 0) {
    st_rec(&P.qi[o], record(root, rinf));
    __hip_atomic_store(&P.claim[root], static_cast<uint32_t>(o), __ATOMIC_RELAXED,
                       __HIP_MEMORY_SCOPE_AGENT);
    __hip_atomic_store(&t.ctl->msum, 0ll, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __hip_atomic_store(&t.ctl->lastkey, kMaxKey, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
  // the root's claims, spread over the whole team (its row may be long)
  for (int32_t k = rinf.x + t.wid * B + threadIdx.x; k < rinf.y; k += t.W * B) {
    const int32_t v = P.colidx[k];
    if (v != root) atomicMin(&P.claim[v], static_cast<uint32_t>(o));
  }
  team_barrier(t, S, false);
  if (t.aborted) return 0;
  int32_t cur_b = o, cur_e = o + 1, levels = 1;
  long long my_m = (t.wid == 0 && threadIdx.x == 0) ? rinf.z : 0;
  bool done = false;
  while (!done) {
    const bool narrow = t.W > 1 && (cur_e - cur_b) < P.narrow_cutoff;
    if (narrow && t.wid != 0) {
      narrow_wait(t, S);
      if (t.aborted) return 0;
      cur_b = S.state[0];
      cur_e = S.state[1];
      levels = S.state[2];
      done = S.state[3] != 0;
      continue;
    }
    if (narrow || t.W == 1) {
      const int32_t stop = narrow ? P.narrow_cutoff : 0x7fffffff;
      int skip = 0;
      while (!done && (cur_e - cur_b) < stop) {
        bool ran = false;
        if (skip == 0) {
          ran = lds_label_levels(P, t, S, end, cur_b, cur_e, levels, done, my_m, stop);
          if (!ran) skip = 8;
        } else {
          --skip;
        }
        if (!ran) global_label_level(P, t, S, end, true, cur_b, cur_e, levels, done, my_m);
        if (t.aborted) return 0;
      }
      if (narrow) {
        narrow_publish(t, cur_b, cur_e, levels, done);
      }
      continue;
    }
    // wide levels; every `rebalance` levels the parents are chunked evenly
    // again instead of taken from each work-group's own list
    for (int since = 0; !done && (cur_e - cur_b) >= P.narrow_cutoff; ++since) {
      global_label_level(P, t, S, end, false, cur_b, cur_e, levels, done, my_m,
                         since % P.rebalance != 0);
      if (t.aborted) return 0;
    }
  }
  if (cur_e != end) {
    if (threadIdx.x == 0 && t.wid == 0)
      flag_error(t.g, RCM_ERR_NOT_SYMMETRIC, 4, t.comp, 0, levels, cur_b, cur_e, end);
    t.aborted = true;
    return 0;
  }
  if (want_lastkey) {
    // the last level is qi[cur_b, cur_e): its records carry the degree
    int32_t lo, hi;
    my_chunk(cur_b, cur_e, t.W, t.wid, lo, hi);
    uint64_t k = kMaxKey;
    for (int32_t p = lo + threadIdx.x; p < hi; p += B) {
      const int4 r = ld_rec(P, p);
      const uint64_t kv = pack_key(r.w, P.relabelled ? P.vinfo[r.x].w : r.x);
      k = kv < k ? kv : k;
    }
    k = wave_min_u64(k);
    if ((threadIdx.x & 63) == 0 && k != kMaxKey) atomicMin(&t.ctl->lastkey, k);
  }
  const long long tot_m = block_sum_i64(my_m, S.red);
  if (threadIdx.x == 0 && tot_m != 0)
    __hip_atomic_fetch_add(&t.ctl->msum, tot_m, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  team_barrier(t, S, false);
  msum = __hip_atomic_load(&t.ctl->msum, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  if (want_lastkey)
    lastkey = __hip_atomic_load(&t.ctl->lastkey, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  if (t.wid == 0 && threadIdx.x == 0) {
    t.ctl->clk[1] += wall_clock64() - clk0;
    t.ctl->clk[3] += levels;
  }
  // msum is reset by the next component's setup, after several barriers
  return levels;
}

// The labelled BFS of a team, run by its first label_team work-groups (the
// labelled levels gain nothing from more, unlike the search's passes) with
// barrier slots of their own; the others sleep until it is done and then
// take its results from the team's control block.
__device__ __forceinline__ int32_t labelled_pass(const BfsParams& P, Team& t, Shared& S, int32_t o,
                                                 int32_t end, int32_t root, long long& msum,
                                                 bool want_lastkey, uint64_t& lastkey) {
  const int Wl = P.label_team < t.W ? P.label_team : t.W;
  if (Wl >= t.W) return label_pass(P, t, S, o, end, root, msum, want_lastkey, lastkey);
  t.ldone += 1;
  if (t.wid < Wl) {
    const int W0 = t.W;
    TeamSlots* const slots0 = t.slots;
    const uint32_t seq0 = t.seq;
    t.W = Wl;
    t.slots = t.sub_slots;
    t.seq = t.sub_seq;
    const int32_t levels = label_pass(P, t, S, o, end, root, msum, want_lastkey, lastkey);
    t.sub_seq = t.seq;
    t.W = W0;
    t.slots = slots0;
    t.seq = seq0;
    if (t.aborted) return 0;
    if (t.wid == 0 && threadIdx.x == 0) {
      // the sub-team's last barrier completed every record and claim;
      // msum and lastkey are already in the control block
      st_relaxed(&t.ctl->llevels, levels);
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
      __hip_atomic_fetch_add(&t.ctl->ldone, 1ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    return levels;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    const bool ok = wait_at_least(t, &t.ctl->ldone, t.ldone, true);
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    S.state[0] = ld_relaxed(&t.ctl->llevels);
    // narrow episodes of the sub-team happened without this work-group
    t.woke = ld_relaxed(&t.ctl->wake);
    S.flag = ok ? 0 : 1;
  }
  __syncthreads();
  t.aborted = S.flag != 0;
  if (t.aborted) return 0;
  msum = __hip_atomic_load(&t.ctl->msum, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  if (want_lastkey)
    lastkey = __hip_atomic_load(&t.ctl->lastkey, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  return S.state[0];
}

__device__ __forceinline__ void order_component(const BfsParams& P, Team& t, Shared& S, const CompTask& task) {
  const int32_t o = task.offset;
  // a task of unknown size (the component of vertex 0) learns it from the
  // first level structure, which visits the whole component
  int32_t size = task.size;
  int32_t end = size >= 0 ? o + size : P.n;
  // Algorithm 2: start at the component's lowest id
  int32_t ecc = 0;
  uint64_t lastkey = 0;
  int32_t nbfs = 1;
  int32_t found = end;
  // level orders' key anchor (the first pass of a component of unknown size
  // writes provisional keys, which later passes replace)
  t.anchor = task.anchor >= 0 ? task.anchor : (size >= 0 ? o + size - 1 : end - 1);
  // A level structure of the search: asynchronous for a team on a large
  // component (it sweeps the vertices of the component's graph once at its
  // end, so the component must be at least an eighth of them), else (or
  // when its ring of records would overflow) level-synchronous.  The tag
  // makes every (component, pass) distinct and grows with the pass.
  const int seg = P.nseg > 1 ? find_segment(P.seg_off, P.nseg, task.seed) : 0;
  const int32_t seg_b = P.nseg > 1 ? P.seg_off[seg] : 0;
  const int32_t seg_e = P.nseg > 1 ? P.seg_off[seg + 1] : P.n;
  const bool try_async =
      P.async_search != 0 && t.W > 1 && task.index < (1 << 25) &&
      (size < 0 || static_cast<long long>(size) * 8 >= static_cast<long long>(seg_e - seg_b));
  bool last_async = false;  // the last search pass ran asynchronously
  auto search_pass = [&](int32_t from, int32_t epoch, int parity, int32_t& e, uint64_t& lk,
                         bool find_end) {
    last_async = false;
    if (try_async && epoch < 64) {
      const uint32_t tag =
          (static_cast<uint32_t>(task.index + 1) << 6) | static_cast<uint32_t>(epoch);
      if (async_bfs_pass(P, t, S, o, end, from, tag, parity, seg_b, seg_e, e, lk, find_end,
                         found)) {
        last_async = true;
        return;
      }
      if (t.aborted) return;
    }
    bfs_pass(P, t, S, o, end, from, epoch, parity, e, lk, find_end, found);
  };
  // the vertex of a (degree, id) key: its caller id, renumbered when the
  // launch runs on a renumbered graph
  auto key_vertex = [&](uint64_t k) {
    const int32_t id = static_cast<int32_t>(k & 0xffffffffu);
    return P.new_of_old != nullptr ? P.new_of_old[id] : id;
  };
  if (P.resume && task.size >= 0 && task.index == 0) {
    // the first level structure ran in an earlier launch (see below)
    ecc = ld_relaxed(&P.gctl->p1_ecc);
    lastkey = ld_relaxed(&P.gctl->p1_lastkey);
  } else {
    search_pass(task.seed, 1, 0, ecc, lastkey, size < 0);
    if (t.aborted) return;
    if (size < 0) {
      size = found - o;
      end = found;
    }
    // a long component: stop here, so that the library renumbers it in
    // this structure's level order (its vertices then sit near their
    // neighbours in memory) and resumes on that copy
    if (P.relabel_levels > 0 && task.size < 0 && task.index == 0 && P.nseg == 1 &&
        P.label_mode == 0 && last_async && ecc + 1 >= P.relabel_levels) {
      if (t.wid == 0 && threadIdx.x == 0) {
        st_relaxed(&P.gctl->p1_ecc, ecc);
        st_relaxed(&P.gctl->p1_size, size);
        __hip_atomic_store(&P.gctl->p1_tag, (static_cast<uint32_t>(task.index + 1) << 6) | 1u,
                           __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __hip_atomic_store(&P.gctl->p1_lastkey, static_cast<unsigned long long>(lastkey),
                           __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        st_relaxed(&P.gctl->p1_stop, 1);
      }
      return;
    }
  }
  t.anchor = task.anchor >= 0 ? task.anchor : o + size - 1;
  int32_t r = task.seed;
  int32_t nlvl = ecc - 1;
  long long m = 0;
  int32_t levels = 0;
  bool labelled = false;
  while (ecc > nlvl) {
    nlvl = ecc;
    const int32_t v = key_vertex(lastkey);  // min degree, last level
    ++nbfs;
    r = v;
    if (P.pp_variant == 0 && nbfs >= 3 && P.label_mode == 0) {
      // Algorithm 2 returns the root of its last search and Algorithm 3
      // starts there, so from the third search on the search is run as the
      // labelled BFS itself: if the eccentricity does not grow, the search
      // ends and the labelling is already done; otherwise the claims of the
      // component are cleared and the search goes on.
      if (labelled) {
        for (int32_t i = t.wid * blockDim.x + threadIdx.x; i < size; i += t.W * blockDim.x)
          __hip_atomic_store(&P.claim[ld_rec(P, o + i).x], kUnclaimed, __ATOMIC_RELAXED,
                             __HIP_MEMORY_SCOPE_AGENT);
        team_barrier(t, S, false);
        if (t.aborted) return;
      }
      levels = labelled_pass(P, t, S, o, end, v, m, true, lastkey);
      if (t.aborted) return;
      ecc = levels - 1;
      labelled = true;
    } else {
      search_pass(v, nbfs, (nbfs - 1) & 1, ecc, lastkey, false);
      if (t.aborted) return;
    }
  }
  const int32_t root = P.pp_variant == 1 ? key_vertex(lastkey) : r;
  // reversal: Cuthill-McKee label t of this component goes to anchor - t
  const int32_t anchor = task.anchor >= 0 ? task.anchor : o + size - 1;
  if (P.label_mode != 0) {
    // level order: the levels come from a level structure rooted at `root`,
    // the search's last one or, for Algorithm 4's pick, one more
    if (P.pp_variant == 1) {
      uint64_t k2 = 0;
      search_pass(root, nbfs + 1, nbfs & 1, ecc, k2, false);
      if (t.aborted) return;
    }
    // every vertex now holds its level and block start; the host sorts
    levels = ecc + 1;
    m = t.pm;
  } else if (!labelled) {
    uint64_t unused_key = 0;
    levels = labelled_pass(P, t, S, o, end, root, m, false, unused_key);
    if (t.aborted) return;
  }
  if (t.wid == 0 && threadIdx.x == 0) {
    CompResult* res = P.results + task.index;
    res->root = P.relabelled ? P.vinfo[root].w : root;
    res->nbfs = nbfs;
    res->levels = levels;
    res->size = size;
    res->m = m;
  }
  if (P.label_mode != 0) return;  // perm is written by the sort
  const int32_t nthreads = t.W * blockDim.x;
  for (int32_t i = t.wid * blockDim.x + threadIdx.x; i < size; i += nthreads) {
    const int32_t x = ld_rec(P, o + i).x;
    const int32_t v = P.relabelled && x >= 0 && x < P.n ? P.vinfo[x].w : x;
    const int32_t pos = anchor - i;
    P.perm[pos] = v;
    if (v >= 0 && v < P.n) P.iperm[v] = pos;
  }
}

// Blocks [0, big_blocks) form teams of team_size work-groups that take large
// components from a queue (largest first); every other block, and the team
// blocks once that queue is empty, orders small components alone, also
// largest first.
__device__ __forceinline__ void order_main(const BfsParams& P) {
  __shared__ Shared S;
  Team t;
  t.g = P.gctl;
  t.slots = nullptr;
  t.seq = 0;
  t.sub_slots = nullptr;
  t.sub_seq = 0;
  t.ldone = 0;
  t.woke = 0;
  if (threadIdx.x == 0) {
    S.lown_ok = 0;
    S.nheavy = 0;
  }
  t.aborted = false;
  t.abort_flag = P.abort_flag;
  t.shuffle = P.shuffle;
  t.polls = 0;
  t.comp = 0;
  if (static_cast<int32_t>(blockIdx.x) < P.big_blocks) {
    // shuffle mode: which work-group plays which team member
    const int32_t b = shuffle_index(static_cast<int32_t>(blockIdx.x), P.big_blocks, P.shuffle);
    t.W = P.team_size;
    t.wid = b % P.team_size;
    t.ctl = P.teams + b / P.team_size;
    t.slots = P.slots + b / P.team_size;
    t.sub_slots = P.sub_slots + b / P.team_size;
    while (true) {
      if (t.wid == 0 && threadIdx.x == 0) {
        int32_t ti = atomicAdd(&P.queues[0], 1);
        // stop at a task boundary once the launch has an error or the
        // caller asks for an abort
        if (t.abort_flag != nullptr) {
          if (ld_relaxed(&t.g->error) != 0) {
            ti = -1;
          } else if (abort_requested(t.abort_flag)) {
            flag_error(t.g, RCM_ERR_ABORTED, 24);
            ti = -1;
          }
        }
        st_relaxed(&t.ctl->task, ti);
      }
      team_barrier(t, S, false);
      if (t.aborted) return;
      const int32_t ti = ld_relaxed(&t.ctl->task);
      if (ti < 0) return;
      if (ti >= P.n_big) break;
      const CompTask task = P.big_tasks[shuffle_index(ti, P.n_big, P.shuffle)];
      t.comp = task.index;
      order_component(P, t, S, task);
      if (t.aborted) return;
    }
  }
  if (P.ntasks <= 0) return;
  t.W = 1;
  t.wid = 0;
  t.ctl = P.small_teams + blockIdx.x;
  t.woke = 0;
  // the small list first, then whatever the teams have not taken yet of
  // the large one
  uint32_t fetched = 0;
  for (int q = 1; q >= 0; --q) {
    const CompTask* list = q == 1 ? P.tasks : P.big_tasks;
    const int32_t count = q == 1 ? P.ntasks : P.n_big;
    while (true) {
      shuffle_delay(P.shuffle, blockIdx.x, fetched);
      if (threadIdx.x == 0) {
        int32_t ti = atomicAdd(&P.queues[q], 1);
        // abort polls: the error word at every task, the caller's flag at
        // every 16th
        if (t.abort_flag != nullptr) {
          if (ld_relaxed(&t.g->error) != 0) {
            ti = -1;
          } else if ((fetched & 15u) == 0 && abort_requested(t.abort_flag)) {
            flag_error(t.g, RCM_ERR_ABORTED, 25);
            ti = -1;
          }
        }
        S.task = ti;
      }
      ++fetched;
      __syncthreads();
      const int32_t ti = S.task;
      __syncthreads();
      if (ti < 0) return;
      if (ti >= count) break;
      const CompTask task = list[shuffle_index(ti, count, q == 1 ? mix32(P.shuffle) : P.shuffle)];
      t.comp = task.index;
      order_component(P, t, S, task);
      if (t.aborted) return;
    }
  }
}

// Two instances of the same kernel, one per work-group size.  Bounded at
// 256 threads, a wave may use all 512 registers of a lane (256 vector and
// 256 accumulator registers) and the kernel compiles without any scratch
// spill; bounded at 512 it gets 256 and spills (about 170 vector registers
// to scratch).  On the 128^3 grid both take the same time (the labelled
// pass is faster without the spills, the asynchronous search slightly
// slower), so 256-thread work-groups, the default, run the spill-free
// instance, and 512-thread ones the other (on the CSR only).
__global__ void __launch_bounds__(256) k_order(BfsParams P) {
  order_main(P);
}

__global__ void __launch_bounds__(512) k_order_wide(BfsParams P) {
  // the fixed-stride row path holds a row per neighbour in registers, which
  // this instance would spill
  BfsParams Q = P;
  Q.ell = nullptr;
  order_main(Q);
}

const void* order_kernel(int32_t threads) {
  return threads > 256 ? reinterpret_cast<const void*>(k_order_wide)
                       : reinterpret_cast<const void*>(k_order);
}

// Cooperative launches of this library in one process never overlap: each
// is sized to what the device holds at once, and two of them resident side
// by side could each hold part of the other's team slots and wait forever.
std::mutex g_coop_mutex;

}  // namespace

int max_team_blocks(int32_t threads) {
  int per_cu = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, order_kernel(threads), threads, 0) !=
      hipSuccess)
    return 0;
  int dev = 0;
  (void)hipGetDevice(&dev);
  int cus = 0;
  (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
  return per_cu * cus;
}

hipError_t launch_order(const BfsParams& p, int32_t blocks, int32_t threads, hipStream_t s) {
  if (blocks <= 0 || (p.n_big <= 0 && p.ntasks <= 0)) return hipSuccess;
  if (threads != 256 && threads != 512) return hipErrorInvalidValue;
  BfsParams q = p;
  if (q.big_blocks > 0 && q.team_size > 1) {
    // held until the kernel has finished, so that another thread's
    // cooperative launch (a second stream of the serving engine, say) cannot
    // take part of the device while this one's teams wait for each other
    std::lock_guard<std::mutex> lk(g_coop_mutex);
    void* args[] = {&q};
    hipError_t e = hipLaunchCooperativeKernel(order_kernel(threads), dim3(blocks), dim3(threads),
                                              args, 0, s);
    if (e != hipSuccess) return e;
    return hipStreamSynchronize(s);
  }
  if (threads > 256)
    k_order_wide<<<blocks, threads, 0, s>>>(q);
  else
    k_order<<<blocks, threads, 0, s>>>(q);
  return hipGetLastError();
}

}  // namespace rcm
