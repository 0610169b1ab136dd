// The ordering itself: for each connected component, the pseudo-peripheral
// search (Algorithm 2: repeated breadth-first searches, each returning its
// eccentricity and the minimum-(degree, id) vertex of its last level) and
// the labelled level-synchronous BFS of Algorithm 3, then the reversal.
//
// One persistent kernel does all of it.  A "team" of W work-groups owns one
// component at a time and walks its levels; between levels the team meets at
// a barrier (a monotone arrival counter with device-scope release/acquire
// fences; for W = 1 the barrier is just __syncthreads).  Two launch shapes:
//   - large components: one team of W co-resident work-groups (cooperative
//     launch), default W = 8 so the team spans the 8 XCDs once;
//   - small components: many single-work-group teams pulling components from
//     an atomic queue.
//
// Level step of the labelled BFS (Algorithm 3), for the frontier
// L_cur = q[cur_b, cur_e) whose labels are exactly the positions p:
//   A. SpMSpV over (select2nd, min): for every edge (u, v) with u = q[p] and
//      v unlabelled, claim[v] = min(claim[v], p) (an atomic min; claim[] of
//      already labelled vertices holds labels < cur_b <= p, so the min leaves
//      them alone -- this is the Select(R == -1) step).
//   B. The children of p are the neighbours v with claim[v] == p.  Each
//      parent counts them.
//   C. An exclusive scan of the counts over the level (in label order) gives
//      each parent's first child label; a child's rank among its siblings is
//      its rank by (degree, id).  Parent label first, then degree, then id:
//      exactly SortPerm's lexicographic (parent label, degree, id) order
//      (Table I), without sorting the whole level.
// Unlabelled BFS (Algorithm 2's level structures): vertices are stamped with
// the pass number (no reset between passes) and appended to the next level
// through an LDS stage and one global atomic per work-group.

#include "rcm_common.hpp"

namespace rcm {

namespace {

constexpr int kStageCap = 2048;

struct Team {
  TeamCtl* ctl;
  GlobalCtl* g;
  int W;
  int wid;
  unsigned long long nbar;  // barrier arrivals expected so far (thread 0 only)
  bool aborted;
};

// Record the first error of the launch (RCM_ERR_ABORTED for a wait that timed
// out, RCM_ERR_NOT_SYMMETRIC when a traversal leaves its component's block,
// which only an asymmetric pattern can cause).
__device__ __forceinline__ void flag_error(GlobalCtl* g, int code) {
  int32_t expected = 0;
  __hip_atomic_compare_exchange_strong(&g->error, &expected, static_cast<int32_t>(code),
                                       __ATOMIC_RELAXED, __ATOMIC_RELAXED,
                                       __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ void team_barrier(Team& t, int* s_flag) {
  if (t.W == 1) {
    __syncthreads();
    return;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    t.nbar += static_cast<unsigned long long>(t.W);
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    __hip_atomic_fetch_add(&t.ctl->bar, 1ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    int ab = 0;
    long spins = 0;
    const long long t0 = wall_clock64();
    while (ld_relaxed(&t.ctl->bar) < t.nbar) {
      if ((++spins & 1023) == 0) {
        if (ld_relaxed(&t.g->error) != 0) {
          ab = 1;
          break;
        }
        if (wall_clock64() - t0 > kWaitLimitTicks) {
          ab = 1;
          flag_error(t.g, RCM_ERR_ABORTED);
          break;
        }
      }
    }
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    *s_flag = ab;
  }
  __syncthreads();
  t.aborted = *s_flag != 0;
}

struct Shared {
  int32_t stage[kStageCap];
  int scan[17];
  long long red[16];
  int32_t cnt;
  int32_t base;
  unsigned long long key;
  int flag;
  int task;
  int32_t wsum[kMaxTeam];
};

// Split [b, e) into W contiguous chunks; chunk of work-group wid.
__device__ __forceinline__ void my_chunk(int32_t b, int32_t e, int W, int wid, int32_t& lo,
                                         int32_t& hi) {
  const int32_t len = e - b;
  const int32_t c = (len + W - 1) / W;
  lo = b + c * wid;
  hi = lo + c < e ? lo + c : e;
  if (lo > e) lo = e;
}

// One level structure (Section II-A) of the component whose label block
// starts at o, rooted at `root`.  Vertices are written level by level into
// q[o ...].  Returns the eccentricity of root and the minimum
// (degree << 32 | id) over the last level.
__device__ void bfs_pass(const BfsParams& P, Team& t, Shared& S, int32_t o, int32_t end,
                         int32_t root, int32_t epoch, int parity, int32_t& ecc,
                         uint64_t& lastkey) {
  int32_t* tail = t.ctl->tail + parity * 3;
  unsigned long long* minkey = t.ctl->minkey + parity * 3;
  if (t.wid == 0 && threadIdx.x == 0) {
    P.q[o] = root;
    P.visit[root] = epoch;
    for (int i = 0; i < 3; ++i) st_relaxed(tail + i, 0);
    __hip_atomic_store(minkey + 0, pack_key(P.deg[root], root), __ATOMIC_RELAXED,
                       __HIP_MEMORY_SCOPE_AGENT);
    __hip_atomic_store(minkey + 1, kMaxKey, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __hip_atomic_store(minkey + 2, kMaxKey, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
  team_barrier(t, &S.flag);
  if (t.aborted) return;
  int32_t cur_b = o, cur_e = o + 1, level = 0;
  const int B = blockDim.x;
  while (true) {
    const int l3 = level % 3;
    if (threadIdx.x == 0) {
      S.cnt = 0;
      S.key = kMaxKey;
    }
    __syncthreads();
    int32_t lo, hi;
    my_chunk(cur_b, cur_e, t.W, t.wid, lo, hi);
    uint64_t mykey = kMaxKey;
    for (int32_t p = lo + threadIdx.x; p < hi; p += B) {
      const int32_t u = P.q[p];
      const int32_t a = P.rowptr[u], b = P.rowptr[u + 1];
      for (int32_t k = a; k < b; ++k) {
        const int32_t v = P.colidx[k];
        if (P.visit[v] == epoch) continue;
        if (atomicExch(&P.visit[v], epoch) == epoch) continue;
        const uint64_t kv = pack_key(P.deg[v], v);
        mykey = kv < mykey ? kv : mykey;
        const int32_t idx = atomicAdd(&S.cnt, 1);
        if (idx < kStageCap) {
          S.stage[idx] = v;
        } else {
          const int32_t at = atomicAdd(tail + l3, 1);
          if (cur_e + at < end) P.q[cur_e + at] = v;
        }
      }
    }
    mykey = wave_min_u64(mykey);
    if ((threadIdx.x & 63) == 0 && mykey != kMaxKey) atomicMin(&S.key, mykey);
    __syncthreads();
    if (threadIdx.x == 0) {
      const int32_t ns = S.cnt < kStageCap ? S.cnt : kStageCap;
      S.base = ns > 0 ? atomicAdd(tail + l3, ns) : 0;
      if (S.key != kMaxKey) atomicMin(minkey + (level + 1) % 3, S.key);
      if (t.wid == 0) {
        // slots of the level after next; nobody reads them any more
        st_relaxed(tail + (level + 1) % 3, 0);
        __hip_atomic_store(minkey + (level + 2) % 3, kMaxKey, __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_AGENT);
      }
    }
    __syncthreads();
    {
      const int32_t ns = S.cnt < kStageCap ? S.cnt : kStageCap;
      for (int32_t i = threadIdx.x; i < ns; i += B)
        if (cur_e + S.base + i < end) P.q[cur_e + S.base + i] = S.stage[i];
    }
    team_barrier(t, &S.flag);
    if (t.aborted) return;
    const int32_t cnt = ld_relaxed(tail + l3);
    if (cnt == 0) {
      ecc = level;
      lastkey = ld_relaxed(minkey + l3);
      break;
    }
    cur_b = cur_e;
    cur_e += cnt;
    ++level;
    if (cur_e > end) {  // left the component: the pattern is not symmetric
      if (threadIdx.x == 0 && t.wid == 0) flag_error(t.g, RCM_ERR_NOT_SYMMETRIC);
      t.aborted = true;
      return;
    }
  }
  if (cur_e != end) {
    if (threadIdx.x == 0 && t.wid == 0) flag_error(t.g, RCM_ERR_NOT_SYMMETRIC);
    t.aborted = true;
    return;
  }
  // every work-group has read the counters before the next pass reuses them
  team_barrier(t, &S.flag);
}

// The labelled BFS of Algorithm 3 from `root`; labels are the positions in
// q[o, o + size).  Returns the number of levels; *msum = sum of degrees.
__device__ int32_t label_pass(const BfsParams& P, Team& t, Shared& S, int32_t o, int32_t end,
                              int32_t root, long long* msum) {
  if (t.wid == 0 && threadIdx.x == 0) {
    P.q[o] = root;
    __hip_atomic_store(&P.claim[root], static_cast<uint32_t>(o), __ATOMIC_RELAXED,
                       __HIP_MEMORY_SCOPE_AGENT);
    __hip_atomic_store(&t.ctl->msum, 0ll, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
  team_barrier(t, &S.flag);
  if (t.aborted) return 0;
  const int B = blockDim.x;
  int32_t cur_b = o, cur_e = o + 1, levels = 1;
  long long my_m = (t.wid == 0 && threadIdx.x == 0) ? P.deg[root] : 0;
  while (true) {
    int32_t lo, hi;
    my_chunk(cur_b, cur_e, t.W, t.wid, lo, hi);
    // A: (select2nd, min) SpMSpV of the frontier, restricted to unlabelled
    for (int32_t p = lo + threadIdx.x; p < hi; p += B) {
      const int32_t u = P.q[p];
      const uint32_t pl = static_cast<uint32_t>(p);
      for (int32_t k = P.rowptr[u]; k < P.rowptr[u + 1]; ++k) {
        const int32_t v = P.colidx[k];
        if (v != u && P.claim[v] > pl) atomicMin(&P.claim[v], pl);
      }
    }
    team_barrier(t, &S.flag);
    if (t.aborted) return 0;
    // B: children per parent
    int wg_total = 0;
    for (int32_t p = lo + threadIdx.x; p < hi; p += B) {
      const int32_t u = P.q[p];
      const uint32_t pl = static_cast<uint32_t>(p);
      int c = 0;
      for (int32_t k = P.rowptr[u]; k < P.rowptr[u + 1]; ++k) {
        const int32_t v = P.colidx[k];
        c += (v != u && P.claim[v] == pl);
      }
      P.tmp[p] = c;
      wg_total += c;
    }
    {
      const long long tot = block_sum_i64(wg_total, S.red);
      if (threadIdx.x == 0)
        st_relaxed(&t.ctl->wg_sum[t.wid], static_cast<int32_t>(tot));
    }
    team_barrier(t, &S.flag);
    if (t.aborted) return 0;
    if (threadIdx.x < t.W) S.wsum[threadIdx.x] = ld_relaxed(&t.ctl->wg_sum[threadIdx.x]);
    __syncthreads();
    int32_t prefix = 0, total = 0;
    for (int w = 0; w < t.W; ++w) {
      prefix += w < t.wid ? S.wsum[w] : 0;
      total += S.wsum[w];
    }
    if (total == 0) break;
    // C: labels = cur_e + (exclusive prefix of counts in label order) +
    //    rank by (degree, id) among siblings
    int32_t run = cur_e + prefix;
    for (int32_t r0 = lo; r0 < hi; r0 += B) {
      const int32_t p = r0 + threadIdx.x;
      const int c = p < hi ? P.tmp[p] : 0;
      int rtot;
      const int ex = block_excl_scan(c, S.scan, &rtot);
      if (c > 0) {
        const int32_t u = P.q[p];
        const uint32_t pl = static_cast<uint32_t>(p);
        const int32_t a = P.rowptr[u], b = P.rowptr[u + 1];
        const int32_t base = run + ex;
        for (int32_t k = a; k < b; ++k) {
          const int32_t v = P.colidx[k];
          if (v == u || P.claim[v] != pl) continue;
          const int32_t dv = P.deg[v];
          const uint64_t kv = pack_key(dv, v);
          int rank = 0;
          for (int32_t k2 = a; k2 < b; ++k2) {
            const int32_t w = P.colidx[k2];
            if (w == u || P.claim[w] != pl) continue;
            rank += pack_key(P.deg[w], w) < kv;
          }
          if (base + rank < end) P.q[base + rank] = v;
          my_m += dv;
        }
      }
      run += rtot;
    }
    team_barrier(t, &S.flag);
    if (t.aborted) return 0;
    cur_b = cur_e;
    cur_e += total;
    ++levels;
    if (cur_e > end) {
      if (threadIdx.x == 0 && t.wid == 0) flag_error(t.g, RCM_ERR_NOT_SYMMETRIC);
      t.aborted = true;
      return 0;
    }
  }
  if (cur_e != end) {
    if (threadIdx.x == 0 && t.wid == 0) flag_error(t.g, RCM_ERR_NOT_SYMMETRIC);
    t.aborted = true;
    return 0;
  }
  const long long tot_m = block_sum_i64(my_m, S.red);
  if (threadIdx.x == 0 && tot_m != 0)
    __hip_atomic_fetch_add(&t.ctl->msum, tot_m, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  team_barrier(t, &S.flag);
  *msum = __hip_atomic_load(&t.ctl->msum, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  // msum is reset by the next component's setup, after several barriers
  return levels;
}

__device__ void order_component(const BfsParams& P, Team& t, Shared& S, const CompTask& task) {
  const int32_t o = task.offset;
  // Algorithm 2: start at the component's lowest id
  int32_t ecc = 0;
  uint64_t lastkey = 0;
  int32_t nbfs = 1;
  const int32_t end = o + task.size;
  bfs_pass(P, t, S, o, end, task.seed, 1, 0, ecc, lastkey);
  if (t.aborted) return;
  int32_t r = task.seed;
  int32_t nlvl = ecc - 1;
  while (ecc > nlvl) {
    nlvl = ecc;
    const int32_t v = static_cast<int32_t>(lastkey & 0xffffffffu);  // min degree, last level
    ++nbfs;
    bfs_pass(P, t, S, o, end, v, nbfs, (nbfs - 1) & 1, ecc, lastkey);
    if (t.aborted) return;
    r = v;
  }
  const int32_t root = P.pp_variant == 1 ? static_cast<int32_t>(lastkey & 0xffffffffu) : r;
  long long m = 0;
  const int32_t levels = label_pass(P, t, S, o, end, root, &m);
  if (t.aborted) return;
  if (t.wid == 0 && threadIdx.x == 0) {
    CompResult* res = P.results + task.index;
    res->root = root;
    res->nbfs = nbfs;
    res->levels = levels;
    res->m = m;
  }
  // reversal: Cuthill-McKee label t of this component goes to anchor - t
  const int32_t nthreads = t.W * blockDim.x;
  for (int32_t i = t.wid * blockDim.x + threadIdx.x; i < task.size; i += nthreads) {
    const int32_t v = P.q[o + i];
    const int32_t pos = task.anchor - i;
    P.perm[pos] = v;
    if (v >= 0 && v < P.n) P.iperm[v] = pos;
  }
}

__global__ void __launch_bounds__(1024) k_order(BfsParams P) {
  __shared__ Shared S;
  Team t;
  t.W = P.team_size;
  t.wid = blockIdx.x % P.team_size;
  const int team = blockIdx.x / P.team_size;
  const int nteams = gridDim.x / P.team_size;
  t.ctl = P.teams + team;
  t.g = P.gctl;
  t.nbar = 0;
  t.aborted = false;
  for (int iter = 0;; ++iter) {
    int ti;
    if (P.use_queue) {
      if (threadIdx.x == 0) S.task = atomicAdd(&P.gctl->queue, 1);
      __syncthreads();
      ti = S.task;
      __syncthreads();
    } else {
      ti = team + iter * nteams;
    }
    if (ti >= P.ntasks) break;
    const CompTask task = P.tasks[ti];
    order_component(P, t, S, task);
    if (t.aborted) break;
  }
}

}  // namespace

int max_team_blocks(int32_t threads) {
  int per_cu = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_order, threads, 0) != hipSuccess)
    return 0;
  int dev = 0;
  (void)hipGetDevice(&dev);
  int cus = 0;
  (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
  return per_cu * cus;
}

hipError_t launch_order_small(const BfsParams& p, int32_t nblocks, int32_t threads,
                              hipStream_t s) {
  if (p.ntasks <= 0) return hipSuccess;
  BfsParams q = p;
  q.team_size = 1;
  q.use_queue = 1;
  k_order<<<nblocks, threads, 0, s>>>(q);
  return hipGetLastError();
}

hipError_t launch_order_big(const BfsParams& p, int32_t threads, hipStream_t s) {
  if (p.ntasks <= 0) return hipSuccess;
  BfsParams q = p;
  q.use_queue = 0;
  void* args[] = {&q};
  return hipLaunchCooperativeKernel(reinterpret_cast<const void*>(k_order), dim3(q.team_size),
                                    dim3(threads), args, 0, s);
}

}  // namespace rcm
