// The ordering of a whole small graph by one work-group with the graph in LDS
// (mode 0 picks it when the graph fits, mode 2 requires it).
//
// Everything of one call runs in this one launch: the CSR checks, degrees and
// the bandwidth / envelope size of the input order (Section II-A), the
// components in increasing lowest-id order (Section III-B), Algorithm 2's
// searches, Algorithm 3's labelled BFS with SortPerm's (parent label, degree,
// id) order, the reversal (Algorithm 1) and the statistics of the result.
// The team kernel pays one or two memory round trips and a barrier per
// level; here a level costs a handful of LDS round trips of one wave, which
// is what the many narrow levels of a small mesh need.
//
// The work-group is one wave of 64 lanes: every phase is wave-synchronous and
// __syncthreads() only orders the wave's LDS accesses.  Per graph the LDS
// holds rowptr (32-bit), the columns, and per vertex its label, degree and
// order entry (16-bit: only graphs of fewer than 65,535 vertices fit) plus a
// 32-bit word for claims and visited stamps (LDS atomics are 32-bit).  The same search/label fusion as the team kernel applies: from
// the third search on, the search pass is the labelled BFS itself.

#include "rcm_common.hpp"

namespace rcm {

namespace {

constexpr int kSW = 64;                     // lanes of the work-group
constexpr uint32_t kFree = 0xFFFFFFFFu;     // claim word: unclaimed, unstamped
constexpr uint32_t kStamp = 0x80000000u;    // visited stamps: kStamp | pass number
constexpr int kBatch = 8;                   // row entries handled together per lane

inline __host__ __device__ size_t al8(size_t x) { return (x + 7) & ~static_cast<size_t>(7); }

template <typename T>
inline __host__ __device__ size_t small_bytes(int64_t n, int64_t nnz) {
  const size_t N = static_cast<size_t>(n);
  return al8(4 * (N + 1)) + al8(sizeof(T) * static_cast<size_t>(nnz)) + 3 * al8(sizeof(T) * N) +
         al8(4 * N);
}

template <typename T>
struct Lds {
  uint32_t* rp;   // rowptr
  T* ci;          // columns
  T* lab;         // label (position) or none
  T* deg;         // off-diagonal entries of the row
  T* ord;         // BFS queue / Cuthill-McKee order of the component being ordered
  uint32_t* clm;  // claims (labelled BFS) and visited stamps (searches)
  T none;         // "no label"
};

struct Acc {                   // per-call totals, kept by every lane alike
  int32_t ncomp = 0, diameter = 0, nbfs = 0, nlevels = 0;
  unsigned long long edges = 0;
  int32_t err = 0;             // rcm_status of a failure
};

// Result of one level structure: eccentricity, minimum (degree << 32 | id)
// of the last level, vertices reached, sum of their degrees.
struct Pass {
  int32_t ecc;
  uint64_t key;
  int32_t count;
  long long msum;
};

__device__ __forceinline__ uint64_t wmin64(uint64_t x) { return wave_min_u64(x); }

// Exclusive prefix over the wave of a per-lane count below 2^bits, and the
// wave's total, from one ballot per bit (a shuffle scan costs several times
// more on this GPU).  Every lane of the wave must call it.
__device__ __forceinline__ int wave_prefix(uint32_t c, int bits, int* total) {
  int pre = 0, tot = 0;
  for (int b = 0; b < bits; ++b) {
    const unsigned long long m = __ballot((c >> b) & 1u);
    const int below = __builtin_amdgcn_mbcnt_hi(static_cast<uint32_t>(m >> 32),
                                                 __builtin_amdgcn_mbcnt_lo(static_cast<uint32_t>(m), 0));
    pre += below << b;
    tot += __popcll(m) << b;
  }
  *total = tot;
  return pre;
}

// Minimum (degree << 32 | id) over the vertices ord[b, e) (one level).
template <typename T>
__device__ __forceinline__ uint64_t level_min_key(const Lds<T>& L, int32_t b, int32_t e) {
  uint64_t k = kMaxKey;
  for (int32_t i = b + static_cast<int32_t>(threadIdx.x); i < e; i += kSW) {
    const uint32_t x = L.ord[i];
    const uint64_t kv = pack_key(static_cast<int32_t>(L.deg[x]), static_cast<int32_t>(x));
    k = kv < k ? kv : k;
  }
  return wmin64(k);
}

// Columns [k0, k0 + kBatch) of a row ending at b (lanes past the end get u).
template <typename T>
__device__ __forceinline__ void row_batch(const Lds<T>& L, uint32_t k0, uint32_t b, uint32_t u,
                                          uint32_t* nb) {
#pragma unroll
  for (int j = 0; j < kBatch; ++j) nb[j] = k0 + j < b ? static_cast<uint32_t>(L.ci[k0 + j]) : u;
}

// Unlabelled level structure from root over the component starting at
// position o (queue ord[o, ...)); stamp marks this pass's visits.  A vertex
// that already carries a label belongs to an ordered component: only an
// asymmetric pattern leads there (flagged, not entered).
template <typename T>
__device__ Pass search_pass(const Lds<T>& L, int32_t n, int32_t o, uint32_t root, uint32_t stamp,
                            int32_t* cnt, int32_t* asym) {
  const int tid = threadIdx.x;
  (void)cnt;
  if (tid == 0) {
    L.ord[o] = static_cast<T>(root);
    L.clm[root] = stamp;
  }
  __syncthreads();
  int32_t fb = o, fe = o + 1, ecc = 0;
  long long msum = tid == 0 ? static_cast<long long>(L.deg[root]) : 0;
  bool bad = false;
  while (true) {
    // the level ord[fb, fe), 64 vertices at a time; every lane runs every
    // step (lanes without a vertex or past their row carry their own
    // vertex, which is never new), so the wave can place its finds with
    // ballots instead of an atomic counter
    int32_t next = 0;
    for (int32_t q = fb; q < fe; q += kSW) {
      const int32_t i = q + tid;
      const bool act = i < fe;
      const uint32_t u = act ? static_cast<uint32_t>(L.ord[i]) : 0u;
      const uint32_t a = act ? L.rp[u] : 0u, b = act ? L.rp[u + 1] : 0u;
      for (uint32_t k0 = a; __any(k0 < b); k0 += kBatch) {
        uint32_t nb[kBatch];
        row_batch(L, k0, b, u, nb);
        // a vertex already stamped in this pass needs no exchange; of the
        // others, the lane whose exchange finds no stamp found it
        uint32_t cl[kBatch];
#pragma unroll
        for (int j = 0; j < kBatch; ++j) cl[j] = L.clm[nb[j]];
        unsigned mask = 0;
#pragma unroll
        for (int j = 0; j < kBatch; ++j) {
          if (nb[j] == u || cl[j] == stamp) continue;
          const T lb = L.lab[nb[j]];
          if (lb != L.none) {
            // a labelled vertex belongs to an ordered component: only an
            // asymmetric pattern leads there
            bad = true;
            continue;
          }
          if (atomicExch(&L.clm[nb[j]], stamp) != stamp) mask |= 1u << j;
        }
        int total;
        const int pre = wave_prefix(static_cast<uint32_t>(__popc(mask)), 4, &total);
        int32_t at = fe + next + pre;
#pragma unroll
        for (int j = 0; j < kBatch; ++j) {
          if (!(mask >> j & 1u)) continue;
          if (at < n) L.ord[at] = static_cast<T>(nb[j]);
          else bad = true;
          ++at;
          msum += static_cast<long long>(L.deg[nb[j]]);
        }
        next += total;
      }
    }
    __syncthreads();
    if (next == 0) break;
    fb = fe;
    fe += next;
    if (fe > n) {
      bad = true;
      fe = n;
      break;
    }
    ++ecc;
  }
  if (__any(bad)) *asym = 1;
  Pass r;
  r.ecc = ecc;
  r.key = level_min_key(L, fb, fe);
  r.count = fe - o;
  r.msum = wave_sum_i64(msum);
  return r;
}

// Children of parent p (vertex u, row [a, b), c children, first label base)
// for a parent with more children than the register ranking holds, placed
// by the whole wave: the lanes take the row 64 entries at a time and write
// the children, in row order, into their label range ord[base, base + c);
// then that range is sorted by (degree, id) in place, which is their rank
// among the siblings.  The sort is a bitonic network whose comparators all
// put the smaller key first (each merge starts with mirrored pairs), so
// positions past c stand for keys above every other without storage.  One
// wave's LDS operations are performed in issue order; the wavefront fence
// keeps the compiler to that order between the steps.  Every lane calls it
// with the same arguments.
template <typename T>
__device__ __forceinline__ uint64_t child_key(const Lds<T>& L, uint32_t x) {
  return pack_key(static_cast<int32_t>(L.deg[x]), static_cast<int32_t>(x));
}

template <typename T>
__device__ __forceinline__ void wave_place_children(const Lds<T>& L, uint32_t p, uint32_t u,
                                                    uint32_t a, uint32_t b, int32_t base,
                                                    int32_t n, int c, bool* bad) {
  const uint32_t lane = threadIdx.x;
  int32_t got = 0;
  for (uint32_t k0 = a; k0 < b; k0 += kSW) {
    const uint32_t k = k0 + lane;
    uint32_t x = 0;
    bool child = false;
    if (k < b) {
      x = L.ci[k];
      child = x != u && L.lab[x] == L.none && L.clm[x] == p;
    }
    const unsigned long long m = __ballot(child);
    const int below = __builtin_amdgcn_mbcnt_hi(static_cast<uint32_t>(m >> 32),
                                                __builtin_amdgcn_mbcnt_lo(static_cast<uint32_t>(m), 0));
    if (child) {
      const int32_t at = base + got + below;
      if (got + below < c && at < n) L.ord[at] = static_cast<T>(x);
      else *bad = true;
    }
    got += __popcll(m);
  }
  if (got != c) *bad = true;
  int32_t len = got < c ? got : c;
  if (base + len > n) len = n - base;
  if (len <= 1) return;
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  T* seg = L.ord + base;
  int32_t pow2 = 1;
  while (pow2 < len) pow2 <<= 1;
  for (int32_t k = 2; k <= pow2; k <<= 1) {
    for (int32_t j = k >> 1; j > 0; j >>= 1) {
      for (int32_t i = static_cast<int32_t>(lane); i < pow2; i += kSW) {
        const int32_t q = j == (k >> 1) ? (i ^ (k - 1)) : (i ^ j);
        if (q > i && q < len) {
          const uint32_t xi = seg[i], xq = seg[q];
          if (child_key(L, xq) < child_key(L, xi)) {
            seg[i] = static_cast<T>(xq);
            seg[q] = static_cast<T>(xi);
          }
        }
      }
      __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    }
  }
}

// Algorithm 3 from root: labels are positions ord[o, ...).  Per level: every
// parent claims its unlabelled neighbours with an LDS atomic minimum of its
// label (the (select2nd, min) product), then each parent counts the
// neighbours whose claim is its own label, a scan over the level in label
// order gives its first child label, and its children are ranked by
// (degree, id) -- SortPerm's (parent label, degree, id) order.  The claim
// words of the component's vertices must be kFree on entry.
template <typename T>
__device__ Pass label_pass(const Lds<T>& L, int32_t n, int32_t o, uint32_t root, int32_t* cnt,
                           int32_t* asym) {
  const int tid = threadIdx.x;
  if (tid == 0) {
    L.ord[o] = static_cast<T>(root);
    L.lab[root] = static_cast<T>(o);
    L.clm[root] = static_cast<uint32_t>(o);
  }
  __syncthreads();
  int32_t b = o, e = o + 1, levels = 1;
  uint64_t last = pack_key(static_cast<int32_t>(L.deg[root]), static_cast<int32_t>(root));
  long long msum = tid == 0 ? static_cast<long long>(L.deg[root]) : 0;
  bool bad = false;
  while (true) {
    // claims: every neighbour of every parent, at once.  A labelled vertex's
    // claim word already holds its parent's label, below every label of
    // this level, so the minimum leaves it alone (and so does u's own word
    // for the lanes past the row end)
    for (int32_t p = b + tid; p < e; p += kSW) {
      const uint32_t u = L.ord[p];
      const uint32_t a = L.rp[u], bb = L.rp[u + 1];
      for (uint32_t k0 = a; k0 < bb; k0 += kBatch) {
        uint32_t nb[kBatch];
        row_batch(L, k0, bb, u, nb);
        // read first: an atomic is only needed where the claim is larger
        uint32_t cl[kBatch];
#pragma unroll
        for (int j = 0; j < kBatch; ++j) cl[j] = L.clm[nb[j]];
#pragma unroll
        for (int j = 0; j < kBatch; ++j)
          if (cl[j] > static_cast<uint32_t>(p)) atomicMin(&L.clm[nb[j]], static_cast<uint32_t>(p));
      }
    }
    __syncthreads();
    // count, scan, place (parents in chunks of one per lane, in label order):
    // a parent's children are its unlabelled neighbours whose claim is its
    // label; up to kBatch of them (in a row of up to kBatch entries) are
    // ranked by (degree, id) from the words the count loaded
    int32_t placed = 0;
    for (int32_t q = b; q < e; q += kSW) {
      const int32_t p = q + tid;
      int c = 0;
      uint32_t u = 0, a = 0, bb = 0;
      uint64_t ck[kBatch];
#pragma unroll
      for (int i = 0; i < kBatch; ++i) ck[i] = kMaxKey;
      if (p < e) {
        u = L.ord[p];
        a = L.rp[u];
        bb = L.rp[u + 1];
        for (uint32_t k0 = a; k0 < bb; k0 += kBatch) {
          uint32_t nb[kBatch];
          row_batch(L, k0, bb, u, nb);
          T lb[kBatch], dg[kBatch];
          uint32_t cl[kBatch];
#pragma unroll
          for (int j = 0; j < kBatch; ++j) lb[j] = L.lab[nb[j]];
#pragma unroll
          for (int j = 0; j < kBatch; ++j) cl[j] = L.clm[nb[j]];
#pragma unroll
          for (int j = 0; j < kBatch; ++j) dg[j] = L.deg[nb[j]];
#pragma unroll
          for (int j = 0; j < kBatch; ++j) {
            // a label of an earlier component: only an asymmetric pattern
            if (nb[j] != u && lb[j] != L.none && static_cast<int32_t>(lb[j]) < o) bad = true;
            const bool child =
                nb[j] != u && lb[j] == L.none && cl[j] == static_cast<uint32_t>(p);
            const uint64_t kv =
                pack_key(static_cast<int32_t>(dg[j]), static_cast<int32_t>(nb[j]));
#pragma unroll
            for (int i = 0; i < kBatch; ++i) ck[i] = (child && i == c) ? kv : ck[i];
            c += child ? 1 : 0;
          }
        }
      }
      // a count above 15 (a long row) needs more bits of the prefix (a row
      // holds fewer than 2^17 entries here)
      int total;
      const int pre = wave_prefix(static_cast<uint32_t>(c), __any(c > 15) ? 17 : 4, &total);
      const int32_t base = e + placed + pre;
      if (c > 0 && c <= kBatch) {
#pragma unroll
        for (int i = 0; i < kBatch; ++i) {
          if (i >= c) continue;
          int rank = 0;
#pragma unroll
          for (int x = 0; x < kBatch; ++x) rank += ck[x] < ck[i] ? 1 : 0;
          const int32_t at = base + rank;
          if (at < n) L.ord[at] = static_cast<T>(ck[i] & 0xffffffffu);
          else bad = true;
        }
      }
      // the parents with more children: the wave places them one by one
      unsigned long long heavy = __ballot(c > kBatch);
      while (heavy != 0) {
        const int l = __ffsll(static_cast<long long>(heavy)) - 1;
        heavy &= heavy - 1;
        wave_place_children(L, static_cast<uint32_t>(__shfl(p, l)), static_cast<uint32_t>(__shfl(static_cast<int>(u), l)),
                            static_cast<uint32_t>(__shfl(static_cast<int>(a), l)),
                            static_cast<uint32_t>(__shfl(static_cast<int>(bb), l)), __shfl(base, l),
                            n, __shfl(c, l), &bad);
      }
      placed += total;
    }
    __syncthreads();
    if (placed == 0) break;
    if (e + placed > n) {
      bad = true;
      break;
    }
    // the new level's labels (which also marks them labelled)
    for (int32_t i = e + tid; i < e + placed; i += kSW) {
      const uint32_t x = L.ord[i];
      L.lab[x] = static_cast<T>(i);
      msum += static_cast<long long>(L.deg[x]);
    }
    __syncthreads();
    b = e;
    e += placed;
    ++levels;
  }
  last = level_min_key(L, b, e);
  (void)cnt;
  if (__any(bad)) *asym = 1;
  Pass r;
  r.ecc = levels - 1;
  r.key = last;
  r.count = e - o;
  r.msum = wave_sum_i64(msum);
  return r;
}

// The claim words of the component's vertices ord[o, o + size) back to kFree
// (the searches left stamps there; a labelled pass that served as a search
// left claims) and, when labels, their labels back to none.
template <typename T>
__device__ __forceinline__ void reset_component(const Lds<T>& L, int32_t o, int32_t size,
                                                bool labels) {
  for (int32_t i = o + threadIdx.x; i < o + size; i += kSW) {
    const uint32_t x = L.ord[i];
    L.clm[x] = kFree;
    if (labels) L.lab[x] = L.none;
  }
  __syncthreads();
}

// One graph: checks, statistics, every component, reversal, result.
template <typename T>
__device__ void order_graph(const SmallJob& J, const SmallOpts& O, char* smem) {
  const int tid = threadIdx.x;
  const int32_t n = J.n;
  // nnz < 0: not known to the host yet (rowptr[n])
  const int32_t nnz = J.nnz >= 0 ? J.nnz : J.rowptr[n];
  __shared__ int32_t cnt[2];
  __shared__ int32_t asym;
  __shared__ int32_t stop;
  SmallResult* R = J.res;
  if (tid == 0) R->nnz = nnz;
  if (nnz < 0) {
    if (tid == 0) R->status = RCM_ERR_BAD_CSR;
    return;
  }
  if (small_bytes<T>(n, nnz) > static_cast<size_t>(O.lds_bytes)) {
    if (tid == 0) R->status = kSmallDeclined;  // the graph does not fit: the host takes over
    return;
  }
  Lds<T> L;
  {
    char* p = smem;
    L.rp = reinterpret_cast<uint32_t*>(p);
    p += al8(4 * (static_cast<size_t>(n) + 1));
    L.ci = reinterpret_cast<T*>(p);
    p += al8(sizeof(T) * static_cast<size_t>(nnz));
    L.lab = reinterpret_cast<T*>(p);
    p += al8(sizeof(T) * static_cast<size_t>(n));
    L.deg = reinterpret_cast<T*>(p);
    p += al8(sizeof(T) * static_cast<size_t>(n));
    L.ord = reinterpret_cast<T*>(p);
    p += al8(sizeof(T) * static_cast<size_t>(n));
    L.clm = reinterpret_cast<uint32_t*>(p);
    L.none = static_cast<T>(~static_cast<T>(0));
  }
  long long tk[7];
  tk[0] = wall_clock64();
  // 1. rows and columns into LDS, with the structural checks.  One wave
  // issues kLoad independent loads per lane before it waits, so that a
  // graph of 20,000 entries costs a few memory round trips, not hundreds.
  bool bad = false;
  constexpr int kLoad = 16;
  for (int32_t i0 = 0; i0 <= n; i0 += kSW * kLoad) {
    int32_t r[kLoad];
#pragma unroll
    for (int j = 0; j < kLoad; ++j) {
      const int32_t i = i0 + j * kSW + tid;
      r[j] = i <= n ? J.rowptr[i] : 0;
    }
#pragma unroll
    for (int j = 0; j < kLoad; ++j) {
      const int32_t i = i0 + j * kSW + tid;
      if (i > n) continue;
      if (r[j] < 0 || r[j] > nnz || (i == 0 && r[j] != 0) || (i == n && r[j] != nnz)) bad = true;
      L.rp[i] = static_cast<uint32_t>(r[j] < 0 ? 0 : (r[j] > nnz ? nnz : r[j]));
    }
  }
  const bool al16 = (reinterpret_cast<uintptr_t>(J.colidx) & 15) == 0;
  if (al16) {
    const int4* c4 = reinterpret_cast<const int4*>(J.colidx);
    const int32_t q = nnz >> 2;  // whole 16-byte groups
    for (int32_t i0 = 0; i0 < q; i0 += kSW * kLoad) {
      int4 v[kLoad];
#pragma unroll
      for (int j = 0; j < kLoad; ++j) {
        const int32_t i = i0 + j * kSW + tid;
        v[j] = i < q ? c4[i] : make_int4(0, 0, 0, 0);
      }
#pragma unroll
      for (int j = 0; j < kLoad; ++j) {
        const int32_t i = i0 + j * kSW + tid;
        if (i >= q) continue;
        const int32_t c[4] = {v[j].x, v[j].y, v[j].z, v[j].w};
#pragma unroll
        for (int h = 0; h < 4; ++h) {
          if (c[h] < 0 || c[h] >= n) bad = true;
          L.ci[4 * i + h] = static_cast<T>(c[h]);
        }
      }
    }
    for (int32_t k = 4 * q + tid; k < nnz; k += kSW) {
      const int32_t c = J.colidx[k];
      if (c < 0 || c >= n) bad = true;
      L.ci[k] = static_cast<T>(c);
    }
  } else {
    for (int32_t k0 = 0; k0 < nnz; k0 += kSW * kLoad) {
      int32_t v[kLoad];
#pragma unroll
      for (int j = 0; j < kLoad; ++j) {
        const int32_t k = k0 + j * kSW + tid;
        v[j] = k < nnz ? J.colidx[k] : 0;
      }
#pragma unroll
      for (int j = 0; j < kLoad; ++j) {
        const int32_t k = k0 + j * kSW + tid;
        if (k >= nnz) continue;
        if (v[j] < 0 || v[j] >= n) bad = true;
        L.ci[k] = static_cast<T>(v[j]);
      }
    }
  }
  __syncthreads();
  // rowptr must not decrease (checked once every entry is in LDS)
  for (int32_t i = tid; i < n; i += kSW) bad |= L.rp[i + 1] < L.rp[i];
  if (__any(bad)) {
    if (tid == 0) R->status = RCM_ERR_BAD_CSR;
    return;
  }
  __syncthreads();
  tk[1] = wall_clock64();
  // 2. degrees, repeated columns, bandwidth and profile of the input order
  long long bw = 0, prof = 0;
  bool dup = false, longrows = false;
  for (int32_t i = tid; i < n; i += kSW) {
    const uint32_t a = L.rp[i], b = L.rp[i + 1];
    const uint32_t me = static_cast<uint32_t>(i);
    uint32_t self = 0, mn = me;
    if (b - a <= kBatch) {
      // the whole row in registers; lanes past its end hold distinct fillers
      uint32_t r[kBatch];
#pragma unroll
      for (int j = 0; j < kBatch; ++j)
        r[j] = a + j < b ? static_cast<uint32_t>(L.ci[a + j]) : 0x80000000u + j;
#pragma unroll
      for (int j = 0; j < kBatch; ++j) {
        if (a + j >= b) continue;
        self += r[j] == me ? 1u : 0u;
        mn = r[j] < mn ? r[j] : mn;
      }
#pragma unroll
      for (int j = 0; j < kBatch; ++j)
#pragma unroll
        for (int k = j + 1; k < kBatch; ++k) dup |= r[j] == r[k];
    } else {
      for (uint32_t k0 = a; k0 < b; k0 += kBatch) {
        uint32_t nb[kBatch];
        row_batch(L, k0, b, me, nb);
#pragma unroll
        for (int j = 0; j < kBatch; ++j) {
          if (k0 + j >= b) continue;
          self += nb[j] == me ? 1u : 0u;
          mn = nb[j] < mn ? nb[j] : mn;
        }
      }
      if (b - a <= 64) {
        for (uint32_t k = a + 1; k < b && !dup; ++k) {
          const uint32_t c = L.ci[k];
          for (uint32_t k2 = a; k2 < k; ++k2) dup |= static_cast<uint32_t>(L.ci[k2]) == c;
        }
      } else {
        longrows = true;
      }
    }
    L.deg[i] = static_cast<T>(b - a - (self > 0 ? 1 : 0));
    L.lab[i] = L.none;
    L.clm[i] = kFree;
    const long long beta = i - static_cast<long long>(mn);
    bw = beta > bw ? beta : bw;
    prof += beta;
  }
  // rows longer than 64 entries, one at a time by the whole wave: each
  // entry swaps the row's number into its column's claim word (all free
  // here), and finding that number there already means the column repeats.
  // The words go back to free afterwards.  (The columns are in range: the
  // load checked them.)
  if (__any(longrows)) {
    for (int32_t i0 = 0; i0 < n; i0 += kSW) {
      const int32_t i = i0 + tid;
      const bool lg = i < n && L.rp[i + 1] - L.rp[i] > 64;
      unsigned long long m = __ballot(lg);
      while (m) {
        const int w = __builtin_ctzll(m);
        m &= m - 1;
        const uint32_t row = static_cast<uint32_t>(i0 + w);
        const uint32_t a = L.rp[row], b = L.rp[row + 1];
        for (uint32_t k = a + tid; k < b; k += kSW)
          dup |= atomicExch(&L.clm[static_cast<uint32_t>(L.ci[k])], row) == row;
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
      }
    }
    for (int32_t i = tid; i < n; i += kSW) L.clm[i] = kFree;
  }
  if (__any(dup)) {
    if (tid == 0) R->status = RCM_ERR_BAD_CSR;
    return;
  }
  if (O.check_full) {
    // (i, c) present needs (c, i) present
    bool miss = false;
    for (int32_t i = tid; i < n; i += kSW) {
      for (uint32_t k = L.rp[i]; k < L.rp[i + 1]; ++k) {
        const uint32_t c = L.ci[k];
        bool found = false;
        for (uint32_t k2 = L.rp[c]; k2 < L.rp[c + 1] && !found; ++k2)
          found = static_cast<uint32_t>(L.ci[k2]) == static_cast<uint32_t>(i);
        miss |= !found;
      }
    }
    if (__any(miss)) {
      if (tid == 0) R->status = RCM_ERR_NOT_SYMMETRIC;
      return;
    }
  }
  bw = wave_max_i64(bw);
  prof = wave_sum_i64(prof);
  if (tid == 0) asym = 0;
  __syncthreads();
  tk[2] = wall_clock64();
  long long t_search = 0, t_label = 0, t_rev = 0;
  // 3. components in increasing lowest-id order
  Acc acc;
  uint32_t pass = 0;
  int32_t o = 0, s_from = 0;
  // abort polls: one PCIe read of the caller's flag whenever 4096 units of
  // work have passed since the last (a level walked is one unit, a
  // component begun 64), checked between passes
  uint32_t since_poll = 0;
  auto abort_poll = [&](uint32_t units) -> bool {
    if (O.abort_flag == nullptr) return false;
    since_poll += units;
    if (since_poll < 4096) return false;
    since_poll = 0;
    if (tid == 0) stop = abort_requested(O.abort_flag) ? 1 : 0;
    __syncthreads();
    const bool hit = stop != 0;
    __syncthreads();
    return hit;
  };
  while (o < n) {
    if (abort_poll(64)) {
      acc.err = RCM_ERR_ABORTED;
      break;
    }
    // the next unlabelled vertex: the next component's lowest id
    int32_t s = -1;
    while (s < 0 && s_from < n) {
      const int32_t i = s_from + tid;
      const unsigned long long m = __ballot(i < n && L.lab[i] == L.none);
      if (m) s = s_from + __builtin_ctzll(m);
      else s_from += kSW;
    }
    if (s < 0) {  // fewer vertices reached than expected: cannot happen
      acc.err = RCM_ERR_NOT_SYMMETRIC;
      break;
    }
    s_from = s + 1;
    int32_t size = 1, nbfs = 2, levels = 1;
    long long mc = 0;
    if (L.deg[s] == 0) {
      // an isolated vertex: its own component (two level structures, one level)
      if (tid == 0) {
        L.ord[o] = static_cast<T>(s);
        L.lab[s] = static_cast<T>(o);
      }
      __syncthreads();
    } else {
      const long long ts0 = wall_clock64();
      Pass r = search_pass(L, n, o, static_cast<uint32_t>(s), kStamp | ++pass, cnt, &asym);
      size = r.count;
      mc = r.msum;
      nbfs = 1;
      uint32_t root = static_cast<uint32_t>(s);
      int32_t nlvl = r.ecc - 1;
      bool labelled = false;
      bool aborted = false;
      __syncthreads();
      while (!asym && r.ecc > nlvl) {
        if (abort_poll(static_cast<uint32_t>(r.ecc) + 1u)) {
          aborted = true;
          break;
        }
        nlvl = r.ecc;
        const uint32_t v = static_cast<uint32_t>(r.key & 0xffffffffu);
        ++nbfs;
        root = v;
        if (O.pp_variant == 0 && nbfs >= 3) {
          // Algorithm 2 would return v if this search does not go deeper, and
          // Algorithm 3 starts there: run this search as the labelled BFS
          const long long tl0 = wall_clock64();
          reset_component(L, o, size, labelled);
          r = label_pass(L, n, o, v, cnt, &asym);
          labelled = true;
          t_label += wall_clock64() - tl0;
        } else {
          r = search_pass(L, n, o, v, kStamp | ++pass, cnt, &asym);
        }
        __syncthreads();
        if (r.count != size) asym = 1;
      }
      if (aborted) {
        acc.err = RCM_ERR_ABORTED;
        break;
      }
      if (O.pp_variant == 1) root = static_cast<uint32_t>(r.key & 0xffffffffu);
      t_search += wall_clock64() - ts0;
      if (!labelled && !asym) {
        const long long tl0 = wall_clock64();
        reset_component(L, o, size, false);
        r = label_pass(L, n, o, root, cnt, &asym);
        __syncthreads();
        if (r.count != size) asym = 1;
        t_label += wall_clock64() - tl0;
      }
      levels = r.ecc + 1;
      __syncthreads();
    }
    if (asym) {
      acc.err = RCM_ERR_NOT_SYMMETRIC;
      break;
    }
    // reversal: Cuthill-McKee label o + t goes to position anchor - t
    const long long tr0 = wall_clock64();
    const int32_t anchor = O.reverse_mode ? n - 1 - o : o + size - 1;
    for (int32_t t = tid; t < size; t += kSW) {
      const uint32_t x = L.ord[o + t];
      const int32_t at = anchor - t;
      J.perm[at] = static_cast<int32_t>(x) + J.id_off;
      if (J.iperm) J.iperm[x] = at + J.pos_off;
      L.lab[x] = static_cast<T>(at);  // final positions, for the statistics below
    }
    __syncthreads();
    t_rev += wall_clock64() - tr0;
    acc.ncomp += 1;
    acc.nbfs += nbfs;
    acc.nlevels += levels;
    acc.diameter = levels - 1 > acc.diameter ? levels - 1 : acc.diameter;
    acc.edges += static_cast<unsigned long long>(nbfs + 1) * static_cast<unsigned long long>(mc);
    o += size;
  }
  if (acc.err != 0) {
    if (tid == 0) R->status = acc.err;
    return;
  }
  // 4. bandwidth and profile of the result: positions are in lab
  tk[3] = wall_clock64();
  long long bw2 = 0, prof2 = 0;
  for (int32_t v = tid; v < n; v += kSW) {
    const int32_t k = static_cast<int32_t>(L.lab[v]);
    int32_t mn = k;
    const uint32_t a = L.rp[v], b = L.rp[v + 1];
    for (uint32_t k0 = a; k0 < b; k0 += kBatch) {
      uint32_t nb[kBatch];
      row_batch(L, k0, b, static_cast<uint32_t>(v), nb);
      T q[kBatch];
#pragma unroll
      for (int j = 0; j < kBatch; ++j) q[j] = L.lab[nb[j]];
#pragma unroll
      for (int j = 0; j < kBatch; ++j) mn = static_cast<int32_t>(q[j]) < mn ? static_cast<int32_t>(q[j]) : mn;
    }
    const long long beta = k - mn;
    bw2 = beta > bw2 ? beta : bw2;
    prof2 += beta;
  }
  bw2 = wave_max_i64(bw2);
  prof2 = wave_sum_i64(prof2);
  if (tid == 0) {
    R->bw_before = static_cast<unsigned long long>(bw);
    R->prof_before = static_cast<unsigned long long>(prof);
    R->bw_after = static_cast<unsigned long long>(bw2);
    R->prof_after = static_cast<unsigned long long>(prof2);
    R->edges = acc.edges;
    R->ncomp = acc.ncomp;
    R->diameter = acc.diameter;
    R->nbfs = acc.nbfs;
    R->nlevels = acc.nlevels;
    // the searches' time includes a labelled pass that served as a search
    R->ticks[0] = tk[1] - tk[0];
    R->ticks[1] = tk[2] - tk[1];
    R->ticks[2] = t_search;
    R->ticks[3] = t_label;
    R->ticks[4] = t_rev;
    R->ticks[5] = wall_clock64() - tk[3];
    R->status = RCM_OK;
  }
}

// One work-group per job; wide is the 32-bit variant (graphs of 65,535
// vertices or more).
// One work-group per job (jobs == nullptr: the single job passed by value).
// Per-vertex words are 16-bit: a graph of 65,535 vertices or more never fits
// one work-group's LDS anyway.
__global__ void __launch_bounds__(kSW) k_small_order(SmallJob single, const SmallJob* jobs,
                                                      int32_t njobs, SmallOpts opts) {
  // the dynamic LDS follows the kernel's static LDS; the alignment keeps
  // every array carved out of it aligned whatever that static part holds
  // (a 1-byte static flag once left it at byte 1, and misaligned 32-bit LDS
  // accesses fault)
  extern __shared__ __align__(16) char smem[];
  for (int32_t j = blockIdx.x; j < njobs; j += gridDim.x) {
    // shuffle mode: which work-group takes which graph
    const int32_t jj = shuffle_index(j, njobs, opts.shuffle);
    order_graph<uint16_t>(jobs ? jobs[jj] : single, opts, smem);
    __syncthreads();
  }
}

}  // namespace

size_t small_lds_bytes(int64_t n, int64_t nnz) {
  if (n <= 0) return 0;
  if (n >= 65535) return ~static_cast<size_t>(0);  // 16-bit words only
  return small_bytes<uint16_t>(n, nnz);
}

size_t small_lds_limit() {
  int dev = 0, v = 0;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess ||
      v <= 0)
    return 0;
  // the kernel's own static LDS (a few counters) comes out of the same budget
  return static_cast<size_t>(v) > 256 ? static_cast<size_t>(v) - 256 : 0;
}

hipError_t launch_small_order(const SmallJob& single, const SmallJob* jobs_dev, int32_t njobs,
                              const SmallOpts& opts, hipStream_t s) {
  if (njobs <= 0) return hipSuccess;
  const int blocks = njobs < 65536 ? njobs : 65536;
  (void)hipFuncSetAttribute(reinterpret_cast<const void*>(k_small_order),
                            hipFuncAttributeMaxDynamicSharedMemorySize, opts.lds_bytes);
  k_small_order<<<blocks, kSW, static_cast<size_t>(opts.lds_bytes), s>>>(single, jobs_dev, njobs,
                                                                         opts);
  return hipGetLastError();
}

}  // namespace rcm
