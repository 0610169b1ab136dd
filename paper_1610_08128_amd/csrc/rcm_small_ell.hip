// The one-work-group engine for small graphs whose rows hold at most eight
// off-diagonal entries (meshes and other bounded-degree patterns): the same
// computation as rcm_small.hip (checks and statistics of Section II-A, the
// components in increasing lowest-id order of Section III-B, Algorithm 2's
// searches, Algorithm 3's labelled BFS in SortPerm's (parent label, degree,
// id) order, the reversal of Algorithm 1), with a data layout and a level
// step cut down to the few dependent LDS round trips a level needs.
//
// - Rows live in LDS as fixed 16-byte records of eight 16-bit columns
//   (diagonal dropped, fillers equal to the row's own vertex), so a level
//   reads a parent's whole row with one load and no row pointer.
// - Every row is sorted once by its columns' (degree, id) keys.  A parent's
//   children in Algorithm 3 are then already in SortPerm's order along its
//   row: a child's rank among its siblings is the number of children before
//   it in the row, a popcount.
// - Every pass claims vertices with LDS atomic minimums that return
//   nothing, and reads the words back once: in a search the claim is a
//   (level, lane, slot) token and the lane that finds its own token back
//   found the vertex; in the labelled BFS it is the parent's label + 1, and
//   the minimum is Algorithm 3's smallest parent label.  A level is then
//   three dependent LDS round trips (its queue entries, their rows, the
//   claims read back) and no exchange-with-return atomics, which cost a
//   full round trip each.
// - The bulk phases (loading with the checks, the row sort, the statistics
//   of the result) run on eight waves; the level loops, whose levels are a
//   wave wide on such graphs, run on the first wave alone while the others
//   wait at the work-group barrier.
//
// The kernel declines (kSmallDeclined) a graph with a longer row or one that
// does not fit, and the host then runs the general engine; a malformed
// pattern gets the status every path gives it.

#include <mutex>

#include "rcm_common.hpp"

namespace rcm {

namespace {

constexpr int kEThreads = 512;              // eight waves for the bulk phases
constexpr int kEWaves = kEThreads / 64;
constexpr int kSlots = 8;                   // columns per row record
constexpr uint32_t kNone16 = 0xFFFFu;       // "no label" (16-bit)
// Claim words (every pass claims with atomic minimums): kFreeW unclaimed,
// kDoneW a vertex of an ordered component, label + 1 in a labelled pass
// (at most 65,535), and in a search the token
//   (kPassTop - pass) << 25 | (level + 1) << 9 | lane << 3 | slot.
// A later search's tokens are smaller than an earlier one's, so a new
// search finds the component unclaimed without resetting it, and every
// token is larger than every label claim, so neither does the labelled
// pass after the searches.  The pass number wraps after kPassTop - 1
// searches (the claim words are reset then).
constexpr uint32_t kFreeW = 0xFFFFFFFFu;
constexpr uint32_t kDoneW = 0u;
constexpr int kTokBits = 9;                 // token: lane (6 bits) and slot (3 bits)
constexpr int kPassShift = 25;              // above 16 bits of level + 1
constexpr uint32_t kPassTop = 127;
constexpr uint32_t kNoKey = 0xFFFFFFFFu;    // (degree << 16 | id) of no vertex

inline __host__ __device__ size_t al16(size_t x) { return (x + 15) & ~static_cast<size_t>(15); }

// LDS bytes for n vertices: row records, degree, label and order (16-bit;
// the order has one spare entry, the target of clamped positions), claim
// words (32-bit).
inline __host__ __device__ size_t ell_bytes(int64_t n) {
  const size_t N = static_cast<size_t>(n);
  return al16(16 * N) + 2 * al16(2 * N) + al16(2 * (N + 1)) + al16(4 * N);
}

struct ELds {
  uint4* row;      // n records of 8 columns (16-bit pairs)
  uint16_t* deg;   // off-diagonal entries of the row
  uint16_t* lab;   // final position once the vertex's component is ordered, else kNone16
  uint16_t* ord;   // queue / Cuthill-McKee order of the component in hand
  uint32_t* clm;   // claims and search stamps
  uint32_t* sink;  // one word per lane of the first wave: the target of the
                   // level loops' masked-off stores, so that they need no
                   // branch (and no exec-mask registers per slot)
};

struct EPass {
  int32_t ecc;     // levels - 1
  uint32_t key;    // minimum (degree << 16 | id) of the last level
  int32_t count;   // vertices reached
};

__device__ __forceinline__ uint32_t lds_ld(const uint32_t* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}
__device__ __forceinline__ void lds_st(uint32_t* p, uint32_t v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}
// Orders the first wave's LDS accesses among its lanes: a wave's LDS
// operations are performed in the order it issues them, so a wavefront-scope
// fence needs no wait, only that the compiler keep that order (in particular
// a token's read-back after the stores and atomics that race for the word).
__device__ __forceinline__ void lds_fence() {
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
}

__device__ __forceinline__ uint32_t wave_min_u32(uint32_t x) {
  for (int o = 32; o > 0; o >>= 1) {
    const uint32_t y = __shfl_xor(x, o, 64);
    x = y < x ? y : x;
  }
  return x;
}

// Exclusive prefix of a per-lane count below 2^bits over the wave, and the
// total, from one ballot per bit.
__device__ __forceinline__ int ell_wave_prefix(uint32_t c, int bits, int* total) {
  int pre = 0, tot = 0;
  for (int b = 0; b < bits; ++b) {
    const unsigned long long m = __ballot((c >> b) & 1u);
    const int below = __builtin_amdgcn_mbcnt_hi(
        static_cast<uint32_t>(m >> 32), __builtin_amdgcn_mbcnt_lo(static_cast<uint32_t>(m), 0));
    pre += below << b;
    tot += __popcll(m) << b;
  }
  *total = tot;
  return pre;
}

// The first W columns of u's record.
template <int W>
__device__ __forceinline__ void load_row(const ELds& L, uint32_t u, uint32_t* nb) {
  if constexpr (W == 8) {
    const uint4 r = L.row[u];
    const uint32_t w[4] = {r.x, r.y, r.z, r.w};
#pragma unroll
    for (int h = 0; h < 4; ++h) {
      nb[2 * h] = w[h] & 0xFFFFu;
      nb[2 * h + 1] = w[h] >> 16;
    }
  } else {
    const uint2 r = reinterpret_cast<const uint2*>(L.row)[2 * u];
    nb[0] = r.x & 0xFFFFu;
    nb[1] = r.x >> 16;
    nb[2] = r.y & 0xFFFFu;
    nb[3] = r.y >> 16;
  }
}

// Columns [S * sub, S * sub + S) of u's record (S = 1, 2, 4 or 8).
template <int S>
__device__ __forceinline__ void load_part(const ELds& L, uint32_t u, uint32_t sub, uint32_t* nb) {
  if constexpr (S == 8) {
    load_row<8>(L, u, nb);
  } else if constexpr (S == 4) {
    const uint2 r = reinterpret_cast<const uint2*>(L.row)[2 * u + sub];
    nb[0] = r.x & 0xFFFFu;
    nb[1] = r.x >> 16;
    nb[2] = r.y & 0xFFFFu;
    nb[3] = r.y >> 16;
  } else if constexpr (S == 2) {
    const uint32_t r = reinterpret_cast<const uint32_t*>(L.row)[4 * u + sub];
    nb[0] = r & 0xFFFFu;
    nb[1] = r >> 16;
  } else {
    static_assert(S == 1, "1, 2, 4 or 8 columns");
    nb[0] = reinterpret_cast<const uint16_t*>(L.row)[8 * u + sub];
  }
}

__device__ __forceinline__ uint32_t vkey(const ELds& L, uint32_t x) {
  return (static_cast<uint32_t>(L.deg[x]) << 16) | x;
}

// Minimum (degree << 16 | id) over ord[b, e).
__device__ __forceinline__ uint32_t ell_level_key(const ELds& L, int32_t b, int32_t e) {
  uint32_t k = kNoKey;
  for (int32_t i = b + static_cast<int32_t>(threadIdx.x); i < e; i += 64) {
    const uint32_t kv = vkey(L, L.ord[i]);
    k = kv < k ? kv : k;
  }
  return wave_min_u32(k);
}

// One level of a search: the vertices ord[fb, fe) claim their neighbours
// and the vertices they find go to ord[fe + next, ...); returns how many.
// LPV lanes share a vertex, each taking S of its W columns (a narrow level
// keeps more lanes busy and each lane's work short); the lanes of a vertex
// are adjacent, so lane order is the (vertex, column) order.  A vertex is
// claimed with an LDS atomic minimum of a token (level + 1, lane, slot) and
// is found by the lane that reads its own token back: a vertex of an
// earlier level keeps its smaller token, an ordered component's kDoneW (0)
// stays, and of the lanes reaching a new vertex exactly one holds the
// minimum.  A level wider than one pass of the wave is taken in chunks; a
// later chunk's tokens are not larger than an earlier chunk's of the same
// level, so there each lane first reads the words and claims only unclaimed
// ones.  With kCheck a neighbour in an ordered component sets badm.
template <int S, int LPV, bool kCheck>
__device__ __forceinline__ int32_t ell_search_level(const ELds& L, int32_t n, int32_t fb,
                                                    int32_t fe, uint32_t lvl,
                                                    unsigned long long& badm) {
  constexpr int32_t kPer = 64 / LPV;  // vertices per chunk
  const uint32_t lane = threadIdx.x;
  uint32_t* const mine = &L.sink[lane];
  uint16_t* const mine16 = reinterpret_cast<uint16_t*>(mine);
  const bool one = fe - fb <= kPer;
  int32_t next = 0;
  for (int32_t q = fb; q < fe; q += kPer) {
    const int32_t i = q + static_cast<int32_t>(lane) / LPV;
    const bool act = i < fe;
    const uint32_t u = act ? static_cast<uint32_t>(L.ord[i]) : 0u;
    uint32_t nb[S];
    load_part<S>(L, u, lane % LPV, nb);
    unsigned nbr = 0;  // (bitwise operators throughout: no branches per slot)
#pragma unroll
    for (int j = 0; j < S; ++j) nbr |= static_cast<unsigned>(act & (nb[j] != u)) << j;
    unsigned cand = nbr;
    if (!one) {
      // unclaimed in this search: kFreeW or an earlier search's token, all
      // of them at least the next larger search field
      const uint32_t unclaimed = ((lvl >> kPassShift) + 1u) << kPassShift;
      cand = 0;
#pragma unroll
      for (int j = 0; j < S; ++j)
        cand |= (nbr >> j & 1u & static_cast<unsigned>(lds_ld(&L.clm[nb[j]]) >= unclaimed)) << j;
    }
#pragma unroll
    for (int j = 0; j < S; ++j)
      atomicMin((cand >> j & 1u) ? &L.clm[nb[j]] : mine,
                lvl | (lane << 3) | static_cast<uint32_t>(j));
    lds_fence();
    unsigned win = 0;
#pragma unroll
    for (int j = 0; j < S; ++j) {
      const uint32_t back = lds_ld(&L.clm[nb[j]]);
      win |= (cand >> j & 1u &
              static_cast<unsigned>(back == (lvl | (lane << 3) | static_cast<uint32_t>(j))))
             << j;
      if (kCheck) badm |= __ballot((nbr >> j & 1u) & (back == kDoneW));
    }
    int total;
    const int pre = ell_wave_prefix(static_cast<uint32_t>(__popc(win)), S >= 4 ? (S == 8 ? 4 : 3)
                                                                            : (S == 2 ? 2 : 1),
                                    &total);
    const int32_t base = fe + next + pre;
    // each vertex is found once per pass, so the positions stay below n;
    // clamped to the spare entry all the same (the caller's level-end check
    // reports a count past n)
#pragma unroll
    for (int j = 0; j < S; ++j) {
      const int32_t at = base + __popc(win & ((1u << j) - 1u));
      *((win >> j & 1u) ? &L.ord[at < n ? at : n] : mine16) = static_cast<uint16_t>(nb[j]);
    }
    next += total;
  }
  lds_fence();
  return next;
}

// Unlabelled level structure from root (Algorithm 2's BFS), queue in
// ord[o, ...), search number pass (1 .. kPassTop - 1).  The component's claim
// words must be kFreeW or tokens of earlier searches on entry.  With
// kCheck, a neighbour in an ordered component sets bad; the first search of
// a component checks, since every later pass must reach the same vertices
// and read the same rows (a different count sets bad).  First wave only.
template <int W, bool kCheck>
__device__ EPass ell_search(const ELds& L, int32_t n, int32_t o, uint32_t root, uint32_t pass,
                            bool& bad) {
  const uint32_t passw = (kPassTop - pass) << kPassShift;
  if (threadIdx.x == 0) {
    L.ord[o] = static_cast<uint16_t>(root);
    lds_st(&L.clm[root], passw | (1u << kTokBits) | ((1u << kTokBits) - 1));
  }
  lds_fence();
  int32_t fb = o, fe = o + 1, ecc = 0;
  unsigned long long badm = 0;
  while (true) {
    // tokens of the level being found: (its level + 1) above lane and slot
    const uint32_t lvl = passw | static_cast<uint32_t>(ecc + 2) << kTokBits;
    const int32_t width = fe - fb;
    int32_t next;
    if (width <= 16)
      next = ell_search_level<W / 4, 4, kCheck>(L, n, fb, fe, lvl, badm);
    else if (width <= 32)
      next = ell_search_level<W / 2, 2, kCheck>(L, n, fb, fe, lvl, badm);
    else
      next = ell_search_level<W, 1, kCheck>(L, n, fb, fe, lvl, badm);
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
  bad |= badm != 0;
  EPass r;
  r.ecc = ecc;
  r.key = ell_level_key(L, fb, fe);
  r.count = fe - o;
  return r;
}

// One level of Algorithm 3: the parents ord[b, e) (labels b ..) claim their
// neighbours with an LDS atomic minimum of their label + 1; a neighbour
// whose claim then equals a parent's is that parent's child (a vertex
// labelled earlier keeps its smaller claim, an ordered component's kDoneW
// (0) stays, and the component's first search has checked that none is a
// neighbour).  The children, already in (degree, id) order along the sorted
// row, take the parent's first child label plus their rank, the number of
// children before them in the row.  Lanes as in ell_search_level (LPV lanes
// per parent, S columns each: lane order is row order).  Returns the number
// of children placed at ord[e, ...).
template <int S, int LPV>
__device__ __forceinline__ int32_t ell_label_level(const ELds& L, int32_t n, int32_t b,
                                                   int32_t e) {
  constexpr int32_t kPer = 64 / LPV;
  const uint32_t lane = threadIdx.x;
  uint32_t* const mine = &L.sink[lane];
  uint16_t* const mine16 = reinterpret_cast<uint16_t*>(mine);
  // claims of every parent of the level; a one-chunk level keeps its rows
  // in registers for the count
  const bool one = e - b <= kPer;
  uint32_t u1 = 0, nb1[S];
#pragma unroll
  for (int j = 0; j < S; ++j) nb1[j] = 0;
  for (int32_t q = b; q < e; q += kPer) {
    const int32_t p = q + static_cast<int32_t>(lane) / LPV;
    const bool act = p < e;
    const uint32_t u = act ? static_cast<uint32_t>(L.ord[p]) : 0u;
    uint32_t nb[S];
    load_part<S>(L, u, lane % LPV, nb);
#pragma unroll
    for (int j = 0; j < S; ++j)
      atomicMin((act & (nb[j] != u)) ? &L.clm[nb[j]] : mine, static_cast<uint32_t>(p) + 1u);
    if (one) {
      u1 = u;
#pragma unroll
      for (int j = 0; j < S; ++j) nb1[j] = nb[j];
    }
  }
  lds_fence();
  int32_t placed = 0;
  for (int32_t q = b; q < e; q += kPer) {
    const int32_t p = q + static_cast<int32_t>(lane) / LPV;
    const bool act = p < e;
    uint32_t u, nb[S];
    if (one) {
      u = u1;
#pragma unroll
      for (int j = 0; j < S; ++j) nb[j] = nb1[j];
    } else {
      u = act ? static_cast<uint32_t>(L.ord[p]) : 0u;
      load_part<S>(L, u, lane % LPV, nb);
    }
    unsigned child = 0;
#pragma unroll
    for (int j = 0; j < S; ++j) {
      const uint32_t c2 = lds_ld(&L.clm[nb[j]]);
      child |= static_cast<unsigned>(act & (nb[j] != u) & (c2 == static_cast<uint32_t>(p) + 1u))
               << j;
    }
    int total;
    const int pre = ell_wave_prefix(static_cast<uint32_t>(__popc(child)),
                                    S >= 4 ? (S == 8 ? 4 : 3) : (S == 2 ? 2 : 1), &total);
    const int32_t base = e + placed + pre;
    // (a vertex is placed once per pass: positions below n, clamped to the
    // spare entry all the same)
#pragma unroll
    for (int j = 0; j < S; ++j) {
      const int32_t at = base + __popc(child & ((1u << j) - 1u));
      *((child >> j & 1u) ? &L.ord[at < n ? at : n] : mine16) = static_cast<uint16_t>(nb[j]);
    }
    placed += total;
  }
  lds_fence();
  return placed;
}

// Algorithm 3 from root: labels are the positions ord[o, ...).  The claim
// words of the component must be kFreeW on entry.  First wave only.
template <int W>
__device__ EPass ell_label(const ELds& L, int32_t n, int32_t o, uint32_t root, bool& bad) {
  if (threadIdx.x == 0) {
    L.ord[o] = static_cast<uint16_t>(root);
    lds_st(&L.clm[root], static_cast<uint32_t>(o) + 1u);
  }
  lds_fence();
  int32_t b = o, e = o + 1, levels = 1;
  while (true) {
    const int32_t width = e - b;
    int32_t placed;
    if (width <= 16)
      placed = ell_label_level<W / 4, 4>(L, n, b, e);
    else if (width <= 32)
      placed = ell_label_level<W / 2, 2>(L, n, b, e);
    else
      placed = ell_label_level<W, 1>(L, n, b, e);
    if (placed == 0) break;
    if (e + placed > n) {
      bad = true;
      break;
    }
    b = e;
    e += placed;
    ++levels;
  }
  EPass r;
  r.ecc = levels - 1;
  r.key = ell_level_key(L, b, e);
  r.count = e - o;
  return r;
}

// The claim words of ord[o, o + size) back to kFreeW.  First wave only.
__device__ __forceinline__ void ell_reset(const ELds& L, int32_t o, int32_t size) {
  for (int32_t i = o + static_cast<int32_t>(threadIdx.x); i < o + size; i += 64)
    lds_st(&L.clm[L.ord[i]], kFreeW);
  lds_fence();
}

// Every claim word back to kFreeW except an ordered component's kDoneW
// (when the search number wraps).  First wave only.
__device__ __forceinline__ void ell_reset_all(const ELds& L, int32_t n) {
  for (int32_t v = static_cast<int32_t>(threadIdx.x); v < n; v += 64)
    if (lds_ld(&L.clm[v]) != kDoneW) lds_st(&L.clm[v], kFreeW);
  lds_fence();
}

struct EAcc {
  int32_t ncomp = 0, diameter = 0, nbfs = 0, nlevels = 0;
  unsigned long long edges = 0;
  int32_t err = 0;
};

// Every component of the graph, in increasing lowest-id order: searches,
// labelled BFS, reversal.  First wave only; t_* accumulate clock ticks.
template <int W>
__device__ EAcc ell_components(const ELds& L, const SmallJob& J, const SmallOpts& O, int32_t n,
                               long long& t_search, long long& t_label, long long& t_rev) {
  const int lane = threadIdx.x;
  EAcc acc;
  int32_t o = 0, s_from = 0;
  uint32_t pass = 0;  // searches since the claim words were last reset
  // the next search number, resetting the claim words when it wraps
  auto next_pass = [&]() -> uint32_t {
    if (++pass >= kPassTop) {
      ell_reset_all(L, n);
      pass = 1;
    }
    return pass;
  };
  uint32_t since_poll = 0;
  // one read of the caller's abort flag per 4096 units of work (a level is
  // one unit, a component 64)
  auto abort_poll = [&](uint32_t units) -> bool {
    if (O.abort_flag == nullptr) return false;
    since_poll += units;
    if (since_poll < 4096) return false;
    since_poll = 0;
    const int hit = lane == 0 && abort_requested(O.abort_flag) ? 1 : 0;
    return __shfl(hit, 0, 64) != 0;
  };
  bool bad = false;
  while (o < n) {
    if (abort_poll(64)) {
      acc.err = RCM_ERR_ABORTED;
      return acc;
    }
    int32_t s = -1;
    while (s < 0 && s_from < n) {
      const int32_t i = s_from + lane;
      const unsigned long long m = __ballot(i < n && L.lab[i] == kNone16);
      if (m) s = s_from + __builtin_ctzll(m);
      else s_from += 64;
    }
    if (s < 0) {
      acc.err = RCM_ERR_NOT_SYMMETRIC;
      return acc;
    }
    s_from = s + 1;
    int32_t size = 1, nbfs = 2, levels = 1;
    long long mc = 0;
    if (L.deg[s] == 0) {
      // an isolated vertex: its own component (two level structures, one level)
      if (lane == 0) L.ord[o] = static_cast<uint16_t>(s);
      lds_fence();
    } else {
      const long long ts0 = wall_clock64();
      // (the component's claim words are kFreeW: no pass has touched them)
      EPass r = ell_search<W, true>(L, n, o, static_cast<uint32_t>(s), next_pass(), bad);
      size = r.count;
      nbfs = 1;
      uint32_t root = static_cast<uint32_t>(s);
      int32_t nlvl = r.ecc - 1;
      bool labelled = false;
      long long tl = 0;
      while (!__any(bad) && r.ecc > nlvl) {
        if (abort_poll(static_cast<uint32_t>(r.ecc) + 1u)) {
          acc.err = RCM_ERR_ABORTED;
          return acc;
        }
        nlvl = r.ecc;
        const uint32_t v = r.key & 0xFFFFu;
        ++nbfs;
        root = v;
        if (O.pp_variant == 0 && nbfs >= 3) {
          // Algorithm 2 returns v unless this search goes deeper, and
          // Algorithm 3 starts there: this search is the labelled BFS
          // (after searches the claim words need no reset; after a
          // labelled pass that went deeper they do)
          const long long tl0 = wall_clock64();
          if (labelled) ell_reset(L, o, size);
          r = ell_label<W>(L, n, o, v, bad);
          labelled = true;
          tl += wall_clock64() - tl0;
        } else {
          r = ell_search<W, false>(L, n, o, v, next_pass(), bad);
        }
        if (r.count != size) bad = true;
      }
      if (O.pp_variant == 1) root = r.key & 0xFFFFu;
      t_search += wall_clock64() - ts0 - tl;
      t_label += tl;
      if (!labelled && !__any(bad)) {
        const long long tl0 = wall_clock64();
        r = ell_label<W>(L, n, o, root, bad);
        if (r.count != size) bad = true;
        t_label += wall_clock64() - tl0;
      }
      levels = r.ecc + 1;
    }
    if (__any(bad)) {
      acc.err = RCM_ERR_NOT_SYMMETRIC;
      return acc;
    }
    // reversal: Cuthill-McKee label o + t goes to position anchor - t; the
    // component's claim words become kDoneW
    const long long tr0 = wall_clock64();
    const int32_t anchor = O.reverse_mode ? n - 1 - o : o + size - 1;
    for (int32_t t = lane; t < size; t += 64) {
      const uint32_t x = L.ord[o + t];
      const int32_t at = anchor - t;
      J.perm[at] = static_cast<int32_t>(x) + J.id_off;
      if (J.iperm) J.iperm[x] = at + J.pos_off;
      L.lab[x] = static_cast<uint16_t>(at);
      lds_st(&L.clm[x], kDoneW);
      mc += L.deg[x];  // the degrees every level structure sums
    }
    mc = wave_sum_i64(mc);
    lds_fence();
    t_rev += wall_clock64() - tr0;
    acc.ncomp += 1;
    acc.nbfs += nbfs;
    acc.nlevels += levels;
    acc.diameter = levels - 1 > acc.diameter ? levels - 1 : acc.diameter;
    acc.edges += static_cast<unsigned long long>(nbfs + 1) * static_cast<unsigned long long>(mc);
    o += size;
  }
  return acc;
}

__global__ void __launch_bounds__(kEThreads)
    k_small_ell(SmallJob J, SmallOpts O) {
  extern __shared__ __align__(16) char smem[];
  __shared__ long long red[16];
  const int tid = threadIdx.x;
  const int32_t n = J.n;
  SmallResult* R = J.res;
  const int32_t nnz = J.nnz >= 0 ? J.nnz : J.rowptr[n];
  if (tid == 0) R->nnz = nnz;
  if (nnz < 0) {
    if (tid == 0) R->status = RCM_ERR_BAD_CSR;
    return;
  }
  if (n <= 0 || n >= 65535 || ell_bytes(n) > static_cast<size_t>(O.lds_bytes)) {
    if (tid == 0) R->status = kSmallDeclined;
    return;
  }
  __shared__ uint32_t sink[64];
  ELds L;
  L.sink = sink;
  {
    char* p = smem;
    const size_t N = static_cast<size_t>(n);
    L.row = reinterpret_cast<uint4*>(p);
    p += al16(16 * N);
    L.deg = reinterpret_cast<uint16_t*>(p);
    p += al16(2 * N);
    L.lab = reinterpret_cast<uint16_t*>(p);
    p += al16(2 * N);
    L.ord = reinterpret_cast<uint16_t*>(p);
    p += al16(2 * (N + 1));
    L.clm = reinterpret_cast<uint32_t*>(p);
  }
  long long tk0 = wall_clock64();
  // 1. rows into LDS records with the structural checks, the degrees and
  // the bandwidth / envelope size of the input order.  The row pointers
  // first go to the claim words (free until the searches), with many loads
  // in flight per thread; then each thread takes kB rows at a time and
  // issues all their entry loads before it waits.
  constexpr int kPtr = 8;
  for (int32_t i0 = tid; i0 < n; i0 += kEThreads * kPtr) {
    int32_t r[kPtr];
#pragma unroll
    for (int j = 0; j < kPtr; ++j) {
      const int32_t i = i0 + j * kEThreads;
      r[j] = i < n ? J.rowptr[i] : 0;
    }
#pragma unroll
    for (int j = 0; j < kPtr; ++j) {
      const int32_t i = i0 + j * kEThreads;
      if (i < n) L.clm[i] = static_cast<uint32_t>(r[j]);
    }
  }
  __syncthreads();
  // (rowptr[n] is the entry count by definition when the job gives none)
  bool bad = tid == 0 && J.nnz >= 0 && J.rowptr[n] != nnz;
  bool longrow = false;
  long long bw = 0, prof = 0;
  int maxdeg = 0;
  constexpr int kB = 8;
  for (int32_t v0 = tid; v0 < n; v0 += kEThreads * kB) {
    int32_t a[kB], b[kB];
    bool take[kB];
#pragma unroll
    for (int q = 0; q < kB; ++q) {
      const int32_t v = v0 + q * kEThreads;
      a[q] = v < n ? static_cast<int32_t>(L.clm[v]) : 0;
      b[q] = v < n ? (v + 1 < n ? static_cast<int32_t>(L.clm[v + 1]) : nnz) : 0;
      const bool broken =
          v < n && (a[q] < 0 || b[q] > nnz || b[q] < a[q] || (v == 0 && a[q] != 0));
      bad |= broken;
      longrow |= v < n && !broken && b[q] - a[q] > kSlots + 1;
      take[q] = v < n && !broken && b[q] - a[q] <= kSlots + 1;
    }
    int32_t c[kB][kSlots + 1];
#pragma unroll
    for (int q = 0; q < kB; ++q)
#pragma unroll
      for (int j = 0; j <= kSlots; ++j)
        c[q][j] = take[q] && a[q] + j < b[q] ? J.colidx[a[q] + j] : -1 - j;
#pragma unroll
    for (int q = 0; q < kB; ++q) {
      if (!take[q]) continue;
      const int32_t v = v0 + q * kEThreads;
      const int32_t len = b[q] - a[q];
      int self = 0, selfpos = kSlots + 1, mn = v;
#pragma unroll
      for (int j = 0; j <= kSlots; ++j) {
        const bool in = j < len;
        const bool me = in & (c[q][j] == v);
        bad |= in & ((c[q][j] < 0) | (c[q][j] >= n));
        self += me ? 1 : 0;
        selfpos = (me & (selfpos > kSlots)) ? j : selfpos;
        mn = (in & (c[q][j] < mn)) ? c[q][j] : mn;
      }
      // a repeated diagonal entry here; repeated off-diagonal ones show up
      // next to each other once the row is sorted
      bad |= self > 1;
      const int d = len - (self > 0 ? 1 : 0);
      if (d > kSlots) {
        longrow = true;
        continue;
      }
      // the off-diagonal columns in row order (the diagonal entry skipped),
      // then fillers (the vertex)
      uint32_t cols[kSlots];
#pragma unroll
      for (int h = 0; h < kSlots; ++h) {
        const int32_t x = h < selfpos ? c[q][h] : c[q][h + 1];
        cols[h] = h < d ? static_cast<uint32_t>(x) & 0xFFFFu : static_cast<uint32_t>(v);
      }
      L.row[v] = make_uint4(cols[0] | cols[1] << 16, cols[2] | cols[3] << 16,
                            cols[4] | cols[5] << 16, cols[6] | cols[7] << 16);
      L.deg[v] = static_cast<uint16_t>(d);
      L.lab[v] = static_cast<uint16_t>(kNone16);
      maxdeg = d > maxdeg ? d : maxdeg;
      const long long beta = static_cast<long long>(v) - mn;
      bw = beta > bw ? beta : bw;
      prof += beta;
    }
  }
  // a malformed pattern is reported as such whatever its rows' lengths
  if (__syncthreads_or(bad)) {
    if (tid == 0) R->status = RCM_ERR_BAD_CSR;
    return;
  }
  if (__syncthreads_or(longrow)) {
    if (tid == 0) R->status = kSmallDeclined;
    return;
  }
  bw = block_max_i64(bw, red);
  prof = block_sum_i64(prof, red);
  const int W = block_max_i64(maxdeg, red) <= 4 ? 4 : 8;
  long long tk1 = wall_clock64();
  // 2. every row sorted by its columns' (degree, id) keys (fillers last),
  // with the check for repeated columns; then optionally the full symmetry
  // check.  (Each thread rewrites only its own rows and reads only the
  // degrees, all complete behind the barriers above.)
  bool dup = false;
  for (int32_t v = tid; v < n; v += kEThreads) {
    uint32_t nb[kSlots], key[kSlots];
    load_row<kSlots>(L, static_cast<uint32_t>(v), nb);
#pragma unroll
    for (int j = 0; j < kSlots; ++j)
      key[j] = nb[j] == static_cast<uint32_t>(v) ? kNoKey : vkey(L, nb[j]);
    // 19-comparator sorting network for eight keys
    constexpr int kNet[19][2] = {{0, 2}, {1, 3}, {4, 6}, {5, 7}, {0, 4}, {1, 5}, {2, 6},
                                 {3, 7}, {0, 1}, {2, 3}, {4, 5}, {6, 7}, {2, 4}, {3, 5},
                                 {1, 4}, {3, 6}, {1, 2}, {3, 4}, {5, 6}};
#pragma unroll
    for (int c = 0; c < 19; ++c) {
      const uint32_t x = key[kNet[c][0]], y = key[kNet[c][1]];
      key[kNet[c][0]] = x < y ? x : y;
      key[kNet[c][1]] = x < y ? y : x;
    }
#pragma unroll
    for (int j = 0; j + 1 < kSlots; ++j) dup |= (key[j] != kNoKey) & (key[j] == key[j + 1]);
#pragma unroll
    for (int j = 0; j < kSlots; ++j)
      nb[j] = key[j] == kNoKey ? static_cast<uint32_t>(v) : (key[j] & 0xFFFFu);
    L.row[v] = make_uint4(nb[0] | nb[1] << 16, nb[2] | nb[3] << 16, nb[4] | nb[5] << 16,
                          nb[6] | nb[7] << 16);
    L.clm[v] = kFreeW;  // (held the row pointers until the barriers above)
  }
  if (__syncthreads_or(dup)) {
    if (tid == 0) R->status = RCM_ERR_BAD_CSR;
    return;
  }
  if (O.check_full) {
    bool miss = false;
    for (int32_t v = tid; v < n; v += kEThreads) {
      uint32_t nb[kSlots];
      load_row<kSlots>(L, static_cast<uint32_t>(v), nb);
#pragma unroll
      for (int j = 0; j < kSlots; ++j) {
        if (nb[j] == static_cast<uint32_t>(v)) continue;
        uint32_t back[kSlots];
        load_row<kSlots>(L, nb[j], back);
        bool found = false;
#pragma unroll
        for (int h = 0; h < kSlots; ++h) found |= back[h] == static_cast<uint32_t>(v);
        miss |= !found;
      }
    }
    if (__syncthreads_or(miss)) {
      if (tid == 0) R->status = RCM_ERR_NOT_SYMMETRIC;
      return;
    }
  }
  __syncthreads();
  long long tk2 = wall_clock64();
  // 3. the components, on the first wave
  long long t_search = 0, t_label = 0, t_rev = 0;
  EAcc acc;
  if (tid < 64) {
    acc = W == 4 ? ell_components<4>(L, J, O, n, t_search, t_label, t_rev)
                 : ell_components<8>(L, J, O, n, t_search, t_label, t_rev);
    if (tid == 0) {
      red[8] = acc.err;
      red[9] = acc.ncomp;
      red[10] = acc.diameter;
      red[11] = acc.nbfs;
      red[12] = acc.nlevels;
      red[13] = static_cast<long long>(acc.edges);
    }
  }
  __syncthreads();
  if (red[8] != 0) {
    if (tid == 0) R->status = static_cast<int32_t>(red[8]);
    return;
  }
  if (tid == 0) {
    acc.ncomp = static_cast<int32_t>(red[9]);
    acc.diameter = static_cast<int32_t>(red[10]);
    acc.nbfs = static_cast<int32_t>(red[11]);
    acc.nlevels = static_cast<int32_t>(red[12]);
    acc.edges = static_cast<unsigned long long>(red[13]);
  }
  __syncthreads();
  // 4. bandwidth and envelope size of the result (lab holds positions)
  long long tk3 = wall_clock64();
  long long bw2 = 0, prof2 = 0;
  for (int32_t v = tid; v < n; v += kEThreads) {
    const int32_t k = L.lab[v];
    uint32_t nb[kSlots];
    load_row<kSlots>(L, static_cast<uint32_t>(v), nb);
    int32_t mn = k;
#pragma unroll
    for (int j = 0; j < kSlots; ++j) {
      const int32_t q = L.lab[nb[j]];
      mn = q < mn ? q : mn;
    }
    const long long beta = k - mn;
    bw2 = beta > bw2 ? beta : bw2;
    prof2 += beta;
  }
  bw2 = block_max_i64(bw2, red);
  prof2 = block_sum_i64(prof2, red);
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
    R->ticks[0] = tk1 - tk0;
    R->ticks[1] = tk2 - tk1;
    R->ticks[2] = t_search;
    R->ticks[3] = t_label;
    R->ticks[4] = t_rev;
    R->ticks[5] = wall_clock64() - tk3;
    R->status = RCM_OK;
  }
}

}  // namespace

// The kernel's static LDS (reduction words and the lanes' sink) comes on
// top of the dynamic part; the budget the host compares with already
// keeps 256 bytes back, this reserve covers the rest.
constexpr size_t kEllStaticReserve = 768;
static_assert(kEllStaticReserve + 256 >= 16 * sizeof(long long) + 64 * sizeof(uint32_t),
              "the static LDS outgrew its reserve");

size_t small_ell_lds_bytes(int64_t n) {
  if (n <= 0) return 0;
  if (n >= 65535) return ~static_cast<size_t>(0);
  return ell_bytes(n) + kEllStaticReserve;
}

hipError_t launch_small_ell(const SmallJob& job, const SmallOpts& opts, hipStream_t s) {
  if (small_ell_lds_bytes(job.n) > static_cast<size_t>(opts.lds_bytes) || job.n <= 0)
    return hipErrorInvalidValue;
  const size_t need = ell_bytes(job.n);
  SmallOpts o = opts;
  o.lds_bytes = static_cast<int32_t>(need);
  // the kernel's dynamic LDS allowance, raised per device as larger graphs
  // come (one attribute call per new maximum instead of one per launch)
  static std::mutex mu;
  static size_t allowed[64] = {};
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return hipErrorInvalidDevice;
  {
    std::lock_guard<std::mutex> lk(mu);
    if (need > allowed[dev]) {
      const hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(k_small_ell),
                                               hipFuncAttributeMaxDynamicSharedMemorySize,
                                               static_cast<int>(need));
      if (e != hipSuccess) return e;
      allowed[dev] = need;
    }
  }
  k_small_ell<<<1, kEThreads, need, s>>>(job, o);
  return hipGetLastError();
}

}  // namespace rcm
