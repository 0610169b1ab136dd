// The remaining level structures of Algorithm 2 and the labelled BFS of
// Algorithm 3 for a long component after its renumbering (rcm_relabel.hip),
// by one work-group with a window of the renumbered vertex ids in LDS.
//
// The renumbering orders the component by its first level structure, so a
// vertex at distance d from that structure's root has its neighbours among
// the ids of distances d - 1 .. d + 1.  On a long narrow component (a
// strip) the frontier of any later BFS then occupies a short id range, and
// so do its neighbours: a window of kWS consecutive ids, held in LDS as a
// ring (slot = id mod kWS) with each vertex's sorted row (four 16-bit
// offsets to its neighbours' ids) and its claim word (12 bytes a vertex),
// follows the frontier.  Each level is
// walked from LDS by the first wave, as in the one-work-group engine
// (rcm_small_ell.hip): three dependent LDS round trips, claims by atomic
// minimum read back once, narrow levels over several lanes per vertex.
// When a level needs an id outside the window, the whole work-group slides
// it (evicted claim words written back to global memory, entering rows,
// keys and claims loaded) and the level runs again.
//
// Rows hold at most 4 off-diagonal entries (k_build_ell4 sorts them by
// their columns' (degree, caller id) keys, so that a parent's children lie
// in SortPerm's order along its row).  The labelled pass writes each
// vertex's label to a global order array; the positions in the caller's
// numbering (perm, iperm) are written from it once the pass is final.  The
// kernel declines -- and the library runs the team kernel on the renumbered
// copy instead -- when a row is longer or reaches further than a 16-bit
// offset, a level is wider than the queue, the ids a level needs do not fit
// the window, or the searches outnumber the pass field; a count that
// differs from the component's size is an asymmetric pattern.

#include <algorithm>
#include <mutex>

#include "rcm_common.hpp"

namespace rcm {

namespace {

constexpr int kWThreads = 512;
constexpr int32_t kWS = 8192;              // window: vertex ids held in LDS (a power of two)
constexpr int32_t kWQ = 2048;              // queue entries per level
constexpr int32_t kWMargin = 64;           // ids kept beyond a slide's target range
// Claim words: kWFree unclaimed; label + 1 in a labelled pass (below 2^29);
// a search's token (7 - pass) << 29 | (level + 1) << 9 | lane << 3 | slot,
// smaller for every later search and larger than every label claim.
constexpr uint32_t kWFree = 0xFFFFFFFFu;
constexpr int kWPassShift = 29;
constexpr uint32_t kWPassTop = 7;          // searches 1 .. 6
constexpr int kWLevelShift = 9;
constexpr int32_t kWMaxLevel = (1 << 20) - 2;

// what the first wave reports at the barrier
enum : int32_t { kRun = 0, kSlide = 1, kPassDone = 2, kDecline = 3, kAsym = 4, kAbort = 5 };

struct WLds {
  uint2* row;                   // [kWS] four 16-bit offsets to the sorted neighbours (0: filler)
  uint32_t* claim;              // [kWS] claim words of the window's ids
  int32_t* q[2];                // [kWQ] each: the current and the next level
};

struct WCtl {
  int32_t w_lo;                 // first id of the window
  int32_t state;                // kRun / kSlide / kPassDone / ...
  int32_t new_lo;               // a slide's target
  int32_t pad;
  int32_t ecc, count;           // the pass's result (first wave)
  unsigned long long lastkey;
};

__device__ __forceinline__ uint32_t wslot(int32_t id) {
  return static_cast<uint32_t>(id) & static_cast<uint32_t>(kWS - 1);
}
__device__ __forceinline__ bool in_window(int32_t id, int32_t w_lo) {
  return static_cast<uint32_t>(id - w_lo) < static_cast<uint32_t>(kWS);
}
__device__ __forceinline__ uint32_t lds_ld32(const uint32_t* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}
// (as in the one-work-group engine: a wave's LDS operations are performed
// in issue order; the fence only keeps the compiler's order)
__device__ __forceinline__ void wfence() { __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront"); }

__device__ __forceinline__ int wprefix(uint32_t c, int bits, int* total) {
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

__device__ __forceinline__ int32_t wave_min_i32(int32_t x) {
  for (int o = 32; o > 0; o >>= 1) {
    const int32_t y = __shfl_xor(x, o, 64);
    x = y < x ? y : x;
  }
  return x;
}
__device__ __forceinline__ int32_t wave_max_i32(int32_t x) {
  for (int o = 32; o > 0; o >>= 1) {
    const int32_t y = __shfl_xor(x, o, 64);
    x = y > x ? y : x;
  }
  return x;
}

// Neighbour ids [S * sub, S * sub + S) of x's row record (S = 1, 2 or 4):
// x plus the sign-extended 16-bit offsets (a filler's offset is 0).
template <int S>
__device__ __forceinline__ void row_part(const WLds& L, int32_t x, uint32_t sub, int32_t* nb) {
  const uint32_t s = wslot(x);
  if constexpr (S == 4) {
    const uint2 r = L.row[s];
    nb[0] = x + (static_cast<int32_t>(r.x << 16) >> 16);
    nb[1] = x + (static_cast<int32_t>(r.x) >> 16);
    nb[2] = x + (static_cast<int32_t>(r.y << 16) >> 16);
    nb[3] = x + (static_cast<int32_t>(r.y) >> 16);
  } else if constexpr (S == 2) {
    const uint32_t r = reinterpret_cast<const uint32_t*>(L.row)[2 * s + sub];
    nb[0] = x + (static_cast<int32_t>(r << 16) >> 16);
    nb[1] = x + (static_cast<int32_t>(r) >> 16);
  } else {
    static_assert(S == 1, "1, 2 or 4 columns");
    nb[0] = x + reinterpret_cast<const int16_t*>(L.row)[4 * s + sub];
  }
}

// The whole work-group moves the window to [new_lo, new_lo + kWS): claim
// words of ids leaving it go back to global memory, and rows and claim
// words of entering ids come in (ids outside the component get an empty
// row and kWFree).  fresh: no id is carried over (a pass's first placement;
// the previous pass's words need not go back, since every later claim is
// below them).
__device__ void slide(const WLds& L, WCtl& C, const WinParams& P, int32_t new_lo, bool fresh) {
  const int32_t old_lo = C.w_lo;
  for (int32_t s = threadIdx.x; s < kWS; s += kWThreads) {
    const int32_t old_id = old_lo + static_cast<int32_t>(wslot(s - old_lo));
    const int32_t new_id = new_lo + static_cast<int32_t>(wslot(s - new_lo));
    if (!fresh && old_id == new_id) continue;
    if (!fresh && old_id >= 0 && old_id < P.size) P.claim[old_id] = L.claim[s];
    if (new_id >= 0 && new_id < P.size) {
      L.row[s] = P.ell[new_id];
      L.claim[s] = P.claim[new_id];
    } else {
      L.row[s] = make_uint2(0, 0);
      L.claim[s] = kWFree;
    }
  }
  __syncthreads();
  if (threadIdx.x == 0) C.w_lo = new_lo;
  __syncthreads();
}

// Where a slide must move the window so that [lo, hi] fits with the
// margin on the side the frontier moves to; false if it cannot.
__device__ __forceinline__ bool slide_target(int32_t lo, int32_t hi, int32_t w_lo,
                                             int32_t* new_lo) {
  if (static_cast<int64_t>(hi) - lo + 1 + 2 * kWMargin > kWS) return false;
  *new_lo = hi >= w_lo + kWS ? lo - kWMargin : hi + 1 + kWMargin - kWS;
  return true;
}

// One level from the queue q[cur][0, F) into q[cur ^ 1], by the first wave.
// Labelled (Algorithm 3): the vertices' labels are b + index, claims are
// label + 1, children go to labels e + position and to perm / iperm.
// Search: claims are the level's tokens (tok: pass and level), the lane and
// the slot.  Of the lanes reaching a vertex exactly one (the minimum) wins:
// all claims are made before any is read back (a wider search level takes
// its chunks one at a time, see below).
// Returns the number of vertices placed, or -1 (with *need_lo / *need_hi)
// when an id the level touches is outside the window (nothing is claimed
// then), or -2 when the next level overflows the queue.
template <int S, int LPV, bool kLabel>
__device__ int32_t wlevel(const WLds& L, const WinParams& P, int32_t w_lo, int32_t cur, int32_t F,
                          uint32_t tok, int32_t b, int32_t e, int32_t* need_lo,
                          int32_t* need_hi) {
  constexpr int32_t kPer = 64 / LPV;
  const uint32_t lane = threadIdx.x;
  const uint32_t sub = lane % LPV;
  const int32_t* qc = L.q[cur];
  int32_t* qn = L.q[cur ^ 1];
  const bool one = F <= kPer;
  // every id the level touches must be in the window; a one-chunk level
  // checks the row it has just read, a wider one reads every chunk first
  auto outside = [&](int32_t x, const int32_t* nb, bool act, int32_t& lo, int32_t& hi) {
    bool o = false;
    if (act) {
      o |= !in_window(x, w_lo);
      lo = x < lo ? x : lo;
      hi = x > hi ? x : hi;
#pragma unroll
      for (int j = 0; j < S; ++j) {
        o |= !in_window(nb[j], w_lo);
        lo = nb[j] < lo ? nb[j] : lo;
        hi = nb[j] > hi ? nb[j] : hi;
      }
    }
    return o;
  };
  int32_t lo = 0x7fffffff, hi = -0x7fffffff;
  if (!one) {
    bool out = false;
    for (int32_t q0 = 0; q0 < F; q0 += kPer) {
      const int32_t i = q0 + static_cast<int32_t>(lane / LPV);
      const bool act = i < F;
      const int32_t x = act ? qc[i] : qc[0];
      int32_t nb[S];
      row_part<S>(L, x, sub, nb);
      out |= outside(x, nb, act, lo, hi);
    }
    if (__any(out)) {
      *need_lo = wave_min_i32(lo);
      *need_hi = wave_max_i32(hi);
      return -1;
    }
  }
  if (!kLabel && !one) {
    // A search level wider than one pass of the wave: a token names the
    // lane and slot but not the chunk, so each chunk claims and reads back
    // on its own, and claims only words no earlier chunk or level of this
    // search has claimed (those of earlier searches and kWFree are at least
    // the next larger pass field).
    const uint32_t unclaimed = ((tok >> kWPassShift) + 1u) << kWPassShift;
    int32_t placed = 0;
    for (int32_t q0 = 0; q0 < F; q0 += kPer) {
      const int32_t i = q0 + static_cast<int32_t>(lane / LPV);
      const bool act = i < F;
      const int32_t x = act ? qc[i] : qc[0];
      int32_t nb[S];
      row_part<S>(L, x, sub, nb);
      unsigned cand = 0;
#pragma unroll
      for (int j = 0; j < S; ++j)
        cand |= static_cast<unsigned>(act & (nb[j] != x) &
                                      (lds_ld32(&L.claim[wslot(nb[j])]) >= unclaimed))
                << j;
      const uint32_t mine = tok | (lane << 3);
#pragma unroll
      for (int j = 0; j < S; ++j)
        if (cand >> j & 1u) atomicMin(&L.claim[wslot(nb[j])], mine | static_cast<uint32_t>(j));
      wfence();
      unsigned win = 0;
#pragma unroll
      for (int j = 0; j < S; ++j)
        win |= (cand >> j & 1u &
                static_cast<unsigned>(lds_ld32(&L.claim[wslot(nb[j])]) ==
                                      (mine | static_cast<uint32_t>(j))))
               << j;
      int total;
      const int pre = wprefix(static_cast<uint32_t>(__popc(win)), S == 4 ? 3 : (S == 2 ? 2 : 1),
                              &total);
      if (placed + total > kWQ) return -2;
#pragma unroll
      for (int j = 0; j < S; ++j)
        if (win >> j & 1u) qn[placed + pre + __popc(win & ((1u << j) - 1u))] = nb[j];
      placed += total;
    }
    wfence();
    return placed;
  }
  int32_t x1 = 0, nb1[S];
#pragma unroll
  for (int j = 0; j < S; ++j) nb1[j] = 0;
  // claims (all of the level before any is read back: a labelled pass's
  // claims are unique across chunks, and a search's one chunk needs no test)
  for (int32_t q0 = 0; q0 < F; q0 += kPer) {
    const int32_t i = q0 + static_cast<int32_t>(lane / LPV);
    const bool act = i < F;
    const int32_t x = act ? qc[i] : qc[0];
    int32_t nb[S];
    row_part<S>(L, x, sub, nb);
    if (one && __any(outside(x, nb, act, lo, hi))) {
      *need_lo = wave_min_i32(lo);
      *need_hi = wave_max_i32(hi);
      return -1;
    }
    const uint32_t mine = kLabel ? static_cast<uint32_t>(b + i) + 1u : tok | (lane << 3);
#pragma unroll
    for (int j = 0; j < S; ++j)
      if (act & (nb[j] != x))
        atomicMin(&L.claim[wslot(nb[j])], kLabel ? mine : (mine | static_cast<uint32_t>(j)));
    if (one) {
      x1 = x;
#pragma unroll
      for (int j = 0; j < S; ++j) nb1[j] = nb[j];
    }
  }
  wfence();
  // children / finds: the words read back
  int32_t placed = 0;
  for (int32_t q0 = 0; q0 < F; q0 += kPer) {
    const int32_t i = q0 + static_cast<int32_t>(lane / LPV);
    const bool act = i < F;
    int32_t x, nb[S];
    if (one) {
      x = x1;
#pragma unroll
      for (int j = 0; j < S; ++j) nb[j] = nb1[j];
    } else {
      x = act ? qc[i] : qc[0];
      row_part<S>(L, x, sub, nb);
    }
    const uint32_t mine = kLabel ? static_cast<uint32_t>(b + i) + 1u : tok | (lane << 3);
    unsigned win = 0;
#pragma unroll
    for (int j = 0; j < S; ++j) {
      const uint32_t back = lds_ld32(&L.claim[wslot(nb[j])]);
      const uint32_t want = kLabel ? mine : (mine | static_cast<uint32_t>(j));
      win |= static_cast<unsigned>(act & (nb[j] != x) & (back == want)) << j;
    }
    int total;
    const int pre = wprefix(static_cast<uint32_t>(__popc(win)), S == 4 ? 3 : (S == 2 ? 2 : 1),
                            &total);
    if (placed + total > kWQ) return -2;
#pragma unroll
    for (int j = 0; j < S; ++j) {
      if (!(win >> j & 1u)) continue;
      const int32_t at = placed + pre + __popc(win & ((1u << j) - 1u));
      qn[at] = nb[j];
      // (a label past the component can only come from an asymmetric
      // pattern, which the level's count then reports)
      if (kLabel && e + at < P.size) P.order[e + at] = nb[j];
    }
    placed += total;
  }
  wfence();
  return placed;
}

struct PassOut {
  int32_t ecc;
  int32_t count;
  unsigned long long lastkey;
  int32_t status;  // kPassDone, kDecline, kAsym, kAbort
};

// One level structure (a search, or with kLabel the labelled BFS) from root,
// run by the whole work-group: the first wave walks the levels, the others
// join it for the slides.
template <bool kLabel>
__device__ PassOut window_pass(const WLds& L, WCtl& C, const WinParams& P, int32_t root,
                               uint32_t pass, uint32_t& polls) {
  const bool w0 = threadIdx.x < 64;
  int32_t start_lo = root - kWS / 2;
  slide(L, C, P, start_lo, true);
  // first-wave state, kept across the slides
  int32_t cur = 0, F = 1, level = 0, b = 0, e = 1, count = 1;
  const uint32_t passw = (kWPassTop - pass) << kWPassShift;
  if (threadIdx.x == 0) {
    L.q[0][0] = root;
    L.claim[wslot(root)] = kLabel ? 1u : passw;
    if (kLabel) P.order[0] = root;
  }
  __syncthreads();
  PassOut out{0, 0, kMaxKey, kPassDone};
  while (true) {
    if (w0) {
      int32_t st = kRun;
      int32_t need_lo = 0, need_hi = 0;
      const int32_t w_lo = C.w_lo;
      while (st == kRun) {
        // every 4096 levels: the caller's abort flag
        if (P.abort_flag != nullptr && ((++polls) & 4095u) == 0) {
          const int hit = threadIdx.x == 0 && abort_requested(P.abort_flag) ? 1 : 0;
          if (__shfl(hit, 0, 64)) {
            st = kAbort;
            break;
          }
        }
        if (level >= kWMaxLevel) {
          st = kDecline;  // (the level field of the tokens is full)
          break;
        }
        const uint32_t tok = passw | (static_cast<uint32_t>(level + 2) << kWLevelShift);
        int32_t placed;
        if (F <= 16)
          placed = wlevel<1, 4, kLabel>(L, P, w_lo, cur, F, tok, b, e, &need_lo, &need_hi);
        else if (F <= 32)
          placed = wlevel<2, 2, kLabel>(L, P, w_lo, cur, F, tok, b, e, &need_lo, &need_hi);
        else
          placed = wlevel<4, 1, kLabel>(L, P, w_lo, cur, F, tok, b, e, &need_lo, &need_hi);
        if (placed == -1) {
          int32_t nl = 0;
          st = slide_target(need_lo, need_hi, w_lo, &nl) ? kSlide : kDecline;
          if (threadIdx.x == 0) C.new_lo = nl;
          break;
        }
        if (placed == -2) {
          st = kDecline;
          break;
        }
        if (placed == 0) {
          // the last level is q[cur][0, F): its minimum (degree, caller id)
          unsigned long long k = kMaxKey;
          for (int32_t i = threadIdx.x; i < F; i += 64) {
            const int4 vi = P.vinfo[L.q[cur][i]];
            const unsigned long long kv = pack_key(vi.z, vi.w);
            k = kv < k ? kv : k;
          }
          k = wave_min_u64(k);
          if (threadIdx.x == 0) {
            C.ecc = level;
            C.count = count;
            C.lastkey = k;
          }
          st = kPassDone;
          break;
        }
        count += placed;
        if (count > P.size) {
          st = kAsym;
          break;
        }
        b = e;
        e += placed;
        F = placed;
        cur ^= 1;
        ++level;
      }
      if (threadIdx.x == 0) C.state = st;
    }
    __syncthreads();
    const int32_t st = C.state;
    if (st == kSlide) {
      slide(L, C, P, C.new_lo, false);
      continue;
    }
    out.status = st;
    if (st == kPassDone) {
      out.ecc = C.ecc;
      out.count = C.count;
      out.lastkey = C.lastkey;
    }
    __syncthreads();
    return out;
  }
}

__global__ void __launch_bounds__(kWThreads) k_window_order(WinParams P) {
  extern __shared__ __align__(16) char smem[];
  __shared__ WCtl C;
  __shared__ long long red[16];
  WLds L;
  {
    char* p = smem;
    L.row = reinterpret_cast<uint2*>(p);
    p += 8 * kWS;
    L.claim = reinterpret_cast<uint32_t*>(p);
    p += 4 * kWS;
    L.q[0] = reinterpret_cast<int32_t*>(p);
    p += 4 * kWQ;
    L.q[1] = reinterpret_cast<int32_t*>(p);
  }
  if (threadIdx.x == 0) {
    C.w_lo = 0;
    C.state = kRun;
  }
  if (*P.ell_flag != 0) {
    // a row longer than the records hold: the team kernel takes the component
    if (threadIdx.x == 0) *P.status = kWindowDeclined;
    return;
  }
  // the component's degree sum (every level structure reaches all of it)
  long long m = 0;
  for (int32_t x = threadIdx.x; x < P.size; x += kWThreads) m += P.vinfo[x].z;
  m = block_sum_i64(m, red);
  __syncthreads();
  uint32_t polls = 0, pass = 0;
  // Algorithm 2 from the first level structure's result, as the team
  // kernel continues it after the renumbering: the root of each search is
  // the minimum (degree, caller id) vertex of the previous search's last
  // level; from the third search on, the search is the labelled BFS itself
  int32_t ecc = P.ecc1;
  unsigned long long lastkey = P.lastkey1;
  int32_t nbfs = 1, nlvl = ecc - 1, r = -1, levels = 0;
  bool labelled = false;
  int32_t status = RCM_OK;
  // the renumbered vertex of a key's caller id (-1 for no vertex)
  auto key_vertex = [&](unsigned long long k) {
    const uint32_t id = static_cast<uint32_t>(k & 0xffffffffu);
    return id < static_cast<uint32_t>(P.n) ? P.new_of_old[id] : -1;
  };
  while (ecc > nlvl && status == RCM_OK) {
    nlvl = ecc;
    const int32_t v = key_vertex(lastkey);
    if (v < 0 || v >= P.size) {
      status = kDecline;
      break;
    }
    ++nbfs;
    r = v;
    PassOut o;
    if (P.pp_variant == 0 && nbfs >= 3) {
      if (labelled) {
        // a labelled pass that went deeper: its claims are below every
        // later one, so the component's words go back to unclaimed
        for (int32_t x = threadIdx.x; x < P.size; x += kWThreads) P.claim[x] = kWFree;
        __syncthreads();
      }
      o = window_pass<true>(L, C, P, v, 0, polls);
      labelled = true;
    } else {
      if (++pass >= kWPassTop) {
        status = kDecline;  // more searches than the pass field holds
        break;
      }
      o = window_pass<false>(L, C, P, v, pass, polls);
    }
    if (o.status != kPassDone) {
      status = o.status;
      break;
    }
    if (o.count != P.size) {
      status = kAsym;
      break;
    }
    ecc = o.ecc;
    lastkey = o.lastkey;
    if (labelled) levels = o.ecc + 1;
  }
  const int32_t root = status == RCM_OK && P.pp_variant == 1 ? key_vertex(lastkey) : r;
  if (status == RCM_OK && (root < 0 || root >= P.size)) status = kDecline;
  if (status == RCM_OK) {
    if (!labelled) {
      const PassOut o = window_pass<true>(L, C, P, root, 0, polls);
      if (o.status != kPassDone) status = o.status;
      else if (o.count != P.size) status = kAsym;
      else levels = o.ecc + 1;
    }
    if (status == RCM_OK) {
      // the final labelled pass's order, in the caller's numbering:
      // Cuthill-McKee label t goes to position anchor - t
      for (int32_t t = threadIdx.x; t < P.size; t += kWThreads) {
        const int32_t caller = P.vinfo[P.order[t]].w;
        const int32_t pos = P.anchor - t;
        P.perm[pos] = caller;
        if (P.iperm) P.iperm[caller] = pos;
      }
      if (threadIdx.x == 0) {
        CompResult* res = P.result;
        res->root = P.vinfo[root].w;
        res->nbfs = nbfs;
        res->levels = levels;
        res->size = P.size;
        res->m = m;
      }
    }
  }
  if (threadIdx.x == 0) {
    *P.status = status == RCM_OK ? 0
                : status == kAsym ? static_cast<int32_t>(RCM_ERR_NOT_SYMMETRIC)
                : status == kAbort ? static_cast<int32_t>(RCM_ERR_ABORTED)
                                   : kWindowDeclined;
  }
}

// Rows of the renumbered component as records of 4 columns sorted by
// (degree, caller id), each the 16-bit offset of the neighbour's id from the
// vertex's (0 for a filler); *flag = 1 when a row has more than 4
// off-diagonal entries or a neighbour further than an offset reaches.
__global__ void k_build_ell4(int32_t size, const int32_t* __restrict__ colidx,
                             const int4* __restrict__ vinfo, uint2* __restrict__ ell,
                             int32_t* __restrict__ flag) {
  for (int32_t x = blockIdx.x * blockDim.x + threadIdx.x; x < size;
       x += gridDim.x * blockDim.x) {
    const int4 r = vinfo[x];
    int32_t ids[4] = {x, x, x, x};
    unsigned long long k[4] = {kMaxKey, kMaxKey, kMaxKey, kMaxKey};
    int c = 0;
    bool longrow = r.y - r.x > 5;
    if (!longrow) {
      for (int32_t q = r.x; q < r.y; ++q) {
        const int32_t y = colidx[q];
        if (y == x) continue;
        if (c == 4) {
          longrow = true;
          break;
        }
        if (y - x > 32767 || x - y > 32767) {
          longrow = true;
          break;
        }
        const int4 vy = vinfo[y];
        ids[c] = y;
        k[c] = pack_key(vy.z, vy.w);
        ++c;
      }
    }
    if (longrow) {
      atomicOr(flag, 1);
      continue;
    }
    // 5-comparator sorting network for four keys
    constexpr int kNet[5][2] = {{0, 1}, {2, 3}, {0, 2}, {1, 3}, {1, 2}};
#pragma unroll
    for (int t = 0; t < 5; ++t) {
      const int a = kNet[t][0], bq = kNet[t][1];
      if (k[bq] < k[a]) {
        const unsigned long long tk = k[a];
        k[a] = k[bq];
        k[bq] = tk;
        const int32_t ti = ids[a];
        ids[a] = ids[bq];
        ids[bq] = ti;
      }
    }
    const uint32_t o[4] = {static_cast<uint32_t>(ids[0] - x) & 0xFFFFu,
                           static_cast<uint32_t>(ids[1] - x) & 0xFFFFu,
                           static_cast<uint32_t>(ids[2] - x) & 0xFFFFu,
                           static_cast<uint32_t>(ids[3] - x) & 0xFFFFu};
    ell[x] = make_uint2(o[0] | o[1] << 16, o[2] | o[3] << 16);
  }
}

constexpr size_t kWindowLds = 8 * kWS + 4 * kWS + 2 * 4 * kWQ;

}  // namespace

size_t window_lds_bytes() { return kWindowLds + 1024; }

hipError_t launch_window_order(const WinParams& P, hipStream_t s) {
  if (P.size <= 0) return hipErrorInvalidValue;
  const int blocks = static_cast<int>(std::min<int64_t>((P.size + 255) / 256, 8192));
  hipError_t e = hipMemsetAsync(P.ell_flag, 0, sizeof(int32_t), s);
  if (e != hipSuccess) return e;
  k_build_ell4<<<blocks, 256, 0, s>>>(P.size, P.colidx, P.vinfo, P.ell, P.ell_flag);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  // the whole claim store unclaimed (the first structure's distance words
  // lived here)
  e = hipMemsetAsync(P.claim, 0xFF, sizeof(uint32_t) * static_cast<size_t>(P.size), s);
  if (e != hipSuccess) return e;
  static std::once_flag once;
  static hipError_t attr = hipSuccess;
  std::call_once(once, [] {
    attr = hipFuncSetAttribute(reinterpret_cast<const void*>(k_window_order),
                               hipFuncAttributeMaxDynamicSharedMemorySize,
                               static_cast<int>(kWindowLds));
  });
  if (attr != hipSuccess) return attr;
  k_window_order<<<1, kWThreads, kWindowLds, s>>>(P);
  return hipGetLastError();
}

}  // namespace rcm
