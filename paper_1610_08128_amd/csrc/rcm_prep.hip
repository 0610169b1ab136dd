// Preparation and finishing kernels of the ordering:
//   - CSR checks, degrees and the bandwidth / envelope size of the input
//     order (Section II-A definitions; degrees form the vector D used by
//     Algorithms 3 and 4);
//   - the optional full check (duplicates, symmetry);
//   - connected components by lock-free union-find (the paper orders each
//     component separately, Section III-B), their sizes, seeds (lowest id)
//     and label offsets;
//   - bandwidth / envelope size of the result and per-graph statistics.
// All of this is plain memory-bound integer work: coalesced row scans, one
// random gather per entry, and block-level reductions that issue one global
// atomic per block and segment.

#include "rcm_common.hpp"

namespace rcm {

namespace {

constexpr int kThreads = 256;

inline int grid_for(int64_t work, int threads, int max_blocks = 8192) {
  int64_t b = (work + threads - 1) / threads;
  if (b < 1) b = 1;
  if (b > max_blocks) b = max_blocks;
  return static_cast<int>(b);
}

// ---------------------------------------------------------------------------
// Row checks + degree + beta of the input order.
// ---------------------------------------------------------------------------
// vinfo[i] = (row begin, row end, degree, i): one 16-byte record per vertex,
// read by the traversal in a single load (the last field is the vertex's id
// in the caller's graph, which the (degree, id) keys use; it differs from
// the vertex's number only in a renumbered graph).
//
// A pattern is a set of positions, so a column repeated within a row is a
// malformed input (rows may come in any order).  Rows of up to kDupRegs
// entries are loaded into registers at once and compared pairwise there;
// rows of up to kDupShort entries are compared by re-reading the row (from
// the cache); longer rows raise *long_rows and are checked by k_dup_long.
// With `ell`, the rows of at most kEllWidth entries are also copied there
// from the registers (the traversal's fixed-stride copy); a longer row
// raises *wide_rows, and the copy is then not used.
constexpr int kDupRegs = 16;
constexpr int kDupShort = 64;

__global__ void k_validate_scan(int32_t n, int32_t nnz, const int32_t* __restrict__ rowptr,
                                const int32_t* __restrict__ colidx, int4* __restrict__ vinfo,
                                int32_t* __restrict__ beta, int32_t* __restrict__ err,
                                int32_t* __restrict__ long_rows, int4* __restrict__ ell,
                                int32_t* __restrict__ wide_rows) {
  for (int32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
    const int32_t a = rowptr[i];
    const int32_t b = rowptr[i + 1];
    if (a < 0 || b < a || b > nnz) {
      vinfo[i] = make_int4(0, 0, 0, i);
      beta[i] = 0;
      atomicOr(err, 1);
      continue;
    }
    const int32_t len = b - a;
    int32_t d = 0;
    int32_t mn = i;
    bool bad = false;
    if (len <= kDupRegs) {
      // all loads of the row in flight together (indices clamped into the
      // row; lanes past its end take distinct negative fillers)
      int32_t r[kDupRegs];
#pragma unroll
      for (int j = 0; j < kDupRegs; ++j) {
        const int32_t k = a + (j < len ? j : (len > 0 ? len - 1 : 0));
        const int32_t c = len > 0 ? colidx[k] : 0;
        r[j] = j < len ? c : -1 - j;
      }
#pragma unroll
      for (int j = 0; j < kDupRegs; ++j) {
        if (j >= len) continue;
        const int32_t c = r[j];
        if (c < 0 || c >= n) { bad = true; continue; }
        d += (c != i);
        mn = c < mn ? c : mn;
      }
#pragma unroll
      for (int j = 0; j < kDupRegs; ++j)
#pragma unroll
        for (int k = j + 1; k < kDupRegs; ++k) bad |= r[j] == r[k];
      if (ell != nullptr) {
        if (len <= kEllWidth) {
          // the row, then the vertex itself in the unused places
          static_assert(kEllWidth == 8, "two 16-byte halves a row");
          int32_t e[8];
#pragma unroll
          for (int j = 0; j < 8; ++j) e[j] = j < len ? r[j] : i;
          ell[2 * static_cast<size_t>(i)] = make_int4(e[0], e[1], e[2], e[3]);
          ell[2 * static_cast<size_t>(i) + 1] = make_int4(e[4], e[5], e[6], e[7]);
        } else {
          atomicOr(wide_rows, 1);
        }
      }
    } else {
      if (ell != nullptr) atomicOr(wide_rows, 1);
      for (int32_t k = a; k < b; ++k) {
        const int32_t c = colidx[k];
        if (c < 0 || c >= n) { bad = true; continue; }
        d += (c != i);
        mn = c < mn ? c : mn;
      }
      if (len <= kDupShort) {
        for (int32_t k = a + 1; k < b && !bad; ++k) {
          const int32_t c = colidx[k];
          for (int32_t k2 = a; k2 < k; ++k2) bad |= colidx[k2] == c;
        }
      } else {
        atomicOr(long_rows, 1);
      }
    }
    if (bad) atomicOr(err, 1);
    vinfo[i] = make_int4(a, b, d, i);
    beta[i] = i - mn;
  }
}

// Duplicates in the rows longer than kDupShort: one work-group per row,
// which inserts the row's columns into a hash set in LDS (open addressing,
// atomic compare-and-swap); finding a column already there is a repeat.  A
// row of L entries takes ceil(L / kDupChunk) passes, pass q over the columns
// c with c mod passes == q, so that each pass holds about kDupChunk keys in
// kDupSlots slots.  A pass whose keys fill the table (columns crowded into
// one residue) ends that row's check with the pairwise comparison.  A row
// with more entries than there are columns repeats one by counting.  Only
// launched when k_validate_scan saw such a row; rows with invalid bounds
// were reported there and are skipped.
constexpr int kDupSlotBits = 14;
constexpr int kDupSlots = 1 << kDupSlotBits;  // 64 KB of LDS
constexpr int kDupChunk = kDupSlots / 2;
constexpr uint32_t kDupEmpty = 0xFFFFFFFFu;  // no column (columns are below 2^31)

__global__ void __launch_bounds__(kThreads)
k_dup_long(int32_t n, int32_t nnz, const int32_t* __restrict__ rowptr,
           const int32_t* __restrict__ colidx, int32_t* __restrict__ err) {
  __shared__ uint32_t table[kDupSlots];
  __shared__ int found, full;
  for (int32_t i = blockIdx.x; i < n; i += gridDim.x) {
    const int32_t a = rowptr[i];
    const int32_t b = rowptr[i + 1];
    if (a < 0 || b < a || b > nnz || b - a <= kDupShort) continue;
    const int32_t len = b - a;
    if (len > n) {
      if (threadIdx.x == 0) atomicOr(err, 1);
      continue;
    }
    const uint32_t passes = static_cast<uint32_t>((len + kDupChunk - 1) / kDupChunk);
    if (threadIdx.x == 0) {
      found = 0;
      full = 0;
    }
    for (uint32_t q = 0; q < passes; ++q) {
      for (int t = threadIdx.x; t < kDupSlots; t += blockDim.x) table[t] = kDupEmpty;
      __syncthreads();
      if (full == 0 && found == 0) {
        for (int32_t k = a + threadIdx.x; k < b; k += blockDim.x) {
          const uint32_t c = static_cast<uint32_t>(colidx[k]);
          if (c % passes != q) continue;
          uint32_t h = (c * 2654435761u) >> (32 - kDupSlotBits);
          bool placed = false;
          for (int probe = 0; probe < kDupSlots; ++probe) {
            const uint32_t old = atomicCAS(&table[h], kDupEmpty, c);
            if (old == kDupEmpty) {
              placed = true;
              break;
            }
            if (old == c) {
              found = 1;
              placed = true;
              break;
            }
            h = (h + 1) & (kDupSlots - 1);
          }
          if (!placed) full = 1;
        }
      }
      __syncthreads();
    }
    if (full != 0 && found == 0) {
      // the pairwise comparison for this row
      for (int32_t k = a + threadIdx.x; k < b; k += blockDim.x) {
        const int32_t c = colidx[k];
        bool dup = false;
        for (int32_t k2 = k + 1; k2 < b && !dup; ++k2) dup = colidx[k2] == c;
        if (dup) found = 1;
      }
      __syncthreads();
    }
    if (threadIdx.x == 0 && found) atomicOr(err, 1);
    __syncthreads();
  }
}

// For graphs made of several segments (batched calls), an entry must stay
// inside its row's segment.  Rows whose bounds are invalid are left to
// k_validate_scan's error (this kernel runs before the host reads it, so it
// must not follow them).
// Every column of a graph's rows lies inside that graph.  Blocks take tiles
// of kSegTile consecutive rows, find the graph of a tile's first row once and
// step forward over the graph boundaries inside it.
constexpr int kSegPer = 8;
constexpr int32_t kSegTile = kThreads * kSegPer;

__global__ void k_check_segments(int32_t n, int32_t nnz, const int32_t* __restrict__ rowptr,
                                 const int32_t* __restrict__ colidx,
                                 const int32_t* __restrict__ seg_off, int nseg,
                                 int32_t* __restrict__ err) {
  const int64_t tiles = (static_cast<int64_t>(n) + kSegTile - 1) / kSegTile;
  for (int64_t t = blockIdx.x; t < tiles; t += gridDim.x) {
    const int64_t base = t * kSegTile;
    int s = find_segment(seg_off, nseg, static_cast<int32_t>(base));
    for (int j = 0; j < kSegPer; ++j) {
      const int64_t x = base + static_cast<int64_t>(j) * kThreads + threadIdx.x;
      if (x >= n) break;
      const int32_t i = static_cast<int32_t>(x);
      while (s + 1 < nseg && i >= seg_off[s + 1]) ++s;
      const int32_t lo = seg_off[s], hi = seg_off[s + 1];
      const int32_t a = rowptr[i];
      const int32_t b = rowptr[i + 1];
      if (a < 0 || b < a || b > nnz) continue;
      for (int32_t k = a; k < b; ++k) {
        const int32_t c = colidx[k];
        if (c < lo || c >= hi) { atomicOr(err, 1); break; }
      }
    }
  }
}

// Segmented max/sum of a per-vertex value.  Block b covers
// [b*chunk, (b+1)*chunk); for every segment intersecting it, one block
// reduction and one pair of atomics.  Segments are contiguous vertex ranges.
__global__ void k_seg_reduce(const int32_t* __restrict__ vals, int32_t count, int32_t chunk,
                             const int32_t* __restrict__ seg_off, int nseg,
                             SegStats* __restrict__ out, int which) {
  __shared__ long long red[16];
  const int32_t c0 = blockIdx.x * chunk;
  if (c0 >= count) return;
  const int32_t c1 = min(count, c0 + chunk);
  int s = find_segment(seg_off, nseg, c0);
  for (; s < nseg && seg_off[s] < c1; ++s) {
    const int32_t lo = max(c0, seg_off[s]);
    const int32_t hi = min(c1, seg_off[s + 1]);
    long long mx = 0, sm = 0;
    for (int32_t i = lo + threadIdx.x; i < hi; i += blockDim.x) {
      const long long v = vals[i];
      mx = v > mx ? v : mx;
      sm += v;
    }
    mx = block_max_i64(mx, red);
    sm = block_sum_i64(sm, red);
    if (threadIdx.x == 0 && hi > lo) {
      unsigned long long* pmax = which == 0 ? &out[s].bw_before : &out[s].bw_after;
      unsigned long long* psum = which == 0 ? &out[s].prof_before : &out[s].prof_after;
      atomicMax(pmax, static_cast<unsigned long long>(mx));
      atomicAdd(psum, static_cast<unsigned long long>(sm));
    }
  }
}

// ---------------------------------------------------------------------------
// Full check: duplicates in a row, and (i, j) present => (j, i) present.
// ---------------------------------------------------------------------------
__global__ void k_full_check(int32_t n, const int32_t* __restrict__ rowptr,
                             const int32_t* __restrict__ colidx, int32_t* __restrict__ err_dup,
                             int32_t* __restrict__ err_sym) {
  for (int32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
    const int32_t a = rowptr[i], b = rowptr[i + 1];
    bool dup = false, asym = false;
    for (int32_t k = a; k < b && !dup; ++k) {
      const int32_t c = colidx[k];
      for (int32_t k2 = k + 1; k2 < b; ++k2)
        if (colidx[k2] == c) { dup = true; break; }
    }
    for (int32_t k = a; k < b && !asym; ++k) {
      const int32_t c = colidx[k];
      bool found = false;
      for (int32_t k2 = rowptr[c]; k2 < rowptr[c + 1]; ++k2)
        if (colidx[k2] == i) { found = true; break; }
      asym = !found;
    }
    if (dup) atomicOr(err_dup, 1);
    if (asym) atomicOr(err_sym, 1);
  }
}

// ---------------------------------------------------------------------------
// Connected components: a forest in which every parent is a smaller id of
// the same component, so the final root of each tree is the component's
// lowest id.  Every vertex starts at its smallest neighbour; a few
// contraction rounds (each vertex hooks its root under the smallest root next
// to it, then the forest is flattened) merge most of each component; one
// large set per graph is marked; exact union-find hooking of the other
// vertices' edges finishes the job.  parent[] changes under other
// work-groups' feet, so while it does it is only read with atomic loads.
// ---------------------------------------------------------------------------

// Root of x without writing anything on the way, through agent-scope loads
// (current values).  The compression below must not halve paths: a halving
// store into parent[i] from another thread could land after i's own root
// store and leave i pointing at a non-root.
__device__ __forceinline__ int32_t uf_root(const int32_t* parent, int32_t x) {
  while (true) {
    const int32_t p = ld_relaxed(parent + x);
    if (p == x) return x;
    x = p;
  }
}

// The root as seen through workgroup-scope loads, which the cache may serve
// with an older value than another work-group's store.  The rounds and the
// hooking below tolerate that: every value parent[x] ever holds is x or a
// smaller id in x's set, and a link, once made, is never replaced (hooks
// only swap a root's own entry; flattening only moves an entry up to the
// root).  So an old value is still an ancestor in the same set and a walk
// over old values still descends to smaller ids and ends; a find may stop at
// a vertex that is no longer a root, and the compare-and-swap on that vertex
// then fails and returns its current parent.  Agent-scope loads, which must
// not come from the cache, made every hop of a find a trip to memory.
__device__ __forceinline__ int32_t ld_cached(const int32_t* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

__device__ __forceinline__ int32_t uf_root_cached(const int32_t* parent, int32_t x) {
  while (true) {
    const int32_t p = ld_cached(parent + x);
    if (p == x) return x;
    x = p;
  }
}

// Union-find start: every vertex points at the smallest of itself and its
// neighbours (skipped vertices and edges into them excluded).  That is
// already a forest inside the components -- every link goes to a smaller id
// in the same component -- and most vertices start next to their root.  The
// same pass reads every row once, so it also clears the pick and done marks
// and reports edges into the skipped set: a skipped (already ordered) component
// is closed under adjacency in a symmetric pattern, so such an edge (u, v)
// lacks its (v, u).
__global__ void k_cc_init(int32_t n, const int32_t* __restrict__ rowptr,
                          const int32_t* __restrict__ colidx, const int32_t* __restrict__ skip,
                          int32_t* __restrict__ parent, int32_t* __restrict__ pick,
                          int32_t* __restrict__ done, int32_t* __restrict__ err) {
  for (int32_t u = blockIdx.x * blockDim.x + threadIdx.x; u < n; u += gridDim.x * blockDim.x) {
    int32_t m = u;
    if (!(skip && skip[u] != 0)) {
      bool bad = false;
      for (int32_t k = rowptr[u]; k < rowptr[u + 1]; ++k) {
        const int32_t v = colidx[k];
        if (skip && skip[v] != 0) {
          bad = true;
          continue;
        }
        if (v < m) m = v;
      }
      if (bad) atomicOr(err, 1);
    }
    parent[u] = m;
    pick[u] = 0;
    done[u] = 0;
  }
}

// One contraction round on a flat forest (every parent a root): each vertex
// takes the smallest parent among itself and its neighbours and hooks its
// root under it, with one compare-and-swap from the root itself and no
// retry, so a root is hooked at most once per round and no link is ever
// replaced: sets only grow, and any parent value ever read stays an ancestor
// of the same set.  There are no finds, so a round costs one pass over the
// rows; hooks lost to a failed swap only wait for the next round or the exact
// hooking.  A vertex whose neighbours all showed its own parent has edges
// inside one set only, for good: done[u] = 1 takes it out of the later
// rounds and of the exact hooking.  The first rounds look at only the first
// cap entries of a row (cap 0: all): their gathers are the cost, and a few
// neighbours per vertex already merge most of a component; a vertex is only
// marked done after a look at its whole row.
__global__ void k_cc_round(int32_t n, const int32_t* __restrict__ rowptr,
                           const int32_t* __restrict__ colidx, const int32_t* __restrict__ skip,
                           int32_t cap, int32_t* __restrict__ done, int32_t* parent) {
  for (int32_t u = blockIdx.x * blockDim.x + threadIdx.x; u < n; u += gridDim.x * blockDim.x) {
    if (done[u] != 0 || (skip && skip[u] != 0)) continue;
    const int32_t pu = ld_cached(parent + u);
    int32_t m = pu;
    const int32_t rb = rowptr[u], len = rowptr[u + 1] - rb;
    const int32_t look = cap > 0 && cap < len ? cap : len;
    bool inside = look == len;
    for (int32_t k = rb; k < rb + look; ++k) {
      const int32_t v = colidx[k];
      if (skip && skip[v] != 0) continue;
      const int32_t pv = ld_cached(parent + v);
      inside = inside && pv == pu;
      m = pv < m ? pv : m;
    }
    if (inside) done[u] = 1;
    // all the vertices of a tree aim at one root: read it first, so that only
    // the ones that may still hook it queue an atomic there
    if (m < pu && ld_cached(parent + pu) == pu) {
      int32_t expected = pu;
      __hip_atomic_compare_exchange_strong(parent + pu, &expected, m, __ATOMIC_RELAXED,
                                           __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
  }
}

// The exact hooking: every edge of every vertex, except the vertices whose
// edges the rounds found inside one set (done) and those whose parent is
// marked in pick (see k_cc_pick for why that loses no connection).
// A root is only ever hooked under a smaller root, so whatever the rounds
// before it left undone, the final root of each tree is its component's
// lowest id.
__global__ void k_cc_link(int32_t n, const int32_t* __restrict__ rowptr,
                          const int32_t* __restrict__ colidx, const int32_t* __restrict__ skip,
                          const int32_t* __restrict__ done, const int32_t* __restrict__ pick,
                          int32_t* parent) {
  for (int32_t u = blockIdx.x * blockDim.x + threadIdx.x; u < n; u += gridDim.x * blockDim.x) {
    if (done[u] != 0 || (skip && skip[u] != 0)) continue;
    if (pick && pick[ld_cached(parent + u)] != 0) continue;
    const int32_t rb = rowptr[u], re = rowptr[u + 1];
    if (rb == re) continue;
    // root of u, found once and kept while it stays u's root
    int32_t a = uf_root_cached(parent, u);
    for (int32_t k = rb; k < re; ++k) {
      const int32_t v = colidx[k];
      if (skip && skip[v] != 0) continue;  // reported by k_cc_init
      int32_t b = uf_root_cached(parent, v);
      if (a == b) continue;
      a = uf_root_cached(parent, a);  // a may have been hooked meanwhile
      while (a != b) {
        if (a < b) { const int32_t t = a; a = b; b = t; }
        // hook the larger root a under the smaller root b
        int32_t expected = a;
        if (__hip_atomic_compare_exchange_strong(parent + a, &expected, b, __ATOMIC_RELAXED,
                                                 __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT))
          break;
        a = uf_root_cached(parent, expected);
        b = uf_root_cached(parent, b);
      }
    }
  }
}

// Every parent[i] becomes its root (the only store into parent[i] is this
// one, by the thread that owns i; concurrent readers see either the old
// parent or the root, both ancestors of i).  With flags, the final pass also
// marks the roots of the components to order.
__global__ void k_cc_compress(int32_t n, int32_t* parent, const int32_t* __restrict__ skip,
                              int32_t* __restrict__ flags) {
  for (int32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
    const int32_t r = uf_root(parent, i);
    __hip_atomic_store(parent + i, r, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (flags) flags[i] = (r == i) && !(skip && skip[i] != 0);
  }
}

// After the contraction rounds and a flattening, one work-group per graph
// segment takes kPickSamples evenly spaced vertices and marks the most
// frequent of their roots: in a graph with a giant component that root's set
// already holds most of the vertices.  The exact hooking then passes over
// every vertex whose parent is a marked root, without losing a connection:
// that set is connected already; an edge with an endpoint outside it is
// hooked from that endpoint; and an edge both of whose endpoints are passed
// over joins two vertices that each had the marked root as an ancestor when
// read, so both already lie in one set.  One mark per segment keeps it so:
// segments share no edges, while two marked sets in one component could be
// joined only by edges between them that nobody hooks.
constexpr int kPickSamples = 64;
constexpr int kContractRounds = 4;
constexpr int kCappedRounds = 2;  // the first rounds look at kRoundCap entries
constexpr int32_t kRoundCap = 4;

__global__ void __launch_bounds__(kPickSamples)
k_cc_pick(const int32_t* __restrict__ seg_off, const int32_t* __restrict__ skip,
          const int32_t* parent, int32_t* __restrict__ pick) {
  __shared__ int32_t roots[kPickSamples];
  const int32_t b = seg_off[blockIdx.x], len = seg_off[blockIdx.x + 1] - b;
  const int j = threadIdx.x;
  int32_t r = -1;
  if (len > 0) {
    const int32_t x = b + static_cast<int32_t>(static_cast<int64_t>(len) * (2 * j + 1) /
                                               (2 * kPickSamples));
    if (!(skip && skip[x] != 0)) r = uf_root(parent, x);
  }
  roots[j] = r;
  __syncthreads();
  int32_t c = 0;
  if (r >= 0)
    for (int i = 0; i < kPickSamples; ++i) c += roots[i] == r;
  // most samples first, then the smaller root
  uint64_t key = r >= 0 ? (static_cast<uint64_t>(c) << 32) | static_cast<uint32_t>(0x7FFFFFFF - r)
                        : 0;
  for (int off = kPickSamples / 2; off > 0; off >>= 1) {
    const uint64_t o = __shfl_xor(key, off, kPickSamples);
    key = o > key ? o : key;
  }
  if (j == 0 && key != 0) pick[0x7FFFFFFF - static_cast<int32_t>(key & 0xFFFFFFFFu)] = 1;
}

// Component sizes: histogram of roots with a small LDS hash per block, so a
// giant component costs one global atomic per block.
__global__ void k_cc_sizes(int32_t n, const int32_t* __restrict__ parent,
                           const int32_t* __restrict__ skip, int32_t* __restrict__ csize) {
  constexpr int H = 256;
  __shared__ int32_t keys[H];
  __shared__ int32_t cnts[H];
  for (int h = threadIdx.x; h < H; h += blockDim.x) { keys[h] = -1; cnts[h] = 0; }
  __syncthreads();
  for (int32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
    if (skip && skip[i] != 0) continue;
    const int32_t r = parent[i];
    uint32_t h = (static_cast<uint32_t>(r) * 2654435761u) >> 24;
    bool done = false;
    for (int probe = 0; probe < 8 && !done; ++probe, h = (h + 1) & (H - 1)) {
      int32_t k = keys[h];
      if (k == -1) {
        k = atomicCAS(&keys[h], -1, r);
        if (k == -1) k = r;
      }
      if (k == r) { atomicAdd(&cnts[h], 1); done = true; }
    }
    if (!done) atomicAdd(&csize[r], 1);
  }
  __syncthreads();
  for (int h = threadIdx.x; h < H; h += blockDim.x)
    if (keys[h] >= 0 && cnts[h] > 0) atomicAdd(&csize[keys[h]], cnts[h]);
}

__global__ void k_scatter_seeds(int32_t n, const int32_t* __restrict__ flags,
                                const int32_t* __restrict__ pos, int32_t* __restrict__ seeds) {
  for (int32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x)
    if (flags[i]) seeds[pos[i]] = i;
}

// ---------------------------------------------------------------------------
// Exclusive scan (int32), 4096 elements per block.
// ---------------------------------------------------------------------------
constexpr int kScanPer = 16;
constexpr int kScanTile = kThreads * kScanPer;

__global__ void k_scan_reduce(const int32_t* __restrict__ in, int32_t count,
                              int32_t* __restrict__ sums) {
  __shared__ long long red[16];
  const int32_t base = blockIdx.x * kScanTile;
  long long s = 0;
  for (int j = 0; j < kScanPer; ++j) {
    const int32_t i = base + j * kThreads + threadIdx.x;
    if (i < count) s += in[i];
  }
  s = block_sum_i64(s, red);
  if (threadIdx.x == 0) sums[blockIdx.x] = static_cast<int32_t>(s);
}

__global__ void k_scan_sums(int32_t* __restrict__ sums, int32_t nb, int32_t* __restrict__ total) {
  __shared__ int scratch[17];
  int run = 0;
  for (int32_t b0 = 0; b0 < nb; b0 += blockDim.x) {
    const int32_t i = b0 + threadIdx.x;
    const int x = i < nb ? sums[i] : 0;
    int tot;
    const int ex = block_excl_scan(x, scratch, &tot);
    if (i < nb) sums[i] = run + ex;
    run += tot;
  }
  if (threadIdx.x == 0 && total) *total = run;
}

__global__ void k_scan_apply(const int32_t* __restrict__ in, int32_t* __restrict__ out,
                             int32_t count, const int32_t* __restrict__ sums) {
  __shared__ int scratch[17];
  const int32_t base = blockIdx.x * kScanTile;
  // each thread owns kScanPer consecutive elements
  int vals[kScanPer];
  int local = 0;
  for (int j = 0; j < kScanPer; ++j) {
    const int32_t i = base + threadIdx.x * kScanPer + j;
    vals[j] = i < count ? in[i] : 0;
    local += vals[j];
  }
  int tot;
  int ex = block_excl_scan(local, scratch, &tot);
  int run = sums[blockIdx.x] + ex;
  for (int j = 0; j < kScanPer; ++j) {
    const int32_t i = base + threadIdx.x * kScanPer + j;
    if (i < count) out[i] = run;
    run += vals[j];
  }
}

// ---------------------------------------------------------------------------
// Component tasks.
// ---------------------------------------------------------------------------
__global__ void k_gather_sizes(int32_t ncomp, const int32_t* __restrict__ seeds,
                               const int32_t* __restrict__ csize, int32_t* __restrict__ sizes) {
  for (int32_t c = blockIdx.x * blockDim.x + threadIdx.x; c < ncomp; c += gridDim.x * blockDim.x)
    sizes[c] = csize[seeds[c]];
}

__device__ __forceinline__ void append_task(CompTask* list, int32_t* counter, const CompTask& t) {
  const int32_t at = atomicAdd(counter, 1);
  list[at] = t;
}

// Size class of a component for largest-first ordering: floor(log2(size)).
__device__ __forceinline__ int size_class(int32_t size) { return 31 - __clz(size); }

// Task lists.  Pass 0 writes the per-component results, appends the
// singletons and counts the other components per (list, size class); pass 1
// places them at cursors that k_class_scan laid out in decreasing size-class
// order, so that teams pulling tasks in list order take the largest
// components first (longest-processing-time-first scheduling).
// sched[0..63]: counts of (list l, class c) at l * 32 + c; sched[64..127]:
// the cursors.
__global__ void k_build_tasks(int32_t ncomp, const int32_t* __restrict__ seeds,
                              const int32_t* __restrict__ sizes, const int32_t* __restrict__ offs,
                              const int32_t* __restrict__ seg_off, int nseg, int32_t small_cutoff,
                              int32_t reverse_mode, int32_t offset_base, int32_t index_base,
                              CompTask* tasks_single, CompTask* tasks_small, CompTask* tasks_big,
                              int32_t* counts, CompResult* results, int32_t* sched, int pass) {
  __shared__ int32_t hist[64];
  if (pass == 0) {
    for (int i = threadIdx.x; i < 64; i += blockDim.x) hist[i] = 0;
    __syncthreads();
  }
  for (int32_t c = blockIdx.x * blockDim.x + threadIdx.x; c < ncomp; c += gridDim.x * blockDim.x) {
    CompTask t;
    t.seed = seeds[c];
    t.size = sizes[c];
    t.offset = offset_base + offs[c];
    t.index = index_base + c;
    const int s = find_segment(seg_off, nseg, t.seed);
    // label t of the component (0-based, Cuthill-McKee order) lands at
    // position anchor - t after reversal
    t.anchor = reverse_mode == 0 ? t.offset + t.size - 1
                                 : seg_off[s] + seg_off[s + 1] - 1 - t.offset;
    const int list = t.size <= small_cutoff ? 0 : 1;
    const int slot = list * 32 + size_class(t.size);
    if (pass == 0) {
      CompResult r;
      r.root = t.seed;
      r.nbfs = 0;
      r.levels = 0;
      r.seg = s;
      r.size = t.size;
      r.pad = 0;
      r.m = 0;
      results[t.index] = r;
      if (t.size == 1)
        append_task(tasks_single, counts + 0, t);
      else
        atomicAdd(&hist[slot], 1);
    } else if (t.size > 1) {
      const int32_t at = atomicAdd(&sched[64 + slot], 1);
      (list == 0 ? tasks_small : tasks_big)[at] = t;
    }
  }
  if (pass == 0) {
    __syncthreads();
    for (int i = threadIdx.x; i < 64; i += blockDim.x)
      if (hist[i] != 0) atomicAdd(&sched[i], hist[i]);
  }
}

// One thread: cursors of each list in decreasing size class; list totals
// into counts[1] (small) and counts[2] (big).
__global__ void k_class_scan(int32_t* sched, int32_t* counts) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  for (int l = 0; l < 2; ++l) {
    int32_t run = 0;
    for (int c = 31; c >= 0; --c) {
      sched[64 + l * 32 + c] = run;
      run += sched[l * 32 + c];
    }
    counts[1 + l] = run;
  }
}

__global__ void k_singletons(const CompTask* __restrict__ tasks, int32_t count,
                             int32_t* __restrict__ perm, int32_t* __restrict__ iperm,
                             int32_t* __restrict__ key, CompResult* __restrict__ results) {
  for (int32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < count; i += gridDim.x * blockDim.x) {
    const CompTask t = tasks[i];
    perm[t.anchor] = t.seed;
    iperm[t.seed] = t.anchor;
    if (key) key[t.seed] = t.anchor;
    // an isolated vertex: Algorithm 2 computes two one-level structures
    results[t.index].root = t.seed;
    results[t.index].nbfs = 2;
    results[t.index].levels = 1;
    results[t.index].size = 1;
    results[t.index].m = 0;
  }
}

// ---------------------------------------------------------------------------
// Result statistics.
// ---------------------------------------------------------------------------
// beta of the result, row by row in the input order (so rowptr and colidx
// stream): the row of vertex u becomes row iperm[u]; its beta is that index
// minus the smallest new index among u's neighbours (the diagonal counts as
// present).  Rows are read in batches of eight with clamped loads so that the
// batch's gathers of new indices are in flight together.
__global__ void k_beta_after(int32_t n, const int32_t* __restrict__ rowptr,
                             const int32_t* __restrict__ colidx,
                             const int32_t* __restrict__ iperm, int32_t* __restrict__ beta) {
  constexpr int R = 8;
  for (int32_t u = blockIdx.x * blockDim.x + threadIdx.x; u < n; u += gridDim.x * blockDim.x) {
    const int32_t i = iperm[u];
    const int32_t a = rowptr[u], b = rowptr[u + 1];
    int32_t f = i;
    for (int32_t k0 = a; k0 < b; k0 += R) {
      int32_t c[R];
#pragma unroll
      for (int j = 0; j < R; ++j) {
        const int32_t k = k0 + j < b ? k0 + j : b - 1;
        const int32_t v = colidx[k];
        c[j] = k0 + j < b ? v : u;
      }
      int32_t x[R];
#pragma unroll
      for (int j = 0; j < R; ++j) x[j] = iperm[c[j]];
#pragma unroll
      for (int j = 0; j < R; ++j) f = x[j] < f ? x[j] : f;
    }
    beta[i] = i - f;
  }
}

// Per-segment component counts: comp_seg_off[g] = number of seeds below seg_off[g].
__global__ void k_comp_seg_bounds(int nseg, const int32_t* __restrict__ seg_off,
                                  const int32_t* __restrict__ seeds, int32_t ncomp,
                                  int32_t* __restrict__ comp_seg_off) {
  for (int g = blockIdx.x * blockDim.x + threadIdx.x; g <= nseg; g += gridDim.x * blockDim.x) {
    const int32_t key = seg_off[g];
    int32_t lo = 0, hi = ncomp;
    while (lo < hi) {
      const int32_t mid = (lo + hi) >> 1;
      if (seeds[mid] < key) lo = mid + 1; else hi = mid;
    }
    comp_seg_off[g] = lo;
  }
}

// labelled_bfs: 1 when a labelled BFS ran after the search (its entries
// are counted too), 0 when the search's last level structure was used.
// Per-graph sums over the component results.  A block takes a chunk of
// components, which may span several graphs of a batch; each wave reduces
// its lanes' share of one graph with shuffles and adds it with atomics, so
// the walk over the graphs needs no block-wide barrier.
__device__ __forceinline__ long long wave_sum_i64(long long x) {
  for (int off = 32; off > 0; off >>= 1) x += __shfl_xor(x, off, 64);
  return x;
}
__device__ __forceinline__ long long wave_max_i64(long long x) {
  for (int off = 32; off > 0; off >>= 1) {
    const long long o = __shfl_xor(x, off, 64);
    x = o > x ? o : x;
  }
  return x;
}

__global__ void k_comp_stats(int32_t ncomp, int32_t chunk, const CompResult* __restrict__ res,
                             const int32_t* __restrict__ comp_seg_off, int nseg,
                             int32_t labelled_bfs, SegStats* __restrict__ out) {
  const int32_t c0 = blockIdx.x * chunk;
  if (c0 >= ncomp) return;
  const int32_t c1 = min(ncomp, c0 + chunk);
  int s = find_segment(comp_seg_off, nseg, c0);
  for (; s < nseg && comp_seg_off[s] < c1; ++s) {
    const int32_t lo = max(c0, comp_seg_off[s]);
    const int32_t hi = min(c1, comp_seg_off[s + 1]);
    long long diam = 0, nb = 0, nl = 0, edges = 0, cnt = 0;
    for (int32_t c = lo + threadIdx.x; c < hi; c += blockDim.x) {
      const CompResult r = res[c];
      diam = (r.levels - 1) > diam ? (r.levels - 1) : diam;
      nb += r.nbfs;
      nl += r.levels;
      edges += static_cast<long long>(r.nbfs + labelled_bfs) * r.m;
      ++cnt;
    }
    cnt = wave_sum_i64(cnt);
    if (cnt == 0) continue;  // uniform across the wave
    diam = wave_max_i64(diam);
    nb = wave_sum_i64(nb);
    nl = wave_sum_i64(nl);
    edges = wave_sum_i64(edges);
    if (threadIdx.x % 64 == 0) {
      atomicAdd(&out[s].ncomp, static_cast<int32_t>(cnt));
      atomicMax(&out[s].diameter, static_cast<int32_t>(diam));
      atomicAdd(&out[s].nbfs, static_cast<int32_t>(nb));
      atomicAdd(&out[s].nlevels, static_cast<int32_t>(nl));
      atomicAdd(&out[s].edges, static_cast<unsigned long long>(edges));
    }
  }
}

}  // namespace

// ---------------------------------------------------------------------------
// Launchers.
// ---------------------------------------------------------------------------
hipError_t launch_exclusive_scan(const int32_t* in, int32_t* out, int32_t count, int32_t* tmp,
                                 int32_t* total_out, hipStream_t s) {
  if (count <= 0) {
    if (total_out) return hipMemsetAsync(total_out, 0, sizeof(int32_t), s);
    return hipSuccess;
  }
  const int nb = (count + kScanTile - 1) / kScanTile;
  k_scan_reduce<<<nb, kThreads, 0, s>>>(in, count, tmp);
  k_scan_sums<<<1, 1024, 0, s>>>(tmp, nb, total_out);
  k_scan_apply<<<nb, kThreads, 0, s>>>(in, out, count, tmp);
  return hipGetLastError();
}

hipError_t launch_validate_scan(const Graph& g, int4* vinfo, int32_t* beta, SegStats* seg,
                                int32_t* err, int32_t* long_rows, int4* ell,
                                int32_t* wide_rows, hipStream_t s) {
  k_validate_scan<<<grid_for(g.n, kThreads), kThreads, 0, s>>>(
      g.n, g.nnz, g.rowptr, g.colidx, vinfo, beta, err, long_rows, ell, wide_rows);
  if (g.nseg > 1)
    k_check_segments<<<grid_for((static_cast<int64_t>(g.n) + kSegTile - 1) / kSegTile, 1),
                       kThreads, 0, s>>>(g.n, g.nnz, g.rowptr, g.colidx, g.seg_off, g.nseg, err);
  constexpr int32_t chunk = 8192;
  const int nb = (g.n + chunk - 1) / chunk;
  k_seg_reduce<<<nb, kThreads, 0, s>>>(beta, g.n, chunk, g.seg_off, g.nseg, seg, 0);
  return hipGetLastError();
}

hipError_t launch_dup_long(const Graph& g, int32_t* err, hipStream_t s) {
  k_dup_long<<<grid_for(g.n, 1, 2048), kThreads, 0, s>>>(g.n, g.nnz, g.rowptr, g.colidx, err);
  return hipGetLastError();
}

hipError_t launch_full_check(const Graph& g, int32_t* err_dup, int32_t* err_sym, hipStream_t s) {
  k_full_check<<<grid_for(g.n, kThreads), kThreads, 0, s>>>(g.n, g.rowptr, g.colidx, err_dup,
                                                             err_sym);
  return hipGetLastError();
}

hipError_t launch_components(const Graph& g, const int32_t* skip, int32_t* parent, int32_t* csize,
                             int32_t* flags, int32_t* scan_tmp, int32_t* seeds,
                             int32_t* num_comps, int32_t* err_asym, hipStream_t s) {
  const int nb = grid_for(g.n, kThreads);
  // flags holds the pick marks until the last compression overwrites it;
  // csize the done marks until it is cleared for the sizes
  k_cc_init<<<nb, kThreads, 0, s>>>(g.n, g.rowptr, g.colidx, skip, parent, flags, csize,
                                    err_asym);
  for (int r = 0; r < kContractRounds; ++r) {
    k_cc_compress<<<nb, kThreads, 0, s>>>(g.n, parent, skip, nullptr);
    k_cc_round<<<nb, kThreads, 0, s>>>(g.n, g.rowptr, g.colidx, skip,
                                       r < kCappedRounds ? kRoundCap : 0, csize, parent);
  }
  k_cc_compress<<<nb, kThreads, 0, s>>>(g.n, parent, skip, nullptr);
  if (g.nseg > 0) k_cc_pick<<<g.nseg, kPickSamples, 0, s>>>(g.seg_off, skip, parent, flags);
  k_cc_link<<<nb, kThreads, 0, s>>>(g.n, g.rowptr, g.colidx, skip, csize, flags, parent);
  k_cc_compress<<<nb, kThreads, 0, s>>>(g.n, parent, skip, flags);
  hipError_t e = hipMemsetAsync(csize, 0, sizeof(int32_t) * static_cast<size_t>(g.n), s);
  if (e != hipSuccess) return e;
  k_cc_sizes<<<grid_for(g.n, kThreads, 2048), kThreads, 0, s>>>(g.n, parent, skip, csize);
  // positions of seeds in ascending id order; reuse seeds as the scan output
  // then scatter into seeds' final slots (scan output lives in scan_tmp tail)
  int32_t* pos = scan_tmp;
  int32_t* blk = scan_tmp + g.n;
  e = launch_exclusive_scan(flags, pos, g.n, blk, num_comps, s);
  if (e != hipSuccess) return e;
  k_scatter_seeds<<<nb, kThreads, 0, s>>>(g.n, flags, pos, seeds);
  return hipGetLastError();
}

hipError_t launch_tasks(const Graph& g, int32_t ncomp, const int32_t* seeds, const int32_t* csize,
                        int32_t small_cutoff, int32_t reverse_mode, int32_t offset_base,
                        int32_t index_base, CompTask* tasks_single, CompTask* tasks_small,
                        CompTask* tasks_big, int32_t* counts, int32_t* sizes, int32_t* offs,
                        int32_t* scan_blk, CompResult* results, int32_t* sched, hipStream_t s) {
  const int nb = grid_for(ncomp, kThreads);
  k_gather_sizes<<<nb, kThreads, 0, s>>>(ncomp, seeds, csize, sizes);
  hipError_t e = launch_exclusive_scan(sizes, offs, ncomp, scan_blk, counts + 3, s);
  if (e != hipSuccess) return e;
  e = hipMemsetAsync(counts, 0, 3 * sizeof(int32_t), s);
  if (e != hipSuccess) return e;
  e = hipMemsetAsync(sched, 0, 128 * sizeof(int32_t), s);
  if (e != hipSuccess) return e;
  for (int pass = 0; pass < 2; ++pass) {
    k_build_tasks<<<nb, kThreads, 0, s>>>(ncomp, seeds, sizes, offs, g.seg_off, g.nseg,
                                          small_cutoff, reverse_mode, offset_base, index_base,
                                          tasks_single, tasks_small, tasks_big, counts, results,
                                          sched, pass);
    if (pass == 0) k_class_scan<<<1, 64, 0, s>>>(sched, counts);
  }
  return hipGetLastError();
}

hipError_t launch_singletons(const CompTask* tasks, int32_t count, int32_t* perm, int32_t* iperm,
                             int32_t* key, CompResult* results, hipStream_t s) {
  if (count <= 0) return hipSuccess;
  k_singletons<<<grid_for(count, kThreads), kThreads, 0, s>>>(tasks, count, perm, iperm, key,
                                                              results);
  return hipGetLastError();
}

hipError_t launch_bw_after(const Graph& g, const int32_t* perm, const int32_t* iperm,
                           int32_t* beta, SegStats* seg, hipStream_t s) {
  (void)perm;
  k_beta_after<<<grid_for(g.n, kThreads), kThreads, 0, s>>>(g.n, g.rowptr, g.colidx, iperm, beta);
  constexpr int32_t chunk = 8192;
  const int nb = (g.n + chunk - 1) / chunk;
  k_seg_reduce<<<nb, kThreads, 0, s>>>(beta, g.n, chunk, g.seg_off, g.nseg, seg, 1);
  return hipGetLastError();
}

hipError_t launch_comp_stats(const Graph& g, int32_t ncomp, const int32_t* seeds,
                             const CompResult* results, int32_t* comp_seg_off, SegStats* seg,
                             int32_t labelled_bfs, hipStream_t s) {
  if (ncomp <= 0) return hipSuccess;
  k_comp_seg_bounds<<<grid_for(g.nseg + 1, kThreads), kThreads, 0, s>>>(g.nseg, g.seg_off, seeds,
                                                                       ncomp, comp_seg_off);
  // one wave per chunk of 64 components: a chunk spans few graphs
  constexpr int32_t chunk = 64;
  const int nb = (ncomp + chunk - 1) / chunk;
  k_comp_stats<<<nb, chunk, 0, s>>>(ncomp, chunk, results, comp_seg_off, g.nseg, labelled_bfs,
                                       seg);
  return hipGetLastError();
}

}  // namespace rcm
