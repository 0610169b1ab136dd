// Locality renumbering of a long component (the ordering's data layout, not
// part of the method: the result is the same in any numbering, since every
// tie is broken by the caller's vertex ids).
//
// A graph with many levels (a long mesh) spends its ordering time walking
// narrow levels one after another, each level a couple of dependent random
// loads; with the caller's (random) vertex numbers every load touches a new
// line and often a new page.  Renumbered in the level order of its first
// level structure, the vertices of consecutive levels sit next to each
// other, and so do their rows, so the later passes' loads hit the caches.
//
// Input: the distances of the component's first (asynchronous) level
// structure, in the distance words (pass tag << 32 | ~distance); vertices
// without the pass's tag belong to other components and keep out.  Steps:
//   1. a histogram of the distances;
//   2. its exclusive scan: the first new number of every level;
//   3. every vertex of the component takes the next number of its level
//      (atomically, in any order within the level);
//   4. the new row lengths, scanned into the new row pointers;
//   5. the rows, copied with their columns renumbered, and the new vertex
//      records (row begin, row end, degree, caller id).

#include "rcm_common.hpp"

namespace rcm {

namespace {

constexpr int kThreads = 256;

inline int grid(int64_t work, int max_blocks = 8192) {
  const int64_t b = (work + kThreads - 1) / kThreads;
  return static_cast<int>(b < 1 ? 1 : (b > max_blocks ? max_blocks : b));
}

__device__ __forceinline__ int32_t distance_of(unsigned long long kv) {
  return static_cast<int32_t>(0xFFFFFFFFu - static_cast<uint32_t>(kv));
}

__global__ void k_rl_hist(int32_t n, const unsigned long long* __restrict__ dkey, uint32_t tag,
                          int32_t ecc, int32_t* __restrict__ hist, int32_t* __restrict__ err) {
  for (int32_t v = blockIdx.x * blockDim.x + threadIdx.x; v < n; v += gridDim.x * blockDim.x) {
    const unsigned long long kv = dkey[v];
    if (static_cast<uint32_t>(kv >> 32) != tag) continue;  // another component
    const int32_t d = distance_of(kv);
    if (d < 0 || d > ecc) {
      atomicOr(err, 1);
      continue;
    }
    atomicAdd(&hist[d], 1);
  }
}

__global__ void k_rl_place(int32_t n, const unsigned long long* __restrict__ dkey, uint32_t tag,
                           int32_t ecc, const int32_t* __restrict__ first,
                           int32_t* __restrict__ cursor, int32_t* __restrict__ new_of_old,
                           int32_t* __restrict__ old_of_new) {
  for (int32_t v = blockIdx.x * blockDim.x + threadIdx.x; v < n; v += gridDim.x * blockDim.x) {
    const unsigned long long kv = dkey[v];
    const int32_t d = distance_of(kv);
    if (static_cast<uint32_t>(kv >> 32) != tag || d < 0 || d > ecc) continue;  // flagged
    const int32_t k = first[d] + atomicAdd(&cursor[d], 1);
    new_of_old[v] = k;
    old_of_new[k] = v;
  }
}

__global__ void k_rl_len(int32_t n, const int32_t* __restrict__ old_of_new,
                         const int4* __restrict__ vinfo, int32_t* __restrict__ len) {
  for (int32_t k = blockIdx.x * blockDim.x + threadIdx.x; k < n; k += gridDim.x * blockDim.x) {
    const int4 r = vinfo[old_of_new[k]];
    len[k] = r.y - r.x;
  }
}

// One thread per new vertex: its row, columns renumbered, and its record.
// Entries past cap (only when the counts disagree, which the caller
// rejects) are flagged instead of written.
__global__ void k_rl_fill(int32_t n, const int32_t* __restrict__ old_of_new,
                         const int32_t* __restrict__ new_of_old, const int4* __restrict__ vinfo,
                         const int32_t* __restrict__ colidx, const int32_t* __restrict__ rowptr_new,
                         int64_t cap, int32_t* __restrict__ colidx_new,
                         int4* __restrict__ vinfo_new, int32_t* __restrict__ err) {
  for (int32_t k = blockIdx.x * blockDim.x + threadIdx.x; k < n; k += gridDim.x * blockDim.x) {
    const int32_t o = old_of_new[k];
    const int4 r = vinfo[o];
    const int32_t b = rowptr_new[k];
    if (b < 0 || static_cast<int64_t>(b) + (r.y - r.x) > cap) {
      atomicOr(err, 1);
      continue;
    }
    for (int32_t j = 0; j < r.y - r.x; ++j) colidx_new[b + j] = new_of_old[colidx[r.x + j]];
    vinfo_new[k] = make_int4(b, b + (r.y - r.x), r.z, r.w);
  }
}

}  // namespace

hipError_t launch_relabel(const Graph& g, const int4* vinfo, const unsigned long long* dkey,
                          uint32_t tag, int32_t ecc, int32_t size, int32_t* hist, int32_t* first,
                          int32_t* cursor, int32_t* scan_tmp, int32_t* new_of_old,
                          int32_t* old_of_new, int32_t* rowptr_new, int32_t* colidx_new,
                          int64_t cap, int4* vinfo_new, int32_t* err, int32_t* counted,
                          hipStream_t s) {
  const int32_t n = g.n;
  const int32_t levels = ecc + 1;
  // both maps start at 0, so that even with a vertex missing (err set; the
  // caller then discards everything) every entry is a valid vertex number
  hipError_t e = hipMemsetAsync(hist, 0, sizeof(int32_t) * levels, s);
  if (e == hipSuccess) e = hipMemsetAsync(cursor, 0, sizeof(int32_t) * levels, s);
  if (e == hipSuccess) e = hipMemsetAsync(new_of_old, 0, sizeof(int32_t) * n, s);
  if (e == hipSuccess) e = hipMemsetAsync(old_of_new, 0, sizeof(int32_t) * n, s);
  if (e != hipSuccess) return e;
  k_rl_hist<<<grid(n), kThreads, 0, s>>>(n, dkey, tag, ecc, hist, err);
  // the first number of each level; the total is the component's size
  e = launch_exclusive_scan(hist, first, levels, scan_tmp, counted, s);
  if (e != hipSuccess) return e;
  k_rl_place<<<grid(n), kThreads, 0, s>>>(n, dkey, tag, ecc, first, cursor, new_of_old,
                                          old_of_new);
  // row lengths in the new order (in cursor, free again), scanned into the
  // new row pointers; rowptr_new[size] (the component's entries) is the
  // scan's total.  old_of_new holds a vertex of the component at every new
  // number below size when counted == size, which the caller checks before
  // it uses the result; otherwise the zeros above keep every index valid.
  k_rl_len<<<grid(size), kThreads, 0, s>>>(size, old_of_new, vinfo, cursor);
  e = launch_exclusive_scan(cursor, rowptr_new, size, scan_tmp, rowptr_new + size, s);
  if (e != hipSuccess) return e;
  k_rl_fill<<<grid(size), kThreads, 0, s>>>(size, old_of_new, new_of_old, vinfo, g.colidx,
                                            rowptr_new, cap, colidx_new, vinfo_new, err);
  return hipGetLastError();
}

}  // namespace rcm
