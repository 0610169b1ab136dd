// Applying an ordering (rcm_apply.h): the permuted matrix B = P A P^T with
// sorted rows, and y = A x as a probe of the locality an ordering buys.
//
// Permutation: new row degrees are gathered and scanned into B's row
// pointer; every row of A is copied to its new place with its columns
// renamed by iperm and sorted: a short row in registers by its thread, a
// long one afterwards by a work-group of its own (a bitonic sort of
// (column, position) pairs, in LDS or, for very long rows, in a scratch
// array).
// Product: a group of eight lanes per row (rows of meshes hold 5 to 13
// entries), each lane striding the row, then a reduction across the group.

#include "rcm_apply.h"

#include <hip/hip_runtime.h>

#include "rcm_common.hpp"

namespace rcm {
namespace {

constexpr int kThreads = 256;

inline size_t align_up(size_t x) { return (x + 255) / 256 * 256; }

inline int grid_for(int64_t work, int threads, int max_blocks = 8192) {
  int64_t b = (work + threads - 1) / threads;
  if (b < 1) b = 1;
  if (b > max_blocks) b = max_blocks;
  return static_cast<int>(b);
}

// Workspace regions of rcm_permute.
struct ApplyLayout {
  size_t deg, blk, keys, vals, sort, total;
};

ApplyLayout apply_layout(int32_t n, int64_t nnz, bool with_values) {
  ApplyLayout L{};
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t at = off;
    off += align_up(bytes);
    return at;
  };
  const size_t N = static_cast<size_t>(n), M = static_cast<size_t>(nnz);
  L.deg = take(4 * N);
  L.blk = take(4 * (N / 4096 + 2));
  L.keys = take(4 * M);
  L.vals = with_values ? take(8 * M) : 0;
  L.sort = take(8 * M);  // (column, position) pairs of rows too long for LDS
  L.total = off;
  return L;
}

__global__ void k_new_degrees(int32_t n, const int32_t* __restrict__ rowptr,
                              const int32_t* __restrict__ perm, int32_t* __restrict__ deg) {
  for (int32_t k = blockIdx.x * blockDim.x + threadIdx.x; k < n; k += gridDim.x * blockDim.x) {
    const int32_t v = perm[k];
    deg[k] = rowptr[v + 1] - rowptr[v];
  }
}

// Row k of B: row perm[k] of A with its columns renamed by iperm.  A row of
// at most kSortReg entries is sorted in registers by one thread, with a fixed
// network of compare-and-swaps of neighbours on strictly greater keys (the
// insertion order, so equal keys keep their input order).  A longer row goes
// to keys / vals_tmp in input order, and k to the list of long rows, which
// k_sort_long_rows sorts.
//
// A block takes kMoveRows consecutive rows of B, whose entries are one
// contiguous range of the output.  If that range fits kStage entries, the
// sorted rows are staged in LDS and the range is written out coalesced (the
// slots of long rows carry nothing; k_sort_long_rows, later on the same
// stream, writes them); otherwise each thread writes its row itself.
constexpr int kSortReg = 16;
constexpr int kMoveRows = 256;
constexpr int kStage = kMoveRows * kSortReg;

__global__ void __launch_bounds__(kMoveRows)
k_move_rows(int32_t n, const int32_t* __restrict__ rowptr, const int32_t* __restrict__ colidx,
            const double* __restrict__ vals, const int32_t* __restrict__ perm,
            const int32_t* __restrict__ iperm, const int32_t* __restrict__ rowptr_out,
            int32_t* __restrict__ keys, double* __restrict__ vals_tmp,
            int32_t* __restrict__ colidx_out, double* __restrict__ vals_out,
            int32_t* __restrict__ long_rows, int32_t* __restrict__ long_count) {
  __shared__ int32_t sc[kStage];
  __shared__ double sx[kStage];
  for (int64_t t = blockIdx.x; t * kMoveRows < n; t += gridDim.x) {
    const int32_t k0 = static_cast<int32_t>(t * kMoveRows);
    const int32_t k1 = min(n, k0 + kMoveRows);
    const int32_t O0 = rowptr_out[k0], span = rowptr_out[k1] - O0;
    const bool stage = span <= kStage;  // the same for the whole block
    const int32_t k = k0 + static_cast<int32_t>(threadIdx.x);
    if (k < k1) {
      const int32_t v = perm[k];
      const int32_t a = rowptr[v], len = rowptr[v + 1] - a;
      const int32_t o = rowptr_out[k];
      if (len > kSortReg) {
        for (int32_t e = 0; e < len; ++e) {
          keys[o + e] = iperm[colidx[a + e]];
          if (vals) vals_tmp[o + e] = vals[a + e];
        }
        long_rows[atomicAdd(long_count, 1)] = k;
      } else {
        int32_t c[kSortReg];
        double x[kSortReg];
#pragma unroll
        for (int j = 0; j < kSortReg; ++j) {
          // past the row: a key above every column, so it sorts last
          c[j] = j < len ? iperm[colidx[a + j]] : 0x7FFFFFFF;
          x[j] = (vals && j < len) ? vals[a + j] : 0.0;
        }
#pragma unroll
        for (int i = 1; i < kSortReg; ++i) {
#pragma unroll
          for (int j = i; j > 0; --j) {
            const bool sw = c[j - 1] > c[j];
            const int32_t lo = sw ? c[j] : c[j - 1], hi = sw ? c[j - 1] : c[j];
            const double xl = sw ? x[j] : x[j - 1], xh = sw ? x[j - 1] : x[j];
            c[j - 1] = lo;
            c[j] = hi;
            x[j - 1] = xl;
            x[j] = xh;
          }
        }
#pragma unroll
        for (int j = 0; j < kSortReg; ++j) {
          if (j < len) {
            if (stage) {
              sc[o - O0 + j] = c[j];
              if (vals) sx[o - O0 + j] = x[j];
            } else {
              colidx_out[o + j] = c[j];
              if (vals) vals_out[o + j] = x[j];
            }
          }
        }
      }
    }
    if (stage) {
      __syncthreads();
      for (int32_t i = threadIdx.x; i < span; i += kMoveRows) {
        colidx_out[O0 + i] = sc[i];
        if (vals) vals_out[O0 + i] = sx[i];
      }
      __syncthreads();
    }
  }
}

// The long rows: one work-group per row (a grid-stride loop over the list
// k_move_rows made).  The row's entries become (column << 32 | position)
// pairs, distinct even if a column repeats, so the sort puts equal columns
// in input order as the short rows do, and the values follow their
// positions.  They are sorted by a bitonic network whose comparators all
// put the smaller pair first (each merge starts by comparing mirrored
// positions), so positions past the row can stand for pairs above every
// other without being stored: a comparator that would reach one is a no-op.
// Rows of up to kLongLds entries sort in LDS, longer ones in place in the
// scratch array, with a barrier of the work-group between the steps.
constexpr int kLongThreads = 256;
constexpr int kLongLds = 8192;

__device__ __forceinline__ void bitonic_pairs(unsigned long long* a, int32_t len, int32_t pow2) {
  for (int32_t k = 2; k <= pow2; k <<= 1) {
    for (int32_t j = k >> 1; j > 0; j >>= 1) {
      for (int32_t i = threadIdx.x; i < pow2; i += kLongThreads) {
        const int32_t p = j == (k >> 1) ? (i ^ (k - 1)) : (i ^ j);
        if (p > i && p < len) {
          const unsigned long long x = a[i], y = a[p];
          if (y < x) {
            a[i] = y;
            a[p] = x;
          }
        }
      }
      __syncthreads();
    }
  }
}

__global__ void __launch_bounds__(kLongThreads)
k_sort_long_rows(const int32_t* __restrict__ rowptr_out, const int32_t* __restrict__ long_rows,
                 const int32_t* __restrict__ long_count, const int32_t* __restrict__ keys,
                 const double* __restrict__ vals_tmp, unsigned long long* __restrict__ pairs,
                 int32_t* __restrict__ colidx_out, double* __restrict__ vals_out) {
  __shared__ unsigned long long sp[kLongLds];
  const int32_t count = *long_count;
  for (int32_t r = blockIdx.x; r < count; r += gridDim.x) {
    const int32_t k = long_rows[r];
    const int32_t o = rowptr_out[k];
    const int32_t len = rowptr_out[k + 1] - o;
    int32_t pow2 = 1;
    while (pow2 < len) pow2 <<= 1;
    unsigned long long* a = len <= kLongLds ? sp : pairs + o;
    for (int32_t i = threadIdx.x; i < len; i += kLongThreads)
      a[i] = (static_cast<unsigned long long>(static_cast<uint32_t>(keys[o + i])) << 32) |
             static_cast<uint32_t>(i);
    __syncthreads();
    bitonic_pairs(a, len, pow2);
    for (int32_t i = threadIdx.x; i < len; i += kLongThreads) {
      const unsigned long long x = a[i];
      colidx_out[o + i] = static_cast<int32_t>(x >> 32);
      if (vals_out) vals_out[o + i] = vals_tmp[o + static_cast<uint32_t>(x)];
    }
    __syncthreads();
  }
}

constexpr int kGroup = 8;  // lanes per row in the product

__global__ void __launch_bounds__(256) k_spmv(int32_t n, const int32_t* __restrict__ rowptr,
                                              const int32_t* __restrict__ colidx,
                                              const double* __restrict__ vals,
                                              const double* __restrict__ x,
                                              double* __restrict__ y) {
  const int lane = threadIdx.x % kGroup;
  const int64_t groups = static_cast<int64_t>(gridDim.x) * (blockDim.x / kGroup);
  for (int64_t row = (static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x) / kGroup;
       row < n; row += groups) {
    const int32_t a = rowptr[row], b = rowptr[row + 1];
    double s = 0.0;
    for (int32_t e = a + lane; e < b; e += kGroup) {
      const double w = vals ? vals[e] : 1.0;
      s = fma(w, x[colidx[e]], s);
    }
#pragma unroll
    for (int off = kGroup / 2; off > 0; off >>= 1) s += __shfl_xor(s, off, kGroup);
    if (lane == 0) y[row] = s;
  }
}

}  // namespace
}  // namespace rcm

using namespace rcm;

extern "C" {

size_t rcm_permute_workspace_bytes(int32_t n, int64_t nnz, int32_t with_values) {
  if (n <= 0 || nnz < 0 || nnz >= (1ll << 31) - 1) return 0;
  return apply_layout(n, nnz, with_values != 0).total;
}

rcm_status rcm_permute(int32_t n, int64_t nnz, const int32_t* rowptr, const int32_t* colidx,
                       const double* vals, const int32_t* perm, const int32_t* iperm,
                       int32_t* rowptr_out, int32_t* colidx_out, double* vals_out,
                       void* workspace, size_t workspace_bytes, void* stream) {
  if (n < 0 || nnz < 0 || nnz >= (1ll << 31) - 1) return RCM_ERR_INVALID_ARGUMENT;
  if (n == 0) return RCM_OK;
  if (!rowptr || !perm || !iperm || !rowptr_out || (nnz > 0 && (!colidx || !colidx_out)))
    return RCM_ERR_INVALID_ARGUMENT;
  if (vals && !vals_out) return RCM_ERR_INVALID_ARGUMENT;
  const ApplyLayout L = apply_layout(n, nnz, vals != nullptr);
  if (!workspace || workspace_bytes < L.total) return RCM_ERR_WORKSPACE_TOO_SMALL;
  hipStream_t s = static_cast<hipStream_t>(stream);
  char* ws = static_cast<char*>(workspace);
  int32_t* deg = reinterpret_cast<int32_t*>(ws + L.deg);
  int32_t* blk = reinterpret_cast<int32_t*>(ws + L.blk);
  int32_t* keys = reinterpret_cast<int32_t*>(ws + L.keys);
  double* vtmp = vals ? reinterpret_cast<double*>(ws + L.vals) : nullptr;
  unsigned long long* pairs = reinterpret_cast<unsigned long long*>(ws + L.sort);
  k_new_degrees<<<grid_for(n, kThreads), kThreads, 0, s>>>(n, rowptr, perm, deg);
  if (hipGetLastError() != hipSuccess) return RCM_ERR_HIP;
  if (launch_exclusive_scan(deg, rowptr_out, n, blk, rowptr_out + n, s) != hipSuccess)
    return RCM_ERR_HIP;
  if (nnz == 0) return RCM_OK;
  // the degrees are scanned by now: deg takes the list of long rows, and
  // the scan's block sums (free again) its length
  int32_t* long_rows = deg;
  int32_t* long_count = blk;
  if (hipMemsetAsync(long_count, 0, sizeof(int32_t), s) != hipSuccess) return RCM_ERR_HIP;
  k_move_rows<<<grid_for(n, kMoveRows), kMoveRows, 0, s>>>(n, rowptr, colidx, vals, perm, iperm,
                                                          rowptr_out, keys, vtmp, colidx_out,
                                                          vals_out, long_rows, long_count);
  if (hipGetLastError() != hipSuccess) return RCM_ERR_HIP;
  k_sort_long_rows<<<1024, kLongThreads, 0, s>>>(rowptr_out, long_rows, long_count, keys, vtmp,
                                                 pairs, colidx_out, vals_out);
  return hipGetLastError() == hipSuccess ? RCM_OK : RCM_ERR_HIP;
}

rcm_status rcm_spmv(int32_t n, const int32_t* rowptr, const int32_t* colidx, const double* vals,
                    const double* x, double* y, void* stream) {
  if (n < 0) return RCM_ERR_INVALID_ARGUMENT;
  if (n == 0) return RCM_OK;
  if (!rowptr || !x || !y) return RCM_ERR_INVALID_ARGUMENT;
  hipStream_t s = static_cast<hipStream_t>(stream);
  const int blocks = grid_for(static_cast<int64_t>(n) * kGroup, kThreads, 1 << 16);
  k_spmv<<<blocks, kThreads, 0, s>>>(n, rowptr, colidx, vals, x, y);
  return hipGetLastError() == hipSuccess ? RCM_OK : RCM_ERR_HIP;
}

}  // extern "C"
