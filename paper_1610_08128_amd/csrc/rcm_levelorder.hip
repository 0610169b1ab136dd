// Level orders: the two alternatives to the per-level sort that the paper
// leaves as future work (Section VI), "no sort" and "one global sort at the
// end".  Both order every component by its root's level structure; within a
// level, "no sort" keeps vertex id order (the order in which the frontier
// vector holds its entries) and the global sort orders by (degree, id), the
// keys SortPerm uses after the parent label.
//
// The ordering kernel leaves, for every vertex, the key anchor - level:
// anchor is the final position of its component's Cuthill-McKee label 0
// (which already accounts for the reversal mode), level its level in the
// root's level structure, so the keys of a component stay inside its block
// and a deeper level gets a smaller key.  The final order is the keys
// ascending and, for equal keys, degree and then id descending: the reverse
// of (level, degree, id) inside each block.  Two stable LSD radix sorts
// produce it, least significant key first: by degree over the vertices in
// descending id order (global sort only), then by key.

#include <hip/hip_runtime.h>

#include <rocprim/device/device_radix_sort.hpp>

#include "rcm_common.hpp"

namespace rcm {
namespace {

constexpr int kThreads = 256;

inline int grid_for(int64_t work) {
  int64_t b = (work + kThreads - 1) / kThreads;
  if (b < 1) b = 1;
  if (b > 8192) b = 8192;
  return static_cast<int>(b);
}

inline unsigned bits_for(int64_t n) {
  unsigned b = 1;
  while (b < 32 && (1ll << b) < n) ++b;
  return b;
}

// vals[i] = n - 1 - i (descending id) and its first sort key: the degree
// complement (ordering by degree) or the position key.
__global__ void k_lo_init(int32_t n, int32_t by_degree, uint32_t deg_max,
                          const int4* __restrict__ vinfo, const int32_t* __restrict__ key,
                          uint32_t* __restrict__ key_out, int32_t* __restrict__ val_out) {
  for (int32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
    const int32_t v = n - 1 - i;
    val_out[i] = v;
    key_out[i] = by_degree ? deg_max - static_cast<uint32_t>(vinfo[v].z)
                           : static_cast<uint32_t>(key[v]);
  }
}

__global__ void k_lo_gather(int32_t n, const int32_t* __restrict__ vals,
                            const int32_t* __restrict__ key, uint32_t* __restrict__ key_out) {
  for (int32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x)
    key_out[i] = static_cast<uint32_t>(key[vals[i]]);
}

__global__ void k_lo_inverse(int32_t n, const int32_t* __restrict__ perm,
                             int32_t* __restrict__ iperm) {
  for (int32_t k = blockIdx.x * blockDim.x + threadIdx.x; k < n; k += gridDim.x * blockDim.x)
    iperm[perm[k]] = k;
}

hipError_t sort_pairs(void* temp, size_t temp_bytes, const uint32_t* kin, uint32_t* kout,
                      const int32_t* vin, int32_t* vout, int32_t n, unsigned end_bit,
                      hipStream_t s) {
  size_t bytes = temp_bytes;
  return rocprim::radix_sort_pairs(temp, bytes, kin, kout, vin, vout, static_cast<unsigned>(n),
                                   0u, end_bit, s);
}

}  // namespace

size_t level_order_temp_bytes(int32_t n) {
  if (n <= 0) return 0;
  size_t bytes = 0;
  if (rocprim::radix_sort_pairs(nullptr, bytes, static_cast<const uint32_t*>(nullptr),
                                static_cast<uint32_t*>(nullptr),
                                static_cast<const int32_t*>(nullptr),
                                static_cast<int32_t*>(nullptr), static_cast<unsigned>(n), 0u,
                                32u) != hipSuccess)
    return 0;
  return bytes;
}

hipError_t launch_level_order(int32_t n, int32_t max_degree_bits, bool by_degree,
                              const int4* vinfo, const int32_t* key, int32_t* perm,
                              int32_t* iperm, void* scratch, void* temp, size_t temp_bytes,
                              hipStream_t s) {
  if (n <= 0) return hipSuccess;
  const size_t N = static_cast<size_t>(n);
  uint32_t* ka = static_cast<uint32_t*>(scratch);
  int32_t* va = reinterpret_cast<int32_t*>(ka + N);
  uint32_t* kb = reinterpret_cast<uint32_t*>(va + N);
  int32_t* vb = reinterpret_cast<int32_t*>(kb + N);
  // keys lie in [0, n); degrees in [0, 2^max_degree_bits)
  const unsigned key_bits = bits_for(n);
  const unsigned deg_bits = static_cast<unsigned>(max_degree_bits);
  const uint32_t deg_max = deg_bits >= 32 ? 0xFFFFFFFFu : ((1u << deg_bits) - 1u);
  const int g = grid_for(n);
  k_lo_init<<<g, kThreads, 0, s>>>(n, by_degree ? 1 : 0, deg_max, vinfo, key, ka, va);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  if (by_degree) {
    e = sort_pairs(temp, temp_bytes, ka, kb, va, vb, n, deg_bits, s);
    if (e != hipSuccess) return e;
    k_lo_gather<<<g, kThreads, 0, s>>>(n, vb, key, ka);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    e = sort_pairs(temp, temp_bytes, ka, kb, vb, perm, n, key_bits, s);
  } else {
    e = sort_pairs(temp, temp_bytes, ka, kb, va, perm, n, key_bits, s);
  }
  if (e != hipSuccess) return e;
  k_lo_inverse<<<g, kThreads, 0, s>>>(n, perm, iperm);
  return hipGetLastError();
}

}  // namespace rcm
