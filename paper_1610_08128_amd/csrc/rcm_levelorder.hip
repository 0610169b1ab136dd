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
//
// The radix sort is this file's own: 8-bit digits; per pass a histogram of
// every 2,048-element tile, one exclusive scan over the histograms laid out
// digit-major (so a digit's tiles follow each other), and a stable scatter
// in which each tile ranks its elements per digit in index order, 256 at a
// time, from ballots of the digit's bits within a wave and per-wave counts
// in LDS.

#include <hip/hip_runtime.h>

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

// ---- stable LSD radix sort of (uint32 key, int32 value) pairs ----
constexpr int kDigitBits = 8;
constexpr int kDigits = 1 << kDigitBits;
constexpr int kSortThreads = kDigits;  // one thread per digit in the per-digit steps
constexpr int kSortRounds = 8;         // rounds of kSortThreads elements per tile
constexpr int kSortTile = kSortThreads * kSortRounds;
constexpr int kSortWaves = kSortThreads / 64;

inline int32_t sort_tiles(int32_t n) { return (n + kSortTile - 1) / kSortTile; }

// counts[d * tiles + t] = elements of tile t whose digit at `shift` is d.
__global__ void __launch_bounds__(kSortThreads)
k_rs_hist(const uint32_t* __restrict__ keys, int32_t n, unsigned shift, int32_t tiles,
          int32_t* __restrict__ counts) {
  __shared__ int32_t h[kDigits];
  h[threadIdx.x] = 0;
  __syncthreads();
  const int64_t base = static_cast<int64_t>(blockIdx.x) * kSortTile;
  for (int r = 0; r < kSortRounds; ++r) {
    const int64_t i = base + r * kSortThreads + threadIdx.x;
    if (i < n) atomicAdd(&h[(keys[i] >> shift) & (kDigits - 1)], 1);
  }
  __syncthreads();
  counts[static_cast<int64_t>(threadIdx.x) * tiles + blockIdx.x] = h[threadIdx.x];
}

// Stable scatter of one tile: offs is the exclusive scan of the digit-major
// histograms, so offs[d * tiles + t] is where tile t's first element of
// digit d goes.  Within the tile, elements go out in index order: round r
// takes elements r * 256 .. r * 256 + 255 in thread order; an element's rank
// is the count of its digit in the earlier waves of the round (per-wave
// counts in LDS) plus the earlier lanes of its own wave with the same digit
// (the lanes whose ballots of the eight digit bits all agree with its own).
__global__ void __launch_bounds__(kSortThreads)
k_rs_scatter(const uint32_t* __restrict__ kin, const int32_t* __restrict__ vin,
             uint32_t* __restrict__ kout, int32_t* __restrict__ vout, int32_t n, unsigned shift,
             int32_t tiles, const int32_t* __restrict__ offs) {
  __shared__ int32_t base[kDigits];
  __shared__ int32_t wc[kSortWaves][kDigits];
  __shared__ int32_t wp[kSortWaves][kDigits];
  const int tid = threadIdx.x;
  const int wave = tid >> 6;
  const int lane = tid & 63;
  const unsigned long long below = (1ull << lane) - 1ull;
  base[tid] = offs[static_cast<int64_t>(tid) * tiles + blockIdx.x];
  const int64_t tile0 = static_cast<int64_t>(blockIdx.x) * kSortTile;
  for (int r = 0; r < kSortRounds; ++r) {
#pragma unroll
    for (int w = 0; w < kSortWaves; ++w) wc[w][tid] = 0;
    __syncthreads();
    const int64_t i = tile0 + r * kSortThreads + tid;
    const bool valid = i < n;
    const uint32_t k = valid ? kin[i] : 0u;
    const int32_t v = valid ? vin[i] : 0;
    const int d = static_cast<int>((k >> shift) & (kDigits - 1));
    unsigned long long same = __ballot(valid);
#pragma unroll
    for (int b = 0; b < kDigitBits; ++b) {
      const bool bit = (d >> b) & 1;
      const unsigned long long on = __ballot(bit);
      same &= bit ? on : ~on;
    }
    const int rank = __popcll(same & below);
    if (valid && rank == 0) wc[wave][d] = __popcll(same);
    __syncthreads();
    int32_t run = 0;
#pragma unroll
    for (int w = 0; w < kSortWaves; ++w) {
      wp[w][tid] = run;
      run += wc[w][tid];
    }
    __syncthreads();
    if (valid) {
      const int32_t at = base[d] + wp[wave][d] + rank;
      kout[at] = k;
      vout[at] = v;
    }
    __syncthreads();
    base[tid] += run;
  }
}

// Scratch of one sort: the histograms, their scan and the scan's block sums.
size_t sort_temp_bytes(int32_t n) {
  const size_t c = static_cast<size_t>(kDigits) * static_cast<size_t>(sort_tiles(n));
  return 2 * 4 * c + 4 * (c / 1024 + 64);
}

// Sorts (ka, va) by the key bits [0, end_bit), stably, with (kb, vb) as the
// other buffers; the sorted values end in vfinal (any of the value buffers
// or another array), the keys in whichever key buffer the last pass wrote.
// The last pass writes the values to vfinal directly unless vfinal is that
// pass's own source, in which case they are copied there after it.
hipError_t sort_pairs(void* temp, size_t temp_bytes, uint32_t* ka, int32_t* va, uint32_t* kb,
                      int32_t* vb, int32_t* vfinal, int32_t n, unsigned end_bit,
                      hipStream_t s) {
  if (n <= 0) return hipSuccess;
  if (temp_bytes < sort_temp_bytes(n)) return hipErrorInvalidValue;
  const int32_t tiles = sort_tiles(n);
  const int32_t c = kDigits * tiles;
  int32_t* counts = static_cast<int32_t*>(temp);
  int32_t* offs = counts + c;
  int32_t* blk = offs + c;
  const unsigned passes = end_bit == 0 ? 1u : (end_bit + kDigitBits - 1) / kDigitBits;
  uint32_t* kin = ka;
  int32_t* vin = va;
  uint32_t* kout = kb;
  int32_t* vout = vb;
  for (unsigned p = 0; p < passes; ++p) {
    const unsigned shift = p * kDigitBits;
    if (p + 1 == passes && vfinal != vin) vout = vfinal;
    k_rs_hist<<<tiles, kSortThreads, 0, s>>>(kin, n, shift, tiles, counts);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    e = launch_exclusive_scan(counts, offs, c, blk, nullptr, s);
    if (e != hipSuccess) return e;
    k_rs_scatter<<<tiles, kSortThreads, 0, s>>>(kin, vin, kout, vout, n, shift, tiles, offs);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    // the next pass reads what this one wrote
    uint32_t* kt = kin;
    int32_t* vt = vin;
    kin = kout;
    vin = vout;
    kout = kt;
    vout = vt;
  }
  if (vin != vfinal)
    return hipMemcpyAsync(vfinal, vin, sizeof(int32_t) * static_cast<size_t>(n),
                          hipMemcpyDeviceToDevice, s);
  return hipSuccess;
}

}  // namespace

size_t level_order_temp_bytes(int32_t n) {
  if (n <= 0) return 0;
  return sort_temp_bytes(n);
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
    // by degree into vb, then the keys gathered again in that order
    e = sort_pairs(temp, temp_bytes, ka, va, kb, vb, vb, n, deg_bits, s);
    if (e != hipSuccess) return e;
    k_lo_gather<<<g, kThreads, 0, s>>>(n, vb, key, ka);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    e = sort_pairs(temp, temp_bytes, ka, vb, kb, va, perm, n, key_bits, s);
  } else {
    e = sort_pairs(temp, temp_bytes, ka, va, kb, vb, perm, n, key_bits, s);
  }
  if (e != hipSuccess) return e;
  k_lo_inverse<<<g, kThreads, 0, s>>>(n, perm, iperm);
  return hipGetLastError();
}

}  // namespace rcm
