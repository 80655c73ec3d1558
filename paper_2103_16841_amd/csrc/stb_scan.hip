// stb_scan.hip -- exclusive prefix sums of per-item counts on the device.
//
// Every list the library lays out (cull candidates per row, lit combos per
// candidate, face candidates, matrix-core quads per block, causal entries
// per row) gets its offsets from one of these scans.  Tiles of 4096 items
// per workgroup: each of the 256 lanes owns 16 consecutive items; a lane
// scans its items serially, the 64 lanes of a wavefront combine their
// totals by a shuffle-up prefix sum, and the four wavefronts by their
// totals in LDS.  Three passes over the device: tile totals, an exclusive
// scan of the tile totals by one workgroup (in chunks of 4096 with a
// carry), and the tiles again with their offsets.  Loads and stores go
// through LDS so that global accesses stay coalesced.  Integer sums: the
// result does not depend on the schedule.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "stb_internal.h"

namespace {

constexpr int kScanThreads = 256;
constexpr int kScanPer = 16;
constexpr int kScanTile = kScanThreads * kScanPer;   // 4096 items per workgroup
constexpr int kWaves = kScanThreads / 64;

// Inclusive prefix sum over the wavefront (lane order).
template <typename T>
__device__ __forceinline__ T wave_inclusive(T v, int lane) {
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    const T y = __shfl_up(v, off, 64);
    if (lane >= off) v += y;
  }
  return v;
}

// Exclusive prefix of the lanes' values over the workgroup, and the total.
template <typename T>
__device__ __forceinline__ T block_exclusive(T v, T* total) {
  __shared__ T wsum[kWaves];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const T inc = wave_inclusive(v, lane);
  if (lane == 63) wsum[wave] = inc;
  __syncthreads();
  T before = 0, all = 0;
#pragma unroll
  for (int w = 0; w < kWaves; ++w) {
    before += w < wave ? wsum[w] : T(0);
    all += wsum[w];
  }
  __syncthreads();   // wsum is reused by the next call
  *total = all;
  return before + inc - v;
}

// Pass 1: the total of each tile.
template <typename T>
__global__ __launch_bounds__(kScanThreads) void k_scan_tile_sums(const T* __restrict__ in, int64_t n,
                                                                 T* __restrict__ sums) {
  const int64_t base = (int64_t)blockIdx.x * kScanTile;
  T s = 0;
#pragma unroll
  for (int k = 0; k < kScanPer; ++k) {
    const int64_t i = base + (int64_t)k * kScanThreads + threadIdx.x;
    if (i < n) s += in[i];
  }
  T tot;
  (void)block_exclusive(s, &tot);
  if (threadIdx.x == 0) sums[blockIdx.x] = tot;
}

// Pass 2: exclusive scan of the nb tile totals in place, one workgroup.
template <typename T>
__global__ __launch_bounds__(kScanThreads) void k_scan_sums(T* __restrict__ sums, int64_t nb) {
  T carry = 0;
  for (int64_t c0 = 0; c0 < nb; c0 += kScanTile) {
    T v[kScanPer];
    T s = 0;
#pragma unroll
    for (int k = 0; k < kScanPer; ++k) {
      const int64_t i = c0 + (int64_t)threadIdx.x * kScanPer + k;
      v[k] = i < nb ? sums[i] : T(0);
      s += v[k];
    }
    T tot;
    T run = carry + block_exclusive(s, &tot);
#pragma unroll
    for (int k = 0; k < kScanPer; ++k) {
      const int64_t i = c0 + (int64_t)threadIdx.x * kScanPer + k;
      if (i < nb) sums[i] = run;
      run += v[k];
    }
    carry += tot;
    __syncthreads();
  }
}

// Pass 3: each tile scanned with its offset; out[i + 1] = sum_{k <= i} in[k],
// out[0] = 0.
template <typename T>
__global__ __launch_bounds__(kScanThreads) void k_scan_tiles(const T* __restrict__ in, int64_t n,
                                                             const T* __restrict__ sums,
                                                             T* __restrict__ out) {
  __shared__ T tile[kScanTile];
  const int64_t base = (int64_t)blockIdx.x * kScanTile;
#pragma unroll
  for (int k = 0; k < kScanPer; ++k) {
    const int j = k * kScanThreads + threadIdx.x;
    tile[j] = base + j < n ? in[base + j] : T(0);
  }
  __syncthreads();
  T v[kScanPer];
  T s = 0;
#pragma unroll
  for (int k = 0; k < kScanPer; ++k) {
    v[k] = tile[threadIdx.x * kScanPer + k];
    s += v[k];
  }
  T tot;
  T run = sums[blockIdx.x] + block_exclusive(s, &tot);
#pragma unroll
  for (int k = 0; k < kScanPer; ++k) {
    run += v[k];
    tile[threadIdx.x * kScanPer + k] = run;   // inclusive
  }
  __syncthreads();
#pragma unroll
  for (int k = 0; k < kScanPer; ++k) {
    const int j = k * kScanThreads + threadIdx.x;
    if (base + j < n) out[base + j + 1] = tile[j];
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) out[0] = 0;
}

}  // namespace

template <typename T>
int64_t stb_scan_tmp_elems(int64_t n) {
  const int64_t nb = (n + kScanTile - 1) / kScanTile;
  return nb > 0 ? nb : 1;
}

template <typename T>
hipError_t stb_scan(const T* in, T* out, int64_t n, T* tmp, hipStream_t st) {
  if (n < 0) return hipErrorInvalidValue;
  const int64_t nb = stb_scan_tmp_elems<T>(n);
  if (nb > (int64_t)0x7fffffff) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_scan_tile_sums<T>, dim3((unsigned)nb), dim3(kScanThreads), 0, st, in, n, tmp);
  hipLaunchKernelGGL(k_scan_sums<T>, dim3(1), dim3(kScanThreads), 0, st, tmp, nb);
  hipLaunchKernelGGL(k_scan_tiles<T>, dim3((unsigned)nb), dim3(kScanThreads), 0, st, in, n, tmp, out);
  return hipGetLastError();
}

template int64_t stb_scan_tmp_elems<int32_t>(int64_t);
template int64_t stb_scan_tmp_elems<int64_t>(int64_t);
template hipError_t stb_scan<int32_t>(const int32_t*, int32_t*, int64_t, int32_t*, hipStream_t);
template hipError_t stb_scan<int64_t>(const int64_t*, int64_t*, int64_t, int64_t*, hipStream_t);
