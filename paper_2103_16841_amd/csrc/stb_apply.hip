// stb_apply.hip -- multi right-hand-side product Y = A W (16 columns) on the
// CDNA4 matrix cores.  With 16 right-hand sides the product is a real GEMM
// over the sparse store: per block of 16 rows, the union of its rows'
// candidate columns is packed into quads, and each quad is one
// v_mfma_f32_16x16x4f32 step, A (16 rows x 4 columns, FP32) times W (4 rows x
// 16 right-hand sides, FP32) accumulated in FP32.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "stb_internal.h"

typedef float f32x4 __attribute__((ext_vector_type(4)));

// One wavefront per 16-row block.  MFMA 16x16x4 (FP32) operand layout:
//   A: lane l holds A[l % 16][l / 16];  B: lane l holds B[l / 16][l % 16];
//   D: lane l, register v holds D[4 (l / 16) + v][l % 16].
__global__ __launch_bounds__(256) void k_bell_mfma(int64_t nblk, int64_t n,
                                                   const int64_t* __restrict__ bptr,
                                                   const int32_t* __restrict__ bcol,
                                                   const float* __restrict__ bval,
                                                   const float* __restrict__ w32,
                                                   double* __restrict__ y) {
  int64_t blk = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  int lane = threadIdx.x & 63;
  if (blk >= nblk) return;
  f32x4 acc = {0.f, 0.f, 0.f, 0.f};
  const int kk = lane >> 4, jj = lane & 15;
  for (int64_t q = bptr[blk]; q < bptr[blk + 1]; ++q) {
    float a = bval[q * 64 + lane];
    int32_t col = bcol[q * 4 + kk];
    float b = col >= 0 ? w32[(int64_t)col * 16 + jj] : 0.f;
    acc = __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, acc, 0, 0, 0);
  }
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    int64_t row = blk * 16 + 4 * kk + v;
    if (row < n) y[row * 16 + jj] = (double)acc[v];
  }
}

__global__ void k_to_f32(int64_t m, const double* __restrict__ a, float* __restrict__ b) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < m) b[i] = (float)a[i];
}

void stb_free_blocked(stb_mat* M) {
  dfree(M->d_bptr);
  dfree(M->d_bcol);
  dfree(M->d_bval);
  M->d_bptr = nullptr;
  M->d_bcol = nullptr;
  M->d_bval = nullptr;
  M->nblk = M->nquad = 0;
}

// Blocked copy, built on the device from the CSR: per 16-row block an LDS
// bitmap over the n columns marks the union of the rows' columns; its
// popcount prefix gives every column its slot, in column order.
constexpr int kBlkThreads = 256;
constexpr int64_t kMaxBlockedN = 262144;   // 2 x n/32 words of LDS <= 64 KiB

__device__ __forceinline__ void blk_mark(int64_t b, int64_t n, const int64_t* rowptr,
                                         const int32_t* cols, uint32_t* bits, int nw) {
  for (int w = threadIdx.x; w < nw; w += kBlkThreads) bits[w] = 0u;
  __syncthreads();
  int64_t r1 = (b + 1) * 16 < n ? (b + 1) * 16 : n;
  for (int64_t r = b * 16; r < r1; ++r)
    for (int64_t k = rowptr[r] + threadIdx.x; k < rowptr[r + 1]; k += kBlkThreads) {
      int32_t c = cols[k];
      atomicOr(&bits[c >> 5], 1u << (c & 31));
    }
  __syncthreads();
}

__global__ __launch_bounds__(kBlkThreads) void k_blk_count(int64_t nblk, int64_t n, int64_t ncols,
                                                           const int64_t* __restrict__ rowptr,
                                                           const int32_t* __restrict__ cols,
                                                           int64_t* __restrict__ nquad) {
  extern __shared__ uint32_t lds[];
  int64_t b = blockIdx.x;
  if (b >= nblk) return;
  int nw = (int)((ncols + 31) / 32);
  blk_mark(b, n, rowptr, cols, lds, nw);
  int c = 0;
  for (int w = threadIdx.x; w < nw; w += kBlkThreads) c += __popc(lds[w]);
  __shared__ int red[kBlkThreads];
  red[threadIdx.x] = c;
  __syncthreads();
  for (int off = kBlkThreads / 2; off > 0; off >>= 1) {
    if (threadIdx.x < off) red[threadIdx.x] += red[threadIdx.x + off];
    __syncthreads();
  }
  if (threadIdx.x == 0) nquad[b] = (red[0] + 3) / 4;
}

__global__ __launch_bounds__(kBlkThreads) void k_blk_fill(int64_t nblk, int64_t n, int64_t ncols,
                                                          const int64_t* __restrict__ rowptr,
                                                          const int32_t* __restrict__ cols,
                                                          const double* __restrict__ vals,
                                                          const int64_t* __restrict__ qptr,
                                                          int32_t* __restrict__ bcol,
                                                          float* __restrict__ bval) {
  extern __shared__ uint32_t lds[];
  int64_t b = blockIdx.x;
  if (b >= nblk) return;
  int nw = (int)((ncols + 31) / 32);
  uint32_t* bits = lds;
  int* pre = reinterpret_cast<int*>(lds + nw);
  blk_mark(b, n, rowptr, cols, bits, nw);
  // exclusive prefix of popcounts over the words: per-thread chunk, then a
  // serial scan of the 256 chunk sums by thread 0
  __shared__ int csum[kBlkThreads];
  int per = (nw + kBlkThreads - 1) / kBlkThreads;
  int w0 = threadIdx.x * per, w1 = min(nw, w0 + per);
  int acc = 0;
  for (int w = w0; w < w1; ++w) { pre[w] = acc; acc += __popc(bits[w]); }
  csum[threadIdx.x] = acc;
  __syncthreads();
  if (threadIdx.x == 0) {
    int run = 0;
    for (int t = 0; t < kBlkThreads; ++t) { int v = csum[t]; csum[t] = run; run += v; }
  }
  __syncthreads();
  for (int w = w0; w < w1; ++w) pre[w] += csum[threadIdx.x];
  __syncthreads();
  int64_t q0 = qptr[b], nq = qptr[b + 1] - q0;
  for (int64_t k = threadIdx.x; k < nq * 4; k += kBlkThreads) bcol[q0 * 4 + k] = -1;
  for (int64_t k = threadIdx.x; k < nq * 64; k += kBlkThreads) bval[q0 * 64 + k] = 0.f;
  __syncthreads();
  for (int w = threadIdx.x; w < nw; w += kBlkThreads) {
    uint32_t m = bits[w];
    int slot = pre[w];
    while (m) {
      int bit = __ffs(m) - 1;
      bcol[q0 * 4 + slot] = w * 32 + bit;
      ++slot;
      m &= m - 1;
    }
  }
  int64_t r1 = (b + 1) * 16 < n ? (b + 1) * 16 : n;
  for (int64_t r = b * 16; r < r1; ++r)
    for (int64_t k = rowptr[r] + threadIdx.x; k < rowptr[r + 1]; k += kBlkThreads) {
      int32_t c = cols[k];
      uint32_t below = bits[c >> 5] & ((1u << (c & 31)) - 1u);
      int slot = pre[c >> 5] + __popc(below);
      bval[(q0 + slot / 4) * 64 + (slot % 4) * 16 + (int)(r - b * 16)] = (float)vals[k];
    }
}

stb_status stb_build_blocked(stb_ctx* ctx, stb_mat* M, hipStream_t st) {
  const int64_t n = M->n, ncols = mat_ncols(M);
  if (ncols > kMaxBlockedN)
    return stb_fail(ctx, STB_E_INVALID_ARG, "16-RHS product supports n <= %lld", (long long)kMaxBlockedN);
  const int64_t nblk = (n + 15) / 16;
  size_t lds = sizeof(uint32_t) * 2 * (size_t)((ncols + 31) / 32);
  int64_t* d_nq = nullptr;
  stb_free_blocked(M);
  HIPCHK(ctx, dalloc(&d_nq, (size_t)nblk));
  HIPCHK(ctx, dalloc(&M->d_bptr, (size_t)nblk + 1));
  hipLaunchKernelGGL(k_blk_count, dim3((unsigned)nblk), dim3(kBlkThreads), lds / 2, st, nblk, n, ncols,
                     M->d_rowptr, M->d_cols, d_nq);
  HIPCHK(ctx, hipGetLastError());
  stb_status s = stb_exclusive_scan(ctx, d_nq, M->d_bptr, nblk, st);
  dfree(d_nq);
  if (s) return s;
  int64_t nquad = 0;
  HIPCHK(ctx, hipMemcpy(&nquad, M->d_bptr + nblk, sizeof(int64_t), hipMemcpyDeviceToHost));
  HIPCHK(ctx, dalloc(&M->d_bcol, (size_t)nquad * 4));
  HIPCHK(ctx, dalloc(&M->d_bval, (size_t)nquad * 64));
  hipLaunchKernelGGL(k_blk_fill, dim3((unsigned)nblk), dim3(kBlkThreads), lds, st, nblk, n, ncols,
                     M->d_rowptr, M->d_cols, M->d_vals, M->d_bptr, M->d_bcol, M->d_bval);
  HIPCHK(ctx, hipGetLastError());
  M->nblk = nblk;
  M->nquad = nquad;
  return STB_OK;
}

stb_status stb_apply16_dev(stb_ctx* ctx, stb_mat* M, const double* w, double* y, hipStream_t st) {
  if (!M->d_bptr) {
    stb_status s = stb_build_blocked(ctx, M, st);
    if (s) return s;
  }
  float* w32 = nullptr;
  HIPCHK(ctx, dalloc(&w32, (size_t)mat_ncols(M) * 16));
  int64_t m = mat_ncols(M) * 16;
  if (m > 0) {
    hipLaunchKernelGGL(k_to_f32, dim3((unsigned)((m + 255) / 256)), dim3(256), 0, st, m, w, w32);
  }
  if (M->nblk > 0) {
    int64_t threads = M->nblk * 64;
    hipLaunchKernelGGL(k_bell_mfma, dim3((unsigned)((threads + 255) / 256)), dim3(256), 0, st, M->nblk,
                       M->n, M->d_bptr, M->d_bcol, M->d_bval, w32, y);
  }
  hipError_t e = hipGetLastError();
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  dfree(w32);
  if (e != hipSuccess) return stb_fail(ctx, STB_E_DEVICE, "16-RHS apply failed: %s", hipGetErrorString(e));
  return STB_OK;
}
