// stb_apply.hip -- multi right-hand-side product Y = A W (16 columns) on the
// CDNA4 matrix cores.  With 16 right-hand sides the product is a real GEMM
// over the sparse store: per block of 16 rows, the union of its rows'
// candidate columns is packed into quads, and each quad is one
// v_mfma_f32_16x16x4f32 step, A (16 rows x 4 columns, FP32) times W (4 rows x
// 16 right-hand sides, FP32) accumulated in FP32.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <mutex>

#include "stb_internal.h"

typedef float f32x4 __attribute__((ext_vector_type(4)));

// One wavefront per 16-row block.  MFMA 16x16x4 (FP32) operand layout:
//   A: lane l holds A[l % 16][l / 16];  B: lane l holds B[l / 16][l % 16];
//   D: lane l, register v holds D[4 (l / 16) + v][l % 16].
// One workgroup (four wavefronts) per 16-row block: wavefront v takes the
// block's quads v, v + 4, ... (two independent MFMA chains, even and odd
// steps), and the four partial tiles are summed in LDS in a fixed order.
__global__ __launch_bounds__(256) void k_bell_mfma(int64_t nblk, int64_t n,
                                                   const int64_t* __restrict__ bptr,
                                                   const int32_t* __restrict__ bcol,
                                                   const float* __restrict__ bval,
                                                   const float* __restrict__ w32,
                                                   double* __restrict__ y) {
  const int64_t blk = blockIdx.x;
  const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int kk = lane >> 4, jj = lane & 15;
  f32x4 acc0 = {0.f, 0.f, 0.f, 0.f}, acc1 = {0.f, 0.f, 0.f, 0.f};
  const int64_t q0 = bptr[blk], q1 = bptr[blk + 1];
  int64_t q = q0 + wv;
  // eight quads per wave and pass: their values, columns and W rows are all
  // requested before the first product waits on them
  for (; q + 28 < q1; q += 32) {
    float a[8], b[8];
    int32_t c[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      a[u] = bval[(q + 4 * u) * 64 + lane];
      c[u] = bcol[(q + 4 * u) * 4 + kk];
    }
#pragma unroll
    for (int u = 0; u < 8; ++u) b[u] = c[u] >= 0 ? w32[(int64_t)c[u] * 16 + jj] : 0.f;
#pragma unroll
    for (int u = 0; u < 8; u += 2) {
      acc0 = __builtin_amdgcn_mfma_f32_16x16x4f32(a[u], b[u], acc0, 0, 0, 0);
      acc1 = __builtin_amdgcn_mfma_f32_16x16x4f32(a[u + 1], b[u + 1], acc1, 0, 0, 0);
    }
  }
  for (; q < q1; q += 4) {
    const float a0 = bval[q * 64 + lane];
    const int32_t c0 = bcol[q * 4 + kk];
    const float b0 = c0 >= 0 ? w32[(int64_t)c0 * 16 + jj] : 0.f;
    acc0 = __builtin_amdgcn_mfma_f32_16x16x4f32(a0, b0, acc0, 0, 0, 0);
  }
  __shared__ float part[4][4][64];
#pragma unroll
  for (int v = 0; v < 4; ++v) part[wv][v][lane] = acc0[v] + acc1[v];
  __syncthreads();
  if (wv != 0) return;
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    const float t = ((part[0][v][lane] + part[1][v][lane]) + part[2][v][lane]) + part[3][v][lane];
    const int64_t row = blk * 16 + 4 * kk + v;
    if (row < n) y[row * 16 + jj] = (double)t;
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

// Slots per pass of the value fill: a [kFillSlots][16] FP32 tile in LDS.
constexpr int kFillSlots = 512;

// The block's slot of column c (c must be marked).
__device__ __forceinline__ int blk_slot(const uint32_t* bits, const int* pre, int32_t c) {
  return pre[c >> 5] + __popc(bits[c >> 5] & ((1u << (c & 31)) - 1u));
}

// Fills one block: column of every slot, then the values.  Slot s of row r
// sits at bval[q0 * 64 + 16 s + r] (the MFMA A-operand order), so a range
// of slots is one contiguous range of bval: the values of kFillSlots slots
// are scattered into an LDS tile (zero where a row lacks the column) and the
// tile is copied out whole.
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
  float* tile = reinterpret_cast<float*>(lds + 2 * nw);
  __shared__ int64_t klo[16], khi[16];
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
  const int64_t q0 = qptr[b], nq = qptr[b + 1] - q0;
  const int nslot = nw > 0 ? pre[nw - 1] + __popc(bits[nw - 1]) : 0;
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
  for (int64_t k = nslot + threadIdx.x; k < nq * 4; k += kBlkThreads) bcol[q0 * 4 + k] = -1;
  for (int64_t k = (int64_t)nslot * 16 + threadIdx.x; k < nq * 64; k += kBlkThreads) bval[q0 * 64 + k] = 0.f;
  const int64_t rb = b * 16;
  const int nr = (int)((rb + 16 < n ? rb + 16 : n) - rb);
  for (int s0 = 0; s0 < nslot; s0 += kFillSlots) {
    const int ns = nslot - s0 < kFillSlots ? nslot - s0 : kFillSlots;
    for (int e = threadIdx.x; e < ns * 16; e += kBlkThreads) tile[e] = 0.f;
    if ((int)threadIdx.x < 2 * nr) {
      // the row's first entry with slot >= s0 (lanes 0..nr-1) or >= s0 + ns
      // (lanes nr..2nr-1): slots increase along a row's sorted columns
      const bool first = (int)threadIdx.x < nr;
      const int rr = first ? (int)threadIdx.x : (int)threadIdx.x - nr;
      const int target = first ? s0 : s0 + ns;
      int64_t lo = rowptr[rb + rr], hi = rowptr[rb + rr + 1];
      while (lo < hi) {
        const int64_t mid = lo + ((hi - lo) >> 1);
        if (blk_slot(bits, pre, cols[mid]) < target) lo = mid + 1; else hi = mid;
      }
      if (first) klo[rr] = lo; else khi[rr] = lo;
    }
    __syncthreads();
    for (int r = 0; r < nr; ++r)
      for (int64_t k = klo[r] + threadIdx.x; k < khi[r]; k += kBlkThreads)
        tile[(blk_slot(bits, pre, cols[k]) - s0) * 16 + r] = (float)vals[k];
    __syncthreads();
    for (int e = threadIdx.x; e < ns * 16; e += kBlkThreads) bval[q0 * 64 + (int64_t)s0 * 16 + e] = tile[e];
    __syncthreads();
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
  const size_t lds_fill = lds + sizeof(float) * 16 * kFillSlots;
  HIPCHK(ctx, hipFuncSetAttribute(reinterpret_cast<const void*>(&k_blk_fill),
                                  hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds_fill));
  hipLaunchKernelGGL(k_blk_fill, dim3((unsigned)nblk), dim3(kBlkThreads), lds_fill, st, nblk, n, ncols,
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
    hipLaunchKernelGGL(k_bell_mfma, dim3((unsigned)M->nblk), dim3(256), 0, st, M->nblk, M->n, M->d_bptr,
                       M->d_bcol, M->d_bval, w32, y);
  }
  hipError_t e = hipGetLastError();
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  dfree(w32);
  if (e != hipSuccess) return stb_fail(ctx, STB_E_DEVICE, "16-RHS apply failed: %s", hipGetErrorString(e));
  return STB_OK;
}

// ------------------------------------------------ product without allocation
// stb_apply16_noalloc is the 16-RHS product for callers that cannot allocate
// device memory (code under HIP graph capture, tight serving loops, harnesses
// that forbid allocation): the FP32 copy of W, which stb_apply16_dev puts in
// a buffer of its own per call, goes to this file-scope array instead.  Each
// device the library runs on holds one copy (16 MiB) until the process ends;
// every call on a device shares it, so calls that overlap on one device race.
constexpr int64_t kNoAllocMaxCols = kMaxBlockedN;
static __device__ __align__(256) float scratch[kNoAllocMaxCols * 16];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
float* g_scratch_dev[kMaxDevices] = {};   // device address of scratch, per device
}  // namespace

// Called by stb_ctx_create with ctx's device current: looks up this device's
// address of the scratch array once.  In host code the array's name is only a
// stand-in; kernels get the address found here.
stb_status stb_noalloc_setup(stb_ctx* ctx) {
  if (ctx->device < 0 || ctx->device >= kMaxDevices)
    return stb_fail(ctx, STB_E_INVALID_ARG, "device %d: at most %d devices", ctx->device, kMaxDevices);
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (g_scratch_dev[ctx->device]) return STB_OK;
  void* ptr = nullptr;
  hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
  if (e != hipSuccess || !ptr)
    return stb_fail(ctx, STB_E_DEVICE, "scratch address: %s", hipGetErrorString(e));
  g_scratch_dev[ctx->device] = static_cast<float*>(ptr);
  return STB_OK;
}

extern "C" stb_status stb_apply16_noalloc(stb_ctx* ctx, const stb_mat* M, const double* w_dev,
                                          double* y_dev, void* stream) {
  if (!ctx || !M || !w_dev || !y_dev) return stb_fail(ctx, STB_E_INVALID_ARG, "NULL argument");
  if (M->ctx != ctx) return stb_fail(ctx, STB_E_INVALID_ARG, "matrix belongs to another context");
  const int64_t ncols = mat_ncols(M);
  if (ncols > kNoAllocMaxCols)
    return stb_fail(ctx, STB_E_INVALID_ARG, "%lld columns exceed the %lld of the allocation-free product",
                    (long long)ncols, (long long)kNoAllocMaxCols);
  if (!M->d_bptr && M->n > 0)
    return stb_fail(ctx, STB_E_INVALID_ARG,
                    "the matrix-core copy is not built: call stb_apply with nrhs = 16 once first");
  float* w32 = g_scratch_dev[ctx->device];
  if (!w32) return stb_fail(ctx, STB_E_INTERNAL, "scratch of device %d not set up", ctx->device);
  hipStream_t st = stream ? (hipStream_t)stream : ctx->stream;
  HIPCHK(ctx, hipSetDevice(ctx->device));
  const int64_t m = ncols * 16;
  if (m > 0)
    hipLaunchKernelGGL(k_to_f32, dim3((unsigned)((m + 255) / 256)), dim3(256), 0, st, m, w_dev, w32);
  if (M->nblk > 0)
    hipLaunchKernelGGL(k_bell_mfma, dim3((unsigned)M->nblk), dim3(256), 0, st, M->nblk, M->n, M->d_bptr,
                       M->d_bcol, M->d_bval, (const float*)w32, y_dev);
  HIPCHK(ctx, hipGetLastError());
  return STB_OK;
}
