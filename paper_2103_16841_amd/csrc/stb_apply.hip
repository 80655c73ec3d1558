// stb_apply.hip -- multi right-hand-side product Y = A W (16 columns) on the
// CDNA4 matrix cores.  With 16 right-hand sides the product is a real GEMM
// over the sparse store: per block of 16 rows, the union of its rows'
// candidate columns is packed into quads, and each quad is one
// v_mfma_f32_16x16x4f32 step, A (16 rows x 4 columns, FP32) times W (4 rows x
// 16 right-hand sides, FP32) accumulated in FP32.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <vector>

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

// Host construction of the blocked copy from the CSR mirror.
static stb_status build_blocked(stb_ctx* ctx, stb_mat* M) {
  stb_status s = stb_mirror_host(M);
  if (s) return s;
  const int64_t n = M->n;
  const int64_t nblk = (n + 15) / 16;
  std::vector<int64_t> bptr((size_t)nblk + 1, 0);
  std::vector<std::vector<int32_t>> ucols((size_t)nblk);
  for (int64_t b = 0; b < nblk; ++b) {
    std::vector<int32_t>& u = ucols[(size_t)b];
    for (int64_t i = b * 16; i < std::min(n, b * 16 + 16); ++i)
      u.insert(u.end(), M->h_cols.begin() + M->h_rowptr[i], M->h_cols.begin() + M->h_rowptr[i + 1]);
    std::sort(u.begin(), u.end());
    u.erase(std::unique(u.begin(), u.end()), u.end());
    bptr[(size_t)b + 1] = bptr[(size_t)b] + (int64_t)((u.size() + 3) / 4);
  }
  const int64_t nquad = bptr[(size_t)nblk];
  std::vector<int32_t> bcol((size_t)nquad * 4, -1);
  std::vector<float> bval((size_t)nquad * 64, 0.f);
  for (int64_t b = 0; b < nblk; ++b) {
    const std::vector<int32_t>& u = ucols[(size_t)b];
    int64_t q0 = bptr[(size_t)b];
    for (size_t k = 0; k < u.size(); ++k) bcol[(size_t)q0 * 4 + k] = u[k];
    for (int64_t i = b * 16; i < std::min(n, b * 16 + 16); ++i) {
      int r = (int)(i - b * 16);
      for (int64_t k = M->h_rowptr[i]; k < M->h_rowptr[i + 1]; ++k) {
        size_t pos = (size_t)(std::lower_bound(u.begin(), u.end(), M->h_cols[k]) - u.begin());
        int64_t q = q0 + (int64_t)(pos / 4);
        int kk = (int)(pos % 4);
        bval[(size_t)q * 64 + (size_t)(kk * 16 + r)] = (float)M->h_vals[k];
      }
    }
  }
  stb_free_blocked(M);
  HIPCHK(ctx, dalloc(&M->d_bptr, (size_t)nblk + 1));
  HIPCHK(ctx, dalloc(&M->d_bcol, (size_t)nquad * 4));
  HIPCHK(ctx, dalloc(&M->d_bval, (size_t)nquad * 64));
  HIPCHK(ctx, hipMemcpy(M->d_bptr, bptr.data(), 8 * (nblk + 1), hipMemcpyHostToDevice));
  if (nquad) {
    HIPCHK(ctx, hipMemcpy(M->d_bcol, bcol.data(), 4 * nquad * 4, hipMemcpyHostToDevice));
    HIPCHK(ctx, hipMemcpy(M->d_bval, bval.data(), 4 * nquad * 64, hipMemcpyHostToDevice));
  }
  M->nblk = nblk;
  M->nquad = nquad;
  return STB_OK;
}

stb_status stb_apply16_dev(stb_ctx* ctx, stb_mat* M, const double* w, double* y, hipStream_t st) {
  if (!M->d_bptr) {
    stb_status s = build_blocked(ctx, M);
    if (s) return s;
  }
  float* w32 = nullptr;
  HIPCHK(ctx, dalloc(&w32, (size_t)M->n * 16));
  int64_t m = M->n * 16;
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
