// stb_solve.hip -- the discrete indirect system (eq. df_ind): restarted
// GMRES over the assembled energetic single-layer matrix, on the device.
//
// Every Krylov step is one FP64 product with the stored matrix (k_spmv)
// plus classical Gram-Schmidt against the basis, done twice for
// orthogonality (CGS2): two batched dot products and two batched updates.
// The small Hessenberg problem (Givens rotations, back substitution) stays
// on the host.  Dot products are fixed-order block reductions, so results
// do not depend on the schedule.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <vector>

#include "stb_internal.h"

namespace {

constexpr int kSolveThreads = 256;

// out[b] = <V_b, w> for b < k (V row-major, k rows of ld doubles).
__global__ __launch_bounds__(kSolveThreads) void k_dots(int64_t n, const double* __restrict__ V,
                                                        int64_t ld, const double* __restrict__ w,
                                                        double* __restrict__ out) {
  const double* v = V + (int64_t)blockIdx.x * ld;
  double s = 0.0;
  for (int64_t i = threadIdx.x; i < n; i += kSolveThreads) s += v[i] * w[i];
  __shared__ double red[kSolveThreads];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int off = kSolveThreads / 2; off > 0; off >>= 1) {
    if ((int)threadIdx.x < off) red[threadIdx.x] += red[threadIdx.x + off];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[blockIdx.x] = red[0];
}

// w -= sum_{b < k} h[b] V_b (b ascending).
__global__ void k_subtract(int64_t n, int k, const double* __restrict__ V, int64_t ld,
                           const double* __restrict__ h, double* __restrict__ w) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double s = w[i];
  for (int b = 0; b < k; ++b) s -= h[b] * V[(int64_t)b * ld + i];
  w[i] = s;
}

// y = a x (+ y when acc).
__global__ void k_axpy(int64_t n, double a, const double* x, double* y, int acc) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  y[i] = acc ? fma(a, x[i], y[i]) : a * x[i];
}

// r = b - r (r holds A x).
__global__ void k_residual(int64_t n, const double* __restrict__ b, double* __restrict__ r) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) r[i] = b[i] - r[i];
}

// b_i = sum_{q < n_i} w_iq g_iq, q ascending: the right-hand side of the
// indirect system from data g at panel i's outer points (eq. df_ind with the
// outer rule of eq. int_bform).
__global__ void k_outer_rhs(int64_t nt, int maxq, const double* __restrict__ w,
                            const int32_t* __restrict__ nq, const double* __restrict__ g,
                            double* __restrict__ b) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nt) return;
  double s = 0.0;
  for (int q = 0; q < nq[i]; ++q) s = fma(w[i * maxq + q], g[i * maxq + q], s);
  b[i] = s;
}


// ------------------------------------------------ marching-on-in-time
// Dense diagonal block D[k][l] = A[row_k][row_l] of the panels of slab 0
// (loc[j] = local index of panel j in its slab, slab[j] its slab).
__global__ void k_mot_block(int64_t K, const int32_t* __restrict__ rows0, const int64_t* __restrict__ rowptr,
                            const int32_t* __restrict__ cols, const double* __restrict__ vals,
                            const int32_t* __restrict__ slab, const int32_t* __restrict__ loc,
                            double* __restrict__ D) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= K) return;
  const int32_t i = rows0[k];
  for (int64_t e = rowptr[i]; e < rowptr[i + 1]; ++e) {
    const int32_t j = cols[e];
    if (slab[j] == 0) D[k * K + loc[j]] = vals[e];
  }
}

// Every stored entry (i, j) has slab[j] <= slab[i] (block lower triangular
// in time); bad[0] counts the entries that do not.
__global__ void k_mot_lower(int64_t n, const int64_t* __restrict__ rowptr, const int32_t* __restrict__ cols,
                            const int32_t* __restrict__ slab, unsigned long long* __restrict__ bad) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  unsigned long long c = 0;
  for (int64_t e = rowptr[i]; e < rowptr[i + 1]; ++e) c += slab[cols[e]] > slab[i] ? 1ull : 0ull;
  if (c) atomicAdd(bad, c);
}

// Gauss-Jordan inversion of D (K x K, row-major) in place, pivot step k,
// part 1 (one workgroup): partial pivot (largest |D[i][k]|, i >= k, first
// such i), row swap, scaling of the pivot row, the column's multipliers
// into f (f[k] = 0) and column k cleared outside the pivot row.
constexpr int kGjThreads = 1024;
__global__ __launch_bounds__(kGjThreads) void k_gj_pivot(int64_t K, int64_t k, double* __restrict__ D,
                                                         int32_t* __restrict__ perm, double* __restrict__ f,
                                                         int* __restrict__ singular) {
  __shared__ double sv[kGjThreads];
  __shared__ int64_t si[kGjThreads];
  double best = -1.0;
  int64_t bi = k;
  for (int64_t i = k + threadIdx.x; i < K; i += kGjThreads) {
    const double v = fabs(D[i * K + k]);
    if (v > best) { best = v; bi = i; }
  }
  sv[threadIdx.x] = best;
  si[threadIdx.x] = bi;
  __syncthreads();
  for (int off = kGjThreads / 2; off > 0; off >>= 1) {
    if ((int)threadIdx.x < off) {
      const double a = sv[threadIdx.x], b = sv[threadIdx.x + off];
      const int64_t ia = si[threadIdx.x], ib = si[threadIdx.x + off];
      if (b > a || (b == a && ib < ia)) { sv[threadIdx.x] = b; si[threadIdx.x] = ib; }
    }
    __syncthreads();
  }
  const int64_t p = si[0];
  if (threadIdx.x == 0) {
    perm[k] = (int32_t)p;
    if (!(sv[0] > 0.0)) *singular = 1;
  }
  if (p != k)
    for (int64_t j = threadIdx.x; j < K; j += kGjThreads) {
      const double t = D[k * K + j];
      D[k * K + j] = D[p * K + j];
      D[p * K + j] = t;
    }
  __syncthreads();
  const double piv = D[k * K + k];
  const double inv = sv[0] > 0.0 ? 1.0 / piv : 0.0;
  __syncthreads();
  for (int64_t j = threadIdx.x; j < K; j += kGjThreads) {
    const double v = j == k ? 1.0 : D[k * K + j];
    D[k * K + j] = v * inv;
  }
  for (int64_t i = threadIdx.x; i < K; i += kGjThreads) {
    if (i == k) { f[i] = 0.0; continue; }
    f[i] = D[i * K + k];
    D[i * K + k] = 0.0;
  }
}

// Part 2: D[i][j] -= f[i] D[k][j] for every row i != k (row k is read only).
__global__ void k_gj_update(int64_t K, int64_t k, double* __restrict__ D, const double* __restrict__ f) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= K * K) return;
  const int64_t i = e / K, j = e - i * K;
  const double fi = f[i];
  if (fi != 0.0) D[e] = fma(-fi, D[k * K + j], D[e]);
}

// Undo the row interchanges on the inverse: its columns k and perm[k] swap,
// k from K - 1 down to 0 (one lane per row).
__global__ void k_gj_unswap(int64_t K, double* __restrict__ D, const int32_t* __restrict__ perm) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= K) return;
  for (int64_t k = K - 1; k >= 0; --k) {
    const int64_t p = perm[k];
    if (p != k) {
      const double t = D[i * K + k];
      D[i * K + k] = D[i * K + p];
      D[i * K + p] = t;
    }
  }
}

// Time step n, part 1: r[k] = b[i] - sum_j A[i][j] x[j] for the rows i =
// rows[k] of the slab (x is zero on this and later slabs, so this is
// b_n - sum_{m<n} A_nm x_m); one wavefront per row, fixed-order reduction.
__global__ __launch_bounds__(256) void k_mot_rhs(int64_t K, const int32_t* __restrict__ rows,
                                                 const int64_t* __restrict__ rowptr,
                                                 const int32_t* __restrict__ cols,
                                                 const double* __restrict__ vals,
                                                 const double* __restrict__ x, const double* __restrict__ b,
                                                 double* __restrict__ r) {
  const int64_t k = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  const int lane = threadIdx.x & 63;
  if (k >= K) return;
  const int32_t i = rows[k];
  double s = 0.0;
  for (int64_t e = rowptr[i] + lane; e < rowptr[i + 1]; e += 64) s += vals[e] * x[cols[e]];
  for (int off = 32; off > 0; off >>= 1) s += __shfl_down(s, off, 64);
  if (lane == 0) r[k] = b[i] - s;
}

// Part 2: x[rows[k]] = sum_l Dinv[k][l] r[l]; one wavefront per row.
__global__ __launch_bounds__(256) void k_mot_apply(int64_t K, const int32_t* __restrict__ rows,
                                                   const double* __restrict__ Dinv,
                                                   const double* __restrict__ r, double* __restrict__ x) {
  const int64_t k = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  const int lane = threadIdx.x & 63;
  if (k >= K) return;
  double s = 0.0;
  for (int64_t l = lane; l < K; l += 64) s += Dinv[k * K + l] * r[l];
  for (int off = 32; off > 0; off >>= 1) s += __shfl_down(s, off, 64);
  if (lane == 0) x[rows[k]] = s;
}

}  // namespace

extern "C" {

stb_status stb_outer_rhs(stb_ctx* ctx, const stb_mesh* mesh_c, int32_t m_q, const double* g,
                         double* b) {
  if (!ctx || !mesh_c || !g || !b) return stb_fail(ctx, STB_E_INVALID_ARG, "NULL argument");
  if (m_q < 1 || m_q > 4) return stb_fail(ctx, STB_E_INVALID_ARG, "m_q must be in [1,4], got %d", m_q);
  stb_mesh* mesh = const_cast<stb_mesh*>(mesh_c);
  if (mesh->ctx != ctx) return stb_fail(ctx, STB_E_INVALID_ARG, "mesh belongs to another context");
  HIPCHK(ctx, hipSetDevice(ctx->device));
  stb_status s = stb_ensure_outer(ctx, mesh, m_q);
  if (s) return s;
  const int64_t nt = mesh->nt, maxq = mesh->maxq;
  if (nt == 0) return STB_OK;
  for (int64_t k = 0; k < nt * maxq; ++k)
    if (!std::isfinite(g[k])) return stb_fail(ctx, STB_E_INVALID_ARG, "non-finite data at outer point %lld", (long long)k);
  double *d_g = nullptr, *d_b = nullptr;
  if (dalloc(&d_g, (size_t)(nt * maxq)) != hipSuccess || dalloc(&d_b, (size_t)nt) != hipSuccess) {
    dfree(d_g); dfree(d_b);
    return stb_fail(ctx, STB_E_NO_MEMORY, "right-hand side buffers");
  }
  hipError_t e = hipMemcpyAsync(d_g, g, sizeof(double) * nt * maxq, hipMemcpyHostToDevice, ctx->stream);
  if (e == hipSuccess) {
    hipLaunchKernelGGL(k_outer_rhs, dim3((unsigned)((nt + 255) / 256)), dim3(256), 0, ctx->stream, nt,
                       (int)maxq, mesh->d_ow, mesh->d_onq, d_g, d_b);
    e = hipGetLastError();
  }
  if (e == hipSuccess) e = hipMemcpyAsync(b, d_b, sizeof(double) * nt, hipMemcpyDeviceToHost, ctx->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
  dfree(d_g);
  dfree(d_b);
  if (e != hipSuccess) return stb_fail(ctx, STB_E_DEVICE, "right-hand side: %s", hipGetErrorString(e));
  return STB_OK;
}

stb_status stb_outer_points(stb_ctx* ctx, const stb_mesh* mesh_c, int32_t m_q, double* pts,
                            double* weights, int32_t* counts) {
  if (!ctx || !mesh_c || !pts || !weights || !counts)
    return stb_fail(ctx, STB_E_INVALID_ARG, "NULL argument");
  if (m_q < 1 || m_q > 4) return stb_fail(ctx, STB_E_INVALID_ARG, "m_q must be in [1,4], got %d", m_q);
  stb_mesh* mesh = const_cast<stb_mesh*>(mesh_c);
  if (mesh->ctx != ctx) return stb_fail(ctx, STB_E_INVALID_ARG, "mesh belongs to another context");
  HIPCHK(ctx, hipSetDevice(ctx->device));
  stb_status s = stb_ensure_outer(ctx, mesh, m_q);
  if (s) return s;
  const int64_t nt = mesh->nt, maxq = mesh->maxq;
  if (nt > 0) {
    HIPCHK(ctx, hipMemcpyAsync(pts, mesh->d_opts, sizeof(double) * nt * maxq * 4, hipMemcpyDeviceToHost,
                               ctx->stream));
    HIPCHK(ctx, hipMemcpyAsync(weights, mesh->d_ow, sizeof(double) * nt * maxq, hipMemcpyDeviceToHost,
                               ctx->stream));
    HIPCHK(ctx, hipMemcpyAsync(counts, mesh->d_onq, sizeof(int32_t) * nt, hipMemcpyDeviceToHost,
                               ctx->stream));
    HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
  }
  // entries past each panel's count are not part of the rule
  for (int64_t i = 0; i < nt; ++i)
    for (int64_t q = counts[i]; q < maxq; ++q) {
      weights[i * maxq + q] = 0.0;
      for (int c = 0; c < 4; ++c) pts[(i * maxq + q) * 4 + c] = 0.0;
    }
  return STB_OK;
}

stb_status stb_solve_gmres(stb_ctx* ctx, const stb_mat* A, const double* b_host, double* x_host,
                           int32_t restart, int32_t maxit, double rtol, int32_t* iters, double* relres) {
  if (!ctx || !A || !b_host || !x_host) return stb_fail(ctx, STB_E_INVALID_ARG, "NULL argument");
  if (A->ncols != 0 && A->ncols != A->n)
    return stb_fail(ctx, STB_E_INVALID_ARG, "GMRES needs the square matrix of a whole mesh");
  if (restart < 1 || restart > 512 || maxit < 1 || !(rtol > 0.0))
    return stb_fail(ctx, STB_E_INVALID_ARG, "restart in [1,512], maxit >= 1 and rtol > 0 required");
  HIPCHK(ctx, hipSetDevice(ctx->device));
  const int64_t n = A->n;
  const int m = restart;
  hipStream_t st = ctx->stream;
  if (iters) *iters = 0;
  if (relres) *relres = 0.0;
  if (n == 0) return STB_OK;
  double *V = nullptr, *w = nullptr, *b = nullptr, *x = nullptr, *h = nullptr, *h2 = nullptr;
  auto cleanup = [&]() { dfree(V); dfree(w); dfree(b); dfree(x); dfree(h); dfree(h2); };
  if (dalloc(&V, (size_t)(m + 1) * n) != hipSuccess || dalloc(&w, (size_t)n) != hipSuccess ||
      dalloc(&b, (size_t)n) != hipSuccess || dalloc(&x, (size_t)n) != hipSuccess ||
      dalloc(&h, (size_t)m + 1) != hipSuccess || dalloc(&h2, (size_t)m + 1) != hipSuccess) {
    cleanup();
    return stb_fail(ctx, STB_E_NO_MEMORY, "GMRES basis of %d vectors of %lld", m + 1, (long long)n);
  }
  const unsigned g = (unsigned)((n + 255) / 256);
  stb_status s = STB_OK;
  hipError_t e = hipMemcpyAsync(b, b_host, sizeof(double) * n, hipMemcpyHostToDevice, st);
  if (e == hipSuccess) e = hipMemcpyAsync(x, x_host, sizeof(double) * n, hipMemcpyHostToDevice, st);
  if (e != hipSuccess) { cleanup(); return stb_fail(ctx, STB_E_DEVICE, "GMRES copy: %s", hipGetErrorString(e)); }
  // one device scalar read back per reduction
  auto dot = [&](const double* u, const double* v, double* out) -> stb_status {
    hipLaunchKernelGGL(k_dots, dim3(1), dim3(kSolveThreads), 0, st, n, u, n, v, h2);
    hipError_t ee = hipMemcpyAsync(out, h2, sizeof(double), hipMemcpyDeviceToHost, st);
    if (ee == hipSuccess) ee = hipStreamSynchronize(st);
    return ee == hipSuccess ? STB_OK : stb_fail(ctx, STB_E_DEVICE, "GMRES dot: %s", hipGetErrorString(ee));
  };
  double bnorm2 = 0.0;
  if ((s = dot(b, b, &bnorm2))) { cleanup(); return s; }
  const double bnorm = std::sqrt(bnorm2);
  if (bnorm == 0.0) {
    for (int64_t i = 0; i < n; ++i) x_host[i] = 0.0;
    cleanup();
    return STB_OK;
  }
  std::vector<double> H((size_t)(m + 1) * m, 0.0), cs(m), sn(m), gv(m + 1), y(m), hh(m + 1), hh2(m + 1);
  int total = 0;
  double res = 0.0;
  for (;;) {
    // r = b - A x, V_0 = r / |r|
    if ((s = stb_apply_dev(ctx, A, 1, x, w, st))) break;
    hipLaunchKernelGGL(k_residual, dim3(g), dim3(256), 0, st, n, b, w);
    double rn2 = 0.0;
    if ((s = dot(w, w, &rn2))) break;
    const double rn = std::sqrt(rn2);
    res = rn / bnorm;
    if (res <= rtol || total >= maxit) break;
    hipLaunchKernelGGL(k_axpy, dim3(g), dim3(256), 0, st, n, 1.0 / rn, w, V, 0);
    std::fill(gv.begin(), gv.end(), 0.0);
    gv[0] = rn;
    int j = 0;
    for (; j < m && total < maxit; ++j, ++total) {
      double* vj1 = V + (int64_t)(j + 1) * n;
      if ((s = stb_apply_dev(ctx, A, 1, V + (int64_t)j * n, vj1, st))) break;
      // classical Gram-Schmidt, twice
      for (int pass = 0; pass < 2 && s == STB_OK; ++pass) {
        hipLaunchKernelGGL(k_dots, dim3((unsigned)(j + 1)), dim3(kSolveThreads), 0, st, n, V, n, vj1, h);
        hipLaunchKernelGGL(k_subtract, dim3(g), dim3(256), 0, st, n, j + 1, V, n, h, vj1);
        e = hipMemcpyAsync(pass == 0 ? hh.data() : hh2.data(), h, sizeof(double) * (j + 1),
                           hipMemcpyDeviceToHost, st);
        if (e != hipSuccess) s = stb_fail(ctx, STB_E_DEVICE, "GMRES: %s", hipGetErrorString(e));
      }
      if (s) break;
      double hn2 = 0.0;
      if ((s = dot(vj1, vj1, &hn2))) break;   // synchronises: hh, hh2 are on the host now
      for (int i = 0; i <= j; ++i) H[(size_t)i * m + j] = hh[i] + hh2[i];
      const double hn = std::sqrt(hn2);
      H[(size_t)(j + 1) * m + j] = hn;
      if (hn > 0.0) hipLaunchKernelGGL(k_axpy, dim3(g), dim3(256), 0, st, n, 1.0 / hn, vj1, vj1, 0);
      // apply the previous rotations, then a new one for row j + 1
      for (int i = 0; i < j; ++i) {
        const double a = H[(size_t)i * m + j], c = H[(size_t)(i + 1) * m + j];
        H[(size_t)i * m + j] = cs[i] * a + sn[i] * c;
        H[(size_t)(i + 1) * m + j] = -sn[i] * a + cs[i] * c;
      }
      const double a = H[(size_t)j * m + j], c = H[(size_t)(j + 1) * m + j];
      const double r = std::hypot(a, c);
      cs[j] = r > 0.0 ? a / r : 1.0;
      sn[j] = r > 0.0 ? c / r : 0.0;
      H[(size_t)j * m + j] = r;
      H[(size_t)(j + 1) * m + j] = 0.0;
      gv[j + 1] = -sn[j] * gv[j];
      gv[j] = cs[j] * gv[j];
      if (std::fabs(gv[j + 1]) <= rtol * bnorm || hn == 0.0) { ++j; ++total; break; }
    }
    if (s) break;
    // x += V y with H y = g (upper triangular, j columns)
    for (int i = j - 1; i >= 0; --i) {
      double t = gv[i];
      for (int k = i + 1; k < j; ++k) t -= H[(size_t)i * m + k] * y[k];
      y[i] = H[(size_t)i * m + i] != 0.0 ? t / H[(size_t)i * m + i] : 0.0;
    }
    for (int i = 0; i < j; ++i)
      hipLaunchKernelGGL(k_axpy, dim3(g), dim3(256), 0, st, n, y[i], V + (int64_t)i * n, x, 1);
    e = hipGetLastError();
    if (e != hipSuccess) { s = stb_fail(ctx, STB_E_DEVICE, "GMRES: %s", hipGetErrorString(e)); break; }
  }
  if (s == STB_OK) {
    e = hipMemcpyAsync(x_host, x, sizeof(double) * n, hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) s = stb_fail(ctx, STB_E_DEVICE, "GMRES copy: %s", hipGetErrorString(e));
  }
  cleanup();
  if (s) return s;
  if (iters) *iters = total;
  if (relres) *relres = res;
  return STB_OK;
}

stb_status stb_solve_mot(stb_ctx* ctx, const stb_mesh* mesh, const stb_mat* A, const double* b_host,
                         double* x_host, double* info4) {
  if (!ctx || !mesh || !A || !b_host || !x_host) return stb_fail(ctx, STB_E_INVALID_ARG, "NULL argument");
  if (mesh->ctx != ctx || A->ctx != ctx)
    return stb_fail(ctx, STB_E_INVALID_ARG, "mesh or matrix of another context");
  if ((A->ncols != 0 && A->ncols != A->n) || A->n != mesh->nt)
    return stb_fail(ctx, STB_E_INVALID_ARG, "marching-on-in-time needs the square matrix of this mesh");
  HIPCHK(ctx, hipSetDevice(ctx->device));
  const int64_t nt = mesh->nt, nv = mesh->nv;
  if (nt == 0) return STB_OK;
  hipStream_t st = ctx->stream;
  // ---- the slab structure, from the vertex times (host)
  std::vector<double> vtx((size_t)nv * 4);
  std::vector<int32_t> tet((size_t)nt * 4);
  HIPCHK(ctx, hipStreamSynchronize(st));
  HIPCHK(ctx, hipMemcpy(vtx.data(), mesh->d_vtx, sizeof(double) * 4 * nv, hipMemcpyDeviceToHost));
  HIPCHK(ctx, hipMemcpy(tet.data(), mesh->d_tet, sizeof(int32_t) * 4 * nt, hipMemcpyDeviceToHost));
  std::vector<double> tv((size_t)nv);
  double tscale = 0.0, xscale = 0.0;
  for (int64_t v = 0; v < nv; ++v) {
    tv[(size_t)v] = vtx[(size_t)v * 4];
    tscale = std::max(tscale, std::fabs(vtx[(size_t)v * 4]));
    for (int c = 1; c < 4; ++c) xscale = std::max(xscale, std::fabs(vtx[(size_t)v * 4 + c]));
  }
  const double ttol = 1e-12 * std::max(tscale, 1.0), xtol = 1e-12 * std::max(xscale, 1.0);
  std::sort(tv.begin(), tv.end());
  std::vector<double> lev;
  for (double t : tv)
    if (lev.empty() || t - lev.back() > ttol) lev.push_back(t);
  const int64_t S = (int64_t)lev.size() - 1;
  if (S < 1) return stb_fail(ctx, STB_E_INVALID_ARG, "no time slabs");
  const double dt = lev[1] - lev[0];
  for (int64_t n = 1; n < S; ++n)
    if (std::fabs((lev[(size_t)n + 1] - lev[(size_t)n]) - dt) > 1e-9 * dt)
      return stb_fail(ctx, STB_E_INVALID_ARG,
                      "time levels are not uniform (slab %lld): use GMRES", (long long)n);
  auto level_of = [&](double t) -> int64_t {
    const int64_t n = (int64_t)(std::lower_bound(lev.begin(), lev.end(), t - ttol) - lev.begin());
    return (n <= S && std::fabs(lev[(size_t)n] - t) <= ttol) ? n : -1;
  };
  std::vector<int32_t> slab((size_t)nt), loc((size_t)nt);
  std::vector<std::vector<int32_t>> rows((size_t)S);
  for (int64_t i = 0; i < nt; ++i) {
    int64_t lo = S + 1, hi = -1;
    for (int k = 0; k < 4; ++k) {
      const int64_t l = level_of(vtx[(size_t)tet[(size_t)i * 4 + k] * 4]);
      if (l < 0) return stb_fail(ctx, STB_E_INTERNAL, "vertex time off the levels");
      lo = std::min(lo, l);
      hi = std::max(hi, l);
    }
    if (hi != lo + 1)
      return stb_fail(ctx, STB_E_INVALID_ARG,
                      "panel %lld does not span exactly one slab between two time levels: use GMRES",
                      (long long)i);
    slab[(size_t)i] = (int32_t)lo;
    loc[(size_t)i] = (int32_t)rows[(size_t)lo].size();
    rows[(size_t)lo].push_back((int32_t)i);
  }
  const int64_t K = (int64_t)rows[0].size();
  for (int64_t n = 1; n < S; ++n)
    if ((int64_t)rows[(size_t)n].size() != K)
      return stb_fail(ctx, STB_E_INVALID_ARG, "slab %lld has %lld panels, slab 0 has %lld: use GMRES",
                      (long long)n, (long long)rows[(size_t)n].size(), (long long)K);
  if (K > 16384) return stb_fail(ctx, STB_E_INVALID_ARG, "%lld panels per slab (at most 16384)", (long long)K);
  // slab n must be slab 0 moved by (lev_n - lev_0) in time, panel by panel
  for (int64_t n = 1; n < S; ++n) {
    const double shift = lev[(size_t)n] - lev[0];
    for (int64_t k = 0; k < K; ++k) {
      const int32_t p = rows[(size_t)n][(size_t)k], q = rows[0][(size_t)k];
      for (int v = 0; v < 4; ++v) {
        const double* X = &vtx[(size_t)tet[(size_t)p * 4 + v] * 4];
        const double* Y = &vtx[(size_t)tet[(size_t)q * 4 + v] * 4];
        bool same = std::fabs(X[0] - Y[0] - shift) <= ttol;
        for (int c = 1; c < 4; ++c) same = same && std::fabs(X[c] - Y[c]) <= xtol;
        if (!same)
          return stb_fail(ctx, STB_E_INVALID_ARG,
                          "slab %lld is not slab 0 moved in time (panel %d vs %d): use GMRES",
                          (long long)n, p, q);
      }
    }
  }
  // ---- device: structure check, inverse of the diagonal block, time steps
  std::vector<int32_t> rflat((size_t)(S * K));
  for (int64_t n = 0; n < S; ++n)
    std::copy(rows[(size_t)n].begin(), rows[(size_t)n].end(), rflat.begin() + n * K);
  int32_t *d_slab = nullptr, *d_loc = nullptr, *d_rows = nullptr, *d_perm = nullptr;
  double *D = nullptr, *f = nullptr, *x = nullptr, *b = nullptr, *r = nullptr;
  unsigned long long* d_bad = nullptr;
  int* d_sing = nullptr;
  auto cleanup = [&]() {
    dfree(d_slab); dfree(d_loc); dfree(d_rows); dfree(d_perm); dfree(D); dfree(f); dfree(x); dfree(b);
    dfree(r); dfree(d_bad); dfree(d_sing);
  };
  if (dalloc(&d_slab, (size_t)nt) != hipSuccess || dalloc(&d_loc, (size_t)nt) != hipSuccess ||
      dalloc(&d_rows, (size_t)(S * K)) != hipSuccess || dalloc(&d_perm, (size_t)K) != hipSuccess ||
      dalloc(&D, (size_t)(K * K)) != hipSuccess || dalloc(&f, (size_t)K) != hipSuccess ||
      dalloc(&x, (size_t)nt) != hipSuccess || dalloc(&b, (size_t)nt) != hipSuccess ||
      dalloc(&r, (size_t)K) != hipSuccess || dalloc(&d_bad, 1) != hipSuccess || dalloc(&d_sing, 1) != hipSuccess) {
    cleanup();
    return stb_fail(ctx, STB_E_NO_MEMORY, "marching-on-in-time buffers (%lld panels per slab)", (long long)K);
  }
  hipError_t e = hipMemcpyAsync(d_slab, slab.data(), 4 * nt, hipMemcpyHostToDevice, st);
  if (e == hipSuccess) e = hipMemcpyAsync(d_loc, loc.data(), 4 * nt, hipMemcpyHostToDevice, st);
  if (e == hipSuccess) e = hipMemcpyAsync(d_rows, rflat.data(), 4 * S * K, hipMemcpyHostToDevice, st);
  if (e == hipSuccess) e = hipMemcpyAsync(b, b_host, 8 * nt, hipMemcpyHostToDevice, st);
  if (e == hipSuccess) e = hipMemsetAsync(d_bad, 0, 8, st);
  if (e == hipSuccess) e = hipMemsetAsync(d_sing, 0, sizeof(int), st);
  if (e == hipSuccess) e = hipMemsetAsync(D, 0, 8 * K * K, st);
  if (e == hipSuccess) e = hipMemsetAsync(x, 0, 8 * nt, st);
  if (e == hipSuccess) {
    hipLaunchKernelGGL(k_mot_lower, dim3((unsigned)((nt + 255) / 256)), dim3(256), 0, st, nt, A->d_rowptr,
                       A->d_cols, d_slab, d_bad);
    hipLaunchKernelGGL(k_mot_block, dim3((unsigned)((K + 255) / 256)), dim3(256), 0, st, K, d_rows,
                       A->d_rowptr, A->d_cols, A->d_vals, d_slab, d_loc, D);
    e = hipGetLastError();
  }
  unsigned long long bad = 0;
  if (e == hipSuccess) e = hipMemcpyAsync(&bad, d_bad, 8, hipMemcpyDeviceToHost, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  if (e != hipSuccess) { cleanup(); return stb_fail(ctx, STB_E_DEVICE, "marching-on-in-time: %s", hipGetErrorString(e)); }
  if (bad) {
    cleanup();
    return stb_fail(ctx, STB_E_INVALID_ARG,
                    "%llu stored entries couple a slab to a later one (not lower triangular in time): use GMRES",
                    bad);
  }
  const auto c0 = std::chrono::steady_clock::now();
  const unsigned gu = (unsigned)((K * K + 255) / 256);
  for (int64_t k = 0; k < K && e == hipSuccess; ++k) {
    hipLaunchKernelGGL(k_gj_pivot, dim3(1), dim3(kGjThreads), 0, st, K, k, D, d_perm, f, d_sing);
    hipLaunchKernelGGL(k_gj_update, dim3(gu), dim3(256), 0, st, K, k, D, f);
    e = hipGetLastError();
  }
  if (e == hipSuccess) {
    hipLaunchKernelGGL(k_gj_unswap, dim3((unsigned)((K + 255) / 256)), dim3(256), 0, st, K, D, d_perm);
    e = hipGetLastError();
  }
  int sing = 0;
  if (e == hipSuccess) e = hipMemcpyAsync(&sing, d_sing, sizeof(int), hipMemcpyDeviceToHost, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  const auto c1 = std::chrono::steady_clock::now();
  if (e == hipSuccess && !sing) {
    const unsigned gw = (unsigned)((K * 64 + 255) / 256);
    for (int64_t n = 0; n < S && e == hipSuccess; ++n) {
      hipLaunchKernelGGL(k_mot_rhs, dim3(gw), dim3(256), 0, st, K, d_rows + n * K, A->d_rowptr, A->d_cols,
                         A->d_vals, x, b, r);
      hipLaunchKernelGGL(k_mot_apply, dim3(gw), dim3(256), 0, st, K, d_rows + n * K, D, r, x);
      e = hipGetLastError();
    }
    if (e == hipSuccess) e = hipMemcpyAsync(x_host, x, 8 * nt, hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
  }
  const auto c2 = std::chrono::steady_clock::now();
  cleanup();
  if (e != hipSuccess) return stb_fail(ctx, STB_E_DEVICE, "marching-on-in-time: %s", hipGetErrorString(e));
  if (sing) return stb_fail(ctx, STB_E_INTERNAL, "the diagonal block is singular");
  if (info4) {
    info4[0] = (double)S;
    info4[1] = (double)K;
    info4[2] = std::chrono::duration<double, std::milli>(c1 - c0).count();
    info4[3] = std::chrono::duration<double, std::milli>(c2 - c1).count();
  }
  return STB_OK;
}

}  // extern "C"
