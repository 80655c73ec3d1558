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

}  // extern "C"
