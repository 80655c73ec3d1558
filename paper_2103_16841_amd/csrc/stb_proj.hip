// stb_proj.hip -- the L2(Sigma) projection Q_h^1 onto V_h^1 (the data
// projection of the direct method, eq. df_dir): find c in V_h^1 with
// (c, lambda_k) = (g, lambda_k) for every vertex hat lambda_k.
//
// On a vertical panel dS = dtau dA is the 3-volume of the tetrahedron in its
// local (tau, u, v) frame, so the mass matrix is the tetrahedral one,
// M_kl = sum_sigma vol_sigma (1 + delta_kl) / 20, and (g, lambda_k) is taken
// with a fixed rule: 27 points per panel, the 3 x 3 x 3 Gauss-Legendre product
// rule on the cube collapsed onto the tetrahedron (xi_1 = a, xi_2 = (1 - a) b,
// xi_3 = (1 - a)(1 - b) c, weight w_a w_b w_c (1 - a)^2 (1 - b)), exact for
// polynomials of degree 3.  The caller evaluates g at the exported points.
// M is applied matrix-free by a gather over each vertex's panels (fixed
// order) and the system solved by Jacobi-preconditioned conjugate gradients
// with fixed-order dot products.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <vector>

#include "stb_internal.h"

using namespace stb;

namespace {

constexpr int kRulePts = STB_L2_POINTS;
constexpr int kThreads = 256;

struct Rule {
  double lam[kRulePts][4];   // barycentric coordinates of the points
  double w[kRulePts];        // weights on the reference tetrahedron (sum 1/6)
};

Rule make_rule() {
  const double g = 0.5 * std::sqrt(0.6);
  const double x[3] = {0.5 - g, 0.5, 0.5 + g};
  const double wt[3] = {5.0 / 18.0, 8.0 / 18.0, 5.0 / 18.0};
  Rule R;
  int p = 0;
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j)
      for (int k = 0; k < 3; ++k) {
        const double a = x[i], b = x[j], c = x[k];
        const double x1 = a, x2 = (1.0 - a) * b, x3 = (1.0 - a) * (1.0 - b) * c;
        R.lam[p][0] = 1.0 - x1 - x2 - x3;
        R.lam[p][1] = x1;
        R.lam[p][2] = x2;
        R.lam[p][3] = x3;
        R.w[p] = wt[i] * wt[j] * wt[k] * (1.0 - a) * (1.0 - a) * (1.0 - b);
        ++p;
      }
  return R;
}

// |det| of the panel's local (tau, u, v) edge vectors = 6 x its 3-volume.
__device__ double vol6_of(const TrialRec& T) {
  double a[3], b[3], c[3];
  for (int q = 0; q < 3; ++q) {
    a[q] = T.V[1][q] - T.V[0][q];
    b[q] = T.V[2][q] - T.V[0][q];
    c[q] = T.V[3][q] - T.V[0][q];
  }
  const double d = a[0] * (b[1] * c[2] - b[2] * c[1]) - a[1] * (b[0] * c[2] - b[2] * c[0]) +
                   a[2] * (b[0] * c[1] - b[1] * c[0]);
  return fabs(d);
}

__global__ void k_vol6(int64_t nt, const TrialRec* __restrict__ trial, double* __restrict__ vol6) {
  int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j < nt) vol6[j] = vol6_of(trial[j]);
}

__global__ void k_l2_points(int64_t nt, const double* __restrict__ vtx, const int32_t* __restrict__ tet,
                            const double* __restrict__ vol6, Rule R, double* __restrict__ pts,
                            double* __restrict__ wts) {
  int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= nt * kRulePts) return;
  const int64_t j = g / kRulePts;
  const int p = (int)(g % kRulePts);
  double x[4] = {0.0, 0.0, 0.0, 0.0};
  for (int m = 0; m < 4; ++m) {
    const double* X = vtx + 4 * (int64_t)tet[4 * j + m];
    for (int c = 0; c < 4; ++c) x[c] += R.lam[p][m] * X[c];
  }
  for (int c = 0; c < 4; ++c) pts[4 * g + c] = x[c];
  wts[g] = vol6[j] * R.w[p];
}

// f_k = sum over the panels at vertex k (ascending panel) of sum_p w g lambda_m.
__global__ void k_l2_rhs(int64_t nv, const int64_t* __restrict__ ptr, const int64_t* __restrict__ adj,
                         const double* __restrict__ gq, const double* __restrict__ vol6, Rule R,
                         double* __restrict__ f) {
  int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= nv) return;
  double s = 0.0;
  for (int64_t e = ptr[k]; e < ptr[k + 1]; ++e) {
    const int64_t j = adj[e] >> 2;
    const int m = (int)(adj[e] & 3);
    double t = 0.0;
    for (int p = 0; p < kRulePts; ++p) t += R.w[p] * gq[j * kRulePts + p] * R.lam[p][m];
    s += vol6[j] * t;
  }
  f[k] = s;
}

// y = M x and the diagonal: M_kl = (vol6 / 6) (1 + delta_kl) / 20 per panel.
__global__ void k_l2_apply(int64_t nv, const int64_t* __restrict__ ptr, const int64_t* __restrict__ adj,
                           const int32_t* __restrict__ tet, const double* __restrict__ vol6,
                           const double* __restrict__ x, double* __restrict__ y, double* __restrict__ diag) {
  int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= nv) return;
  double s = 0.0, d = 0.0;
  for (int64_t e = ptr[k]; e < ptr[k + 1]; ++e) {
    const int64_t j = adj[e] >> 2;
    const int32_t* tv = tet + 4 * j;
    const double c = vol6[j] / 120.0;
    s += c * (((x[tv[0]] + x[tv[1]]) + (x[tv[2]] + x[tv[3]])) + x[k]);
    d += 2.0 * c;
  }
  y[k] = s;
  if (diag) diag[k] = d;
}

// out[0] = <a, b> (one block, fixed order).
__global__ __launch_bounds__(kThreads) void k_dot(int64_t n, const double* __restrict__ a,
                                                  const double* __restrict__ b, double* __restrict__ out) {
  double s = 0.0;
  for (int64_t i = threadIdx.x; i < n; i += kThreads) s += a[i] * b[i];
  __shared__ double red[kThreads];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int off = kThreads / 2; off > 0; off >>= 1) {
    if ((int)threadIdx.x < off) red[threadIdx.x] += red[threadIdx.x + off];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[0] = red[0];
}

// CG steps: x += alpha p, r -= alpha q, z = r / diag.
__global__ void k_cg_step(int64_t n, double alpha, const double* __restrict__ p, const double* __restrict__ q,
                          const double* __restrict__ diag, double* __restrict__ x, double* __restrict__ r,
                          double* __restrict__ z) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  x[i] = fma(alpha, p[i], x[i]);
  const double ri = fma(-alpha, q[i], r[i]);
  r[i] = ri;
  z[i] = ri / diag[i];
}

// p = z + beta p; with init: r = f - y, z = r / diag, p = z.
__global__ void k_cg_dir(int64_t n, double beta, const double* __restrict__ z, double* __restrict__ p) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = fma(beta, p[i], z[i]);
}

__global__ void k_cg_init(int64_t n, const double* __restrict__ f, const double* __restrict__ y,
                          const double* __restrict__ diag, double* __restrict__ r, double* __restrict__ z,
                          double* __restrict__ p) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double ri = f[i] - y[i];
  r[i] = ri;
  z[i] = ri / diag[i];
  p[i] = z[i];
}

unsigned blocks(int64_t n) { return (unsigned)((n + kThreads - 1) / kThreads); }

}  // namespace

// Vertex -> (panel, local vertex) lists and panel volumes, built once per mesh.
static stb_status ensure_adjacency(stb_ctx* ctx, stb_mesh* m) {
  if (m->d_v2t_ptr) return STB_OK;
  const int64_t nt = m->nt, nv = m->nv;
  std::vector<int32_t> tet((size_t)nt * 4);
  HIPCHK(ctx, hipMemcpyAsync(tet.data(), m->d_tet, sizeof(int32_t) * 4 * nt, hipMemcpyDeviceToHost, ctx->stream));
  HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
  std::vector<int64_t> ptr((size_t)nv + 1, 0), adj((size_t)nt * 4);
  for (int64_t e = 0; e < 4 * nt; ++e) ++ptr[(size_t)tet[e] + 1];
  for (int64_t k = 0; k < nv; ++k) ptr[k + 1] += ptr[k];
  std::vector<int64_t> fill(ptr.begin(), ptr.end() - 1);
  for (int64_t j = 0; j < nt; ++j)          // ascending panel within each vertex
    for (int q = 0; q < 4; ++q) adj[(size_t)fill[tet[4 * j + q]]++] = 4 * j + q;
  int64_t *d_ptr = nullptr, *d_adj = nullptr;
  double* d_vol6 = nullptr;
  if (dalloc(&d_ptr, (size_t)nv + 1) != hipSuccess || dalloc(&d_adj, (size_t)nt * 4) != hipSuccess ||
      dalloc(&d_vol6, (size_t)nt) != hipSuccess) {
    dfree(d_ptr); dfree(d_adj); dfree(d_vol6);
    return stb_fail(ctx, STB_E_NO_MEMORY, "projection adjacency");
  }
  hipError_t e = hipMemcpyAsync(d_ptr, ptr.data(), sizeof(int64_t) * (nv + 1), hipMemcpyHostToDevice, ctx->stream);
  if (e == hipSuccess)
    e = hipMemcpyAsync(d_adj, adj.data(), sizeof(int64_t) * 4 * nt, hipMemcpyHostToDevice, ctx->stream);
  if (e == hipSuccess && nt > 0) {
    hipLaunchKernelGGL(k_vol6, dim3(blocks(nt)), dim3(kThreads), 0, ctx->stream, nt, m->d_trial, d_vol6);
    e = hipGetLastError();
  }
  if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
  if (e != hipSuccess) {
    dfree(d_ptr); dfree(d_adj); dfree(d_vol6);
    return stb_fail(ctx, STB_E_DEVICE, "projection adjacency: %s", hipGetErrorString(e));
  }
  m->d_v2t_ptr = d_ptr;
  m->d_v2t = d_adj;
  m->d_vol6 = d_vol6;
  return STB_OK;
}

void stb_free_projection(stb_mesh* m) {
  dfree(m->d_v2t_ptr); dfree(m->d_v2t); dfree(m->d_vol6);
  m->d_v2t_ptr = nullptr;
  m->d_v2t = nullptr;
  m->d_vol6 = nullptr;
}

extern "C" {

stb_status stb_l2_points(stb_ctx* ctx, const stb_mesh* mesh_c, double* pts, double* wts) {
  if (!ctx || !mesh_c || !pts || !wts) return stb_fail(ctx, STB_E_INVALID_ARG, "bad arguments");
  stb_mesh* m = const_cast<stb_mesh*>(mesh_c);
  if (m->ctx != ctx) return stb_fail(ctx, STB_E_INVALID_ARG, "mesh belongs to another context");
  const int64_t nt = m->nt;
  if (nt == 0) return STB_OK;
  HIPCHK(ctx, hipSetDevice(ctx->device));
  stb_status s = ensure_adjacency(ctx, m);
  if (s) return s;
  double *d_pts = nullptr, *d_w = nullptr;
  if (dalloc(&d_pts, (size_t)nt * kRulePts * 4) != hipSuccess || dalloc(&d_w, (size_t)nt * kRulePts) != hipSuccess) {
    dfree(d_pts); dfree(d_w);
    return stb_fail(ctx, STB_E_NO_MEMORY, "projection points");
  }
  hipLaunchKernelGGL(k_l2_points, dim3(blocks(nt * kRulePts)), dim3(kThreads), 0, ctx->stream, nt, m->d_vtx,
                     m->d_tet, m->d_vol6, make_rule(), d_pts, d_w);
  hipError_t e = hipGetLastError();
  if (e == hipSuccess)
    e = hipMemcpyAsync(pts, d_pts, sizeof(double) * nt * kRulePts * 4, hipMemcpyDeviceToHost, ctx->stream);
  if (e == hipSuccess) e = hipMemcpyAsync(wts, d_w, sizeof(double) * nt * kRulePts, hipMemcpyDeviceToHost, ctx->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
  dfree(d_pts);
  dfree(d_w);
  if (e != hipSuccess) return stb_fail(ctx, STB_E_DEVICE, "projection points: %s", hipGetErrorString(e));
  return STB_OK;
}

stb_status stb_project_V1(stb_ctx* ctx, const stb_mesh* mesh_c, const double* gq, double* out,
                          int32_t* iters) {
  if (!ctx || !mesh_c || !gq || !out) return stb_fail(ctx, STB_E_INVALID_ARG, "bad arguments");
  stb_mesh* m = const_cast<stb_mesh*>(mesh_c);
  if (m->ctx != ctx) return stb_fail(ctx, STB_E_INVALID_ARG, "mesh belongs to another context");
  const int64_t nt = m->nt, nv = m->nv;
  for (int64_t i = 0; i < nt * kRulePts; ++i)
    if (!std::isfinite(gq[i])) return stb_fail(ctx, STB_E_INVALID_ARG, "non-finite value %lld", (long long)i);
  if (iters) *iters = 0;
  HIPCHK(ctx, hipSetDevice(ctx->device));
  stb_status s = ensure_adjacency(ctx, m);
  if (s) return s;
  double *d_g = nullptr, *d_f = nullptr, *d_x = nullptr, *d_r = nullptr, *d_z = nullptr, *d_p = nullptr,
         *d_q = nullptr, *d_d = nullptr, *d_s = nullptr;
  auto cleanup = [&]() {
    dfree(d_g); dfree(d_f); dfree(d_x); dfree(d_r); dfree(d_z); dfree(d_p); dfree(d_q); dfree(d_d); dfree(d_s);
  };
  if (dalloc(&d_g, (size_t)nt * kRulePts) != hipSuccess || dalloc(&d_f, (size_t)nv) != hipSuccess ||
      dalloc(&d_x, (size_t)nv) != hipSuccess || dalloc(&d_r, (size_t)nv) != hipSuccess ||
      dalloc(&d_z, (size_t)nv) != hipSuccess || dalloc(&d_p, (size_t)nv) != hipSuccess ||
      dalloc(&d_q, (size_t)nv) != hipSuccess || dalloc(&d_d, (size_t)nv) != hipSuccess ||
      dalloc(&d_s, 2) != hipSuccess) {
    cleanup();
    return stb_fail(ctx, STB_E_NO_MEMORY, "projection buffers");
  }
  hipStream_t st = ctx->stream;
  auto dot = [&](const double* a, const double* b, double* res) -> hipError_t {
    hipLaunchKernelGGL(k_dot, dim3(1), dim3(kThreads), 0, st, nv, a, b, d_s);
    hipError_t e = hipGetLastError();
    if (e == hipSuccess) e = hipMemcpyAsync(res, d_s, sizeof(double), hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    return e;
  };
  const Rule R = make_rule();
  hipError_t e = hipMemcpyAsync(d_g, gq, sizeof(double) * nt * kRulePts, hipMemcpyHostToDevice, st);
  if (e == hipSuccess) {
    hipLaunchKernelGGL(k_l2_rhs, dim3(blocks(nv)), dim3(kThreads), 0, st, nv, m->d_v2t_ptr, m->d_v2t, d_g,
                       m->d_vol6, R, d_f);
    e = hipGetLastError();
  }
  int it = 0;
  bool done = false;
  if (e == hipSuccess) e = hipMemsetAsync(d_x, 0, sizeof(double) * nv, st);   // x0 = 0
  if (e == hipSuccess) {
    hipLaunchKernelGGL(k_l2_apply, dim3(blocks(nv)), dim3(kThreads), 0, st, nv, m->d_v2t_ptr, m->d_v2t,
                       m->d_tet, m->d_vol6, d_x, d_q, d_d);
    hipLaunchKernelGGL(k_cg_init, dim3(blocks(nv)), dim3(kThreads), 0, st, nv, d_f, d_q, d_d, d_r, d_z, d_p);
    e = hipGetLastError();
  }
  double ff = 0.0, rz = 0.0;
  if (e == hipSuccess) e = dot(d_f, d_f, &ff);
  if (e == hipSuccess) e = dot(d_r, d_z, &rz);
  const double tol2 = 1e-26 * ff;   // relative residual 1e-13
  const int maxit = 1000;
  double rr = ff;
  while (e == hipSuccess && !done) {
    if (rr <= tol2 || ff == 0.0) { done = true; break; }
    if (it >= maxit) break;
    hipLaunchKernelGGL(k_l2_apply, dim3(blocks(nv)), dim3(kThreads), 0, st, nv, m->d_v2t_ptr, m->d_v2t,
                       m->d_tet, m->d_vol6, d_p, d_q, nullptr);
    double pq = 0.0;
    if ((e = hipGetLastError()) != hipSuccess || (e = dot(d_p, d_q, &pq)) != hipSuccess) break;
    if (!(pq > 0.0)) break;
    const double alpha = rz / pq;
    hipLaunchKernelGGL(k_cg_step, dim3(blocks(nv)), dim3(kThreads), 0, st, nv, alpha, d_p, d_q, d_d, d_x, d_r,
                       d_z);
    double rz1 = 0.0;
    if ((e = hipGetLastError()) != hipSuccess || (e = dot(d_r, d_z, &rz1)) != hipSuccess ||
        (e = dot(d_r, d_r, &rr)) != hipSuccess)
      break;
    hipLaunchKernelGGL(k_cg_dir, dim3(blocks(nv)), dim3(kThreads), 0, st, nv, rz1 / rz, d_z, d_p);
    if ((e = hipGetLastError()) != hipSuccess) break;
    rz = rz1;
    ++it;
  }
  if (e == hipSuccess) e = hipMemcpyAsync(out, d_x, sizeof(double) * nv, hipMemcpyDeviceToHost, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  cleanup();
  if (iters) *iters = it;
  if (e != hipSuccess) return stb_fail(ctx, STB_E_DEVICE, "projection failed: %s", hipGetErrorString(e));
  if (!done) return stb_fail(ctx, STB_E_INTERNAL, "projection: CG did not converge in %d steps", it);
  return STB_OK;
}

}  // extern "C"
