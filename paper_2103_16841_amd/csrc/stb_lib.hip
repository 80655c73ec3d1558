// stb_lib.hip -- MI355X (gfx950) implementation of the C ABI in include/stb.h.
//
// Pipeline of stb_assemble_V (energetic single-layer Galerkin matrix,
// Poelz & Schanz arXiv 2103.16841, eq. df_ind / eq. int_bform):
//   k_geometry   per panel: frame, face half-spaces (eq. pnl_ilf), bounds;
//   k_outer      per test panel: outer points and weights of the composite
//                centroid rule on its faces (Fig. int_tri_mid);
//   k_cull_*     conservative causal cull of (test, trial) pairs from the
//                bounding balls and time ranges (superset of the lit pairs of
//                Sec. 3.3), compacted per row with wavefront ballots;
//   pair pipeline (stb_pairs.hip): lit test, breakpoints, empty-piece tests,
//                Gauss nodes, ordered sums, store.
// The store is CSR over the candidate columns (values aligned with them).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "stb.h"
#include "stb_device.h"

using namespace stb;

#include "stb_internal.h"
#include "stb_pairs.h"

static std::mutex g_err_mu;
static std::string g_err;

stb_status stb_fail(stb_ctx* ctx, stb_status s, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  if (ctx) ctx->err = buf;
  else {
    std::lock_guard<std::mutex> g(g_err_mu);
    g_err = buf;
  }
  return s;
}
#define fail stb_fail


// ---------------------------------------------------------------- kernels

// status[j] = 5 when a vertex index of panel j is out of range.
__global__ void k_check_index(int64_t nt, int64_t nv, const int32_t* __restrict__ tet,
                              int32_t* __restrict__ status) {
  int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= nt) return;
  int bad = 0;
  for (int k = 0; k < 4; ++k) bad |= (tet[4 * j + k] < 0 || tet[4 * j + k] >= nv);
  status[j] = bad ? 5 : 0;
}

// Panel geometry.  status[j]: 0 ok, 1 non-finite, else as make_trial.
__global__ void k_geometry(int64_t nt, const double* __restrict__ vtx,
                           const int32_t* __restrict__ tet, TrialRec* __restrict__ out,
                           FaceAng* __restrict__ fang, int32_t* __restrict__ status) {
  int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= nt) return;
  double X[4][4];
  int st = 0;
  for (int k = 0; k < 4; ++k) {
    const double* v = vtx + 4 * (int64_t)tet[4 * j + k];
    for (int c = 0; c < 4; ++c) {
      X[k][c] = v[c];
      if (!isfinite(v[c])) st = 1;
    }
  }
  if (st == 0) {
    TrialRec R;
    st = make_trial(X, R);
    if (st == 0) {
      out[j] = R;
      FaceAng F;
      face_angles(R, F);
      fang[j] = F;
    }
  }
  status[j] = st;
}

// Outer points of eq. int_bform: centroids of the m^2 congruent sub-triangles
// of every face with nu_t != 0, weight -nu_t |F| / m^2; plus the apex box.
__global__ void k_outer(int64_t nt, const TrialRec* __restrict__ rec, int m, int maxq,
                        double* __restrict__ pts, double* __restrict__ wts,
                        int32_t* __restrict__ nq, ApexBox* __restrict__ box) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nt) return;
  const TrialRec& R = rec[i];
  double* P = pts + (int64_t)i * maxq * 4;
  double* W = wts + (int64_t)i * maxq;
  int cnt = make_outer(R, m, P, W);
  nq[i] = cnt;
  ApexBox B;
  B.tlo = 1e300; B.thi = -1e300;
  double c[3] = {0, 0, 0};
  for (int q = 0; q < cnt; ++q) {
    B.tlo = fmin(B.tlo, P[4 * q]);
    B.thi = fmax(B.thi, P[4 * q]);
    for (int d = 0; d < 3; ++d) c[d] += P[4 * q + 1 + d] / cnt;
  }
  double rho = 0.0;
  for (int q = 0; q < cnt; ++q) {
    double dx = P[4 * q + 1] - c[0], dy = P[4 * q + 2] - c[1], dz = P[4 * q + 3] - c[2];
    rho = fmax(rho, sqrt(dx * dx + dy * dy + dz * dz));
  }
  B.cx = c[0]; B.cy = c[1]; B.cz = c[2]; B.rho = rho * (1.0 + 1e-12);
  B.pad[0] = B.pad[1] = 0.0;
  box[i] = B;
}

// Apex boxes of single evaluation points.
__global__ void k_point_boxes(int64_t np, const double* __restrict__ pts, ApexBox* __restrict__ box) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= np) return;
  ApexBox B;
  B.tlo = B.thi = pts[4 * i];
  B.cx = pts[4 * i + 1]; B.cy = pts[4 * i + 2]; B.cz = pts[4 * i + 3];
  B.rho = 0.0;
  B.pad[0] = B.pad[1] = 0.0;
  box[i] = B;
}

// Conservative causal test: some apex of the box and some point of the
// panel with |x - y| = t - tau requires t - tau >= dist >= lower bound, and a
// crossing needs a point outside the cone: t - tau < dist <= upper bound.
// The panel fields the cull reads.
struct CullPanel {
  double cx, cy, cz, rad, tmin, tmax, diam;
};

__device__ __forceinline__ CullPanel cull_panel(const TrialRec& T) {
  return CullPanel{T.cx, T.cy, T.cz, T.rad, T.tmin, T.tmax, T.diam};
}

__device__ __forceinline__ bool maybe_lit(const ApexBox& b, const CullPanel& T) {
  double dx = b.cx - T.cx, dy = b.cy - T.cy, dz = b.cz - T.cz;
  double dc = sqrt(dx * dx + dy * dy + dz * dz);
  double lb = dc - b.rho - T.rad, ub = dc + b.rho + T.rad;
  double slack = 1e-9 * (fabs(b.thi - T.tmin) + T.diam + b.rho);
  return (b.thi - T.tmin > lb - slack) && (b.tlo - T.tmax < ub + slack);
}

constexpr int kCullThreads = 256;
// Rows per block: each panel record read from L2 serves this many rows.
constexpr int kCullRows = 8;

__global__ __launch_bounds__(kCullThreads) void k_cull_count(int64_t nrows,
                                                             const ApexBox* __restrict__ rows,
                                                             int64_t nt,
                                                             const TrialRec* __restrict__ T,
                                                             int64_t* __restrict__ cnt) {
  const int64_t i0 = (int64_t)blockIdx.x * kCullRows;
  if (i0 >= nrows) return;
  const int nr = (int)std::min<int64_t>(kCullRows, nrows - i0);
  __shared__ ApexBox s_b[kCullRows];
  __shared__ int red[kCullRows][kCullThreads];
  if ((int)threadIdx.x < nr) s_b[threadIdx.x] = rows[i0 + threadIdx.x];
  __syncthreads();
  int c[kCullRows];
#pragma unroll
  for (int r = 0; r < kCullRows; ++r) c[r] = 0;
  for (int64_t j = threadIdx.x; j < nt; j += kCullThreads) {
    const CullPanel P = cull_panel(T[j]);
#pragma unroll
    for (int r = 0; r < kCullRows; ++r)
      if (r < nr) c[r] += maybe_lit(s_b[r], P) ? 1 : 0;
  }
#pragma unroll
  for (int r = 0; r < kCullRows; ++r) red[r][threadIdx.x] = c[r];
  __syncthreads();
  for (int off = kCullThreads / 2; off > 0; off >>= 1) {
    if ((int)threadIdx.x < off)
#pragma unroll
      for (int r = 0; r < kCullRows; ++r) red[r][threadIdx.x] += red[r][threadIdx.x + off];
    __syncthreads();
  }
  if ((int)threadIdx.x < nr) cnt[i0 + threadIdx.x] = red[threadIdx.x][0];
}

// Fill the candidate columns of each row in ascending order: per 256-wide
// chunk of panels (read once for the block's rows), a wavefront ballot +
// mbcnt gives each lane its rank inside the wave per row; an LDS prefix
// over the four waves orders the chunk.
__global__ __launch_bounds__(kCullThreads) void k_cull_fill(int64_t nrows,
                                                            const ApexBox* __restrict__ rows,
                                                            int64_t nt,
                                                            const TrialRec* __restrict__ T,
                                                            const int64_t* __restrict__ rowptr,
                                                            int32_t* __restrict__ cols,
                                                            int32_t* __restrict__ rowof) {
  const int64_t i0 = (int64_t)blockIdx.x * kCullRows;
  if (i0 >= nrows) return;
  const int nr = (int)std::min<int64_t>(kCullRows, nrows - i0);
  constexpr int kWaves = kCullThreads / 64;
  __shared__ ApexBox s_b[kCullRows];
  __shared__ int wave_cnt[kCullRows][kWaves];
  if ((int)threadIdx.x < nr) s_b[threadIdx.x] = rows[i0 + threadIdx.x];
  __syncthreads();
  int64_t base[kCullRows];
#pragma unroll
  for (int r = 0; r < kCullRows; ++r) base[r] = r < nr ? rowptr[i0 + r] : 0;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  for (int64_t j0 = 0; j0 < nt; j0 += kCullThreads) {
    const int64_t j = j0 + threadIdx.x;
    CullPanel P{};
    if (j < nt) P = cull_panel(T[j]);
    uint32_t pm = 0;   // rows for which panel j is a candidate
    int rank[kCullRows];
#pragma unroll
    for (int r = 0; r < kCullRows; ++r) {
      const bool p = r < nr && j < nt && maybe_lit(s_b[r], P);
      const uint64_t bal = __ballot(p);
      rank[r] = __builtin_amdgcn_mbcnt_hi((uint32_t)(bal >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)bal, 0));
      if (lane == 0) wave_cnt[r][wave] = __popcll(bal);
      pm |= (p ? 1u : 0u) << r;
    }
    __syncthreads();
#pragma unroll
    for (int r = 0; r < kCullRows; ++r) {
      int off = 0, tot = 0;
      for (int w = 0; w < kWaves; ++w) {
        off += w < wave ? wave_cnt[r][w] : 0;
        tot += wave_cnt[r][w];
      }
      if ((pm >> r) & 1u) {
        cols[base[r] + off + rank[r]] = (int32_t)j;
        rowof[base[r] + off + rank[r]] = (int32_t)(i0 + r);
      }
      base[r] += tot;
    }
    __syncthreads();
  }
}

// One lane per (point, panel) pair: the whole inner integral serially.
__global__ void k_inner_values(int64_t k, const TrialRec* __restrict__ trial,
                               const double* __restrict__ pts, const int32_t* __restrict__ panel,
                               const double* __restrict__ gl, int ng, double* __restrict__ out) {
  int64_t m = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (m >= k) return;
  double x4[4] = {pts[4 * m], pts[4 * m + 1], pts[4 * m + 2], pts[4 * m + 3]};
  out[m] = inner_serial(trial[panel[m]], x4, ng, gl, gl + kMaxNg, nullptr);
}

// Potential per evaluation point: ordered sum over its candidates of
// w_j I_j (exact zeros skipped).
// u(p) = sum_j w_j I_pj over the point's candidates: one wavefront per
// point, lane-strided partial sums and a fixed-order shuffle reduction.
__global__ __launch_bounds__(256) void k_point_sum(int64_t np, const int64_t* __restrict__ rowptr,
                                                   const int32_t* __restrict__ cols,
                                                   const double* __restrict__ I,
                                                   const double* __restrict__ w,
                                                   double* __restrict__ out) {
  const int lane = threadIdx.x & 63;
  const int64_t waves = ((int64_t)gridDim.x * blockDim.x) >> 6;
  for (int64_t i = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6; i < np; i += waves) {
    double s = 0.0;
    for (int64_t c = rowptr[i] + lane; c < rowptr[i + 1]; c += 64)
      if (I[c] != 0.0) s += w[cols[c]] * I[c];
    for (int off = 32; off > 0; off >>= 1) s += __shfl_down(s, off, 64);
    if (lane == 0) out[i] = s;
  }
}

// y = A w (FP64 CSR), one wavefront per row, fixed-order reduction.  Eight
// (then four) entries per lane and pass, with four partial sums: the loads
// of a pass are all in flight before the first product needs them (one
// entry per pass waits out a column load and a gather every time).
__global__ __launch_bounds__(256) void k_spmv(int64_t n, const int64_t* __restrict__ rowptr,
                                              const int32_t* __restrict__ cols,
                                              const double* __restrict__ vals,
                                              const double* __restrict__ w, int nrhs, int col,
                                              double* __restrict__ y) {
  const int lane = threadIdx.x & 63;
  const int64_t waves = ((int64_t)gridDim.x * blockDim.x) >> 6;
  for (int64_t row = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6; row < n; row += waves) {
    const int64_t e = rowptr[row + 1];
    int64_t k = rowptr[row] + lane;
    double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
    for (; k + 448 < e; k += 512) {
      int32_t c[8];
      double v[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        c[u] = cols[k + 64 * u];
        v[u] = vals[k + 64 * u];
      }
      double x[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) x[u] = w[(int64_t)c[u] * nrhs + col];
      s0 = fma(v[0], x[0], s0);
      s1 = fma(v[1], x[1], s1);
      s2 = fma(v[2], x[2], s2);
      s3 = fma(v[3], x[3], s3);
      s0 = fma(v[4], x[4], s0);
      s1 = fma(v[5], x[5], s1);
      s2 = fma(v[6], x[6], s2);
      s3 = fma(v[7], x[7], s3);
    }
    for (; k + 192 < e; k += 256) {
      const int32_t c0 = cols[k], c1 = cols[k + 64], c2 = cols[k + 128], c3 = cols[k + 192];
      const double v0 = vals[k], v1 = vals[k + 64], v2 = vals[k + 128], v3 = vals[k + 192];
      s0 = fma(v0, w[(int64_t)c0 * nrhs + col], s0);
      s1 = fma(v1, w[(int64_t)c1 * nrhs + col], s1);
      s2 = fma(v2, w[(int64_t)c2 * nrhs + col], s2);
      s3 = fma(v3, w[(int64_t)c3 * nrhs + col], s3);
    }
    for (; k < e; k += 64) s0 = fma(vals[k], w[(int64_t)cols[k] * nrhs + col], s0);
    double s = (s0 + s1) + (s2 + s3);
    for (int off = 32; off > 0; off >>= 1) s += __shfl_down(s, off, 64);
    if (lane == 0) y[row * nrhs + col] = s;
  }
}

// Compaction of a store to its causal entries: one wavefront per row counts
// the row's flags; after the scan of the counts, one wavefront per row
// copies the flagged entries in order (ballot + mbcnt give each lane its
// slot among the 64 entries in flight).
__global__ __launch_bounds__(256) void k_keep_count(int64_t n, const int64_t* __restrict__ rowptr,
                                                    const uint8_t* __restrict__ flag,
                                                    int64_t* __restrict__ cnt) {
  const int64_t row = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  const int lane = threadIdx.x & 63;
  if (row >= n) return;
  int64_t c = 0;
  for (int64_t k = rowptr[row] + lane; k < rowptr[row + 1]; k += 64) c += flag[k] ? 1 : 0;
  for (int off = 32; off > 0; off >>= 1) c += __shfl_down(c, off, 64);
  if (lane == 0) cnt[row] = c;
}

__global__ __launch_bounds__(256) void k_keep_fill(int64_t n, const int64_t* __restrict__ rowptr,
                                                   const int32_t* __restrict__ cols,
                                                   const double* __restrict__ vals,
                                                   const uint8_t* __restrict__ flag,
                                                   const int64_t* __restrict__ nrowptr,
                                                   int32_t* __restrict__ ncols,
                                                   double* __restrict__ nvals) {
  const int64_t row = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  const int lane = threadIdx.x & 63;
  if (row >= n) return;
  int64_t out = nrowptr[row];
  for (int64_t k0 = rowptr[row]; k0 < rowptr[row + 1]; k0 += 64) {
    const int64_t k = k0 + lane;
    const bool p = k < rowptr[row + 1] && flag[k] != 0;
    const uint64_t bal = __ballot(p);
    const int rank = (int)__builtin_amdgcn_mbcnt_hi((uint32_t)(bal >> 32),
                                                    __builtin_amdgcn_mbcnt_lo((uint32_t)bal, 0));
    if (p) {
      ncols[out + rank] = cols[k];
      nvals[out + rank] = vals[k];
    }
    out += __popcll(bal);
  }
}

// Entries (row[m], col[m]) of a CSR store with ascending columns: one lane
// per entry, bisection in the row; 0.0 where the column is not stored.
__global__ void k_mat_get(int64_t k, const int64_t* __restrict__ rowptr, const int32_t* __restrict__ cols,
                          const double* __restrict__ vals, const int32_t* __restrict__ row,
                          const int32_t* __restrict__ col, double* __restrict__ out) {
  const int64_t m = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (m >= k) return;
  int64_t lo = rowptr[row[m]], hi = rowptr[row[m] + 1];
  const int64_t end = hi;
  const int32_t c = col[m];
  while (lo < hi) {
    const int64_t mid = lo + ((hi - lo) >> 1);
    if (cols[mid] < c) lo = mid + 1;
    else hi = mid;
  }
  out[m] = (lo < end && cols[lo] == c) ? vals[lo] : 0.0;
}

// ---------------------------------------------------------------- host helpers

// Gauss-Legendre on [0,1] by Newton iteration on the three-term recurrence.
static void gauss_legendre01(int n, double* x, double* w) {
  for (int i = 0; i < n; ++i) {
    double z = std::cos(kPi * (i + 0.75) / (n + 0.5)), pn = 0.0, dpn = 1.0;
    for (int it = 0; it < 100; ++it) {
      double p_prev = 1.0, p = z;
      for (int k = 2; k <= n; ++k) {
        double p_next = ((2 * k - 1) * z * p - (k - 1) * p_prev) / k;
        p_prev = p;
        p = p_next;
      }
      if (n == 1) { p = z; p_prev = 1.0; }
      pn = p;
      dpn = n * (z * p - p_prev) / (z * z - 1.0);
      double dz = pn / dpn;
      z -= dz;
      if (std::fabs(dz) < 1e-16) break;
    }
    double p_prev = 1.0, p = z;
    for (int k = 2; k <= n; ++k) {
      double p_next = ((2 * k - 1) * z * p - (k - 1) * p_prev) / k;
      p_prev = p;
      p = p_next;
    }
    dpn = n * (z * p - p_prev) / (z * z - 1.0);
    x[i] = 0.5 * (1.0 - z);
    w[i] = 1.0 / ((1.0 - z * z) * dpn * dpn);
  }
}

stb_status stb_ensure_gl(stb_ctx* ctx, int ng) {
  if (ctx->gl_n == ng && ctx->d_gl) return STB_OK;
  // nodes u_g and weights w_g on [0, 1], then per node the offset of its
  // smoothstep-mapped angle from a piece's midpoint, 1/2 - s(u_g), and its
  // weight factor s'(u_g) w_g (s(u) = 3u^2 - 2u^3), both per unit length
  double h[4 * kMaxNg] = {0};
  gauss_legendre01(ng, h, h + kMaxNg);
  for (int g = 0; g < ng; ++g) {
    const double u = h[g];
    h[2 * kMaxNg + g] = 0.5 - u * u * (3.0 - 2.0 * u);
    h[3 * kMaxNg + g] = (6.0 * u * (1.0 - u)) * h[kMaxNg + g];
  }
  if (!ctx->d_gl) HIPCHK(ctx, dalloc(&ctx->d_gl, 4 * kMaxNg));
  HIPCHK(ctx, hipMemcpyAsync(ctx->d_gl, h, sizeof(h), hipMemcpyHostToDevice, ctx->stream));
  HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
  ctx->gl_n = ng;
  return STB_OK;
}

stb_status stb_check_params(stb_ctx* ctx, const stb_quad_params* p) {
  if (p->m_q < 1 || p->m_q > 4) return fail(ctx, STB_E_INVALID_ARG, "m_q must be in [1,4], got %d", p->m_q);
  if (p->n_g < 2 || p->n_g > kMaxNg) return fail(ctx, STB_E_INVALID_ARG, "n_g must be in [2,%d], got %d", kMaxNg, p->n_g);
  if (p->prec != STB_FP64 && p->prec != STB_MIXED) return fail(ctx, STB_E_INVALID_ARG, "bad precision");
  if (!(p->eta_far >= 0.0) || !std::isfinite(p->eta_far))
    return fail(ctx, STB_E_INVALID_ARG, "eta_far must be finite and >= 0");
  if (p->lit_search != STB_LIT_TREE && p->lit_search != STB_LIT_FLAT)
    return fail(ctx, STB_E_INVALID_ARG, "bad lit search %d", p->lit_search);
  if (p->n_min < 1 || p->n_min > 4096) return fail(ctx, STB_E_INVALID_ARG, "n_min must be in [1,4096], got %d", p->n_min);
  return STB_OK;
}

stb_status stb_ensure_outer(stb_ctx* ctx, stb_mesh* m, int mq) {
  if (m->mq == mq && m->d_opts) return STB_OK;
  dfree(m->d_opts); dfree(m->d_ow); dfree(m->d_onq); dfree(m->d_box);
  m->d_opts = nullptr; m->d_ow = nullptr; m->d_onq = nullptr; m->d_box = nullptr;
  int maxq = 4 * mq * mq;
  HIPCHK(ctx, dalloc(&m->d_opts, (size_t)m->nt * maxq * 4));
  HIPCHK(ctx, dalloc(&m->d_ow, (size_t)m->nt * maxq));
  HIPCHK(ctx, dalloc(&m->d_onq, (size_t)m->nt));
  HIPCHK(ctx, dalloc(&m->d_box, (size_t)m->nt));
  if (m->nt > 0) {
    hipLaunchKernelGGL(k_outer, dim3((unsigned)((m->nt + 127) / 128)), dim3(128), 0, ctx->stream,
                       m->nt, m->d_trial, mq, maxq, m->d_opts, m->d_ow, m->d_onq, m->d_box);
    HIPCHK(ctx, hipGetLastError());
  }
  m->mq = mq;
  m->maxq = maxq;
  return STB_OK;
}

// Exclusive scan of n int64 counts into out[0..n] (device), with the
// library's own three-pass scan (stb_scan.hip); synchronises st.
stb_status stb_exclusive_scan(stb_ctx* ctx, const int64_t* in, int64_t* out, int64_t n,
                              hipStream_t st) {
  int64_t* tmp = nullptr;
  HIPCHK(ctx, dalloc(&tmp, (size_t)stb_scan_tmp_elems<int64_t>(n)));
  hipError_t e = stb_scan<int64_t>(in, out, n, tmp, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  dfree(tmp);
  if (e != hipSuccess) return fail(ctx, STB_E_DEVICE, "scan failed: %s", hipGetErrorString(e));
  return STB_OK;
}

static stb_status device_exclusive_scan(stb_ctx* ctx, const int64_t* in, int64_t* out, int64_t n) {
  return stb_exclusive_scan(ctx, in, out, n, ctx->stream);
}

// Apex boxes of evaluation points (enqueued on ctx's stream).
void stb_point_boxes(stb_ctx* ctx, int64_t np, const double* d_pts, ApexBox* d_box) {
  if (np > 0)
    hipLaunchKernelGGL(k_point_boxes, dim3((unsigned)((np + 255) / 256)), dim3(256), 0, ctx->stream, np,
                       d_pts, d_box);
}

// Exclusive prefix of the candidate counts of these rows (count pass only),
// copied to the host.
stb_status stb_cull_rowptr(stb_ctx* ctx, int64_t nrows, const ApexBox* d_rows, const stb_mesh* m,
                           int64_t* rowptr_host) {
  rowptr_host[0] = 0;
  if (nrows <= 0) return STB_OK;
  int64_t *d_cnt = nullptr, *d_scan = nullptr;
  HIPCHK(ctx, dalloc(&d_cnt, (size_t)nrows));
  if (dalloc(&d_scan, (size_t)nrows + 1) != hipSuccess) {
    dfree(d_cnt);
    return fail(ctx, STB_E_NO_MEMORY, "cull counts");
  }
  hipLaunchKernelGGL(k_cull_count, dim3((unsigned)((nrows + kCullRows - 1) / kCullRows)), dim3(kCullThreads), 0,
                     ctx->stream, nrows,
                     d_rows, m->nt, m->d_trial, d_cnt);
  hipError_t e = hipGetLastError();
  stb_status s = e == hipSuccess ? device_exclusive_scan(ctx, d_cnt, d_scan, nrows)
                                 : fail(ctx, STB_E_DEVICE, "cull count: %s", hipGetErrorString(e));
  if (s == STB_OK &&
      hipMemcpy(rowptr_host, d_scan, sizeof(int64_t) * (nrows + 1), hipMemcpyDeviceToHost) != hipSuccess)
    s = fail(ctx, STB_E_DEVICE, "cull count copy");
  dfree(d_cnt);
  dfree(d_scan);
  return s;
}

// Number of candidates the cull would produce for these rows.
stb_status stb_cull_count(stb_ctx* ctx, int64_t nrows, const ApexBox* d_rows, const stb_mesh* m,
                          int64_t* nnz) {
  std::vector<int64_t> rp((size_t)std::max<int64_t>(nrows, 0) + 1);
  stb_status s = stb_cull_rowptr(ctx, nrows, d_rows, m, rp.data());
  *nnz = rp.back();
  return s;
}

// Cull rows (apex boxes) against all trial panels into CSR candidates, with
// the row of every candidate alongside.
stb_status stb_cull(stb_ctx* ctx, int64_t nrows, const ApexBox* d_rows, const stb_mesh* m,
                       int64_t** d_rowptr, int32_t** d_cols, int32_t** d_rowof, int64_t* nnz, bool lend) {
  int64_t* d_cnt = nullptr;
  HIPCHK(ctx, dalloc(&d_cnt, (size_t)nrows));
  HIPCHK(ctx, dalloc(d_rowptr, (size_t)nrows + 1));
  if (nrows > 0) {
    hipLaunchKernelGGL(k_cull_count, dim3((unsigned)((nrows + kCullRows - 1) / kCullRows)), dim3(kCullThreads),
                       0, ctx->stream,
                       nrows, d_rows, m->nt, m->d_trial, d_cnt);
    HIPCHK(ctx, hipGetLastError());
  }
  stb_status s = device_exclusive_scan(ctx, d_cnt, *d_rowptr, nrows);
  dfree(d_cnt);
  if (s) return s;
  HIPCHK(ctx, hipMemcpy(nnz, *d_rowptr + nrows, sizeof(int64_t), hipMemcpyDeviceToHost));
  HIPCHK(ctx, lend ? kalloc(ctx, d_cols, (size_t)*nnz) : dalloc(d_cols, (size_t)*nnz));
  HIPCHK(ctx, lend ? kalloc(ctx, d_rowof, (size_t)*nnz) : dalloc(d_rowof, (size_t)*nnz));
  if (nrows > 0) {
    hipLaunchKernelGGL(k_cull_fill, dim3((unsigned)((nrows + kCullRows - 1) / kCullRows)), dim3(kCullThreads),
                       0, ctx->stream,
                       nrows, d_rows, m->nt, m->d_trial, *d_rowptr, *d_cols, *d_rowof);
    HIPCHK(ctx, hipGetLastError());
  }
  return STB_OK;
}

stb_status stb_cull_points(stb_ctx* ctx, stb_mesh* m, const stb_quad_params& p, int64_t np,
                           const double* d_pts, int64_t** d_rowptr, int32_t** d_cols, int32_t** d_rowof,
                           int64_t* nnz) {
  if (p.lit_search == STB_LIT_TREE)
    return stb_tree_cull(ctx, m, p.n_min, np, d_pts, d_rowptr, d_cols, d_rowof, nnz, nullptr);
  ApexBox* d_box = nullptr;
  if (dalloc(&d_box, (size_t)std::max<int64_t>(np, 1)) != hipSuccess)
    return fail(ctx, STB_E_NO_MEMORY, "point boxes");
  stb_point_boxes(ctx, np, d_pts, d_box);
  stb_status s = stb_cull(ctx, np, d_box, m, d_rowptr, d_cols, d_rowof, nnz);
  HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
  dfree(d_box);
  ctx->lit_search[0] = 0;
  ctx->lit_search[1] = np * m->nt;   // every panel examined for every point
  ctx->lit_search[2] = s == STB_OK ? *nnz : 0;
  return s;
}

stb_status stb_keep_causal(stb_ctx* ctx, stb_mat* M, const uint8_t* d_flag, hipStream_t st) {
  const int64_t n = M->n;
  int64_t *cnt = nullptr, *rp = nullptr;
  int32_t* cols = nullptr;
  double* vals = nullptr;
  auto cleanup = [&]() { dfree(cnt); dfree(rp); dfree(cols); dfree(vals); };
  if (dalloc(&cnt, (size_t)std::max<int64_t>(n, 1)) != hipSuccess || dalloc(&rp, (size_t)n + 1) != hipSuccess) {
    cleanup();
    return fail(ctx, STB_E_NO_MEMORY, "causal store: row counts");
  }
  const unsigned g = (unsigned)((n * 64 + 255) / 256);
  if (n > 0) hipLaunchKernelGGL(k_keep_count, dim3(g), dim3(256), 0, st, n, M->d_rowptr, d_flag, cnt);
  HIPCHK(ctx, hipGetLastError());
  stb_status s = stb_exclusive_scan(ctx, cnt, rp, n, st);
  if (s) { cleanup(); return s; }
  int64_t nk = 0;
  hipError_t e = hipMemcpy(&nk, rp + n, sizeof(int64_t), hipMemcpyDeviceToHost);
  if (e != hipSuccess) { cleanup(); return fail(ctx, STB_E_DEVICE, "causal store: %s", hipGetErrorString(e)); }
  if (dalloc(&cols, (size_t)nk) != hipSuccess || dalloc(&vals, (size_t)nk) != hipSuccess) {
    cleanup();
    return fail(ctx, STB_E_NO_MEMORY, "causal store of %lld entries", (long long)nk);
  }
  if (n > 0)
    hipLaunchKernelGGL(k_keep_fill, dim3(g), dim3(256), 0, st, n, M->d_rowptr, M->d_cols, M->d_vals, d_flag,
                       rp, cols, vals);
  e = hipGetLastError();
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  if (e != hipSuccess) { cleanup(); return fail(ctx, STB_E_DEVICE, "causal store: %s", hipGetErrorString(e)); }
  dfree(cnt);
  dfree(M->d_rowptr);
  ctx_keep(ctx, M->d_cols);
  ctx_keep(ctx, M->d_vals);
  dfree(M->d_vals32);
  M->d_vals32 = nullptr;
  stb_free_blocked(M);
  M->d_rowptr = rp;
  M->d_cols = cols;
  M->d_vals = vals;
  M->nnz = nk;
  M->host_valid = false;
  return STB_OK;
}

// Host copy of a matrix store (for stb_mat_get / stb_mat_to_dense).
static stb_status mirror_host(stb_mat* M) {
  if (M->host_valid) return STB_OK;
  stb_ctx* ctx = M->ctx;
  HIPCHK(ctx, hipSetDevice(ctx->device));
  M->h_rowptr.resize((size_t)M->n + 1);
  M->h_cols.resize((size_t)M->nnz);
  M->h_vals.resize((size_t)M->nnz);
  HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
  HIPCHK(ctx, hipMemcpy(M->h_rowptr.data(), M->d_rowptr, 8 * (M->n + 1), hipMemcpyDeviceToHost));
  if (M->nnz) {
    HIPCHK(ctx, hipMemcpy(M->h_cols.data(), M->d_cols, 4 * M->nnz, hipMemcpyDeviceToHost));
    HIPCHK(ctx, hipMemcpy(M->h_vals.data(), M->d_vals, 8 * M->nnz, hipMemcpyDeviceToHost));
  }
  M->host_valid = true;
  return STB_OK;
}

// ---------------------------------------------------------------- C ABI
hipError_t ctx_alloc(stb_ctx* ctx, void** p, size_t bytes) {
  *p = nullptr;
  size_t best = (size_t)-1;
  int bi = -1;
  for (size_t k = 0; k < ctx->kept.size(); ++k) {
    const size_t n = ctx->kept[k].second;
    if (n >= bytes && n / 2 <= bytes && n < best) {
      best = n;
      bi = (int)k;
    }
  }
  if (bi >= 0) {
    ctx->lent.push_back(ctx->kept[(size_t)bi]);
    ctx->kept_bytes -= ctx->kept[(size_t)bi].second;
    ctx->kept.erase(ctx->kept.begin() + bi);
    *p = ctx->lent.back().first;
    return hipSuccess;
  }
  hipError_t e = hipMalloc(p, bytes);
  if (e == hipErrorOutOfMemory && !ctx->kept.empty()) {
    (void)hipGetLastError();
    for (auto& b : ctx->kept) (void)hipFree(b.first);
    ctx->kept.clear();
    ctx->kept_bytes = 0;
    e = hipMalloc(p, bytes);
  }
  if (e != hipSuccess) {
    *p = nullptr;
    return e;
  }
  ctx->lent.push_back({*p, bytes});
  return hipSuccess;
}

void ctx_keep(stb_ctx* ctx, void* p) {
  if (!p) return;
  for (size_t k = 0; k < ctx->lent.size(); ++k)
    if (ctx->lent[k].first == p) {
      const size_t n = ctx->lent[k].second;
      if (ctx->kept_bytes + n <= kKeptMaxBytes) {
        ctx->kept.push_back(ctx->lent[k]);
        ctx->kept_bytes += n;
      } else {
        (void)hipFree(p);
      }
      ctx->lent.erase(ctx->lent.begin() + (long)k);
      return;
    }
  (void)hipFree(p);   // not lent by ctx_alloc
}

void ctx_drop_kept(stb_ctx* ctx) {
  for (auto& b : ctx->kept) (void)hipFree(b.first);
  for (auto& b : ctx->lent) (void)hipFree(b.first);
  ctx->kept.clear();
  ctx->lent.clear();
  ctx->kept_bytes = 0;
}

extern "C" {

stb_quad_params stb_default_params(void) {
  stb_quad_params p;
  p.m_q = 3;
  p.n_g = 16;
  p.eta_far = 0.5;
  p.prec = STB_FP64;
  p.lit_search = STB_LIT_FLAT;
  p.n_min = 64;
  return p;
}

const char* stb_status_str(stb_status s) {
  switch (s) {
    case STB_OK: return "ok";
    case STB_E_INVALID_ARG: return "invalid argument";
    case STB_E_INVALID_MESH: return "invalid mesh";
    case STB_E_NO_MEMORY: return "out of memory";
    case STB_E_DEVICE: return "device error";
    case STB_E_NOT_FOUND: return "not found";
    case STB_E_BUSY: return "busy";
    case STB_E_INTERNAL: return "internal error";
  }
  return "unknown status";
}

const char* stb_last_error(const stb_ctx* ctx) {
  if (ctx) return ctx->err.c_str();
  std::lock_guard<std::mutex> g(g_err_mu);
  return g_err.c_str();
}

stb_status stb_ctx_create(int32_t device, stb_ctx** out) {
  if (!out) return fail(nullptr, STB_E_INVALID_ARG, "out is NULL");
  *out = nullptr;
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || ndev == 0)
    return fail(nullptr, STB_E_DEVICE, "no HIP device available");
  if (device < 0 || device >= ndev)
    return fail(nullptr, STB_E_INVALID_ARG, "device %d out of range [0,%d)", device, ndev);
  if (hipSetDevice(device) != hipSuccess) return fail(nullptr, STB_E_DEVICE, "hipSetDevice failed");
  stb_ctx* c = new stb_ctx();
  c->device = device;
  if (hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking) != hipSuccess) {
    delete c;
    return fail(nullptr, STB_E_DEVICE, "hipStreamCreate failed");
  }
  for (auto& e : c->ev)
    if (hipEventCreate(&e) != hipSuccess) {
      delete c;
      return fail(nullptr, STB_E_DEVICE, "hipEventCreate failed");
    }
  // this device's address of the allocation-free product's scratch array
  if (stb_noalloc_setup(c) != STB_OK) {
    std::string m = c->err;
    stb_ctx_destroy(c);
    return fail(nullptr, STB_E_DEVICE, "%s", m.c_str());
  }
  *out = c;
  return STB_OK;
}

void stb_ctx_destroy(stb_ctx* ctx) {
  if (!ctx) return;
  (void)hipSetDevice(ctx->device);
  (void)hipStreamSynchronize(ctx->stream);
  dfree(ctx->d_gl);
  stb_free_workspace(ctx);
  ctx_drop_kept(ctx);
  for (auto& e : ctx->ev) if (e) (void)hipEventDestroy(e);
  for (auto& e : ctx->kev) if (e) (void)hipEventDestroy(e);
  if (ctx->stream) (void)hipStreamDestroy(ctx->stream);
  delete ctx;
}

static stb_status mesh_create_impl(stb_ctx* ctx, int64_t nv, const double* vtx, int64_t nt,
                                   const int32_t* tet, bool dev, hipStream_t ust, stb_mesh** out) {
  if (!ctx || !out) return fail(ctx, STB_E_INVALID_ARG, "NULL argument");
  *out = nullptr;
  if (nv <= 0 || nt <= 0 || !vtx || !tet)
    return fail(ctx, STB_E_INVALID_ARG, "empty mesh or NULL arrays (nv=%lld nt=%lld)",
                (long long)nv, (long long)nt);
  if (nt > (int64_t)INT32_MAX || nv > (int64_t)INT32_MAX)
    return fail(ctx, STB_E_INVALID_ARG, "too many panels or vertices");
  if (!dev)
    for (int64_t i = 0; i < 4 * nt; ++i)
      if (tet[i] < 0 || tet[i] >= nv)
        return fail(ctx, STB_E_INVALID_MESH, "panel %lld: vertex index %d out of range",
                    (long long)(i / 4), tet[i]);
  HIPCHK(ctx, hipSetDevice(ctx->device));
  if (dev && ust) HIPCHK(ctx, hipStreamSynchronize(ust));
  stb_mesh* m = new stb_mesh();
  m->ctx = ctx;
  m->nv = nv;
  m->nt = nt;
  int32_t* d_status = nullptr;
  auto cleanup = [&]() {
    dfree(d_status);
    stb_mesh_destroy(m);
  };
  if (dalloc(&m->d_vtx, (size_t)nv * 4) != hipSuccess || dalloc(&m->d_tet, (size_t)nt * 4) != hipSuccess ||
      dalloc(&m->d_trial, (size_t)nt) != hipSuccess || dalloc(&m->d_fang, (size_t)nt) != hipSuccess ||
      dalloc(&d_status, (size_t)nt) != hipSuccess) {
    cleanup();
    return fail(ctx, STB_E_NO_MEMORY, "device allocation for %lld panels failed", (long long)nt);
  }
  hipMemcpyKind kind = dev ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice;
  hipError_t e = hipMemcpyAsync(m->d_vtx, vtx, sizeof(double) * 4 * nv, kind, ctx->stream);
  if (e == hipSuccess) e = hipMemcpyAsync(m->d_tet, tet, sizeof(int32_t) * 4 * nt, kind, ctx->stream);
  std::vector<int32_t> status((size_t)nt);
  if (dev && e == hipSuccess) {
    // indices first, on the device: the geometry kernel gathers through them
    hipLaunchKernelGGL(k_check_index, dim3((unsigned)((nt + 255) / 256)), dim3(256), 0, ctx->stream, nt, nv,
                       m->d_tet, d_status);
    e = hipGetLastError();
    if (e == hipSuccess)
      e = hipMemcpyAsync(status.data(), d_status, sizeof(int32_t) * nt, hipMemcpyDeviceToHost, ctx->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
    if (e == hipSuccess)
      for (int64_t j = 0; j < nt; ++j)
        if (status[j] != 0) {
          cleanup();
          return fail(ctx, STB_E_INVALID_MESH, "panel %lld: vertex index out of range", (long long)j);
        }
  }
  if (e == hipSuccess) {
    hipLaunchKernelGGL(k_geometry, dim3((unsigned)((nt + 127) / 128)), dim3(128), 0, ctx->stream, nt,
                       m->d_vtx, m->d_tet, m->d_trial, m->d_fang, d_status);
    e = hipGetLastError();
  }
  if (e == hipSuccess)
    e = hipMemcpyAsync(status.data(), d_status, sizeof(int32_t) * nt, hipMemcpyDeviceToHost, ctx->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
  if (e != hipSuccess) {
    cleanup();
    return fail(ctx, STB_E_DEVICE, "mesh upload failed: %s", hipGetErrorString(e));
  }
  static const char* why[] = {"ok", "non-finite coordinate", "degenerate spatial projection",
                              "not vertical (spatial projection not planar)", "zero 3-volume"};
  for (int64_t j = 0; j < nt; ++j)
    if (status[j] != 0) {
      int s = status[j];
      cleanup();
      return fail(ctx, STB_E_INVALID_MESH, "panel %lld: %s", (long long)j, why[s >= 0 && s <= 4 ? s : 0]);
    }
  dfree(d_status);
  *out = m;
  return STB_OK;
}

stb_status stb_mesh_create(stb_ctx* ctx, int64_t nv, const double* vtx, int64_t nt,
                           const int32_t* tet, stb_mesh** out) {
  return mesh_create_impl(ctx, nv, vtx, nt, tet, false, nullptr, out);
}

stb_status stb_mesh_create_dev(stb_ctx* ctx, int64_t nv, const double* vtx_dev, int64_t nt,
                               const int32_t* tet_dev, void* stream, stb_mesh** out) {
  return mesh_create_impl(ctx, nv, vtx_dev, nt, tet_dev, true, (hipStream_t)stream, out);
}

void stb_mesh_destroy(stb_mesh* m) {
  if (!m) return;
  dfree(m->d_vtx); dfree(m->d_tet); dfree(m->d_trial); dfree(m->d_fang);
  dfree(m->d_nsign);
  stb_free_projection(m);
  dfree(m->d_opts); dfree(m->d_ow); dfree(m->d_onq); dfree(m->d_box);
  stb_free_faces(m);
  stb_free_tree(m);
  delete m;
}

int64_t stb_mesh_size(const stb_mesh* m) { return m ? m->nt : 0; }

stb_status stb_assemble_V(stb_ctx* ctx, const stb_mesh* mesh_c, const stb_quad_params* params,
                          stb_mat** out) {
  if (!ctx || !mesh_c || !out) return fail(ctx, STB_E_INVALID_ARG, "NULL argument");
  *out = nullptr;
  stb_mesh* mesh = const_cast<stb_mesh*>(mesh_c);
  if (mesh->ctx != ctx) return fail(ctx, STB_E_INVALID_ARG, "mesh belongs to another context");
  stb_quad_params p = params ? *params : stb_default_params();
  stb_status s = stb_check_params(ctx, &p);
  if (s) return s;
  HIPCHK(ctx, hipSetDevice(ctx->device));
  if ((s = stb_ensure_gl(ctx, p.n_g))) return s;
  HIPCHK(ctx, hipEventRecord(ctx->ev[0], ctx->stream));
  if ((s = stb_ensure_outer(ctx, mesh, p.m_q))) return s;
  HIPCHK(ctx, hipEventRecord(ctx->ev[1], ctx->stream));
  stb_mat* M = new stb_mat();
  M->ctx = ctx;
  M->n = mesh->nt;
  // the candidate store (columns, values), the candidates' rows and their
  // causal flags are blocks lent by the context until the causal-only
  // store replaces them
  int32_t* d_rowof = nullptr;
  auto drop = [&]() {
    ctx_keep(ctx, d_rowof);
    d_rowof = nullptr;
    ctx_keep(ctx, M->d_cols);
    M->d_cols = nullptr;
    ctx_keep(ctx, M->d_vals);
    M->d_vals = nullptr;
  };
  s = stb_cull(ctx, mesh->nt, mesh->d_box, mesh, &M->d_rowptr, &M->d_cols, &d_rowof, &M->nnz, true);
  if (s) { drop(); stb_mat_destroy(M); return s; }
  HIPCHK(ctx, hipEventRecord(ctx->ev[2], ctx->stream));
  uint8_t* d_keep = nullptr;
  if (kalloc(ctx, &M->d_vals, (size_t)M->nnz) != hipSuccess || kalloc(ctx, &d_keep, (size_t)M->nnz) != hipSuccess) {
    drop(); ctx_keep(ctx, d_keep); stb_mat_destroy(M);
    return fail(ctx, STB_E_NO_MEMORY, "store of %lld entries does not fit", (long long)M->nnz);
  }
  unsigned long long causal = 0, work[4];
  if (p.prec == STB_FP64) {
    // through the shared faces' outer points
    FaceUnit U;
    U.mesh = mesh;
    U.r0 = 0;
    U.r1 = mesh->nt;
    U.rowptr = M->d_rowptr;
    U.rowof = d_rowof;
    U.cols = M->d_cols;
    U.nnz = M->nnz;
    U.vals = M->d_vals;
    U.keep = d_keep;
    s = stb_face_assemble(ctx, p, &U, 1, work);
    causal = (unsigned long long)U.n_causal;
  } else {
    PairJob J;
    J.nnz = M->nnz;
    J.rows = d_rowof;
    J.cols = M->d_cols;
    J.trial = mesh->d_trial;
    J.fang = mesh->d_fang;
    J.apex = mesh->d_opts;
    J.apex_w = mesh->d_ow;
    J.apex_n = mesh->d_onq;
    J.maxq = mesh->maxq;
    J.gl = ctx->d_gl;
    J.ng = p.n_g;
    J.mixed = true;
    J.eta_far = p.eta_far;
    J.out = M->d_vals;
    J.lit_out = d_keep;
    J.n_causal = &causal;
    s = stb_run_pairs(ctx, J, work);
  }
  ctx_keep(ctx, d_rowof);
  d_rowof = nullptr;
  // the resident store keeps the causal entries only (and hands the
  // candidate store back to the context)
  if (s == STB_OK) s = stb_keep_causal(ctx, M, d_keep, ctx->stream);
  ctx_keep(ctx, d_keep);
  if (s) { drop(); stb_mat_destroy(M); return s; }
  HIPCHK(ctx, hipEventRecord(ctx->ev[3], ctx->stream));
  HIPCHK(ctx, hipEventSynchronize(ctx->ev[3]));
  M->n_causal = (int64_t)causal;
  for (int k = 0; k < 4; ++k) ctx->work[k] = (int64_t)work[k];
  float t01 = 0, t12 = 0, t23 = 0, t03 = 0;
  (void)hipEventElapsedTime(&t01, ctx->ev[0], ctx->ev[1]);
  (void)hipEventElapsedTime(&t12, ctx->ev[1], ctx->ev[2]);
  (void)hipEventElapsedTime(&t23, ctx->ev[2], ctx->ev[3]);
  (void)hipEventElapsedTime(&t03, ctx->ev[0], ctx->ev[3]);
  ctx->timings[0] = t01; ctx->timings[1] = t12; ctx->timings[2] = t23; ctx->timings[3] = t03;
  *out = M;
  return STB_OK;
}

void stb_mat_destroy(stb_mat* M) {
  if (!M) return;
  dfree(M->d_rowptr); dfree(M->d_cols); dfree(M->d_vals); dfree(M->d_vals32);
  stb_free_blocked(M);
  delete M;
}

stb_status stb_mat_info(const stb_mat* M, int64_t* n, int64_t* nc, int64_t* nstored, int64_t* bytes) {
  if (!M) return fail(nullptr, STB_E_INVALID_ARG, "NULL matrix");
  if (n) *n = M->n;
  if (nc) *nc = M->n_causal;
  if (nstored) *nstored = M->nnz;
  if (bytes)
    *bytes = (M->n + 1) * 8 + M->nnz * (4 + 8) + (M->d_vals32 ? M->nnz * 4 : 0);
  return STB_OK;
}

stb_status stb_mat_to_dense(const stb_mat* Mc, double* out) {
  if (!Mc || !out) return fail(Mc ? Mc->ctx : nullptr, STB_E_INVALID_ARG, "NULL argument");
  stb_mat* M = const_cast<stb_mat*>(Mc);
  stb_status s = mirror_host(M);
  if (s) return s;
  std::memset(out, 0, sizeof(double) * (size_t)M->n * (size_t)M->n);
  for (int64_t i = 0; i < M->n; ++i)
    for (int64_t k = M->h_rowptr[i]; k < M->h_rowptr[i + 1]; ++k) out[i * M->n + M->h_cols[k]] = M->h_vals[k];
  return STB_OK;
}

stb_status stb_mat_get(const stb_mat* Mc, int64_t k, const int32_t* row, const int32_t* col, double* out) {
  if (!Mc || (k > 0 && (!row || !col || !out)) || k < 0)
    return fail(Mc ? Mc->ctx : nullptr, STB_E_INVALID_ARG, "bad arguments");
  stb_mat* M = const_cast<stb_mat*>(Mc);
  const int64_t ncols = mat_ncols(M);
  for (int64_t m = 0; m < k; ++m)
    if (row[m] < 0 || row[m] >= M->n || col[m] < 0 || col[m] >= ncols)
      return fail(M->ctx, STB_E_INVALID_ARG, "entry %lld out of range", (long long)m);
  if (k == 0) return STB_OK;
  if (M->host_valid) {
    for (int64_t m = 0; m < k; ++m) {
      const int32_t* b = M->h_cols.data() + M->h_rowptr[row[m]];
      const int32_t* e = M->h_cols.data() + M->h_rowptr[row[m] + 1];
      const int32_t* it = std::lower_bound(b, e, col[m]);
      out[m] = (it != e && *it == col[m]) ? M->h_vals[it - M->h_cols.data()] : 0.0;
    }
    return STB_OK;
  }
  // on the device: no host copy of a store that may hold billions of entries
  stb_ctx* ctx = M->ctx;
  HIPCHK(ctx, hipSetDevice(ctx->device));
  int32_t *d_rc = nullptr;
  double* d_out = nullptr;
  if (dalloc(&d_rc, (size_t)(2 * k)) != hipSuccess || dalloc(&d_out, (size_t)k) != hipSuccess) {
    dfree(d_rc); dfree(d_out);
    return fail(ctx, STB_E_NO_MEMORY, "entry lookup buffers");
  }
  hipError_t e = hipMemcpyAsync(d_rc, row, 4 * k, hipMemcpyHostToDevice, ctx->stream);
  if (e == hipSuccess) e = hipMemcpyAsync(d_rc + k, col, 4 * k, hipMemcpyHostToDevice, ctx->stream);
  if (e == hipSuccess) {
    hipLaunchKernelGGL(k_mat_get, dim3((unsigned)((k + 255) / 256)), dim3(256), 0, ctx->stream, k,
                       M->d_rowptr, M->d_cols, M->d_vals, d_rc, d_rc + k, d_out);
    e = hipGetLastError();
  }
  if (e == hipSuccess) e = hipMemcpyAsync(out, d_out, 8 * k, hipMemcpyDeviceToHost, ctx->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
  dfree(d_rc);
  dfree(d_out);
  if (e != hipSuccess) return fail(ctx, STB_E_DEVICE, "entry lookup: %s", hipGetErrorString(e));
  return STB_OK;
}

stb_status stb_mat_export(const stb_mat* M, int64_t* rowptr, int32_t* cols, double* vals) {
  if (!M) return fail(nullptr, STB_E_INVALID_ARG, "NULL matrix");
  stb_ctx* ctx = M->ctx;
  HIPCHK(ctx, hipSetDevice(ctx->device));
  HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
  if (rowptr) HIPCHK(ctx, hipMemcpy(rowptr, M->d_rowptr, 8 * (M->n + 1), hipMemcpyDeviceToHost));
  if (cols && M->nnz) HIPCHK(ctx, hipMemcpy(cols, M->d_cols, 4 * M->nnz, hipMemcpyDeviceToHost));
  if (vals && M->nnz) HIPCHK(ctx, hipMemcpy(vals, M->d_vals, 8 * M->nnz, hipMemcpyDeviceToHost));
  return STB_OK;
}

stb_status stb_apply_dev(stb_ctx* ctx, const stb_mat* M, int32_t nrhs, const double* w, double* y,
                         void* stream) {
  if (!ctx || !M || !w || !y || nrhs < 1) return fail(ctx, STB_E_INVALID_ARG, "bad arguments");
  hipStream_t st = stream ? (hipStream_t)stream : ctx->stream;
  HIPCHK(ctx, hipSetDevice(ctx->device));
  if (nrhs == 16) return stb_apply16_dev(ctx, const_cast<stb_mat*>(M), w, y, st);
  int64_t threads = M->n * 64;
  for (int c = 0; c < nrhs; ++c) {
    if (M->n > 0) {
      hipLaunchKernelGGL(k_spmv, dim3((unsigned)std::min<int64_t>((threads + 255) / 256, 1 << 20)), dim3(256), 0, st, M->n,
                         M->d_rowptr, M->d_cols, M->d_vals, w, nrhs, c, y);
      HIPCHK(ctx, hipGetLastError());
    }
  }
  return STB_OK;
}

stb_status stb_apply(stb_ctx* ctx, const stb_mat* M, int32_t nrhs, const double* w, double* y) {
  if (!ctx || !M || !w || !y || nrhs < 1) return fail(ctx, STB_E_INVALID_ARG, "bad arguments");
  HIPCHK(ctx, hipSetDevice(ctx->device));
  double *dw = nullptr, *dy = nullptr;
  size_t bytes = sizeof(double) * (size_t)M->n * nrhs;
  if (dalloc(&dw, (size_t)M->n * nrhs) != hipSuccess || dalloc(&dy, (size_t)M->n * nrhs) != hipSuccess) {
    dfree(dw); dfree(dy);
    return fail(ctx, STB_E_NO_MEMORY, "apply buffers");
  }
  hipError_t e = hipMemcpyAsync(dw, w, bytes, hipMemcpyHostToDevice, ctx->stream);
  stb_status s = e == hipSuccess ? stb_apply_dev(ctx, M, nrhs, dw, dy, nullptr)
                                 : fail(ctx, STB_E_DEVICE, "copy failed");
  if (s == STB_OK) {
    e = hipMemcpyAsync(y, dy, bytes, hipMemcpyDeviceToHost, ctx->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
    if (e != hipSuccess) s = fail(ctx, STB_E_DEVICE, "apply failed: %s", hipGetErrorString(e));
  }
  dfree(dw);
  dfree(dy);
  return s;
}

}  // extern "C"

// Potential with device inputs and output, on the context stream.
stb_status stb_potential_core(stb_ctx* ctx, stb_mesh* mesh, const stb_quad_params& p,
                              const double* d_w, int64_t np, const double* d_pts, double* d_out) {
  stb_status s;
  if ((s = stb_ensure_gl(ctx, p.n_g))) return s;
  double* d_I = nullptr;
  int64_t* d_rowptr = nullptr;
  int32_t *d_cols = nullptr, *d_rowof = nullptr;
  auto cleanup = [&]() {
    dfree(d_I); dfree(d_rowptr); dfree(d_cols); dfree(d_rowof);
  };
  HIPCHK(ctx, hipEventRecord(ctx->ev[0], ctx->stream));
  HIPCHK(ctx, hipEventRecord(ctx->ev[1], ctx->stream));
  int64_t nnz = 0;
  s = stb_cull_points(ctx, mesh, p, np, d_pts, &d_rowptr, &d_cols, &d_rowof, &nnz);
  if (s) { cleanup(); return s; }
  HIPCHK(ctx, hipEventRecord(ctx->ev[2], ctx->stream));
  if (dalloc(&d_I, (size_t)nnz) != hipSuccess) { cleanup(); return fail(ctx, STB_E_NO_MEMORY, "candidates"); }
  PairJob J;
  J.nnz = nnz;
  J.rows = d_rowof;
  J.cols = d_cols;
  J.trial = mesh->d_trial;
  J.fang = mesh->d_fang;
  J.apex = d_pts;
  J.apex_w = nullptr;
  J.apex_n = nullptr;
  J.maxq = 1;
  J.gl = ctx->d_gl;
  J.ng = p.n_g;
  J.mixed = false;   // the potential is a plain sum over panels: always FP64
  J.out = d_I;
  unsigned long long work[4];
  s = stb_run_pairs(ctx, J, work);
  if (s) { cleanup(); return s; }
  for (int k = 0; k < 4; ++k) ctx->work[k] = (int64_t)work[k];
  hipLaunchKernelGGL(k_point_sum, dim3((unsigned)std::min<int64_t>((np * 64 + 255) / 256, 1 << 20)), dim3(256), 0,
                     ctx->stream, np, d_rowptr, d_cols, d_I, d_w, d_out);
  hipError_t e = hipGetLastError();
  if (e == hipSuccess) e = hipEventRecord(ctx->ev[3], ctx->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
  cleanup();
  if (e != hipSuccess) return fail(ctx, STB_E_DEVICE, "potential failed: %s", hipGetErrorString(e));
  float t01 = 0, t12 = 0, t23 = 0, t03 = 0;
  (void)hipEventElapsedTime(&t01, ctx->ev[0], ctx->ev[1]);
  (void)hipEventElapsedTime(&t12, ctx->ev[1], ctx->ev[2]);
  (void)hipEventElapsedTime(&t23, ctx->ev[2], ctx->ev[3]);
  (void)hipEventElapsedTime(&t03, ctx->ev[0], ctx->ev[3]);
  ctx->timings[0] = t01; ctx->timings[1] = t12; ctx->timings[2] = t23; ctx->timings[3] = t03;
  return STB_OK;
}

extern "C" {

stb_status stb_potential_S(stb_ctx* ctx, const stb_mesh* mesh_c, const stb_quad_params* params,
                           const double* w, int64_t np, const double* pts, double* out) {
  if (!ctx || !mesh_c || !w || (np > 0 && (!pts || !out)) || np < 0)
    return fail(ctx, STB_E_INVALID_ARG, "bad arguments");
  stb_mesh* mesh = const_cast<stb_mesh*>(mesh_c);
  if (mesh->ctx != ctx) return fail(ctx, STB_E_INVALID_ARG, "mesh belongs to another context");
  stb_quad_params p = params ? *params : stb_default_params();
  stb_status s = stb_check_params(ctx, &p);
  if (s) return s;
  if (np == 0) return STB_OK;
  for (int64_t i = 0; i < 4 * np; ++i)
    if (!std::isfinite(pts[i])) return fail(ctx, STB_E_INVALID_ARG, "non-finite point %lld", (long long)(i / 4));
  HIPCHK(ctx, hipSetDevice(ctx->device));
  double *d_pts = nullptr, *d_w = nullptr, *d_out = nullptr;
  if (dalloc(&d_pts, (size_t)np * 4) != hipSuccess || dalloc(&d_w, (size_t)mesh->nt) != hipSuccess ||
      dalloc(&d_out, (size_t)np) != hipSuccess) {
    dfree(d_pts); dfree(d_w); dfree(d_out);
    return fail(ctx, STB_E_NO_MEMORY, "potential buffers");
  }
  hipError_t e = hipMemcpyAsync(d_pts, pts, sizeof(double) * 4 * np, hipMemcpyHostToDevice, ctx->stream);
  if (e == hipSuccess) e = hipMemcpyAsync(d_w, w, sizeof(double) * mesh->nt, hipMemcpyHostToDevice, ctx->stream);
  s = e == hipSuccess ? stb_potential_core(ctx, mesh, p, d_w, np, d_pts, d_out)
                      : fail(ctx, STB_E_DEVICE, "copy failed");
  if (s == STB_OK) {
    e = hipMemcpy(out, d_out, sizeof(double) * np, hipMemcpyDeviceToHost);
    if (e != hipSuccess) s = fail(ctx, STB_E_DEVICE, "copy back failed: %s", hipGetErrorString(e));
  }
  dfree(d_pts); dfree(d_w); dfree(d_out);
  return s;
}

stb_status stb_potential_S_dev(stb_ctx* ctx, const stb_mesh* mesh_c, const stb_quad_params* params,
                               const double* w_dev, int64_t np, const double* pts_dev, double* out_dev,
                               void* stream) {
  if (!ctx || !mesh_c || !w_dev || (np > 0 && (!pts_dev || !out_dev)) || np < 0)
    return fail(ctx, STB_E_INVALID_ARG, "bad arguments");
  stb_mesh* mesh = const_cast<stb_mesh*>(mesh_c);
  if (mesh->ctx != ctx) return fail(ctx, STB_E_INVALID_ARG, "mesh belongs to another context");
  stb_quad_params p = params ? *params : stb_default_params();
  stb_status s = stb_check_params(ctx, &p);
  if (s) return s;
  if (np == 0) return STB_OK;
  HIPCHK(ctx, hipSetDevice(ctx->device));
  if (stream) HIPCHK(ctx, hipStreamSynchronize((hipStream_t)stream));
  return stb_potential_core(ctx, mesh, p, w_dev, np, pts_dev, out_dev);
}

stb_status stb_inner_values(stb_ctx* ctx, const stb_mesh* mesh, const stb_quad_params* params,
                            int64_t k, const double* pts, const int32_t* panel, double* out) {
  if (!ctx || !mesh || k < 0 || (k > 0 && (!pts || !panel || !out)))
    return fail(ctx, STB_E_INVALID_ARG, "bad arguments");
  stb_quad_params p = params ? *params : stb_default_params();
  stb_status s = stb_check_params(ctx, &p);
  if (s) return s;
  for (int64_t m = 0; m < k; ++m)
    if (panel[m] < 0 || panel[m] >= mesh->nt)
      return fail(ctx, STB_E_INVALID_ARG, "panel index %d out of range", panel[m]);
  if (k == 0) return STB_OK;
  HIPCHK(ctx, hipSetDevice(ctx->device));
  if ((s = stb_ensure_gl(ctx, p.n_g))) return s;
  double *d_pts = nullptr, *d_out = nullptr;
  int32_t* d_pan = nullptr;
  if (dalloc(&d_pts, (size_t)k * 4) != hipSuccess || dalloc(&d_out, (size_t)k) != hipSuccess ||
      dalloc(&d_pan, (size_t)k) != hipSuccess) {
    dfree(d_pts); dfree(d_out); dfree(d_pan);
    return fail(ctx, STB_E_NO_MEMORY, "buffers");
  }
  hipError_t e = hipMemcpyAsync(d_pts, pts, 32 * k, hipMemcpyHostToDevice, ctx->stream);
  if (e == hipSuccess) e = hipMemcpyAsync(d_pan, panel, 4 * k, hipMemcpyHostToDevice, ctx->stream);
  if (e == hipSuccess) {
    hipLaunchKernelGGL(k_inner_values, dim3((unsigned)((k + 127) / 128)), dim3(128), 0, ctx->stream, k,
                       mesh->d_trial, d_pts, d_pan, ctx->d_gl, p.n_g, d_out);
    e = hipGetLastError();
  }
  if (e == hipSuccess) e = hipMemcpyAsync(out, d_out, 8 * k, hipMemcpyDeviceToHost, ctx->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
  dfree(d_pts); dfree(d_out); dfree(d_pan);
  if (e != hipSuccess) return fail(ctx, STB_E_DEVICE, "inner values failed: %s", hipGetErrorString(e));
  return STB_OK;
}

stb_status stb_last_timings(const stb_ctx* ctx, double* ms4) {
  if (!ctx || !ms4) return fail(nullptr, STB_E_INVALID_ARG, "NULL argument");
  for (int k = 0; k < 4; ++k) ms4[k] = ctx->timings[k];
  return STB_OK;
}

stb_status stb_last_kernel_times(const stb_ctx* ctx, double* ms8, int64_t* launches8,
                                 int64_t* units8) {
  if (!ctx || !ms8 || !launches8 || !units8) return fail(nullptr, STB_E_INVALID_ARG, "NULL argument");
  for (int k = 0; k < 8; ++k) {
    ms8[k] = ctx->kern_ms[k];
    launches8[k] = ctx->kern_n[k];
    units8[k] = ctx->kern_units[k];
  }
  return STB_OK;
}

stb_status stb_last_path_counts(const stb_ctx* ctx, int64_t* counts4) {
  if (!ctx || !counts4) return fail(nullptr, STB_E_INVALID_ARG, "NULL argument");
  for (int k = 0; k < 4; ++k) counts4[k] = ctx->path_counts[k];
  return STB_OK;
}

stb_status stb_last_lit_search(const stb_ctx* ctx, int64_t* counts3) {
  if (!ctx || !counts3) return fail(nullptr, STB_E_INVALID_ARG, "NULL argument");
  for (int k = 0; k < 3; ++k) counts3[k] = ctx->lit_search[k];
  return STB_OK;
}

stb_status stb_last_work(const stb_ctx* ctx, int64_t* counts4) {
  if (!ctx || !counts4) return fail(nullptr, STB_E_INVALID_ARG, "NULL argument");
  for (int k = 0; k < 4; ++k) counts4[k] = ctx->work[k];
  return STB_OK;
}

}  // extern "C"
