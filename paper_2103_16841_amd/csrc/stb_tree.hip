// stb_tree.hip -- lit-panel search for evaluation points by a cluster tree
// (Sec. 3.3: Def. bct, Theorem phi_xi_sphere, Alg. lit_leaves).
//
// The paper descends a binary cluster tree recursively per point on a CPU.
// Here the tree is a perfect binary tree over the panels sorted along a
// space-time Morton curve (leaves of at most n_min panels; a cluster is a
// contiguous range of that order, so its two sons split it in the middle:
// disjoint, non-empty where the range is, union the father), with one
// bounding 4-ball per cluster.  All points descend together, level by level:
// the frontier is a flat list of (point, cluster) pairs; every pair is tested
// with the theorem's exact extrema of phi_Xi over the ball, and the survivors'
// sons (or, on the last level, the surviving leaves) are laid out by a prefix
// sum of their counts, which keeps each point's entries in tree order.  The
// leaves that survive give the candidate panels X_N(x); the exact lit test of
// the pair pipeline then decides Sigma_N^Xi(x).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <mutex>
#include <numeric>
#include <vector>

#include "stb_internal.h"

using namespace stb;

namespace {

// A cluster's bounding ball (t, x, y, z, r); r < 0: empty cluster.
struct Ball {
  double c[4];
  double r;
};

// Spread the low 16 bits of v over every fourth bit.
inline uint64_t spread4(uint64_t v) {
  uint64_t x = v & 0xffffull;
  uint64_t out = 0;
  for (int b = 0; b < 16; ++b) out |= ((x >> b) & 1ull) << (4 * b);
  return out;
}

// Theorem phi_xi_sphere: for the ball B_r(y), y = (tau, y), and the point
// x = (t, x), phi = |x - y| - (t - tau) ranges over [phi - d_r(|x - y|),
// phi + r sqrt 2] on the ball, d_r(a) = a + sqrt(r^2 - a^2) below
// a = r / sqrt 2 and r sqrt 2 above.  The cone meets the ball iff that range
// contains 0.  A relative slack keeps the test conservative under rounding.
__device__ __forceinline__ bool ball_maybe_lit(const double* __restrict__ x, const Ball& B) {
  if (B.r < 0.0) return false;
  const double dx = x[1] - B.c[1], dy = x[2] - B.c[2], dz = x[3] - B.c[3];
  const double a = sqrt(dx * dx + dy * dy + dz * dz);
  const double phi = a - (x[0] - B.c[0]);
  const double r2 = B.r * 1.4142135623730951;
  const double dr = a < B.r * 0.7071067811865476 ? a + sqrt(fmax(B.r * B.r - a * a, 0.0)) : r2;
  const double slack = 1e-9 * (fabs(x[0] - B.c[0]) + a + B.r);
  return phi - dr <= slack && phi + r2 >= -slack;
}

constexpr int kTreeThreads = 256;

// Blocks for n threads' worth of work, capped: the kernels loop over their
// items (a dispatch holds fewer than 2^32 work-items).
inline unsigned tree_grid(int64_t nthreads) {
  const int64_t b = (nthreads + kTreeThreads - 1) / kTreeThreads;
  return (unsigned)std::max<int64_t>(1, std::min<int64_t>(b, (int64_t)1 << 20));
}

// Level of the descent: cnt[e] = 2 (inner cluster) or 1 (leaf, on the last
// level) when entry e = (point, cluster) survives, else 0.
__global__ __launch_bounds__(kTreeThreads) void k_tree_test(int64_t nf, const int32_t* __restrict__ fp,
                                                            const int32_t* __restrict__ fv,
                                                            const double* __restrict__ pts,
                                                            const Ball* __restrict__ balls, int last,
                                                            int64_t* __restrict__ cnt) {
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < nf; e += (int64_t)gridDim.x * blockDim.x) {
    const double* x = pts + 4 * (int64_t)fp[e];
    const bool keep = ball_maybe_lit(x, balls[fv[e]]);
    cnt[e] = keep ? (last ? 1 : 2) : 0;
  }
}

// Survivors' sons (heap order: sons of v are 2v + 1, 2v + 2) or, on the last
// level, the surviving leaves themselves, at their prefix offsets.
__global__ __launch_bounds__(kTreeThreads) void k_tree_push(int64_t nf, const int32_t* __restrict__ fp,
                                                            const int32_t* __restrict__ fv,
                                                            const int64_t* __restrict__ off, int last,
                                                            int32_t* __restrict__ np_, int32_t* __restrict__ nv_) {
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < nf; e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t o = off[e], n = off[e + 1] - o;
    if (n == 0) continue;
    if (last) {
      np_[o] = fp[e];
      nv_[o] = fv[e];
    } else {
      np_[o] = fp[e];
      nv_[o] = 2 * fv[e] + 1;
      np_[o + 1] = fp[e];
      nv_[o + 1] = 2 * fv[e] + 2;
    }
  }
}

// Per-panel bounds of the leaves' panels, in the tree's (Morton) order:
// the spatial bounding ball and the time range of each panel.
struct PanelBound {
  double cx, cy, cz, rad, tmin, tmax, diam, pad;
};

// The point x can reach the panel only if some |x - y| over the panel's
// ball equals t - tau for tau in its time range (a conservative test with a
// relative slack, as the flat cull's).
__device__ __forceinline__ bool panel_maybe_lit(const double* __restrict__ x, const PanelBound& P) {
  const double dx = x[1] - P.cx, dy = x[2] - P.cy, dz = x[3] - P.cz;
  const double dc = sqrt(dx * dx + dy * dy + dz * dz);
  const double lb = dc - P.rad, ub = dc + P.rad;
  const double slack = 1e-9 * (fabs(x[0] - P.tmin) + P.diam);
  return (x[0] - P.tmin > lb - slack) && (x[0] - P.tmax < ub + slack);
}

// Panels of the surviving leaves that pass the per-panel test: one
// wavefront per (point, leaf) entry, 64 of the leaf's panels at a time (one
// per lane); a ballot counts them (pass 1) and its mbcnt ranks give each its
// slot (pass 2), in the leaf's panel order.
__global__ __launch_bounds__(kTreeThreads) void k_tree_leafcount(int64_t nf, const int32_t* __restrict__ fp,
                                                                 const int32_t* __restrict__ fv,
                                                                 int64_t first_leaf,
                                                                 const int64_t* __restrict__ leafptr,
                                                                 const PanelBound* __restrict__ pb,
                                                                 const double* __restrict__ pts,
                                                                 int64_t* __restrict__ cnt) {
  const int lane = threadIdx.x & 63;
  const int64_t waves = ((int64_t)gridDim.x * blockDim.x) >> 6;
  for (int64_t e = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6; e < nf; e += waves) {
    const double* x = pts + 4 * (int64_t)fp[e];
    const int64_t l = fv[e] - first_leaf;
    const int64_t b = leafptr[l], n = leafptr[l + 1] - b;
    int64_t c = 0;
    for (int64_t k0 = 0; k0 < n; k0 += 64) {
      const bool ok = k0 + lane < n && panel_maybe_lit(x, pb[b + k0 + lane]);
      c += __popcll(__ballot(ok));
    }
    if (lane == 0) cnt[e] = c;
  }
}

__global__ __launch_bounds__(kTreeThreads) void k_tree_leaffill(int64_t nf, const int32_t* __restrict__ fp,
                                                                const int32_t* __restrict__ fv,
                                                                int64_t first_leaf,
                                                                const int64_t* __restrict__ leafptr,
                                                                const PanelBound* __restrict__ pb,
                                                                const int32_t* __restrict__ perm,
                                                                const double* __restrict__ pts,
                                                                const int64_t* __restrict__ off,
                                                                int32_t* __restrict__ rows,
                                                                int32_t* __restrict__ cols) {
  const int lane = threadIdx.x & 63;
  const int64_t waves = ((int64_t)gridDim.x * blockDim.x) >> 6;
  for (int64_t e = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6; e < nf; e += waves) {
    const int32_t p = fp[e];
    const double* x = pts + 4 * (int64_t)p;
    const int64_t l = fv[e] - first_leaf;
    const int64_t b = leafptr[l], n = leafptr[l + 1] - b;
    int64_t o = off[e];
    for (int64_t k0 = 0; k0 < n; k0 += 64) {
      const bool ok = k0 + lane < n && panel_maybe_lit(x, pb[b + k0 + lane]);
      const uint64_t bal = __ballot(ok);
      const int rank = (int)__builtin_amdgcn_mbcnt_hi((uint32_t)(bal >> 32),
                                                      __builtin_amdgcn_mbcnt_lo((uint32_t)bal, 0));
      if (ok) {
        rows[o + rank] = p;
        cols[o + rank] = perm[b + k0 + lane];
      }
      o += __popcll(bal);
    }
  }
}

// Panels in the surviving leaves, before the per-panel test (the size of
// X_N(x) summed over the points): cnt[e] = size of entry e's leaf.
__global__ __launch_bounds__(kTreeThreads) void k_tree_leafsize(int64_t nf, const int32_t* __restrict__ fv,
                                                                int64_t first_leaf,
                                                                const int64_t* __restrict__ leafptr,
                                                                unsigned long long* __restrict__ total) {
  unsigned long long n = 0;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < nf; e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t l = fv[e] - first_leaf;
    n += (unsigned long long)(leafptr[l + 1] - leafptr[l]);
  }
  for (int off = 32; off > 0; off >>= 1) n += __shfl_down(n, off, 64);
  if ((threadIdx.x & 63) == 0 && n) atomicAdd(total, n);
}

// rowptr[p] = first candidate of point p (candidates grouped by point in
// increasing order), rowptr[np] = nnz.
__global__ __launch_bounds__(kTreeThreads) void k_rows_to_ptr(int64_t np, int64_t nnz,
                                                              const int32_t* __restrict__ rows,
                                                              int64_t* __restrict__ rowptr) {
  for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p <= np; p += (int64_t)gridDim.x * blockDim.x) {
    int64_t lo = 0, hi = nnz;
    while (lo < hi) {
      const int64_t mid = lo + ((hi - lo) >> 1);
      if (rows[mid] < p) lo = mid + 1;
      else hi = mid;
    }
    rowptr[p] = lo;
  }
}

__global__ void k_root_frontier(int64_t np, int32_t* __restrict__ fp, int32_t* __restrict__ fv) {
  for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < np; p += (int64_t)gridDim.x * blockDim.x) {
    fp[p] = (int32_t)p;
    fv[p] = 0;
  }
}

}  // namespace

// The mesh's cluster tree for leaves of at most nmin panels (host build once
// per mesh and nmin, kept on the device).
struct stb_tree {
  int nmin = 0;
  int depth = 0;            // leaves at depth `depth` (root at 0)
  int64_t nleaf = 0;        // 2^depth leaves (the last ones may be empty)
  int32_t* d_perm = nullptr;     // [nt] panels in Morton order
  int64_t* d_leafptr = nullptr;  // [nleaf + 1] leaf l: d_perm[leafptr[l] .. leafptr[l + 1])
  Ball* d_ball = nullptr;        // [2 nleaf - 1], heap order
  PanelBound* d_pb = nullptr;    // [nt] per-panel bounds in d_perm's order
};

void stb_free_tree(stb_mesh* m) {
  if (!m->tree) return;
  dfree(m->tree->d_perm);
  dfree(m->tree->d_leafptr);
  dfree(m->tree->d_ball);
  dfree(m->tree->d_pb);
  delete m->tree;
  m->tree = nullptr;
}

static stb_status build_tree(stb_ctx* ctx, stb_mesh* m, int nmin) {
  const int64_t nt = m->nt, nv = m->nv;
  std::vector<double> vtx((size_t)nv * 4);
  std::vector<int32_t> tet((size_t)nt * 4);
  HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
  HIPCHK(ctx, hipMemcpy(vtx.data(), m->d_vtx, sizeof(double) * 4 * nv, hipMemcpyDeviceToHost));
  HIPCHK(ctx, hipMemcpy(tet.data(), m->d_tet, sizeof(int32_t) * 4 * nt, hipMemcpyDeviceToHost));
  // Morton order of the panels' space-time centroids, one scale for all four
  // coordinates (the light cone is at 45 degrees in (t, x))
  double lo[4] = {1e300, 1e300, 1e300, 1e300}, hi[4] = {-1e300, -1e300, -1e300, -1e300};
  std::vector<double> cen((size_t)nt * 4);
  for (int64_t i = 0; i < nt; ++i)
    for (int c = 0; c < 4; ++c) {
      double s = 0.0;
      for (int k = 0; k < 4; ++k) s += vtx[(size_t)tet[(size_t)i * 4 + k] * 4 + c];
      cen[(size_t)i * 4 + c] = 0.25 * s;
      lo[c] = std::min(lo[c], cen[(size_t)i * 4 + c]);
      hi[c] = std::max(hi[c], cen[(size_t)i * 4 + c]);
    }
  double ext = 0.0;
  for (int c = 0; c < 4; ++c) ext = std::max(ext, hi[c] - lo[c]);
  if (!(ext > 0.0)) ext = 1.0;
  std::vector<uint64_t> code((size_t)nt);
  for (int64_t i = 0; i < nt; ++i) {
    uint64_t k = 0;
    for (int c = 0; c < 4; ++c) {
      const double u = (cen[(size_t)i * 4 + c] - lo[c]) / ext;
      const uint64_t q = (uint64_t)std::min(65535.0, std::max(0.0, std::floor(u * 65536.0)));
      k |= spread4(q) << (3 - c);
    }
    code[(size_t)i] = k;
  }
  std::vector<int32_t> perm((size_t)nt);
  std::iota(perm.begin(), perm.end(), 0);
  std::stable_sort(perm.begin(), perm.end(), [&](int32_t a, int32_t b) { return code[(size_t)a] < code[(size_t)b]; });
  // perfect binary tree over ceil(nt / nmin) leaves
  const int64_t nreal = (nt + nmin - 1) / nmin;
  int depth = 0;
  while (((int64_t)1 << depth) < nreal) ++depth;
  const int64_t nleaf = (int64_t)1 << depth;
  std::vector<int64_t> leafptr((size_t)nleaf + 1);
  for (int64_t l = 0; l <= nleaf; ++l) leafptr[(size_t)l] = std::min(nt, l * (int64_t)nmin);
  // balls: per cluster, the centre of the bounding box of its panels'
  // vertices and the largest distance to them (a non-minimal bounding ball)
  const int64_t nnode = 2 * nleaf - 1;
  std::vector<Ball> ball((size_t)nnode);
  for (int d = depth; d >= 0; --d) {
    const int64_t first = ((int64_t)1 << d) - 1, cnt = (int64_t)1 << d, span = nleaf >> d;
    for (int64_t q = 0; q < cnt; ++q) {
      const int64_t p0 = leafptr[(size_t)(q * span)], p1 = leafptr[(size_t)((q + 1) * span)];
      Ball B;
      if (p1 <= p0) {
        for (double& c : B.c) c = 0.0;
        B.r = -1.0;
      } else {
        double bl[4] = {1e300, 1e300, 1e300, 1e300}, bh[4] = {-1e300, -1e300, -1e300, -1e300};
        for (int64_t k = p0; k < p1; ++k)
          for (int v = 0; v < 4; ++v) {
            const double* X = &vtx[(size_t)tet[(size_t)perm[(size_t)k] * 4 + v] * 4];
            for (int c = 0; c < 4; ++c) { bl[c] = std::min(bl[c], X[c]); bh[c] = std::max(bh[c], X[c]); }
          }
        for (int c = 0; c < 4; ++c) B.c[c] = 0.5 * (bl[c] + bh[c]);
        double r2 = 0.0;
        for (int64_t k = p0; k < p1; ++k)
          for (int v = 0; v < 4; ++v) {
            const double* X = &vtx[(size_t)tet[(size_t)perm[(size_t)k] * 4 + v] * 4];
            double s = 0.0;
            for (int c = 0; c < 4; ++c) s += (X[c] - B.c[c]) * (X[c] - B.c[c]);
            r2 = std::max(r2, s);
          }
        B.r = std::sqrt(r2) * (1.0 + 1e-12) + 1e-300;
      }
      ball[(size_t)(first + q)] = B;
    }
  }
  // per-panel bounds in tree order: spatial bounding ball (centre of the
  // vertices' box, largest distance to them), time range, size
  std::vector<PanelBound> pb((size_t)nt);
  for (int64_t k = 0; k < nt; ++k) {
    const int32_t i = perm[(size_t)k];
    double bl[4] = {1e300, 1e300, 1e300, 1e300}, bh[4] = {-1e300, -1e300, -1e300, -1e300};
    for (int v = 0; v < 4; ++v) {
      const double* X = &vtx[(size_t)tet[(size_t)i * 4 + v] * 4];
      for (int c = 0; c < 4; ++c) { bl[c] = std::min(bl[c], X[c]); bh[c] = std::max(bh[c], X[c]); }
    }
    PanelBound P;
    P.cx = 0.5 * (bl[1] + bh[1]);
    P.cy = 0.5 * (bl[2] + bh[2]);
    P.cz = 0.5 * (bl[3] + bh[3]);
    double r2 = 0.0, span = 0.0;
    for (int v = 0; v < 4; ++v) {
      const double* X = &vtx[(size_t)tet[(size_t)i * 4 + v] * 4];
      const double dx = X[1] - P.cx, dy = X[2] - P.cy, dz = X[3] - P.cz;
      r2 = std::max(r2, dx * dx + dy * dy + dz * dz);
      for (int w = 0; w < 4; ++w) {
        const double* Y = &vtx[(size_t)tet[(size_t)i * 4 + w] * 4];
        span = std::max(span, std::sqrt((X[1] - Y[1]) * (X[1] - Y[1]) + (X[2] - Y[2]) * (X[2] - Y[2]) +
                                        (X[3] - Y[3]) * (X[3] - Y[3])));
      }
    }
    P.rad = std::sqrt(r2) * (1.0 + 1e-12);
    P.tmin = bl[0];
    P.tmax = bh[0];
    P.diam = std::max(span, bh[0] - bl[0]);
    P.pad = 0.0;
    pb[(size_t)k] = P;
  }
  stb_tree* T = new stb_tree();
  T->nmin = nmin;
  T->depth = depth;
  T->nleaf = nleaf;
  if (dalloc(&T->d_perm, (size_t)std::max<int64_t>(nt, 1)) != hipSuccess ||
      dalloc(&T->d_leafptr, (size_t)nleaf + 1) != hipSuccess || dalloc(&T->d_ball, (size_t)nnode) != hipSuccess ||
      dalloc(&T->d_pb, (size_t)std::max<int64_t>(nt, 1)) != hipSuccess) {
    dfree(T->d_perm); dfree(T->d_leafptr); dfree(T->d_ball); dfree(T->d_pb);
    delete T;
    return stb_fail(ctx, STB_E_NO_MEMORY, "cluster tree");
  }
  hipError_t e = hipMemcpy(T->d_perm, perm.data(), 4 * nt, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(T->d_leafptr, leafptr.data(), 8 * (nleaf + 1), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(T->d_ball, ball.data(), sizeof(Ball) * nnode, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(T->d_pb, pb.data(), sizeof(PanelBound) * nt, hipMemcpyHostToDevice);
  if (e != hipSuccess) {
    dfree(T->d_perm); dfree(T->d_leafptr); dfree(T->d_ball); dfree(T->d_pb);
    delete T;
    return stb_fail(ctx, STB_E_DEVICE, "cluster tree upload: %s", hipGetErrorString(e));
  }
  stb_free_tree(m);
  m->tree = T;
  return STB_OK;
}

stb_status stb_ensure_tree(stb_ctx* ctx, stb_mesh* m, int nmin) {
  if (nmin < 1 || nmin > 4096) return stb_fail(ctx, STB_E_INVALID_ARG, "n_min must be in [1, 4096]");
  // contexts that share the mesh (server slots) build it once
  std::lock_guard<std::mutex> lk(m->tree_mu);
  if (m->tree && m->tree->nmin == nmin) return STB_OK;
  return build_tree(ctx, m, nmin);
}

// Candidates of np points (d_pts, device, (t, x, y, z)) by the tree:
// *d_rowptr [np + 1], *d_cols and *d_rowof [*nnz] (allocated here; each
// point's candidates in the tree's leaf order).  *nleaves (optional): the
// (point, leaf) pairs that survived.
stb_status stb_tree_cull(stb_ctx* ctx, stb_mesh* m, int nmin, int64_t np, const double* d_pts,
                         int64_t** d_rowptr, int32_t** d_cols, int32_t** d_rowof, int64_t* nnz,
                         int64_t* nleaves) {
  stb_status s = stb_ensure_tree(ctx, m, nmin);
  if (s) return s;
  const stb_tree* T = m->tree;
  hipStream_t st = ctx->stream;
  int32_t *fp = nullptr, *fv = nullptr, *gp = nullptr, *gv = nullptr;
  int64_t *cnt = nullptr, *off = nullptr, *tmp = nullptr;
  auto cleanup = [&]() { dfree(fp); dfree(fv); dfree(gp); dfree(gv); dfree(cnt); dfree(off); dfree(tmp); };
  int64_t nf = np;
  if (dalloc(&fp, (size_t)np) != hipSuccess || dalloc(&fv, (size_t)np) != hipSuccess) {
    cleanup();
    return stb_fail(ctx, STB_E_NO_MEMORY, "tree frontier");
  }
  if (np > 0)
    hipLaunchKernelGGL(k_root_frontier, dim3(tree_grid(np)), dim3(kTreeThreads), 0, st, np, fp, fv);
  for (int d = 0; d <= T->depth && nf > 0; ++d) {
    const int last = d == T->depth;
    if (dalloc(&cnt, (size_t)nf) != hipSuccess || dalloc(&off, (size_t)nf + 1) != hipSuccess ||
        dalloc(&tmp, (size_t)stb_scan_tmp_elems<int64_t>(nf)) != hipSuccess) {
      cleanup();
      return stb_fail(ctx, STB_E_NO_MEMORY, "tree frontier of %lld entries", (long long)nf);
    }
    const unsigned g = tree_grid(nf);
    hipLaunchKernelGGL(k_tree_test, dim3(g), dim3(kTreeThreads), 0, st, nf, fp, fv, d_pts, T->d_ball, last, cnt);
    hipError_t e = stb_scan<int64_t>(cnt, off, nf, tmp, st);
    int64_t nn = 0;
    if (e == hipSuccess) e = hipMemcpyAsync(&nn, off + nf, 8, hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) { cleanup(); return stb_fail(ctx, STB_E_DEVICE, "tree level: %s", hipGetErrorString(e)); }
    if (nn > (int64_t)INT32_MAX * 4) { cleanup(); return stb_fail(ctx, STB_E_NO_MEMORY, "tree frontier too large"); }
    if (dalloc(&gp, (size_t)nn) != hipSuccess || dalloc(&gv, (size_t)nn) != hipSuccess) {
      cleanup();
      return stb_fail(ctx, STB_E_NO_MEMORY, "tree frontier of %lld entries", (long long)nn);
    }
    hipLaunchKernelGGL(k_tree_push, dim3(g), dim3(kTreeThreads), 0, st, nf, fp, fv, off, last, gp, gv);
    HIPCHK(ctx, hipGetLastError());
    dfree(fp); dfree(fv); dfree(cnt); dfree(off); dfree(tmp);
    fp = gp; fv = gv; gp = gv = nullptr; cnt = off = tmp = nullptr;
    nf = nn;
  }
  if (nleaves) *nleaves = nf;
  // panels of the surviving leaves that pass the per-panel bound test
  const int64_t first_leaf = T->nleaf - 1;
  unsigned long long* d_union = nullptr;
  if (dalloc(&cnt, (size_t)std::max<int64_t>(nf, 1)) != hipSuccess || dalloc(&off, (size_t)nf + 1) != hipSuccess ||
      dalloc(&tmp, (size_t)stb_scan_tmp_elems<int64_t>(nf)) != hipSuccess || dalloc(&d_union, 1) != hipSuccess) {
    dfree(d_union);
    cleanup();
    return stb_fail(ctx, STB_E_NO_MEMORY, "tree leaves");
  }
  const unsigned gw = tree_grid(std::max<int64_t>(nf, 1) * 64);
  const unsigned g1 = tree_grid(std::max<int64_t>(nf, 1));
  hipError_t e = hipMemsetAsync(d_union, 0, 8, st);
  if (nf > 0) {
    hipLaunchKernelGGL(k_tree_leafsize, dim3(g1), dim3(kTreeThreads), 0, st, nf, fv, first_leaf, T->d_leafptr,
                       d_union);
    hipLaunchKernelGGL(k_tree_leafcount, dim3(gw), dim3(kTreeThreads), 0, st, nf, fp, fv, first_leaf,
                       T->d_leafptr, T->d_pb, d_pts, cnt);
  }
  if (e == hipSuccess) e = stb_scan<int64_t>(cnt, off, nf, tmp, st);
  int64_t total = 0;
  unsigned long long uni = 0;
  if (e == hipSuccess) e = hipMemcpyAsync(&total, off + nf, 8, hipMemcpyDeviceToHost, st);
  if (e == hipSuccess) e = hipMemcpyAsync(&uni, d_union, 8, hipMemcpyDeviceToHost, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  dfree(d_union);
  if (e != hipSuccess) { cleanup(); return stb_fail(ctx, STB_E_DEVICE, "tree leaves: %s", hipGetErrorString(e)); }
  ctx->lit_search[0] = nf;
  ctx->lit_search[1] = (int64_t)uni;
  ctx->lit_search[2] = total;
  *d_rowptr = nullptr; *d_cols = nullptr; *d_rowof = nullptr;
  if (dalloc(d_rowptr, (size_t)np + 1) != hipSuccess || dalloc(d_cols, (size_t)std::max<int64_t>(total, 1)) != hipSuccess ||
      dalloc(d_rowof, (size_t)std::max<int64_t>(total, 1)) != hipSuccess) {
    cleanup();
    dfree(*d_rowptr); dfree(*d_cols); dfree(*d_rowof);
    *d_rowptr = nullptr; *d_cols = nullptr; *d_rowof = nullptr;
    return stb_fail(ctx, STB_E_NO_MEMORY, "tree candidates (%lld)", (long long)total);
  }
  if (nf > 0)
    hipLaunchKernelGGL(k_tree_leaffill, dim3(gw), dim3(kTreeThreads), 0, st, nf, fp, fv, first_leaf,
                       T->d_leafptr, T->d_pb, T->d_perm, d_pts, off, *d_rowof, *d_cols);
  hipLaunchKernelGGL(k_rows_to_ptr, dim3(tree_grid(np + 1)), dim3(kTreeThreads), 0, st, np, total, *d_rowof,
                     *d_rowptr);
  e = hipGetLastError();
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  cleanup();
  if (e != hipSuccess) return stb_fail(ctx, STB_E_DEVICE, "tree candidates: %s", hipGetErrorString(e));
  *nnz = total;
  return STB_OK;
}
