// stb_dl.hip -- retarded double-layer potential (eq. dlp, kernels k2 and k3
// of eq. kfunc) of a density in V_h^1 (continuous, linear on every panel;
// def. st_be), at points off or on the surface.
//
// The candidates (point, panel) come from the single layer's cull.  Three
// stages give the potentials of each candidate panel's four hat functions:
// per candidate the lit test and the breakpoints, which list the pieces;
// per piece the empty-piece test and the Gauss nodes (dense work); per
// candidate the sum of its pieces.  A last kernel sums the hats per point
// against the vertex values in a fixed order.  stb_inner_values_D keeps one
// lane per pair (inner_dl_serial) for checks.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <vector>

#include "stb_internal.h"

using namespace stb;

namespace {

// nsign[j] = +1 where the given outward normal has a positive component along
// the frame normal n of panel j, -1 where negative; status 1 where the given
// normal is not finite or is within 60 degrees of the panel's plane.
__global__ void k_normal_sign(int64_t nt, const TrialRec* __restrict__ trial,
                              const double* __restrict__ nrm, double* __restrict__ nsign,
                              int32_t* __restrict__ status) {
  int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= nt) return;
  const double* g = nrm + 3 * j;
  const TrialRec& T = trial[j];
  double l = sqrt(g[0] * g[0] + g[1] * g[1] + g[2] * g[2]);
  double c = g[0] * T.n[0] + g[1] * T.n[1] + g[2] * T.n[2];
  bool ok = l > 0.0 && isfinite(l) && fabs(c) >= 0.5 * l;
  nsign[j] = c > 0.0 ? 1.0 : -1.0;
  status[j] = ok ? 0 : 1;
}

// u(p) = sum over p's candidates and the panel's vertices of v(vertex) *
// hat potential: one wavefront per point, lane-strided partial sums and a
// fixed-order shuffle reduction.
__global__ __launch_bounds__(256) void k_dl_point_sum(int64_t np, const int64_t* __restrict__ rowptr,
                                                      const int32_t* __restrict__ cols,
                                                      const int32_t* __restrict__ tet,
                                                      const double* __restrict__ v,
                                                      const double* __restrict__ h4,
                                                      double* __restrict__ out) {
  int64_t i = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  int lane = threadIdx.x & 63;
  if (i >= np) return;
  double s = 0.0;
  for (int64_t c = rowptr[i] + lane; c < rowptr[i + 1]; c += 64) {
    const int32_t* tv = tet + 4 * (int64_t)cols[c];
    const double* h = h4 + 4 * c;
    s += ((v[tv[0]] * h[0] + v[tv[1]] * h[1]) + v[tv[2]] * h[2]) + v[tv[3]] * h[3];
  }
  for (int off = 32; off > 0; off >>= 1) s += __shfl_down(s, off, 64);
  if (lane == 0) out[i] = s;
}

__global__ void k_dl_pairs(int64_t k, const TrialRec* __restrict__ trial,
                           const FaceAng* __restrict__ fang, const double* __restrict__ nsign,
                           const double* __restrict__ pts, const int32_t* __restrict__ panel,
                           const double* __restrict__ gl, int ng, double* __restrict__ out4) {
  int64_t m = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (m >= k) return;
  const int32_t j = panel[m];
  double x4[4] = {pts[4 * m], pts[4 * m + 1], pts[4 * m + 2], pts[4 * m + 3]};
  double h[4];
  inner_dl_serial(trial[j], fang[j], x4, nsign[j], ng, gl, gl + kMaxNg, h);
  for (int q = 0; q < 4; ++q) out4[4 * m + q] = h[q];
}

// ---- split evaluation: candidates -> pieces -> nodes -> candidates ----
//
// Stage 1 (one lane per candidate): apex data, lit test, w-range,
// breakpoints; the pieces the ray test does not rule out are appended to a
// list, each candidate's contiguously and in phi order (a block takes one
// range of the list with one atomic); the candidate keeps C_k, d^2, the
// w-range and the factor nsign d / 4 pi.  Stage 2 (one lane per piece): the
// empty-piece test and the Gauss nodes, three sums per piece.  Stage 3 (one
// lane per candidate): its pieces summed in order, then the four hats.
constexpr int kDlCb = 8;   // C[4], d2, wlo, whi, factor
// Pieces narrower than this take the full evaluation at every node: their
// nodes sit within rounding of the breakpoints, where the gap structure is
// ambiguous.
constexpr double kDlRecipeMinH = 1e-8;

// Breakpoint slots 0..23 of a lane in LDS (slot s of lane t at s * B + t),
// the rare rest in private memory: the private lists of all resident lanes
// would not stay in the caches.
constexpr int kDlBpLds = 24;
struct DlBp {
  double* lds;
  int stride;
  double* spill;
  __device__ __forceinline__ void put(int i, double v) {
    if (i < kDlBpLds) lds[i * stride] = v;
    else spill[i - kDlBpLds] = v;
  }
  __device__ __forceinline__ double get(int i) const {
    return i < kDlBpLds ? lds[i * stride] : spill[i - kDlBpLds];
  }
};

__global__ __launch_bounds__(256) void k_dl_split(int64_t c0, int64_t n, const int32_t* __restrict__ rowof,
                                                  const int32_t* __restrict__ cols,
                                                  const TrialRec* __restrict__ trial,
                                                  const FaceAng* __restrict__ fang,
                                                  const double* __restrict__ nsign,
                                                  const double* __restrict__ pts, double* __restrict__ cb,
                                                  int64_t* __restrict__ poff, int32_t* __restrict__ pcnt,
                                                  double* __restrict__ pa, double* __restrict__ ph,
                                                  int32_t* __restrict__ pc, int64_t cap,
                                                  unsigned long long* __restrict__ counter) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const bool valid = k < n;
  __shared__ double s_bp[kDlBpLds * 256];
  double spill[kMaxBp - kDlBpLds];
  DlBp bp{s_bp + threadIdx.x, (int)blockDim.x, spill};
  int nb = -1;   // -1: nothing to integrate; 0: periodic (two trapezoid halves)
  unsigned np = 0;
  Apex A;
  const TrialRec* T = nullptr;
  if (valid) {
    const int64_t c = c0 + k;
    const int32_t j = cols[c];
    T = trial + j;
    const double* xp = pts + 4 * (int64_t)rowof[c];
    double x4[4] = {xp[0], xp[1], xp[2], xp[3]};
    apex_of(*T, x4, A);
    double wlo = 0.0, whi = 0.0;
    double* o = cb + kDlCb * k;
    o[7] = 0.0;
    if (A.d != 0.0) {
      const int lq = lit_quick(*T, x4, A);
      const bool lit = lq == 1 || (lq == 2 && lit_test(*T, x4, A));
      if (lit && w_range(*T, A, wlo, whi)) {
        for (int q = 0; q < 4; ++q) o[q] = A.C[q];
        o[4] = A.d * A.d;
        o[5] = wlo;
        o[6] = whi;
        o[7] = nsign[j] * A.d / (4.0 * kPi);
        nb = breakpoints_t(*T, fang[j], A, bp);
        sort_bp_t(bp, nb);
        if (nb == 0) {
          np = 2;
        } else {
          for (int m = 0; m < nb; ++m) {
            const double a = bp.get(m), e = (m + 1 < nb) ? bp.get(m + 1) : bp.get(0) + kTwoPi;
            if (e - a > 0.0 && !piece_misses(*T, A, a, e - a)) ++np;
          }
        }
      }
    }
  }
  __shared__ unsigned s_cnt;
  __shared__ unsigned long long s_base;
  if (threadIdx.x == 0) s_cnt = 0;
  __syncthreads();
  const unsigned my = np ? atomicAdd(&s_cnt, np) : 0u;
  __syncthreads();
  if (threadIdx.x == 0) s_base = s_cnt ? atomicAdd(counter, (unsigned long long)s_cnt) : 0ull;
  __syncthreads();
  if (!valid) return;
  const unsigned long long base = s_base + my;
  poff[k] = (int64_t)base;
  pcnt[k] = (int32_t)np;
  if (np == 0 || base + np > (unsigned long long)cap) return;
  int64_t w = (int64_t)base;
  if (nb == 0) {
    for (int h = 0; h < 2; ++h, ++w) { pa[w] = (double)h; ph[w] = -1.0; pc[w] = (int32_t)k; }
    return;
  }
  for (int m = 0; m < nb; ++m) {
    const double a = bp.get(m), e = (m + 1 < nb) ? bp.get(m + 1) : bp.get(0) + kTwoPi;
    if (!(e - a > 0.0) || piece_misses(*T, A, a, e - a)) continue;
    pa[w] = a; ph[w] = e - a; pc[w] = (int32_t)k; ++w;
  }
}

// Stage 2: one lane per piece.  A trapezoid half (ph < 0) takes its n_g
// nodes of the periodic rule; a Gauss piece is tested at its midpoint and
// quarter points first, and that test's recipe (the endpoint formulas of at
// most two gaps) gives every node its gaps from two faces per gap instead of
// the four-face sweep; without a recipe, the full evaluation (dl_eval).
__global__ __launch_bounds__(256) void k_dl_piece_nodes(int64_t npc, int64_t c0, const double* __restrict__ pa,
                                                        const double* __restrict__ ph,
                                                        const int32_t* __restrict__ pc,
                                                        const double* __restrict__ cb,
                                                        const int32_t* __restrict__ cols,
                                                        const TrialRec* __restrict__ trial,
                                                        const double* __restrict__ gl, int ng,
                                                        double* __restrict__ out3) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= npc) return;
  const int64_t k = pc[p];
  const double* o = cb + kDlCb * k;
  const TrialRec& T = trial[cols[c0 + k]];
  ComboL L;
  FaceSet F;
  for (int q = 0; q < 4; ++q) {
    L.C[q] = o[q]; L.fa[q] = T.fa[q]; L.fb[q] = T.fb[q]; L.fc[q] = T.fc[q];
    F.fa[q] = T.fa[q]; F.fb[q] = T.fb[q]; F.fc[q] = T.fc[q];
  }
  L.d2 = o[4]; L.wlo = o[5]; L.whi = o[6];
  const double a = pa[p], H = ph[p];
  double ia = 0.0, ic = 0.0, is = 0.0;
  auto node = [&](double phi, double wt) {
    double sn, cs, sa, sh;
    sincos_small(phi, &sn, &cs);
    dl_eval(F, L.C, L.d2, L.wlo, L.whi, cs, sn, sa, sh);
    ia += wt * sa;
    ic += (wt * sh) * cs;
    is += (wt * sh) * sn;
  };
  if (H < 0.0) {
    const double ht = kTwoPi / (2 * ng);
    for (int g = 0; g < ng; ++g) node((a * ng + g) * ht, ht);
  } else {
    // the empty-piece test also yields the piece's recipe (the gap
    // structure at its midpoint, else at the first non-zero quarter point)
    uint32_t rec = 0u;
    double sn, cs;
    sincos_small(a + 0.5 * H, &sn, &cs);
    bool ne = L_eval_recipe(L, cs, sn, &rec) != 0.0;
    if (!ne) {
      sincos_small(a + 0.25 * H, &sn, &cs);
      ne = L_eval_recipe(L, cs, sn, &rec) != 0.0;
    }
    if (!ne) {
      sincos_small(a + 0.75 * H, &sn, &cs);
      ne = L_eval_recipe(L, cs, sn, &rec) != 0.0;
    }
    const int ngap = recipe_gaps(rec);
    if (ne && rec != 0u && H >= kDlRecipeMinH) {
      // every node from the recipe's endpoint formulas only
      Endpoint E[2 * kRecipeGaps];
      for (int q = 0; q < 2 * ngap; ++q) {
        const uint32_t id = (rec >> (8 * (q >> 1) + ((q & 1) ? 0 : 4))) & 15u;
        const int f = id >= 2 ? (int)(id - 2) >> 1 : 0;
        E[q].a = L.fa[f]; E[q].fb = L.fb[f]; E[q].fc = L.fc[f]; E[q].C = L.C[f];
        E[q].cst = id < 2;
        E[q].cval = id == 0 ? L.wlo : L.whi;
        E[q].isb = id >= 2 && ((id - 2) & 1u);
      }
      for (int g = 0; g < ng; ++g) {
        const double u = gl[g];
        const double sm = u * u * (3.0 - 2.0 * u);
        const double wt = H * (6.0 * u * (1.0 - u)) * gl[kMaxNg + g];
        sincos_small(a + H * sm, &sn, &cs);
        double sa = 0.0, sh = 0.0;
        for (int q = 0; q < ngap; ++q) {
          const double w0 = endpoint_value(E[2 * q], L.d2, L.wlo, L.whi, cs, sn);
          const double w1 = endpoint_value(E[2 * q + 1], L.d2, L.wlo, L.whi, cs, sn);
          if (w1 > w0) {
            const double q0 = 1.0 / fma(w0, w0, L.d2), q1 = 1.0 / fma(w1, w1, L.d2);
            sa += 2.0 * (w0 * q0 - w1 * q1);
            sh += log(w1 / w0) + 2.0 * L.d2 * (q1 - q0);
          }
        }
        ia += wt * sa;
        ic += (wt * sh) * cs;
        is += (wt * sh) * sn;
      }
    } else if (ne) {
      for (int g = 0; g < ng; ++g) {
        const double u = gl[g];
        const double sm = u * u * (3.0 - 2.0 * u);
        const double ds = 6.0 * u * (1.0 - u);
        node(a + H * sm, H * ds * gl[kMaxNg + g]);
      }
    }
  }
  out3[3 * p] = ia;
  out3[3 * p + 1] = ic;
  out3[3 * p + 2] = is;
}

// Stage 3: per candidate, its pieces in order, then the hats
// lambda_m(t, p) = C_m / D_m and grad lambda_m = -(b_m, c_m) / D_m.
__global__ void k_dl_finish(int64_t c0, int64_t n, const int32_t* __restrict__ cols,
                            const TrialRec* __restrict__ trial, const double* __restrict__ cb,
                            const int64_t* __restrict__ poff, const int32_t* __restrict__ pcnt,
                            const double* __restrict__ out3, double* __restrict__ out4) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n) return;
  double ia = 0.0, ic = 0.0, is = 0.0;
  for (int64_t p = poff[k]; p < poff[k] + pcnt[k]; ++p) {
    ia += out3[3 * p];
    ic += out3[3 * p + 1];
    is += out3[3 * p + 2];
  }
  const double* o = cb + kDlCb * k;
  const TrialRec& T = trial[cols[c0 + k]];
  double* h = out4 + 4 * (c0 + k);
  for (int m = 0; m < 4; ++m) {
    const double Dm = T.fh[m] - T.fa[m] * T.V[m][0] - T.fb[m] * T.V[m][1] - T.fc[m] * T.V[m][2];
    h[m] = pcnt[k] ? o[7] * (o[m] * ia - T.fb[m] * ic - T.fc[m] * is) / Dm : 0.0;
  }
}

// The points of entities [r0, r0 + nr) (faces), maxq slots each, packed
// without padding: point q of entity i goes to off[i] - off[r0] + q (off:
// exclusive prefix of the counts).
__global__ void k_pack_outer(int64_t r0, int64_t nr, int maxq, const double* __restrict__ opts,
                             const int64_t* __restrict__ off, double* __restrict__ pts) {
  int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= nr * maxq) return;
  const int64_t i = r0 + g / maxq;
  const int q = (int)(g % maxq);
  if (q >= off[i + 1] - off[i]) return;
  const double* src = opts + (i * maxq + q) * 4;
  double* dst = pts + (off[i] - off[r0] + q) * 4;
  for (int c = 0; c < 4; ++c) dst[c] = src[c];
}

// Sum of K v over each face's points: kf[f] = sum_q kv[off[f] - off[f0] + q]
// for faces [f0, f0 + nf) (off: exclusive prefix of the faces' counts).
__global__ void k_face_ksum(int64_t f0, int64_t nf, const int64_t* __restrict__ off,
                            const double* __restrict__ kv, double* __restrict__ kf) {
  int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= nf) return;
  const int64_t f = f0 + g;
  double s = 0.0;
  for (int64_t k = off[f]; k < off[f + 1]; ++k) s += kv[k - off[f0]];
  kf[f] = s;
}

// out[i] = sum_q w_iq (c_id v_h(x_iq) + (K v)(x_iq)): the energetic forms of
// eq. int_bform with A = I and A = K.  v_h at an outer point of panel i is
// panel i's own linear function: its hats are (h_m - a_m tau - b_m u -
// c_m v) / D_m in the local frame.  The K part comes per slot (face) of the
// panel: its per-point weight times the face's sum kf (the outer points of a
// face are the same for both panels that share it).
__global__ void k_dl_outer_sum(int64_t nt, int maxq, const TrialRec* __restrict__ trial,
                               const int32_t* __restrict__ tet, const double* __restrict__ v,
                               const double* __restrict__ opts, const double* __restrict__ ow,
                               const int32_t* __restrict__ onq, const int32_t* __restrict__ pf,
                               const double* __restrict__ pw, const double* __restrict__ kf,
                               double c_id, double* __restrict__ out) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nt) return;
  const TrialRec& T = trial[i];
  double coef[4];
  for (int m = 0; m < 4; ++m) {
    const double Dm = T.fh[m] - T.fa[m] * T.V[m][0] - T.fb[m] * T.V[m][1] - T.fc[m] * T.V[m][2];
    coef[m] = v[tet[4 * i + m]] / Dm;
  }
  double id = 0.0;
  for (int q = 0; q < onq[i]; ++q) {
    const double* x = opts + (i * maxq + q) * 4;
    const double dx = x[1] - T.o[0], dy = x[2] - T.o[1], dz = x[3] - T.o[2];
    const double u = dx * T.e1[0] + dy * T.e1[1] + dz * T.e1[2];
    const double w = dx * T.e2[0] + dy * T.e2[1] + dz * T.e2[2];
    double vq = 0.0;
    for (int m = 0; m < 4; ++m) vq += coef[m] * (T.fh[m] - T.fa[m] * x[0] - T.fb[m] * u - T.fc[m] * w);
    id += ow[i * maxq + q] * vq;
  }
  double kk = 0.0;
  for (int k = 0; k < 4; ++k) {
    const int32_t f = pf[4 * i + k];
    if (f >= 0) kk += pw[4 * i + k] * kf[f];
  }
  out[i] = c_id * id + kk;
}

unsigned grid_for(int64_t n, int b) { return (unsigned)((n + b - 1) / b); }

}  // namespace

// Candidates per pass of the split evaluation, and initial pieces per candidate.
constexpr int64_t kDlCandChunk = int64_t(1) << 23;
constexpr int64_t kDlPiecesPer = 12;

// The hats of candidates [0, nnz) into h4 through the three stages.
static stb_status dl_split(stb_ctx* ctx, stb_mesh* mesh, const stb_quad_params& p, int64_t nnz,
                           const int32_t* d_rowof, const int32_t* d_cols, const double* d_pts, double* d_h4) {
  if (nnz == 0) return STB_OK;
  hipStream_t st = ctx->stream;
  const int64_t chunk = std::min(nnz, kDlCandChunk);
  double *d_cb = nullptr, *d_pa = nullptr, *d_ph = nullptr, *d_o3 = nullptr;
  int64_t* d_poff = nullptr;
  int32_t *d_pcnt = nullptr, *d_pc = nullptr;
  unsigned long long* d_ctr = nullptr;
  int64_t cap = chunk * kDlPiecesPer;
  auto free_pieces = [&]() { dfree(d_pa); dfree(d_ph); dfree(d_pc); dfree(d_o3); d_pa = d_ph = d_o3 = nullptr; d_pc = nullptr; };
  auto cleanup = [&]() { dfree(d_cb); dfree(d_poff); dfree(d_pcnt); dfree(d_ctr); free_pieces(); };
  auto alloc_pieces = [&]() {
    return dalloc(&d_pa, (size_t)cap) == hipSuccess && dalloc(&d_ph, (size_t)cap) == hipSuccess &&
           dalloc(&d_pc, (size_t)cap) == hipSuccess && dalloc(&d_o3, (size_t)cap * 3) == hipSuccess;
  };
  if (dalloc(&d_cb, (size_t)chunk * kDlCb) != hipSuccess || dalloc(&d_poff, (size_t)chunk) != hipSuccess ||
      dalloc(&d_pcnt, (size_t)chunk) != hipSuccess || dalloc(&d_ctr, 1) != hipSuccess || !alloc_pieces()) {
    cleanup();
    return stb_fail(ctx, STB_E_NO_MEMORY, "double-layer pieces");
  }
  hipError_t e = hipSuccess;
  for (int64_t c0 = 0; c0 < nnz && e == hipSuccess;) {
    const int64_t n = std::min(chunk, nnz - c0);
    unsigned long long npc = 0;
    for (;;) {
      e = hipMemsetAsync(d_ctr, 0, sizeof(unsigned long long), st);
      if (e != hipSuccess) break;
      hipLaunchKernelGGL(k_dl_split, dim3(grid_for(n, 256)), dim3(256), 0, st, c0, n, d_rowof, d_cols,
                         mesh->d_trial, mesh->d_fang, mesh->d_nsign, d_pts, d_cb, d_poff, d_pcnt, d_pa, d_ph,
                         d_pc, cap, d_ctr);
      if ((e = hipGetLastError()) != hipSuccess) break;
      if ((e = hipMemcpyAsync(&npc, d_ctr, sizeof(npc), hipMemcpyDeviceToHost, st)) != hipSuccess) break;
      if ((e = hipStreamSynchronize(st)) != hipSuccess) break;
      if ((int64_t)npc <= cap) break;
      free_pieces();                       // the list overflowed: grow it and redo the pass
      cap = (int64_t)npc + npc / 8 + 1024;
      if (!alloc_pieces()) { cleanup(); return stb_fail(ctx, STB_E_NO_MEMORY, "double-layer pieces"); }
    }
    if (e != hipSuccess) break;
    if (npc > 0)
      hipLaunchKernelGGL(k_dl_piece_nodes, dim3(grid_for((int64_t)npc, 256)), dim3(256), 0, st, (int64_t)npc, c0,
                         d_pa, d_ph, d_pc, d_cb, d_cols, mesh->d_trial, ctx->d_gl, p.n_g, d_o3);
    hipLaunchKernelGGL(k_dl_finish, dim3(grid_for(n, 256)), dim3(256), 0, st, c0, n, d_cols, mesh->d_trial, d_cb,
                       d_poff, d_pcnt, d_o3, d_h4);
    e = hipGetLastError();
    c0 += n;
  }
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  cleanup();
  if (e != hipSuccess) return stb_fail(ctx, STB_E_DEVICE, "double layer failed: %s", hipGetErrorString(e));
  return STB_OK;
}

// Double-layer potential with device inputs and output on the context stream.
static stb_status dl_core(stb_ctx* ctx, stb_mesh* mesh, const stb_quad_params& p, const double* d_v,
                          int64_t np, const double* d_pts, double* d_out) {
  stb_status s;
  if ((s = stb_ensure_gl(ctx, p.n_g))) return s;
  double* d_h = nullptr;
  int64_t* d_rowptr = nullptr;
  int32_t *d_cols = nullptr, *d_rowof = nullptr;
  auto cleanup = [&]() {
    dfree(d_h); dfree(d_rowptr); dfree(d_cols); dfree(d_rowof);
  };
  int64_t nnz = 0;
  s = stb_cull_points(ctx, mesh, p, np, d_pts, &d_rowptr, &d_cols, &d_rowof, &nnz);
  if (s) { cleanup(); return s; }
  if (dalloc(&d_h, (size_t)nnz * 4) != hipSuccess) {
    cleanup();
    return stb_fail(ctx, STB_E_NO_MEMORY, "double-layer candidates");
  }
  if ((s = dl_split(ctx, mesh, p, nnz, d_rowof, d_cols, d_pts, d_h))) { cleanup(); return s; }
  hipLaunchKernelGGL(k_dl_point_sum, dim3(grid_for(np * 64, 256)), dim3(256), 0, ctx->stream, np, d_rowptr,
                     d_cols, mesh->d_tet, d_v, d_h, d_out);
  hipError_t e = hipGetLastError();
  if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
  cleanup();
  ctx->work[0] = 0;
  ctx->work[1] = 0;
  ctx->work[2] = nnz;
  ctx->work[3] = 0;
  if (e != hipSuccess) return stb_fail(ctx, STB_E_DEVICE, "double layer failed: %s", hipGetErrorString(e));
  return STB_OK;
}

static stb_status dl_check(stb_ctx* ctx, const stb_mesh* mesh, const stb_quad_params* params,
                           stb_quad_params* p) {
  if (mesh->ctx != ctx) return stb_fail(ctx, STB_E_INVALID_ARG, "mesh belongs to another context");
  if (!mesh->d_nsign)
    return stb_fail(ctx, STB_E_INVALID_ARG, "the mesh has no outward normals (stb_mesh_set_normals)");
  *p = params ? *params : stb_default_params();
  return stb_check_params(ctx, p);
}

extern "C" {

stb_status stb_mesh_set_normals(stb_ctx* ctx, stb_mesh* mesh, const double* nrm) {
  if (!ctx || !mesh || !nrm) return stb_fail(ctx, STB_E_INVALID_ARG, "bad arguments");
  if (mesh->ctx != ctx) return stb_fail(ctx, STB_E_INVALID_ARG, "mesh belongs to another context");
  const int64_t nt = mesh->nt;
  if (nt == 0) return STB_OK;
  HIPCHK(ctx, hipSetDevice(ctx->device));
  double* d_n = nullptr;
  int32_t* d_st = nullptr;
  if (!mesh->d_nsign && dalloc(&mesh->d_nsign, (size_t)nt) != hipSuccess)
    return stb_fail(ctx, STB_E_NO_MEMORY, "normal signs");
  if (dalloc(&d_n, (size_t)nt * 3) != hipSuccess || dalloc(&d_st, (size_t)nt) != hipSuccess) {
    dfree(d_n); dfree(d_st);
    return stb_fail(ctx, STB_E_NO_MEMORY, "normals");
  }
  std::vector<int32_t> st((size_t)nt);
  hipError_t e = hipMemcpyAsync(d_n, nrm, sizeof(double) * 3 * nt, hipMemcpyHostToDevice, ctx->stream);
  if (e == hipSuccess) {
    hipLaunchKernelGGL(k_normal_sign, dim3(grid_for(nt, 256)), dim3(256), 0, ctx->stream, nt,
                       mesh->d_trial, d_n, mesh->d_nsign, d_st);
    e = hipGetLastError();
  }
  if (e == hipSuccess)
    e = hipMemcpyAsync(st.data(), d_st, sizeof(int32_t) * nt, hipMemcpyDeviceToHost, ctx->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
  dfree(d_n);
  dfree(d_st);
  if (e != hipSuccess) return stb_fail(ctx, STB_E_DEVICE, "normals failed: %s", hipGetErrorString(e));
  for (int64_t j = 0; j < nt; ++j)
    if (st[j]) {
      dfree(mesh->d_nsign);
      mesh->d_nsign = nullptr;
      return stb_fail(ctx, STB_E_INVALID_ARG,
                      "normal of panel %lld is not finite or not transversal to the panel's plane",
                      (long long)j);
    }
  return STB_OK;
}

stb_status stb_potential_D(stb_ctx* ctx, const stb_mesh* mesh_c, const stb_quad_params* params,
                           const double* v, int64_t np, const double* pts, double* out) {
  if (!ctx || !mesh_c || !v || (np > 0 && (!pts || !out)) || np < 0)
    return stb_fail(ctx, STB_E_INVALID_ARG, "bad arguments");
  stb_mesh* mesh = const_cast<stb_mesh*>(mesh_c);
  stb_quad_params p;
  stb_status s = dl_check(ctx, mesh, params, &p);
  if (s) return s;
  if (np == 0) return STB_OK;
  for (int64_t i = 0; i < 4 * np; ++i)
    if (!std::isfinite(pts[i]))
      return stb_fail(ctx, STB_E_INVALID_ARG, "non-finite point %lld", (long long)(i / 4));
  HIPCHK(ctx, hipSetDevice(ctx->device));
  double *d_pts = nullptr, *d_v = nullptr, *d_out = nullptr;
  if (dalloc(&d_pts, (size_t)np * 4) != hipSuccess || dalloc(&d_v, (size_t)mesh->nv) != hipSuccess ||
      dalloc(&d_out, (size_t)np) != hipSuccess) {
    dfree(d_pts); dfree(d_v); dfree(d_out);
    return stb_fail(ctx, STB_E_NO_MEMORY, "double-layer buffers");
  }
  hipError_t e = hipMemcpyAsync(d_pts, pts, sizeof(double) * 4 * np, hipMemcpyHostToDevice, ctx->stream);
  if (e == hipSuccess) e = hipMemcpyAsync(d_v, v, sizeof(double) * mesh->nv, hipMemcpyHostToDevice, ctx->stream);
  s = e == hipSuccess ? dl_core(ctx, mesh, p, d_v, np, d_pts, d_out)
                      : stb_fail(ctx, STB_E_DEVICE, "copy failed");
  if (s == STB_OK) {
    e = hipMemcpy(out, d_out, sizeof(double) * np, hipMemcpyDeviceToHost);
    if (e != hipSuccess) s = stb_fail(ctx, STB_E_DEVICE, "copy back failed: %s", hipGetErrorString(e));
  }
  dfree(d_pts); dfree(d_v); dfree(d_out);
  return s;
}

stb_status stb_potential_D_dev(stb_ctx* ctx, const stb_mesh* mesh_c, const stb_quad_params* params,
                               const double* v_dev, int64_t np, const double* pts_dev, double* out_dev,
                               void* stream) {
  if (!ctx || !mesh_c || !v_dev || (np > 0 && (!pts_dev || !out_dev)) || np < 0)
    return stb_fail(ctx, STB_E_INVALID_ARG, "bad arguments");
  stb_mesh* mesh = const_cast<stb_mesh*>(mesh_c);
  stb_quad_params p;
  stb_status s = dl_check(ctx, mesh, params, &p);
  if (s) return s;
  if (np == 0) return STB_OK;
  HIPCHK(ctx, hipSetDevice(ctx->device));
  if (stream) HIPCHK(ctx, hipStreamSynchronize((hipStream_t)stream));
  return dl_core(ctx, mesh, p, v_dev, np, pts_dev, out_dev);
}

// Face points per chunk of the energetic form (candidates are about 1e3-1e4
// per point: a chunk's candidate lists stay within a few GB).
constexpr int64_t kDlChunkPoints = 32768;

stb_status stb_dl_energetic(stb_ctx* ctx, const stb_mesh* mesh_c, const stb_quad_params* params,
                            const double* v, double c_id, double* out) {
  if (!ctx || !mesh_c || !v || !out || !std::isfinite(c_id))
    return stb_fail(ctx, STB_E_INVALID_ARG, "bad arguments");
  stb_mesh* mesh = const_cast<stb_mesh*>(mesh_c);
  stb_quad_params p;
  stb_status s = dl_check(ctx, mesh, params, &p);
  if (s) return s;
  const int64_t nt = mesh->nt;
  if (nt == 0) return STB_OK;
  HIPCHK(ctx, hipSetDevice(ctx->device));
  if ((s = stb_ensure_outer(ctx, mesh, p.m_q))) return s;
  if ((s = stb_ensure_faces(ctx, mesh, p.m_q))) return s;
  const int maxq = mesh->maxq, fq = p.m_q * p.m_q;
  const int64_t nf = mesh->nf;
  std::vector<int32_t> nq((size_t)std::max<int64_t>(nf, 1));
  std::vector<int64_t> off((size_t)nf + 1, 0);
  if (nf > 0) {
    HIPCHK(ctx, hipMemcpyAsync(nq.data(), mesh->d_fnq, sizeof(int32_t) * nf, hipMemcpyDeviceToHost,
                               ctx->stream));
    HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
  }
  for (int64_t f = 0; f < nf; ++f) off[f + 1] = off[f] + nq[f];
  double *d_v = nullptr, *d_out = nullptr, *d_pts = nullptr, *d_kv = nullptr, *d_kf = nullptr;
  int64_t* d_off = nullptr;
  const int64_t cap = std::max<int64_t>(kDlChunkPoints, fq);
  auto cleanup = [&]() { dfree(d_v); dfree(d_out); dfree(d_pts); dfree(d_kv); dfree(d_kf); dfree(d_off); };
  if (dalloc(&d_v, (size_t)mesh->nv) != hipSuccess || dalloc(&d_out, (size_t)nt) != hipSuccess ||
      dalloc(&d_pts, (size_t)cap * 4) != hipSuccess || dalloc(&d_kv, (size_t)cap) != hipSuccess ||
      dalloc(&d_kf, (size_t)std::max<int64_t>(nf, 1)) != hipSuccess ||
      dalloc(&d_off, (size_t)nf + 1) != hipSuccess) {
    cleanup();
    return stb_fail(ctx, STB_E_NO_MEMORY, "double-layer energetic buffers");
  }
  hipError_t e = hipMemcpyAsync(d_v, v, sizeof(double) * mesh->nv, hipMemcpyHostToDevice, ctx->stream);
  if (e == hipSuccess)
    e = hipMemcpyAsync(d_off, off.data(), sizeof(int64_t) * (nf + 1), hipMemcpyHostToDevice, ctx->stream);
  if (e != hipSuccess) { cleanup(); return stb_fail(ctx, STB_E_DEVICE, "copy failed"); }
  // K v at every distinct face point, in chunks of faces
  int64_t cand = 0;
  for (int64_t f0 = 0; f0 < nf;) {
    int64_t f1 = f0 + 1;
    while (f1 < nf && off[f1 + 1] - off[f0] <= cap) ++f1;
    const int64_t nfc = f1 - f0, np = off[f1] - off[f0];
    hipLaunchKernelGGL(k_pack_outer, dim3(grid_for(nfc * fq, 256)), dim3(256), 0, ctx->stream, f0, nfc, fq,
                       mesh->d_fpts, d_off, d_pts);
    if ((e = hipGetLastError()) != hipSuccess) break;
    if (np > 0) {
      s = dl_core(ctx, mesh, p, d_v, np, d_pts, d_kv);
      if (s) { cleanup(); return s; }
      cand += ctx->work[2];
    }
    hipLaunchKernelGGL(k_face_ksum, dim3(grid_for(nfc, 256)), dim3(256), 0, ctx->stream, f0, nfc, d_off, d_kv,
                       d_kf);
    if ((e = hipGetLastError()) != hipSuccess) break;
    f0 = f1;
  }
  if (e == hipSuccess) {
    hipLaunchKernelGGL(k_dl_outer_sum, dim3(grid_for(nt, 128)), dim3(128), 0, ctx->stream, nt, maxq,
                       mesh->d_trial, mesh->d_tet, d_v, mesh->d_opts, mesh->d_ow, mesh->d_onq, mesh->d_pf,
                       mesh->d_pw, d_kf, c_id, d_out);
    e = hipGetLastError();
  }
  if (e == hipSuccess) e = hipMemcpyAsync(out, d_out, sizeof(double) * nt, hipMemcpyDeviceToHost, ctx->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
  cleanup();
  ctx->work[2] = cand;
  if (e != hipSuccess) return stb_fail(ctx, STB_E_DEVICE, "double-layer energetic form failed: %s",
                                       hipGetErrorString(e));
  return STB_OK;
}

stb_status stb_inner_values_D(stb_ctx* ctx, const stb_mesh* mesh, const stb_quad_params* params,
                              int64_t k, const double* pts, const int32_t* panel, double* out) {
  if (!ctx || !mesh || k < 0 || (k > 0 && (!pts || !panel || !out)))
    return stb_fail(ctx, STB_E_INVALID_ARG, "bad arguments");
  stb_quad_params p;
  stb_status s = dl_check(ctx, mesh, params, &p);
  if (s) return s;
  for (int64_t m = 0; m < k; ++m)
    if (panel[m] < 0 || panel[m] >= mesh->nt)
      return stb_fail(ctx, STB_E_INVALID_ARG, "panel index %d out of range", panel[m]);
  if (k == 0) return STB_OK;
  HIPCHK(ctx, hipSetDevice(ctx->device));
  if ((s = stb_ensure_gl(ctx, p.n_g))) return s;
  double *d_pts = nullptr, *d_out = nullptr;
  int32_t* d_pan = nullptr;
  if (dalloc(&d_pts, (size_t)k * 4) != hipSuccess || dalloc(&d_out, (size_t)k * 4) != hipSuccess ||
      dalloc(&d_pan, (size_t)k) != hipSuccess) {
    dfree(d_pts); dfree(d_out); dfree(d_pan);
    return stb_fail(ctx, STB_E_NO_MEMORY, "buffers");
  }
  hipError_t e = hipMemcpyAsync(d_pts, pts, 32 * k, hipMemcpyHostToDevice, ctx->stream);
  if (e == hipSuccess) e = hipMemcpyAsync(d_pan, panel, 4 * k, hipMemcpyHostToDevice, ctx->stream);
  if (e == hipSuccess) {
    hipLaunchKernelGGL(k_dl_pairs, dim3(grid_for(k, 128)), dim3(128), 0, ctx->stream, k, mesh->d_trial,
                       mesh->d_fang, mesh->d_nsign, d_pts, d_pan, ctx->d_gl, p.n_g, d_out);
    e = hipGetLastError();
  }
  if (e == hipSuccess) e = hipMemcpyAsync(out, d_out, 32 * k, hipMemcpyDeviceToHost, ctx->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
  dfree(d_pts); dfree(d_out); dfree(d_pan);
  if (e != hipSuccess)
    return stb_fail(ctx, STB_E_DEVICE, "double-layer values failed: %s", hipGetErrorString(e));
  return STB_OK;
}

}  // extern "C"
