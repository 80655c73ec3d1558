// stb_faces.hip -- FP64 assembly through the outer points of shared faces.
//
// The outer rule of eq. int_bform puts its points on the faces of the test
// panel with nu_t != 0, and in a conforming space-time mesh each such face
// is shared by two panels (the slab above or below, or the neighbouring
// tetrahedron of the same prism), with outward time normals of opposite
// sign.  The inner integrals Vphi_j(x_{F,q}) at a face's points are
// therefore the same numbers for both panels.  Here the pair pipeline runs
// once per unique face F and trial panel j and returns
//   S(F, j) = sum_q Vphi_j(x_{F,q})          (fixed order in q),
// and every matrix entry is
//   A_ij = sum over the active faces F of panel i of w_{i,F} S(F, j),
//   w_{i,F} = -nu_{F,t} |F| / m_q^2          (nu outward for panel i),
// exactly +0.0 unless some point of one of its faces is lit (Sec. 3.3).
//
// Faces are identified by their sorted global vertex ids; a face's points
// are computed once from its vertices in that order (the set of sub-triangle
// centroids does not depend on the vertex order).  A face's candidate trial
// panels are those of the first panel row of the unit that has it.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <vector>

#include "stb_device.h"

using namespace stb;

#include "stb_internal.h"
#include "stb_pairs.h"

namespace {

// Outer weight of each face slot k of every panel (the face opposite local
// vertex k): -nu_t |F| / m^2 with the panel's outward normal, 0 for a
// vertical face.  Same arithmetic as the per-panel outer points.
__global__ void k_slot_weights(int64_t nt, const TrialRec* __restrict__ rec, int m,
                               double* __restrict__ pw) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nt) return;
  const TrialRec& R = rec[i];
  for (int k = 0; k < 4; ++k) {
    const int i0 = k == 0 ? 1 : 0, i1 = k <= 1 ? 2 : 1, i2 = k <= 2 ? 3 : 2;
    double u1[3], u2[3], tk[3];
    for (int c = 0; c < 3; ++c) {
      u1[c] = R.V[i1][c] - R.V[i0][c];
      u2[c] = R.V[i2][c] - R.V[i0][c];
      tk[c] = R.V[k][c] - R.V[i0][c];
    }
    const double N[3] = {u1[1] * u2[2] - u1[2] * u2[1], u1[2] * u2[0] - u1[0] * u2[2],
                         u1[0] * u2[1] - u1[1] * u2[0]};
    const double sg = dot3(N, tk) > 0.0 ? -1.0 : 1.0;
    const double nut_area = sg * N[0] * 0.5;
    pw[4 * i + k] = nut_area == 0.0 ? 0.0 : -nut_area / (double)(m * m);
  }
}

// Outer points of each face from its sorted vertices: centroids of the m^2
// congruent sub-triangles (Fig. int_tri_mid), in the per-panel order of
// (a, b, up); unit weights (the sums S are unweighted).
__global__ void k_face_points(int64_t nf, const double* __restrict__ vtx,
                              const int32_t* __restrict__ fv, int m, int maxq,
                              double* __restrict__ pts, double* __restrict__ ones,
                              int32_t* __restrict__ nq) {
  const int64_t f = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (f >= nf) return;
  const double* X0 = vtx + 4 * (int64_t)fv[3 * f];
  const double* X1 = vtx + 4 * (int64_t)fv[3 * f + 1];
  const double* X2 = vtx + 4 * (int64_t)fv[3 * f + 2];
  double* P = pts + f * maxq * 4;
  const double inv = 1.0 / m;
  int cnt = 0;
  for (int a = 0; a < m; ++a)
    for (int b = 0; a + b < m; ++b)
      for (int up = 0; up < 2; ++up) {
        double al, be;
        if (up == 0) {
          al = (a + 1.0 / 3.0) * inv;
          be = (b + 1.0 / 3.0) * inv;
        } else {
          if (a + b > m - 2) continue;
          al = (a + 2.0 / 3.0) * inv;
          be = (b + 2.0 / 3.0) * inv;
        }
        for (int c = 0; c < 4; ++c) P[4 * cnt + c] = X0[c] + al * (X1[c] - X0[c]) + be * (X2[c] - X0[c]);
        ones[f * maxq + cnt] = 1.0;
        ++cnt;
      }
  nq[f] = cnt;
}

// Candidates of each face: those of its primary panel row (the first row of
// the unit that has the face; the panel's apex box contains the face's
// points, so its cull is a superset of the face's).  -1: no such row.
__global__ void k_face_rows_count(int64_t nfu, const int32_t* __restrict__ prim,
                                  const int64_t* __restrict__ rowptr, int64_t* __restrict__ cnt) {
  const int64_t f = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (f >= nfu) return;
  const int32_t r = prim[f];
  cnt[f] = r < 0 ? 0 : rowptr[r + 1] - rowptr[r];
}

// One block per face row: copy the primary row's columns.
__global__ void k_face_rows_fill(int64_t nfu, const int32_t* __restrict__ prim,
                                 const int64_t* __restrict__ rowptr, const int32_t* __restrict__ cols,
                                 const int64_t* __restrict__ frowptr, int32_t* __restrict__ fcols,
                                 int32_t* __restrict__ frowof) {
  const int64_t f = blockIdx.x;
  if (f >= nfu) return;
  const int32_t r = prim[f];
  if (r < 0) return;
  const int64_t src = rowptr[r], n = rowptr[r + 1] - src, dst = frowptr[f];
  for (int64_t k = threadIdx.x; k < n; k += blockDim.x) {
    fcols[dst + k] = cols[src + k];
    frowof[dst + k] = (int32_t)f;
  }
}

__global__ void k_face_shift(int64_t n, const int32_t* __restrict__ in, int32_t add,
                             int32_t* __restrict__ out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = in[i] + add;
}

// Matrix entries of panel rows r0 .. r0 + nrow from the face sums, one lane
// per candidate: per active face slot of the row's panel (slot order), the
// candidate's column is looked up among the face's candidate columns
// (ascending).  A face's columns are those of the panel that owns the face
// row, a neighbour across the face whose cull found nearly the same columns,
// so the search starts at the candidate's own rank in its row and gallops
// from there before it bisects.
__global__ void k_face_combine(int64_t nnz, int64_t r0, const int32_t* __restrict__ rowof,
                               const int32_t* __restrict__ cols, const int32_t* __restrict__ pf,
                               const double* __restrict__ pw, int64_t f0, int64_t nfu,
                               const int64_t* __restrict__ frowptr,
                               const int32_t* __restrict__ fcols, const int32_t* __restrict__ prim,
                               const int64_t* __restrict__ rowptr, const double* __restrict__ S,
                               const uint8_t* __restrict__ lit, double* __restrict__ vals,
                               uint8_t* __restrict__ keep,
                               unsigned long long* __restrict__ causal) {
  unsigned long long n = 0;
  for (int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; c < nnz;
       c += (int64_t)gridDim.x * blockDim.x) {
    const int32_t li = rowof[c];
    const int64_t i = r0 + li;
    const int32_t j = cols[c];
    double acc = 0.0;
    bool any = false;
    for (int s = 0; s < 4; ++s) {
      const int64_t lf = (int64_t)pf[4 * i + s] - f0;
      if (pf[4 * i + s] < 0 || lf < 0 || lf >= nfu) continue;
      int64_t lo = frowptr[lf], hi = frowptr[lf + 1];
      if (prim[lf] == li) {
        lo += c - rowptr[li];   // the face's candidates are this row's, in order
      } else if (lo < hi) {
        // first position in [lo, hi) whose column is >= j: bracket it by
        // steps of 1, 2, 4, ... from the guess, then bisect the bracket
        const int64_t g = std::min(std::max(lo + (c - rowptr[li]), lo), hi - 1);
        int64_t a, b;   // the position lies in [a, b] (b = hi: none)
        if (fcols[g] < j) {
          a = g + 1;
          b = hi;
          for (int64_t step = 1;; step <<= 1) {
            const int64_t q = g + step;
            if (q >= hi) break;
            if (fcols[q] >= j) { b = q; break; }
            a = q + 1;
          }
        } else {
          a = lo;
          b = g;
          for (int64_t step = 1;; step <<= 1) {
            const int64_t q = g - step;
            if (q < lo) break;
            if (fcols[q] < j) { a = q + 1; break; }
            b = q;
          }
        }
        while (a < b) {
          const int64_t mid = a + ((b - a) >> 1);
          if (fcols[mid] < j) a = mid + 1;
          else b = mid;
        }
        lo = a;
      }
      if (lo < frowptr[lf + 1] && fcols[lo] == j) {
        acc += pw[4 * i + s] * S[lo];
        any = any || lit[lo] != 0;
      }
    }
    vals[c] = any ? acc : 0.0;
    if (keep) keep[c] = any ? 1 : 0;
    n += any ? 1ull : 0ull;
  }
  for (int off = 32; off > 0; off >>= 1) n += __shfl_down(n, off, 64);
  if ((threadIdx.x & 63) == 0 && n) atomicAdd(causal, n);
}

inline uint64_t hash3(const int32_t* k) {
  uint64_t h = (uint64_t)(uint32_t)k[0] * 0x9E3779B97F4A7C15ull;
  h ^= (uint64_t)(uint32_t)k[1] + 0x7F4A7C159E3779B9ull + (h << 6) + (h >> 2);
  h ^= (uint64_t)(uint32_t)k[2] + 0x94D049BB133111EBull + (h << 6) + (h >> 2);
  return h ^ (h >> 29);
}

}  // namespace

void stb_free_faces(stb_mesh* m) {
  dfree(m->d_fpts); dfree(m->d_fones); dfree(m->d_fnq);
  dfree(m->d_pf); dfree(m->d_pw);
  m->d_fpts = m->d_fones = nullptr;
  m->d_fnq = nullptr;
  m->d_pf = nullptr;
  m->d_pw = nullptr;
  m->h_pf.clear();
  m->nf = 0;
  m->face_mq = 0;
}

stb_status stb_ensure_faces(stb_ctx* ctx, stb_mesh* m, int mq) {
  if (m->face_mq == mq && m->d_pf) return STB_OK;
  stb_free_faces(m);
  const int64_t nt = m->nt;
  const int fq = mq * mq;
  std::vector<double> pw((size_t)nt * 4);
  std::vector<int32_t> tet((size_t)nt * 4);
  HIPCHK(ctx, dalloc(&m->d_pw, (size_t)nt * 4));
  if (nt > 0) {
    hipLaunchKernelGGL(k_slot_weights, dim3((unsigned)((nt + 127) / 128)), dim3(128), 0, ctx->stream, nt,
                       m->d_trial, mq, m->d_pw);
    HIPCHK(ctx, hipGetLastError());
    HIPCHK(ctx, hipMemcpyAsync(pw.data(), m->d_pw, sizeof(double) * 4 * nt, hipMemcpyDeviceToHost,
                               ctx->stream));
    HIPCHK(ctx, hipMemcpyAsync(tet.data(), m->d_tet, sizeof(int32_t) * 4 * nt, hipMemcpyDeviceToHost,
                               ctx->stream));
    HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
  }
  // unique active faces by sorted vertex ids, numbered in order of first
  // appearance (panel, slot); open addressing in a power-of-two table of at
  // least 8 entries per panel: at most half full (4 faces per panel, each
  // shared faces counted once; an eighth for conforming slab meshes)
  size_t tcap = 16;
  while (tcap < (size_t)nt * 8) tcap <<= 1;
  std::vector<int32_t> table(tcap, -1);
  const size_t tmask = tcap - 1;
  std::vector<int32_t> fv;
  fv.reserve((size_t)nt * 6);
  m->h_pf.assign((size_t)nt * 4, -1);
  for (int64_t i = 0; i < nt; ++i)
    for (int k = 0; k < 4; ++k) {
      if (pw[4 * i + k] == 0.0) continue;
      std::array<int32_t, 3> key;
      int c = 0;
      for (int v = 0; v < 4; ++v)
        if (v != k) key[c++] = tet[4 * i + v];
      std::sort(key.begin(), key.end());
      size_t h = (size_t)hash3(key.data()) & tmask;
      int32_t f;
      for (;;) {
        const int32_t t = table[h];
        if (t < 0) {
          f = (int32_t)(fv.size() / 3);
          table[h] = f;
          fv.insert(fv.end(), key.begin(), key.end());
          break;
        }
        if (fv[3 * (size_t)t] == key[0] && fv[3 * (size_t)t + 1] == key[1] && fv[3 * (size_t)t + 2] == key[2]) {
          f = t;
          break;
        }
        h = (h + 1) & tmask;
      }
      m->h_pf[4 * i + k] = f;
    }
  const int64_t nf = (int64_t)(fv.size() / 3);
  int32_t* d_fv = nullptr;
  HIPCHK(ctx, dalloc(&m->d_pf, (size_t)nt * 4));
  HIPCHK(ctx, dalloc(&m->d_fpts, (size_t)std::max<int64_t>(nf, 1) * fq * 4));
  HIPCHK(ctx, dalloc(&m->d_fones, (size_t)std::max<int64_t>(nf, 1) * fq));
  HIPCHK(ctx, dalloc(&m->d_fnq, (size_t)std::max<int64_t>(nf, 1)));
  HIPCHK(ctx, dalloc(&d_fv, (size_t)std::max<int64_t>(nf, 1) * 3));
  hipError_t e = hipSuccess;
  if (nt > 0)
    e = hipMemcpyAsync(m->d_pf, m->h_pf.data(), sizeof(int32_t) * 4 * nt, hipMemcpyHostToDevice, ctx->stream);
  if (e == hipSuccess && nf > 0)
    e = hipMemcpyAsync(d_fv, fv.data(), sizeof(int32_t) * 3 * nf, hipMemcpyHostToDevice, ctx->stream);
  if (e == hipSuccess && nf > 0) {
    hipLaunchKernelGGL(k_face_points, dim3((unsigned)((nf + 127) / 128)), dim3(128), 0, ctx->stream, nf,
                       m->d_vtx, d_fv, mq, fq, m->d_fpts, m->d_fones, m->d_fnq);
    e = hipGetLastError();
  }
  if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
  dfree(d_fv);
  if (e != hipSuccess) {
    stb_free_faces(m);
    return stb_fail(ctx, STB_E_DEVICE, "face table: %s", hipGetErrorString(e));
  }
  m->nf = nf;
  m->face_mq = mq;
  return STB_OK;
}

// Face range [f0, f1) referenced by panel rows [r0, r1) (host table).
static void face_range(const stb_mesh* m, int64_t r0, int64_t r1, int64_t* f0, int64_t* f1) {
  int64_t lo = m->nf, hi = 0;
  for (int64_t i = r0; i < r1; ++i)
    for (int k = 0; k < 4; ++k) {
      const int32_t f = m->h_pf[4 * i + k];
      if (f < 0) continue;
      lo = std::min<int64_t>(lo, f);
      hi = std::max<int64_t>(hi, (int64_t)f + 1);
    }
  if (hi <= lo) lo = hi = 0;
  *f0 = lo;
  *f1 = hi;
}

// Face CSR of a unit (faces f0 .. f1, local rows): each face's row is its
// primary panel's candidate row.
static stb_status face_rows(stb_ctx* ctx, const FaceUnit& fu, int64_t f0, int64_t f1,
                            int64_t** frowptr, int32_t** fcols, int32_t** frowof, int32_t** fprim,
                            int64_t* fnnz) {
  const int64_t nfu = f1 - f0;
  std::vector<int32_t> prim((size_t)std::max<int64_t>(nfu, 1), -1);
  for (int64_t i = fu.r0; i < fu.r1; ++i)
    for (int k = 0; k < 4; ++k) {
      const int32_t f = fu.mesh->h_pf[4 * i + k];
      if (f < 0 || f < f0 || f >= f1) continue;
      if (prim[(size_t)(f - f0)] < 0) prim[(size_t)(f - f0)] = (int32_t)(i - fu.r0);
    }
  int32_t* d_prim = nullptr;
  int64_t* d_cnt = nullptr;
  *fnnz = 0;
  HIPCHK(ctx, dalloc(frowptr, (size_t)nfu + 1));
  if (dalloc(&d_prim, (size_t)nfu) != hipSuccess || dalloc(&d_cnt, (size_t)nfu) != hipSuccess) {
    dfree(d_prim);
    dfree(d_cnt);
    return stb_fail(ctx, STB_E_NO_MEMORY, "face rows");
  }
  hipStream_t st = ctx->stream;
  hipError_t e = hipSuccess;
  if (nfu > 0) {
    e = hipMemcpyAsync(d_prim, prim.data(), sizeof(int32_t) * nfu, hipMemcpyHostToDevice, st);
    if (e == hipSuccess) {
      hipLaunchKernelGGL(k_face_rows_count, dim3((unsigned)((nfu + 255) / 256)), dim3(256), 0, st, nfu,
                         d_prim, fu.rowptr, d_cnt);
      e = hipGetLastError();
    }
  }
  stb_status s = e == hipSuccess ? stb_exclusive_scan(ctx, d_cnt, *frowptr, nfu, st)
                                 : stb_fail(ctx, STB_E_DEVICE, "face rows: %s", hipGetErrorString(e));
  if (s == STB_OK && hipMemcpy(fnnz, *frowptr + nfu, sizeof(int64_t), hipMemcpyDeviceToHost) != hipSuccess)
    s = stb_fail(ctx, STB_E_DEVICE, "face rows copy");
  if (s == STB_OK && (kalloc(ctx, fcols, (size_t)*fnnz) != hipSuccess ||
                      kalloc(ctx, frowof, (size_t)*fnnz) != hipSuccess))
    s = stb_fail(ctx, STB_E_NO_MEMORY, "face candidates (%lld)", (long long)*fnnz);
  if (s == STB_OK && nfu > 0) {
    hipLaunchKernelGGL(k_face_rows_fill, dim3((unsigned)nfu), dim3(256), 0, st, nfu, d_prim, fu.rowptr,
                       fu.cols, *frowptr, *fcols, *frowof);
    e = hipGetLastError();
    if (e != hipSuccess) s = stb_fail(ctx, STB_E_DEVICE, "face rows: %s", hipGetErrorString(e));
  }
  if (s == STB_OK) {
    e = hipStreamSynchronize(st);
    if (e != hipSuccess) s = stb_fail(ctx, STB_E_DEVICE, "face rows: %s", hipGetErrorString(e));
  }
  if (s == STB_OK) *fprim = d_prim;   // kept for the combine (primary rows index directly)
  else dfree(d_prim);
  dfree(d_cnt);
  return s;
}

stb_status stb_face_assemble(stb_ctx* ctx, const stb_quad_params& p, FaceUnit* units, int nunit,
                             unsigned long long work[4]) {
  for (int k = 0; k < 4; ++k) work[k] = 0;
  hipStream_t st = ctx->stream;
  const int fq = p.m_q * p.m_q;
  struct U {
    int64_t f0 = 0, f1 = 0, fnnz = 0, of = 0, op = 0, oc = 0;
    int64_t* frowptr = nullptr;
    int32_t *fcols = nullptr, *frowof = nullptr, *fprim = nullptr;
  };
  std::vector<U> u((size_t)nunit);
  TrialRec* trial_g = nullptr;
  FaceAng* fang_g = nullptr;
  double *apex_g = nullptr, *ones_g = nullptr, *S_g = nullptr;
  int32_t *apexn_g = nullptr, *rows_g = nullptr, *cols_g = nullptr;
  uint8_t* lit_g = nullptr;
  unsigned long long* d_causal = nullptr;
  auto cleanup = [&]() {
    for (auto& x : u) { dfree(x.frowptr); ctx_keep(ctx, x.fcols); ctx_keep(ctx, x.frowof); dfree(x.fprim); }
    dfree(trial_g); dfree(fang_g); dfree(apex_g); dfree(ones_g); ctx_keep(ctx, S_g);
    dfree(apexn_g); dfree(rows_g); dfree(cols_g); ctx_keep(ctx, lit_g); dfree(d_causal);
  };
  stb_status s = STB_OK;
  int64_t F = 0, C = 0, P = 0;
  for (int k = 0; k < nunit; ++k) {
    FaceUnit& fu = units[k];
    U& x = u[(size_t)k];
    if ((s = stb_ensure_faces(ctx, fu.mesh, p.m_q))) { cleanup(); return s; }
    face_range(fu.mesh, fu.r0, fu.r1, &x.f0, &x.f1);
    if ((s = face_rows(ctx, fu, x.f0, x.f1, &x.frowptr, &x.fcols, &x.frowof, &x.fprim, &x.fnnz))) {
      cleanup();
      return s;
    }
    x.of = F;
    x.oc = C;
    x.op = P;
    F += x.f1 - x.f0;
    C += x.fnnz;
    P += fu.mesh->nt;
  }
  if (F > 0x7fffffffll || P > 0x7fffffffll) {
    cleanup();
    return stb_fail(ctx, STB_E_INVALID_ARG, "face batch too large");
  }
  // one unit: the pipeline reads the mesh's arrays and the unit's face CSR
  // in place (its rows and columns need no offsets); several: staged into
  // concatenated arrays with per-unit offsets
  const bool direct = nunit == 1;
  bool ok = kalloc(ctx, &S_g, (size_t)std::max<int64_t>(C, 1)) == hipSuccess &&
            kalloc(ctx, &lit_g, (size_t)std::max<int64_t>(C, 1)) == hipSuccess &&
            dalloc(&d_causal, (size_t)nunit) == hipSuccess;
  if (ok && !direct)
    ok = dalloc(&trial_g, (size_t)std::max<int64_t>(P, 1)) == hipSuccess &&
         dalloc(&fang_g, (size_t)std::max<int64_t>(P, 1)) == hipSuccess &&
         dalloc(&apex_g, (size_t)std::max<int64_t>(F, 1) * fq * 4) == hipSuccess &&
         dalloc(&ones_g, (size_t)std::max<int64_t>(F, 1) * fq) == hipSuccess &&
         dalloc(&apexn_g, (size_t)std::max<int64_t>(F, 1)) == hipSuccess &&
         dalloc(&rows_g, (size_t)std::max<int64_t>(C, 1)) == hipSuccess &&
         dalloc(&cols_g, (size_t)std::max<int64_t>(C, 1)) == hipSuccess;
  if (!ok) {
    cleanup();
    return stb_fail(ctx, STB_E_NO_MEMORY, "face lists of %lld candidates do not fit", (long long)C);
  }
  hipError_t e = hipMemsetAsync(d_causal, 0, sizeof(unsigned long long) * nunit, st);
  for (int k = 0; k < nunit && e == hipSuccess && !direct; ++k) {
    const FaceUnit& fu = units[k];
    const U& x = u[(size_t)k];
    const stb_mesh* me = fu.mesh;
    const int64_t nfu = x.f1 - x.f0;
    e = hipMemcpyAsync(trial_g + x.op, me->d_trial, sizeof(TrialRec) * me->nt, hipMemcpyDeviceToDevice, st);
    if (e == hipSuccess)
      e = hipMemcpyAsync(fang_g + x.op, me->d_fang, sizeof(FaceAng) * me->nt, hipMemcpyDeviceToDevice, st);
    if (e == hipSuccess && nfu > 0)
      e = hipMemcpyAsync(apex_g + x.of * fq * 4, me->d_fpts + x.f0 * fq * 4, sizeof(double) * nfu * fq * 4,
                         hipMemcpyDeviceToDevice, st);
    if (e == hipSuccess && nfu > 0)
      e = hipMemcpyAsync(ones_g + x.of * fq, me->d_fones + x.f0 * fq, sizeof(double) * nfu * fq,
                         hipMemcpyDeviceToDevice, st);
    if (e == hipSuccess && nfu > 0)
      e = hipMemcpyAsync(apexn_g + x.of, me->d_fnq + x.f0, sizeof(int32_t) * nfu, hipMemcpyDeviceToDevice, st);
    if (e == hipSuccess && x.fnnz > 0) {
      const unsigned g = (unsigned)((x.fnnz + 255) / 256);
      hipLaunchKernelGGL(k_face_shift, dim3(g), dim3(256), 0, st, x.fnnz, x.frowof, (int32_t)x.of,
                         rows_g + x.oc);
      hipLaunchKernelGGL(k_face_shift, dim3(g), dim3(256), 0, st, x.fnnz, x.fcols, (int32_t)x.op,
                         cols_g + x.oc);
      e = hipGetLastError();
    }
  }
  if (e != hipSuccess) {
    cleanup();
    return stb_fail(ctx, STB_E_DEVICE, "face staging: %s", hipGetErrorString(e));
  }
  PairJob J;
  J.nnz = C;
  if (direct) {
    const stb_mesh* me = units[0].mesh;
    const int64_t f0 = u[0].f0;
    J.rows = u[0].frowof;
    J.cols = u[0].fcols;
    J.trial = me->d_trial;
    J.fang = me->d_fang;
    J.apex = me->d_fpts + f0 * fq * 4;
    J.apex_w = me->d_fones + f0 * fq;
    J.apex_n = me->d_fnq + f0;
  } else {
    J.rows = rows_g;
    J.cols = cols_g;
    J.trial = trial_g;
    J.fang = fang_g;
    J.apex = apex_g;
    J.apex_w = ones_g;
    J.apex_n = apexn_g;
  }
  J.maxq = fq;
  J.gl = ctx->d_gl;
  J.ng = p.n_g;
  J.mixed = false;
  J.eta_far = p.eta_far;
  J.out = S_g;
  J.lit_out = lit_g;
  s = stb_run_pairs(ctx, J, work);
  if (s) { cleanup(); return s; }
  for (int k = 0; k < nunit; ++k) {
    const FaceUnit& fu = units[k];
    const U& x = u[(size_t)k];
    if (fu.nnz <= 0) continue;
    const int64_t blocks = std::min<int64_t>((fu.nnz + 255) / 256, (int64_t)std::max(ctx->ncu, 1) * 32);
    hipLaunchKernelGGL(k_face_combine, dim3((unsigned)blocks), dim3(256), 0, st, fu.nnz, fu.r0, fu.rowof,
                       fu.cols, fu.mesh->d_pf, fu.mesh->d_pw, x.f0, x.f1 - x.f0, x.frowptr, x.fcols,
                       x.fprim, fu.rowptr, S_g + x.oc, lit_g + x.oc, fu.vals, fu.keep, d_causal + k);
    e = hipGetLastError();
    if (e != hipSuccess) break;
  }
  std::vector<unsigned long long> hc((size_t)nunit, 0);
  if (e == hipSuccess)
    e = hipMemcpyAsync(hc.data(), d_causal, sizeof(unsigned long long) * nunit, hipMemcpyDeviceToHost, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  cleanup();
  if (e != hipSuccess) return stb_fail(ctx, STB_E_DEVICE, "face combine: %s", hipGetErrorString(e));
  for (int k = 0; k < nunit; ++k) units[k].n_causal = (int64_t)hc[(size_t)k];
  return STB_OK;
}
