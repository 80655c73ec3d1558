// stb_batch.hip -- many meshes through one pass of the pair pipeline.
//
// The meshes of a batch differ in size (here 780 to 245,760 panels) and
// their pairs in cost; launching one pipeline per mesh would leave the GPU
// idle on every small mesh and pay one launch chain each.  Instead the
// candidate sets of all meshes of a wave are concatenated into one work list
// (panel records, outer points and candidate indices shifted by each mesh's
// panel offset) and the pipeline runs once over it: every kernel launch
// covers all meshes, and the flat lists even out the per-pair cost.  Waves
// group consecutive meshes whose stores fit the HBM budget; after a wave the
// optional per-mesh products Y_m = A_m W_m run and, unless the caller keeps
// the matrices, the stores are released.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <vector>

#include "stb_internal.h"
#include "stb_pairs.h"

using namespace stb;

extern "C" stb_status stb_autotune(stb_ctx* ctx, const stb_mesh* mesh, const stb_quad_params* params,
                                   int32_t* cfg16);

__global__ void k_shift_idx(int64_t n, const int32_t* __restrict__ in, int32_t add,
                            int32_t* __restrict__ out) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = in[i] + add;
}

__global__ void k_gather_stride(int64_t n, int64_t stride, const int32_t* __restrict__ rows,
                                const int32_t* __restrict__ cols, int32_t* __restrict__ rs,
                                int32_t* __restrict__ cs) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) {
    rs[i] = rows[i * stride];
    cs[i] = cols[i * stride];
  }
}

namespace {

// Device bytes per candidate held during a wave: the mesh's store (cols,
// vals), the candidate's row, the concatenated row/column/value copies, the
// causal flag, and at most as much again for the compacted store.
constexpr int64_t kBytesPerCand = 4 + 8 + 4 + 4 + 4 + 8 + 1 + 12;

struct WaveMesh {
  int idx;
  stb_mesh* mesh;
  int64_t r0 = 0, r1 = 0, nnz = 0;   // rows [r0, r1) of the mesh, their candidates
  stb_mat* M = nullptr;
  int32_t* rowof = nullptr;
  int64_t off_panel = 0, off_cand = 0;
};

void release(std::vector<WaveMesh>& w, bool keep) {
  for (auto& x : w) {
    dfree(x.rowof);
    x.rowof = nullptr;
    if (!keep && x.M) {
      stb_mat_destroy(x.M);
      x.M = nullptr;
    }
  }
}

}  // namespace

extern "C" stb_status stb_batch_assemble(stb_ctx* ctx, int32_t nmesh, stb_mesh* const* meshes,
                                         const stb_quad_params* params, int64_t hbm_budget,
                                         stb_mat** mats, int32_t nrhs, const double* const* W_dev,
                                         double* const* Y_dev, int64_t* n_causal) {
  if (!ctx || nmesh < 1 || !meshes) return stb_fail(ctx, STB_E_INVALID_ARG, "bad arguments");
  if (!mats && !(W_dev && Y_dev)) return stb_fail(ctx, STB_E_INVALID_ARG, "nothing to return");
  if ((W_dev || Y_dev) && (!W_dev || !Y_dev || nrhs < 1))
    return stb_fail(ctx, STB_E_INVALID_ARG, "W and Y need each other and nrhs >= 1");
  if (hbm_budget < 0) return stb_fail(ctx, STB_E_INVALID_ARG, "negative HBM budget");
  for (int k = 0; k < nmesh; ++k) {
    if (!meshes[k]) return stb_fail(ctx, STB_E_INVALID_ARG, "mesh %d is NULL", k);
    if (meshes[k]->ctx != ctx) return stb_fail(ctx, STB_E_INVALID_ARG, "mesh %d: other context", k);
    if (W_dev && (!W_dev[k] || !Y_dev[k])) return stb_fail(ctx, STB_E_INVALID_ARG, "W/Y %d NULL", k);
  }
  if (mats)
    for (int k = 0; k < nmesh; ++k) mats[k] = nullptr;
  stb_quad_params p = params ? *params : stb_default_params();
  stb_status s = stb_check_params(ctx, &p);
  if (s) return s;
  HIPCHK(ctx, hipSetDevice(ctx->device));
  if ((s = stb_ensure_gl(ctx, p.n_g))) return s;
  HIPCHK(ctx, hipEventRecord(ctx->ev[0], ctx->stream));
  for (int k = 0; k < nmesh; ++k)
    if ((s = stb_ensure_outer(ctx, meshes[k], p.m_q))) return s;
  const int maxq = meshes[0]->maxq;
  if (!ctx->tuned) {
    int big = 0;
    for (int k = 1; k < nmesh; ++k)
      if (meshes[k]->nt > meshes[big]->nt) big = k;
    if ((s = stb_autotune(ctx, meshes[big], &p, nullptr))) return s;
  }
  if (hbm_budget == 0) {
    size_t fr = 0, tot = 0;
    HIPCHK(ctx, hipMemGetInfo(&fr, &tot));
    hbm_budget = (int64_t)(0.4 * (double)fr);
  }
  // candidate counts per row, for the wave plan
  std::vector<std::vector<int64_t>> rp(nmesh);
  for (int k = 0; k < nmesh; ++k) {
    rp[k].resize((size_t)meshes[k]->nt + 1);
    if ((s = stb_cull_rowptr(ctx, meshes[k]->nt, meshes[k]->d_box, meshes[k], rp[k].data()))) return s;
  }
  HIPCHK(ctx, hipEventRecord(ctx->ev[1], ctx->stream));
  // units: whole meshes, or (without kept matrices) row blocks of a mesh
  // whose candidates alone exceed the budget
  struct Unit { int mesh; int64_t r0, r1, nnz, bytes; };
  std::vector<Unit> units;
  for (int k = 0; k < nmesh; ++k) {
    const int64_t nt = meshes[k]->nt;
    const int64_t fixed = nt * (int64_t)(sizeof(TrialRec) + 40 * maxq);
    if (mats) {
      units.push_back({k, 0, nt, rp[k][nt], rp[k][nt] * kBytesPerCand + fixed});
      continue;
    }
    int64_t r0 = 0;
    while (r0 < nt) {
      int64_t r1 = r0 + 1;
      // largest r1 whose block fits (binary search on the row prefix)
      int64_t lo = r0 + 1, hi = nt;
      while (lo < hi) {
        int64_t mid = (lo + hi + 1) / 2;
        if ((rp[k][mid] - rp[k][r0]) * kBytesPerCand + fixed <= hbm_budget) lo = mid; else hi = mid - 1;
      }
      r1 = lo;
      int64_t nz = rp[k][r1] - rp[k][r0];
      units.push_back({k, r0, r1, nz, nz * kBytesPerCand + fixed});
      r0 = r1;
    }
  }
  HIPCHK(ctx, hipEventRecord(ctx->ev[2], ctx->stream));
  unsigned long long work_tot[4] = {0, 0, 0, 0};
  double kms[8] = {0}, kunits[8] = {0};
  int64_t npath[4] = {0, 0, 0, 0};
  int64_t kn[8] = {0};
  std::vector<int64_t> causal(nmesh, 0);
  size_t u0 = 0;
  while (u0 < units.size()) {
    // wave: consecutive units within the budget (at least one); kept
    // matrices stay resident, so with mats the whole batch is one wave
    size_t u1 = u0;
    int64_t bytes = 0, panels = 0, cands = 0;
    while (u1 < units.size()) {
      if (u1 > u0 && bytes + units[u1].bytes > hbm_budget && !mats) break;
      bytes += units[u1].bytes;
      panels += meshes[units[u1].mesh]->nt;
      cands += units[u1].nnz;
      ++u1;
    }
    if (panels > (int64_t)INT32_MAX) return stb_fail(ctx, STB_E_INVALID_ARG, "batch wave exceeds 2^31 panels");
    std::vector<WaveMesh> w;
    for (size_t u = u0; u < u1; ++u) {
      WaveMesh x;
      x.idx = units[u].mesh;
      x.mesh = meshes[units[u].mesh];
      x.r0 = units[u].r0;
      x.r1 = units[u].r1;
      x.nnz = units[u].nnz;
      w.push_back(x);
    }
    TrialRec* trial_g = nullptr;
    FaceAng* fang_g = nullptr;
    uint8_t* keep_g = nullptr;   // [cands] 1 where the pair is causal
    double *apex_g = nullptr, *apexw_g = nullptr, *vals_g = nullptr;
    int32_t *apexn_g = nullptr, *rows_g = nullptr, *cols_g = nullptr;
    int64_t* seg_off = nullptr;
    unsigned long long* seg_causal = nullptr;
    auto cleanup = [&](bool keep) {
      dfree(trial_g); dfree(fang_g); dfree(apex_g); dfree(apexw_g); dfree(apexn_g); dfree(rows_g); dfree(cols_g);
      dfree(vals_g); dfree(seg_off); dfree(seg_causal); dfree(keep_g);
      release(w, keep);
    };
    // FP64: through the shared faces (stb_faces.hip), which stages its own
    // lists; mixed precision: the panels' outer points, staged here
    const bool faces = p.prec == STB_FP64;
    bool ok = dalloc(&keep_g, (size_t)std::max<int64_t>(cands, 1)) == hipSuccess;
    ok = ok && (faces || (dalloc(&trial_g, (size_t)panels) == hipSuccess &&
                        dalloc(&fang_g, (size_t)panels) == hipSuccess &&
                        dalloc(&apex_g, (size_t)panels * maxq * 4) == hipSuccess &&
                        dalloc(&apexw_g, (size_t)panels * maxq) == hipSuccess &&
                        dalloc(&apexn_g, (size_t)panels) == hipSuccess &&
                        dalloc(&rows_g, (size_t)cands) == hipSuccess &&
                        dalloc(&cols_g, (size_t)cands) == hipSuccess &&
                        dalloc(&vals_g, (size_t)cands) == hipSuccess &&
                        dalloc(&seg_off, w.size() + 1) == hipSuccess &&
                        dalloc(&seg_causal, w.size()) == hipSuccess));
    if (!ok) {
      cleanup(false);
      return stb_fail(ctx, STB_E_NO_MEMORY, "batch wave of %lld candidates does not fit", (long long)cands);
    }
    std::vector<int64_t> h_off(w.size() + 1, 0);
    int64_t op = 0, oc = 0;
    hipStream_t st = ctx->stream;
    for (size_t m = 0; m < w.size(); ++m) {
      WaveMesh& x = w[m];
      stb_mesh* me = x.mesh;
      const bool whole = x.r0 == 0 && x.r1 == me->nt;
      x.M = new stb_mat();
      x.M->ctx = ctx;
      x.M->n = x.r1 - x.r0;
      x.M->ncols = whole ? 0 : me->nt;
      int64_t nz = 0;
      s = stb_cull(ctx, x.r1 - x.r0, me->d_box + x.r0, me, &x.M->d_rowptr, &x.M->d_cols, &x.rowof, &nz);
      if (s == STB_OK && nz != x.nnz) s = stb_fail(ctx, STB_E_INTERNAL, "cull count changed");
      if (s == STB_OK && dalloc(&x.M->d_vals, (size_t)nz) != hipSuccess)
        s = stb_fail(ctx, STB_E_NO_MEMORY, "store of mesh %d", x.idx);
      if (s) { cleanup(false); return s; }
      x.M->nnz = nz;
      x.off_panel = op;
      x.off_cand = oc;
      h_off[m] = oc;
      if (faces) {
        op += me->nt;
        oc += nz;
        continue;
      }
      hipError_t e = hipMemcpyAsync(trial_g + op, me->d_trial, sizeof(TrialRec) * me->nt,
                                    hipMemcpyDeviceToDevice, st);
      if (e == hipSuccess)
        e = hipMemcpyAsync(fang_g + op, me->d_fang, sizeof(FaceAng) * me->nt, hipMemcpyDeviceToDevice, st);
      if (e == hipSuccess)
        e = hipMemcpyAsync(apex_g + op * maxq * 4, me->d_opts, sizeof(double) * me->nt * maxq * 4,
                           hipMemcpyDeviceToDevice, st);
      if (e == hipSuccess)
        e = hipMemcpyAsync(apexw_g + op * maxq, me->d_ow, sizeof(double) * me->nt * maxq,
                           hipMemcpyDeviceToDevice, st);
      if (e == hipSuccess)
        e = hipMemcpyAsync(apexn_g + op, me->d_onq, sizeof(int32_t) * me->nt, hipMemcpyDeviceToDevice, st);
      if (e == hipSuccess && nz > 0) {
        unsigned g = (unsigned)((nz + 255) / 256);
        hipLaunchKernelGGL(k_shift_idx, dim3(g), dim3(256), 0, st, nz, x.rowof, (int32_t)(op + x.r0),
                           rows_g + oc);
        hipLaunchKernelGGL(k_shift_idx, dim3(g), dim3(256), 0, st, nz, x.M->d_cols, (int32_t)op,
                           cols_g + oc);
        e = hipGetLastError();
      }
      if (e != hipSuccess) {
        cleanup(false);
        return stb_fail(ctx, STB_E_DEVICE, "batch staging: %s", hipGetErrorString(e));
      }
      op += me->nt;
      oc += nz;
    }
    h_off[w.size()] = oc;
    if (faces) {
      std::vector<FaceUnit> fu(w.size());
      for (size_t m = 0; m < w.size(); ++m) {
        fu[m].mesh = w[m].mesh;
        fu[m].r0 = w[m].r0;
        fu[m].r1 = w[m].r1;
        fu[m].rowptr = w[m].M->d_rowptr;
        fu[m].rowof = w[m].rowof;
        fu[m].cols = w[m].M->d_cols;
        fu[m].nnz = w[m].M->nnz;
        fu[m].vals = w[m].M->d_vals;
        fu[m].keep = keep_g + w[m].off_cand;
      }
      unsigned long long work[4];
      s = stb_face_assemble(ctx, p, fu.data(), (int)fu.size(), work);
      if (s) { cleanup(false); return s; }
      for (int q = 0; q < 4; ++q) work_tot[q] += work[q];
      for (int q = 0; q < 8; ++q) { kms[q] += ctx->kern_ms[q]; kn[q] += ctx->kern_n[q]; kunits[q] += (double)ctx->kern_units[q]; }
      for (int q = 0; q < 4; ++q) npath[q] += ctx->path_counts[q];
      for (size_t m = 0; m < w.size(); ++m) {
        w[m].M->n_causal = fu[m].n_causal;
        causal[(size_t)w[m].idx] += fu[m].n_causal;
      }
    } else {
    HIPCHK(ctx, hipMemcpyAsync(seg_off, h_off.data(), 8 * h_off.size(), hipMemcpyHostToDevice, st));
    HIPCHK(ctx, hipMemsetAsync(seg_causal, 0, 8 * w.size(), st));
    PairJob J;
    J.nnz = oc;
    J.rows = rows_g;
    J.cols = cols_g;
    J.trial = trial_g;
    J.fang = fang_g;
    J.apex = apex_g;
    J.apex_w = apexw_g;
    J.apex_n = apexn_g;
    J.maxq = maxq;
    J.gl = ctx->d_gl;
    J.ng = p.n_g;
    J.mixed = p.prec == STB_MIXED;
    J.eta_far = p.eta_far;
    J.out = vals_g;
    J.lit_out = keep_g;
    J.nseg = (int)w.size();
    J.seg_off = seg_off;
    J.seg_causal = seg_causal;
    unsigned long long work[4];
    s = stb_run_pairs(ctx, J, work);
    if (s) { cleanup(false); return s; }
    for (int q = 0; q < 4; ++q) work_tot[q] += work[q];
    for (int q = 0; q < 8; ++q) { kms[q] += ctx->kern_ms[q]; kn[q] += ctx->kern_n[q]; kunits[q] += (double)ctx->kern_units[q]; }
    for (int q = 0; q < 4; ++q) npath[q] += ctx->path_counts[q];
    std::vector<unsigned long long> h_causal(w.size());
    HIPCHK(ctx, hipMemcpyAsync(h_causal.data(), seg_causal, 8 * w.size(), hipMemcpyDeviceToHost, st));
    for (size_t m = 0; m < w.size(); ++m) {
      WaveMesh& x = w[m];
      if (x.M->nnz)
        HIPCHK(ctx, hipMemcpyAsync(x.M->d_vals, vals_g + x.off_cand, 8 * x.M->nnz,
                                   hipMemcpyDeviceToDevice, st));
    }
    HIPCHK(ctx, hipStreamSynchronize(st));
    for (size_t m = 0; m < w.size(); ++m) {
      w[m].M->n_causal = (int64_t)h_causal[m];
      causal[(size_t)w[m].idx] += (int64_t)h_causal[m];
    }
    }
    // each store keeps its causal entries only
    for (size_t m = 0; m < w.size(); ++m) {
      s = stb_keep_causal(ctx, w[m].M, keep_g + w[m].off_cand, st);
      if (s) { cleanup(false); return s; }
    }
    // products of the wave's row blocks, then release (or hand over) the stores
    for (size_t m = 0; m < w.size() && W_dev; ++m) {
      WaveMesh& x = w[m];
      s = stb_apply_dev(ctx, x.M, nrhs, W_dev[x.idx], Y_dev[x.idx] + x.r0 * nrhs, nullptr);
      if (s) { cleanup(false); return s; }
    }
    if (W_dev) HIPCHK(ctx, hipStreamSynchronize(st));
    if (mats)
      for (auto& x : w) mats[x.idx] = x.M;
    cleanup(mats != nullptr);
    u0 = u1;
  }
  if (n_causal)
    for (int k = 0; k < nmesh; ++k) n_causal[k] = causal[(size_t)k];
  HIPCHK(ctx, hipEventRecord(ctx->ev[3], ctx->stream));
  HIPCHK(ctx, hipEventSynchronize(ctx->ev[3]));
  for (int q = 0; q < 4; ++q) ctx->work[q] = (int64_t)work_tot[q];
  for (int q = 0; q < 4; ++q) ctx->path_counts[q] = npath[q];
  for (int q = 0; q < 8; ++q) {
    ctx->kern_ms[q] = kms[q];
    ctx->kern_n[q] = kn[q];
    ctx->kern_units[q] = (int64_t)kunits[q];
  }
  float t01 = 0, t12 = 0, t23 = 0, t03 = 0;
  (void)hipEventElapsedTime(&t01, ctx->ev[0], ctx->ev[1]);
  (void)hipEventElapsedTime(&t12, ctx->ev[1], ctx->ev[2]);
  (void)hipEventElapsedTime(&t23, ctx->ev[2], ctx->ev[3]);
  (void)hipEventElapsedTime(&t03, ctx->ev[0], ctx->ev[3]);
  ctx->timings[0] = t01; ctx->timings[1] = t12; ctx->timings[2] = t23; ctx->timings[3] = t03;
  return STB_OK;
}

// Autotune the pair pipeline on a strided sample (about 2^22 candidates) of
// one mesh's assembly.
extern "C" stb_status stb_autotune(stb_ctx* ctx, const stb_mesh* mesh_c,
                                   const stb_quad_params* params, int32_t* cfg16) {
  if (!ctx || !mesh_c) return stb_fail(ctx, STB_E_INVALID_ARG, "NULL argument");
  stb_mesh* mesh = const_cast<stb_mesh*>(mesh_c);
  if (mesh->ctx != ctx) return stb_fail(ctx, STB_E_INVALID_ARG, "mesh belongs to another context");
  stb_quad_params p = params ? *params : stb_default_params();
  stb_status s = stb_check_params(ctx, &p);
  if (s) return s;
  HIPCHK(ctx, hipSetDevice(ctx->device));
  if ((s = stb_ensure_gl(ctx, p.n_g))) return s;
  if ((s = stb_ensure_outer(ctx, mesh, p.m_q))) return s;
  int64_t *rowptr = nullptr;
  int32_t *cols = nullptr, *rowof = nullptr, *rs = nullptr, *cs = nullptr;
  double* out = nullptr;
  int64_t nnz = 0;
  auto cleanup = [&]() { dfree(rowptr); dfree(cols); dfree(rowof); dfree(rs); dfree(cs); dfree(out); };
  s = stb_cull(ctx, mesh->nt, mesh->d_box, mesh, &rowptr, &cols, &rowof, &nnz);
  if (s) { cleanup(); return s; }
  const int64_t want = (int64_t)1 << 22;
  const int64_t stride = std::max<int64_t>(1, nnz / want);
  const int64_t n = nnz / stride;
  if (n > 0) {
    if (dalloc(&rs, (size_t)n) != hipSuccess || dalloc(&cs, (size_t)n) != hipSuccess ||
        dalloc(&out, (size_t)n) != hipSuccess) {
      cleanup();
      return stb_fail(ctx, STB_E_NO_MEMORY, "autotune sample");
    }
    hipLaunchKernelGGL(k_gather_stride, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, ctx->stream, n,
                       stride, rowof, cols, rs, cs);
    PairJob J;
    J.nnz = n;
    J.rows = rs;
    J.cols = cs;
    J.trial = mesh->d_trial;
    J.fang = mesh->d_fang;
    J.apex = mesh->d_opts;
    J.apex_w = mesh->d_ow;
    J.apex_n = mesh->d_onq;
    J.maxq = mesh->maxq;
    J.gl = ctx->d_gl;
    J.ng = p.n_g;
    J.mixed = p.prec == STB_MIXED;
    J.eta_far = p.eta_far;
    J.out = out;
    s = stb_tune_pairs(ctx, J);
  }
  cleanup();
  if (s) return s;
  ctx->tuned = true;
  if (cfg16)
    for (int k = 0; k < 8; ++k) {
      cfg16[k] = ctx->tune_block[k];
      cfg16[8 + k] = ctx->tune_per_cu[k];
    }
  return STB_OK;
}

extern "C" stb_status stb_set_tuning(stb_ctx* ctx, const int32_t* cfg16) {
  if (!ctx) return stb_fail(nullptr, STB_E_INVALID_ARG, "NULL context");
  for (int k = 0; k < 8; ++k) {
    int b = cfg16 ? cfg16[k] : 256, pc = cfg16 ? cfg16[8 + k] : kDefaultPerCu[k];
    if (b < 64 || b > 256 || (b & 63) || pc < 1 || pc > 64)
      return stb_fail(ctx, STB_E_INVALID_ARG, "stage %d: block %d / blocks per CU %d out of range", k, b, pc);
  }
  for (int k = 0; k < 8; ++k) {
    ctx->tune_block[k] = cfg16 ? cfg16[k] : 256;
    ctx->tune_per_cu[k] = cfg16 ? cfg16[8 + k] : kDefaultPerCu[k];
  }
  ctx->tuned = cfg16 != nullptr;
  return STB_OK;
}
