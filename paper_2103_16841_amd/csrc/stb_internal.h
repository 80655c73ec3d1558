// stb_internal.h -- handle layouts shared by the library's translation units.
#pragma once
#include <hip/hip_runtime.h>

#include <mutex>
#include <string>
#include <utility>
#include <vector>

#include "stb.h"
#include "stb_device.h"

// ---------------------------------------------------------------- handles
// Default resident blocks per CU of the pair pipeline's stages (kinds of
// stb_last_kernel_times): the lit test, breakpoint and empty-piece stages
// gain from 32 (more blocks to even out their per-item work), the Gauss
// nodes run best at 16 (measured on the 30,720-panel bench assembly).
constexpr int kDefaultPerCu[8] = {32, 32, 32, 16, 16, 16, 16, 16};

struct stb_ctx {
  int device = 0;
  hipStream_t stream = nullptr;
  hipEvent_t ev[5] = {};
  std::string err;
  double timings[4] = {0, 0, 0, 0};
  int64_t work[4] = {0, 0, 0, 0};   // last assembly: L evals, lit combos, apexes, pieces
  // last potential's lit search: (point, leaf) pairs kept by the tree, the
  // panels of those leaves, candidates after the per-panel bound test
  int64_t lit_search[3] = {0, 0, 0};
  struct PairWorkspace* ws = nullptr;   // pair pipeline lists (grown on demand)
  hipEvent_t kev[16] = {};              // pair pipeline: start/stop per kernel kind
  double kern_ms[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  int64_t kern_n[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  int64_t kern_units[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  // evaluations of L in the FP64 node launches (kind 4) by path: one-gap
  // recipe, two-gap recipe, full evaluation; [3] pieces found empty by the
  // ray test (no evaluation of L)
  int64_t path_counts[4] = {0, 0, 0, 0};
  // launch shapes of the pair pipeline's stages (autotuned or defaults):
  // threads per block and blocks per compute unit, indexed like kern_ms
  int tune_block[8] = {256, 256, 256, 256, 256, 256, 256, 256};
  int tune_per_cu[8] = {kDefaultPerCu[0], kDefaultPerCu[1], kDefaultPerCu[2], kDefaultPerCu[3],
                        kDefaultPerCu[4], kDefaultPerCu[5], kDefaultPerCu[6], kDefaultPerCu[7]};
  bool tuned = false;
  int ncu = 0;
  // caller's upper limits on the pair lists' lengths: candidates, lit
  // combos, pieces per chunk (0: none; stb_set_pair_lists)
  int64_t list_limit[3] = {0, 0, 0};
  // Gauss-Legendre nodes on [0,1] for the last n_g used (device copy)
  int gl_n = 0;
  double* d_gl = nullptr;   // [4 * kMaxNg]: x, w, 1/2 - s(x), s'(x) w
  // large temporaries of the assembly kept for later calls (ctx_alloc,
  // ctx_keep): free blocks and the blocks lent out, (address, bytes); the
  // free ones hold kept_bytes <= kKeptMaxBytes
  std::vector<std::pair<void*, size_t>> kept, lent;
  size_t kept_bytes = 0;
};

struct stb_mesh {
  stb_ctx* ctx = nullptr;
  int64_t nv = 0, nt = 0;
  double* d_vtx = nullptr;
  int32_t* d_tet = nullptr;
  stb::TrialRec* d_trial = nullptr;
  stb::FaceAng* d_fang = nullptr;   // [nt] polar form of the face normals
  // double layer: +1 where the outward normal of Gamma is the panel frame's
  // normal n, else -1 (set by stb_mesh_set_normals)
  double* d_nsign = nullptr;        // [nt]
  // L2 projection onto V_h^1: vertex -> (4 panel + local vertex), ascending
  // panel per vertex; 6 x the panels' 3-volumes (built on first use)
  int64_t* d_v2t_ptr = nullptr;     // [nv + 1]
  int64_t* d_v2t = nullptr;         // [4 nt]
  double* d_vol6 = nullptr;         // [nt]
  // outer points for one m_q (recomputed when m_q changes)
  int mq = 0;
  int maxq = 0;
  double* d_opts = nullptr;   // [nt][4*mq*mq][4]
  double* d_ow = nullptr;     // [nt][4*mq*mq]
  int32_t* d_onq = nullptr;   // [nt]
  stb::ApexBox* d_box = nullptr;   // [nt]
  // unique faces with nu_t != 0 and their outer points (for one m_q)
  int face_mq = 0;
  int64_t nf = 0;
  double* d_fpts = nullptr;        // [nf][mq*mq][4], from the sorted vertex ids
  double* d_fones = nullptr;       // [nf][mq*mq] unit weights
  int32_t* d_fnq = nullptr;        // [nf] points per face
  int32_t* d_pf = nullptr;         // [nt][4] face of each slot (-1: vertical), device
  double* d_pw = nullptr;          // [nt][4] outer weight of the slot for this panel
  std::vector<int32_t> h_pf;       // host copy of d_pf
  // cluster tree of the panels for the lit search of evaluation points
  // (stb_tree.hip; built on first use)
  struct stb_tree* tree = nullptr;
  std::mutex tree_mu;
};

struct stb_mat {
  stb_ctx* ctx = nullptr;
  int64_t n = 0, nnz = 0, n_causal = 0;
  int64_t ncols = 0;             // columns (0: n; a row block of a batch: the mesh's panels)
  int64_t* d_rowptr = nullptr;
  int32_t* d_cols = nullptr;
  double* d_vals = nullptr;
  float* d_vals32 = nullptr;     // lazily made for the 16-RHS product
  // host mirror for stb_mat_get / to_dense
  std::vector<int64_t> h_rowptr;
  std::vector<int32_t> h_cols;
  std::vector<double> h_vals;
  bool host_valid = false;
  // blocked copy for the 16-RHS matrix-core product: per 16-row block, the
  // union of its rows' columns in quads; FP32 values in MFMA A-operand order
  int64_t nblk = 0, nquad = 0;
  int64_t* d_bptr = nullptr;     // [nblk + 1] quad offsets
  int32_t* d_bcol = nullptr;     // [nquad * 4] column of each quad slot (-1 = pad)
  float* d_bval = nullptr;       // [nquad * 64]
};


stb_status stb_fail(stb_ctx* ctx, stb_status s, const char* fmt, ...);


#define HIPCHK(ctx, call)                                                                    \
  do {                                                                                       \
    hipError_t e_ = (call);                                                                  \
    if (e_ != hipSuccess)                                                                    \
      return stb_fail(ctx, e_ == hipErrorOutOfMemory ? STB_E_NO_MEMORY : STB_E_DEVICE,       \
                      "%s failed: %s", #call, hipGetErrorString(e_));                        \
  } while (0)

static inline int64_t mat_ncols(const stb_mat* M) { return M->ncols ? M->ncols : M->n; }

template <typename T>
static inline hipError_t dalloc(T** p, size_t count) {
  *p = nullptr;
  if (count == 0) count = 1;
  return hipMalloc((void**)p, count * sizeof(T));
}

static inline void dfree(void* p) {
  if (p) (void)hipFree(p);
}

// Large temporaries that the context keeps between calls (freeing a block
// of hundreds of MB takes about 0.3 ms): ctx_alloc lends a kept block of at
// least `bytes` and at most twice that, else allocates (dropping the kept
// blocks and retrying once when the device is full); ctx_keep takes a lent
// block back, or frees it when the kept blocks would exceed kKeptMaxBytes
// (a context that assembled a very large mesh does not go on holding its
// temporaries).  The blocks are freed with the context (ctx_drop_kept).
constexpr size_t kKeptMaxBytes = (size_t)8 << 30;
hipError_t ctx_alloc(stb_ctx* ctx, void** p, size_t bytes);
void ctx_keep(stb_ctx* ctx, void* p);
void ctx_drop_kept(stb_ctx* ctx);

template <typename T>
static inline hipError_t kalloc(stb_ctx* ctx, T** p, size_t count) {
  void* v = nullptr;
  const hipError_t e = ctx_alloc(ctx, &v, (count ? count : 1) * sizeof(T));
  *p = (T*)v;
  return e;
}

// Shared steps (stb_lib.hip).
stb_status stb_ensure_gl(stb_ctx* ctx, int ng);
stb_status stb_check_params(stb_ctx* ctx, const stb_quad_params* p);
stb_status stb_ensure_outer(stb_ctx* ctx, stb_mesh* m, int mq);
// Conservative cull of rows (apex boxes) against all panels of m into CSR
// candidates (rowptr, cols ascending per row) and the row of each candidate.
// lend: cols and rowof are blocks lent by ctx (ctx_alloc), to be handed
// back with ctx_keep.
stb_status stb_cull(stb_ctx* ctx, int64_t nrows, const stb::ApexBox* d_rows, const stb_mesh* m,
                    int64_t** d_rowptr, int32_t** d_cols, int32_t** d_rowof, int64_t* nnz,
                    bool lend = false);
stb_status stb_cull_count(stb_ctx* ctx, int64_t nrows, const stb::ApexBox* d_rows, const stb_mesh* m,
                          int64_t* nnz);
// Exclusive prefix of the per-row candidate counts (nrows + 1 entries, host).
stb_status stb_cull_rowptr(stb_ctx* ctx, int64_t nrows, const stb::ApexBox* d_rows, const stb_mesh* m,
                           int64_t* rowptr_host);
void stb_point_boxes(stb_ctx* ctx, int64_t np, const double* d_pts, stb::ApexBox* d_box);

// FP64 assembly through shared faces (stb_faces.hip).  A unit is a range
// of panel rows of one mesh with its candidate CSR (rows local to r0).
struct FaceUnit {
  stb_mesh* mesh = nullptr;
  int64_t r0 = 0, r1 = 0;
  const int64_t* rowptr = nullptr;  // [r1 - r0 + 1] candidate rows (local)
  const int32_t* rowof = nullptr;   // [nnz] local row of each candidate
  const int32_t* cols = nullptr;    // [nnz] trial panel (mesh-local)
  int64_t nnz = 0;
  double* vals = nullptr;           // [nnz] out
  uint8_t* keep = nullptr;          // optional [nnz] out: 1 where the pair is causal
  int64_t n_causal = 0;             // out
};
stb_status stb_ensure_faces(stb_ctx* ctx, stb_mesh* m, int mq);
void stb_free_faces(stb_mesh* m);
// One pass of the pair pipeline over the faces of all units; writes each
// unit's values and causal count; work as stb_run_pairs.
stb_status stb_face_assemble(stb_ctx* ctx, const stb_quad_params& p, FaceUnit* units, int nunit,
                             unsigned long long work[4]);

// Drops the stored candidates whose flag is 0 (non-causal pairs): M keeps
// exactly its causal entries, rows and column order unchanged, nnz =
// the number of flags set; the candidate store's columns and values go to
// ctx_keep (lent blocks back to the context, others freed).  Synchronises
// st.
stb_status stb_keep_causal(stb_ctx* ctx, stb_mat* M, const uint8_t* d_flag, hipStream_t st);

// Lit search of evaluation points by the cluster tree (stb_tree.hip): the
// tree for leaves of at most nmin panels is built on first use; candidates
// as by stb_cull (CSR per point, row of each candidate), nleaves (optional)
// the surviving (point, leaf) pairs.
stb_status stb_ensure_tree(stb_ctx* ctx, stb_mesh* m, int nmin);
stb_status stb_tree_cull(stb_ctx* ctx, stb_mesh* m, int nmin, int64_t np, const double* d_pts,
                         int64_t** d_rowptr, int32_t** d_cols, int32_t** d_rowof, int64_t* nnz,
                         int64_t* nleaves);
void stb_free_tree(stb_mesh* m);
// Candidates of evaluation points by the search p.lit_search selects (the
// cluster tree or the flat cull); records the surviving leaves in
// ctx->work.
stb_status stb_cull_points(stb_ctx* ctx, stb_mesh* m, const stb_quad_params& p, int64_t np,
                           const double* d_pts, int64_t** d_rowptr, int32_t** d_cols, int32_t** d_rowof,
                           int64_t* nnz);

// Frees the L2 projection's adjacency (stb_proj.hip).
void stb_free_projection(stb_mesh* m);

// Potential with device inputs/outputs on ctx's stream and workspace (the
// mesh may belong to another context of the same device).
stb_status stb_potential_core(stb_ctx* ctx, stb_mesh* mesh, const stb_quad_params& p,
                              const double* d_w, int64_t np, const double* d_pts, double* d_out);

// 16-RHS product (stb_apply.hip): builds the blocked copy on first use.
stb_status stb_build_blocked(stb_ctx* ctx, stb_mat* M, hipStream_t st);
stb_status stb_apply16_dev(stb_ctx* ctx, stb_mat* M, const double* w, double* y, hipStream_t st);
void stb_free_blocked(stb_mat* M);
// Looks up this device's address of the allocation-free product's scratch
// array (stb_apply.hip); called once per context with its device current.
stb_status stb_noalloc_setup(stb_ctx* ctx);
// Exclusive prefix sum of n counts into out[0..n] (device memory); syncs st.
stb_status stb_exclusive_scan(stb_ctx* ctx, const int64_t* in, int64_t* out, int64_t n, hipStream_t st);

// Device-wide exclusive prefix sum (stb_scan.hip): out[0] = 0, out[i + 1] =
// in[0] + ... + in[i] for i < n (n + 1 outputs), enqueued on st; tmp holds
// stb_scan_tmp_elems<T>(n) elements.  No allocation, no memset.
template <typename T>
int64_t stb_scan_tmp_elems(int64_t n);
template <typename T>
hipError_t stb_scan(const T* in, T* out, int64_t n, T* tmp, hipStream_t st);
