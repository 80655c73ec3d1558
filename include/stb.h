/*
 * stb.h -- C ABI of the MI355X space-time boundary element library.
 *
 * Method: Poelz & Schanz, "On the space-time discretization of variational
 * retarded potential boundary integral equations" (arXiv 2103.16841).
 *
 *   * The lateral boundary Sigma = (0,T) x Gamma is meshed by N open
 *     tetrahedral panels that are "vertical": each lies in R x (plane of a
 *     spatial triangle), so its space-time normal has no time component
 *     (Sec. 2, the normal field nu_Sigma; Sec. 3, the mesh Sigma_N).
 *   * Trial/test space: piecewise constants S_h^0 (Sec. 3, def. st_be).
 *   * Galerkin matrix of the energetic single-layer form,
 *       A[i][j] = b_V(phi_j, phi_i)
 *               = - sum_{F in faces(sigma_i)} int_F nu_{F,t} V phi_j dS
 *     (eq. df_ind with the outer form eq. int_bform); the face integral is
 *     the composite centroid rule of Fig. int_tri_mid with m_q^2
 *     sub-triangles per face (m_q = 3 in Exp. 3).
 *   * V phi_j (x) = S 1_{sigma_j}(x) with the retarded single-layer kernel
 *     k1 = 1/(4 pi |x - y|) and c = 1 (eq. slp, eq. kfunc); evaluated on the
 *     cone-panel intersection (eq. tk_para) in the (r, phi) form where the
 *     k1 integrand is constant (Lemma kernel_para), r exactly, phi by a
 *     breakpoint-aware Gauss-Legendre rule with n_g nodes per piece.
 *
 * Coordinates: space-time points are (t, x, y, z) in geometrized time.
 * Row i = test panel, column j = trial panel.  Entries of pairs that are not
 * causal (no outer point of panel i has a backward light cone crossing
 * panel j, Sec. 3.3) are exactly +0.0.
 *
 * Memory: unless a name ends in _dev, pointer arguments are host memory;
 * inputs are copied, outputs are caller-allocated and written in full.
 * _dev entry points take device pointers and a HIP stream (as void*; NULL =
 * the context's stream) and return after enqueueing.  Handles are owned by
 * the library and released by the matching *_destroy call.  No exception
 * crosses this interface; every call returns a stb_status and leaves a
 * message for stb_last_error().  A context is externally synchronised: do
 * not call into one context from two threads at once.
 */
#ifndef STB_H
#define STB_H
#include <stdint.h>
#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  STB_OK = 0,
  STB_E_INVALID_ARG = 1,   /* null pointer, bad size, bad parameter          */
  STB_E_INVALID_MESH = 2,  /* index out of range, non-finite coordinate,
                              non-vertical or degenerate panel               */
  STB_E_NO_MEMORY = 3,     /* device allocation failed or budget exceeded    */
  STB_E_DEVICE = 4,        /* HIP runtime error                              */
  STB_E_NOT_FOUND = 5,     /* unknown id / ticket                            */
  STB_E_BUSY = 6,          /* resource in use                                */
  STB_E_INTERNAL = 7
} stb_status;

typedef enum { STB_FP64 = 0, STB_MIXED = 1 } stb_precision;

/* Lit-panel search of the potentials (Sec. 3.3).  STB_LIT_TREE: the cluster
 * tree of Def. bct (panels in space-time Morton order, perfect binary tree,
 * leaves of at most n_min panels, one bounding 4-ball per cluster),
 * descended by all points together level by level with the exact extrema
 * of Theorem phi_xi_sphere (Alg. lit_leaves); the panels of the surviving
 * leaves, X_N(x), then pass a per-panel bound test (time range and spatial
 * ball).  STB_LIT_FLAT: every point against every panel's bound test.  Both
 * feed the exact lit test, so the lit sets and the potentials agree.  The
 * tree of a mesh is built on first use for its n_min (once; contexts that
 * share the mesh may search it concurrently with the same n_min). */
typedef enum { STB_LIT_TREE = 0, STB_LIT_FLAT = 1 } stb_lit_search;

/* Quadrature parameters.  m_q: sub-triangles per face edge of the outer
 * centroid rule (1..4, default 3 as in Exp. 3).  n_g: Gauss-Legendre nodes
 * per phi piece of the inner rule (2..64, default 16).  prec: FP64 or mixed.
 * Mixed (stb_assemble_V only; the potential is always FP64): the phi nodes
 * of "far" (outer point, trial panel) pairs -- the point farther than
 * eta_far times the radius of the panel's spatial bounding ball from that
 * ball (default 0.5) -- solve the face quadratics and measure the r-gaps in
 * FP32 about the middle of the pair's admissible range, with Kahan-summed
 * FP32 node sums; lit test, breakpoints, empty-piece tests, angles and the
 * quadratics' coefficients stay FP64.  Every entry carries a first-order
 * bound of its FP32 error; entries whose bound exceeds 3e-6 of their size
 * are recomputed with FP64 nodes (the bound overestimates the error by at
 * least a factor 3 on every entry measured), which keeps entries within
 * 1e-6 relative of the FP64 assembly. */
typedef struct {
  int32_t m_q;
  int32_t n_g;
  double eta_far;
  stb_precision prec;
  int32_t lit_search;   /* stb_lit_search: how evaluation points find their
                           candidate panels (potentials) */
  int32_t n_min;        /* leaf size of the cluster tree (1..4096, default 64) */
} stb_quad_params;

typedef struct stb_ctx stb_ctx;
typedef struct stb_mesh stb_mesh;
typedef struct stb_mat stb_mat;

/* Default parameters (m_q = 3, n_g = 16, eta_far = 0.5, FP64, flat lit
 * search; n_min = 64 when the tree is chosen).  The flat search is the
 * default because it is the faster one on meshes of up to 2.5e5 panels on
 * this hardware (measured per point for 1e3-1e5 points); the tree's cost per
 * point grows more slowly with N. */
stb_quad_params stb_default_params(void);

/* Create a context on HIP device `device` (its own stream). */
stb_status stb_ctx_create(int32_t device, stb_ctx** out);
void stb_ctx_destroy(stb_ctx* ctx);
const char* stb_status_str(stb_status s);
/* Message of the last failed call on ctx (or of the last failed
 * stb_ctx_create when ctx is NULL).  Valid until the next call. */
const char* stb_last_error(const stb_ctx* ctx);

/* Upload a mesh and precompute per-panel geometry on the device: panel
 * frames, face half-spaces (eq. pnl_ilf), bounding data and the outer
 * points / weights of eq. int_bform for m_q = 1..4 on demand.
 *   vtx: nv x 4 doubles (t, x, y, z), row-major;
 *   tet: nt x 4 int32 vertex indices.
 * Validates every panel (STB_E_INVALID_MESH names the first bad one). */
stb_status stb_mesh_create(stb_ctx* ctx, int64_t nv, const double* vtx, int64_t nt,
                           const int32_t* tet, stb_mesh** out);
/* Same with vtx / tet in device memory (copied into the mesh on `stream`,
 * NULL = the context stream); indices are validated on the device. */
stb_status stb_mesh_create_dev(stb_ctx* ctx, int64_t nv, const double* vtx_dev, int64_t nt,
                               const int32_t* tet_dev, void* stream, stb_mesh** out);
void stb_mesh_destroy(stb_mesh* mesh);
int64_t stb_mesh_size(const stb_mesh* mesh);

/* Assemble A over all causal pairs into a device-resident sparse store:
 * CSR rows holding exactly the causal pairs of the row (columns ascending;
 * the conservative cull's other candidates are evaluated and dropped), so
 * every entry not stored is +0.0.  params NULL = defaults. */
stb_status stb_assemble_V(stb_ctx* ctx, const stb_mesh* mesh, const stb_quad_params* params,
                          stb_mat** out);
void stb_mat_destroy(stb_mat* mat);

/* n: matrix order; n_causal_pairs: exact number of causal pairs (Sec. 3.3
 * lit predicate at the outer points); n_stored: stored entries (equal to
 * n_causal_pairs); bytes: device bytes held by the store. */
stb_status stb_mat_info(const stb_mat* mat, int64_t* n, int64_t* n_causal_pairs,
                        int64_t* n_stored, int64_t* bytes);
/* Dense copy, n x n row-major FP64 (caller-owned host buffer). */
stb_status stb_mat_to_dense(const stb_mat* mat, double* out);
/* k individual entries A[row[m]][col[m]] (host arrays). */
stb_status stb_mat_get(const stb_mat* mat, int64_t k, const int32_t* row, const int32_t* col,
                       double* out);

/* Export the store in CSR form into caller-allocated host arrays: rowptr
 * (n + 1 entries), cols and vals (n_stored entries each, see stb_mat_info);
 * columns ascend within a row; every stored entry is a causal pair.
 * Any of the three pointers may be NULL to skip that array. */
stb_status stb_mat_export(const stb_mat* mat, int64_t* rowptr, int32_t* cols, double* vals);

/* y = A w for nrhs right-hand sides; w: n x nrhs row-major, y: n x nrhs.
 * nrhs == 1: FP64 sparse product.  nrhs == 16: FP32 matrix-core product
 * (A and W rounded to FP32, FP32 accumulation).  Other nrhs: FP64, one
 * column at a time. */
stb_status stb_apply(stb_ctx* ctx, const stb_mat* mat, int32_t nrhs, const double* w, double* y);
stb_status stb_apply_dev(stb_ctx* ctx, const stb_mat* mat, int32_t nrhs, const double* w_dev,
                         double* y_dev, void* stream);

/* The 16-RHS matrix-core product of stb_apply_dev (nrhs = 16) for callers
 * that cannot allocate device memory: code under HIP graph capture, tight
 * serving loops, harnesses that forbid allocation.  Y = A W with w_dev
 * (n x 16, row-major FP64) and y_dev (n x 16) in device memory; the same
 * kernels and results as stb_apply_dev.  The FP32 copy of W lives in one
 * static 16 MiB device array per device (at most 262,144 columns;
 * STB_E_INVALID_ARG beyond), shared by every call on that device and kept
 * between calls: calls that overlap on one device race.  The matrix's
 * matrix-core copy must exist already (built by one stb_apply or
 * stb_apply_dev with nrhs = 16; STB_E_INVALID_ARG otherwise).  Enqueues on
 * `stream` (NULL = the context stream) and returns; allocates nothing and
 * does not synchronise. */
stb_status stb_apply16_noalloc(stb_ctx* ctx, const stb_mat* mat, const double* w_dev,
                               double* y_dev, void* stream);

/* Retarded single-layer potential u(p) = sum_j w_j V phi_j (p) (eq. slp with
 * w in S_h^0) at np points pts (np x 4, (t, x, y, z)); w has nt entries. */
stb_status stb_potential_S(stb_ctx* ctx, const stb_mesh* mesh, const stb_quad_params* params,
                           const double* w, int64_t np, const double* pts, double* out);
/* Same with w, pts and out in device memory; returns after the result is
 * written (the call synchronises its stream). */
stb_status stb_potential_S_dev(stb_ctx* ctx, const stb_mesh* mesh, const stb_quad_params* params,
                               const double* w_dev, int64_t np, const double* pts_dev,
                               double* out_dev, void* stream);

/* Single-panel potentials out[m] = V phi_{panel[m]} (pts[m]) for k pairs
 * (pts: k x 4 (t, x, y, z); panel: k indices into the mesh), the inner
 * integral of eq. tk_para for one panel, one lane per pair with the same
 * arithmetic as the assembly.  For checks and diagnostics. */
stb_status stb_inner_values(stb_ctx* ctx, const stb_mesh* mesh, const stb_quad_params* params,
                            int64_t k, const double* pts, const int32_t* panel, double* out);

/* Outward spatial normals of the panels, needed by the double layer (its
 * kernels k2, k3 of eq. kfunc contain <n_Gamma(y), x - y>): nrm is nt x 3
 * (host, any length); only the side matters: each normal must be finite
 * and within 60 degrees of the panel's plane normal (STB_E_INVALID_ARG
 * otherwise, and the mesh is left without normals).  The mesh keeps one
 * sign per panel. */
stb_status stb_mesh_set_normals(stb_ctx* ctx, stb_mesh* mesh, const double* nrm);

/* Retarded double-layer potential u(p) = D v (p) (eq. dlp: kernels k3 v +
 * k2 dv/dtau of eq. kfunc, behind the light cone) of the density v in
 * V_h^1 (def. st_be: continuous, linear on every panel) given by its nv
 * vertex values, at np points pts (np x 4, (t, x, y, z), host).  Needs the
 * mesh's outward normals (stb_mesh_set_normals; STB_E_INVALID_ARG
 * otherwise).  Panels whose plane contains the point contribute 0 (k2 = k3
 * = 0 there), so points on the surface get the direct value of the
 * integral.  Same phi-rule as the single layer, closed-form r-integrals;
 * FP64. */
stb_status stb_potential_D(stb_ctx* ctx, const stb_mesh* mesh, const stb_quad_params* params,
                           const double* v, int64_t np, const double* pts, double* out);
/* Same with v, pts and out in device memory; returns after the result is
 * written (the call synchronises its stream). */
stb_status stb_potential_D_dev(stb_ctx* ctx, const stb_mesh* mesh, const stb_quad_params* params,
                               const double* v_dev, int64_t np, const double* pts_dev,
                               double* out_dev, void* stream);
/* Double-layer potentials of the four hat functions of one panel at one
 * point: out[4 m + q] = D lambda_q (pts[m]) for panel[m], lambda_q the
 * linear function that is 1 at the panel's vertex q (its q-th index in the
 * tetrahedra array) and 0 at the other three.  For checks. */
stb_status stb_inner_values_D(stb_ctx* ctx, const stb_mesh* mesh, const stb_quad_params* params,
                              int64_t k, const double* pts, const int32_t* panel, double* out);

/* Energetic forms of the identity and the double layer with the outer rule
 * of eq. int_bform (A = I, A = K, the same rule as the single layer's
 * matrix rows): out[i] = c_id b_I(v, phi_i) + b_K(v, phi_i) for every test
 * panel i (out: nt entries, host), v in V_h^1 by its nv vertex values
 * (host).  b_I(v, phi_i) = sum_q w_iq v(x_iq) with panel i's own linear
 * function; b_K(v, phi_i) = sum_q w_iq (K v)(x_iq), K v the direct value of
 * the double layer at the outer points.  With v the data g (or its
 * interpolant), c_id = 1/2 gives the right-hand side of the direct method
 * (eq. df_dir) for the interior problem, c_id = -1/2 for the exterior one.
 * Needs the mesh's outward normals.  Works through the outer points in
 * chunks of 32,768. */
stb_status stb_dl_energetic(stb_ctx* ctx, const stb_mesh* mesh, const stb_quad_params* params,
                            const double* v, double c_id, double* out);

/* L2 projection Q_h^1 onto V_h^1 (the data projection of the direct method,
 * eq. df_dir): c in V_h^1 with (c, lambda_k) = (g, lambda_k) in L2(Sigma)
 * for every vertex hat lambda_k.  (g, lambda_k) uses a fixed rule of
 * STB_L2_POINTS points per panel (the 3 x 3 x 3 Gauss-Legendre product rule
 * collapsed onto the tetrahedron, exact for degree 3):
 * stb_l2_points writes them, pts [nt][STB_L2_POINTS][4] (t, x, y, z) and
 * weights [nt][STB_L2_POINTS] (host); the caller evaluates g there and
 * stb_project_V1 takes those values gq [nt][STB_L2_POINTS] (host) and
 * writes the nv vertex values of Q_h^1 g (host).  The mass system is solved
 * by Jacobi-preconditioned CG on the device to a relative residual of
 * 1e-13 (STB_E_INTERNAL if 1,000 steps do not reach it); iters (optional)
 * receives the steps. */
#define STB_L2_POINTS 27
stb_status stb_l2_points(stb_ctx* ctx, const stb_mesh* mesh, double* pts, double* wts);
stb_status stb_project_V1(stb_ctx* ctx, const stb_mesh* mesh, const double* gq, double* out,
                          int32_t* iters);

/* Batched assembly of nmesh meshes of one context (Exp. 3 style workloads
 * of many independent scatterers): the candidate sets of all meshes are one
 * work list of the pair pipeline, so every kernel launch covers the whole
 * batch.  Meshes are processed in waves of consecutive meshes whose stores
 * fit hbm_budget bytes of device memory (0: 40% of the free memory).
 * mats (optional): receives each mesh's matrix, as stb_assemble_V would
 * return it (then the whole batch forms one wave and must fit).
 * W_dev, Y_dev (optional, together): per mesh a device array of n_m x nrhs
 * inputs and outputs, Y_m = A_m W_m computed after the mesh's wave (nrhs = 16:
 * FP32 matrix cores), so that a batch larger than HBM can be assembled and
 * applied without keeping its matrices.  At least one of mats and W_dev/Y_dev
 * must be given.  n_causal (optional, host, nmesh entries): causal pairs
 * per mesh.  Results are identical to per-mesh stb_assemble_V calls.
 * Timings, work and kernel times describe the whole batch. */
stb_status stb_batch_assemble(stb_ctx* ctx, int32_t nmesh, stb_mesh* const* meshes,
                              const stb_quad_params* params, int64_t hbm_budget, stb_mat** mats,
                              int32_t nrhs, const double* const* W_dev, double* const* Y_dev,
                              int64_t* n_causal);

/* Launch-shape autotuner of the pair pipeline: times every stage (lit
 * test, breakpoints, empty-piece test, FP64 and FP32 Gauss nodes) on a
 * strided sample of about 2^22 of mesh's (test, trial) candidates for each
 * threads-per-block in {64, 128, 256} and resident blocks per CU in
 * {4, 8, 16, 32}, keeps the fastest per stage in ctx (used by every later
 * assembly, potential and batch on ctx) and, when cfg16 is not NULL, writes
 * the choice: cfg16[k] threads per block and cfg16[8 + k] blocks per CU of
 * stage k (numbered as in stb_last_kernel_times).  stb_batch_assemble runs
 * it on its largest mesh when ctx has not been tuned. */
stb_status stb_autotune(stb_ctx* ctx, const stb_mesh* mesh, const stb_quad_params* params,
                        int32_t* cfg16);

/* Set the launch shapes (cfg16 as written by stb_autotune; block sizes
 * multiples of 64 in [64, 256], 1..64 blocks per CU), or restore the
 * defaults (256 threads; 32 blocks per CU for stages 0-2, 16 for the
 * others) with cfg16 = NULL. */
stb_status stb_set_tuning(stb_ctx* ctx, const int32_t* cfg16);

/* Upper limits on the lengths of the pair pipeline's lists on ctx, per
 * chunk of candidates: max_cand candidates, max_combo lit (outer point,
 * trial panel) combos, max_piece phi pieces; 0 = no limit (the default).
 * The pipeline cuts the candidates into chunks whose lists fit and redoes a
 * chunk whose lists overflowed with a smaller one, so the values assembled
 * do not depend on the limits.  Set before the first assembly on ctx, they
 * bound the workspace it allocates (one already larger is kept) at the cost
 * of more chunks.  Nonzero limits are at least 64 (else STB_E_INVALID_ARG);
 * a candidate whose own combos or pieces exceed them fails with
 * STB_E_INTERNAL. */
stb_status stb_set_pair_lists(stb_ctx* ctx, int64_t max_cand, int64_t max_combo, int64_t max_piece);

/* ------------------------------------------------------------ serving
 * A server answers matvec and potential requests on meshes (and their
 * matrices) resident on one device, with continuous batching: nslots worker
 * slots, each with its own stream and workspace, take requests in arrival
 * order; a request starts as soon as a slot is free and its device
 * footprint (inputs, outputs and, for a potential, its exact candidate
 * arrays and the growth of its slot's pipeline workspace) fits
 * hbm_budget_bytes beside the requests in flight and the workspaces the
 * slots hold (0: half of the free device memory).  Requests in different
 * slots run concurrently on the device.  Results do not depend on what else
 * is in flight.  stb_server_submit, stb_server_wait and
 * stb_server_add_mesh are thread-safe (a mesh may be added while requests
 * run). */
typedef struct stb_server stb_server;

typedef enum { STB_REQ_MATVEC16 = 0, STB_REQ_POTENTIAL = 1 } stb_request_kind;

/* kind STB_REQ_MATVEC16: out (n x 16, row-major) = A w, w n x 16 row-major,
 *   A the matrix registered with the mesh (FP32 matrix cores).
 * kind STB_REQ_POTENTIAL: out[k] = S w (pts[k]) for np points (t, x, y, z),
 *   w the density (n values), FP64 (default quadrature parameters).
 * All pointers are host memory owned by the caller and must stay valid until
 * stb_server_wait for the ticket returns; out is written before that. */
typedef struct {
  int32_t kind;
  int32_t mesh;        /* id from stb_server_add_mesh */
  int64_t np;
  const double* w;
  const double* pts;
  double* out;
} stb_request;

stb_status stb_server_create(stb_ctx* ctx, int64_t hbm_budget_bytes, int32_t nslots,
                             stb_server** out);
/* Register a mesh of ctx and, for matvec requests, its matrix (both stay
 * owned by the caller and must outlive the server); *id receives the id. */
stb_status stb_server_add_mesh(stb_server* server, const stb_mesh* mesh, const stb_mat* mat,
                               int32_t* id);
/* Queue a request (the descriptor is copied, the data is not); *ticket
 * receives its ticket.  STB_E_NOT_FOUND for an unknown mesh id. */
stb_status stb_server_submit(stb_server* server, const stb_request* req, uint64_t* ticket);
/* Block until the request completes; returns its status (STB_E_NO_MEMORY if
 * its footprint exceeds the whole budget) and, if latency_s is not NULL, the
 * time from submit to completion in seconds.  Wait for each ticket once. */
stb_status stb_server_wait(stb_server* server, uint64_t ticket, double* latency_s);
/* Finish the queued and running requests, then release the server. */
void stb_server_destroy(stb_server* server);

/* The outer rule of eq. int_bform for every panel of mesh, the points the
 * matrix rows are built from: pts [nt][4 m_q^2][4] (t, x, y, z), weights
 * [nt][4 m_q^2] (-nu_{F,t} |F| / m_q^2 for the panel's faces with nu_t != 0,
 * Fig. int_tri_mid), counts [nt]; host arrays owned by the caller; entries
 * past a panel's count are zero.  With g sampled at these points,
 * b_i = sum_q w_iq g(x_q) is the right-hand side b(g, phi_i) of the discrete
 * indirect system (eq. df_ind, the same integration by parts as
 * eq. int_bform with g in place of V w). */
stb_status stb_outer_points(stb_ctx* ctx, const stb_mesh* mesh, int32_t m_q, double* pts,
                            double* weights, int32_t* counts);

/* Right-hand side of the discrete indirect system (eq. df_ind) for boundary
 * data g: b[i] = b(g, phi_i) = sum_q w_iq g(x_iq), the outer rule of
 * eq. int_bform with g in place of V w (the same integration by parts).
 * g: the data at the outer points of stb_outer_points for the same m_q,
 * [nt][4 m_q^2] (host; entries past a panel's count are ignored, must be
 * finite); b: nt doubles (host, caller-allocated).  Sums in q order. */
stb_status stb_outer_rhs(stb_ctx* ctx, const stb_mesh* mesh, int32_t m_q, const double* g,
                         double* b);

/* Solves the discrete indirect system A x = b (eq. df_ind) for the square
 * matrix of one whole mesh by restarted GMRES(restart) on the device: FP64
 * products with the stored matrix, classical Gram-Schmidt with one
 * re-orthogonalisation, Givens rotations on the host.  x_host holds the
 * initial guess and receives the solution (n doubles each, host).  Stops
 * when the true residual |b - A x| <= rtol |b| (checked at each restart) or
 * after maxit products; iters (optional) receives the products used,
 * relres (optional) the last true relative residual.  STB_E_INVALID_ARG for
 * a row block (not square), restart outside [1, 512], maxit < 1 or
 * rtol <= 0. */
stb_status stb_solve_gmres(stb_ctx* ctx, const stb_mat* A, const double* b_host, double* x_host,
                           int32_t restart, int32_t maxit, double rtol, int32_t* iters, double* relres);

/* Marching-on-in-time solve of the discrete indirect system A x = b
 * (eq. df_ind) for a mesh made of S time slabs that repeat: the vertex
 * times take S + 1 equally spaced values, every panel spans one slab
 * between two consecutive ones, every slab has the same number K of panels
 * and slab n is slab 0 moved by n dt in time, panel by panel in index
 * order (an unjittered extrusion).  Causality then makes A block lower
 * triangular in the slab index with the same diagonal block D (the coupling
 * of a slab with itself) on every slab, so x follows slab by slab:
 *   x_n = D^{-1} (b_n - sum_{m < n} A_nm x_m).
 * D is inverted once on the device (Gauss-Jordan, partial pivoting); each
 * time step is one product over the slab's rows with the solution so far
 * and one dense K x K product.  A: the matrix stb_assemble_V returned for
 * mesh; b_host, x_host: nt doubles (host).  info4 (optional): slabs S,
 * panels per slab K, milliseconds of the inversion and of the time steps.
 * STB_E_INVALID_ARG when the mesh or the stored matrix do not have that
 * structure (jittered or non-uniform time levels, a stored entry coupling
 * a slab to a later one, K > 16384): use stb_solve_gmres then. */
stb_status stb_solve_mot(stb_ctx* ctx, const stb_mesh* mesh, const stb_mat* A, const double* b_host,
                         double* x_host, double* info4);

/* Timing of the last stb_assemble_V or potential (stb_potential_S, _D) on
 * ctx, in milliseconds measured with HIP events on the context stream:
 * [0] geometry/outer points (0 for a potential), [1] cull and compaction
 * (the lit search of the points for a potential), [2] clip + quadrature +
 * store (+ the point sums), [3] total. */
stb_status stb_last_timings(const stb_ctx* ctx, double* ms4);

/* Path counts of the last assembly or batch on ctx.  [0..2]: evaluations of
 * L(phi) in the FP64 Gauss-node launches (kernel kind 4 of
 * stb_last_kernel_times) by the path that evaluated them: [0] pieces with
 * one gap of a fixed endpoint structure (two endpoint formulas per node),
 * [1] two gaps (four formulas), [2] the full evaluation over the four faces
 * (Sec. 3.2, the (r, phi) rule).  [3]: phi pieces found empty without
 * evaluating L, because the rays of all three test points (midpoint and
 * quarter points) miss the panel's spatial shadow (each would otherwise
 * cost three evaluations). */
stb_status stb_last_path_counts(const stb_ctx* ctx, int64_t* counts4);

/* Lit search of the last potential on ctx (stb_potential_S, _D):
 * [0] (point, leaf) pairs the cluster tree kept, [1] panels in those leaves
 * summed over the points (the sets X_N(x) of Sec. 3.3), [2] candidate
 * (point, panel) pairs after the per-panel bound test, which the exact lit
 * test then decides.  The flat search reports 0, points x panels examined,
 * and its candidates. */
stb_status stb_last_lit_search(const stb_ctx* ctx, int64_t* counts3);

/* Work of the last stb_assemble_V or potential on ctx: [0] evaluations of L(phi)
 * (empty-piece tests and Gauss nodes), [1] lit (outer point, trial panel)
 * pairs, [2] candidate (outer point, trial panel) pairs examined, [3] phi
 * pieces. */
stb_status stb_last_work(const stb_ctx* ctx, int64_t* counts4);

/* Per-kernel device time of the pair pipeline in the last stb_assemble_V or
 * potential call on ctx (HIP events on the context stream around every
 * launch): ms8[k] total milliseconds, launches8[k] launch count and
 * units8[k] work units for kernel kind k = 0 lit test (units: apexes
 * tested), 1 breakpoints (lit combos), 2 empty-piece test (L evaluations
 * at midpoints and quarter points), 3 mixed precision: second sums and
 * store (entries recomputed in FP64), 4 Gauss nodes FP64 (L evaluations),
 * 5 Gauss nodes FP32 of far pairs (L evaluations), 6 piece/apex sums and
 * store (candidates), 7 mixed precision: FP64 Gauss nodes of the
 * recomputed entries (L evaluations).  All three arrays are caller-allocated with
 * 8 entries. */
stb_status stb_last_kernel_times(const stb_ctx* ctx, double* ms8, int64_t* launches8,
                                 int64_t* units8);

#ifdef __cplusplus
}
#endif
#endif
