/*
 * stb_oracle.h -- plain FP64 CPU oracle for the energetic single-layer
 * space-time Galerkin BEM (Poelz & Schanz, arXiv 2103.16841).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library may include,
 * link or call this file; only the tests, the smoke check and the CPU
 * baseline leg of the benchmark use it.  It shares no code with the HIP
 * path.
 *
 * Conventions (all FP64):
 *   space-time points are (t, x, y, z) with wave speed c = 1 (geometrized
 *   time, Sec. 2);  a tetrahedral panel is given by 4 such points, all four
 *   spatial projections coplanar (vertical panel, Sec. 2: the space-time
 *   normal has no time component);  k1 = 1/(4 pi |x-y|)  (eq. kfunc).
 *
 * Matrix convention:  A[i][j] = b_V(phi_j, phi_i), row i = test panel,
 * column j = trial panel (eq. df_ind with the outer form eq. int_bform).
 */
#ifndef STB_ORACLE_H
#define STB_ORACLE_H
#include <stdint.h>
#ifdef __cplusplus
extern "C" {
#endif

/* Work counters of one inner integral (summed by the callers). */
typedef struct {
  int64_t n_eval;      /* evaluations of L(phi) (midpoint tests + nodes)  */
  int64_t n_sub;       /* non-empty phi sub-intervals                     */
  int64_t n_bp;        /* breakpoints collected                           */
  int64_t n_lit;       /* inner integrals with a non-zero value           */
} orc_stats;

/* Gauss-Legendre rule with n nodes on [0,1] (Newton on P_n). */
int orc_gauss_legendre01(int n, double* x, double* w);

/* Inner integral V phi_j (x) = S 1_sigma (x) (eq. slp, Lemma kernel_para):
 * x4 = (t,x,y,z); tet = 4 points x 4 coords, row-major.  n_g = Gauss
 * nodes per phi sub-interval.  Returns 0 and writes *out, or a negative
 * code for an invalid (non-vertical / degenerate) panel. */
int orc_inner(const double* x4, const double* tet, int n_g, double* out,
              orc_stats* st);

/* L(phi) on its own (for tests): length of the r-set at one angle phi,
 * measured from the panel's local axis e1 (see orc_panel_frame). */
int orc_L(const double* x4, const double* tet, double phi, double* out);

/* Local frame of a panel: origin o[3], axes e1[3], e2[3], unit normal n[3]. */
int orc_panel_frame(const double* tet, double* o, double* e1, double* e2,
                    double* n);

/* Outer points of test panel tet for the composite centroid rule with
 * m_q^2 sub-triangles per face (Fig. int_tri_mid, eq. int_bform).  Writes
 * up to 4*m_q^2 points pts[k*4+c] and weights w[k] = -nu_t |F| / m_q^2;
 * faces with nu_t == 0 are skipped.  Returns the number of points or a
 * negative code. */
int orc_outer_points(const double* tet, int m_q, double* pts, double* w);

/* One matrix entry A_ij. */
int orc_entry(const double* vtx, const int32_t* tets, int64_t i, int64_t j,
              int m_q, int n_g, double* out, orc_stats* st);

/* Rows of A: out[r*nt + j] = A[rows[r]][j], all nt columns; OpenMP over
 * rows.  Returns 0 or a negative code. */
int orc_assemble_rows(int64_t nv, const double* vtx, int64_t nt,
                      const int32_t* tets, int64_t nrows, const int64_t* rows,
                      int m_q, int n_g, double* out, orc_stats* st);

/* Same rows and, when mag is not NULL, mag[r*nt + j] = sum_q |w_q I_q|:
 * the size of the outer-sum terms of entry (rows[r], j) of eq. int_bform,
 * whose top- and bottom-face terms cancel in A itself. */
int orc_assemble_rows_mag(int64_t nv, const double* vtx, int64_t nt,
                          const int32_t* tets, int64_t nrows, const int64_t* rows,
                          int m_q, int n_g, double* out, double* mag,
                          orc_stats* st);

/* y[r] = sum_j A[rows[r]][j] w[j]  (compensated sum, Neumaier). */
int orc_matvec_rows(int64_t nv, const double* vtx, int64_t nt,
                    const int32_t* tets, int64_t nrows, const int64_t* rows,
                    int m_q, int n_g, const double* w, double* y);

/* u(p) = sum_j w_j V phi_j (p) at np points (eq. slp with w in S_h^0). */
int orc_potential(int64_t nv, const double* vtx, int64_t nt,
                  const int32_t* tets, const double* w, int64_t np,
                  const double* pts, int n_g, double* out);

/* Retarded double-layer potential (eq. dlp, kernels k2, k3 of eq. kfunc)
 * at x4 of the density that is linear on the panel tet with values vv[4]
 * at its vertices; nrm[3] = the panel's outward spatial normal (its sign
 * is what matters; it must not be tangent to the panel).  Same phi-rule as
 * orc_inner; the r-integral is closed-form. */
int orc_inner_dl(const double* x4, const double* tet, const double* nrm,
                 const double* vv, int n_g, double* out);
/* u(p) = D v (p) at np points for v in V_h^1 (vertex values v[nv]); nrm =
 * per-panel outward spatial normals [nt][3]. */
int orc_potential_dl(int64_t nv, const double* vtx, int64_t nt,
                     const int32_t* tets, const double* nrm, const double* v,
                     int64_t np, const double* pts, int n_g, double* out);
/* c_id b_I(v, phi_i) + b_K(v, phi_i) for the given test panels (eq.
 * int_bform with A = I and A = K: outer rule of m_q^2 points per face);
 * v in V_h^1 (vertex values), nrm per-panel outward normals.  K v at an
 * outer point is the direct value of the double layer there. */
int orc_dl_energetic_rows(int64_t nv, const double* vtx, int64_t nt,
                          const int32_t* tets, const double* nrm, const double* v,
                          int64_t nrows, const int64_t* rows, int m_q, int n_g,
                          double c_id, double* out);
/* L2 projection onto V_h^1: orc_l2_points writes the 27 points (pts[27][4])
 * and weights of the fixed panel rule; orc_l2_projection takes g at those
 * points for every panel (gq[nt][27]) and writes the nv vertex values of
 * Q_h^1 g (dense solve, nv <= 20000). */
int orc_l2_points(const double* tet, double* pts, double* w);
int orc_l2_projection(int64_t nv, const double* vtx, int64_t nt,
                      const int32_t* tets, const double* gq, double* out);
/* Exact lit predicate of Sec. 3.3: 1 iff the backward cone of x meets the
 * open panel, i.e. min < 0 < max of phi_Xi(x - y) over the closed panel
 * (eq. sgn_dist_cone).  Also returns min and max when non-NULL. */
int orc_lit(const double* x4, const double* tet, double* mn, double* mx);

/* Causal pair predicate: some outer point of panel i lights panel j. */
int orc_pair_causal(const double* vtx, const int32_t* tets, int64_t i,
                    int64_t j, int m_q);

/* Number of causal pairs over the given rows (all columns); OpenMP. */
int64_t orc_count_causal_rows(int64_t nv, const double* vtx, int64_t nt,
                              const int32_t* tets, int64_t nrows,
                              const int64_t* rows, int m_q);

/* Per-row causal counts (for the row-sampled workloads). */
int orc_count_causal_per_row(int64_t nv, const double* vtx, int64_t nt,
                             const int32_t* tets, int64_t nrows,
                             const int64_t* rows, int m_q, int64_t* out);

int orc_num_threads(void);

/* Breakpoint angles of L for one (apex, panel) pair (sorted); returns count. */
int orc_breakpoints(const double* x4, const double* tet, double* out, int cap);

#ifdef __cplusplus
}
#endif
#endif
