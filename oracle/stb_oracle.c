/*
 * stb_oracle.c -- plain FP64 CPU oracle (TEST INFRASTRUCTURE ONLY).
 *
 * Computes what the hot path computes, written for clarity, not speed:
 *
 *   A_ij = sum_{faces F of sigma_i} (-nu_{F,t} |F| / m_q^2)
 *          * sum_{q = 1..m_q^2} V phi_j (x_{F,q})                 (eq. int_bform,
 *                                                  composite centroid rule of
 *                                                  Fig. int_tri_mid, m_q = 3
 *                                                  in Exp. 3)
 *
 *   V phi_j (x) = (1 / 4 pi) int_0^{2 pi} L(phi) dphi,
 *   L(phi) = | { r >= |d| : (t - r, p + sqrt(r^2 - d^2) e(phi)) in sigma_j } |
 *
 * The second line is eq. slp restricted to one vertical panel: with the
 * panel in R x Pi_j, dS = dtau dA, the delta fixes tau = t - |x - y|, and
 * polar coordinates (s, phi) about the foot point p of x on Pi_j with
 * r = sqrt(s^2 + d^2) turn dA / |x - y| into dr dphi.  The k1 integrand is
 * thus constant in (r, phi) -- the statement of Lemma kernel_para for
 * rho_0 = 0 (k_psi,1 = r_0) and the form I = r_0 int_U d(rho, phi) used in
 * the appendix.  Only r is integrated exactly; phi uses the rule below.
 *
 * phi-rule (the paper's quadtree scheme of Sec. 3.1 is not reproducible
 * from the paper; this rule replaces it and is shared by definition, not by
 * code, with the GPU path):
 *   breakpoints = angles where the cone meets a panel edge (edge events),
 *                 angles where a face plane is tangent to the cone section
 *                 at a point of the closed panel (C_k^2 + d^2 (B_k^2 - a_k^2)
 *                 = 0), angles with B_k = 0 when the hyperboloid vertex
 *                 (t - |d|, p) lies on face k's plane, and angles with
 *                 B_k = a_k when the apex lies on face k's plane inside the
 *                 panel's hyperplane (d = 0, C_k = 0: L jumps there);
 *   between consecutive breakpoints (periodic), skip the piece if L is 0 at
 *   its midpoint and at its quarter points, else apply n_g-point
 *   Gauss-Legendre in the smoothstep
 *   variable phi = a + (b - a)(3u^2 - 2u^3);
 *   with no breakpoint at all, the periodic trapezoid rule with 2 n_g nodes.
 *
 * L(phi) itself is found the plain way: all roots of the squared face
 * equations inside the admissible r-range are candidate endpoints, and each
 * candidate sub-interval is kept iff its midpoint satisfies every face
 * inequality of eq. pnl_ilf.  Spurious roots of the squaring only add
 * harmless extra split points.
 *
 * The lit predicate (Sec. 3.3) uses the exact min / max of phi_Xi(x - y)
 * over the closed panel: the max at a vertex (convexity), the min among
 * vertex, edge-stationary and face-stationary candidates.
 *
 * Parity pins of every function live in tests/ (closed forms of the
 * appendix, polyhedral Laplace potentials, brute force, identities).
 */
#include "stb_oracle.h"
#include <math.h>
#include <string.h>
#include <stdlib.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORC_PI 3.14159265358979323846
#define ORC_TWO_PI (2.0 * ORC_PI)
#define ORC_MAX_BP 64
#define ORC_MAX_NG 96
/* Breakpoint hints are added within these fractions of the pair scale
 * |t - tau_min| + diam (see breakpoints()). */
#define ORC_TANG_TOL 0.05
#define ORC_VTX_TOL 0.05
#define ORC_FLAT_TOL 1e-10
/* edge parameters within this of [0, 1] count as on the closed edge */
#define ORC_EDGE_TOL 1e-10

enum { ORC_OK = 0, ORC_E_ARG = -1, ORC_E_PANEL = -2 };

typedef struct {
  double o[3], e1[3], e2[3], n[3];
  double V[4][3];              /* vertices in local (tau, u, v) */
  double fa[4], fb[4], fc[4];  /* unit outward face normals, local coords */
  double fh[4];                /* face k: fa tau + fb u + fc v < fh        */
  double tmin, tmax, diam;
} orc_panel;

static double dot3(const double* a, const double* b) {
  return a[0] * b[0] + a[1] * b[1] + a[2] * b[2];
}
static void cross3(const double* a, const double* b, double* c) {
  c[0] = a[1] * b[2] - a[2] * b[1];
  c[1] = a[2] * b[0] - a[0] * b[2];
  c[2] = a[0] * b[1] - a[1] * b[0];
}
static void sub3(const double* a, const double* b, double* c) {
  c[0] = a[0] - b[0]; c[1] = a[1] - b[1]; c[2] = a[2] - b[2];
}

/* Panel in its tangent hyperplane: frame + the 4 face half-spaces of
 * eq. pnl_ilf.  Rejects panels whose spatial projection is not planar
 * (space-time normal with a time component) or that are degenerate. */
static int panel_setup(const double* tet, orc_panel* P) {
  const double* X[4];
  double T[4];
  for (int k = 0; k < 4; ++k) {
    X[k] = tet + 4 * k + 1;
    T[k] = tet[4 * k];
    for (int c = 0; c < 4; ++c)
      if (!isfinite(tet[4 * k + c])) return ORC_E_PANEL;
  }
  int ia = 0, ib = 1;
  double best = -1.0;
  for (int a = 0; a < 4; ++a)
    for (int b = a + 1; b < 4; ++b) {
      double dv[3];
      sub3(X[b], X[a], dv);
      double l2 = dot3(dv, dv);
      if (l2 > best) { best = l2; ia = a; ib = b; }
    }
  if (!(best > 0.0)) return ORC_E_PANEL;
  double diam = sqrt(best);
  double e1[3];
  sub3(X[ib], X[ia], e1);
  for (int c = 0; c < 3; ++c) e1[c] /= diam;
  double nbest = -1.0, nrm[3] = {0, 0, 0};
  for (int c = 0; c < 4; ++c) {
    if (c == ia || c == ib) continue;
    double v[3], cr[3];
    sub3(X[c], X[ia], v);
    cross3(e1, v, cr);
    double l = sqrt(dot3(cr, cr));
    if (l > nbest) { nbest = l; nrm[0] = cr[0] / l; nrm[1] = cr[1] / l; nrm[2] = cr[2] / l; }
  }
  if (!(nbest > 1e-12 * diam)) return ORC_E_PANEL;
  double e2[3];
  cross3(nrm, e1, e2);
  for (int c = 0; c < 3; ++c) {
    P->o[c] = X[ia][c]; P->e1[c] = e1[c]; P->e2[c] = e2[c]; P->n[c] = nrm[c];
  }
  P->tmin = T[0]; P->tmax = T[0];
  double tspan;
  for (int k = 0; k < 4; ++k) {
    double v[3];
    sub3(X[k], P->o, v);
    if (fabs(dot3(v, nrm)) > 1e-12 * diam) return ORC_E_PANEL;
    P->V[k][0] = T[k];
    P->V[k][1] = dot3(v, e1);
    P->V[k][2] = dot3(v, e2);
    if (T[k] < P->tmin) P->tmin = T[k];
    if (T[k] > P->tmax) P->tmax = T[k];
  }
  tspan = P->tmax - P->tmin;
  P->diam = diam > tspan ? diam : tspan;
  /* 3-volume in (tau, u, v) must be positive */
  double a1[3], a2[3], a3[3], cr[3];
  sub3(P->V[1], P->V[0], a1);
  sub3(P->V[2], P->V[0], a2);
  sub3(P->V[3], P->V[0], a3);
  cross3(a1, a2, cr);
  double vol6 = fabs(dot3(cr, a3));
  if (!(vol6 > 1e-14 * P->diam * P->diam * P->diam)) return ORC_E_PANEL;
  for (int k = 0; k < 4; ++k) {
    int id[3], m = 0;
    for (int c = 0; c < 4; ++c) if (c != k) id[m++] = c;
    double u1[3], u2[3], N[3], toK[3];
    sub3(P->V[id[1]], P->V[id[0]], u1);
    sub3(P->V[id[2]], P->V[id[0]], u2);
    cross3(u1, u2, N);
    sub3(P->V[k], P->V[id[0]], toK);
    if (dot3(N, toK) > 0) { N[0] = -N[0]; N[1] = -N[1]; N[2] = -N[2]; }
    double l = sqrt(dot3(N, N));
    P->fa[k] = N[0] / l; P->fb[k] = N[1] / l; P->fc[k] = N[2] / l;
    P->fh[k] = (N[0] * P->V[id[0]][0] + N[1] * P->V[id[0]][1] + N[2] * P->V[id[0]][2]) / l;
  }
  return ORC_OK;
}

int orc_panel_frame(const double* tet, double* o, double* e1, double* e2, double* n) {
  orc_panel P;
  int rc = panel_setup(tet, &P);
  if (rc) return rc;
  for (int c = 0; c < 3; ++c) { o[c] = P.o[c]; e1[c] = P.e1[c]; e2[c] = P.e2[c]; n[c] = P.n[c]; }
  return ORC_OK;
}

/* ---------------- Gauss-Legendre ---------------- */
int orc_gauss_legendre01(int n, double* x, double* w) {
  if (n < 1 || n > ORC_MAX_NG) return ORC_E_ARG;
  for (int i = 0; i < n; ++i) {
    double z = cos(ORC_PI * (i + 0.75) / (n + 0.5));
    double dp = 1.0;
    for (int it = 0; it < 100; ++it) {
      double p0 = 1.0, p1 = z;           /* P_0, P_1 */
      for (int k = 2; k <= n; ++k) {
        double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
        p0 = p1; p1 = p2;
      }
      if (n == 1) { p1 = z; p0 = 1.0; }
      dp = n * (z * p1 - p0) / (z * z - 1.0);  /* P_n' */
      double dz = p1 / dp;
      z -= dz;
      if (fabs(dz) < 1e-16) break;
    }
    {
      double p0 = 1.0, p1 = z;
      for (int k = 2; k <= n; ++k) {
        double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
        p0 = p1; p1 = p2;
      }
      dp = n * (z * p1 - p0) / (z * z - 1.0);
    }
    /* node z in (-1,1) -> [0,1], weight 2/((1-z^2) P_n'^2) -> half */
    x[i] = 0.5 * (1.0 - z);
    w[i] = 1.0 / ((1.0 - z * z) * dp * dp);
  }
  return ORC_OK;
}

/* ---------------- apex data relative to one panel ---------------- */
typedef struct {
  double t, pu, pv, d;   /* apex time, foot point (local), signed distance */
  double C[4];           /* C_k = h_k - a_k t - b_k p_u - c_k p_v          */
} orc_apex;

static void apex_setup(const orc_panel* P, const double* x4, orc_apex* A) {
  double v[3] = {x4[1] - P->o[0], x4[2] - P->o[1], x4[3] - P->o[2]};
  A->t = x4[0];
  A->pu = dot3(v, P->e1);
  A->pv = dot3(v, P->e2);
  A->d = dot3(v, P->n);
  /* apex in the panel's hyperplane up to rounding: d = 0 exactly (a d of
   * order 1e-17 would turn C_k / d in the tangency condition into noise) */
  if (fabs(A->d) <= ORC_FLAT_TOL * (fabs(A->t - P->tmin) + P->diam)) A->d = 0.0;
  for (int k = 0; k < 4; ++k)
    A->C[k] = P->fh[k] - P->fa[k] * A->t - P->fb[k] * A->pu - P->fc[k] * A->pv;
}

static void sort_small(double* a, int n) {
  for (int i = 1; i < n; ++i) {
    double v = a[i];
    int j = i - 1;
    while (j >= 0 && a[j] > v) { a[j + 1] = a[j]; --j; }
    a[j + 1] = v;
  }
}

/* Roots of A2 r^2 + A1 r + A0 = 0 (numerically stable form). */
static int quad_roots(double A2, double A1, double A0, double* r) {
  if (A2 == 0.0) {
    if (A1 == 0.0) return 0;
    r[0] = -A0 / A1;
    return 1;
  }
  double disc = A1 * A1 - 4.0 * A2 * A0;
  if (disc < 0.0) return 0;
  double sq = sqrt(disc);
  double q = -0.5 * (A1 + copysign(sq, A1));
  if (q == 0.0) { r[0] = 0.0; return 1; }
  r[0] = q / A2;
  r[1] = A0 / q;
  return 2;
}

/* Roots of the squared face equation (B^2 - a^2) r^2 - 2 a C r
 * - (B^2 d^2 + C^2) = 0.  Its discriminant is 4 B^2 D with
 * D = C^2 + d^2 (B^2 - a^2); using the factored form avoids the
 * cancellation near B = 0, where the true and the spurious root meet. */
static int face_roots(double B, double a, double C, double d2, double* r) {
  double A2 = B * B - a * a, A1 = -2.0 * a * C, A0 = -(B * B * d2 + C * C);
  if (A2 == 0.0) {
    if (A1 == 0.0) return 0;
    r[0] = -A0 / A1;
    return 1;
  }
  double D = C * C + d2 * A2;
  if (D < 0.0) return 0;
  double sq = fabs(B) * sqrt(D);
  double q = a * C + copysign(sq, a * C);
  if (q == 0.0) { r[0] = 0.0; return 1; }
  r[0] = q / A2;
  r[1] = A0 / q;
  return 2;
}

/* The admissible r-set at angle phi as sub-intervals [seg[2m], seg[2m+1]]
 * in increasing order (see header comment); returns their number.  Adjacent
 * kept sub-intervals are not merged. */
static int r_segments(const orc_panel* P, const orc_apex* A, double phi, double* seg) {
  double rlo = fabs(A->d);
  if (A->t - P->tmax > rlo) rlo = A->t - P->tmax;
  double rhi = A->t - P->tmin;
  if (!(rhi > rlo)) return 0;
  double cs = cos(phi), sn = sin(phi);
  double B[4], cand[16];
  int nc = 0;
  cand[nc++] = rlo;
  cand[nc++] = rhi;
  double d2 = A->d * A->d;
  for (int k = 0; k < 4; ++k) {
    B[k] = P->fb[k] * cs + P->fc[k] * sn;
    double a = P->fa[k], C = A->C[k];
    double r[2];
    int nr = face_roots(B[k], a, C, d2, r);
    for (int m = 0; m < nr; ++m)
      if (r[m] > rlo && r[m] < rhi) cand[nc++] = r[m];
  }
  sort_small(cand, nc);
  int ns = 0;
  for (int m = 0; m + 1 < nc; ++m) {
    double r1 = cand[m], r2 = cand[m + 1];
    if (!(r2 > r1)) continue;
    double rm = 0.5 * (r1 + r2);
    double s2 = rm * rm - d2;
    double s = s2 > 0.0 ? sqrt(s2) : 0.0;
    int inside = 1;
    for (int k = 0; k < 4 && inside; ++k)
      if (!(B[k] * s - P->fa[k] * rm - A->C[k] < 0.0)) inside = 0;
    if (inside) { seg[2 * ns] = r1; seg[2 * ns + 1] = r2; ++ns; }
  }
  return ns;
}

/* L(phi): measure of the admissible r-set (see header comment). */
static double L_phi(const orc_panel* P, const orc_apex* A, double phi) {
  double seg[32];
  int ns = r_segments(P, A, phi, seg);
  double len = 0.0;
  for (int m = 0; m < ns; ++m) len += seg[2 * m + 1] - seg[2 * m];
  return len;
}

int orc_L(const double* x4, const double* tet, double phi, double* out) {
  orc_panel P;
  int rc = panel_setup(tet, &P);
  if (rc) return rc;
  orc_apex A;
  apex_setup(&P, x4, &A);
  *out = L_phi(&P, &A, phi);
  return ORC_OK;
}

static double wrap_angle(double a) {
  double r = fmod(a, ORC_TWO_PI);
  if (r < 0.0) r += ORC_TWO_PI;
  if (r >= ORC_TWO_PI) r -= ORC_TWO_PI;
  return r;
}

/* Tolerance scale of one (apex, panel) pair: |t - tau_min| + panel size. */
static double pair_scale(const orc_panel* P, double t) {
  return fabs(t - P->tmin) + P->diam;
}

/* Breakpoints of L (see header comment).  Returns count.
 *  - edge events: the cone meets one of the 6 panel edges;
 *  - tangencies: face k touches the cone section (D_k = 0) at a point of
 *    the closed panel (L has a square-root end there); also kept when the
 *    point lies within ORC_TANG_TOL * scale outside, where L is analytic but
 *    steep, so that the smoothstep nodes cluster there;
 *  - hyperboloid vertex (t - |d|, p) on face k's plane (a_k |d| + C_k = 0):
 *    angles with B_k = 0 (the second root crosses r = |d| there); kept as a
 *    hint while |a_k |d| + C_k| <= ORC_VTX_TOL * scale;
 *  - apex on face k's plane inside the panel's hyperplane (d = 0, C_k = 0):
 *    L jumps where B_k = a_k. */
static int breakpoints(const orc_panel* P, const orc_apex* A, double* bp) {
  int nb = 0;
  double d2 = A->d * A->d;
  double sc = pair_scale(P, A->t);
  /* edge events: cone meets edge V_i V_j */
  for (int i = 0; i < 4; ++i)
    for (int j = i + 1; j < 4; ++j) {
      const double* Pv = P->V[i];
      const double* Qv = P->V[j];
      double a0 = A->t - Pv[0], a1 = -(Qv[0] - Pv[0]);
      double bu = Pv[1] - A->pu, bv = Pv[2] - A->pv;
      double du = Qv[1] - Pv[1], dv = Qv[2] - Pv[2];
      double qa = a1 * a1 - du * du - dv * dv;
      double qb = 2.0 * (a0 * a1 - bu * du - bv * dv);
      double qc = a0 * a0 - bu * bu - bv * bv - d2;
      double lam[2];
      int nl;
      double disc = qb * qb - 4.0 * qa * qc;
      if (qa != 0.0 && disc < 0.0 && disc >= -1e-12 * (qb * qb + fabs(4.0 * qa * qc))) {
        /* the cone touches the edge: a double root lost to rounding */
        lam[0] = -qb / (2.0 * qa);
        nl = 1;
      } else {
        nl = quad_roots(qa, qb, qc, lam);
      }
      for (int m = 0; m < nl; ++m) {
        double l = lam[m];
        /* closed edges: a cone through a vertex gives roots at 0 or 1 up to
         * rounding, which are kept (at the vertex) */
        if (!(l >= -ORC_EDGE_TOL && l <= 1.0 + ORC_EDGE_TOL)) continue;
        if (l < 0.0) l = 0.0;
        if (l > 1.0) l = 1.0;
        if (a0 + a1 * l < 0.0) continue;   /* forward cone branch */
        double ou = bu + l * du, ov = bv + l * dv;
        /* a crossing at the foot point itself (s = 0) has no angle */
        if (ou * ou + ov * ov <= 1e-20 * sc * sc) continue;
        bp[nb++] = wrap_angle(atan2(ov, ou));
      }
    }
  for (int k = 0; k < 4; ++k) {
    double a = P->fa[k], b = P->fb[k], c = P->fc[k], C = A->C[k];
    double beta = sqrt(b * b + c * c);
    if (!(beta > 1e-12)) continue;   /* horizontal face: B_k = 0 for all phi */
    double phik = atan2(c, b);
    /* tangency: beta^2 cos^2(psi) = a^2 - C^2/d^2, psi = phi - phi_k */
    if (d2 > 0.0) {
      double rhs = a * a - C * C / d2;
      if (rhs >= 0.0 && rhs <= beta * beta) {
        double cv = sqrt(rhs) / beta;
        if (cv > 1.0) cv = 1.0;
        double g = acos(cv);
        double cand[4] = {phik + g, phik - g, phik + ORC_PI - g, phik + ORC_PI + g};
        for (int m = 0; m < 4; ++m) {
          double ph = cand[m];
          double Bt = b * cos(ph) + c * sin(ph);
          double den = Bt * Bt - a * a;
          if (den == 0.0 || Bt == 0.0) continue;
          double rt = a * C / den;               /* double root of the squared eq. */
          double st = (a * rt + C) / Bt;         /* B s = a r + C on the true branch */
          if (!(st >= 0.0) || !(rt >= fabs(A->d))) continue;
          double Y[3] = {A->t - rt, A->pu + st * cos(ph), A->pv + st * sin(ph)};
          double worst = -INFINITY;
          for (int m2 = 0; m2 < 4; ++m2) {
            double v = P->fa[m2] * Y[0] + P->fb[m2] * Y[1] + P->fc[m2] * Y[2] - P->fh[m2];
            if (v > worst) worst = v;
          }
          if (worst <= ORC_TANG_TOL * sc) bp[nb++] = wrap_angle(ph);
        }
      }
    }
    /* hyperboloid vertex (t - |d|, p) on the face plane */
    if (fabs(a * fabs(A->d) + C) <= ORC_VTX_TOL * sc) {
      bp[nb++] = wrap_angle(phik + 0.5 * ORC_PI);
      bp[nb++] = wrap_angle(phik - 0.5 * ORC_PI);
    }
    /* apex on the face plane inside the panel hyperplane: jump at B_k = a_k */
    if (fabs(A->d) <= ORC_FLAT_TOL * sc && fabs(C) <= ORC_FLAT_TOL * sc && fabs(a) <= beta) {
      double cv = a / beta;
      if (cv > 1.0) cv = 1.0;
      if (cv < -1.0) cv = -1.0;
      double g = acos(cv);
      bp[nb++] = wrap_angle(phik + g);
      bp[nb++] = wrap_angle(phik - g);
    }
  }
  sort_small(bp, nb);
  return nb;
}

/* Exact extrema of f(y) = |x - y| - (t - tau) over the closed panel. */
static double f_cone(const double* x4, const double* y4) {
  double dx = x4[1] - y4[1], dy = x4[2] - y4[2], dz = x4[3] - y4[3];
  return sqrt(dx * dx + dy * dy + dz * dz) - (x4[0] - y4[0]);
}

static void lit_extrema(const double* x4, const double* tet, const orc_panel* P,
                        double* mn_out, double* mx_out) {
  double mn = INFINITY, mx = -INFINITY;
  for (int k = 0; k < 4; ++k) {
    double f = f_cone(x4, tet + 4 * k);
    if (f < mn) mn = f;
    if (f > mx) mx = f;
  }
  /* edges: stationary points of sqrt(a l^2 + b l + c) + D l */
  for (int i = 0; i < 4; ++i)
    for (int j = i + 1; j < 4; ++j) {
      const double* Pp = tet + 4 * i;
      const double* Qq = tet + 4 * j;
      double U[3] = {Qq[1] - Pp[1], Qq[2] - Pp[2], Qq[3] - Pp[3]};
      double Av[3] = {Pp[1] - x4[1], Pp[2] - x4[2], Pp[3] - x4[3]};
      double Dt = Qq[0] - Pp[0];
      /* f(l) = sqrt(a l^2 + b l + c) + Dt l + const; the squared stationary
       * condition has roots -b/(2a) +- |Dt| sqrt((4ac - b^2) / g) / (2a) with
       * g = a - Dt^2 > 0 (space-like edge) and 4ac - b^2 = 4 |A x U|^2. */
      double a = dot3(U, U), b = 2.0 * dot3(Av, U);
      double g = a - Dt * Dt;
      if (!(a > 0.0 && g > 0.0)) continue;
      double cr[3];
      cross3(Av, U, cr);
      double disc = 4.0 * dot3(cr, cr);
      double hw = fabs(Dt) / (2.0 * a) * sqrt(disc / g);
      double lam[2] = {-b / (2.0 * a) - hw, -b / (2.0 * a) + hw};
      int nl = 2;
      for (int m = 0; m < nl; ++m) {
        double l = lam[m];
        if (!(l > 0.0 && l < 1.0)) continue;
        double y[4];
        for (int cc = 0; cc < 4; ++cc) y[cc] = Pp[cc] + l * (Qq[cc] - Pp[cc]);
        double f = f_cone(x4, y);
        if (f < mn) mn = f;
      }
    }
  /* faces: interior stationary point p - g |d| / sqrt(1 - |g|^2) */
  double v[3] = {x4[1] - P->o[0], x4[2] - P->o[1], x4[3] - P->o[2]};
  double pu = dot3(v, P->e1), pv = dot3(v, P->e2), d = dot3(v, P->n);
  for (int k = 0; k < 4; ++k) {
    int id[3], m = 0;
    for (int c = 0; c < 4; ++c) if (c != k) id[m++] = c;
    const double* V0 = P->V[id[0]];
    double Uu = P->V[id[1]][1] - V0[1], Uv = P->V[id[1]][2] - V0[2];
    double Wu = P->V[id[2]][1] - V0[1], Wv = P->V[id[2]][2] - V0[2];
    double D1 = P->V[id[1]][0] - V0[0], D2 = P->V[id[2]][0] - V0[0];
    double det = Uu * Wv - Uv * Wu;               /* spatial area x 2 */
    double sc = P->diam * P->diam;
    if (!(fabs(det) > 1e-12 * sc)) continue;      /* vertical face */
    /* tau = tau0 + g . (y - V0), g from [U W]^T g = [D1 D2] */
    double gu = (D1 * Wv - D2 * Uv) / det;
    double gv = (Uu * D2 - Wu * D1) / det;
    double g2 = gu * gu + gv * gv;
    if (!(g2 < 1.0)) continue;
    double fac = fabs(d) / sqrt(1.0 - g2);
    double yu = pu - gu * fac, yv = pv - gv * fac;
    /* barycentric of (yu,yv) in the face's spatial triangle */
    double ru = yu - V0[1], rv = yv - V0[2];
    double al = (ru * Wv - rv * Wu) / det;
    double be = (Uu * rv - Uv * ru) / det;
    if (!(al >= 0.0 && be >= 0.0 && al + be <= 1.0)) continue;
    double tau = V0[0] + gu * ru + gv * rv;
    double du = pu - yu, dv = pv - yv;
    double f = sqrt(du * du + dv * dv + d * d) - (x4[0] - tau);
    if (f < mn) mn = f;
  }
  *mn_out = mn;
  *mx_out = mx;
}

/* Lit decision with a relative dead zone: the cone must cross the panel by
 * more than delta = 1e-12 (|t - tau_min| + diam) on both sides.  An apex on
 * the panel's closure (shared faces, min = 0 up to rounding) is thus not
 * lit; a grazing contact of that size has no measurable integral. */
static int lit_decide(double mn, double mx, double t, const orc_panel* P) {
  double delta = 1e-12 * (fabs(t - P->tmin) + P->diam);
  return (mn < -delta && mx > delta) ? 1 : 0;
}

int orc_lit(const double* x4, const double* tet, double* mn, double* mx) {
  orc_panel P;
  int rc = panel_setup(tet, &P);
  if (rc) return rc;
  double a, b;
  lit_extrema(x4, tet, &P, &a, &b);
  if (mn) *mn = a;
  if (mx) *mx = b;
  return lit_decide(a, b, x4[0], &P);
}

/* ---------------- the inner integral ---------------- */
static double inner_panel(const orc_panel* P, const double* tet, const double* x4,
                          int n_g, const double* gx, const double* gw, orc_stats* st) {
  orc_apex A;
  apex_setup(P, x4, &A);
  if (!(A.t - P->tmin > fabs(A.d))) return 0.0;   /* cone misses the plane slab */
  double mn, mx;
  lit_extrema(x4, tet, P, &mn, &mx);
  if (!lit_decide(mn, mx, A.t, P)) return 0.0;    /* not lit (Sec. 3.3) */
  double bp[ORC_MAX_BP];
  int nb = breakpoints(P, &A, bp);
  double sum = 0.0;
  int64_t nev = 0, nsub = 0;
  if (nb == 0) {
    int m = 2 * n_g;
    double h = ORC_TWO_PI / m;
    for (int k = 0; k < m; ++k) sum += h * L_phi(P, &A, k * h);
    nev += m;
    nsub = 1;
  } else {
    for (int k = 0; k < nb; ++k) {
      double a = bp[k];
      double b = (k + 1 < nb) ? bp[k + 1] : bp[0] + ORC_TWO_PI;
      double H = b - a;
      if (!(H > 0.0)) continue;
      /* empty-piece test: L at the midpoint, then at the quarter points
       * (an isolated zero where the cone touches an edge must not empty a
       * piece) */
      ++nev;
      if (L_phi(P, &A, a + 0.5 * H) == 0.0) {
        nev += 2;
        if (L_phi(P, &A, a + 0.25 * H) == 0.0 && L_phi(P, &A, a + 0.75 * H) == 0.0) continue;
      }
      ++nsub;
      for (int g = 0; g < n_g; ++g) {
        double u = gx[g];
        double s = u * u * (3.0 - 2.0 * u);
        double ds = 6.0 * u * (1.0 - u);
        sum += H * ds * gw[g] * L_phi(P, &A, a + H * s);
      }
      nev += n_g;
    }
  }
  if (st) {
    st->n_eval += nev;
    st->n_sub += nsub;
    st->n_bp += nb;
    if (sum != 0.0) st->n_lit += 1;
  }
  return sum / (4.0 * ORC_PI);
}

int orc_inner(const double* x4, const double* tet, int n_g, double* out, orc_stats* st) {
  if (n_g < 1 || n_g > ORC_MAX_NG) return ORC_E_ARG;
  orc_panel P;
  int rc = panel_setup(tet, &P);
  if (rc) return rc;
  double gx[ORC_MAX_NG], gw[ORC_MAX_NG];
  orc_gauss_legendre01(n_g, gx, gw);
  *out = inner_panel(&P, tet, x4, n_g, gx, gw, st);
  return ORC_OK;
}

/* ---------------- double layer (eq. dlp) ----------------
 *
 * For a density v linear on the panel, eq. dlp restricted to the panel
 * reads, after the delta fixes tau = t - |x - y| and with the polar
 * coordinates of the single layer (dA = r dr dphi, r = |x - y|,
 * s = sqrt(r^2 - d^2)):
 *
 *   D v (x) = (d_n / 4 pi) int dphi int_{R(phi)} [ v(t - r, y) / r^2
 *                                                  + dv/dtau / r ] dr,
 *
 * with d_n = <n_Gamma, x - y> the distance of x from the panel's plane
 * along the outward normal (constant on the plane), so that k3 = d_n /
 * (4 pi r^3) and k2 = d_n / (4 pi r^2) (eq. kfunc).  Writing
 * v = c0 + c_tau tau + c_u u + c_v v in the local frame, the retarded
 * value is v(t - r, p + s e(phi)) = alpha - c_tau r + s gamma(phi) with
 * alpha = v(t, p) and gamma = c_u cos phi + c_v sin phi, so the c_tau terms
 * cancel and the r-integrand is alpha / r^2 + gamma s / r^2, integrated in
 * closed form over every sub-interval [r0, r1] of R(phi):
 *
 *   alpha (1/r0 - 1/r1) + gamma (H(r1) - H(r0)),  H(r) = ln(r + s) - s / r.
 *
 * The phi-rule (breakpoints, empty-piece test on L, smoothstep Gauss) is
 * the single layer's: the r-set is the same. */

/* v = c[0] + c[1] tau + c[2] u + c[3] v from its values at the 4 local
 * vertices (Gaussian elimination with partial pivoting). */
static int linear_coeffs(const orc_panel* P, const double* vv, double* c) {
  double M[4][5];
  for (int k = 0; k < 4; ++k) {
    M[k][0] = 1.0; M[k][1] = P->V[k][0]; M[k][2] = P->V[k][1]; M[k][3] = P->V[k][2];
    M[k][4] = vv[k];
  }
  for (int col = 0; col < 4; ++col) {
    int piv = col;
    for (int r = col + 1; r < 4; ++r)
      if (fabs(M[r][col]) > fabs(M[piv][col])) piv = r;
    if (M[piv][col] == 0.0) return ORC_E_PANEL;
    for (int q = 0; q < 5; ++q) { double t = M[col][q]; M[col][q] = M[piv][q]; M[piv][q] = t; }
    for (int r = col + 1; r < 4; ++r) {
      double f = M[r][col] / M[col][col];
      for (int q = col; q < 5; ++q) M[r][q] -= f * M[col][q];
    }
  }
  for (int r = 3; r >= 0; --r) {
    double x = M[r][4];
    for (int q = r + 1; q < 4; ++q) x -= M[r][q] * c[q];
    c[r] = x / M[r][r];
  }
  return ORC_OK;
}

static double H_dl(double r, double d2) {
  double s2 = r * r - d2;
  double s = s2 > 0.0 ? sqrt(s2) : 0.0;
  return log(r + s) - s / r;
}

/* The double-layer r-integral at angle phi (without the factor d_n). */
static double F_phi(const orc_panel* P, const orc_apex* A, double phi, double alpha,
                    double cu, double cv) {
  double seg[32];
  int ns = r_segments(P, A, phi, seg);
  double d2 = A->d * A->d, gam = cu * cos(phi) + cv * sin(phi);
  double f = 0.0;
  for (int m = 0; m < ns; ++m) {
    double r0 = seg[2 * m], r1 = seg[2 * m + 1];
    f += alpha * (1.0 / r0 - 1.0 / r1) + gam * (H_dl(r1, d2) - H_dl(r0, d2));
  }
  return f;
}

/* D v_j (x) for the outward-normal sign sgn (+1 when the outward normal is
 * the frame normal P->n) and vertex values vv. */
static double inner_panel_dl(const orc_panel* P, const double* tet, const double* x4, double sgn,
                             const double* vv, int n_g, const double* gx, const double* gw) {
  orc_apex A;
  apex_setup(P, x4, &A);
  if (A.d == 0.0) return 0.0;                     /* k2 = k3 = 0 in the plane */
  if (!(A.t - P->tmin > fabs(A.d))) return 0.0;
  double mn, mx;
  lit_extrema(x4, tet, P, &mn, &mx);
  if (!lit_decide(mn, mx, A.t, P)) return 0.0;
  double c[4];
  if (linear_coeffs(P, vv, c)) return 0.0;
  double alpha = c[0] + c[1] * A.t + c[2] * A.pu + c[3] * A.pv;
  double bp[ORC_MAX_BP];
  int nb = breakpoints(P, &A, bp);
  double sum = 0.0;
  if (nb == 0) {
    int m = 2 * n_g;
    double h = ORC_TWO_PI / m;
    for (int k = 0; k < m; ++k) sum += h * F_phi(P, &A, k * h, alpha, c[2], c[3]);
  } else {
    for (int k = 0; k < nb; ++k) {
      double a = bp[k];
      double b = (k + 1 < nb) ? bp[k + 1] : bp[0] + ORC_TWO_PI;
      double H = b - a;
      if (!(H > 0.0)) continue;
      if (L_phi(P, &A, a + 0.5 * H) == 0.0 && L_phi(P, &A, a + 0.25 * H) == 0.0 &&
          L_phi(P, &A, a + 0.75 * H) == 0.0)
        continue;
      for (int g = 0; g < n_g; ++g) {
        double u = gx[g];
        double s = u * u * (3.0 - 2.0 * u);
        double ds = 6.0 * u * (1.0 - u);
        sum += H * ds * gw[g] * F_phi(P, &A, a + H * s, alpha, c[2], c[3]);
      }
    }
  }
  return sgn * A.d * sum / (4.0 * ORC_PI);
}

static int normal_sign(const orc_panel* P, const double* nrm, double* sgn) {
  double l = sqrt(dot3(nrm, nrm)), c = dot3(nrm, P->n);
  if (!(l > 0.0) || !isfinite(l) || !(fabs(c) >= 0.5 * l)) return ORC_E_ARG;
  *sgn = c > 0.0 ? 1.0 : -1.0;
  return ORC_OK;
}

int orc_inner_dl(const double* x4, const double* tet, const double* nrm, const double* vv,
                 int n_g, double* out) {
  if (n_g < 1 || n_g > ORC_MAX_NG) return ORC_E_ARG;
  orc_panel P;
  int rc = panel_setup(tet, &P);
  if (rc) return rc;
  double sgn;
  if ((rc = normal_sign(&P, nrm, &sgn))) return rc;
  double gx[ORC_MAX_NG], gw[ORC_MAX_NG];
  orc_gauss_legendre01(n_g, gx, gw);
  *out = inner_panel_dl(&P, tet, x4, sgn, vv, n_g, gx, gw);
  return ORC_OK;
}

/* ---------------- outer rule ---------------- */
int orc_outer_points(const double* tet, int m_q, double* pts, double* w) {
  if (m_q < 1 || m_q > 16) return ORC_E_ARG;
  orc_panel P;
  int rc = panel_setup(tet, &P);
  if (rc) return rc;
  int np = 0;
  double inv = 1.0 / m_q;
  for (int k = 0; k < 4; ++k) {
    int id[3], m = 0;
    for (int c = 0; c < 4; ++c) if (c != k) id[m++] = c;
    double u1[3], u2[3], N[3], toK[3];
    sub3(P.V[id[1]], P.V[id[0]], u1);
    sub3(P.V[id[2]], P.V[id[0]], u2);
    cross3(u1, u2, N);
    sub3(P.V[k], P.V[id[0]], toK);
    double sgn = (dot3(N, toK) > 0) ? -1.0 : 1.0;   /* outward orientation */
    double nut_area = sgn * N[0] * 0.5;             /* nu_{F,t} |F|        */
    if (nut_area == 0.0) continue;                  /* vertical face       */
    double wq = -nut_area / (double)(m_q * m_q);
    const double* Pa = tet + 4 * id[0];
    const double* Pb = tet + 4 * id[1];
    const double* Pc = tet + 4 * id[2];
    for (int i = 0; i < m_q; ++i)
      for (int j = 0; i + j < m_q; ++j) {
        for (int up = 0; up < 2; ++up) {
          double al, be;
          if (up == 0) { al = (i + 1.0 / 3.0) * inv; be = (j + 1.0 / 3.0) * inv; }
          else {
            if (i + j > m_q - 2) continue;
            al = (i + 2.0 / 3.0) * inv; be = (j + 2.0 / 3.0) * inv;
          }
          for (int c = 0; c < 4; ++c)
            pts[4 * np + c] = Pa[c] + al * (Pb[c] - Pa[c]) + be * (Pc[c] - Pa[c]);
          w[np] = wq;
          ++np;
        }
      }
  }
  return np;
}

static void gather_tet(const double* vtx, const int32_t* tets, int64_t i, double* tet) {
  for (int k = 0; k < 4; ++k)
    for (int c = 0; c < 4; ++c) tet[4 * k + c] = vtx[4 * (int64_t)tets[4 * i + k] + c];
}

int orc_entry(const double* vtx, const int32_t* tets, int64_t i, int64_t j, int m_q, int n_g,
              double* out, orc_stats* st) {
  double ti[16], tj[16], pts[4 * 4 * 256], w[4 * 256];
  if (n_g < 1 || n_g > ORC_MAX_NG) return ORC_E_ARG;
  gather_tet(vtx, tets, i, ti);
  gather_tet(vtx, tets, j, tj);
  int np = orc_outer_points(ti, m_q, pts, w);
  if (np < 0) return np;
  orc_panel P;
  int rc = panel_setup(tj, &P);
  if (rc) return rc;
  double gx[ORC_MAX_NG], gw[ORC_MAX_NG];
  orc_gauss_legendre01(n_g, gx, gw);
  double s = 0.0;
  for (int q = 0; q < np; ++q) {
    double I = inner_panel(&P, tj, pts + 4 * q, n_g, gx, gw, st);
    if (I != 0.0) s += w[q] * I;
  }
  *out = s;
  return ORC_OK;
}

static int check_mesh(int64_t nv, const double* vtx, int64_t nt, const int32_t* tets) {
  if (nv <= 0 || nt < 0 || !vtx || (nt > 0 && !tets)) return ORC_E_ARG;
  for (int64_t i = 0; i < 4 * nt; ++i)
    if (tets[i] < 0 || tets[i] >= nv) return ORC_E_ARG;
  return ORC_OK;
}

/* Compensated running sum (Neumaier's variant of Kahan's: the rounding
 * error of every addition is kept, whichever operand is larger, so a
 * compensation is not lost when a large term follows small ones). */
typedef struct { double s, c; } orc_csum;
static void csum_add(orc_csum* a, double x) {
  double t = a->s + x;
  if (fabs(a->s) >= fabs(x)) a->c += (a->s - t) + x;
  else a->c += (x - t) + a->s;
  a->s = t;
}
static double csum_value(const orc_csum* a) { return a->s + a->c; }

/* Rows of A and, when mag is not NULL, the size of each entry's terms
 * mag[r*nt + j] = sum_q |w_q I_q| (the outer sum of eq. int_bform before
 * its top- and bottom-face terms cancel). */
int orc_assemble_rows_mag(int64_t nv, const double* vtx, int64_t nt, const int32_t* tets,
                          int64_t nrows, const int64_t* rows, int m_q, int n_g, double* out,
                          double* mag, orc_stats* st) {
  int rc = check_mesh(nv, vtx, nt, tets);
  if (rc) return rc;
  if (n_g < 1 || n_g > ORC_MAX_NG || m_q < 1 || m_q > 16) return ORC_E_ARG;
  orc_panel* panels = (orc_panel*)malloc(sizeof(orc_panel) * (size_t)(nt > 0 ? nt : 1));
  double* tetc = (double*)malloc(sizeof(double) * 16 * (size_t)(nt > 0 ? nt : 1));
  for (int64_t j = 0; j < nt; ++j) {
    gather_tet(vtx, tets, j, tetc + 16 * j);
    if (panel_setup(tetc + 16 * j, panels + j)) { free(panels); free(tetc); return ORC_E_PANEL; }
  }
  double gx[ORC_MAX_NG], gw[ORC_MAX_NG];
  orc_gauss_legendre01(n_g, gx, gw);
  int64_t s_eval = 0, s_sub = 0, s_bp = 0, s_lit = 0;
  int bad = 0;
#pragma omp parallel for schedule(dynamic, 1) reduction(+ : s_eval, s_sub, s_bp, s_lit)
  for (int64_t r = 0; r < nrows; ++r) {
    int64_t i = rows[r];
    if (i < 0 || i >= nt) { bad = 1; continue; }
    double pts[4 * 4 * 256], w[4 * 256];
    int np = orc_outer_points(tetc + 16 * i, m_q, pts, w);
    orc_stats ls = {0, 0, 0, 0};
    for (int64_t j = 0; j < nt; ++j) {
      double s = 0.0, a = 0.0;
      for (int q = 0; q < np; ++q) {
        double I = inner_panel(panels + j, tetc + 16 * j, pts + 4 * q, n_g, gx, gw, &ls);
        if (I != 0.0) {
          s += w[q] * I;
          a += fabs(w[q] * I);
        }
      }
      out[r * nt + j] = s;
      if (mag) mag[r * nt + j] = a;
    }
    s_eval += ls.n_eval; s_sub += ls.n_sub; s_bp += ls.n_bp; s_lit += ls.n_lit;
  }
  free(panels);
  free(tetc);
  if (bad) return ORC_E_ARG;
  if (st) { st->n_eval += s_eval; st->n_sub += s_sub; st->n_bp += s_bp; st->n_lit += s_lit; }
  return ORC_OK;
}

int orc_assemble_rows(int64_t nv, const double* vtx, int64_t nt, const int32_t* tets,
                      int64_t nrows, const int64_t* rows, int m_q, int n_g, double* out,
                      orc_stats* st) {
  return orc_assemble_rows_mag(nv, vtx, nt, tets, nrows, rows, m_q, n_g, out, NULL, st);
}

int orc_matvec_rows(int64_t nv, const double* vtx, int64_t nt, const int32_t* tets,
                    int64_t nrows, const int64_t* rows, int m_q, int n_g, const double* w,
                    double* y) {
  int rc = check_mesh(nv, vtx, nt, tets);
  if (rc) return rc;
  double* A = (double*)malloc(sizeof(double) * (size_t)nt);
  if (!A && nt) return ORC_E_ARG;
  for (int64_t r = 0; r < nrows; ++r) {
    rc = orc_assemble_rows(nv, vtx, nt, tets, 1, rows + r, m_q, n_g, A, NULL);
    if (rc) { free(A); return rc; }
    orc_csum acc = {0.0, 0.0};
    for (int64_t j = 0; j < nt; ++j) csum_add(&acc, A[j] * w[j]);
    y[r] = csum_value(&acc);
  }
  free(A);
  return ORC_OK;
}

int orc_potential(int64_t nv, const double* vtx, int64_t nt, const int32_t* tets,
                  const double* w, int64_t np, const double* pts, int n_g, double* out) {
  int rc = check_mesh(nv, vtx, nt, tets);
  if (rc) return rc;
  if (n_g < 1 || n_g > ORC_MAX_NG) return ORC_E_ARG;
  orc_panel* panels = (orc_panel*)malloc(sizeof(orc_panel) * (size_t)(nt > 0 ? nt : 1));
  double* tetc = (double*)malloc(sizeof(double) * 16 * (size_t)(nt > 0 ? nt : 1));
  for (int64_t j = 0; j < nt; ++j) {
    gather_tet(vtx, tets, j, tetc + 16 * j);
    if (panel_setup(tetc + 16 * j, panels + j)) { free(panels); free(tetc); return ORC_E_PANEL; }
  }
  double gx[ORC_MAX_NG], gw[ORC_MAX_NG];
  orc_gauss_legendre01(n_g, gx, gw);
#pragma omp parallel for schedule(dynamic, 1)
  for (int64_t p = 0; p < np; ++p) {
    orc_csum acc = {0.0, 0.0};
    for (int64_t j = 0; j < nt; ++j) {
      double I = inner_panel(panels + j, tetc + 16 * j, pts + 4 * p, n_g, gx, gw, NULL);
      if (I != 0.0) csum_add(&acc, w[j] * I);
    }
    out[p] = csum_value(&acc);
  }
  free(panels);
  free(tetc);
  return ORC_OK;
}

int orc_potential_dl(int64_t nv, const double* vtx, int64_t nt, const int32_t* tets,
                     const double* nrm, const double* v, int64_t np, const double* pts, int n_g,
                     double* out) {
  int rc = check_mesh(nv, vtx, nt, tets);
  if (rc) return rc;
  if (n_g < 1 || n_g > ORC_MAX_NG) return ORC_E_ARG;
  orc_panel* panels = (orc_panel*)malloc(sizeof(orc_panel) * (size_t)(nt > 0 ? nt : 1));
  double* tetc = (double*)malloc(sizeof(double) * 16 * (size_t)(nt > 0 ? nt : 1));
  double* sg = (double*)malloc(sizeof(double) * (size_t)(nt > 0 ? nt : 1));
  for (int64_t j = 0; j < nt; ++j) {
    gather_tet(vtx, tets, j, tetc + 16 * j);
    rc = panel_setup(tetc + 16 * j, panels + j);
    if (!rc) rc = normal_sign(panels + j, nrm + 3 * j, sg + j);
    if (rc) { free(panels); free(tetc); free(sg); return rc; }
  }
  double gx[ORC_MAX_NG], gw[ORC_MAX_NG];
  orc_gauss_legendre01(n_g, gx, gw);
#pragma omp parallel for schedule(dynamic, 1)
  for (int64_t p = 0; p < np; ++p) {
    orc_csum acc = {0.0, 0.0};
    for (int64_t j = 0; j < nt; ++j) {
      double vv[4];
      for (int k = 0; k < 4; ++k) vv[k] = v[tets[4 * j + k]];
      double I = inner_panel_dl(panels + j, tetc + 16 * j, pts + 4 * p, sg[j], vv, n_g, gx, gw);
      if (I != 0.0) csum_add(&acc, I);
    }
    out[p] = csum_value(&acc);
  }
  free(panels);
  free(tetc);
  free(sg);
  return ORC_OK;
}

/* Energetic forms of the double layer and the identity with the outer rule
 * of eq. int_bform (A = K, A = I): for every given test panel i,
 *   out[r] = c_id * sum_q w_q v(x_q) + sum_q w_q (K v)(x_q),
 * v in V_h^1 with vertex values v[nv]; v(x_q) is panel i's own linear
 * function at its outer point, (K v)(x_q) the direct value of the double
 * layer there (panels in x_q's plane contribute 0). */
int orc_dl_energetic_rows(int64_t nv, const double* vtx, int64_t nt, const int32_t* tets,
                          const double* nrm, const double* v, int64_t nrows, const int64_t* rows,
                          int m_q, int n_g, double c_id, double* out) {
  int rc = check_mesh(nv, vtx, nt, tets);
  if (rc) return rc;
  if (n_g < 1 || n_g > ORC_MAX_NG || m_q < 1 || m_q > 16) return ORC_E_ARG;
  orc_panel* panels = (orc_panel*)malloc(sizeof(orc_panel) * (size_t)(nt > 0 ? nt : 1));
  double* tetc = (double*)malloc(sizeof(double) * 16 * (size_t)(nt > 0 ? nt : 1));
  double* sg = (double*)malloc(sizeof(double) * (size_t)(nt > 0 ? nt : 1));
  for (int64_t j = 0; j < nt; ++j) {
    gather_tet(vtx, tets, j, tetc + 16 * j);
    rc = panel_setup(tetc + 16 * j, panels + j);
    if (!rc) rc = normal_sign(panels + j, nrm + 3 * j, sg + j);
    if (rc) { free(panels); free(tetc); free(sg); return rc; }
  }
  double gx[ORC_MAX_NG], gw[ORC_MAX_NG];
  orc_gauss_legendre01(n_g, gx, gw);
  int bad = 0;
#pragma omp parallel for schedule(dynamic, 1)
  for (int64_t r = 0; r < nrows; ++r) {
    int64_t i = rows[r];
    if (i < 0 || i >= nt) { bad = 1; continue; }
    double pts[4 * 4 * 256], w[4 * 256], vi[4], c[4];
    int np = orc_outer_points(tetc + 16 * i, m_q, pts, w);
    for (int k = 0; k < 4; ++k) vi[k] = v[tets[4 * i + k]];
    linear_coeffs(panels + i, vi, c);
    double acc = 0.0;
    for (int q = 0; q < np; ++q) {
      const double* x = pts + 4 * q;
      double d3[3] = {x[1] - panels[i].o[0], x[2] - panels[i].o[1], x[3] - panels[i].o[2]};
      double vq = c[0] + c[1] * x[0] + c[2] * dot3(d3, panels[i].e1) + c[3] * dot3(d3, panels[i].e2);
      double kv = 0.0;
      for (int64_t j = 0; j < nt; ++j) {
        double vv[4];
        for (int k = 0; k < 4; ++k) vv[k] = v[tets[4 * j + k]];
        kv += inner_panel_dl(panels + j, tetc + 16 * j, x, sg[j], vv, n_g, gx, gw);
      }
      acc += w[q] * (c_id * vq + kv);
    }
    out[r] = acc;
  }
  free(panels);
  free(tetc);
  free(sg);
  return bad ? ORC_E_ARG : ORC_OK;
}

/* ---------------- L2 projection onto V_h^1 (eq. df_dir's Q_h^1) ----------------
 * (c, lambda_k) = (g, lambda_k) in L2(Sigma), dS = the 3-volume of the
 * panel in its (tau, u, v) frame.  The integrals of g use a fixed rule
 * (ORC_L2_PTS points per panel): the 3 x 3 x 3 Gauss-Legendre product rule
 * on the unit cube pulled back to the tetrahedron by
 * (a, b, c) -> (a, (1 - a) b, (1 - a)(1 - b) c), Jacobian (1 - a)^2 (1 - b);
 * the mass matrix is exact, vol (1 + delta_kl) / 20 per panel.  Dense
 * Gaussian elimination (small meshes only). */
#define ORC_L2_PTS 27

static void l2_rule(double lam[ORC_L2_PTS][4], double w[ORC_L2_PTS]) {
  double gx[3], gw[3];
  orc_gauss_legendre01(3, gx, gw);
  int p = 0;
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j)
      for (int k = 0; k < 3; ++k) {
        double a = gx[i], b = gx[j], c = gx[k];
        double xi1 = a, xi2 = (1.0 - a) * b, xi3 = (1.0 - a) * (1.0 - b) * c;
        lam[p][0] = 1.0 - xi1 - xi2 - xi3;
        lam[p][1] = xi1;
        lam[p][2] = xi2;
        lam[p][3] = xi3;
        w[p] = gw[i] * gw[j] * gw[k] * (1.0 - a) * (1.0 - a) * (1.0 - b);
        ++p;
      }
}

static double panel_volume(const orc_panel* P) {
  double a1[3], a2[3], a3[3], cr[3];
  sub3(P->V[1], P->V[0], a1);
  sub3(P->V[2], P->V[0], a2);
  sub3(P->V[3], P->V[0], a3);
  cross3(a1, a2, cr);
  return fabs(dot3(cr, a3)) / 6.0;
}

int orc_l2_points(const double* tet, double* pts, double* w) {
  orc_panel P;
  int rc = panel_setup(tet, &P);
  if (rc) return rc;
  double lam[ORC_L2_PTS][4], wr[ORC_L2_PTS];
  l2_rule(lam, wr);
  double vol = panel_volume(&P);
  for (int p = 0; p < ORC_L2_PTS; ++p) {
    for (int c = 0; c < 4; ++c) {
      double x = 0.0;
      for (int m = 0; m < 4; ++m) x += lam[p][m] * tet[4 * m + c];
      pts[4 * p + c] = x;
    }
    w[p] = 6.0 * vol * wr[p];
  }
  return ORC_L2_PTS;
}

int orc_l2_projection(int64_t nv, const double* vtx, int64_t nt, const int32_t* tets,
                      const double* gq, double* out) {
  int rc = check_mesh(nv, vtx, nt, tets);
  if (rc) return rc;
  if (nv > 20000) return ORC_E_ARG;
  double lam[ORC_L2_PTS][4], wr[ORC_L2_PTS];
  l2_rule(lam, wr);
  double* M = (double*)calloc((size_t)nv * (size_t)(nv + 1), sizeof(double));   /* [nv][nv + 1] */
  if (!M) return ORC_E_ARG;
  for (int64_t j = 0; j < nt; ++j) {
    double tet[16];
    orc_panel P;
    gather_tet(vtx, tets, j, tet);
    if ((rc = panel_setup(tet, &P))) { free(M); return rc; }
    double vol = panel_volume(&P);
    for (int a = 0; a < 4; ++a) {
      int64_t k = tets[4 * j + a];
      for (int b = 0; b < 4; ++b) M[k * (nv + 1) + tets[4 * j + b]] += vol * (a == b ? 2.0 : 1.0) / 20.0;
      double f = 0.0;
      for (int p = 0; p < ORC_L2_PTS; ++p) f += 6.0 * vol * wr[p] * gq[j * ORC_L2_PTS + p] * lam[p][a];
      M[k * (nv + 1) + nv] += f;
    }
  }
  for (int64_t col = 0; col < nv; ++col) {
    int64_t piv = col;
    for (int64_t r = col + 1; r < nv; ++r)
      if (fabs(M[r * (nv + 1) + col]) > fabs(M[piv * (nv + 1) + col])) piv = r;
    if (M[piv * (nv + 1) + col] == 0.0) { free(M); return ORC_E_PANEL; }
    if (piv != col)
      for (int64_t q = 0; q <= nv; ++q) {
        double t = M[col * (nv + 1) + q];
        M[col * (nv + 1) + q] = M[piv * (nv + 1) + q];
        M[piv * (nv + 1) + q] = t;
      }
    for (int64_t r = col + 1; r < nv; ++r) {
      double f = M[r * (nv + 1) + col] / M[col * (nv + 1) + col];
      if (f == 0.0) continue;
      for (int64_t q = col; q <= nv; ++q) M[r * (nv + 1) + q] -= f * M[col * (nv + 1) + q];
    }
  }
  for (int64_t r = nv - 1; r >= 0; --r) {
    double x = M[r * (nv + 1) + nv];
    for (int64_t q = r + 1; q < nv; ++q) x -= M[r * (nv + 1) + q] * out[q];
    out[r] = x / M[r * (nv + 1) + r];
  }
  free(M);
  return ORC_OK;
}

int orc_pair_causal(const double* vtx, const int32_t* tets, int64_t i, int64_t j, int m_q) {
  double ti[16], tj[16], pts[4 * 4 * 256], w[4 * 256];
  gather_tet(vtx, tets, i, ti);
  gather_tet(vtx, tets, j, tj);
  int np = orc_outer_points(ti, m_q, pts, w);
  if (np < 0) return np;
  orc_panel P;
  if (panel_setup(tj, &P)) return ORC_E_PANEL;
  for (int q = 0; q < np; ++q) {
    double mn, mx;
    lit_extrema(pts + 4 * q, tj, &P, &mn, &mx);
    if (lit_decide(mn, mx, pts[4 * q], &P)) return 1;
  }
  return 0;
}

int orc_count_causal_per_row(int64_t nv, const double* vtx, int64_t nt, const int32_t* tets,
                             int64_t nrows, const int64_t* rows, int m_q, int64_t* out) {
  int rc = check_mesh(nv, vtx, nt, tets);
  if (rc) return rc;
  int bad = 0;
#pragma omp parallel for schedule(dynamic, 4)
  for (int64_t r = 0; r < nrows; ++r) {
    int64_t i = rows[r];
    if (i < 0 || i >= nt) { bad = 1; continue; }
    int64_t c = 0;
    for (int64_t j = 0; j < nt; ++j) {
      int v = orc_pair_causal(vtx, tets, i, j, m_q);
      if (v < 0) { bad = 1; break; }
      c += v;
    }
    out[r] = c;
  }
  return bad ? ORC_E_ARG : ORC_OK;
}

int64_t orc_count_causal_rows(int64_t nv, const double* vtx, int64_t nt, const int32_t* tets,
                              int64_t nrows, const int64_t* rows, int m_q) {
  int64_t* per = (int64_t*)malloc(sizeof(int64_t) * (size_t)(nrows > 0 ? nrows : 1));
  int rc = orc_count_causal_per_row(nv, vtx, nt, tets, nrows, rows, m_q, per);
  int64_t s = 0;
  if (rc == 0)
    for (int64_t r = 0; r < nrows; ++r) s += per[r];
  free(per);
  return rc ? (int64_t)rc : s;
}

int orc_num_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

int orc_breakpoints(const double* x4, const double* tet, double* out, int cap) {
  orc_panel P;
  int rc = panel_setup(tet, &P);
  if (rc) return rc;
  orc_apex A;
  apex_setup(&P, x4, &A);
  double bp[ORC_MAX_BP];
  int nb = breakpoints(&P, &A, bp);
  for (int k = 0; k < nb && k < cap; ++k) out[k] = bp[k];
  return nb;
}
