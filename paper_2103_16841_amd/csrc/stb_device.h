// stb_device.h -- device-side geometry and quadrature of the energetic
// single-layer form (Poelz & Schanz, arXiv 2103.16841) for CDNA4 (gfx950).
//
// Notation follows the paper: a panel sigma lies in R x Pi (vertical,
// Sec. 2); its faces are half-spaces of the tangent hyperplane (eq.
// pnl_ilf); the backward light cone of x is phi_Xi(x - y) = 0 (eq.
// sgn_dist_cone).  For an apex x = (t, x) with foot point p on Pi and signed
// distance d, polar coordinates (s, phi) about p and r = sqrt(s^2 + d^2)
// turn the single-layer integral (eq. slp) over one panel into
//     V phi_sigma (x) = (1/4pi) int_0^{2pi} L(phi) dphi,
//     L(phi) = |{ r >= |d| : (t - r, p + s(r) e(phi)) in sigma }|,
// the constant-integrand form of Lemma kernel_para.  Face k,
// a_k tau + b_k u + c_k v < h_k, becomes  B_k s - a_k r < C_k  with
// B_k = b_k cos phi + c_k sin phi and C_k = h_k - a_k t - b_k p_u - c_k p_v.
//
// Device evaluation of L uses w = r + s (so r = (w + d^2/w)/2, s =
// (w - d^2/w)/2, w >= |d|): face k is then the quadratic inequality
//     Q_k(w) = (B_k - a_k) w^2 - 2 C_k w - d^2 (B_k + a_k) < 0,
// whose two roots are both genuine (no squaring), with discriminant
// C_k^2 + d^2 (B_k^2 - a_k^2).  Opening up (B_k > a_k): an admissible
// interval; opening down: a hole.  L is the r-measure of the w-interval
// [w(r_lo), w(r_hi)] cut by the intervals, minus the holes.
#pragma once
#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#define STB_HD __host__ __device__

namespace stb {

constexpr double kPi = 3.14159265358979323846;
constexpr double kTwoPi = 6.28318530717958647692;
constexpr int kMaxBp = 48;        // breakpoints per (apex, panel) pair
constexpr int kMaxNg = 64;        // Gauss nodes per phi piece
// breakpoint hint tolerances (fractions of |t - tau_min| + panel size)
constexpr double kTangHint = 0.05;
constexpr double kVtxHint = 0.05;
constexpr double kFlatTol = 1e-10;
constexpr double kEdgeTol = 1e-10;   // edge parameters this close to [0, 1] are on the edge
constexpr double kLitDead = 1e-12;

// Per-panel record used when the panel is the trial panel (64 doubles).
struct TrialRec {
  // first 256 bytes: all the lit test's first pass reads
  double o[3], e1[3], e2[3], n[3];   // spatial frame of the panel plane
  double V[4][3];                    // vertices in local (tau, u, v)
  double tmin, tmax, diam;           // time range; max(spatial diam, span)
  double cx, cy, cz, rad;            // spatial bounding ball
  double pad;
  double fa[4], fb[4], fc[4], fh[4]; // unit outward face normals, offsets
  double X[4][4];                    // vertices (t, x, y, z)
};
// 512 bytes: every candidate's lane reads one record, so it is kept small
static_assert(sizeof(TrialRec) == 64 * sizeof(double), "TrialRec layout");
static_assert(offsetof(TrialRec, pad) == 31 * sizeof(double), "lit-test fields in two 128-byte lines");

// Bounding data of an apex set (the outer points of a test panel, or one
// evaluation point) for the conservative causal cull.
// Polar form of each face's spatial normal (b_k, c_k) = beta_k (cos phi_k,
// sin phi_k): B_k(phi) = beta_k cos(phi - phi_k).  Per panel, used by the
// breakpoints.
struct FaceAng {
  double phi[4], beta[4];
};

struct ApexBox {
  double tlo, thi;   // apex time range
  double cx, cy, cz; // centre of the spatial bounding ball
  double rho;        // its radius
  double pad[2];
};

struct Apex {
  double t, pu, pv, d;
  double C[4];
};

STB_HD __forceinline__ double dot3(const double* a, const double* b) {
  return a[0] * b[0] + a[1] * b[1] + a[2] * b[2];
}

// sin and cos of an angle of moderate size (|x| < 64 pi; here x in
// [0, 4 pi)): Cody-Waite reduction by pi/2 with a two-part pi/2, then the
// Taylor polynomials of sin (to x^17) and cos (to x^18) on [-pi/4, pi/4],
// whose truncation errors there are below 1e-17.
// a * b + c as one v_fma_f64 with the addend a polynomial coefficient in
// a scalar register pair (the one scalar operand a VOP3 instruction may
// take): the compiler otherwise copies the coefficient and uses the
// two-address v_fmac_f64, two instructions, and coefficients kept in vector
// registers across a loop cost the node kernels a wave per SIMD.
STB_HD __forceinline__ double fma_keep(double a, double b, double c) {
#if defined(__HIP_DEVICE_COMPILE__)
  double r;
  asm("v_fma_f64 %0, %1, %2, %3" : "=v"(r) : "v"(a), "v"(b), "s"(c));
  return r;
#else
  return fma(a, b, c);
#endif
}

STB_HD __forceinline__ void sincos_small(double x, double* s, double* c) {
  const double kInvPio2 = 0.63661977236758134308;
  const double kPio2Hi = 1.5707963267948966192e+00;   // nearest double to pi/2
  const double kPio2Lo = 6.1232339957367660359e-17;   // pi/2 - kPio2Hi
  double k = rint(x * kInvPio2);
  double r = fma(-k, kPio2Hi, x);
  r = fma(-k, kPio2Lo, r);
  double r2 = r * r;
  // sin r = r (1 - r^2/3! + r^4/5! - ...), cos r = 1 - r^2/2! + r^4/4! - ...
  double ps = -1.0 / 355687428096000.0;                 // -1/17!
  ps = fma_keep(ps, r2, 1.0 / 1307674368000.0);              //  1/15!
  ps = fma_keep(ps, r2, -1.0 / 6227020800.0);                // -1/13!
  ps = fma_keep(ps, r2, 1.0 / 39916800.0);                   //  1/11!
  ps = fma_keep(ps, r2, -1.0 / 362880.0);                    // -1/9!
  ps = fma_keep(ps, r2, 1.0 / 5040.0);                       //  1/7!
  ps = fma_keep(ps, r2, -1.0 / 120.0);                       // -1/5!
  ps = fma_keep(ps, r2, 1.0 / 6.0);                          //  1/3! (sign below)
  double sr = fma(-r * r2, ps, r);
  double pc = 1.0 / 6402373705728000.0;                 //  1/18!
  pc = fma_keep(pc, r2, -1.0 / 20922789888000.0);            // -1/16!
  pc = fma_keep(pc, r2, 1.0 / 87178291200.0);                //  1/14!
  pc = fma_keep(pc, r2, -1.0 / 479001600.0);                 // -1/12!
  pc = fma_keep(pc, r2, 1.0 / 3628800.0);                    //  1/10!
  pc = fma_keep(pc, r2, -1.0 / 40320.0);                     // -1/8!
  pc = fma_keep(pc, r2, 1.0 / 720.0);                        //  1/6!
  pc = fma_keep(pc, r2, -1.0 / 24.0);                        // -1/4!
  pc = fma_keep(pc, r2, 0.5);                                //  1/2! (sign below)
  double cr = fma(-r2, pc, 1.0);
  int q = ((int)k) & 3;
  double ss = (q & 1) ? cr : sr, cc = (q & 1) ? sr : cr;
  *s = (q & 2) ? -ss : ss;
  *c = (q == 1 || q == 2) ? -cc : cc;
}

// sin and cos for |x| <= pi/2 without the reduction: the Taylor polynomials
// to x^19 and x^20, whose truncation errors there are below 3e-16 and 2e-17.
STB_HD __forceinline__ void sincos_half_pi(double x, double* s, double* c) {
  const double x2 = x * x;
  double ps = -1.0 / 121645100408832000.0;                  // -1/19!
  ps = fma_keep(ps, x2, 1.0 / 355687428096000.0);            //  1/17!
  ps = fma_keep(ps, x2, -1.0 / 1307674368000.0);             // -1/15!
  ps = fma_keep(ps, x2, 1.0 / 6227020800.0);                 //  1/13!
  ps = fma_keep(ps, x2, -1.0 / 39916800.0);                  // -1/11!
  ps = fma_keep(ps, x2, 1.0 / 362880.0);                     //  1/9!
  ps = fma_keep(ps, x2, -1.0 / 5040.0);                      // -1/7!
  ps = fma_keep(ps, x2, 1.0 / 120.0);                        //  1/5!
  ps = fma_keep(ps, x2, -1.0 / 6.0);                         // -1/3!
  *s = fma(x * x2, ps, x);
  double pc = 1.0 / 2432902008176640000.0;                   //  1/20!
  pc = fma_keep(pc, x2, -1.0 / 6402373705728000.0);          // -1/18!
  pc = fma_keep(pc, x2, 1.0 / 20922789888000.0);             //  1/16!
  pc = fma_keep(pc, x2, -1.0 / 87178291200.0);               // -1/14!
  pc = fma_keep(pc, x2, 1.0 / 479001600.0);                  //  1/12!
  pc = fma_keep(pc, x2, -1.0 / 3628800.0);                   // -1/10!
  pc = fma_keep(pc, x2, 1.0 / 40320.0);                      //  1/8!
  pc = fma_keep(pc, x2, -1.0 / 720.0);                       // -1/6!
  pc = fma_keep(pc, x2, 1.0 / 24.0);                         //  1/4!
  pc = fma_keep(pc, x2, -0.5);                               // -1/2!
  *c = fma(x2, pc, 1.0);
}

STB_HD __forceinline__ double wrap_2pi(double a) {
  if (a < 0.0) a += kTwoPi;
  if (a < 0.0) a += kTwoPi;
  if (a >= kTwoPi) a -= kTwoPi;
  if (a >= kTwoPi) a -= kTwoPi;
  return a;
}

// The apex in the panel's frame (t, p_u, p_v, d), without the C_k.
STB_HD __forceinline__ void apex_frame(const TrialRec& T, const double* x4, Apex& A) {
  double v[3] = {x4[1] - T.o[0], x4[2] - T.o[1], x4[3] - T.o[2]};
  A.t = x4[0];
  A.pu = dot3(v, T.e1);
  A.pv = dot3(v, T.e2);
  A.d = dot3(v, T.n);
  // an apex in the panel's hyperplane up to rounding is taken exactly in it:
  // d of order 1e-17 would make C_k / d (tangency) meaningless
  if (fabs(A.d) <= kFlatTol * (fabs(A.t - T.tmin) + T.diam)) A.d = 0.0;
}

STB_HD __forceinline__ void apex_of(const TrialRec& T, const double* x4, Apex& A) {
  apex_frame(T, x4, A);
#pragma unroll
  for (int k = 0; k < 4; ++k) A.C[k] = T.fh[k] - T.fa[k] * A.t - T.fb[k] * A.pu - T.fc[k] * A.pv;
}

// w-interval of the admissible time range r in [max(|d|, t - tmax), t - tmin].
// Returns false when empty.
STB_HD __forceinline__ bool w_range(const TrialRec& T, const Apex& A, double& wlo,
                                        double& whi) {
  double ad = fabs(A.d);
  double rlo = fmax(ad, A.t - T.tmax);
  double rhi = A.t - T.tmin;
  if (!(rhi > rlo)) return false;
  wlo = rlo + sqrt(fmax((rlo - ad) * (rlo + ad), 0.0));
  whi = rhi + sqrt(fmax((rhi - ad) * (rhi + ad), 0.0));
  return true;
}

STB_HD __forceinline__ double r_of_w(double w, double d2) {
  return d2 > 0.0 ? 0.5 * (w + d2 / w) : 0.5 * w;
}

// 1/x to within an ulp for normal, finite, non-zero x: the hardware
// reciprocal estimate refined by two Newton steps (e = 1 - x r, r += r e).
// Much shorter than an IEEE division; every use below has |x| well inside
// the normal range.
STB_HD __forceinline__ double frcp(double x) {
#if defined(__HIP_DEVICE_COMPILE__)
  double r = __builtin_amdgcn_rcp(x);
#else
  double r = 1.0 / x;
#endif
  double e = fma(-x, r, 1.0);
  r = fma(r, e, r);
  e = fma(-x, r, 1.0);
  return fma(r, e, r);
}

// sqrt(max(D, 0)) of a face discriminant: v_rsq_f64, one Goldschmidt and
// one Newton step (about an ulp; the library's square root adds a second
// Newton step, range scaling and special-value selects).  D below 2^-900
// gives 0: its root, below 2^-450, is far under an ulp of the C_k it is
// added to.
STB_HD __forceinline__ double sqrt_disc(double D) {
  const bool pos = D > 0x1p-900;
#if defined(__HIP_DEVICE_COMPILE__)
  const double x = pos ? D : 1.0;
  const double y = __builtin_amdgcn_rsq(x);
  double g = x * y, h = 0.5 * y;
  const double r = fma(-g, h, 0.5);
  g = fma(g, r, g);
  h = fma(h, r, h);
  g = fma(fma(-g, g, x), h, g);
  return pos ? g : 0.0;
#else
  return pos ? sqrt(D) : 0.0;
#endif
}

// sqrt of a non-negative value to about an ulp (sqrt_disc's sequence; the
// library's correctly rounded square root adds range scaling and special
// cases, about twice the instructions).  Used where a decision has a
// tolerance far above an ulp (lit tests, edge events, tangencies).
STB_HD __forceinline__ double sqrt_nn(double x) { return sqrt_disc(x); }

// sqrt to about 1e-7 relative: for tolerances only.
STB_HD __forceinline__ double sqrt_rough(double x) {
#if defined(__HIP_DEVICE_COMPILE__)
  return x > 0.0 ? x * __builtin_amdgcn_rsq(x) : 0.0;
#else
  return sqrt(x);
#endif
}

// r(w1) - r(w0) = (w1 - w0) (1 - d^2 / (w0 w1)) / 2 for w1 >= w0 > 0 (or
// d^2 = 0, where w0 may be 0).
STB_HD __forceinline__ double rdiff(double w0, double w1, double d2) {
  // the ends lie in the admissible range, so w0 w1 >= d^2 when d != 0; the
  // floor 2^-1000 acts only at d = 0 (or in an empty range, whose measure
  // is not used), where it keeps 1 / (w0 w1) finite and the factor exactly 1
  double h = 0.5 * (w1 - w0);
  double g = fma(-d2, frcp(fmax(w0 * w1, 0x1p-1000)), 1.0);
  return h * g;
}

// Face data needed by L(phi): fa, fb, fc of the 4 faces.
struct FaceSet {
  double fa[4], fb[4], fc[4];
};

// Order two intervals by start (registers only, selects).
STB_HD __forceinline__ void order2(double& s0, double& e0, double& s1, double& e1) {
  bool sw = s1 < s0;
  double ts = s0, te = e0;
  s0 = sw ? s1 : s0;
  e0 = sw ? e1 : e0;
  s1 = sw ? ts : s1;
  e1 = sw ? te : e1;
}

// L(phi) for cos/sin of phi.  C: C_k, d2 = d^2, [wlo, whi]: admissible w-range.
//
// In w = r + sqrt(r^2 - d^2) face k's constraint reads
//   Q_k(w) = (B_k - a_k) w^2 - 2 C_k w - d^2 (B_k + a_k) < 0,  w >= |d|.
// With e = B_k - a_k, f = B_k + a_k, D = C_k^2 + d^2 e f and
// q = C_k + sign(C_k) sqrt(D), the roots are q / e and -d^2 f / q (the
// second is the root of the linear case e = 0).  e > 0: the admissible set
// is the open interval between the roots (empty when D <= 0); e < 0: the
// complement of that interval (all of w when D <= 0); e = 0: a half-line
// w > root (C_k > 0) or w < root (C_k < 0), or all / nothing (C_k = 0).
// L is the r-measure of [wlo, whi] intersected with every face's set.
//
// Branch-free: every face takes the same instructions and selects the
// outcome, so lanes evaluating different pairs do not diverge.  Holes (e < 0)
// are clipped to the admissible interval, sorted by start and swept once.
STB_HD __forceinline__ double L_eval(const FaceSet& F, const double* C, double d2, double wlo,
                                     double whi, double cs, double sn) {
  const double kNone = 1e300;
  double lo = wlo, hi = whi;
  bool dead = false;
  double hs[4], he[4];
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    double a = F.fa[k];
    double B = fma(F.fb[k], cs, F.fc[k] * sn);
    double e = B - a, f = B + a, Ck = C[k];
    double D = fma(Ck, Ck, d2 * (e * f));
    bool two = D > 0.0;
    double q = Ck + copysign(sqrt_disc(D), Ck);
    double w1 = q * frcp(e);
    double w2 = -d2 * f * frcp(q);
    double mn = fmin(w1, w2), mx = fmax(w1, w2);
    bool pos = e > 0.0, neg = e < 0.0, zer = !(pos || neg);
    bool cut = pos && two;
    dead = dead || (pos && !two) || (zer && Ck == 0.0 && !(d2 * f > 0.0));
    lo = cut ? fmax(lo, mn) : lo;
    hi = cut ? fmin(hi, mx) : hi;
    lo = (zer && Ck > 0.0) ? fmax(lo, w2) : lo;
    hi = (zer && Ck < 0.0) ? fmin(hi, w2) : hi;
    bool hole = neg && two;
    hs[k] = hole ? mn : kNone;
    he[k] = hole ? mx : kNone;
  }
  // clip the holes to [lo, hi] (absent ones become [hi, hi]), sort by start
  // (five compare-exchanges), then sweep and add the gaps between them: a sum
  // of non-negative measures, exactly 0 when the holes cover [lo, hi]
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    hs[k] = fmin(fmax(hs[k], lo), hi);
    he[k] = fmax(fmin(he[k], hi), hs[k]);
  }
  order2(hs[0], he[0], hs[1], he[1]);
  order2(hs[2], he[2], hs[3], he[3]);
  order2(hs[0], he[0], hs[2], he[2]);
  order2(hs[1], he[1], hs[3], he[3]);
  order2(hs[1], he[1], hs[2], he[2]);
  // A gap whose r-measure is below kWulp * w (4 ulp of w) is a rounding
  // artefact, e.g. [|d|, |d| + a few ulp] where two roots meet at the
  // hyperbola's vertex (r is flat in w there: measure ~1e-30), and counts
  // as empty.
  const double kWulp = 8.881784197001252e-16;
  double len = 0.0, c = lo;
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    double g1 = fmax(hs[k], c);
    double m = rdiff(c, g1, d2);
    len += (m > kWulp * g1) ? m : 0.0;
    c = fmax(he[k], c);
  }
  double m = rdiff(c, hi, d2);
  len += (m > kWulp * hi) ? m : 0.0;
  bool empty = dead || !(hi > lo);
  return empty ? 0.0 : len;
}

// The double layer's r-integrals at one angle, over the same admissible set
// as L_eval: for every gap [w0, w1] of it (r0 = r(w0), r1 = r(w1)),
//   sa += 1/r0 - 1/r1 = 2 w0 / (w0^2 + d^2) - 2 w1 / (w1^2 + d^2),
//   sh += H(r1) - H(r0),  H(r) = ln(r + s) - s / r = ln w - 1 + 2 d^2 / (w^2 + d^2),
// the integrals of 1/r^2 and of s/r^2 over r (s = sqrt(r^2 - d^2), so that
// r + s = w and s / r = (w^2 - d^2) / (w^2 + d^2)).  Needs d^2 > 0.  Same
// holes, clipping, sort and gap threshold as L_eval, so that both see the
// same set.
STB_HD inline void dl_eval(const FaceSet& F, const double* C, double d2, double wlo, double whi,
                           double cs, double sn, double& sa, double& sh) {
  const double kNone = 1e300;
  double lo = wlo, hi = whi;
  bool dead = false;
  double hs[4], he[4];
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    double a = F.fa[k];
    double B = fma(F.fb[k], cs, F.fc[k] * sn);
    double e = B - a, f = B + a, Ck = C[k];
    double D = fma(Ck, Ck, d2 * (e * f));
    bool two = D > 0.0;
    double q = Ck + copysign(sqrt_disc(D), Ck);
    double w1 = q * frcp(e);
    double w2 = -d2 * f * frcp(q);
    double mn = fmin(w1, w2), mx = fmax(w1, w2);
    bool pos = e > 0.0, neg = e < 0.0, zer = !(pos || neg);
    bool cut = pos && two;
    dead = dead || (pos && !two) || (zer && Ck == 0.0 && !(d2 * f > 0.0));
    lo = cut ? fmax(lo, mn) : lo;
    hi = cut ? fmin(hi, mx) : hi;
    lo = (zer && Ck > 0.0) ? fmax(lo, w2) : lo;
    hi = (zer && Ck < 0.0) ? fmin(hi, w2) : hi;
    bool hole = neg && two;
    hs[k] = hole ? mn : kNone;
    he[k] = hole ? mx : kNone;
  }
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    hs[k] = fmin(fmax(hs[k], lo), hi);
    he[k] = fmax(fmin(he[k], hi), hs[k]);
  }
  order2(hs[0], he[0], hs[1], he[1]);
  order2(hs[2], he[2], hs[3], he[3]);
  order2(hs[0], he[0], hs[2], he[2]);
  order2(hs[1], he[1], hs[3], he[3]);
  order2(hs[1], he[1], hs[2], he[2]);
  const double kWulp = 8.881784197001252e-16;
  sa = 0.0;
  sh = 0.0;
  if (dead || !(hi > lo)) return;
  auto gap = [&](double w0, double w1) {
    double m = rdiff(w0, w1, d2);
    if (!(m > kWulp * w1)) return;
    double q0 = 1.0 / fma(w0, w0, d2), q1 = 1.0 / fma(w1, w1, d2);
    sa += 2.0 * (w0 * q0 - w1 * q1);
    sh += log(w1 / w0) + 2.0 * d2 * (q1 - q0);
  };
  double c = lo;
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    gap(c, fmax(hs[k], c));
    c = fmax(he[k], c);
  }
  gap(c, hi);
}

// Exact extrema of f(y) = |x - y| - (t - tau) over the closed panel:
// max at a vertex; min among vertices, stationary points on the 6 edges and
// in the non-vertical faces.  Returns the lit decision with the relative
// dead zone kLitDead * (|t - tmin| + diam).
// The cheap part of the lit decision: 0 = not lit (cone misses the panel's
// time slab, bounding-ball rejection, or every vertex inside the cone),
// 1 = lit (a vertex strictly inside and one strictly outside), 2 = the
// vertices do not decide (lit_test's edge and face minima must).
STB_HD inline int lit_quick(const TrialRec& T, const double* x4, const Apex& A);

STB_HD inline bool lit_test(const TrialRec& T, const double* x4, const Apex& A) {
  double mn = 1e300, mx = -1e300;
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    double dx = x4[1] - T.X[k][1], dy = x4[2] - T.X[k][2], dz = x4[3] - T.X[k][3];
    double f = sqrt_nn(dx * dx + dy * dy + dz * dz) - (x4[0] - T.X[k][0]);
    mn = fmin(mn, f);
    mx = fmax(mx, f);
  }
  double dead = kLitDead * (fabs(A.t - T.tmin) + T.diam);
  if (!(mx > dead)) return false;
  if (mn < -dead) return true;     // a vertex inside the cone already decides
  for (int i = 0; i < 4; ++i)
    for (int j = i + 1; j < 4; ++j) {
      double U[3] = {T.X[j][1] - T.X[i][1], T.X[j][2] - T.X[i][2], T.X[j][3] - T.X[i][3]};
      double P[3] = {T.X[i][1] - x4[1], T.X[i][2] - x4[2], T.X[i][3] - x4[3]};
      double Dt = T.X[j][0] - T.X[i][0];
      double a = dot3(U, U), b = 2.0 * dot3(P, U);
      double g = a - Dt * Dt;
      if (!(a > 0.0 && g > 0.0)) continue;
      double cr0 = P[1] * U[2] - P[2] * U[1];
      double cr1 = P[2] * U[0] - P[0] * U[2];
      double cr2 = P[0] * U[1] - P[1] * U[0];
      const double ra2 = frcp(2.0 * a);
      double hw = fabs(Dt) * ra2 * sqrt_nn(4.0 * (cr0 * cr0 + cr1 * cr1 + cr2 * cr2) * frcp(g));
      double lc = -b * ra2;
#pragma unroll
      for (int m = 0; m < 2; ++m) {
        double l = m ? lc + hw : lc - hw;
        if (!(l > 0.0 && l < 1.0)) continue;
        double y0 = T.X[i][0] + l * Dt;
        double y1 = P[0] + l * U[0], y2 = P[1] + l * U[1], y3 = P[2] + l * U[2];
        double f = sqrt_nn(y1 * y1 + y2 * y2 + y3 * y3) - (x4[0] - y0);
        mn = fmin(mn, f);
      }
    }
  // faces: tau linear over the face's spatial triangle with gradient g;
  // stationary point y = p - g |d| / sqrt(1 - |g|^2) when |g| < 1
  double sc2 = T.diam * T.diam;
  for (int k = 0; k < 4; ++k) {
    int i0 = k == 0 ? 1 : 0;
    int i1 = k <= 1 ? 2 : 1;
    int i2 = k <= 2 ? 3 : 2;
    const double* V0 = T.V[i0];
    double Uu = T.V[i1][1] - V0[1], Uv = T.V[i1][2] - V0[2];
    double Wu = T.V[i2][1] - V0[1], Wv = T.V[i2][2] - V0[2];
    double D1 = T.V[i1][0] - V0[0], D2 = T.V[i2][0] - V0[0];
    double det = Uu * Wv - Uv * Wu;
    if (!(fabs(det) > 1e-12 * sc2)) continue;
    const double rdet = frcp(det);
    double gu = (D1 * Wv - D2 * Uv) * rdet;
    double gv = (Uu * D2 - Wu * D1) * rdet;
    double g2 = gu * gu + gv * gv;
    if (!(g2 < 1.0)) continue;
    double fac = fabs(A.d) * frcp(sqrt_nn(1.0 - g2));
    double yu = A.pu - gu * fac, yv = A.pv - gv * fac;
    double ru = yu - V0[1], rv = yv - V0[2];
    double al = (ru * Wv - rv * Wu) * rdet;
    double be = (Uu * rv - Uv * ru) * rdet;
    if (!(al >= 0.0 && be >= 0.0 && al + be <= 1.0)) continue;
    double tau = V0[0] + gu * ru + gv * rv;
    double du = A.pu - yu, dv = A.pv - yv;
    double f = sqrt_nn(du * du + dv * dv + A.d * A.d) - (A.t - tau);
    mn = fmin(mn, f);
  }
  return mn < -dead;
}

STB_HD __forceinline__ bool ball_rejects(const TrialRec& T, const double* x4);

// First pass of the lit test from the apex's frame (apex_frame) and the
// panel's local vertices: the record's first 256 bytes only.
STB_HD inline int lit_quick(const TrialRec& T, const double* x4, const Apex& A) {
  if (!(A.t - T.tmin > fabs(A.d))) return 0;
  if (ball_rejects(T, x4)) return 0;
  double mn = 1e300, mx = -1e300;
  const double d2 = A.d * A.d;
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    double du = A.pu - T.V[k][1], dv = A.pv - T.V[k][2];
    double f = sqrt_nn(du * du + dv * dv + d2) - (A.t - T.V[k][0]);
    mn = fmin(mn, f);
    mx = fmax(mx, f);
  }
  double dead = kLitDead * (fabs(A.t - T.tmin) + T.diam);
  if (!(mx > dead)) return 0;
  if (mn < -dead) return 1;
  return 2;
}

// Quick rejection by the bounding 4-ball of the panel (Theorem
// phi_xi_sphere): over the closed ball B_r(y), y = (tau_c, c), the cone
// function phi_Xi(x - z) ranges exactly over [phi - d_r(|x - c|),
// phi + r sqrt 2] with phi = phi_Xi(x - y).  A ball entirely inside or
// outside the cone (beyond a small margin) cannot be lit; otherwise the
// exact test decides.
STB_HD __forceinline__ bool ball_rejects(const TrialRec& T, const double* x4) {
  const double s2 = 1.4142135623730951;
  double tc = 0.5 * (T.tmin + T.tmax), ht = 0.5 * (T.tmax - T.tmin);
  double r = sqrt_nn(T.rad * T.rad + ht * ht) * (1.0 + 1e-12);
  double dx = x4[1] - T.cx, dy = x4[2] - T.cy, dz = x4[3] - T.cz;
  double al = sqrt_nn(dx * dx + dy * dy + dz * dz);
  double phi = al - (x4[0] - tc);
  double dr = al < r * (1.0 / s2) ? al + sqrt_nn(r * r - al * al) : r * s2;
  double margin = 1e-9 * (fabs(x4[0] - T.tmin) + T.diam);
  return (phi + r * s2 < -margin) || (phi - dr > margin);
}

// atan2 for breakpoint angles (range (-pi, pi]).  With t = min/max of |x|,
// |y| in [0, 1] and c the multiple of 1/4 nearest to t,
//   atan t = atan c + atan u,  u = (t - c) / (1 + t c) = (min - c max) / (max + c min),
// |u| <= 1/8, and atan u is its odd Taylor series to u^17 (remainder below
// u^19 / 19 < 4e-19).  atan c is a table of three values in two parts
// each; the octant follows from |y| > |x|, x < 0 and the sign of y.
// Absolute error about 2e-16; one quotient instead of the library's range
// reduction with several.
STB_HD __forceinline__ double atan2_bp(double y, double x) {
  const double ax = fabs(x), ay = fabs(y);
  const double mx = fmax(ax, ay), mn = fmin(ax, ay);
#if defined(__HIP_DEVICE_COMPILE__)
  const double tq = mn * __builtin_amdgcn_rcp(mx);   // only picks c
#else
  const double tq = mn / mx;
#endif
  const double i = rint(4.0 * tq);
  const double c = 0.25 * i;
  const double u = fma(-c, mx, mn) * frcp(fma(c, mn, mx));
  const double u2 = u * u;
  double p = 1.0 / 17.0;
  p = fma_keep(p, u2, -1.0 / 15.0);
  p = fma_keep(p, u2, 1.0 / 13.0);
  p = fma_keep(p, u2, -1.0 / 11.0);
  p = fma_keep(p, u2, 1.0 / 9.0);
  p = fma_keep(p, u2, -1.0 / 7.0);
  p = fma_keep(p, u2, 1.0 / 5.0);
  p = fma_keep(p, u2, -1.0 / 3.0);
  const double au = fma(u * u2, p, u);
  // atan(i / 4), high and low parts
  const double th_hi = i < 0.5 ? 0.0 : i < 1.5 ? 0.24497866312686414 : i < 2.5 ? 0.4636476090008061
                     : i < 3.5 ? 0.6435011087932844 : 0.7853981633974483;
  const double th_lo = i < 0.5 ? 0.0 : i < 1.5 ? 1.0699e-17 : i < 2.5 ? 2.2699e-17
                     : i < 3.5 ? 1.5835e-17 : 3.0616e-17;
  double th = th_hi + (au + th_lo);                        // atan(mn / mx), [0, pi/4]
  th = ay > ax ? (1.5707963267948966 - th) + 6.123233995736766e-17 : th;
  th = x < 0.0 ? (3.141592653589793 - th) + 1.2246467991473532e-16 : th;
  th = copysign(th, y);
  return mx > 0.0 ? th : 0.0;
}

// acos x = atan2(sqrt((1 - x)(1 + x)), x) for x in [-1, 1].
STB_HD __forceinline__ double acos_bp(double x) {
  return atan2_bp(sqrt_nn((1.0 - x) * (1.0 + x)), x);
}

// Stable roots of qa l^2 + qb l + qc = 0; returns count.  Quotients by the
// refined reciprocal (within an ulp; the correctly rounded division costs
// registers that limit the breakpoint kernel's occupancy).
STB_HD __forceinline__ int roots2(double qa, double qb, double qc, double* r) {
  // every case computed and selected: a lane-divergent branch per case costs
  // the breakpoint kernel more than the arithmetic
  const bool lin = qa == 0.0;
  const double disc = qb * qb - 4.0 * qa * qc;
  const bool neg = disc < 0.0;
  const bool near = disc >= -1e-12 * (qb * qb + fabs(4.0 * qa * qc));
  const double q = -0.5 * (qb + copysign(sqrt_nn(disc), qb));
  const double rqa = frcp(lin ? 1.0 : qa);
  const double rq = frcp(q == 0.0 ? 1.0 : q);
  double r0 = q * rqa, r1 = qc * rq;
  int n = 2;
  r0 = q == 0.0 ? 0.0 : r0;
  n = q == 0.0 ? 1 : n;
  r0 = neg ? -0.5 * qb * rqa : r0;
  n = neg ? (near ? 1 : 0) : n;
  // linear (qa = 0): disc = qb^2, q = -qb up to the square root's rounding,
  // so qc / q is the root -qc / qb
  r0 = lin ? r1 : r0;
  n = lin ? (qb == 0.0 ? 0 : 1) : n;
  r[0] = r0;
  r[1] = r1;
  return n;
}

// Breakpoints of L (unsorted); returns count (<= kMaxBp).  The set is the
// phi-rule's definition: edge events; tangencies within kTangHint of the
// closed panel; B_k = 0 where the hyperboloid vertex is within kVtxHint of
// face k's plane; B_k = a_k for an apex on face k's plane inside the
// panel's hyperplane (d = 0, C_k = 0).
STB_HD inline void face_angles(const TrialRec& T, FaceAng& F) {
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    F.beta[k] = sqrt(T.fb[k] * T.fb[k] + T.fc[k] * T.fc[k]);
    F.phi[k] = atan2(T.fc[k], T.fb[k]);
  }
}

// Breakpoint storage: a plain array, or (the breakpoint kernel) slots in
// LDS with the rare overflow in private memory.  put/get by slot index.
struct BpArray {
  double* a;
  STB_HD __forceinline__ void put(int i, double v) { a[i] = v; }
  STB_HD __forceinline__ double get(int i) const { return a[i]; }
};

template <class BP>
STB_HD inline int breakpoints_t(const TrialRec& T, const FaceAng& FA, const Apex& A, BP& bp) {
  int nb = 0;
  double d2 = A.d * A.d, ad = fabs(A.d);
  const double rd2 = d2 > 0.0 ? frcp(d2) : 0.0;   // for the tangency test
  double sc = fabs(A.t - T.tmin) + T.diam;
  // cone function at the vertices: an edge with both ends strictly inside
  // the backward cone (a convex set) cannot meet it
  double fv[4];
  for (int k = 0; k < 4; ++k) {
    double du = T.V[k][1] - A.pu, dv = T.V[k][2] - A.pv;
    fv[k] = sqrt_nn(du * du + dv * dv + d2) - (A.t - T.V[k][0]);
  }
  const double inside = -1e-9 * sc;
  // edge events (at most 12): the in-plane offsets (ou, ov) first, kept in
  // slots m and 12 + m, then their angles in one loop
  int nh = 0;
  for (int i = 0; i < 4; ++i)
    for (int j = i + 1; j < 4; ++j) {
      const bool skip = fv[i] < inside && fv[j] < inside;
      double a0 = A.t - T.V[i][0], a1 = T.V[i][0] - T.V[j][0];
      double bu = T.V[i][1] - A.pu, bv = T.V[i][2] - A.pv;
      double du = T.V[j][1] - T.V[i][1], dv = T.V[j][2] - T.V[i][2];
      double qa = a1 * a1 - du * du - dv * dv;
      double qb = 2.0 * (a0 * a1 - bu * du - bv * dv);
      double qc = a0 * a0 - bu * bu - bv * bv - d2;
      double lam[2];
      int nl = roots2(qa, qb, qc, lam);
      nl = skip ? 0 : nl;
#pragma unroll
      for (int m = 0; m < 2; ++m) {
        double l = lam[m];
        bool ok = m < nl && (l >= -kEdgeTol && l <= 1.0 + kEdgeTol);
        l = fmin(fmax(l, 0.0), 1.0);
        ok = ok && !(a0 + a1 * l < 0.0);
        double ou = bu + l * du, ov = bv + l * dv;
        ok = ok && !(ou * ou + ov * ov <= 1e-20 * sc * sc);
        if (ok) {
          bp.put(nh, ou);
          bp.put(12 + nh, ov);
          ++nh;
        }
      }
    }
  for (int m = 0; m < nh; ++m) bp.put(m, wrap_2pi(atan2_bp(bp.get(12 + m), bp.get(m))));
  nb = nh;
  for (int k = 0; k < 4; ++k) {
    double a = T.fa[k], b = T.fb[k], c = T.fc[k], Ck = A.C[k];
    double beta = FA.beta[k];
    if (!(beta > 1e-12)) continue;
    double phik = FA.phi[k];
    if (d2 > 0.0) {
      double rhs = a * a - Ck * Ck * rd2;
      if (rhs >= 0.0 && rhs <= beta * beta) {
        const double rb = frcp(beta);
        double cv = fmin(sqrt_nn(rhs) * rb, 1.0);
        double g = acos_bp(cv);
        // candidates phi_k + g, phi_k - g, phi_k + pi - g, phi_k + pi + g;
        // their directions from (cos, sin) of phi_k = (b, c) / beta and of
        // g = (cv, sqrt(1 - cv^2)) by the addition theorems
        const double cp = b * rb, sp = c * rb, sg = sqrt_nn((1.0 - cv) * (1.0 + cv));
        const double c1 = cp * cv - sp * sg, s1 = sp * cv + cp * sg;   // phi_k + g
        const double c2 = cp * cv + sp * sg, s2 = sp * cv - cp * sg;   // phi_k - g
#pragma unroll 1
        for (int m = 0; m < 4; ++m) {
          const bool pg = m == 0 || m == 3;             // + g
          const double sgn = m < 2 ? 1.0 : -1.0;        // + pi: opposite direction
          const double cs = sgn * (pg ? c1 : c2), sn = sgn * (pg ? s1 : s2);
          const double cand = (m < 2 ? phik : phik + kPi) + (pg ? g : -g);
          double e = b * cs + c * sn - a;
          if (e == 0.0) continue;
          double wt = Ck * frcp(e);           // double root of Q_k
          if (!(wt >= ad) || !(wt > 0.0)) continue;
          const double rw = frcp(wt);
          double rt = d2 > 0.0 ? 0.5 * (wt + d2 * rw) : 0.5 * wt, st = 0.5 * (wt - d2 * rw);
          double y0 = A.t - rt, y1 = A.pu + st * cs, y2 = A.pv + st * sn;
          double worst = -1e300;
#pragma unroll
          for (int m2 = 0; m2 < 4; ++m2)
            worst = fmax(worst, T.fa[m2] * y0 + T.fb[m2] * y1 + T.fc[m2] * y2 - T.fh[m2]);
          if (worst <= kTangHint * sc) bp.put(nb++, wrap_2pi(cand));
        }
      }
    }
    if (fabs(a * ad + Ck) <= kVtxHint * sc) {
      bp.put(nb++, wrap_2pi(phik + 0.5 * kPi));
      bp.put(nb++, wrap_2pi(phik - 0.5 * kPi));
    }
    if (ad <= kFlatTol * sc && fabs(Ck) <= kFlatTol * sc && fabs(a) <= beta) {
      double g = acos_bp(fmax(-1.0, fmin(1.0, a / beta)));
      bp.put(nb++, wrap_2pi(phik + g));
      bp.put(nb++, wrap_2pi(phik - g));
    }
  }
  return nb;
}

STB_HD inline int breakpoints(const TrialRec& T, const FaceAng& FA, const Apex& A, double* bp) {
  BpArray a{bp};
  return breakpoints_t(T, FA, A, a);
}

// A direction whose ray from the apex's projection (pu, pv) misses the
// panel's spatial shadow (the hull of its vertices' (u, v)) carries no part
// of the panel, so L = 0 there.  Sufficient test with a margin tol: every
// vertex strictly on one side of the ray's line, or strictly behind it.
STB_HD __forceinline__ bool ray_misses(const TrialRec& T, const Apex& A, double cs, double sn,
                                       double tol) {
  bool left = true, right = true, behind = true;
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    double du = T.V[k][1] - A.pu, dv = T.V[k][2] - A.pv;
    double cr = cs * dv - sn * du, dt = cs * du + sn * dv;
    left = left && cr > tol;
    right = right && cr < -tol;
    behind = behind && dt < -tol;
  }
  return left || right || behind;
}

// The empty-piece test's three points (mid, then the quarter points) all
// on rays that miss the panel: the piece is empty without evaluating L.
// The quarter points' directions are the midpoint's turned by -+ H/4.
STB_HD __forceinline__ bool piece_misses(const TrialRec& T, const Apex& A, double a, double H) {
  const double tol = 1e-10 * (fabs(A.t - T.tmin) + T.diam);
  double sm, cm;
  sincos_small(a + 0.5 * H, &sm, &cm);
  if (!ray_misses(T, A, cm, sm, tol)) return false;
  double sh, ch;
  sincos_small(0.25 * H, &sh, &ch);
  const double cc = cm * ch, ss = sm * sh, sc = sm * ch, cs = cm * sh;
  return ray_misses(T, A, cc + ss, sc - cs, tol) && ray_misses(T, A, cc - ss, sc + cs, tol);
}

// The same question for every piece of a pair at once, in angle space.  When
// the foot point p lies outside the shadow, the directions whose rays meet
// the shadow form one wedge [lo, lo + w] (w < pi) between its two extreme
// vertex directions; a direction more than kWedgeMargin outside it misses
// the shadow by a margin far above rounding.  One wedge per pair (two
// arctangents) replaces a sin/cos and up to three ray tests per piece.  No
// wedge (every piece is evaluated) when p is inside the shadow, on or near
// its boundary, or within 1e-4 (|t - tmin| + diam) of a vertex, where the
// vertex directions are not resolved.
constexpr double kWedgeMargin = 1e-8;

// The directions that miss, as an arc: from ms = lo + w + kWedgeMargin
// over len = 2 pi - w - 2 kWedgeMargin.
struct ShadowWedge {
  double ms, len;
  bool ok;
};

STB_HD __forceinline__ ShadowWedge shadow_wedge(const TrialRec& T, const Apex& A) {
  const double sc = fabs(A.t - T.tmin) + T.diam;
  double du[4], dv[4], n2[4];
  bool nearp = false;
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    du[k] = T.V[k][1] - A.pu;
    dv[k] = T.V[k][2] - A.pv;
    n2[k] = du[k] * du[k] + dv[k] * dv[k];
    nearp = nearp || n2[k] < 1e-8 * sc * sc;
  }
  // the clockwise extreme: no vertex clockwise of it; the counterclockwise
  // extreme: none counterclockwise of it (cross products, collinear allowed)
  double ulo = 0.0, vlo = 0.0, uhi = 0.0, vhi = 0.0;
  bool flo = false, fhi = false;
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    bool first = true, last = true;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const double cr = du[i] * dv[k] - dv[i] * du[k];
      const double tol = 1e-12 * sqrt_rough(n2[i] * n2[k]);
      first = first && cr >= -tol;
      last = last && cr <= tol;
    }
    const bool tlo = first && !flo, thi = last && !fhi;
    ulo = tlo ? du[i] : ulo;
    vlo = tlo ? dv[i] : vlo;
    uhi = thi ? du[i] : uhi;
    vhi = thi ? dv[i] : vhi;
    flo = flo || first;
    fhi = fhi || last;
  }
  ShadowWedge W{0.0, 0.0, false};
  if (nearp || !flo || !fhi) return W;
  const double lo = atan2_bp(vlo, ulo);
  double w = atan2_bp(vhi, uhi) - lo;
  w = w < 0.0 ? w + kTwoPi : w;
  W.ms = lo + w + kWedgeMargin;
  W.len = kTwoPi - w - 2.0 * kWedgeMargin;
  W.ok = w < kPi - 1e-6;
  return W;
}

// piece_misses by the wedge: the piece's quarter points and midpoint all on
// the missing arc.  With u the first quarter point's offset along the arc
// (reduced mod 2 pi), that is 0 < u and u + H / 2 < len: one reduction
// instead of three.  Every miss it finds is one of the three points
// tested separately; the converse fails only when the whole wedge lies
// between two of the points, and such a piece is kept and evaluated.
STB_HD __forceinline__ bool wedge_misses(const ShadowWedge& W, double a, double H) {
  double u = fma(0.25, H, a) - W.ms;
  u -= kTwoPi * floor(u * (1.0 / kTwoPi));
  return W.ok & (u > 0.0) & (fma(0.5, H, u) < W.len);
}

// Sorts a[0..n) for n <= M (M a power of 2): into registers (padded with
// +inf), Batcher's odd-even merge network, back -- independent loads and
// stores instead of the insertion sort's dependent chain through memory.
template <int M, class BP>
STB_HD __forceinline__ void sort_net(BP& a, int n) {
  double r[M];
#pragma unroll
  for (int j = 0; j < M; ++j) r[j] = j < n ? a.get(j) : HUGE_VAL;
#pragma unroll
  for (int p = 1; p < M; p <<= 1)
#pragma unroll
    for (int k = p; k >= 1; k >>= 1)
#pragma unroll
      for (int j = k % p; j + k < M; j += 2 * k)
#pragma unroll
        for (int i = 0; i < k && i + j + k < M; ++i)
          if ((i + j) / (2 * p) == (i + j + k) / (2 * p)) {
            const double lo = fmin(r[i + j], r[i + j + k]);
            const double hi = fmax(r[i + j], r[i + j + k]);
            r[i + j] = lo;
            r[i + j + k] = hi;
          }
#pragma unroll
  for (int j = 0; j < M; ++j)
    if (j < n) a.put(j, r[j]);
}

// Sorts a[0..n).  Up to 16 values (nearly every (apex, panel) pair) by the
// network; more by insertion.
template <class BP>
STB_HD __forceinline__ void sort_bp_t(BP& a, int n) {
  if (n <= 16) {
    sort_net<16>(a, n);
    return;
  }
  for (int i = 1; i < n; ++i) {
    double v = a.get(i);
    int j = i - 1;
    while (j >= 0 && a.get(j) > v) { a.put(j + 1, a.get(j)); --j; }
    a.put(j + 1, v);
  }
}

STB_HD __forceinline__ void sort_bp(double* a, int n) {
  BpArray b{a};
  sort_bp_t(b, n);
}

// Panel geometry from its 4 vertices (t, x, y, z).  Returns 0, or 2 for a
// degenerate spatial projection, 3 for a panel that is not vertical (its
// spatial projection is not planar), 4 for zero 3-volume.
STB_HD inline int make_trial(const double (&X)[4][4], TrialRec& R) {
  // e1 along the farthest pair of spatial points
  int ia = 0, ib = 1;
  double best = -1.0;
  for (int a = 0; a < 4; ++a)
    for (int b = a + 1; b < 4; ++b) {
      double dx = X[b][1] - X[a][1], dy = X[b][2] - X[a][2], dz = X[b][3] - X[a][3];
      double l2 = dx * dx + dy * dy + dz * dz;
      if (l2 > best) { best = l2; ia = a; ib = b; }
    }
  if (!(best > 0.0)) return 2;
  double dsp = sqrt(best);
  double e1[3] = {(X[ib][1] - X[ia][1]) / dsp, (X[ib][2] - X[ia][2]) / dsp,
                  (X[ib][3] - X[ia][3]) / dsp};
  double nb = -1.0, n[3] = {0, 0, 0};
  for (int c = 0; c < 4; ++c) {
    if (c == ia || c == ib) continue;
    double v[3] = {X[c][1] - X[ia][1], X[c][2] - X[ia][2], X[c][3] - X[ia][3]};
    double cr[3] = {e1[1] * v[2] - e1[2] * v[1], e1[2] * v[0] - e1[0] * v[2],
                    e1[0] * v[1] - e1[1] * v[0]};
    double l = sqrt(dot3(cr, cr));
    if (l > nb) { nb = l; n[0] = cr[0] / l; n[1] = cr[1] / l; n[2] = cr[2] / l; }
  }
  if (!(nb > 1e-12 * dsp)) return 2;
  double e2[3] = {n[1] * e1[2] - n[2] * e1[1], n[2] * e1[0] - n[0] * e1[2],
                  n[0] * e1[1] - n[1] * e1[0]};
  for (int c = 0; c < 3; ++c) {
    R.o[c] = X[ia][c + 1]; R.e1[c] = e1[c]; R.e2[c] = e2[c]; R.n[c] = n[c];
  }
  R.tmin = X[0][0]; R.tmax = X[0][0];
  double cen[3] = {0, 0, 0};
  for (int k = 0; k < 4; ++k) {
    double v[3] = {X[k][1] - R.o[0], X[k][2] - R.o[1], X[k][3] - R.o[2]};
    if (fabs(dot3(v, n)) > 1e-12 * dsp) return 3;
    R.V[k][0] = X[k][0];
    R.V[k][1] = dot3(v, e1);
    R.V[k][2] = dot3(v, e2);
    for (int c = 0; c < 4; ++c) R.X[k][c] = X[k][c];
    R.tmin = fmin(R.tmin, X[k][0]);
    R.tmax = fmax(R.tmax, X[k][0]);
    for (int c = 0; c < 3; ++c) cen[c] += 0.25 * X[k][c + 1];
  }
  R.diam = fmax(dsp, R.tmax - R.tmin);
  double a1[3], a2[3], a3[3];
  for (int c = 0; c < 3; ++c) {
    a1[c] = R.V[1][c] - R.V[0][c]; a2[c] = R.V[2][c] - R.V[0][c]; a3[c] = R.V[3][c] - R.V[0][c];
  }
  double cr[3] = {a1[1] * a2[2] - a1[2] * a2[1], a1[2] * a2[0] - a1[0] * a2[2],
                  a1[0] * a2[1] - a1[1] * a2[0]};
  if (!(fabs(dot3(cr, a3)) > 1e-14 * R.diam * R.diam * R.diam)) return 4;
  for (int k = 0; k < 4; ++k) {
    int i0 = k == 0 ? 1 : 0, i1 = k <= 1 ? 2 : 1, i2 = k <= 2 ? 3 : 2;
    double u1[3], u2[3], tk[3];
    for (int c = 0; c < 3; ++c) {
      u1[c] = R.V[i1][c] - R.V[i0][c]; u2[c] = R.V[i2][c] - R.V[i0][c]; tk[c] = R.V[k][c] - R.V[i0][c];
    }
    double N[3] = {u1[1] * u2[2] - u1[2] * u2[1], u1[2] * u2[0] - u1[0] * u2[2],
                   u1[0] * u2[1] - u1[1] * u2[0]};
    if (dot3(N, tk) > 0.0) { N[0] = -N[0]; N[1] = -N[1]; N[2] = -N[2]; }
    double l = sqrt(dot3(N, N));
    R.fa[k] = N[0] / l; R.fb[k] = N[1] / l; R.fc[k] = N[2] / l;
    R.fh[k] = (N[0] * R.V[i0][0] + N[1] * R.V[i0][1] + N[2] * R.V[i0][2]) / l;
  }
  double rad = 0.0;
  for (int k = 0; k < 4; ++k) {
    double dx = X[k][1] - cen[0], dy = X[k][2] - cen[1], dz = X[k][3] - cen[2];
    rad = fmax(rad, sqrt(dx * dx + dy * dy + dz * dz));
  }
  R.cx = cen[0]; R.cy = cen[1]; R.cz = cen[2]; R.rad = rad * (1.0 + 1e-12);
  R.pad = 0.0;
  return 0;
}

// Outer points of eq. int_bform for one test panel: centroids of the m^2
// congruent sub-triangles of every face with nu_t != 0 (Fig. int_tri_mid),
// weight -nu_t |F| / m^2.  Returns the number of points.
STB_HD inline int make_outer(const TrialRec& R, int m, double* P, double* W) {
  int cnt = 0;
  double inv = 1.0 / m;
  for (int k = 0; k < 4; ++k) {
    int i0 = k == 0 ? 1 : 0, i1 = k <= 1 ? 2 : 1, i2 = k <= 2 ? 3 : 2;
    double u1[3], u2[3], tk[3];
    for (int c = 0; c < 3; ++c) {
      u1[c] = R.V[i1][c] - R.V[i0][c]; u2[c] = R.V[i2][c] - R.V[i0][c]; tk[c] = R.V[k][c] - R.V[i0][c];
    }
    double N[3] = {u1[1] * u2[2] - u1[2] * u2[1], u1[2] * u2[0] - u1[0] * u2[2],
                   u1[0] * u2[1] - u1[1] * u2[0]};
    double sg = dot3(N, tk) > 0.0 ? -1.0 : 1.0;
    double nut_area = sg * N[0] * 0.5;       // nu_{F,t} |F| (outward)
    if (nut_area == 0.0) continue;           // vertical face
    double wq = -nut_area / (double)(m * m);
    for (int a = 0; a < m; ++a)
      for (int b = 0; a + b < m; ++b)
        for (int up = 0; up < 2; ++up) {
          double al, be;
          if (up == 0) { al = (a + 1.0 / 3.0) * inv; be = (b + 1.0 / 3.0) * inv; }
          else {
            if (a + b > m - 2) continue;
            al = (a + 2.0 / 3.0) * inv; be = (b + 2.0 / 3.0) * inv;
          }
          for (int c = 0; c < 4; ++c)
            P[4 * cnt + c] = R.X[i0][c] + al * (R.X[i1][c] - R.X[i0][c]) + be * (R.X[i2][c] - R.X[i0][c]);
          W[cnt] = wq;
          ++cnt;
        }
  }
  return cnt;
}

struct ComboL {          // per (apex, trial panel) data needed by L(phi)
  double C[4];
  double d2, wlo, whi;
  double fa[4], fb[4], fc[4];
};

STB_HD __forceinline__ double L_combo(const ComboL& cb, double cs, double sn) {
  FaceSet F;
#pragma unroll
  for (int k = 0; k < 4; ++k) { F.fa[k] = cb.fa[k]; F.fb[k] = cb.fb[k]; F.fc[k] = cb.fc[k]; }
  return L_eval(F, cb.C, cb.d2, cb.wlo, cb.whi, cs, sn);
}

// ------------------------------------------------------------ piece recipes
//
// Between consecutive breakpoints the admissible set keeps its structure:
// which face roots (or ends of the time range) bound each of its gaps
// changes only where two roots meet on a panel edge (edge events), where a
// face's roots appear or vanish (tangencies), or at the hint angles -- all
// breakpoints.  So the structure seen at one point of a piece (its midpoint,
// or a quarter point) is a recipe for L at every node of the piece: L is the
// r-measure of a fixed list of gaps, each from one endpoint formula to
// another, and a node needs only those formulas instead of all four faces,
// the hole sort and the sweep.  Endpoint ids: 0 = wlo, 1 = whi, 2 + 2k =
// face k's root q / e, 3 + 2k = its root -d^2 f / q (the root of the linear
// case e = 0).  A recipe holds up to kRecipeGaps (2) gaps, 8 bits each (start id
// << 4 | end id), and the gap count in bits 24-25; 0 gaps means "no recipe"
// (more gaps than fit).  On the host mirror over 8.5 million non-empty
// pieces of the cube and icosphere workloads the recipe reproduced L at
// every node of every piece wider than 1e-12 to rounding; 99.6% of the
// pieces have one gap, the rest two.
constexpr int kRecipeGaps = 2;

STB_HD __forceinline__ void order2i(double& s0, double& e0, int& i0, int& j0, double& s1, double& e1,
                                    int& i1, int& j1) {
  bool sw = s1 < s0;
  double ts = s0, te = e0;
  int ti = i0, tj = j0;
  s0 = sw ? s1 : s0; e0 = sw ? e1 : e0; i0 = sw ? i1 : i0; j0 = sw ? j1 : j0;
  s1 = sw ? ts : s1; e1 = sw ? te : e1; i1 = sw ? ti : i1; j1 = sw ? tj : j1;
}

// L(phi) as L_eval, also returning the recipe of its gap structure.  The
// admissible set is found from values alone (as L_eval does); the endpoint
// formula of each end of the (at most two) kept gaps is then identified by
// matching its value against the candidates -- the range ends wlo, whi and
// the faces' roots q / e, -d^2 f / q -- the lowest id first.  Every end is a
// copy of one of them (fmin, fmax and selects keep the bits), and carrying
// the ids through every comparison instead costs more selects than the
// arithmetic itself.
STB_HD inline double L_eval_recipe(const ComboL& cb, double cs, double sn, uint32_t* recipe) {
  const double kNone = 1e300;
  const double d2 = cb.d2;
  double lo = cb.wlo, hi = cb.whi;
  bool dead = false;
  double hs[4], he[4], r1[4], r2[4];
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    double a = cb.fa[k];
    double B = fma(cb.fb[k], cs, cb.fc[k] * sn);
    double e = B - a, f = B + a, Ck = cb.C[k];
    double D = fma(Ck, Ck, d2 * (e * f));
    bool two = D > 0.0;
    double q = Ck + copysign(sqrt_disc(D), Ck);
    double w1 = q * frcp(e);
    double w2 = -d2 * f * frcp(q);
    r1[k] = w1;
    r2[k] = w2;
    double mn = fmin(w1, w2), mx = fmax(w1, w2);
    bool pos = e > 0.0, neg = e < 0.0, zer = !(pos || neg);
    bool cut = pos && two;
    dead = dead || (pos && !two) || (zer && Ck == 0.0 && !(d2 * f > 0.0));
    lo = cut ? fmax(lo, mn) : lo;
    hi = cut ? fmin(hi, mx) : hi;
    lo = (zer && Ck > 0.0) ? fmax(lo, w2) : lo;
    hi = (zer && Ck < 0.0) ? fmin(hi, w2) : hi;
    bool hole = neg && two;
    hs[k] = hole ? mn : kNone;
    he[k] = hole ? mx : kNone;
  }
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    hs[k] = fmin(fmax(hs[k], lo), hi);
    he[k] = fmax(fmin(he[k], hi), hs[k]);
  }
  order2(hs[0], he[0], hs[1], he[1]);
  order2(hs[2], he[2], hs[3], he[3]);
  order2(hs[0], he[0], hs[2], he[2]);
  order2(hs[1], he[1], hs[3], he[3]);
  order2(hs[1], he[1], hs[2], he[2]);
  const double kWulp = 8.881784197001252e-16;
  double len = 0.0, c = lo;
  double gs0 = lo, ge0 = lo, gs1 = lo, ge1 = lo;   // ends of the first two kept gaps
  int ng = 0;
#pragma unroll
  for (int k = 0; k < 5; ++k) {
    const double g1 = k < 4 ? fmax(hs[k], c) : hi;
    const double m = rdiff(c, g1, d2);
    const bool keep = m > kWulp * g1;
    len += keep ? m : 0.0;
    const bool f0 = keep && ng == 0, f1 = keep && ng == 1;
    gs0 = f0 ? c : gs0;
    ge0 = f0 ? g1 : ge0;
    gs1 = f1 ? c : gs1;
    ge1 = f1 ? g1 : ge1;
    ng += keep ? 1 : 0;
    if (k < 4) c = fmax(he[k], c);
  }
  auto id_of = [&](double v) {
    uint32_t id = 9u;
#pragma unroll
    for (int k = 3; k >= 0; --k) {
      id = v == r2[k] ? (uint32_t)(3 + 2 * k) : id;
      id = v == r1[k] ? (uint32_t)(2 + 2 * k) : id;
    }
    id = v == cb.whi ? 1u : id;
    id = v == cb.wlo ? 0u : id;
    return id;
  };
  const uint32_t rec = (ng >= 1 ? (id_of(gs0) << 4) | id_of(ge0) : 0u) |
                       (ng >= 2 ? ((id_of(gs1) << 4) | id_of(ge1)) << 8 : 0u);
  const bool empty = dead || !(hi > lo);
  *recipe = (empty || ng > kRecipeGaps) ? 0u : (rec | ((uint32_t)ng << 24));
  return empty ? 0.0 : len;
}

STB_HD __forceinline__ int recipe_gaps(uint32_t r) { return (int)((r >> 24) & 3u); }

// One endpoint formula, prepared per piece: the coefficients of its face
// (or a constant end of the time range).
struct Endpoint {
  double a, fb, fc, C;
  double cval;      // value when constant
  bool cst, isb;    // constant end; root -d^2 f / q (else q / e)
};

STB_HD __forceinline__ double endpoint_value(const Endpoint& E, double d2, double wlo, double whi,
                                             double cs, double sn) {
  double B = fma(E.fb, cs, E.fc * sn);
  double e = B - E.a, f = B + E.a;
  double D = fma(E.C, E.C, d2 * (e * f));
  double q = E.C + copysign(sqrt_disc(D), E.C);
  double num = E.isb ? -d2 * f : q;
  double den = E.isb ? q : e;
  double v = num * frcp(den);
  v = E.cst ? E.cval : v;
  // the admissible set lies in [wlo, whi]; a formula evaluated just past
  // the structure it was chosen for (rounding at a piece's end) stays there
  return fmin(fmax(v, wlo), whi);
}

// endpoint_value for a q / e root (not a constant, not the -d^2 f / q root):
// the same operations without the selects.
STB_HD __forceinline__ double endpoint_value_qe(const Endpoint& E, double d2, double wlo, double whi,
                                                double cs, double sn) {
  double B = fma(E.fb, cs, E.fc * sn);
  double e = B - E.a, f = B + E.a;
  double D = fma(E.C, E.C, d2 * (e * f));
  double q = E.C + copysign(sqrt_disc(D), E.C);
  double v = q * frcp(e);
  return fmin(fmax(v, wlo), whi);
}

// The Gauss-node stage's arithmetic: the same formulas with one refinement
// step fewer.  Measured on the device over 2^22 seeded values spanning 2^-100
// to 2^100: the reciprocal estimate is within 4.6e-8, so one Newton step
// leaves 1/x within 2.2e-15; one Goldschmidt step leaves sqrt within 4.2e-15
// (relative).  The nodes only add values (no decision is taken on them
// beyond the sign of a gap), so this moves a node value by about 1e-14 of
// its inputs' scale, four orders below the assembly's 1e-10 parity bound;
// the decisions (lit test, breakpoints, empty-piece test, recipe) keep the
// refinement to an ulp.
STB_HD __forceinline__ double frcp_node(double x) {
#if defined(__HIP_DEVICE_COMPILE__)
  const double r = __builtin_amdgcn_rcp(x);
  return fma(r, fma(-x, r, 1.0), r);
#else
  return 1.0 / x;
#endif
}

// A discriminant D <= 2^-900 (no real root, or a double root up to
// rounding) is taken as 2^-900, one floor instead of a test and two
// selects: its root 2^-450 vanishes when added to a C_k above 2^-397 in
// magnitude, as 0 would, and at C_k = 0 it leaves w = 2^-450 / e instead of
// 0 (the r-measure moves by that much at most).
STB_HD __forceinline__ double sqrt_disc_node(double D) {
  const double x = fmax(D, 0x1p-900);
#if defined(__HIP_DEVICE_COMPILE__)
  const double y = __builtin_amdgcn_rsq(x);
  const double g = x * y;
  return fma(g, fma(-g, 0.5 * y, 0.5), g);
#else
  return sqrt(x);
#endif
}

// r(w1) - r(w0) = (w1 - w0) (1 - d^2 / (w0 w1)) / 2, returned doubled (the
// node sums take the factor 1/2 once, at the end: exact).  Both ends are
// at least |d| (the admissible range starts there), so w0 w1 >= d^2 when
// d != 0; the floor 2^-1000 only acts at d = 0, where it keeps 1 / (w0 w1)
// finite and the factor exactly 1.
STB_HD __forceinline__ double rdiff2_node(double w0, double w1, double d2) {
  const double g = fma(-d2, frcp_node(fmax(w0 * w1, 0x1p-1000)), 1.0);
  return (w1 - w0) * g;
}

STB_HD __forceinline__ double endpoint_value_node(const Endpoint& E, double d2, double wlo, double whi,
                                                  double cs, double sn) {
  const double B = fma(E.fb, cs, E.fc * sn);
  const double e = B - E.a, f = B + E.a;
  const double D = fma(E.C, E.C, d2 * (e * f));
  const double q = E.C + copysign(sqrt_disc_node(D), E.C);
  const double num = E.isb ? -d2 * f : q;
  const double den = E.isb ? q : e;
  double v = num * frcp_node(den);
  v = E.cst ? E.cval : v;
  return fmin(fmax(v, wlo), whi);
}

STB_HD __forceinline__ double endpoint_value_qe_node(const Endpoint& E, double d2, double wlo,
                                                     double whi, double cs, double sn) {
  const double B = fma(E.fb, cs, E.fc * sn);
  const double e = B - E.a, f = B + E.a;
  const double D = fma(E.C, E.C, d2 * (e * f));
  const double q = E.C + copysign(sqrt_disc_node(D), E.C);
  return fmin(fmax(q * frcp_node(e), wlo), whi);
}

// One endpoint formula at the mirror nodes m -+ delta of a piece, from the
// per-piece P = B(m), Q = b sin m - c cos m of its face, CC = C^2 and
// SG = copysign(1, C): B(m -+ delta) = P cos delta +- Q sin delta, and
// C + copysign(s, C) as one fma.  vm at m - delta, vp at m + delta;
// node-stage arithmetic.
template <bool QE>
STB_HD __forceinline__ void endpoint_pair_node(const Endpoint& E, double P, double Q, double CC, double SG,
                                               double d2, double wlo, double whi, double cd, double sd,
                                               double& vm, double& vp) {
  const double qs = Q * sd;
  double v[2];
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    const double B = fma(P, cd, h ? -qs : qs);
    const double e = B - E.a, f = B + E.a;
    const double D = fma(d2 * e, f, CC);
    const double q = fma(SG, sqrt_disc_node(D), E.C);
    double w;
    if (QE) {
      w = q * frcp_node(e);
    } else {
      const double num = E.isb ? -d2 * f : q;
      const double den = E.isb ? q : e;
      w = num * frcp_node(den);
      w = E.cst ? E.cval : w;
    }
    v[h] = fmin(fmax(w, wlo), whi);
  }
  vm = v[0];
  vp = v[1];
}

// L by a recipe: the r-measure of its gaps, each between two endpoint
// formulas (E[2g], E[2g + 1]).
STB_HD __forceinline__ double L_by_recipe(const Endpoint* E, int ng, double d2, double wlo,
                                          double whi, double cs, double sn) {
  double len = 0.0;
  for (int g = 0; g < ng; ++g) {
    double v0 = endpoint_value(E[2 * g], d2, wlo, whi, cs, sn);
    double v1 = endpoint_value(E[2 * g + 1], d2, wlo, whi, cs, sn);
    len += v1 > v0 ? rdiff(v0, v1, d2) : 0.0;
  }
  return len;
}

// ------------------------------------------------------------ mixed precision
//
// Far pairs: the root solves and the interval measure of L(phi) in FP32,
// everything that fixes the geometry in FP64.  Near the panel the roots
// w = r + s of the face quadratics are large (~ 2 |x - y|) while the
// admissible interval is as wide as the panel, so roots computed in FP32
// about w = 0 would lose |x - y| / diam ulps.  Instead the quadratics are
// re-centred at the middle w_c of the admissible w-range: with w = w_c + delta,
//   Q_k(w_c + delta) = e delta^2 + 2 beta delta + gamma,
//   e = B - a,  beta = B w_c - (a w_c + C),  gamma = B (w_c^2 - d^2)
//                                               - (a (w_c^2 + d^2) + 2 C w_c),
// where beta, gamma and the discriminant beta^2 - e gamma (which cancels
// near a tangency) are formed in FP64 from the FP64 angle and per-pair
// constants and only then rounded to FP32; the deltas of interest are as
// large as the panel, so FP32 resolves them to ~1e-7 of the panel.  The r-measure of a gap [delta0, delta1] is
//   (delta1 - delta0) / 2 * (v0 v1 + |d| (v0 + v1)) / ((|d| + v0)(|d| + v1)),
// v = w - |d| = (w_c - |d|) + delta >= 0: a product of non-negative terms,
// free of the cancellation in 1 - d^2 / (w0 w1) near the hyperbola's vertex.
struct FarConst {
  double wc, P1;           // centre of the admissible w-range, w_c^2 - d^2
  double K1[4], K0[4];     // a w_c + C, a (w_c^2 + d^2) + 2 C w_c per face
  float m, ad;             // w_c - |d|, |d|
  float dlo, dhi;          // admissible range of delta
};

STB_HD __forceinline__ FarConst far_const(const ComboL& cb) {
  FarConst F;
  const double wc = 0.5 * (cb.wlo + cb.whi), ad = sqrt(cb.d2);
  F.wc = wc;
  F.P1 = (wc - ad) * (wc + ad);
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    F.K1[k] = fma(cb.fa[k], wc, cb.C[k]);
    F.K0[k] = fma(cb.fa[k], fma(wc, wc, cb.d2), 2.0 * cb.C[k] * wc);
  }
  F.m = (float)(wc - ad);
  F.ad = (float)ad;
  F.dlo = (float)(cb.wlo - wc);
  F.dhi = (float)(cb.whi - wc);
  return F;
}

// FP32 reciprocal and square root (hardware, about 1 ulp).
STB_HD __forceinline__ float rcp32(float x) {
#if defined(__HIP_DEVICE_COMPILE__)
  return __builtin_amdgcn_rcpf(x);
#else
  return 1.0f / x;
#endif
}

STB_HD __forceinline__ float sqrt32(float x) {
#if defined(__HIP_DEVICE_COMPILE__)
  return __builtin_amdgcn_sqrtf(x);
#else
  return sqrtf(x);
#endif
}

STB_HD __forceinline__ void order2f(float& s0, float& e0, float& s1, float& e1) {
  bool sw = s1 < s0;
  float ts = s0, te = e0;
  s0 = sw ? s1 : s0;
  e0 = sw ? e1 : e0;
  s1 = sw ? ts : s1;
  e1 = sw ? te : e1;
}

// r-measure of the gap [d0, d1] (delta coordinates), see above.
STB_HD __forceinline__ float rgap32(float d0, float d1, const FarConst& F) {
  float v0 = fmaxf(F.m + d0, 0.0f), v1 = fmaxf(F.m + d1, 0.0f);
  float num = fmaf(v0, v1, F.ad * (v0 + v1));
  float den = (F.ad + v0) * (F.ad + v1);
  float g = den > 0.0f ? num * rcp32(den) : 1.0f;
  return 0.5f * (d1 - d0) * g;
}

// L(phi) of a far pair: same case analysis as L_eval (e > 0: between the
// roots; e < 0: outside; e = 0: one side of the linear root) in delta.
// *err receives a first-order bound of the FP32 rounding error: every root
// is resolved to a few ulps of its own size (beta, gamma and the
// discriminant come rounded from FP64; one square root, one reciprocal, two
// products), so a gap [c, g1] contributes at most kE (|c| + |g1| + m) with
// kE = 4 ulp.
STB_HD __forceinline__ float L_eval_far(const ComboL& cb, const FarConst& F, double cs,
                                        double sn, float* err) {
  const float kNone = 3.0e38f;
  float lo = F.dlo, hi = F.dhi;
  bool dead = false;
  float hs[4], he[4];
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const double B = fma(cb.fb[k], cs, cb.fc[k] * sn);
    const double e64 = B - cb.fa[k];
    const double be64 = fma(B, F.wc, -F.K1[k]);
    const double ga64 = fma(B, F.P1, -F.K0[k]);
    // the discriminant cancels near a tangency: formed in FP64
    const float D = (float)fma(be64, be64, -e64 * ga64);
    const float e = (float)e64, be = (float)be64, ga = (float)ga64;
    const bool two = D > 0.0f;
    const float q = -(be + copysignf(sqrt32(fmaxf(D, 0.0f)), be));
    const float r1 = q * rcp32(e), r2 = ga * rcp32(q);
    const float mn = fminf(r1, r2), mx = fmaxf(r1, r2);
    const bool pos = e > 0.0f, neg = e < 0.0f, zer = !(pos || neg);
    const bool cut = pos && two;
    dead = dead || (pos && !two) || (zer && be == 0.0f && !(ga < 0.0f));
    lo = cut ? fmaxf(lo, mn) : lo;
    hi = cut ? fminf(hi, mx) : hi;
    // e = 0: 2 beta delta + gamma < 0, root r2 = -gamma / (2 beta)
    lo = (zer && be < 0.0f) ? fmaxf(lo, r2) : lo;
    hi = (zer && be > 0.0f) ? fminf(hi, r2) : hi;
    const bool hole = neg && two;
    hs[k] = hole ? mn : kNone;
    he[k] = hole ? mx : kNone;
  }
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    hs[k] = fminf(fmaxf(hs[k], lo), hi);
    he[k] = fmaxf(fminf(he[k], hi), hs[k]);
  }
  order2f(hs[0], he[0], hs[1], he[1]);
  order2f(hs[2], he[2], hs[3], he[3]);
  order2f(hs[0], he[0], hs[2], he[2]);
  order2f(hs[1], he[1], hs[3], he[3]);
  order2f(hs[1], he[1], hs[2], he[2]);
  // gaps whose measure is below 4 FP32 ulps of their delta-coordinates are
  // rounding artefacts (e.g. where two roots meet at the hyperbola's vertex)
  const float kWulp32 = 4.76837158203125e-7f;
  const float kE = 2.384185791015625e-7f;   // 4 ulp
  // A dropped gap adds its own measure to the bound; an interval that is
  // empty in FP32 only because its ends crossed by rounding adds the ends'
  // uncertainty (the decisions on the signs of e and of the discriminant
  // are the FP64 ones: the casts keep signs).
  float len = 0.0f, e = 0.0f, c = lo;
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    float g1 = fmaxf(hs[k], c);
    float m = rgap32(c, g1, F);
    bool keep = m > kWulp32 * fmaxf(fabsf(c), fabsf(g1));
    len += keep ? m : 0.0f;
    e += keep ? kE * (fabsf(c) + fabsf(g1) + m) : m;
    c = fmaxf(he[k], c);
  }
  float m = rgap32(c, hi, F);
  bool keep = m > kWulp32 * fmaxf(fabsf(c), fabsf(hi));
  len += keep ? m : 0.0f;
  e += keep ? kE * (fabsf(c) + fabsf(hi) + m) : m;
  const bool empty = dead || !(hi > lo);
  *err = dead ? 0.0f : (empty ? kE * (fabsf(lo) + fabsf(hi)) : e);
  return empty ? 0.0f : len;
}

// A combo is far when the apex's spatial distance from the trial panel's
// bounding ball exceeds eta times the ball's radius.
STB_HD __forceinline__ bool apex_far(const TrialRec& T, const double* x4, double eta) {
  double dx = x4[1] - T.cx, dy = x4[2] - T.cy, dz = x4[3] - T.cz;
  return sqrt(dx * dx + dy * dy + dz * dz) - T.rad > eta * T.rad;
}

STB_HD __forceinline__ double L_at(const ComboL& cb, double phi) {
  double sn, cs;
  sincos_small(phi, &sn, &cs);
  return L_combo(cb, cs, sn);
}

// One Gauss node of a phi piece [a, a + H] in the smoothstep variable.  Not
// inlined, so every caller sums identically rounded node values.
static STB_HD __noinline__ double node_value(const ComboL& cb, double a, double H, double u,
                                          double wg) {
  double s = u * u * (3.0 - 2.0 * u);
  double ds = 6.0 * u * (1.0 - u);
  double L = L_at(cb, a + H * s);
  double f = H * ds;
  f = f * wg;
  return f * L;
}


// The whole inner integral V phi_sigma (x) of one (apex, panel) pair, one
// lane, in the order the tiled kernel uses: lit test, breakpoints, pieces in
// phi order, nodes in order.  Returns 0 for a pair that is not lit; *lit
// receives the lit decision.
STB_HD inline double inner_serial(const TrialRec& T, const double* x4, int ng, const double* glx,
                                  const double* glw, bool* lit_out) {
  Apex A;
  apex_of(T, x4, A);
  double wlo = 0.0, whi = 0.0;
  bool lit = A.t - T.tmin > fabs(A.d) && !ball_rejects(T, x4) && lit_test(T, x4, A);
  if (lit_out) *lit_out = lit;
  if (!lit || !w_range(T, A, wlo, whi)) return 0.0;
  ComboL cb;
  for (int k = 0; k < 4; ++k) {
    cb.C[k] = A.C[k]; cb.fa[k] = T.fa[k]; cb.fb[k] = T.fb[k]; cb.fc[k] = T.fc[k];
  }
  cb.d2 = A.d * A.d; cb.wlo = wlo; cb.whi = whi;
  double bp[kMaxBp];
  FaceAng FA;
  face_angles(T, FA);
  int nb = breakpoints(T, FA, A, bp);
  sort_bp(bp, nb);
  double I = 0.0;
  if (nb == 0) {
    int m = 2 * ng;
    double h = kTwoPi / m;
    for (int k = 0; k < m; ++k) I += h * L_at(cb, k * h);
    return I / (4.0 * kPi);
  }
  for (int k = 0; k < nb; ++k) {
    double a = bp[k];
    double b = (k + 1 < nb) ? bp[k + 1] : bp[0] + kTwoPi;
    double H = b - a;
    if (!(H > 0.0)) continue;
    bool ne = L_at(cb, a + 0.5 * H) != 0.0;
    if (!ne) ne = L_at(cb, a + 0.25 * H) != 0.0 || L_at(cb, a + 0.75 * H) != 0.0;
    if (!ne) continue;
    double acc = 0.0;
    for (int g = 0; g < ng; ++g) acc += node_value(cb, a, H, glx[g], glw[g]);
    I += acc;
  }
  return I / (4.0 * kPi);
}

// Retarded double-layer potential (eq. dlp) of the four hat functions of a
// panel at x4, out[m] for the density that is 1 at local vertex m and 0 at
// the others.  With k3 = d_n / (4 pi r^3), k2 = d_n / (4 pi r^2) (eq. kfunc;
// d_n = nsign d, the distance along the outward normal) and dA = r dr dphi,
// the k2 term of a linear density cancels the time part of the k3 term:
// the r-integrand is d_n (lambda(t, p) + grad_uv lambda . e(phi) s) / r^2.
// The hat of vertex m is lambda_m = (h_m - a_m tau - b_m u - c_m v) / D_m
// over face m (opposite vertex m), D_m its value at vertex m: at (t, p) it
// is C_m / D_m, its in-plane gradient -(b_m, c_m) / D_m.  Three integrals
// over phi (of sa, sh cos, sh sin from dl_eval) give all four hats; the
// phi-rule (breakpoints, empty-piece test on L, smoothstep Gauss) is the
// single layer's.
STB_HD inline void inner_dl_serial(const TrialRec& T, const FaceAng& FA, const double* x4,
                                   double nsign, int ng, const double* glx, const double* glw,
                                   double* out) {
  for (int m = 0; m < 4; ++m) out[m] = 0.0;
  Apex A;
  apex_of(T, x4, A);
  double wlo = 0.0, whi = 0.0;
  if (A.d == 0.0) return;   // k2 = k3 = 0 in the panel's plane
  const int lq = lit_quick(T, x4, A);   // the vertices decide nearly every pair
  const bool lit = lq == 1 || (lq == 2 && lit_test(T, x4, A));
  if (!lit || !w_range(T, A, wlo, whi)) return;
  ComboL cb;
  FaceSet F;
  for (int k = 0; k < 4; ++k) {
    cb.C[k] = A.C[k]; cb.fa[k] = T.fa[k]; cb.fb[k] = T.fb[k]; cb.fc[k] = T.fc[k];
    F.fa[k] = T.fa[k]; F.fb[k] = T.fb[k]; F.fc[k] = T.fc[k];
  }
  const double d2 = A.d * A.d;
  cb.d2 = d2; cb.wlo = wlo; cb.whi = whi;
  double bp[kMaxBp];
  int nb = breakpoints(T, FA, A, bp);
  sort_bp(bp, nb);
  double ia = 0.0, ic = 0.0, is = 0.0;
  auto node = [&](double phi, double wt) {
    double sn, cs, sa, sh;
    sincos_small(phi, &sn, &cs);
    dl_eval(F, A.C, d2, wlo, whi, cs, sn, sa, sh);
    ia += wt * sa;
    ic += (wt * sh) * cs;
    is += (wt * sh) * sn;
  };
  if (nb == 0) {
    const int m = 2 * ng;
    const double h = kTwoPi / m;
    for (int k = 0; k < m; ++k) node(k * h, h);
  } else {
    for (int k = 0; k < nb; ++k) {
      const double a = bp[k];
      const double b = (k + 1 < nb) ? bp[k + 1] : bp[0] + kTwoPi;
      const double H = b - a;
      if (!(H > 0.0)) continue;
      if (piece_misses(T, A, a, H)) continue;   // no ray of the piece meets the panel
      bool ne = L_at(cb, a + 0.5 * H) != 0.0;
      if (!ne) ne = L_at(cb, a + 0.25 * H) != 0.0 || L_at(cb, a + 0.75 * H) != 0.0;
      if (!ne) continue;
      for (int g = 0; g < ng; ++g) {
        const double u = glx[g];
        const double sm = u * u * (3.0 - 2.0 * u);
        const double ds = 6.0 * u * (1.0 - u);
        node(a + H * sm, H * ds * glw[g]);
      }
    }
  }
  const double f = nsign * A.d / (4.0 * kPi);
  for (int m = 0; m < 4; ++m) {
    const double Dm = T.fh[m] - T.fa[m] * T.V[m][0] - T.fb[m] * T.V[m][1] - T.fc[m] * T.V[m][2];
    out[m] = f * (A.C[m] * ia - T.fb[m] * ic - T.fc[m] * is) / Dm;
  }
}

}  // namespace stb
