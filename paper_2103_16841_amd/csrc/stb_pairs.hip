// stb_pairs.hip -- the pair pipeline: every (outer point, trial panel)
// combination of a candidate set, through the lit test, the phi-breakpoints,
// the empty-piece tests and the Gauss nodes, as a chain of flat kernels that
// hand their work on through lists in HBM.
//
// A candidate is one (row, trial panel) pair of the cull's CSR: a row is a
// test panel (matrix) or an evaluation point (potential); its apexes are the
// row's outer points of eq. int_bform (matrix) or the point itself.
//
//   k_lit     one lane per candidate: for each of its apexes the exact lit
//             test of Sec. 3.3 (bounding-ball pre-test of Theorem
//             phi_xi_sphere first); lit (candidate, apex) combos are appended
//             to the combo list, contiguous per candidate, by wave-aggregated
//             atomics (ballot-free prefix of the per-lane counts).
//   k_bp      one lane per lit combo: apex data, admissible w-range, the
//             phi-breakpoints (sorted) and the pieces between them, appended
//             to the piece list, contiguous per combo in phi order; a combo
//             without breakpoints gets two half-periods of the trapezoid rule.
//             A piece whose three test points all lie outside the wedge of
//             directions that meet the panel's spatial shadow is empty and is
//             not listed.
//   k_empty   one lane per piece: L at the midpoint; the pieces where it is
//             zero are queued for k_quarter (L at the quarter points); the
//             non-empty pieces go to the job lists.
//   k_nodes   one lane per job: the n_g Gauss nodes of the piece in order
//             (smoothstep map), summed in order.
//   k_combine one lane per combo: ordered sum over its pieces, / (4 pi).
//   k_store   one lane per candidate: matrix entry = ordered sum over the
//             apexes of w_q I_q (eq. int_bform); potential: I itself.
//
// Every list position is handed out by atomics, but every sum runs in a
// fixed order (nodes, pieces in phi order, apexes in q order), so results do
// not depend on the schedule.  The candidate range is processed in chunks
// sized to the workspace; a chunk whose lists would overflow is split and
// redone.  Lists cost a few hundred bytes per combo: the HBM traffic is a few
// percent of what the FP64 arithmetic takes, while each stage runs at full
// lane occupancy with its own register budget.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstddef>

#include "stb_internal.h"
#include "stb_pairs.h"

using namespace stb;

namespace {

constexpr int kBlk = 256;
constexpr int kMaxBlocks = 256 * 16;

enum {
  CNT_COMBO = 0, CNT_DEEP, CNT_PIECE, CNT_JOB, CNT_JOB1X, CNT_JOB2, CNT_JOBF, CNT_JOB32, CNT_REDO, CNT_JOBR, CNT_PAIRS, CNT_CAUSAL, CNT_EVAL_MID,
  CNT_EVAL_QUARTER, CNT_EVAL_NODES, CNT_EVAL_NODES32, CNT_EVAL_REDO, CNT_MISS, CNT_QZ, CNT_N
};

// Combo key: (candidate in chunk) << kKeyShift | far << 6 | q, q < 64
// (4 m_q^2 outer points at most): 25 bits of candidate index.
constexpr int kKeyShift = 7;
constexpr uint32_t kKeyFar = 1u << 6;
constexpr uint32_t kKeyQ = 63u;

// Block-wide list allocation: every thread of the block calls it (n = 0
// when it has nothing to append), with the same LDS scratch; one atomic per
// block.  Same-address atomics serialise in the memory system, so they are
// kept to one per few hundred list entries.  Returns the first slot of this
// thread's n entries; slots are in thread order within the block.
struct AllocLds {
  unsigned wtot[kBlk / 64];
  unsigned long long base;
};

__device__ __forceinline__ unsigned long long block_alloc(unsigned long long* ctr, unsigned n,
                                                          AllocLds& sh) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  unsigned incl = n;
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    unsigned v = __shfl_up(incl, off, 64);
    if (lane >= off) incl += v;
  }
  if (lane == 63) sh.wtot[wave] = incl;
  __syncthreads();
  if (threadIdx.x == 0) {
    unsigned run = 0;
#pragma unroll
    for (int w = 0; w < (int)(blockDim.x >> 6); ++w) {
      unsigned t = sh.wtot[w];
      sh.wtot[w] = run;
      run += t;
    }
    sh.base = run ? atomicAdd(ctr, (unsigned long long)run) : 0ull;
  }
  __syncthreads();
  unsigned long long r = sh.base + sh.wtot[wave] + (incl - n);
  __syncthreads();   // the scratch is reused by the next call
  return r;
}

// Sum of a per-lane count over the block, added to *ctr once per block.
__device__ __forceinline__ void block_count(unsigned long long* ctr, unsigned long long v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
  if ((threadIdx.x & 63) == 0 && v) atomicAdd(ctr, v);
}

struct Lists {
  // per candidate of the chunk
  uint64_t* mask;        // lit apexes (bit q)
  int32_t* combo0;       // first combo of the candidate
  int32_t* ccnt;         // [cap_cand + 1] lit apexes per candidate, then ...
  int32_t* coff;         // [cap_cand + 1] ... their exclusive prefix
  void* scan_tmp;        // prefix-sum scratch
  size_t scan_bytes;
  // per combo
  uint32_t* key;         // (candidate in chunk) << kKeyShift | far << 6 | q
  uint32_t* deep;        // (candidate in chunk) << kKeyShift | q of lit tests the vertices left open
  double* cb;            // C_k, d^2, w-range: structure of arrays, field f at f * cap_combo
  int32_t* ccol;         // trial panel of the combo (its face normals are read from there)
  int32_t* p0;           // first piece
  int32_t* np;           // pieces
  double* I;             // inner integral
  float* Ie;             // its FP32 rounding bound (mixed)
  // per piece
  double* pa;            // start angle (trapezoid half: 0 or 1)
  double* ph;            // length (trapezoid half: -1)
  int32_t* pc;           // owning combo
  double* pv;            // ordered node sum
  int32_t* pz;           // pieces whose quarter points decide (shares pv's memory: the
                         // node sums are written only after k_quarter has read the queue)
  float* pe;             // FP32 rounding bound of the node sum (far pieces, mixed)
  int32_t* job;          // non-empty pieces, FP64 nodes by a one-gap recipe
  int32_t* job2;         // ... by a two-gap recipe
  int32_t* jobf;         // ... full evaluation (no recipe, slivers, trapezoid halves)
  uint32_t* prec;        // per piece: recipe of its gap structure
  int32_t* job32;        // non-empty pieces of far combos, FP32 nodes (mixed)
  uint8_t* pne;          // per piece: non-empty
  uint8_t* redo;         // per candidate (mixed): entry recomputed in FP64
  unsigned long long* cnt;
  int64_t cap_cand, cap_combo, cap_piece;
  const TrialRec* trial; // panel records of the run
};

// Item count of a list for a kernel: given by the host (n >= 0), or read
// from the list's device counter -n - 1, so that the host need not wait for
// the producer before it launches the consumer.  With a device count the
// kernel does nothing when one of the first `done` lists (deep, combo,
// piece: those whose producers have finished) overflowed: a producer skips
// an allocation that crosses the capacity, so slots below it can be stale,
// and the host redoes such a chunk with a smaller one (k_store writes
// nothing for it).
__device__ __forceinline__ int64_t list_count(const Lists& L, int64_t n, int64_t cap, int done) {
  if (n >= 0) return n;
  bool ok = L.cnt[CNT_DEEP] <= (unsigned long long)L.cap_combo;
  if (done >= 2) ok = ok && L.cnt[CNT_COMBO] <= (unsigned long long)L.cap_combo;
  if (done >= 3) ok = ok && L.cnt[CNT_PIECE] <= (unsigned long long)L.cap_piece;
  if (!ok) return 0;
  const unsigned long long c = L.cnt[-n - 1];
  return (int64_t)(c < (unsigned long long)cap ? c : (unsigned long long)cap);
}

// Field positions of ComboL's apex-dependent part in the combo list; the
// face normals (fa, fb, fc) are the trial panel's and are read from its
// record, not stored per combo.
constexpr int64_t kCbC = offsetof(ComboL, C) / sizeof(double);
constexpr int64_t kCbD2 = offsetof(ComboL, d2) / sizeof(double);
constexpr int64_t kCbWlo = offsetof(ComboL, wlo) / sizeof(double);
constexpr int64_t kCbWhi = offsetof(ComboL, whi) / sizeof(double);
constexpr int kComboStored = 7;
static_assert(kCbC == 0 && kCbD2 == 4 && kCbWlo == 5 && kCbWhi == 6, "ComboL layout");

// Combo data in structure-of-arrays form: lanes reading neighbouring combos
// touch neighbouring addresses of each field.
__device__ __forceinline__ void store_combo(const Lists& L, int64_t k, const ComboL& cb, int32_t col) {
  const int64_t cap = L.cap_combo;
#pragma unroll
  for (int f = 0; f < 4; ++f) L.cb[(kCbC + f) * cap + k] = cb.C[f];
  L.cb[kCbD2 * cap + k] = cb.d2;
  L.cb[kCbWlo * cap + k] = cb.wlo;
  L.cb[kCbWhi * cap + k] = cb.whi;
  L.ccol[k] = col;
}

// One endpoint formula of a recipe: only the selected face's coefficients,
// C_k from the combo list and (a, b, c)_k from the panel record.  (Selecting
// the face among all four in registers lets the compiler turn the selects
// into an indexed load from a private copy of the arrays.)
__device__ __forceinline__ Endpoint endpoint_load(const Lists& L, int64_t c, int id, double wlo,
                                                  double whi) {
  const int64_t cap = L.cap_combo;
  const int k = id >= 2 ? (id - 2) >> 1 : 0;
  const TrialRec* T = L.trial + L.ccol[c];
  Endpoint E;
  E.C = L.cb[(kCbC + k) * cap + c];
  E.a = T->fa[k];
  E.fb = T->fb[k];
  E.fc = T->fc[k];
  E.cst = id < 2;
  E.cval = id == 0 ? wlo : whi;
  E.isb = id >= 2 && ((id - 2) & 1);
  return E;
}

__device__ __forceinline__ ComboL load_combo(const Lists& L, int64_t k) {
  const int64_t cap = L.cap_combo;
  const TrialRec& T = L.trial[L.ccol[k]];
  ComboL cb;
#pragma unroll
  for (int f = 0; f < 4; ++f) {
    cb.C[f] = L.cb[(kCbC + f) * cap + k];
    cb.fa[f] = T.fa[f];
    cb.fb[f] = T.fb[f];
    cb.fc[f] = T.fc[f];
  }
  cb.d2 = L.cb[kCbD2 * cap + k];
  cb.wlo = L.cb[kCbWlo * cap + k];
  cb.whi = L.cb[kCbWhi * cap + k];
  return cb;
}

struct Geo {
  const int32_t* rows;   // row of each candidate (global index)
  const int32_t* cols;   // trial panel of each candidate
  const TrialRec* trial;
  const FaceAng* fang;   // per trial panel
  const double* apex;    // [rows][maxq][4]
  const double* apex_w;  // [rows][maxq] (matrix) or nullptr (potential)
  uint8_t* lit_out;      // optional per candidate: some apex lit
  const int32_t* apex_n; // [rows] or nullptr (one apex)
  int maxq;
  int mixed;             // far combos' nodes in FP32
  double eta_far;
};

// Lit test in two passes: the cheap part (slab, bounding ball, vertices)
// for every (candidate, apex), then the edge and face minima only for the
// few apexes the vertices leave open, densely -- a wave that ran them
// inline would pay the long path whenever one of its 64 lanes needs it.
// The first pass's fields of a panel record (its first 256 bytes), copied
// into registers once per candidate: read through the reference, the loads
// sink into the tests' branches and every apex waits for them again.
__device__ __forceinline__ TrialRec lit_fields(const TrialRec* __restrict__ p) {
  const double2* s = reinterpret_cast<const double2*>(p);
  double2 r[16];
#pragma unroll
  for (int i = 0; i < 16; ++i) r[i] = s[i];
  TrialRec T;
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    T.o[c] = (&r[0].x)[c];
    T.e1[c] = (&r[0].x)[3 + c];
    T.e2[c] = (&r[0].x)[6 + c];
    T.n[c] = (&r[0].x)[9 + c];
  }
#pragma unroll
  for (int k = 0; k < 4; ++k)
#pragma unroll
    for (int c = 0; c < 3; ++c) T.V[k][c] = (&r[0].x)[12 + 3 * k + c];
  T.tmin = r[12].x;
  T.tmax = r[12].y;
  T.diam = r[13].x;
  T.cx = r[13].y;
  T.cy = r[14].x;
  T.cz = r[14].y;
  T.rad = r[15].x;
  return T;
}
static_assert(offsetof(TrialRec, tmin) == 24 * sizeof(double) && offsetof(TrialRec, rad) == 30 * sizeof(double),
              "lit_fields layout");

__global__ __launch_bounds__(kBlk, 4) void k_lit(Geo g, Lists L, int64_t c0, int64_t nc) {
  const int B = (int)blockDim.x;
  __shared__ AllocLds sh;
  unsigned long long pairs = 0;
  for (int64_t base = (int64_t)blockIdx.x * B; base < nc; base += (int64_t)gridDim.x * B) {
    const int64_t c = base + threadIdx.x;
    const bool v = c < nc;
    uint64_t m = 0, und = 0;
    int nq = 0;
    if (v) {
      const int64_t cg = c0 + c;
      const int32_t i = g.rows[cg];
      const TrialRec T = lit_fields(g.trial + g.cols[cg]);
      nq = g.apex_n ? g.apex_n[i] : 1;
      // (points passed in by a caller are only known to be 8-byte aligned)
      const double* xr = g.apex + (int64_t)i * g.maxq * 4;
      // the next apex is loaded while this one is tested
      double xn[4] = {xr[0], xr[1], xr[2], xr[3]};
      for (int q = 0; q < nq; ++q) {
        double x4[4] = {xn[0], xn[1], xn[2], xn[3]};
        if (q + 1 < nq)
#pragma unroll
          for (int c = 0; c < 4; ++c) xn[c] = xr[4 * (q + 1) + c];
        Apex A;
        apex_frame(T, x4, A);
        const int r = lit_quick(T, x4, A);
        m |= (uint64_t)(r == 1) << q;
        und |= (uint64_t)(r == 2) << q;
      }
      pairs += (unsigned long long)nq;
      L.mask[c] = m;
    }
    const unsigned n = (unsigned)__popcll(und);
    unsigned long long k = block_alloc(L.cnt + CNT_DEEP, n, sh);
    if (v && k + n <= (unsigned long long)L.cap_combo)
      for (int q = 0; q < nq; ++q)
        if ((und >> q) & 1ull) L.deep[k++] = ((uint32_t)c << kKeyShift) | (uint32_t)q;
  }
  block_count(L.cnt + CNT_PAIRS, pairs);
}

// The second pass's fields: the first pass's and the vertices (t, x, y, z).
__device__ __forceinline__ TrialRec deep_fields(const TrialRec* __restrict__ p) {
  TrialRec T = lit_fields(p);
  const double2* s = reinterpret_cast<const double2*>(&p->X[0][0]);
  double2 r[8];
#pragma unroll
  for (int i = 0; i < 8; ++i) r[i] = s[i];
#pragma unroll
  for (int k = 0; k < 4; ++k)
#pragma unroll
    for (int c = 0; c < 4; ++c) T.X[k][c] = (&r[0].x)[4 * k + c];
  return T;
}

__global__ __launch_bounds__(kBlk) void k_lit_deep(Geo g, Lists L, int64_t c0, int64_t ndeep_arg) {
  const int B = (int)blockDim.x;
  const int64_t ndeep = list_count(L, ndeep_arg, L.cap_combo, 1);
  for (int64_t k = (int64_t)blockIdx.x * B + threadIdx.x; k < ndeep; k += (int64_t)gridDim.x * B) {
    const uint32_t key = L.deep[k];
    const int64_t c = key >> kKeyShift;
    const int q = (int)(key & kKeyQ);
    const int64_t cg = c0 + c;
    const int32_t i = g.rows[cg];
    const TrialRec T = deep_fields(g.trial + g.cols[cg]);
    const double* xq = g.apex + ((int64_t)i * g.maxq + q) * 4;
    double x4[4] = {xq[0], xq[1], xq[2], xq[3]};
    Apex A;
    apex_frame(T, x4, A);   // the lit test needs the frame only, not the C_k
    if (lit_test(T, x4, A)) atomicOr(reinterpret_cast<unsigned long long*>(L.mask + c), 1ull << q);
  }
}

// Lit combos contiguous per candidate, in apex order, candidates in order:
// counts, an exclusive prefix sum (stb_scan.hip), then the keys.
__global__ void k_emit_count(Lists L, int64_t nc) {
  const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (c < nc) L.ccnt[c] = __popcll(L.mask[c]);
  else if (c == nc) L.ccnt[nc] = 0;
}

__global__ __launch_bounds__(kBlk) void k_emit(Lists L, int64_t nc) {
  const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (c == 0) L.cnt[CNT_COMBO] = (unsigned long long)L.coff[nc];
  if (c >= nc) return;
  const uint64_t m = L.mask[c];
  const int32_t b = L.coff[c];
  L.combo0[c] = b;
  if ((int64_t)b + __popcll(m) <= L.cap_combo) {
    int64_t k = b;
    uint64_t mm = m;
    while (mm) {
      const int q = __ffsll((long long)mm) - 1;
      L.key[k++] = ((uint32_t)c << kKeyShift) | (uint32_t)q;
      mm &= mm - 1;
    }
  }
}

// Breakpoints of a lane: the first kBpLds slots in LDS (slot s of lane t at
// s * B + t: neighbouring lanes, neighbouring banks), the rest (nearly never
// used) in private memory.  Private memory of every resident lane is tens of
// MB, past the L2 caches: keeping the lists there cost most of the kernel's
// memory traffic.
constexpr int kBpLds = 24;
struct BpLds {
  double* lds;
  int stride;
  double* spill;
  __device__ __forceinline__ void put(int i, double v) {
    if (i < kBpLds) lds[i * stride] = v;
    else spill[i - kBpLds] = v;
  }
  __device__ __forceinline__ double get(int i) const {
    return i < kBpLds ? lds[i * stride] : spill[i - kBpLds];
  }
};

__global__ __launch_bounds__(kBlk, 3) void k_bp(Geo g, Lists L, int64_t c0, int64_t ncombo_arg) {
  const int B = (int)blockDim.x;
  const int64_t ncombo = list_count(L, ncombo_arg, L.cap_combo, 2);
  __shared__ AllocLds sh;
  __shared__ double s_bp[kBpLds * kBlk];
  unsigned long long nmiss = 0;
  double spill[kMaxBp - kBpLds];
  BpLds bp{s_bp + threadIdx.x, B, spill};
  for (int64_t base = (int64_t)blockIdx.x * B; base < ncombo; base += (int64_t)gridDim.x * B) {
    const int64_t k = base + threadIdx.x;
    const bool v = k < ncombo;
    int nb = 0;
    unsigned np = 0;
    unsigned long long miss = 0;   // pieces (by start breakpoint) found empty by the ray test
    if (v) {
      const uint32_t key = L.key[k];
      const int64_t cg = c0 + (key >> kKeyShift);
      const int q = (int)(key & kKeyQ);
      const int32_t i = g.rows[cg];
      const int32_t col = g.cols[cg];
      const TrialRec& T = g.trial[col];
      const double* xq = g.apex + ((int64_t)i * g.maxq + q) * 4;
      double x4[4] = {xq[0], xq[1], xq[2], xq[3]};
      Apex A;
      apex_of(T, x4, A);
      double wlo = 0.0, whi = 0.0;
      if (w_range(T, A, wlo, whi)) {
        ComboL cb;
#pragma unroll
        for (int f = 0; f < 4; ++f) {
          cb.C[f] = A.C[f]; cb.fa[f] = T.fa[f]; cb.fb[f] = T.fb[f]; cb.fc[f] = T.fc[f];
        }
        cb.d2 = A.d * A.d; cb.wlo = wlo; cb.whi = whi;
        store_combo(L, k, cb, col);
        if (g.mixed && apex_far(T, x4, g.eta_far)) L.key[k] = key | kKeyFar;
        nb = breakpoints_t(T, g.fang[col], A, bp);
        // the 8-wide network when every lane of the wave has at most 8
        // breakpoints (about half the waves), the 16-wide one otherwise
        if (__ballot(nb > 8) == 0) sort_net<8>(bp, nb);
        else sort_bp_t(bp, nb);
        if (nb == 0) {
          np = 2;
        } else {
          const ShadowWedge W = shadow_wedge(T, A);
          for (int m = 0; m < nb; ++m) {
            const double a = bp.get(m);
            double e = (m + 1 < nb) ? bp.get(m + 1) : bp.get(0) + kTwoPi;
            const bool pos = e - a > 0.0;
            const bool wm = pos & wedge_misses(W, a, e - a);
            miss |= (uint64_t)wm << m;
            nmiss += wm ? 1 : 0;
            np += (pos && !wm) ? 1u : 0u;
          }
        }
      }
    }
    const unsigned long long p0 = block_alloc(L.cnt + CNT_PIECE, np, sh);
    if (v) {
      L.p0[k] = (int32_t)std::min<unsigned long long>(p0, 0x7fffffffull);
      L.np[k] = (int32_t)np;
      if (np && p0 + np <= (unsigned long long)L.cap_piece) {
        if (nb == 0) {
          for (int h = 0; h < 2; ++h) {
            L.pa[p0 + h] = (double)h;
            L.ph[p0 + h] = -1.0;
            L.pc[p0 + h] = (int32_t)k;
          }
        } else {
          unsigned long long s = p0;
          for (int m = 0; m < nb; ++m) {
            double a = bp.get(m);
            double e = (m + 1 < nb) ? bp.get(m + 1) : bp.get(0) + kTwoPi;
            const bool keep = (e - a > 0.0) && !((miss >> m) & 1ull);
            if (keep) {
              L.pa[s] = a;
              L.ph[s] = e - a;
              L.pc[s] = (int32_t)k;
            }
            s += keep ? 1 : 0;
          }
        }
      }
    }
  }
  block_count(L.cnt + CNT_MISS, nmiss);
}

// The empty-piece test, kEmptyPer pieces per lane and pass: a wave takes
// kEmptyPer runs of 64 consecutive pieces (coalesced reads; the job lists
// keep piece order), so that one list allocation covers 64 kEmptyPer
// pieces.  L at the midpoint (k_empty); the pieces where it is zero are
// queued for the quarter points (k_quarter).
constexpr int kEmptyPer = 8;

// Job lists the empty-piece test routes a non-empty piece to.
// One-gap recipes whose two endpoints are both q / e roots (nearly all of
// them) go to the front of the one-gap list, the other one-gap recipes to
// its back (filled downward from the end).
enum { JOB_R1Q = 0, JOB_R2 = 1, JOB_FULL = 2, JOB_FP32 = 3, JOB_R1X = 4 };

// Pieces narrower than this take the full evaluation: their nodes sit
// within rounding of the breakpoints, where the structure is ambiguous.
constexpr double kRecipeMinH = 1e-8;

// Route of a non-empty piece among the FP64 node kernels by its recipe.
__device__ __forceinline__ unsigned route_fp64(const Lists& L, int32_t p, uint32_t rec) {
  const double H = L.ph[p];
  const int ng = recipe_gaps(rec);
  if (rec == 0u || !(H >= kRecipeMinH)) return JOB_FULL;
  if (ng != 1) return JOB_R2;
  const uint32_t i0 = (rec >> 4) & 15u, i1 = rec & 15u;
  const bool qe = i0 >= 2 && i1 >= 2 && !((i0 - 2) & 1u) && !((i1 - 2) & 1u);
  return qe ? JOB_R1Q : JOB_R1X;
}

__device__ __forceinline__ unsigned route_of(const Lists& L, int32_t p, uint32_t rec) {
  if (L.key[L.pc[p]] & kKeyFar) return JOB_FP32;
  return route_fp64(L, p, rec);
}

// Job lists of one pass: every lane routes up to kEmptyPer pieces (3 bits
// of route each in `route`, presence in `has`, piece j from piece_of(j)).
// Slots are handed out per wave, for the six lists at once: the lane's
// counts (at most kEmptyPer each) in 10-bit fields of one 64-bit word, one
// shuffle scan over the wave, and lane f reserves list f's slots with one
// atomic when the wave has any (no block barriers; the rare lists are
// rarely touched).  Every lane of the wave must call it.
constexpr int JOB_QZ = 5;   // not a job list: the queue for the quarter points
static_assert(kEmptyPer * 64 < 1024, "per-wave list counts fit 10 bits");

template <class F>
__device__ __forceinline__ void route_pieces(Lists& L, unsigned has, unsigned route, F piece_of) {
  const int lane = threadIdx.x & 63;
  unsigned long long v = 0;
  for (int j = 0; j < kEmptyPer; ++j)
    if ((has >> j) & 1u) v += 1ull << (10 * ((route >> (3 * j)) & 7u));
  unsigned long long incl = v;
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    const unsigned long long t = __shfl_up(incl, off, 64);
    if (lane >= off) incl += t;
  }
  const unsigned long long tot = __shfl(incl, 63, 64);
  unsigned long long b = 0;
  if (lane < 6) {
    const int ctr = lane == JOB_R1Q ? CNT_JOB : lane == JOB_R2 ? CNT_JOB2 : lane == JOB_FULL ? CNT_JOBF
                  : lane == JOB_FP32 ? CNT_JOB32 : lane == JOB_R1X ? CNT_JOB1X : CNT_QZ;
    const unsigned long long n = (tot >> (10 * lane)) & 1023u;
    if (n) b = atomicAdd(L.cnt + ctr, n);
  }
  const unsigned long long ex = incl - v;
  // the one-gap q/e jobs (nearly every piece) in piece order: item j of
  // every lane before item j + 1, lanes in order within an item, so that
  // neighbouring jobs read neighbouring pieces and combos
  unsigned long long s0 = __shfl(b, JOB_R1Q, 64);
  const unsigned long long below = (1ull << lane) - 1ull;
  for (int j = 0; j < kEmptyPer; ++j) {
    const bool q = ((has >> j) & 1u) && ((route >> (3 * j)) & 7u) == JOB_R1Q;
    const unsigned long long bal = __ballot(q);
    if (q) L.job[s0 + __popcll(bal & below)] = piece_of(j);
    s0 += __popcll(bal);
  }
  unsigned long long s1 = __shfl(b, JOB_R2, 64) + ((ex >> 10) & 1023u);
  unsigned long long s2 = __shfl(b, JOB_FULL, 64) + ((ex >> 20) & 1023u);
  unsigned long long s3 = __shfl(b, JOB_FP32, 64) + ((ex >> 30) & 1023u);
  unsigned long long s4 = __shfl(b, JOB_R1X, 64) + ((ex >> 40) & 1023u);
  unsigned long long s5 = __shfl(b, JOB_QZ, 64) + ((ex >> 50) & 1023u);
  // the other lists: only the lane's items that go there (nearly always
  // none or one of its kEmptyPer), so the wave runs the slowest lane's few
  unsigned rare = 0;
  for (int j = 0; j < kEmptyPer; ++j)
    rare |= (((has >> j) & 1u) && ((route >> (3 * j)) & 7u) != JOB_R1Q ? 1u : 0u) << j;
  while (rare) {
    const int j = __ffs(rare) - 1;
    rare &= rare - 1u;
    const unsigned r = (route >> (3 * j)) & 7u;
    const int32_t p = piece_of(j);
    int32_t* dst = r == JOB_R2 ? L.job2 + s1 : r == JOB_FULL ? L.jobf + s2 : r == JOB_FP32 ? L.job32 + s3
                 : r == JOB_R1X ? L.job + (L.cap_piece - 1 - (int64_t)s4) : L.pz + s5;
    *dst = p;
    s1 += r == JOB_R2 ? 1 : 0;
    s2 += r == JOB_FULL ? 1 : 0;
    s3 += r == JOB_FP32 ? 1 : 0;
    s4 += r == JOB_R1X ? 1 : 0;
    s5 += r == JOB_QZ ? 1 : 0;
  }
}

// The empty-piece test at the midpoints: L and its recipe there; the
// non-empty pieces go to the job lists, the others to the queue of pieces
// whose quarter points decide (k_quarter).  The quarter-point path has a
// kernel of its own so that this one, run on every piece, needs fewer
// registers and keeps more waves resident.
__global__ __launch_bounds__(kBlk, 4) void k_empty(Lists L, int64_t npiece_arg) {
  const int B = (int)blockDim.x;
  const int64_t npiece = list_count(L, npiece_arg, L.cap_piece, 3);
  unsigned long long ev_mid = 0;
  const int64_t step = (int64_t)gridDim.x * B * kEmptyPer;
  for (int64_t base = (int64_t)blockIdx.x * B * kEmptyPer; base < npiece; base += step) {
    unsigned has = 0, route = 0;   // route: 3 bits per item
    // each wave takes kEmptyPer runs of 64 consecutive pieces
    const int64_t wbase = base + (int64_t)(threadIdx.x >> 6) * 64 * kEmptyPer + (threadIdx.x & 63);
    auto piece_of = [&](int j) { return (int32_t)(wbase + (int64_t)j * 64); };
#pragma unroll 1
    for (int j = 0; j < kEmptyPer; ++j) {
      const int64_t p = wbase + (int64_t)j * 64;
      if (p >= npiece) break;
      const double H = L.ph[p];
      bool nz = true;   // trapezoid half (H < 0): always evaluated
      uint32_t rec = 0u;
      if (!(H < 0.0)) {
        double sn, cs;
        sincos_small(L.pa[p] + 0.5 * H, &sn, &cs);
        nz = L_eval_recipe(load_combo(L, L.pc[p]), cs, sn, &rec) != 0.0;
        ++ev_mid;
      }
      L.pne[p] = nz ? 1 : 0;
      L.prec[p] = rec;
      has |= 1u << j;
      route |= (nz ? route_of(L, (int32_t)p, rec) : (unsigned)JOB_QZ) << (3 * j);
    }
    route_pieces(L, has, route, piece_of);
  }
  block_count(L.cnt + CNT_EVAL_MID, ev_mid);
}

// The queued pieces (L zero at the midpoint): L at the quarter points; the
// recipe of a piece found non-empty is taken at the point that decided.
__global__ __launch_bounds__(kBlk, 3) void k_quarter(Lists L, int64_t nq_arg) {
  const int B = (int)blockDim.x;
  const int64_t nq = list_count(L, nq_arg, L.cap_piece, 3);
  unsigned long long ev_quarter = 0;
  const int64_t step = (int64_t)gridDim.x * B * kEmptyPer;
  for (int64_t base = (int64_t)blockIdx.x * B * kEmptyPer; base < nq; base += step) {
    unsigned ne = 0, route = 0;
    auto piece_of = [&](int j) { return L.pz[base + (int64_t)j * B + threadIdx.x]; };
#pragma unroll 1
    for (int j = 0; j < kEmptyPer; ++j) {
      const int64_t e = base + (int64_t)j * B + threadIdx.x;
      if (e >= nq) break;
      const int32_t p = L.pz[e];
      const ComboL cb = load_combo(L, L.pc[p]);
      const double a = L.pa[p], H = L.ph[p];
      // the test in plain arithmetic; the recipe only for the (few) pieces
      // it finds non-empty, at the point that decided
      // (both points, independent of each other: a wave nearly always has a
      // lane that needs the second)
      uint32_t rec = 0u;
      const double v1 = L_at(cb, a + 0.25 * H), v3 = L_at(cb, a + 0.75 * H);
      const bool nz = v1 != 0.0 || v3 != 0.0;
      const double phq = v1 != 0.0 ? a + 0.25 * H : a + 0.75 * H;
      ev_quarter += 2;
      if (nz) {
        double sn, cs;
        sincos_small(phq, &sn, &cs);
        (void)L_eval_recipe(cb, cs, sn, &rec);
        L.pne[p] = 1;
        L.prec[p] = rec;
        route |= route_of(L, p, rec) << (3 * j);
      }
      ne |= (nz ? 1u : 0u) << j;
    }
    route_pieces(L, ne, route, piece_of);
  }
  block_count(L.cnt + CNT_EVAL_QUARTER, ev_quarter);
}

// The n_g nodes of a piece by its recipe (NG gaps): per node only the
// endpoint formulas of the recipe, not all four faces (see L_eval_recipe).
// jobs_arg: the job list, or nullptr for the one-gap list's back part (its
// last njob slots of L.job); njob_arg as for list_count.
template <int NG, bool QE>
__global__ __launch_bounds__(kBlk, 4) void k_nodes_rec(Lists L, const int32_t* __restrict__ jobs_arg,
                                                       int64_t njob_arg, const double* __restrict__ gl,
                                                       int ng, int ctr) {
  const int B = (int)blockDim.x;
  unsigned long long evals = 0;
  const int64_t njob = list_count(L, njob_arg, L.cap_piece, 3);
  const int32_t* __restrict__ jobs = jobs_arg ? jobs_arg : L.job + (L.cap_piece - njob);
  for (int64_t base = (int64_t)blockIdx.x * B; base < njob; base += (int64_t)gridDim.x * B) {
    const int64_t k = base + threadIdx.x;
    if (k >= njob) continue;
    const int32_t p = jobs[k];
    const double H = L.ph[p], a = L.pa[p];
    const uint32_t rec = L.prec[p];
    const int64_t c = L.pc[p];
    const int64_t cap = L.cap_combo;
    const double d2 = L.cb[kCbD2 * cap + c], wlo = L.cb[kCbWlo * cap + c],
                 whi = L.cb[kCbWhi * cap + c];
    Endpoint E[2 * NG];
#pragma unroll
    for (int g = 0; g < NG; ++g) {
      E[2 * g] = endpoint_load(L, c, (rec >> (8 * g + 4)) & 15u, wlo, whi);
      E[2 * g + 1] = endpoint_load(L, c, (rec >> (8 * g)) & 15u, wlo, whi);
    }
    // The nodes come in mirror pairs about the piece's midpoint m:
    // phi = m -+ delta with delta = H (1/2 - s(u_g)) (the Gauss nodes are
    // symmetric and s(1 - u) = 1 - s(u)), sharing one weight.  With
    // P = B(m) and Q = b sin m - c cos m per endpoint face, the addition
    // theorems give B(m -+ delta) = P cos(delta) +- Q sin(delta): one sin/cos
    // per pair, two products per face and node.
    const double m = a + 0.5 * H;
    double sm, cm;
    sincos_small(m, &sm, &cm);
    double P[2 * NG], Q[2 * NG], CC[2 * NG], SG[2 * NG];
#pragma unroll
    for (int e = 0; e < 2 * NG; ++e) {
      P[e] = fma(E[e].fb, cm, E[e].fc * sm);
      Q[e] = fma(E[e].fb, sm, -(E[e].fc * cm));
      CC[e] = E[e].C * E[e].C;
      SG[e] = copysign(1.0, E[e].C);
    }
    // twice L at m - delta (lm) and m + delta (lp): the sum takes the 1/2
    auto L_pair = [&](double cd, double sd, double& lm, double& lp) {
      lm = 0.0;
      lp = 0.0;
#pragma unroll
      for (int g = 0; g < NG; ++g) {
        double vm[2], vp[2];
#pragma unroll
        for (int t = 0; t < 2; ++t) {
          const int e = 2 * g + t;
          endpoint_pair_node<QE>(E[e], P[e], Q[e], CC[e], SG[e], d2, wlo, whi, cd, sd, vm[t], vp[t]);
        }
        // a gap that closed (end <= start) measures 0: rdiff of equal ends,
        // so no branch (w >= |d| > 0 when d^2 > 0; rdiff ignores 1/w at d = 0)
        lm += rdiff2_node(vm[0], fmax(vm[1], vm[0]), d2);
        lp += rdiff2_node(vp[0], fmax(vp[1], vp[0]), d2);
      }
    };
    double acc = 0.0;
    // |delta| < H / 2: a piece shorter than pi (all but the rare long ones)
    // needs no reduction for its sin/cos.  Decided per piece, so that a
    // piece's value does not depend on the pieces that share its wave.
    const bool short_piece = H <= kPi;
    // the next pair's table entries are loaded while this pair is evaluated
    double t_off = gl[2 * kMaxNg], t_wf = gl[3 * kMaxNg];
    for (int gi = 0; gi < (ng >> 1); ++gi) {
      const double off = t_off, wf = t_wf;
      if (gi + 1 < (ng >> 1)) {
        t_off = gl[2 * kMaxNg + gi + 1];
        t_wf = gl[3 * kMaxNg + gi + 1];
      }
      double sd, cd;
      if (short_piece) sincos_half_pi(H * off, &sd, &cd);
      else sincos_small(H * off, &sd, &cd);
      double lm, lp;
      L_pair(cd, sd, lm, lp);
      acc += wf * (lm + lp);
    }
    if (ng & 1) {   // u = 1/2: the midpoint itself
      double lm, lp;
      L_pair(1.0, 0.0, lm, lp);
      acc += (1.5 * gl[kMaxNg + (ng >> 1)]) * lm;
    }
    evals += (unsigned long long)ng;
    // the weights' common factor H, and the 1/2 the doubled r-measures left
    L.pv[p] = (0.5 * H) * acc;
  }
  block_count(L.cnt + ctr, evals);
}

// The n_g nodes of one piece.  Gauss piece [a, a + H]: phi = a + H s(u_g),
// weight H s'(u_g) w_g with s(u) = 3u^2 - 2u^3.  Trapezoid half h of the
// period (no breakpoints): phi = (h n_g + g) 2 pi / (2 n_g), weight
// 2 pi / (2 n_g).
__global__ __launch_bounds__(kBlk, 4) void k_nodes(Lists L, const int32_t* __restrict__ jobs,
                                                   int64_t njob_arg, const double* __restrict__ gl,
                                                   int ng, int ctr) {
  const int B = (int)blockDim.x;
  unsigned long long evals = 0;
  const int64_t njob = list_count(L, njob_arg, L.cap_piece, 3);
  const double ht = kTwoPi / (2 * ng);
  for (int64_t base = (int64_t)blockIdx.x * B; base < njob; base += (int64_t)gridDim.x * B) {
    const int64_t k = base + threadIdx.x;
    if (k >= njob) continue;
    const int32_t p = jobs[k];
    const double H = L.ph[p], a = L.pa[p];
    const ComboL cb = load_combo(L, L.pc[p]);
    const bool trap = H < 0.0;
    double acc = 0.0;
    for (int gi = 0; gi < ng; ++gi) {
      const double u = gl[gi];
      const double s = u * u * (3.0 - 2.0 * u);
      const double ds = 6.0 * u * (1.0 - u);
      const double phi = trap ? (a * ng + gi) * ht : a + H * s;
      const double wt = trap ? ht : (H * ds) * gl[kMaxNg + gi];
      acc += wt * L_at(cb, phi);
    }
    evals += (unsigned long long)ng;
    L.pv[p] = acc;
  }
  block_count(L.cnt + ctr, evals);
}

// The n_g nodes of a far piece in mixed precision: node angle, sin/cos and
// the per-face coefficients in FP64, root solves and interval measure in
// FP32 (L_eval_far), node sum in FP32 with Kahan compensation.
__global__ __launch_bounds__(kBlk, 4) void k_nodes32(Lists L, int64_t njob_arg,
                                                     const double* __restrict__ gl, int ng) {
  const int B = (int)blockDim.x;
  unsigned long long evals = 0;
  const int64_t njob = list_count(L, njob_arg, L.cap_piece, 3);
  const double ht = kTwoPi / (2 * ng);
  for (int64_t base = (int64_t)blockIdx.x * B; base < njob; base += (int64_t)gridDim.x * B) {
    const int64_t k = base + threadIdx.x;
    if (k >= njob) continue;
    const int32_t p = L.job32[k];
    const double H = L.ph[p], a = L.pa[p];
    const ComboL cb = load_combo(L, L.pc[p]);
    const FarConst F = far_const(cb);
    const bool trap = H < 0.0;
    float acc = 0.0f, comp = 0.0f, eacc = 0.0f;
    for (int gi = 0; gi < ng; ++gi) {
      const double u = gl[gi];
      const double s = u * u * (3.0 - 2.0 * u);
      const double ds = 6.0 * u * (1.0 - u);
      const double phi = trap ? (a * ng + gi) * ht : a + H * s;
      const double wt = trap ? ht : (H * ds) * gl[kMaxNg + gi];
      double sn, cs;
      sincos_small(phi, &sn, &cs);
      float el;
      const float term = (float)wt * L_eval_far(cb, F, cs, sn, &el);
      eacc = fmaf((float)wt, el, eacc);
      const float y = term - comp;
      const float t = acc + y;
      comp = (t - acc) - y;
      acc = t;
    }
    evals += (unsigned long long)ng;
    L.pv[p] = (double)acc;
    // the bound also covers the summation: Kahan leaves O(ulp) of the sum.
    // The piece is non-empty (its FP64 test found L > 0): a sum of zero means
    // FP32 lost the whole lit sliver, so the entry must be recomputed.
    L.pe[p] = acc == 0.0f ? INFINITY : eacc + 1.2e-7f * fabsf(acc);
  }
  block_count(L.cnt + CNT_EVAL_NODES32, evals);
}

__global__ __launch_bounds__(kBlk) void k_combine(Lists L, int64_t ncombo_arg) {
  const int64_t ncombo = list_count(L, ncombo_arg, L.cap_combo, 3);
  int64_t k = (int64_t)blockIdx.x * kBlk + threadIdx.x;
  for (; k < ncombo; k += (int64_t)gridDim.x * kBlk) {
    const int32_t p0 = L.p0[k], np = L.np[k];
    // empty pieces have no node sum (not written); far combos' non-empty
    // pieces went through the FP32 nodes and carry a rounding bound
    const bool far = (L.key[k] & kKeyFar) != 0;
    double I = 0.0;
    float e = 0.0f;
    for (int s = 0; s < np; ++s) {
      if (!L.pne[p0 + s]) continue;
      I += L.pv[p0 + s];
      if (far) e += L.pe[p0 + s];
    }
    L.I[k] = I / (4.0 * kPi);
    L.Ie[k] = e * (float)(1.0 / (4.0 * kPi));
  }
}

// Matrix: out[c] = sum over lit apexes q (ascending) of w_q I_q, skipping
// exact zeros; a candidate with any lit apex is a causal pair.  Potential:
// out[c] = I of the single apex (0 when not lit).
//
// Mixed precision (check = 1): the entry is a sum of outer-point terms that
// can cancel (the energetic form differences the test panel's top and
// bottom faces), so a small relative error of the far terms can be a large
// one of the entry.  Each far I_q carries a first-order bound of its FP32
// rounding error (from the node evaluations, see L_eval_far); when
// sum_q |w_q| bound_q exceeds kMixedTol |entry|, the candidate is flagged for
// recomputation with FP64 nodes.  The largest error/bound ratio seen is
// 0.32, so kMixedTol = 3e-6 keeps every kept FP32 entry within
// 0.32 * 3e-6 < 1e-6 of its FP64 value without relying on the terms' errors
// cancelling.  Causal pairs are counted when check = 0.
constexpr double kMixedTol = 3e-6;

// Segment of global candidate cg: last s with off[s] <= cg.
__device__ __forceinline__ int seg_of(const int64_t* off, int nseg, int64_t cg) {
  int lo = 0, hi = nseg;
  while (hi - lo > 1) {
    int mid = (lo + hi) >> 1;
    if (off[mid] <= cg) lo = mid; else hi = mid;
  }
  return lo;
}

__global__ __launch_bounds__(kBlk) void k_store(Geo g, Lists L, int64_t c0, int64_t nc,
                                                double* __restrict__ out, int check, int nseg,
                                                const int64_t* __restrict__ seg_off,
                                                unsigned long long* __restrict__ seg_causal) {
  // a chunk whose lists overflowed is redone by the host: write nothing
  if (L.cnt[CNT_DEEP] > (unsigned long long)L.cap_combo || L.cnt[CNT_COMBO] > (unsigned long long)L.cap_combo ||
      L.cnt[CNT_PIECE] > (unsigned long long)L.cap_piece)
    return;
  unsigned long long causal = 0, redo = 0;
  for (int64_t base = (int64_t)blockIdx.x * kBlk; base < nc; base += (int64_t)gridDim.x * kBlk) {
    const int64_t c = base + threadIdx.x;
    bool is_causal = false;
    if (c < nc) {
      const uint64_t m = L.mask[c];
      int32_t idx = L.combo0[c];
      double s = 0.0, bound = 0.0;
      if (g.apex_w) {
        const int32_t i = g.rows[c0 + c];
        const double* wq = g.apex_w + (int64_t)i * g.maxq;
        const int nq = g.apex_n ? g.apex_n[i] : 1;
        for (int q = 0; q < nq; ++q) {
          if (!((m >> q) & 1ull)) continue;
          const int32_t k = idx++;
          const double I = L.I[k];
          if (I != 0.0) s += wq[q] * I;
          if (check && (L.key[k] & kKeyFar)) bound += fabs(wq[q]) * (double)L.Ie[k];
        }
      } else if (m) {
        s = L.I[idx];
      }
      out[c0 + c] = s;
      if (g.lit_out) g.lit_out[c0 + c] = m ? 1 : 0;
      if (check) {
        const bool r = bound > kMixedTol * fabs(s);
        L.redo[c] = r ? 1 : 0;
        redo += r ? 1ull : 0ull;
      } else {
        causal += m ? 1ull : 0ull;
        is_causal = m != 0;
      }
    }
    if (seg_off && !check) {
      // per-segment counts: one atomic per wave unless the wave straddles
      // a segment boundary (candidates of a wave are consecutive)
      const int lane = threadIdx.x & 63;
      const int64_t cf = c0 + base + (threadIdx.x & ~63);
      const int64_t cl = std::min<int64_t>(cf + 63, c0 + nc - 1);
      const uint64_t bal = __ballot(is_causal);
      if (cf <= cl) {
        const int sa = seg_of(seg_off, nseg, cf), sb = seg_of(seg_off, nseg, cl);
        if (sa == sb) {
          if (lane == 0 && bal) atomicAdd(seg_causal + sa, (unsigned long long)__popcll(bal));
        } else if (is_causal) {
          atomicAdd(seg_causal + seg_of(seg_off, nseg, c0 + c), 1ull);
        }
      }
    }
  }
  block_count(L.cnt + CNT_CAUSAL, causal);
  block_count(L.cnt + CNT_REDO, redo);
}

// Mixed precision: the non-empty pieces of the far combos of every flagged
// candidate go to the FP64 node kernels again, routed by their recipes as in
// the FP64 pass (the job lists and their counters start empty), so that a
// recomputed entry is the FP64 assembly's value through the same outer
// points, bit for bit.
__global__ __launch_bounds__(kBlk) void k_redo(Geo g, Lists L, int64_t nc) {
  __shared__ AllocLds sh;
  for (int64_t base = (int64_t)blockIdx.x * kBlk; base < nc; base += (int64_t)gridDim.x * kBlk) {
    const int64_t c = base + threadIdx.x;
    const bool v = c < nc && L.redo[c];
    unsigned cnt[5] = {0, 0, 0, 0, 0};
    int32_t k0 = 0, nk = 0;
    if (v) {
      k0 = L.combo0[c];
      nk = __popcll(L.mask[c]);
      for (int32_t k = k0; k < k0 + nk; ++k) {
        if (!(L.key[k] & kKeyFar)) continue;
        for (int32_t p = L.p0[k]; p < L.p0[k] + L.np[k]; ++p)
          if (L.pne[p]) ++cnt[route_fp64(L, p, L.prec[p])];
      }
    }
    unsigned long long sl[5];
    sl[JOB_R1Q] = block_alloc(L.cnt + CNT_JOB, cnt[JOB_R1Q], sh);
    sl[JOB_R2] = block_alloc(L.cnt + CNT_JOB2, cnt[JOB_R2], sh);
    sl[JOB_FULL] = block_alloc(L.cnt + CNT_JOBF, cnt[JOB_FULL], sh);
    sl[JOB_R1X] = block_alloc(L.cnt + CNT_JOB1X, cnt[JOB_R1X], sh);
    if (v) {
      for (int32_t k = k0; k < k0 + nk; ++k) {
        if (!(L.key[k] & kKeyFar)) continue;
        for (int32_t p = L.p0[k]; p < L.p0[k] + L.np[k]; ++p) {
          if (!L.pne[p]) continue;
          const unsigned r = route_fp64(L, p, L.prec[p]);
          if (r == JOB_R1X) L.job[L.cap_piece - 1 - (int64_t)(sl[r]++)] = p;
          else if (r == JOB_R1Q) L.job[sl[r]++] = p;
          else if (r == JOB_R2) L.job2[sl[r]++] = p;
          else L.jobf[sl[r]++] = p;
        }
      }
    }
  }
}

unsigned grid_for(int64_t n, int per = 1, int block = kBlk, int64_t max_blocks = kMaxBlocks) {
  int64_t b = (n + (int64_t)block * per - 1) / ((int64_t)block * per);
  return (unsigned)std::max<int64_t>(1, std::min<int64_t>(b, max_blocks));
}

}  // namespace

// ------------------------------------------------------------------ host

struct PairWorkspace {
  int64_t cap_cand = 0, cap_combo = 0, cap_piece = 0;
  void* base = nullptr;
  Lists L{};
};

void stb_free_workspace(stb_ctx* ctx) {
  if (!ctx->ws) return;
  dfree(ctx->ws->base);
  delete ctx->ws;
  ctx->ws = nullptr;
}

static size_t align256(size_t b) { return (b + 255) & ~size_t(255); }

// Lay the lists out in one allocation.
static size_t scan_bytes_for(int64_t cc) {
  return (size_t)stb_scan_tmp_elems<int32_t>(cc) * sizeof(int32_t);
}

static size_t ws_bytes(int64_t cc, int64_t cb, int64_t cp) {
  size_t b = 0;
  b += 2 * align256((cc + 1) * 4) + align256(scan_bytes_for(cc));
  b += align256(cc * 8) + align256(cc * 4);
  b += 2 * align256(cb * 4) + align256(cb * kComboStored * 8) + align256(cb * 4) + 2 * align256(cb * 4) +
       align256(cb * 8);
  b += 2 * align256(cp * 8) + align256(cp * 4) + align256(cp * 8) + 2 * align256(cp * 4);
  b += align256(cp) + align256(cc) + align256(cb * 4) + align256(cp * 4);
  b += 3 * align256(cp * 4);
  b += align256(CNT_N * 8);
  return b;
}

// List capacities a run over nnz candidates with maxq apexes each asks for.
static void ws_want(int64_t nnz, int maxq, int64_t* cc, int64_t* cb, int64_t* cp) {
  const int64_t kCandMax = std::min<int64_t>((int64_t)1 << (32 - kKeyShift),
                                             (int64_t)INT32_MAX / std::max(maxq, 1));
  *cc = std::min<int64_t>(nnz, kCandMax);
  *cb = std::min<int64_t>(*cc * maxq, (int64_t)1 << 27);
  *cp = std::min<int64_t>(*cb * 8, (int64_t)1 << 28);
}

int64_t stb_pairs_ws_held(const stb_ctx* ctx) {
  const PairWorkspace* w = ctx->ws;
  return w ? (int64_t)ws_bytes(w->cap_cand, w->cap_combo, w->cap_piece) : 0;
}

int64_t stb_pairs_ws_need(const stb_ctx* ctx, int64_t nnz, int maxq) {
  if (nnz <= 0) return stb_pairs_ws_held(ctx);
  int64_t cc, cb, cp;
  ws_want(nnz, maxq, &cc, &cb, &cp);
  const PairWorkspace* w = ctx->ws;
  if (w) {
    if (w->cap_cand >= cc && w->cap_combo >= cb && w->cap_piece >= cp) return stb_pairs_ws_held(ctx);
    cc = std::max(cc, w->cap_cand);
    cb = std::max(cb, w->cap_combo);
    cp = std::max(cp, w->cap_piece);
  }
  return (int64_t)ws_bytes(cc, cb, cp);
}

static stb_status ensure_workspace(stb_ctx* ctx, int64_t want_cand, int64_t want_combo,
                                   int64_t want_piece) {
  PairWorkspace* w = ctx->ws;
  if (w && w->cap_cand >= want_cand && w->cap_combo >= want_combo && w->cap_piece >= want_piece)
    return STB_OK;
  if (w) {
    want_cand = std::max(want_cand, w->cap_cand);
    want_combo = std::max(want_combo, w->cap_combo);
    want_piece = std::max(want_piece, w->cap_piece);
  }
  stb_free_workspace(ctx);
  void* base = nullptr;
  // halve the request until it fits
  for (;;) {
    if (hipMalloc(&base, ws_bytes(want_cand, want_combo, want_piece)) == hipSuccess) break;
    (void)hipGetLastError();
    base = nullptr;
    if (want_combo <= 4096) return stb_fail(ctx, STB_E_NO_MEMORY, "pair workspace does not fit");
    want_cand = std::max<int64_t>(want_cand / 2, 1024);
    want_combo /= 2;
    want_piece /= 2;
  }
  w = new PairWorkspace();
  w->base = base;
  w->cap_cand = want_cand;
  w->cap_combo = want_combo;
  w->cap_piece = want_piece;
  char* p = (char*)base;
  auto take = [&](size_t bytes) { char* r = p; p += align256(bytes); return (void*)r; };
  Lists& L = w->L;
  L.scan_bytes = scan_bytes_for(want_cand);
  L.ccnt = (int32_t*)take((want_cand + 1) * 4);
  L.coff = (int32_t*)take((want_cand + 1) * 4);
  L.scan_tmp = take(L.scan_bytes);
  L.mask = (uint64_t*)take(want_cand * 8);
  L.combo0 = (int32_t*)take(want_cand * 4);
  L.key = (uint32_t*)take(want_combo * 4);
  L.deep = (uint32_t*)take(want_combo * 4);
  L.cb = (double*)take(want_combo * kComboStored * 8);
  L.ccol = (int32_t*)take(want_combo * 4);
  L.p0 = (int32_t*)take(want_combo * 4);
  L.np = (int32_t*)take(want_combo * 4);
  L.I = (double*)take(want_combo * 8);
  L.Ie = (float*)take(want_combo * 4);
  L.pa = (double*)take(want_piece * 8);
  L.ph = (double*)take(want_piece * 8);
  L.pc = (int32_t*)take(want_piece * 4);
  L.pv = (double*)take(want_piece * 8);
  L.pz = reinterpret_cast<int32_t*>(L.pv);
  L.pe = (float*)take(want_piece * 4);
  L.job = (int32_t*)take(want_piece * 4);
  L.job2 = (int32_t*)take(want_piece * 4);
  L.jobf = (int32_t*)take(want_piece * 4);
  L.prec = (uint32_t*)take(want_piece * 4);
  L.job32 = (int32_t*)take(want_piece * 4);
  L.pne = (uint8_t*)take(want_piece);
  L.redo = (uint8_t*)take(want_cand);
  L.cnt = (unsigned long long*)take(CNT_N * 8);
  L.cap_cand = want_cand;
  L.cap_combo = want_combo;
  L.cap_piece = want_piece;
  ctx->ws = w;
  return STB_OK;
}

stb_status stb_run_pairs(stb_ctx* ctx, const PairJob& job, unsigned long long work[4]) {
  for (int k = 0; k < 4; ++k) work[k] = 0;
  if (job.nnz <= 0) return STB_OK;
  // sizes: the whole candidate set when it is small, else chunks of up to
  // 2^25 candidates (the combo key holds 25 bits of candidate index; the
  // int32 combo offsets, at most maxq per candidate, bound it too)
  int64_t want_cand, want_combo, want_piece;
  ws_want(job.nnz, job.maxq, &want_cand, &want_combo, &want_piece);
  int64_t* const want[3] = {&want_cand, &want_combo, &want_piece};
  for (int k = 0; k < 3; ++k)
    if (ctx->list_limit[k]) *want[k] = std::min(*want[k], ctx->list_limit[k]);
  stb_status s = ensure_workspace(ctx, want_cand, want_combo, want_piece);
  if (s) return s;
  PairWorkspace* w = ctx->ws;
  Lists L = w->L;
  // the lists' lengths in use: the workspace's, within the caller's limits
  // (the combo fields' stride follows cap_combo, so a shorter length only
  // narrows the fields inside their allocation)
  if (ctx->list_limit[0]) L.cap_cand = std::min(L.cap_cand, ctx->list_limit[0]);
  if (ctx->list_limit[1]) L.cap_combo = std::min(L.cap_combo, ctx->list_limit[1]);
  if (ctx->list_limit[2]) L.cap_piece = std::min(L.cap_piece, ctx->list_limit[2]);
  L.trial = job.trial;
  Geo g;
  g.rows = job.rows; g.cols = job.cols; g.trial = job.trial; g.fang = job.fang;
  g.lit_out = job.lit_out;
  g.apex = job.apex; g.apex_w = job.apex_w; g.apex_n = job.apex_n; g.maxq = job.maxq;
  g.mixed = job.mixed ? 1 : 0;
  g.eta_far = job.eta_far;
  hipStream_t st = ctx->stream;
  unsigned long long h[CNT_N];
  // first guess: ~4 lit apexes and ~4 pieces per lit apex; adapted below
  int64_t chunk = std::min<int64_t>(L.cap_cand, std::max<int64_t>(1, L.cap_combo / 4));
  chunk = std::min<int64_t>(chunk, std::max<int64_t>(1, L.cap_piece / 16));
  int64_t c0 = 0;
  // device count argument of list counter k (see list_count)
  auto dev = [](int k) { return -(int64_t)k - 1; };
  for (int k = 0; k < 8; ++k) { ctx->kern_ms[k] = 0.0; ctx->kern_n[k] = 0; ctx->kern_units[k] = 0; }
  for (int k = 0; k < 4; ++k) ctx->path_counts[k] = 0;
  for (auto& e : ctx->kev)
    if (!e) HIPCHK(ctx, hipEventCreate(&e));
  bool used[8] = {false, false, false, false, false, false, false, false};
  // brackets a launch of kernel kind k with events (per chunk, read after
  // the chunk's synchronisation)
  auto t0 = [&](int k) { used[k] = true; return hipEventRecord(ctx->kev[2 * k], st); };
  if (!ctx->ncu) {
    HIPCHK(ctx, hipDeviceGetAttribute(&ctx->ncu, hipDeviceAttributeMultiprocessorCount, ctx->device));
    if (ctx->ncu < 1) ctx->ncu = 1;
  }
  // grid of stage k: enough blocks for n items (per items per thread), at
  // most the stage's blocks per CU times the CU count
  auto gfor = [&](int k, unsigned long long n, int per = 1) {
    return grid_for((int64_t)n, per, ctx->tune_block[k], (int64_t)ctx->tune_per_cu[k] * ctx->ncu);
  };
  auto t1 = [&](int k) { return hipEventRecord(ctx->kev[2 * k + 1], st); };
  while (c0 < job.nnz) {
    const int64_t nc = std::min<int64_t>(chunk, job.nnz - c0);
    for (auto& u : used) u = false;
    HIPCHK(ctx, hipMemsetAsync(L.cnt, 0, CNT_N * 8, st));
    HIPCHK(ctx, t0(0));
    hipLaunchKernelGGL(k_lit, dim3(gfor(0, nc)), dim3(ctx->tune_block[0]), 0, st, g, L, c0, nc);
    HIPCHK(ctx, hipGetLastError());
    // the consumers read their counts from the device counters (see
    // list_count); grids for the lists' upper bounds: at most maxq lit
    // apexes per candidate, at most the piece list's capacity of jobs
    const int64_t ub_combo = std::min<int64_t>(nc * job.maxq, L.cap_combo);
    const int64_t ub_piece = L.cap_piece;
    hipLaunchKernelGGL(k_lit_deep, dim3(gfor(0, ub_combo)), dim3(ctx->tune_block[0]), 0, st, g, L, c0,
                       dev(CNT_DEEP));
    hipLaunchKernelGGL(k_emit_count, dim3((unsigned)((nc + 1 + 255) / 256)), dim3(256), 0, st, L, nc);
    HIPCHK(ctx, hipGetLastError());
    HIPCHK(ctx, stb_scan<int32_t>(L.ccnt, L.coff, nc, (int32_t*)L.scan_tmp, st));
    hipLaunchKernelGGL(k_emit, dim3((unsigned)((nc + 255) / 256)), dim3(256), 0, st, L, nc);
    HIPCHK(ctx, hipGetLastError());
    HIPCHK(ctx, t1(0));
    HIPCHK(ctx, t0(1));
    hipLaunchKernelGGL(k_bp, dim3(gfor(1, ub_combo)), dim3(ctx->tune_block[1]), 0, st, g, L, c0,
                       dev(CNT_COMBO));
    HIPCHK(ctx, hipGetLastError());
    HIPCHK(ctx, t1(1));
    HIPCHK(ctx, t0(2));
    hipLaunchKernelGGL(k_empty, dim3(gfor(2, ub_piece, kEmptyPer)), dim3(ctx->tune_block[2]), 0, st, L,
                       dev(CNT_PIECE));
    hipLaunchKernelGGL(k_quarter, dim3(gfor(2, ub_piece, kEmptyPer)), dim3(ctx->tune_block[2]), 0, st, L,
                       dev(CNT_QZ));
    HIPCHK(ctx, hipGetLastError());
    HIPCHK(ctx, t1(2));
    // FP64 nodes: one-gap recipes (front and back of the one-gap list),
    // two-gap recipes, full evaluations
    HIPCHK(ctx, t0(4));
    hipLaunchKernelGGL((k_nodes_rec<1, true>), dim3(gfor(4, ub_piece)), dim3(ctx->tune_block[4]), 0, st, L,
                       L.job, dev(CNT_JOB), job.gl, job.ng, (int)CNT_EVAL_NODES);
    hipLaunchKernelGGL((k_nodes_rec<1, false>), dim3(gfor(4, ub_piece)), dim3(ctx->tune_block[4]), 0, st,
                       L, nullptr, dev(CNT_JOB1X), job.gl, job.ng, (int)CNT_EVAL_NODES);
    hipLaunchKernelGGL((k_nodes_rec<2, false>), dim3(gfor(4, ub_piece)), dim3(ctx->tune_block[4]), 0, st,
                       L, L.job2, dev(CNT_JOB2), job.gl, job.ng, (int)CNT_EVAL_NODES);
    hipLaunchKernelGGL(k_nodes, dim3(gfor(4, ub_piece)), dim3(ctx->tune_block[4]), 0, st, L, L.jobf,
                       dev(CNT_JOBF), job.gl, job.ng, (int)CNT_EVAL_NODES);
    HIPCHK(ctx, hipGetLastError());
    HIPCHK(ctx, t1(4));
    if (g.mixed) {
      HIPCHK(ctx, t0(5));
      hipLaunchKernelGGL(k_nodes32, dim3(gfor(5, ub_piece)), dim3(ctx->tune_block[5]), 0, st, L,
                         dev(CNT_JOB32), job.gl, job.ng);
      HIPCHK(ctx, hipGetLastError());
      HIPCHK(ctx, t1(5));
    }
    HIPCHK(ctx, t0(6));
    hipLaunchKernelGGL(k_combine, dim3(grid_for(ub_combo)), dim3(kBlk), 0, st, L, dev(CNT_COMBO));
    HIPCHK(ctx, hipGetLastError());
    const bool check = g.mixed && g.apex_w;
    hipLaunchKernelGGL(k_store, dim3(grid_for(nc)), dim3(kBlk), 0, st, g, L, c0, nc, job.out,
                       check ? 1 : 0, job.nseg, job.seg_off, job.seg_causal);
    HIPCHK(ctx, hipGetLastError());
    HIPCHK(ctx, t1(6));
    // the chunk's one wait: its list counts
    unsigned long long hc[CNT_N];
    HIPCHK(ctx, hipMemcpyAsync(hc, L.cnt, sizeof(hc), hipMemcpyDeviceToHost, st));
    HIPCHK(ctx, hipStreamSynchronize(st));
    {
      // a list overflowed: nothing was stored; redo with a smaller chunk
      // (a count after an overflowed list is a lower bound)
      double f = 1.0;
      if (hc[CNT_DEEP] > (unsigned long long)L.cap_combo) f = std::min(f, (double)L.cap_combo / hc[CNT_DEEP]);
      if (hc[CNT_COMBO] > (unsigned long long)L.cap_combo) f = std::min(f, (double)L.cap_combo / hc[CNT_COMBO]);
      if (hc[CNT_PIECE] > (unsigned long long)L.cap_piece) f = std::min(f, (double)L.cap_piece / hc[CNT_PIECE]);
      if (f < 1.0) {
        if (nc == 1) return stb_fail(ctx, STB_E_INTERNAL, "pair lists too small for one candidate");
        chunk = std::max<int64_t>(1, (int64_t)((double)nc * f * 0.8));
        continue;
      }
    }
    const unsigned long long ncombo = hc[CNT_COMBO], npiece = hc[CNT_PIECE];
    const unsigned long long njob = hc[CNT_JOB], njob1x = hc[CNT_JOB1X], njob2 = hc[CNT_JOB2];
    if (check) {
      // mixed: entries whose FP32 error bound is too large for their size
      // are recomputed with FP64 nodes
      unsigned long long nredo = hc[CNT_REDO], njr = 0;
      if (nredo) {
        // the FP64 job lists were consumed by the launches above (same stream)
        HIPCHK(ctx, hipMemsetAsync(L.cnt + CNT_JOB, 0, 4 * sizeof(unsigned long long), st));
        static_assert(CNT_JOB1X == CNT_JOB + 1 && CNT_JOB2 == CNT_JOB + 2 && CNT_JOBF == CNT_JOB + 3,
                      "job counters contiguous");
        hipLaunchKernelGGL(k_redo, dim3(grid_for(nc)), dim3(kBlk), 0, st, g, L, nc);
        HIPCHK(ctx, hipGetLastError());
        unsigned long long hr[CNT_N];
        HIPCHK(ctx, hipMemcpyAsync(hr, L.cnt, sizeof(hr), hipMemcpyDeviceToHost, st));
        HIPCHK(ctx, hipStreamSynchronize(st));
        const unsigned long long r1 = hr[CNT_JOB], r1x = hr[CNT_JOB1X], r2 = hr[CNT_JOB2], rf = hr[CNT_JOBF];
        njr = r1 + r1x + r2 + rf;
        if (njr) {
          HIPCHK(ctx, t0(7));
          if (r1)
            hipLaunchKernelGGL((k_nodes_rec<1, true>), dim3(gfor(4, r1)), dim3(ctx->tune_block[4]), 0, st, L,
                               L.job, (int64_t)r1, job.gl, job.ng, (int)CNT_EVAL_REDO);
          if (r1x)
            hipLaunchKernelGGL((k_nodes_rec<1, false>), dim3(gfor(4, r1x)), dim3(ctx->tune_block[4]), 0, st,
                               L, L.job + (L.cap_piece - (int64_t)r1x), (int64_t)r1x, job.gl, job.ng,
                               (int)CNT_EVAL_REDO);
          if (r2)
            hipLaunchKernelGGL((k_nodes_rec<2, false>), dim3(gfor(4, r2)), dim3(ctx->tune_block[4]), 0, st,
                               L, L.job2, (int64_t)r2, job.gl, job.ng, (int)CNT_EVAL_REDO);
          if (rf)
            hipLaunchKernelGGL(k_nodes, dim3(gfor(4, rf)), dim3(ctx->tune_block[4]), 0, st, L, L.jobf,
                               (int64_t)rf, job.gl, job.ng, (int)CNT_EVAL_REDO);
          HIPCHK(ctx, hipGetLastError());
          HIPCHK(ctx, t1(7));
        }
      }
      HIPCHK(ctx, t0(3));
      if (njr)
        hipLaunchKernelGGL(k_combine, dim3(grid_for(ncombo)), dim3(kBlk), 0, st, L, (int64_t)ncombo);
      hipLaunchKernelGGL(k_store, dim3(grid_for(nc)), dim3(kBlk), 0, st, g, L, c0, nc, job.out, 0,
                         job.nseg, job.seg_off, job.seg_causal);
      HIPCHK(ctx, hipGetLastError());
      HIPCHK(ctx, t1(3));
    }
    if (check) {
      HIPCHK(ctx, hipMemcpyAsync(h, L.cnt, sizeof(h), hipMemcpyDeviceToHost, st));
      HIPCHK(ctx, hipStreamSynchronize(st));
    } else {
      for (int k = 0; k < CNT_N; ++k) h[k] = hc[k];
    }
    for (int k = 0; k < 8; ++k) {
      if (!used[k]) continue;
      float ms = 0.0f;
      HIPCHK(ctx, hipEventElapsedTime(&ms, ctx->kev[2 * k], ctx->kev[2 * k + 1]));
      ctx->kern_ms[k] += ms;
      ctx->kern_n[k] += 1;
    }
    const unsigned long long evals = h[CNT_EVAL_MID] + h[CNT_EVAL_QUARTER] + h[CNT_EVAL_NODES] +
                                     h[CNT_EVAL_NODES32] + h[CNT_EVAL_REDO];
    ctx->kern_units[0] += (int64_t)h[CNT_PAIRS];
    ctx->kern_units[1] += (int64_t)ncombo;
    ctx->kern_units[2] += (int64_t)(h[CNT_EVAL_MID] + h[CNT_EVAL_QUARTER]);
    ctx->kern_units[4] += (int64_t)h[CNT_EVAL_NODES];
    ctx->path_counts[0] += (int64_t)(njob + njob1x) * job.ng;
    ctx->path_counts[1] += (int64_t)njob2 * job.ng;
    ctx->path_counts[2] += (int64_t)h[CNT_EVAL_NODES] - (int64_t)(njob + njob1x + njob2) * job.ng;
    ctx->path_counts[3] += (int64_t)h[CNT_MISS];
    ctx->kern_units[5] += (int64_t)h[CNT_EVAL_NODES32];
    ctx->kern_units[7] += (int64_t)h[CNT_EVAL_REDO];
    ctx->kern_units[3] += (int64_t)h[CNT_REDO];
    ctx->kern_units[6] += (int64_t)nc;
    work[0] += evals;
    work[1] += h[CNT_COMBO];
    work[2] += h[CNT_PAIRS];
    work[3] += h[CNT_PIECE];
    if (job.n_causal) *job.n_causal += h[CNT_CAUSAL];
    c0 += nc;
    // next chunk: as large as the lists allow at this chunk's densities
    double fc = (double)L.cap_combo / std::max<unsigned long long>(ncombo, 1);
    double fp = (double)L.cap_piece / std::max<unsigned long long>(npiece, 1);
    int64_t next = (int64_t)((double)nc * std::min(fc, fp) * 0.7);
    chunk = std::max<int64_t>(1, std::min<int64_t>(next, L.cap_cand));
  }
  return STB_OK;
}

extern "C" stb_status stb_set_pair_lists(stb_ctx* ctx, int64_t max_cand, int64_t max_combo,
                                         int64_t max_piece) {
  if (!ctx) return stb_fail(nullptr, STB_E_INVALID_ARG, "NULL context");
  const int64_t v[3] = {max_cand, max_combo, max_piece};
  for (int k = 0; k < 3; ++k)
    if (v[k] < 0 || (v[k] > 0 && v[k] < 64))
      return stb_fail(ctx, STB_E_INVALID_ARG, "list limit %d = %lld: 0 or at least 64", k, (long long)v[k]);
  for (int k = 0; k < 3; ++k) ctx->list_limit[k] = v[k];
  return STB_OK;
}

// Launch-shape autotuner.  The flat lists make every stage a loop over
// items of one cost class (apexes to test, lit combos, pieces, Gauss jobs),
// so what is left to tune per stage is the launch shape: threads per block
// (64, 128, 256) and resident blocks per CU (4, 8, 16, 32), which trade
// latency hiding against tail effects and L2 locality of neighbouring
// items.  Each stage is timed on the sample (HIP events) for every shape
// with the other stages at their current choice, in order of their share of
// the time (the better of two runs per shape); a shape replaces the stage's
// current one only when it is faster by more than 5% (the sample's timing
// noise and its difference from the full assembly are about that size).
stb_status stb_tune_pairs(stb_ctx* ctx, const PairJob& sample) {
  static const int kStages[] = {4, 5, 2, 1, 0};
  static const int kBlocks[] = {64, 128, 256};
  static const int kPerCu[] = {4, 8, 16, 32};
  unsigned long long work[4];
  stb_status s = stb_run_pairs(ctx, sample, work);   // warm-up, lists sized
  if (s) return s;
  for (int stage : kStages) {
    if (ctx->kern_n[stage] == 0) continue;   // stage unused on this sample
    int bb = ctx->tune_block[stage], bp = ctx->tune_per_cu[stage];
    // the stage's time at the current shapes: the better of two runs
    auto timed = [&](double* ms) -> stb_status {
      double t = 1e300;
      for (int r = 0; r < 2; ++r) {
        stb_status e = stb_run_pairs(ctx, sample, work);
        if (e) return e;
        t = std::min(t, ctx->kern_ms[stage]);
      }
      *ms = t;
      return STB_OK;
    };
    double best = 0.0;   // the current shape
    if ((s = timed(&best))) return s;
    for (int b : kBlocks)
      for (int pc : kPerCu) {
        ctx->tune_block[stage] = b;
        ctx->tune_per_cu[stage] = pc;
        double t = 0.0;
        if ((s = timed(&t))) return s;
        if (t < 0.95 * best) {
          best = t;
          bb = b;
          bp = pc;
        }
      }
    ctx->tune_block[stage] = bb;
    ctx->tune_per_cu[stage] = bp;
  }
  ctx->tuned = true;
  return STB_OK;
}
