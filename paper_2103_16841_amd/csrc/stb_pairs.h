// stb_pairs.h -- the pair pipeline (stb_pairs.hip) as seen by the library.
#pragma once
#include "stb_internal.h"

// One pipeline run over a candidate set (device arrays, context stream).
struct PairJob {
  int64_t nnz = 0;                   // candidates
  const int32_t* rows = nullptr;     // [nnz] row of each candidate
  const int32_t* cols = nullptr;     // [nnz] trial panel of each candidate
  const stb::TrialRec* trial = nullptr;
  const stb::FaceAng* fang = nullptr;  // [panels]
  const double* apex = nullptr;      // [rows][maxq][4] (t, x, y, z)
  const double* apex_w = nullptr;    // [rows][maxq] outer weights; nullptr: potential
  const int32_t* apex_n = nullptr;   // [rows] apexes per row; nullptr: one
  int maxq = 1;
  const double* gl = nullptr;        // [4 kMaxNg]: Gauss nodes on [0,1], weights, 1/2 - s(x), s'(x) w
  int ng = 0;
  bool mixed = false;                // far combos' Gauss nodes in FP32
  double eta_far = 2.0;              // far: apex farther than eta_far radii from the panel's ball
  double* out = nullptr;             // [nnz] matrix entry or inner integral
  uint8_t* lit_out = nullptr;        // optional [nnz]: 1 where some apex is lit
  unsigned long long* n_causal = nullptr;   // host: += candidates with a lit apex
  // optional segments of the candidate range (batches of meshes): candidate
  // offsets [nseg + 1] and per-segment causal counts [nseg], both device
  int nseg = 0;
  const int64_t* seg_off = nullptr;
  unsigned long long* seg_causal = nullptr;
};

// Runs the pipeline; work[0..3] receive L evaluations, lit combos, apexes
// tested and pieces.  Synchronises the context stream.
stb_status stb_run_pairs(stb_ctx* ctx, const PairJob& job, unsigned long long work[4]);
void stb_free_workspace(stb_ctx* ctx);
// Device bytes of ctx's pipeline workspace now, and after a run over nnz
// candidates with maxq apexes each (the workspace only grows).
int64_t stb_pairs_ws_held(const stb_ctx* ctx);
int64_t stb_pairs_ws_need(const stb_ctx* ctx, int64_t nnz, int maxq);
// Chooses the launch shape of every stage on a sample job (see stb_pairs.hip).
stb_status stb_tune_pairs(stb_ctx* ctx, const PairJob& sample);
