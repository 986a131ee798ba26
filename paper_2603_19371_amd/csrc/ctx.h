// The context of one registration pair (shared by api.cpp and api_batch.cpp).
#pragma once

#include <hip/hip_runtime.h>

#include <vector>

#include "lmr_internal.h"

// Event pairs recorded around the kernels of sampled attempts.
struct Profiler {
  bool on = false;
  int stride = 1;
  int max_attempts = 0;
  int recorded = 0;   // attempts recorded
  long long seen = 0; // attempts enqueued while on
  std::vector<hipEvent_t> ev;  // LMR_NUM_KERNELS + 1 per recorded attempt
};

struct lmr_ctx {
  Profiler prof;
  lmr::Geom g;
  lmr_dtype img;
  lmr_params p;
  lmr::DecideParams dp;
  hipStream_t stream;
  void* arena;
  float* U[2];
  float* G;
  float* graw;
  float* maps;
  float* Mw;
  double* fstat;  // window mean and variance of the fixed image [2][N]
  const void* fstat_of;  // the fixed image fstat was computed from
  double* partials;
  int nparts;
  lmr::DevState* st;
  lmr::DevState* st_next;  // the state a backward pass decided, until P5 stores it in st
  double* probe;
  lmr::DevState* st_probe;
  double* part_probe;
  unsigned long long* counter;
  bool begun;
  size_t arena_bytes;  // the whole workspace (lmr_workspace_bytes)
  int forced = -1;     // lmr_force_decision: the decision of later lmr_step attempts
  // tile_size > 1 (eq. tilen): mean g g^T per tile [tiles][6]
  double* H;
  int tiles[3];  // tiles along x, y, z
  // Adam comparator: first and second moments [3][N] each
  float* am;
  float* av;
  // mutual information: partial histograms, p, gradient table, bin maps
  unsigned long long* mi_hpart;
  double* mi_p;
  double* mi_tab;
  double* mi_map;
  float* mi_rpart;
  const void* mi_of[2];  // the images the bin maps were taken from
  lmr::StepExtra extra() const;
};

namespace lmr {
// Records the text of a failing HIP call for lmr_last_error and returns LMR_EHIP.
lmr_status hip_fail(hipError_t e);
bool params_ok(const lmr_params* p);
}  // namespace lmr

#define LMR_HIP(expr)                                \
  do {                                               \
    hipError_t e_ = (expr);                          \
    if (e_ != hipSuccess) return lmr::hip_fail(e_);  \
  } while (0)
