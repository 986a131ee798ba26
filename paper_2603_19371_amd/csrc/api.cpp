// C-ABI of liblmreg: contexts, workspace and the step sequence of one LM
// attempt (include/lmreg.h documents every entry point).
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <map>
#include <new>
#include <tuple>
#include <vector>

#include "ctx.h"
#include "pass_decision.h"
#include "pyramid.h"
#include "lmr_internal.h"

using namespace lmr;

namespace {

thread_local char g_err[256] = "";

}  // namespace

lmr_status lmr::hip_fail(hipError_t e) {
  snprintf(g_err, sizeof g_err, "%s", hipGetErrorString(e));
  return LMR_EHIP;
}

bool lmr::params_ok(const lmr_params* p) {
  if (!p) return false;
  if (p->window < 3 || p->window > 9 || (p->window % 2) == 0) return false;
  if (!(p->grad_sigma >= 0.0 && p->grad_sigma <= 2.0)) return false;
  if (!(p->cc_eps >= 0.0)) return false;
  if (!(p->step_eps > 0.0)) return false;
  if (p->accum != LMR_ACC_F64 && p->accum != LMR_ACC_F32C) return false;
  if (!(p->lambda_inc > 1.0) || !(p->lambda_dec > 0.0 && p->lambda_dec < 1.0)) return false;
  if (!(p->lambda_min > 0.0) || !(p->lambda_max >= p->lambda_min)) return false;
  if (p->max_retries < 1) return false;
  if (p->tile < 1 || p->tile > 16) return false;
  if (p->optimizer != LMR_OPT_LM && p->optimizer != LMR_OPT_ADAM) return false;
  if (p->similarity != LMR_SIM_LNCC && p->similarity != LMR_SIM_MSE &&
      p->similarity != LMR_SIM_DEMONS && p->similarity != LMR_SIM_MI)
    return false;
  if (p->similarity == LMR_SIM_MI && (p->mi_bins < 8 || p->mi_bins > 32)) return false;
  if (p->stencil != LMR_STENCIL_AUTO && p->stencil != LMR_STENCIL_MARCH &&
      p->stencil != LMR_STENCIL_CUBE)
    return false;
  if (p->similarity == LMR_SIM_DEMONS && (p->optimizer != LMR_OPT_LM || p->tile != 1))
    return false;
  if (p->optimizer == LMR_OPT_ADAM) {
    if (p->tile != 1 || !(p->adam_lr > 0.0) || !(p->adam_eps > 0.0)) return false;
    if (!(p->adam_beta1 >= 0.0 && p->adam_beta1 < 1.0)) return false;
    if (!(p->adam_beta2 >= 0.0 && p->adam_beta2 < 1.0)) return false;
  }
  return true;
}

lmr::StepExtra lmr_ctx::extra() const {
  lmr::StepExtra x{};
  if (p.similarity == LMR_SIM_DEMONS) {
    x.mode = 3;
  } else if (p.optimizer == LMR_OPT_ADAM) {
    x.mode = 2;
    x.m = am;
    x.v = av;
    x.b1 = static_cast<float>(p.adam_beta1);
    x.ob1 = static_cast<float>(1.0 - p.adam_beta1);
    x.b2 = static_cast<float>(p.adam_beta2);
    x.ob2 = static_cast<float>(1.0 - p.adam_beta2);
    x.lr = static_cast<float>(p.adam_lr);
    x.aeps = static_cast<float>(p.adam_eps);
  } else if (p.tile > 1) {
    x.mode = 1;
    x.H = H;
    x.k = p.tile;
    x.tx = tiles[0];
    x.ty = tiles[1];
  }
  return x;
}

namespace {

size_t align256(size_t n) { return (n + 255) & ~size_t(255); }

// One attempt: P1 update, P2 forward, P3 decide, P4 backward, P5 smooth.
// Squared error: P2 is the squared-error reduction and P4 its gradient.
// Demons: the step field is formed and smoothed before P1 (timed with P1),
// and P4 keeps the residuals of an accepted field (no P5).
lmr_status enqueue_attempt(lmr_ctx* c, const void* F, const void* M, int force) {
  hipStream_t s = c->stream;
  Profiler& pr = c->prof;
  hipEvent_t* ev = nullptr;
  if (pr.on) {
    if (pr.seen % pr.stride == 0 && pr.recorded < pr.max_attempts)
      ev = &pr.ev[(LMR_NUM_KERNELS + 1) * pr.recorded++];
    ++pr.seen;
  }
  // one event before the first kernel and one after each kernel: kernel k
  // runs between events k and k + 1 (each event costs a few microseconds of
  // stream time, so a kernel's start is the previous kernel's end)
  auto mark = [&](int k, int end) -> hipError_t {
    if (!ev || (!end && k > 0)) return hipSuccess;
    return hipEventRecord(ev[end ? k + 1 : 0], s);
  };
  const int sim = c->p.similarity;
  // the Adam comparator keeps every step
  if (c->p.optimizer == LMR_OPT_ADAM) force = 1;
  const StepExtra ex = c->extra();
  LMR_HIP(mark(LMR_K_UPDATE, 0));
  if (sim == LMR_SIM_DEMONS) {
    // du from the kept residuals of the accepted field, smoothed into G
    LMR_HIP(launch_demons_force(c->maps, c->g, c->st, c->graw, s));
    LMR_HIP(launch_smooth(c->graw, c->g, c->p, nullptr, c->G, s));
  }
  // the derivative of the candidate's warped image goes to graw, where P4
  // reads it (voxel by voxel, before overwriting it with the raw gradient)
  LMR_HIP(launch_update(M, c->img, c->g, c->p, c->st, c->G, c->U[0], c->U[1], nullptr,
                        nullptr, 0.0, 0.0, c->Mw, c->graw, s, &ex));
  LMR_HIP(mark(LMR_K_UPDATE, 1));
  LMR_HIP(mark(LMR_K_FWD, 0));
  if (sim == LMR_SIM_LNCC)
    LMR_HIP(launch_fwd(F, c->img, c->Mw, c->fstat, c->g, c->p, c->st, c->maps, c->partials,
                       c->nparts, nullptr, s));
  else if (sim == LMR_SIM_MI)
    LMR_HIP(launch_mi_fwd(F, c->img, c->Mw, c->g, c->p.mi_bins, c->mi_map, c->mi_hpart,
                          c->mi_p, c->mi_tab, c->partials, c->st, s));
  else
    LMR_HIP(launch_mse_fwd(F, c->img, c->Mw, c->g, c->nparts, c->partials, nullptr, c->st, s));
  LMR_HIP(mark(LMR_K_FWD, 1));
  // levels with few partials take the decision in the backward pass, which
  // stages the decided state; the smoothing pass makes it the pair state
  const bool dec_in_bwd = sim == LMR_SIM_LNCC && bwd_takes_decision(c->g, c->p, c->nparts);
  LMR_HIP(mark(LMR_K_DECIDE, 0));
  if (!dec_in_bwd)
    LMR_HIP(launch_decide(c->st, c->partials, sim == LMR_SIM_MI ? 1 : c->nparts, c->g.N,
                          c->dp, 0, force, 0.0, nullptr, s));
  LMR_HIP(mark(LMR_K_DECIDE, 1));
  LMR_HIP(mark(LMR_K_BWD, 0));
  if (dec_in_bwd) {
    PassDecision pd{};
    pd.partials = c->partials;
    pd.nparts = c->nparts;
    pd.N = c->g.N;
    pd.dp = c->dp;
    pd.force = force;
    pd.next = c->st_next;
    LMR_HIP(launch_bwd_decide(F, M, c->img, c->Mw, c->maps, c->g, c->p, c->st, c->U[0],
                              c->U[1], c->graw, c->graw, pd, s));
  } else if (sim == LMR_SIM_LNCC)
    LMR_HIP(launch_bwd(F, M, c->img, c->Mw, c->maps, c->g, c->p, c->st, c->U[0], c->U[1],
                       nullptr, c->graw, c->graw, s));
  else if (sim == LMR_SIM_MSE)
    LMR_HIP(launch_mse_bwd(F, c->img, c->Mw, c->graw, c->g, c->st, nullptr, c->graw, s));
  else if (sim == LMR_SIM_MI)
    LMR_HIP(launch_mi_bwd(F, c->img, c->Mw, c->graw, c->g, c->p.mi_bins, c->mi_map, c->mi_tab,
                          c->st, c->graw, s));
  else
    LMR_HIP(launch_demons_keep(F, c->img, c->Mw, c->graw, c->g, c->st, c->maps, s));
  LMR_HIP(mark(LMR_K_BWD, 1));
  LMR_HIP(mark(LMR_K_SMOOTH, 0));
  if (dec_in_bwd) {
    LMR_HIP(launch_smooth_commit(c->graw, c->g, c->p, c->st_next, c->st, c->G, s));
    if (ex.mode == 1) LMR_HIP(launch_tile_hessian(c->G, c->g, c->p.tile, c->H, c->st, 2, s));
  } else if (sim != LMR_SIM_DEMONS) {
    LMR_HIP(launch_smooth(c->graw, c->g, c->p, c->st, c->G, s));
    // eq. tilen: the pooled matrices of the new gradient (timed with P5)
    if (ex.mode == 1) LMR_HIP(launch_tile_hessian(c->G, c->g, c->p.tile, c->H, c->st, 2, s));
  }
  LMR_HIP(mark(LMR_K_SMOOTH, 1));
  return LMR_OK;
}

void profile_release(Profiler& pr) {
  for (hipEvent_t e : pr.ev) (void)hipEventDestroy(e);
  pr.ev.clear();
  pr.on = false;
}

}  // namespace

extern "C" {

const char* lmr_strerror(lmr_status s) {
  switch (s) {
    case LMR_OK: return "ok";
    case LMR_EINVAL: return "invalid argument";
    case LMR_ENOMEM: return "out of device memory";
    case LMR_EHIP: return "HIP runtime error";
    case LMR_ESTATE: return "call out of order";
    case LMR_ESTALLED: return "pair is frozen";
    case LMR_EBUSY: return "batched launch not co-resident (GPU held by other work)";
  }
  return "unknown status";
}

const char* lmr_last_error(void) { return g_err; }

void lmr_default_params(lmr_params* p) {
  if (!p) return;
  p->window = 5;
  p->grad_sigma = 1.0;
  p->cc_eps = 1e-5;
  p->step_eps = 1.0;
  p->compositive = 1;
  p->accum = LMR_ACC_F64;
  p->lambda_inc = 2.0;
  p->lambda_dec = 0.5;
  p->lambda_min = 1e-12;
  p->lambda_max = 1e6;
  p->tau = 0.0;
  p->max_retries = 10;
  p->tile = 1;
  p->optimizer = LMR_OPT_LM;
  p->adam_lr = 0.1;
  p->adam_beta1 = 0.9;
  p->adam_beta2 = 0.999;
  p->adam_eps = 1e-8;
  p->similarity = LMR_SIM_LNCC;
  p->mi_bins = 32;
  p->stencil = LMR_STENCIL_AUTO;
}

lmr_status lmr_create(lmr_ctx** out, int nz, int ny, int nx, lmr_dtype img,
                      const lmr_params* p, hipStream_t stream) {
  if (!out) return LMR_EINVAL;
  *out = nullptr;
  if (nz < 1 || ny < 1 || nx < 1 || nz > 65535) return LMR_EINVAL;
  long long N = (long long)nz * ny * nx;
  if (N >= (1LL << 30)) return LMR_EINVAL;
  if (img != LMR_F32 && img != LMR_BF16) return LMR_EINVAL;
  if (!params_ok(p)) return LMR_EINVAL;

  lmr_ctx* c = new (std::nothrow) lmr_ctx();
  if (!c) return LMR_ENOMEM;
  c->g = Geom{nz, ny, nx, N};
  c->img = img;
  c->p = *p;
  c->dp = DecideParams{p->lambda_inc, p->lambda_dec,     p->lambda_min,
                       p->lambda_max, p->tau,            p->max_retries,
                       p->adam_beta1, p->adam_beta2,     p->similarity,
                       p->mi_bins};
  c->stream = stream;
  c->nparts = fwd_num_blocks(c->g, *p);

  const size_t f3 = align256(sizeof(float) * 3 * N);
  const size_t sizes[] = {f3,
                          f3,
                          f3,
                          f3,
                          align256(sizeof(float) * 4 * N),
                          align256(sizeof(float) * N),
                          align256(sizeof(double) * c->nparts),
                          align256(2 * sizeof(DevState)),  // the pair state and its staging slot
                          align256(sizeof(double)),
                          align256(sizeof(DevState)),
                          align256(sizeof(double)),
                          align256(sizeof(unsigned long long)),
                          align256(sizeof(double) * 2 * N)};
  const int k = p->tile;
  c->tiles[0] = (nx + k - 1) / k;
  c->tiles[1] = (ny + k - 1) / k;
  c->tiles[2] = (nz + k - 1) / k;
  const size_t h_bytes =
      k > 1 ? align256(sizeof(double) * 6 * (size_t)c->tiles[0] * c->tiles[1] * c->tiles[2])
            : 0;
  const size_t mv_bytes = p->optimizer == LMR_OPT_ADAM ? f3 : 0;
  const bool mi = p->similarity == LMR_SIM_MI;
  const size_t bb = mi ? static_cast<size_t>(p->mi_bins) * p->mi_bins : 0;
  const size_t mi_sizes[5] = {align256(8 * bb * kMiBlocks), align256(8 * bb), align256(8 * bb),
                              mi ? align256(32) : 0, mi ? align256(16 * kMiBlocks) : 0};
  size_t mi_bytes = 0;
  for (size_t v : mi_sizes) mi_bytes += v;
  size_t total = h_bytes + 2 * mv_bytes + mi_bytes;
  for (size_t s : sizes) total += s;
  c->arena_bytes = total;
  hipError_t e = hipMalloc(&c->arena, total);
  if (e != hipSuccess) {
    snprintf(g_err, sizeof g_err, "%s", hipGetErrorString(e));
    delete c;
    return LMR_ENOMEM;
  }
  char* q = static_cast<char*>(c->arena);
  c->U[0] = reinterpret_cast<float*>(q); q += sizes[0];
  c->U[1] = reinterpret_cast<float*>(q); q += sizes[1];
  c->G = reinterpret_cast<float*>(q); q += sizes[2];
  c->graw = reinterpret_cast<float*>(q); q += sizes[3];
  c->maps = reinterpret_cast<float*>(q); q += sizes[4];
  c->Mw = reinterpret_cast<float*>(q); q += sizes[5];
  c->partials = reinterpret_cast<double*>(q); q += sizes[6];
  c->st = reinterpret_cast<DevState*>(q); q += sizes[7];
  c->st_next = c->st + 1;
  c->probe = reinterpret_cast<double*>(q); q += sizes[8];
  c->st_probe = reinterpret_cast<DevState*>(q); q += sizes[9];
  c->part_probe = reinterpret_cast<double*>(q); q += sizes[10];
  c->counter = reinterpret_cast<unsigned long long*>(q);
  q += sizes[11];
  c->fstat = reinterpret_cast<double*>(q);
  q += sizes[12];
  c->H = h_bytes ? reinterpret_cast<double*>(q) : nullptr;
  q += h_bytes;
  c->am = mv_bytes ? reinterpret_cast<float*>(q) : nullptr;
  c->av = mv_bytes ? reinterpret_cast<float*>(q + mv_bytes) : nullptr;
  q += 2 * mv_bytes;
  c->mi_hpart = mi ? reinterpret_cast<unsigned long long*>(q) : nullptr;
  q += mi_sizes[0];
  c->mi_p = mi ? reinterpret_cast<double*>(q) : nullptr;
  q += mi_sizes[1];
  c->mi_tab = mi ? reinterpret_cast<double*>(q) : nullptr;
  q += mi_sizes[2];
  c->mi_map = mi ? reinterpret_cast<double*>(q) : nullptr;
  q += mi_sizes[3];
  c->mi_rpart = mi ? reinterpret_cast<float*>(q) : nullptr;
  c->mi_of[0] = c->mi_of[1] = nullptr;
  c->begun = false;
  *out = c;
  return LMR_OK;
}

void lmr_destroy(lmr_ctx* c) {
  if (!c) return;
  (void)hipStreamSynchronize(c->stream);
  profile_release(c->prof);
  (void)hipFree(c->arena);
  delete c;
}

lmr_status lmr_begin(lmr_ctx* c, const void* F, const void* M, const float* field,
                     double lambda0) {
  if (!c || !F || !M || !(lambda0 > 0.0)) return LMR_EINVAL;
  hipStream_t s = c->stream;
  const size_t bytes = sizeof(float) * 3 * c->g.N;
  if (!field)
    LMR_HIP(launch_fill(c->U[0], 3 * c->g.N, 0.0f, s));
  else if (field != c->U[0])  // a field already in place is kept as it is
    LMR_HIP(hipMemcpyAsync(c->U[0], field, bytes, hipMemcpyDeviceToDevice, s));
  const int sim = c->p.similarity;
  if (sim == LMR_SIM_LNCC) {
    LMR_HIP(launch_fstat(F, c->img, c->g, c->p, c->fstat, s));
    c->fstat_of = F;
    LMR_HIP(launch_warp(M, c->img, c->U[0], c->g, c->Mw, nullptr, s));
    LMR_HIP(launch_fwd(F, c->img, c->Mw, c->fstat, c->g, c->p, nullptr, c->maps,
                       c->partials, c->nparts, nullptr, s));
  } else if (sim == LMR_SIM_MI) {
    LMR_HIP(launch_mi_range(F, M, c->img, c->g, c->p.mi_bins, c->mi_rpart, c->mi_map, s));
    c->mi_of[0] = F;
    c->mi_of[1] = M;
    LMR_HIP(launch_warp(M, c->img, c->U[0], c->g, c->Mw, c->graw, s));
    LMR_HIP(launch_mi_fwd(F, c->img, c->Mw, c->g, c->p.mi_bins, c->mi_map, c->mi_hpart,
                          c->mi_p, c->mi_tab, c->partials, nullptr, s));
  } else {
    LMR_HIP(launch_warp(M, c->img, c->U[0], c->g, c->Mw, c->graw, s));
    LMR_HIP(launch_mse_fwd(F, c->img, c->Mw, c->g, c->nparts, c->partials, nullptr, nullptr,
                           s));
  }
  LMR_HIP(launch_decide(c->st, c->partials, sim == LMR_SIM_MI ? 1 : c->nparts, c->g.N, c->dp,
                        1, -1, lambda0, nullptr, s));
  if (sim == LMR_SIM_LNCC) {
    LMR_HIP(launch_bwd(F, M, c->img, c->Mw, c->maps, c->g, c->p, nullptr, nullptr,
                       nullptr, c->U[0], nullptr, c->graw, s));
    LMR_HIP(launch_smooth(c->graw, c->g, c->p, nullptr, c->G, s));
  } else if (sim == LMR_SIM_MSE) {
    // the state holds r = sqrt(L) of the starting field
    LMR_HIP(launch_mse_bwd(F, c->img, c->Mw, c->graw, c->g, c->st, nullptr, c->graw, s));
    LMR_HIP(launch_smooth(c->graw, c->g, c->p, nullptr, c->G, s));
  } else if (sim == LMR_SIM_MI) {
    LMR_HIP(launch_mi_bwd(F, c->img, c->Mw, c->graw, c->g, c->p.mi_bins, c->mi_map, c->mi_tab,
                          c->st, c->graw, s));
    LMR_HIP(launch_smooth(c->graw, c->g, c->p, nullptr, c->G, s));
  } else {
    LMR_HIP(launch_demons_keep(F, c->img, c->Mw, c->graw, c->g, nullptr, c->maps, s));
  }
  if (c->H) LMR_HIP(launch_tile_hessian(c->G, c->g, c->p.tile, c->H, nullptr, 0, s));
  if (c->am) {
    LMR_HIP(launch_fill(c->am, 3 * c->g.N, 0.0f, s));
    LMR_HIP(launch_fill(c->av, 3 * c->g.N, 0.0f, s));
  }
  c->begun = true;
  return LMR_OK;
}

// The statistics of F are kept from lmr_begin; a step given another fixed
// image buffer recomputes them first (an image rewritten in place is the
// caller's to avoid, as documented).
static lmr_status refresh_fstat(lmr_ctx* c, const void* F, const void* M) {
  if (c->p.similarity == LMR_SIM_MI && (F != c->mi_of[0] || M != c->mi_of[1])) {
    LMR_HIP(launch_mi_range(F, M, c->img, c->g, c->p.mi_bins, c->mi_rpart, c->mi_map,
                            c->stream));
    c->mi_of[0] = F;
    c->mi_of[1] = M;
    return LMR_OK;
  }
  if (F == c->fstat_of || c->p.similarity != LMR_SIM_LNCC) return LMR_OK;
  LMR_HIP(launch_fstat(F, c->img, c->g, c->p, c->fstat, c->stream));
  c->fstat_of = F;
  return LMR_OK;
}

lmr_status lmr_step(lmr_ctx* c, const void* F, const void* M, int n) {
  if (!c || !F || !M || n < 0) return LMR_EINVAL;
  if (!c->begun) return LMR_ESTATE;
  if (n > 0) {
    const lmr_status r = refresh_fstat(c, F, M);
    if (r != LMR_OK) return r;
  }
  for (int i = 0; i < n; ++i) {
    lmr_status r = enqueue_attempt(c, F, M, c->forced);
    if (r != LMR_OK) return r;
  }
  return LMR_OK;
}

lmr_status lmr_force_decision(lmr_ctx* c, int decision) {
  if (!c || decision < -1 || decision > 1) return LMR_EINVAL;
  if (decision == 0 && c->p.optimizer == LMR_OPT_ADAM) return LMR_EINVAL;
  c->forced = decision;
  return LMR_OK;
}

lmr_status lmr_step_forced(lmr_ctx* c, const void* F, const void* M,
                           const int* decisions, int n) {
  if (!c || !F || !M || n < 0 || (n > 0 && !decisions)) return LMR_EINVAL;
  if (c->p.optimizer == LMR_OPT_ADAM)
    for (int i = 0; i < n; ++i)
      if (decisions[i] == 0) return LMR_EINVAL;
  if (!c->begun) return LMR_ESTATE;
  if (n > 0) {
    const lmr_status r = refresh_fstat(c, F, M);
    if (r != LMR_OK) return r;
  }
  for (int i = 0; i < n; ++i) {
    int d = decisions[i] < 0 ? -1 : (decisions[i] ? 1 : 0);
    lmr_status r = enqueue_attempt(c, F, M, d);
    if (r != LMR_OK) return r;
  }
  return LMR_OK;
}

lmr_status lmr_workspace_bytes(const lmr_ctx* c, size_t* out) {
  if (!c || !out) return LMR_EINVAL;
  *out = c->arena_bytes;
  return LMR_OK;
}

lmr_status lmr_get_field(lmr_ctx* c, float* out) {
  if (!c || !out) return LMR_EINVAL;
  if (!c->begun) return LMR_ESTATE;
  LMR_HIP(launch_copy_cur(c->st, c->U[0], c->U[1], out, 3 * c->g.N, c->stream));
  return LMR_OK;
}

lmr_status lmr_get_grad(lmr_ctx* c, float* out) {
  if (!c || !out) return LMR_EINVAL;
  if (!c->begun) return LMR_ESTATE;
  LMR_HIP(hipMemcpyAsync(out, c->G, sizeof(float) * 3 * c->g.N,
                         hipMemcpyDeviceToDevice, c->stream));
  return LMR_OK;
}

lmr_status lmr_get_state(lmr_ctx* c, lmr_pair_state* out) {
  if (!c || !out) return LMR_EINVAL;
  if (!c->begun) return LMR_ESTATE;
  DevState h;
  LMR_HIP(hipMemcpyAsync(&h, c->st, sizeof h, hipMemcpyDeviceToHost, c->stream));
  LMR_HIP(hipStreamSynchronize(c->stream));
  out->lambda = h.lambda;
  out->loss = h.loss;
  out->loss_prev = h.loss_prev;
  out->cand_loss = h.cand_loss;
  out->n_hist = h.n_hist;
  out->retries = h.retries;
  out->accepted = h.accepted;
  out->stalled = h.stalled;
  out->attempts = h.attempts;
  return LMR_OK;
}

lmr_status lmr_set_state(lmr_ctx* c, const lmr_pair_state* in) {
  if (!c || !in || c->p.optimizer == LMR_OPT_ADAM) return LMR_EINVAL;
  if (!c->begun) return LMR_ESTATE;
  if (!(in->lambda > 0.0) || in->n_hist < 1 || in->retries < 0) return LMR_EINVAL;
  DevState v{};
  v.lambda = in->lambda;
  v.loss = in->loss;
  v.loss_prev = in->loss_prev;
  v.cand_loss = in->cand_loss;
  v.r = residual_of(in->loss, c->p.similarity, c->p.mi_bins);
  v.n_hist = in->n_hist;
  v.retries = in->retries;
  v.accepted = in->accepted;
  v.stalled = in->stalled;
  v.attempts = in->attempts;
  LMR_HIP(launch_set_state(c->st, v, c->stream));
  return LMR_OK;
}

lmr_status lmr_loss_grad(lmr_ctx* c, const void* F, const void* M, const float* u,
                         double* loss_out, float* g_raw, float* g_smooth,
                         float* cc_map) {
  if (!c || !F || !M || !u) return LMR_EINVAL;
  hipStream_t s = c->stream;
  if (c->p.similarity == LMR_SIM_LNCC) {
    // a stage call may pass any fixed image: its statistics are taken here
    LMR_HIP(launch_fstat(F, c->img, c->g, c->p, c->fstat, s));
    c->fstat_of = F;
    LMR_HIP(launch_warp(M, c->img, u, c->g, c->Mw, nullptr, s));
    LMR_HIP(launch_fwd(F, c->img, c->Mw, c->fstat, c->g, c->p, nullptr, c->maps,
                       c->partials, c->nparts, cc_map, s));
  } else if (c->p.similarity == LMR_SIM_MI) {
    if (cc_map) return LMR_EINVAL;
    LMR_HIP(launch_mi_range(F, M, c->img, c->g, c->p.mi_bins, c->mi_rpart, c->mi_map, s));
    c->mi_of[0] = F;
    c->mi_of[1] = M;
    LMR_HIP(launch_warp(M, c->img, u, c->g, c->Mw, c->graw, s));
    LMR_HIP(launch_mi_fwd(F, c->img, c->Mw, c->g, c->p.mi_bins, c->mi_map, c->mi_hpart,
                          c->mi_p, c->mi_tab, c->partials, nullptr, s));
  } else {
    // squared error (cc_map receives the squared errors)
    LMR_HIP(launch_warp(M, c->img, u, c->g, c->Mw, c->graw, s));
    LMR_HIP(launch_mse_fwd(F, c->img, c->Mw, c->g, c->nparts, c->partials, cc_map, nullptr,
                           s));
  }
  LMR_HIP(launch_decide(c->st, c->partials,
                        c->p.similarity == LMR_SIM_MI ? 1 : c->nparts, c->g.N, c->dp, 2, -1,
                        0.0, c->probe, s));
  if (g_raw || g_smooth) {
    float* gr = g_raw ? g_raw : c->graw;
    if (c->p.similarity == LMR_SIM_LNCC)
      LMR_HIP(launch_bwd(F, M, c->img, c->Mw, c->maps, c->g, c->p, nullptr, nullptr,
                         nullptr, u, nullptr, gr, s));
    else if (c->p.similarity == LMR_SIM_MI)
      LMR_HIP(launch_mi_bwd(F, c->img, c->Mw, c->graw, c->g, c->p.mi_bins, c->mi_map,
                            c->mi_tab, nullptr, gr, s));
    else
      LMR_HIP(launch_mse_bwd(F, c->img, c->Mw, c->graw, c->g, nullptr, c->probe, gr, s));
    if (g_smooth) LMR_HIP(launch_smooth(gr, c->g, c->p, nullptr, g_smooth, s));
  }
  double L = 0.0;
  LMR_HIP(hipMemcpyAsync(&L, c->probe, sizeof L, hipMemcpyDeviceToHost, s));
  LMR_HIP(hipStreamSynchronize(s));
  if (loss_out) *loss_out = L;
  return LMR_OK;
}

lmr_status lmr_update(lmr_ctx* c, const float* u, const float* g_smooth, double r,
                      double lambda, float* u_out) {
  if (!c || !u || !g_smooth || !u_out || u == u_out) return LMR_EINVAL;
  if (c->p.optimizer == LMR_OPT_ADAM || c->p.similarity == LMR_SIM_DEMONS) return LMR_EINVAL;
  StepExtra ex = c->extra();
  if (ex.mode == 1) {
    LMR_HIP(launch_tile_hessian(g_smooth, c->g, c->p.tile, c->H, nullptr, 0, c->stream));
    ex.H = c->H;
  }
  LMR_HIP(launch_update(nullptr, LMR_F32, c->g, c->p, nullptr, g_smooth, nullptr,
                        nullptr, u, u_out, r, lambda, c->Mw, nullptr, c->stream, &ex));
  return LMR_OK;
}

lmr_status lmr_folded_count(lmr_ctx* c, const float* u, long long* count_out,
                            float* det_out) {
  if (!c || !count_out) return LMR_EINVAL;
  if (!u) {
    if (!c->begun) return LMR_ESTATE;
    // the accepted field, copied so that the kernel sees a fixed pointer
    LMR_HIP(launch_copy_cur(c->st, c->U[0], c->U[1], c->graw, 3 * c->g.N, c->stream));
    u = c->graw;
  }
  LMR_HIP(launch_folds(u, c->g, c->counter, det_out, c->stream));
  unsigned long long n = 0;
  LMR_HIP(hipMemcpyAsync(&n, c->counter, sizeof n, hipMemcpyDeviceToHost, c->stream));
  LMR_HIP(hipStreamSynchronize(c->stream));
  *count_out = static_cast<long long>(n);
  return LMR_OK;
}

lmr_status lmr_smooth(lmr_ctx* c, const float* g, float* out) {
  if (!c || !g || !out || g == out) return LMR_EINVAL;
  LMR_HIP(launch_smooth(g, c->g, c->p, nullptr, out, c->stream));
  return LMR_OK;
}

lmr_status lmr_decide_probe(lmr_ctx* c, const lmr_pair_state* in, double cand_loss,
                            int force, lmr_pair_state* out) {
  if (!c || !in || !out || force < -1 || force > 1) return LMR_EINVAL;
  DevState h{};
  h.lambda = in->lambda;
  h.loss = in->loss;
  h.loss_prev = in->loss_prev;
  h.cand_loss = in->cand_loss;
  h.r = residual_of(in->loss, c->p.similarity, c->p.mi_bins);
  h.n_hist = in->n_hist;
  h.retries = in->retries;
  h.accepted = in->accepted;
  h.stalled = in->stalled;
  h.cur = 0;
  h.attempts = in->attempts;
  // one partial of -cand_loss over N = 1 reproduces cand_loss exactly
  const double part = -cand_loss;
  hipStream_t s = c->stream;
  LMR_HIP(hipMemcpyAsync(c->st_probe, &h, sizeof h, hipMemcpyHostToDevice, s));
  LMR_HIP(hipMemcpyAsync(c->part_probe, &part, sizeof part, hipMemcpyHostToDevice, s));
  LMR_HIP(launch_decide(c->st_probe, c->part_probe, 1, 1, c->dp, 0, force, 0.0,
                        nullptr, s));
  LMR_HIP(hipMemcpyAsync(&h, c->st_probe, sizeof h, hipMemcpyDeviceToHost, s));
  LMR_HIP(hipStreamSynchronize(s));
  out->lambda = h.lambda;
  out->loss = h.loss;
  out->loss_prev = h.loss_prev;
  out->cand_loss = h.cand_loss;
  out->n_hist = h.n_hist;
  out->retries = h.retries;
  out->accepted = h.accepted;
  out->stalled = h.stalled;
  out->attempts = h.attempts;
  return LMR_OK;
}

lmr_status lmr_warp(const void* M, lmr_dtype img, const float* u, int nz, int ny,
                    int nx, float* Mw, float* dMw, hipStream_t stream) {
  if (!M || !u || !Mw || nz < 1 || ny < 1 || nx < 1 || nz > 65535) return LMR_EINVAL;
  if (img != LMR_F32 && img != LMR_BF16) return LMR_EINVAL;
  long long N = (long long)nz * ny * nx;
  if (N >= (1LL << 30)) return LMR_EINVAL;
  LMR_HIP(launch_warp(M, img, u, Geom{nz, ny, nx, N}, Mw, dMw, stream));
  return LMR_OK;
}

// ------------------------------------------------------------ kernel timing
const char* lmr_kernel_name(int k) {
  static const char* names[LMR_NUM_KERNELS] = {"update", "lncc_fwd", "decide",
                                               "lncc_bwd", "smooth"};
  return (k >= 0 && k < LMR_NUM_KERNELS) ? names[k] : "unknown";
}

lmr_status lmr_profile_start(lmr_ctx* c, int max_attempts, int stride) {
  if (!c || max_attempts < 1 || stride < 1) return LMR_EINVAL;
  profile_release(c->prof);
  Profiler& pr = c->prof;
  pr.ev.resize((LMR_NUM_KERNELS + 1) * (size_t)max_attempts);
  for (auto& e : pr.ev) {
    hipError_t err = hipEventCreate(&e);
    if (err != hipSuccess) {
      e = nullptr;
      profile_release(pr);
      return hip_fail(err);
    }
  }
  pr.on = true;
  pr.stride = stride;
  pr.max_attempts = max_attempts;
  pr.recorded = 0;
  pr.seen = 0;
  return LMR_OK;
}

lmr_status lmr_profile_stop(lmr_ctx* c, lmr_kernel_time out[LMR_NUM_KERNELS]) {
  if (!c || !out) return LMR_EINVAL;
  Profiler& pr = c->prof;
  if (!pr.on) return LMR_ESTATE;
  for (int k = 0; k < LMR_NUM_KERNELS; ++k) out[k] = lmr_kernel_time{0, 0.0, 0.0, 0.0};
  hipError_t err = hipStreamSynchronize(c->stream);
  if (err != hipSuccess) {
    profile_release(pr);
    return hip_fail(err);
  }
  for (int a = 0; a < pr.recorded; ++a)
    for (int k = 0; k < LMR_NUM_KERNELS; ++k) {
      float ms = 0.0f;
      hipEvent_t* e = &pr.ev[(LMR_NUM_KERNELS + 1) * a + k];
      if (hipEventElapsedTime(&ms, e[0], e[1]) != hipSuccess) continue;
      lmr_kernel_time& t = out[k];
      if (t.count == 0 || ms < t.min_ms) t.min_ms = ms;
      if (ms > t.max_ms) t.max_ms = ms;
      t.total_ms += ms;
      t.count += 1;
    }
  profile_release(pr);
  return LMR_OK;
}

// ---------------------------------------------------------------- pyramid
lmr_status lmr_avgpool(const void* img, lmr_dtype t, int nz, int ny, int nx, int f,
                       float* out, hipStream_t stream) {
  if (!img || !out || f < 1 || nz < 1 || ny < 1 || nx < 1) return LMR_EINVAL;
  if (t != LMR_F32 && t != LMR_BF16) return LMR_EINVAL;
  if (nz % f || ny % f || nx % f) return LMR_EINVAL;
  LMR_HIP(launch_avgpool(img, t, nz, ny, nx, f, out, stream));
  return LMR_OK;
}

lmr_status lmr_upsample_field(const float* uc, int nzc, int nyc, int nxc, float* uf,
                              hipStream_t stream) {
  if (!uc || !uf || nzc < 1 || nyc < 1 || nxc < 1) return LMR_EINVAL;
  if (8LL * nzc * nyc * nxc >= (1LL << 30)) return LMR_EINVAL;
  LMR_HIP(launch_upsample_field(uc, nzc, nyc, nxc, uf, stream));
  return LMR_OK;
}

}  // extern "C"

struct lmr_pyramid {
  int nlevels;
  int factors[8];
  int dims[8][3];
  lmr_dtype img;
  hipStream_t stream;
  lmr_ctx* lv[8];
  float* Fl[8];   // pooled fixed image (null at factor 1)
  float* Ml[8];   // pooled moving image
  void* arena = nullptr;
  // HIP graphs of the attempt sequences, keyed by (level, images, attempts);
  // captured on a private stream, launched on the pyramid's stream
  bool use_graphs = true;
  hipStream_t cap = nullptr;
  std::map<std::tuple<int, const void*, const void*, int>, hipGraphExec_t> graphs;
};

namespace {

void drop_graphs(lmr_pyramid* y) {
  for (auto& kv : y->graphs) (void)hipGraphExecDestroy(kv.second);
  y->graphs.clear();
}

// n automatic attempts of level l as one graph launch on the pyramid's stream.
lmr_status step_graph(lmr_pyramid* y, int l, const void* Fl, const void* Ml, int n) {
  lmr_ctx* c = y->lv[l];
  const auto key = std::make_tuple(l, Fl, Ml, n);
  auto it = y->graphs.find(key);
  if (it == y->graphs.end()) {
    if (!y->cap) LMR_HIP(hipStreamCreateWithFlags(&y->cap, hipStreamNonBlocking));
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    const hipStream_t own = c->stream;
    c->stream = y->cap;
    hipError_t e = hipStreamBeginCapture(y->cap, hipStreamCaptureModeThreadLocal);
    lmr_status st = e == hipSuccess ? lmr_step(c, Fl, Ml, n) : LMR_OK;
    if (e == hipSuccess) e = hipStreamEndCapture(y->cap, &graph);
    c->stream = own;
    if (st != LMR_OK) {
      if (graph) (void)hipGraphDestroy(graph);
      return st;
    }
    if (e == hipSuccess) e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    if (graph) (void)hipGraphDestroy(graph);
    LMR_HIP(e);
    it = y->graphs.emplace(key, exec).first;
  }
  LMR_HIP(hipGraphLaunch(it->second, y->stream));
  return LMR_OK;
}

// n attempts of level l. Without kernel timing they are one graph launch. With
// timing every stride-th attempt (stride > 1) runs eagerly between its events
// and the attempts in between run as graphs, so the timed sequence is the
// graph sequence but for the sampled attempts.
lmr_status step_sampled(lmr_pyramid* y, int l, const void* Fl, const void* Ml, int n) {
  lmr_ctx* c = y->lv[l];
  Profiler& pr = c->prof;
  if (!pr.on) return step_graph(y, l, Fl, Ml, n);
  for (int done = 0; done < n;) {
    int k = static_cast<int>(pr.stride - pr.seen % pr.stride) % pr.stride;
    if (k == 0) {
      lmr_status st = lmr_step(c, Fl, Ml, 1);  // records its events
      if (st != LMR_OK) return st;
      ++done;
      continue;
    }
    k = std::min(k, n - done);
    pr.on = false;  // nothing of the profiler goes into a captured graph
    lmr_status st = step_graph(y, l, Fl, Ml, k);
    pr.on = true;
    if (st != LMR_OK) return st;
    pr.seen += k;
    done += k;
  }
  return LMR_OK;
}

}  // namespace

extern "C" {

void lmr_pyramid_destroy(lmr_pyramid* y) {
  if (!y) return;
  (void)hipStreamSynchronize(y->stream);
  drop_graphs(y);
  if (y->cap) (void)hipStreamDestroy(y->cap);
  for (int l = 0; l < y->nlevels; ++l) lmr_destroy(y->lv[l]);
  (void)hipFree(y->arena);
  delete y;
}

lmr_status lmr_pyramid_use_graphs(lmr_pyramid* y, int enable) {
  if (!y) return LMR_EINVAL;
  y->use_graphs = enable != 0;
  return LMR_OK;
}

lmr_status lmr_pyramid_create(lmr_pyramid** out, int nz, int ny, int nx, lmr_dtype img,
                              const lmr_params* p, int nlevels, const int* factors,
                              hipStream_t stream) {
  if (!out || !factors || nlevels < 1 || nlevels > 8) return LMR_EINVAL;
  *out = nullptr;
  if (factors[nlevels - 1] != 1) return LMR_EINVAL;
  for (int l = 0; l + 1 < nlevels; ++l)
    if (factors[l] != 2 * factors[l + 1]) return LMR_EINVAL;
  const int f0 = factors[0];
  if (nz < 1 || ny < 1 || nx < 1 || nz % f0 || ny % f0 || nx % f0) return LMR_EINVAL;
  if (!params_ok(p)) return LMR_EINVAL;
  lmr_pyramid* y = new (std::nothrow) lmr_pyramid();
  if (!y) return LMR_ENOMEM;
  y->nlevels = nlevels;
  y->img = img;
  y->stream = stream;
  size_t total = 0;
  for (int l = 0; l < nlevels; ++l) {
    const int f = factors[l];
    y->factors[l] = f;
    y->dims[l][0] = nz / f;
    y->dims[l][1] = ny / f;
    y->dims[l][2] = nx / f;
    const size_t n = (size_t)(nz / f) * (ny / f) * (nx / f);
    total += f > 1 ? 2 * align256(4 * n) : 0;
  }
  if (total > 0 && hipMalloc(&y->arena, total) != hipSuccess) {
    delete y;
    return LMR_ENOMEM;
  }
  char* q = static_cast<char*>(y->arena);
  for (int l = 0; l < nlevels; ++l) {
    const size_t n = (size_t)y->dims[l][0] * y->dims[l][1] * y->dims[l][2];
    y->Fl[l] = y->Ml[l] = nullptr;
    if (factors[l] > 1) {
      y->Fl[l] = reinterpret_cast<float*>(q);
      q += align256(4 * n);
      y->Ml[l] = reinterpret_cast<float*>(q);
      q += align256(4 * n);
    }
    lmr_status st = lmr_create(&y->lv[l], y->dims[l][0], y->dims[l][1], y->dims[l][2],
                               factors[l] > 1 ? LMR_F32 : img, p, stream);
    if (st != LMR_OK) {
      y->nlevels = l;
      lmr_pyramid_destroy(y);
      return st;
    }
  }
  *out = y;
  return LMR_OK;
}

lmr_ctx* lmr_pyramid_level(lmr_pyramid* y, int l) {
  return (y && l >= 0 && l < y->nlevels) ? y->lv[l] : nullptr;
}

lmr_status lmr_pyramid_run(lmr_pyramid* y, const void* F, const void* M,
                           const int* iters, double lambda0, const int* decisions,
                           float* field_out) {
  if (!y || !F || !M || !iters || !field_out || !(lambda0 > 0.0)) return LMR_EINVAL;
  for (int l = 0; l < y->nlevels; ++l)
    if (iters[l] < 0) return LMR_EINVAL;
  const int* d = decisions;
  const int* fine = y->dims[y->nlevels - 1];
  for (int l = 0; l < y->nlevels; ++l) {
    lmr_ctx* c = y->lv[l];
    const void* Fl = F;
    const void* Ml = M;
    if (y->factors[l] > 1) {
      LMR_HIP(launch_avgpool(F, y->img, fine[0], fine[1], fine[2], y->factors[l], y->Fl[l],
                             y->stream));
      LMR_HIP(launch_avgpool(M, y->img, fine[0], fine[1], fine[2], y->factors[l], y->Ml[l],
                             y->stream));
      Fl = y->Fl[l];
      Ml = y->Ml[l];
    }
    const float* u0 = nullptr;
    if (l > 0) {
      // the coarse level's current field, upsampled straight into this
      // level's first field buffer (lmr_begin then copies nothing)
      const lmr_ctx* pc = y->lv[l - 1];
      LMR_HIP(launch_upsample_cur(pc->st, pc->U[0], pc->U[1], y->dims[l - 1][0],
                                  y->dims[l - 1][1], y->dims[l - 1][2], c->U[0], y->stream));
      u0 = c->U[0];
    }
    lmr_status st = lmr_begin(c, Fl, Ml, u0, lambda0);
    if (st != LMR_OK) return st;
    if (d)
      st = lmr_step_forced(c, Fl, Ml, d, iters[l]);
    else if (y->use_graphs && iters[l] > 0 && !(c->prof.on && c->prof.stride == 1))
      st = step_sampled(y, l, Fl, Ml, iters[l]);
    else
      st = lmr_step(c, Fl, Ml, iters[l]);
    if (st != LMR_OK) return st;
    if (d) d += iters[l];
  }
  return lmr_get_field(y->lv[y->nlevels - 1], field_out);
}

}  // extern "C"
