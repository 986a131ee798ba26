// C-ABI of the batched persistent form: many uneven-size pairs advance by one
// LM attempt per persistent launch; the launches of a step are captured once
// in a HIP graph and replayed.  Tile shapes and the persistent grid are
// chosen by a measuring autotuner whose choices are cached in a text file.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stddef.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <map>
#include <new>
#include <string>
#include <vector>

#include "ctx.h"
#include "lmr_batch.h"

using namespace lmr;

struct lmr_batch {
  int npairs = 0;
  lmr_dtype img = LMR_F32;
  lmr_params p{};
  DecideParams dp{};
  hipStream_t stream = nullptr;
  std::vector<lmr_ctx*> ctx;
  std::vector<BatchPair> host;
  BatchPair* dev_pairs = nullptr;
  BatchCtl* ctl = nullptr;
  std::vector<double*> partials;  // per pair, sized for the smallest z-chunk
  const void* kernel = nullptr;
  int cus = 0, max_blocks_per_cu = 0;
  bool any_march = false, any_bricks = false;  // the stencil forms of the pairs
  // tuned configuration
  // target_tiles 0: each pair tiled as a stand-alone context's march tiles it;
  // blocks_per_cu -1: one launch per phase (no persistent kernel)
  int target_tiles = 0, min_cz = 16, blocks_per_cu = -1;
  int n_update_items = 0, n_tiles = 0;
  unsigned long long timeout = 0;  // barrier timeout in wall-clock ticks
  unsigned long long start_timeout = 0;  // co-residency check, wall-clock ticks
  int missing = 0;                       // test hook (lmr_batch_test_residency)
  std::map<int, hipGraphExec_t> graphs;  // n_iters -> instantiated graph
  bool begun = false;
};

namespace {

int gauss_r(double sigma) { return sigma > 0.0 ? (int)ceil(3.0 * sigma - 1e-12) : 0; }

void drop_graphs(lmr_batch* b) {
  for (auto& kv : b->graphs) (void)hipGraphExecDestroy(kv.second);
  b->graphs.clear();
}

// Rebuild the work lists for the current tiling knobs and upload the table.
lmr_status layout(lmr_batch* b) {
  int vox = 0, tiles = 0;
  const int ty = batch_tile_rows();
  for (int i = 0; i < b->npairs; ++i) {
    BatchPair& P = b->host[i];
    P.t = b->target_tiles > 0
              ? make_tiling(P.g.nz, P.g.ny, P.g.nx, ty, b->target_tiles, b->min_cz)
              : march_tiling(P.g, b->p.window / 2);
    const int ucols = ((P.g.nx + kBatchUpdateTX - 1) / kBatchUpdateTX) *
                      ((P.g.ny + kBatchUpdateTY - 1) / kBatchUpdateTY);
    P.ucz = static_cast<int>(((long long)P.g.nz * ucols + kBatchUpdateItems - 1) /
                             kBatchUpdateItems);
    P.ucz = std::min(std::max(P.ucz, kBatchUpdateMinCz), kBatchUpdateMaxCz);
    P.ntiles = P.bricks ? brick_count(P.g, kBatchBrickTZ) : P.t.tiles();
    P.utile0 = vox;
    P.tile0 = tiles;
    vox += ucols * ((P.g.nz + P.ucz - 1) / P.ucz);
    tiles += P.ntiles;
  }
  b->n_update_items = vox;
  b->n_tiles = tiles;
  LMR_HIP(hipMemcpyAsync(b->dev_pairs, b->host.data(), sizeof(BatchPair) * b->npairs,
                         hipMemcpyHostToDevice, b->stream));
  // the barrier counters count arrivals of one grid size: start them over
  // (the error flag stays until lmr_batch_sync reports it)
  LMR_HIP(hipMemsetAsync(b->ctl, 0, offsetof(BatchCtl, error), b->stream));
  drop_graphs(b);
  return LMR_OK;
}

int grid_of(const lmr_batch* b) {
  const int per = b->blocks_per_cu > 0 ? std::min(b->blocks_per_cu, b->max_blocks_per_cu)
                                       : b->max_blocks_per_cu;
  return std::max(1, per * b->cus);
}

lmr_status enqueue_steps(lmr_batch* b, int n) {
  if (b->blocks_per_cu < 0) {  // one launch per phase
    const int rb = b->p.window / 2, rg = gauss_r(b->p.grad_sigma);
    for (int i = 0; i < n; ++i)
      LMR_HIP(launch_batch_phases(b->img, static_cast<lmr_accum>(b->p.accum), rb, rg,
                                  b->any_march, b->any_bricks, b->dev_pairs, b->npairs,
                                  b->n_update_items, b->n_tiles, b->dp, b->stream));
    return LMR_OK;
  }
  const int grid = grid_of(b);
  for (int i = 0; i < n; ++i)
    LMR_HIP(launch_batch_attempt(b->kernel, grid, b->dev_pairs, b->npairs, b->n_update_items,
                                 b->n_tiles, b->ctl, b->dp, b->timeout, b->start_timeout,
                                 b->missing, b->stream));
  return LMR_OK;
}

std::string cache_key(const lmr_batch* b) {
  char buf[128];
  snprintf(buf, sizeof buf, "gfx950|v2|img%d|acc%d|w%d|s%.3f|", (int)b->img, b->p.accum,
           b->p.window, b->p.grad_sigma);
  std::string k = buf;
  for (const auto& P : b->host) {
    snprintf(buf, sizeof buf, "%dx%dx%d,", P.g.nz, P.g.ny, P.g.nx);
    k += buf;
  }
  return k;
}

}  // namespace

extern "C" {

void lmr_batch_destroy(lmr_batch* b) {
  if (!b) return;
  (void)hipStreamSynchronize(b->stream);
  drop_graphs(b);
  for (lmr_ctx* c : b->ctx) lmr_destroy(c);
  for (double* p : b->partials) (void)hipFree(p);
  (void)hipFree(b->dev_pairs);
  (void)hipFree(b->ctl);
  if (b->stream) (void)hipStreamDestroy(b->stream);
  delete b;
}

lmr_status lmr_batch_create(lmr_batch** out, int npairs, const int* shapes, lmr_dtype img,
                            const lmr_params* p) {
  if (!out || npairs < 1 || npairs > 4096 || !shapes) return LMR_EINVAL;
  *out = nullptr;
  if (!params_ok(p) || (img != LMR_F32 && img != LMR_BF16)) return LMR_EINVAL;
  // the batched kernel runs the rank-1 LM attempt only
  if (p->tile != 1 || p->optimizer != LMR_OPT_LM || p->similarity != LMR_SIM_LNCC)
    return LMR_EINVAL;
  const int rb = p->window / 2, rg = gauss_r(p->grad_sigma);
  // pair i runs its stencils on 4-plane bricks where a stand-alone context
  // does (small pairs), else it marches; the pair's own begin uses that form
  std::vector<char> bricks(npairs, 0);
  bool any_bricks = false;
  for (int i = 0; i < npairs; ++i) {
    const int nz = shapes[3 * i], ny = shapes[3 * i + 1], nx = shapes[3 * i + 2];
    if (nz < 1 || ny < 1 || nx < 1) return LMR_EINVAL;
    const Geom gi{nz, ny, nx, (long long)nz * ny * nx};
    bricks[i] = brick_depth(gi, *p) == kBatchBrickTZ;
    any_bricks = any_bricks || bricks[i];
  }
  const void* kernel =
      batch_kernel(img, static_cast<lmr_accum>(p->accum), rb, rg, any_bricks);
  if (!kernel) return LMR_EINVAL;  // Gaussian radius beyond the instantiated range
  lmr_batch* b = new (std::nothrow) lmr_batch();
  if (!b) return LMR_ENOMEM;
  b->npairs = npairs;
  b->img = img;
  b->p = *p;
  b->dp = DecideParams{p->lambda_inc, p->lambda_dec, p->lambda_min, p->lambda_max,
                       p->tau, p->max_retries};
  b->kernel = kernel;
  b->any_bricks = any_bricks;
  for (int i = 0; i < npairs; ++i) b->any_march = b->any_march || !bricks[i];
  auto fail = [&](lmr_status s) {
    lmr_batch_destroy(b);
    return s;
  };
  if (hipStreamCreateWithFlags(&b->stream, hipStreamNonBlocking) != hipSuccess)
    return fail(LMR_EHIP);
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&b->cus, hipDeviceAttributeMultiprocessorCount, dev) !=
          hipSuccess ||
      hipOccupancyMaxActiveBlocksPerMultiprocessor(&b->max_blocks_per_cu, kernel,
                                                   batch_block_threads(), 0) != hipSuccess ||
      b->max_blocks_per_cu < 1)
    return fail(LMR_EHIP);
  int wall_khz = 0;
  if (hipDeviceGetAttribute(&wall_khz, hipDeviceAttributeWallClockRate, dev) != hipSuccess ||
      wall_khz <= 0)
    wall_khz = 100000;
  b->timeout = (unsigned long long)wall_khz * 250;  // 0.25 s per barrier wait
  // blocks of one launch start within microseconds of each other when the
  // GPU is free: 2 ms at the first barrier with some block not started means
  // the grid is not co-resident
  b->start_timeout = (unsigned long long)wall_khz * 2;
  float taps[16] = {0};
  {
    const int R = rg;
    double t[16], tot = 0.0;
    for (int k = -R; k <= R; ++k) {
      t[k + R] = R == 0 ? 1.0 : exp(-(double)k * k / (2.0 * p->grad_sigma * p->grad_sigma));
      tot += t[k + R];
    }
    for (int k = 0; k <= 2 * R; ++k) taps[k] = static_cast<float>(t[k] / tot);
  }
  b->ctx.resize(npairs, nullptr);
  b->host.resize(npairs);
  b->partials.resize(npairs, nullptr);
  for (int i = 0; i < npairs; ++i) {
    const int nz = shapes[3 * i], ny = shapes[3 * i + 1], nx = shapes[3 * i + 2];
    const Geom gi{nz, ny, nx, (long long)nz * ny * nx};
    lmr_params pc = *p;
    pc.stencil = bricks[i] ? LMR_STENCIL_CUBE : LMR_STENCIL_MARCH;
    lmr_status st = lmr_create(&b->ctx[i], nz, ny, nx, img, &pc, b->stream);
    if (st != LMR_OK) return fail(st);
    lmr_ctx* c = b->ctx[i];
    // partial slots for the largest tile count any tuning can produce (cz >=
    // 2), or the pair's bricks
    const int ty = batch_tile_rows();
    const size_t maxt =
        bricks[i] ? (size_t)brick_count(gi, kBatchBrickTZ)
               : (size_t)((nx + kTX - 1) / kTX) * ((ny + ty - 1) / ty) * ((nz + 1) / 2);
    if (hipMalloc(&b->partials[i], sizeof(double) * maxt) != hipSuccess)
      return fail(LMR_ENOMEM);
    BatchPair& P = b->host[i];
    memset(&P, 0, sizeof P);
    P.g = c->g;
    P.bricks = bricks[i] ? 1 : 0;
    P.U0 = c->U[0];
    P.U1 = c->U[1];
    P.G = c->G;
    P.graw = c->graw;
    P.maps = c->maps;
    P.Mw = c->Mw;
    P.fstat = c->fstat;
    P.partials = b->partials[i];
    P.st = c->st;
    P.eps = static_cast<float>(p->step_eps);
    P.compositive = p->compositive;
    P.inv_n = 1.0 / ((double)p->window * p->window * p->window);
    P.cc_eps = p->cc_eps;
    memcpy(P.gw, taps, sizeof taps);
  }
  if (hipMalloc(&b->dev_pairs, sizeof(BatchPair) * npairs) != hipSuccess ||
      hipMalloc(&b->ctl, sizeof(BatchCtl)) != hipSuccess)
    return fail(LMR_ENOMEM);
  if (hipMemsetAsync(b->ctl, 0, sizeof(BatchCtl), b->stream) != hipSuccess)
    return fail(LMR_EHIP);
  if (layout(b) != LMR_OK) return fail(LMR_EHIP);
  *out = b;
  return LMR_OK;
}

lmr_status lmr_batch_begin(lmr_batch* b, const void* const* fixed,
                           const void* const* moving, const double* lambda0) {
  if (!b || !fixed || !moving) return LMR_EINVAL;
  for (int i = 0; i < b->npairs; ++i) {
    const double l0 = lambda0 ? lambda0[i] : 1.0;
    lmr_status st = lmr_begin(b->ctx[i], fixed[i], moving[i], nullptr, l0);
    if (st != LMR_OK) return st;
    b->host[i].F = fixed[i];
    b->host[i].M = moving[i];
  }
  LMR_HIP(hipMemcpyAsync(b->dev_pairs, b->host.data(), sizeof(BatchPair) * b->npairs,
                         hipMemcpyHostToDevice, b->stream));
  // no begin kernel of this batch may still run when any batch's persistent
  // launch needs the whole GPU
  LMR_HIP(hipStreamSynchronize(b->stream));
  b->begun = true;
  return LMR_OK;
}

lmr_status lmr_batch_step(lmr_batch* b, int n_iters, int use_graph) {
  if (!b || n_iters < 0) return LMR_EINVAL;
  if (!b->begun) return LMR_ESTATE;
  if (n_iters == 0) return LMR_OK;
  if (!use_graph) return enqueue_steps(b, n_iters);
  auto it = b->graphs.find(n_iters);
  if (it == b->graphs.end()) {
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    LMR_HIP(hipStreamBeginCapture(b->stream, hipStreamCaptureModeThreadLocal));
    lmr_status st = enqueue_steps(b, n_iters);
    hipError_t e = hipStreamEndCapture(b->stream, &graph);
    if (st != LMR_OK) {
      if (graph) (void)hipGraphDestroy(graph);
      return st;
    }
    LMR_HIP(e);
    e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    LMR_HIP(e);
    it = b->graphs.emplace(n_iters, exec).first;
  }
  LMR_HIP(hipGraphLaunch(it->second, b->stream));
  return LMR_OK;
}

lmr_status lmr_batch_sync(lmr_batch* b) {
  if (!b) return LMR_EINVAL;
  LMR_HIP(hipStreamSynchronize(b->stream));
  BatchCtl h;
  LMR_HIP(hipMemcpy(&h, b->ctl, sizeof h, hipMemcpyDeviceToHost));
  if (h.error.v) {
    // clear the flag so that the batch can be used again
    LMR_HIP(hipMemset(b->ctl, 0, sizeof(BatchCtl)));
    return h.error.v == 2 ? LMR_EBUSY : LMR_EHIP;
  }
  return LMR_OK;
}

lmr_status lmr_batch_test_residency(lmr_batch* b, int late_block) {
  if (!b || late_block < 0 || late_block > 1) return LMR_EINVAL;
  b->missing = late_block;
  drop_graphs(b);  // captured launches hold the old value
  return LMR_OK;
}

lmr_ctx* lmr_batch_pair(lmr_batch* b, int i) {
  return (b && i >= 0 && i < b->npairs) ? b->ctx[i] : nullptr;
}

lmr_status lmr_batch_get_config(lmr_batch* b, int cfg[3]) {
  if (!b || !cfg) return LMR_EINVAL;
  cfg[0] = b->target_tiles;
  cfg[1] = b->min_cz;
  cfg[2] = b->blocks_per_cu != 0 ? b->blocks_per_cu : b->max_blocks_per_cu;
  return LMR_OK;
}

lmr_status lmr_batch_set_config(lmr_batch* b, int target_tiles, int min_cz,
                                int blocks_per_cu) {
  if (!b || (target_tiles != 0 && (target_tiles < 64 || target_tiles > (1 << 20))) ||
      min_cz < 4 || min_cz > 256 || blocks_per_cu < -1)
    return LMR_EINVAL;
  b->target_tiles = target_tiles;
  b->min_cz = min_cz;
  b->blocks_per_cu = blocks_per_cu;
  return layout(b);
}

lmr_status lmr_batch_tune(lmr_batch* b, const void* const* fixed, const void* const* moving,
                          const char* cache_path, int iters_per_trial, double* best_ms) {
  if (!b || !fixed || !moving || iters_per_trial < 1) return LMR_EINVAL;
  const std::string key = cache_key(b);
  if (cache_path) {
    if (FILE* f = fopen(cache_path, "r")) {
      char line[4096];
      while (fgets(line, sizeof line, f)) {
        char k[3000];
        int tt, mc, bpc;
        double ms;
        if (sscanf(line, "%2999s %d %d %d %lf", k, &tt, &mc, &bpc, &ms) == 5 && key == k) {
          fclose(f);
          if (best_ms) *best_ms = ms;
          return lmr_batch_set_config(b, tt, mc, bpc);
        }
      }
      fclose(f);
    }
  }
  hipEvent_t e0, e1;
  LMR_HIP(hipEventCreate(&e0));
  LMR_HIP(hipEventCreate(&e1));
  double best = 1e30;
  int bt = b->target_tiles, bm = b->min_cz, bb = b->blocks_per_cu;
  // target 0 (the per-pair tiling) does not use the chunk minimum
  const int tts[] = {0, 1024, 2048, 4096, 8192};
  const int mcs[] = {8, 16, 32};
  for (int tt : tts)
    for (int mc : mcs)
      for (int bpc = -1; bpc <= b->max_blocks_per_cu; ++bpc) {
        if (bpc == 0 || (tt == 0 && mc != 16)) continue;
        lmr_status st = lmr_batch_set_config(b, tt, mc, bpc);
        if (st == LMR_OK) st = lmr_batch_begin(b, fixed, moving, nullptr);
        if (st == LMR_OK) st = lmr_batch_step(b, 1, 0);  // warm-up
        if (st == LMR_OK && hipEventRecord(e0, b->stream) != hipSuccess) st = LMR_EHIP;
        if (st == LMR_OK) st = lmr_batch_step(b, iters_per_trial, 0);
        if (st == LMR_OK && hipEventRecord(e1, b->stream) != hipSuccess) st = LMR_EHIP;
        if (st == LMR_OK) st = lmr_batch_sync(b);
        if (st != LMR_OK) {
          (void)hipEventDestroy(e0);
          (void)hipEventDestroy(e1);
          return st;
        }
        float ms = 0.0f;
        (void)hipEventElapsedTime(&ms, e0, e1);
        const double per = ms / iters_per_trial;
        if (per < best) {
          best = per;
          bt = tt;
          bm = mc;
          bb = bpc;
        }
      }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  b->begun = false;  // the trials overwrote the pair states
  if (best_ms) *best_ms = best;
  if (cache_path) {
    if (FILE* f = fopen(cache_path, "a")) {
      fprintf(f, "%s %d %d %d %.17g\n", key.c_str(), bt, bm, bb, best);
      fclose(f);
    }
  }
  return lmr_batch_set_config(b, bt, bm, bb);
}

}  // extern "C"
