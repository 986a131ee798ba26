// C-ABI of the learned initializer's U-Net (include/lmreg_unet.h): buffers,
// the layer graph, forward, backward and Adam.
#include <hip/hip_runtime.h>
#include <math.h>

#include <new>
#include <vector>

#include "ctx.h"
#include "lmreg_unet.h"
#include "unet_internal.h"

using namespace lmr;

namespace {

struct LayerDef {
  int cin, cout, relu, level;
};
// Network definition (header comment of lmreg_unet.h).
constexpr LayerDef kLayers[LMR_UNET_LAYERS] = {
    {2, 16, 1, 0},    {16, 16, 1, 0},  {16, 32, 1, 1},  {32, 32, 1, 1},  {32, 64, 1, 2},
    {64, 64, 1, 2},   {64, 128, 1, 3}, {128, 128, 1, 3}, {192, 64, 1, 2}, {64, 64, 1, 2},
    {96, 32, 1, 1},   {32, 32, 1, 1},  {48, 16, 1, 0},  {16, 16, 1, 0},  {16, 3, 0, 0}};

int pad16(int c) { return (c + 15) / 16 * 16; }

long long layer_offset(int l) {
  long long o = 0;
  for (int i = 0; i < l; ++i) o += 27LL * kLayers[i].cin * kLayers[i].cout + kLayers[i].cout;
  return o;
}

long long param_count() { return layer_offset(LMR_UNET_LAYERS); }

// A channels-last BF16 view: base pointer and channel stride.
struct T {
  uint16_t* p;
  int ld;
  T at(int c) const { return T{p + c, ld}; }
};

}  // namespace

struct lmr_unet {
  int dims[4][3];  // level d: (nz, ny, nx) >> d
  long long n[4];
  hipStream_t stream;
  std::vector<void*> allocs;
  float *params, *grads, *m1, *m2;
  uint16_t* Wf[LMR_UNET_LAYERS];
  uint16_t* Wb[LMR_UNET_LAYERS];
  // activations
  T x, e1a, c1, p1, e2a, c2, p2, e3a, c3, p3, e4a, e4, f3a, f3, f2a, f2, f1a, f1;
  float* yf;  // head output, FP32, stride 4
  // gradients (with respect to post-activation values)
  T d_out, d_f1, d_f1a, d_c1, d_f2, d_f2a, d_c2, d_f3, d_f3a, d_c3, d_e4, d_e4a, d_p3,
      d_e3a, d_p2, d_e2a, d_p1, d_e1a;
  float *part, *partb;
  double *mse_part, *loss_scratch;
  long long step;
  bool have_forward;
};

namespace {

lmr_status alloc(lmr_unet* u, size_t bytes, void** out) {
  void* p = nullptr;
  if (hipMalloc(&p, bytes) != hipSuccess) return LMR_ENOMEM;
  u->allocs.push_back(p);
  *out = p;
  return LMR_OK;
}

lmr_status alloc_t(lmr_unet* u, int level, int ld, T* t) {
  void* p;
  const size_t bytes = static_cast<size_t>(u->n[level]) * ld * sizeof(uint16_t);
  lmr_status s = alloc(u, bytes, &p);
  if (s != LMR_OK) return s;
  t->p = static_cast<uint16_t*>(p);
  t->ld = ld;
  return LMR_OK;
}

void free_all(lmr_unet* u) {
  for (void* p : u->allocs) (void)hipFree(p);
  u->allocs.clear();
}

float* W_of(float* flat, int l) { return flat + layer_offset(l); }
float* b_of(float* flat, int l) {
  return flat + layer_offset(l) + 27LL * kLayers[l].cin * kLayers[l].cout;
}

hipError_t pack_all(lmr_unet* u) {
  for (int l = 0; l < LMR_UNET_LAYERS; ++l) {
    hipError_t e = unet_pack(W_of(u->params, l), kLayers[l].cin, kLayers[l].cout,
                             pad16(kLayers[l].cin), pad16(kLayers[l].cout), u->Wf[l],
                             u->Wb[l], u->stream);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

// y = act(conv_l(x) + b_l)
hipError_t conv_fwd(lmr_unet* u, int l, T x, int cin_valid, T y, float* yf, int ldf) {
  const LayerDef& L = kLayers[l];
  const int* d = u->dims[L.level];
  ConvArgs a{};
  a.X = x.p;
  a.ldx = x.ld;
  a.cin_valid = cin_valid;
  a.cin_p = pad16(L.cin);
  a.W = u->Wf[l];
  a.bias = b_of(u->params, l);
  a.cout = L.cout;
  a.cout_p = pad16(L.cout);
  a.Y = y.p;
  a.ldy = y.ld;
  a.yf = yf;
  a.ldf = ldf;
  a.nz = d[0];
  a.ny = d[1];
  a.nx = d[2];
  a.relu = L.relu;
  return unet_conv(a, u->stream);
}

// Gradients of layer l from its input x and the gradient dz of its
// pre-activation output; dx (may have p == NULL) receives the input gradient.
hipError_t conv_bwd(lmr_unet* u, int l, T x, T dz, T dx, int accumulate) {
  const LayerDef& L = kLayers[l];
  const int* d = u->dims[L.level];
  hipError_t e = unet_wgrad(x.p, x.ld, L.cin, pad16(L.cin), dz.p, dz.ld, L.cout,
                            pad16(L.cout), d[0], d[1], d[2], u->part, u->partb,
                            W_of(u->grads, l), b_of(u->grads, l), accumulate, u->stream);
  if (e != hipSuccess || !dx.p) return e;
  ConvArgs a{};
  a.X = dz.p;
  a.ldx = dz.ld;
  a.cin_valid = L.cout;
  a.cin_p = pad16(L.cout);
  a.W = u->Wb[l];
  a.bias = nullptr;
  a.cout = L.cin;
  a.cout_p = pad16(L.cin);
  a.Y = dx.p;
  a.ldy = dx.ld;
  a.yf = nullptr;
  a.ldf = 0;
  a.nz = d[0];
  a.ny = d[1];
  a.nx = d[2];
  a.relu = 0;
  return unet_conv(a, u->stream);
}

hipError_t mask(lmr_unet* u, int level, T d, T a, int C) {
  return unet_relu_mask(d.p, d.ld, a.p, a.ld, C, u->n[level], u->stream);
}

#define LMR_TRY(expr)                                \
  do {                                               \
    hipError_t e_ = (expr);                          \
    if (e_ != hipSuccess) return lmr::hip_fail(e_);  \
  } while (0)

}  // namespace

extern "C" {

int64_t lmr_unet_param_count(void) { return param_count(); }

lmr_status lmr_unet_layer_info(int layer, int* cin, int* cout, int* relu, int64_t* offset) {
  if (layer < 0 || layer >= LMR_UNET_LAYERS) return LMR_EINVAL;
  if (cin) *cin = kLayers[layer].cin;
  if (cout) *cout = kLayers[layer].cout;
  if (relu) *relu = kLayers[layer].relu;
  if (offset) *offset = layer_offset(layer);
  return LMR_OK;
}

void lmr_unet_destroy(lmr_unet* u) {
  if (!u) return;
  free_all(u);
  delete u;
}

lmr_status lmr_unet_create(lmr_unet** out, int nz, int ny, int nx, hipStream_t stream) {
  if (!out) return LMR_EINVAL;
  *out = nullptr;
  if (nz < 8 || ny < 8 || nx < 8 || nz % 8 || ny % 8 || nx % 8) return LMR_EINVAL;
  if ((long long)nz * ny * nx >= (1LL << 28)) return LMR_EINVAL;
  lmr_unet* u = new (std::nothrow) lmr_unet();
  if (!u) return LMR_ENOMEM;
  u->stream = stream;
  for (int d = 0; d < 4; ++d) {
    u->dims[d][0] = nz >> d;
    u->dims[d][1] = ny >> d;
    u->dims[d][2] = nx >> d;
    u->n[d] = (long long)u->dims[d][0] * u->dims[d][1] * u->dims[d][2];
  }
  lmr_status s = LMR_OK;
  auto A = [&](size_t bytes, void** p) {
    if (s == LMR_OK) s = alloc(u, bytes, p);
  };
  auto AT = [&](int level, int ld, T* t) {
    if (s == LMR_OK) s = alloc_t(u, level, ld, t);
  };
  const size_t np = static_cast<size_t>(param_count());
  A(np * 4, reinterpret_cast<void**>(&u->params));
  A(np * 4, reinterpret_cast<void**>(&u->grads));
  A(np * 4, reinterpret_cast<void**>(&u->m1));
  A(np * 4, reinterpret_cast<void**>(&u->m2));
  long long part_n = 0, partb_n = 0;
  for (int l = 0; l < LMR_UNET_LAYERS; ++l) {
    const size_t pk = 27ULL * pad16(kLayers[l].cin) * pad16(kLayers[l].cout) * 2;
    A(pk, reinterpret_cast<void**>(&u->Wf[l]));
    A(pk, reinterpret_cast<void**>(&u->Wb[l]));
    const int* d = u->dims[kLayers[l].level];
    const long long a = unet_wgrad_part_floats(pad16(kLayers[l].cin),
                                               pad16(kLayers[l].cout), d[0], d[1], d[2]);
    const long long b = unet_wgrad_bias_floats(pad16(kLayers[l].cin),
                                               pad16(kLayers[l].cout), d[0], d[1], d[2]);
    if (a > part_n) part_n = a;
    if (b > partb_n) partb_n = b;
  }
  A(static_cast<size_t>(part_n) * 4, reinterpret_cast<void**>(&u->part));
  A(static_cast<size_t>(partb_n) * 4, reinterpret_cast<void**>(&u->partb));
  A(static_cast<size_t>(unet_mse_blocks(u->n[0])) * 8, reinterpret_cast<void**>(&u->mse_part));
  A(8, reinterpret_cast<void**>(&u->loss_scratch));
  AT(0, 4, &u->x);
  AT(0, 16, &u->e1a);
  AT(0, 48, &u->c1);
  AT(1, 16, &u->p1);
  AT(1, 32, &u->e2a);
  AT(1, 96, &u->c2);
  AT(2, 32, &u->p2);
  AT(2, 64, &u->e3a);
  AT(2, 192, &u->c3);
  AT(3, 64, &u->p3);
  AT(3, 128, &u->e4a);
  AT(3, 128, &u->e4);
  AT(2, 64, &u->f3a);
  AT(2, 64, &u->f3);
  AT(1, 32, &u->f2a);
  AT(1, 32, &u->f2);
  AT(0, 16, &u->f1a);
  AT(0, 16, &u->f1);
  A(static_cast<size_t>(u->n[0]) * 4 * 4, reinterpret_cast<void**>(&u->yf));
  AT(0, 4, &u->d_out);
  AT(0, 16, &u->d_f1);
  AT(0, 16, &u->d_f1a);
  AT(0, 48, &u->d_c1);
  AT(1, 32, &u->d_f2);
  AT(1, 32, &u->d_f2a);
  AT(1, 96, &u->d_c2);
  AT(2, 64, &u->d_f3);
  AT(2, 64, &u->d_f3a);
  AT(2, 192, &u->d_c3);
  AT(3, 128, &u->d_e4);
  AT(3, 128, &u->d_e4a);
  AT(3, 64, &u->d_p3);
  AT(2, 64, &u->d_e3a);
  AT(2, 32, &u->d_p2);
  AT(1, 32, &u->d_e2a);
  AT(1, 16, &u->d_p1);
  AT(0, 16, &u->d_e1a);
  if (s != LMR_OK) {
    lmr_unet_destroy(u);
    return s;
  }
  // zero parameters, moments and the padding channel of d_out
  hipError_t e = hipMemsetAsync(u->params, 0, np * 4, stream);
  if (e == hipSuccess) e = hipMemsetAsync(u->grads, 0, np * 4, stream);
  if (e == hipSuccess) e = hipMemsetAsync(u->m1, 0, np * 4, stream);
  if (e == hipSuccess) e = hipMemsetAsync(u->m2, 0, np * 4, stream);
  if (e == hipSuccess) e = unet_zero(u->d_out.p, u->n[0] * 4, stream);
  if (e == hipSuccess) e = unet_zero(u->x.p, u->n[0] * 4, stream);
  if (e == hipSuccess) e = pack_all(u);
  if (e == hipSuccess) e = hipStreamSynchronize(stream);
  if (e != hipSuccess) {
    lmr_unet_destroy(u);
    return hip_fail(e);
  }
  *out = u;
  return LMR_OK;
}

lmr_status lmr_unet_set_params(lmr_unet* u, const float* params) {
  if (!u || !params) return LMR_EINVAL;
  const size_t bytes = static_cast<size_t>(param_count()) * 4;
  LMR_TRY(hipMemcpyAsync(u->params, params, bytes, hipMemcpyDeviceToDevice, u->stream));
  LMR_TRY(hipMemsetAsync(u->m1, 0, bytes, u->stream));
  LMR_TRY(hipMemsetAsync(u->m2, 0, bytes, u->stream));
  LMR_TRY(pack_all(u));
  u->step = 0;
  return LMR_OK;
}

lmr_status lmr_unet_get_params(lmr_unet* u, float* params) {
  if (!u || !params) return LMR_EINVAL;
  LMR_TRY(hipMemcpyAsync(params, u->params, static_cast<size_t>(param_count()) * 4,
                         hipMemcpyDeviceToDevice, u->stream));
  return LMR_OK;
}

lmr_status lmr_unet_get_grads(lmr_unet* u, float* grads) {
  if (!u || !grads) return LMR_EINVAL;
  LMR_TRY(hipMemcpyAsync(grads, u->grads, static_cast<size_t>(param_count()) * 4,
                         hipMemcpyDeviceToDevice, u->stream));
  return LMR_OK;
}

lmr_status lmr_unet_forward(lmr_unet* u, const void* F, const void* M, lmr_dtype img,
                            int pool, float* field) {
  if (!u || !F || !M || (img != LMR_F32 && img != LMR_BF16) || (pool != 0 && pool != 1))
    return LMR_EINVAL;
  hipStream_t s = u->stream;
  const int* d0 = u->dims[0];
  const int* d1 = u->dims[1];
  const int* d2 = u->dims[2];
  LMR_TRY(unet_input(F, M, img, d0[0], d0[1], d0[2], pool, u->x.p, s));
  LMR_TRY(conv_fwd(u, 0, u->x, 2, u->e1a, nullptr, 0));
  LMR_TRY(conv_fwd(u, 1, u->e1a, 16, u->c1.at(32), nullptr, 0));
  LMR_TRY(unet_pool2(u->c1.p + 32, 48, 16, d0[0], d0[1], d0[2], u->p1.p, 16, s));
  LMR_TRY(conv_fwd(u, 2, u->p1, 16, u->e2a, nullptr, 0));
  LMR_TRY(conv_fwd(u, 3, u->e2a, 32, u->c2.at(64), nullptr, 0));
  LMR_TRY(unet_pool2(u->c2.p + 64, 96, 32, d1[0], d1[1], d1[2], u->p2.p, 32, s));
  LMR_TRY(conv_fwd(u, 4, u->p2, 32, u->e3a, nullptr, 0));
  LMR_TRY(conv_fwd(u, 5, u->e3a, 64, u->c3.at(128), nullptr, 0));
  LMR_TRY(unet_pool2(u->c3.p + 128, 192, 64, d2[0], d2[1], d2[2], u->p3.p, 64, s));
  LMR_TRY(conv_fwd(u, 6, u->p3, 64, u->e4a, nullptr, 0));
  LMR_TRY(conv_fwd(u, 7, u->e4a, 128, u->e4, nullptr, 0));
  LMR_TRY(unet_up2(u->e4.p, 128, 128, d2[0], d2[1], d2[2], u->c3.p, 192, s));
  LMR_TRY(conv_fwd(u, 8, u->c3, 192, u->f3a, nullptr, 0));
  LMR_TRY(conv_fwd(u, 9, u->f3a, 64, u->f3, nullptr, 0));
  LMR_TRY(unet_up2(u->f3.p, 64, 64, d1[0], d1[1], d1[2], u->c2.p, 96, s));
  LMR_TRY(conv_fwd(u, 10, u->c2, 96, u->f2a, nullptr, 0));
  LMR_TRY(conv_fwd(u, 11, u->f2a, 32, u->f2, nullptr, 0));
  LMR_TRY(unet_up2(u->f2.p, 32, 32, d0[0], d0[1], d0[2], u->c1.p, 48, s));
  LMR_TRY(conv_fwd(u, 12, u->c1, 48, u->f1a, nullptr, 0));
  LMR_TRY(conv_fwd(u, 13, u->f1a, 16, u->f1, nullptr, 0));
  LMR_TRY(conv_fwd(u, 14, u->f1, 16, T{nullptr, 0}, u->yf, 4));
  if (field) LMR_TRY(unet_head_to_field(u->yf, 4, u->n[0], field, s));
  u->have_forward = true;
  return LMR_OK;
}

lmr_status lmr_unet_backward(lmr_unet* u, const float* target, double target_scale,
                             int accumulate, double* loss) {
  if (!u || !target || !isfinite(target_scale)) return LMR_EINVAL;
  if (!u->have_forward) return LMR_ESTATE;
  hipStream_t s = u->stream;
  const int* d0 = u->dims[0];
  const int* d1 = u->dims[1];
  const int* d2 = u->dims[2];
  const T none{nullptr, 0};
  const int acc = accumulate ? 1 : 0;
  LMR_TRY(unet_mse(u->yf, 4, target, static_cast<float>(target_scale), u->n[0], u->d_out.p,
                   4, u->mse_part, loss ? loss : u->loss_scratch, s));
  // level-0 decoder
  LMR_TRY(conv_bwd(u, 14, u->f1, u->d_out, u->d_f1, acc));
  LMR_TRY(mask(u, 0, u->d_f1, u->f1, 16));
  LMR_TRY(conv_bwd(u, 13, u->f1a, u->d_f1, u->d_f1a, acc));
  LMR_TRY(mask(u, 0, u->d_f1a, u->f1a, 16));
  LMR_TRY(conv_bwd(u, 12, u->c1, u->d_f1a, u->d_c1, acc));
  // d_c1 = [d up(f2) | d e1]; d e1 stays in place (channels 32..47)
  LMR_TRY(unet_up2_back(u->d_c1.p, 48, 32, d0[0], d0[1], d0[2], u->d_f2.p, 32, 0, s));
  LMR_TRY(mask(u, 1, u->d_f2, u->f2, 32));
  LMR_TRY(conv_bwd(u, 11, u->f2a, u->d_f2, u->d_f2a, acc));
  LMR_TRY(mask(u, 1, u->d_f2a, u->f2a, 32));
  LMR_TRY(conv_bwd(u, 10, u->c2, u->d_f2a, u->d_c2, acc));
  LMR_TRY(unet_up2_back(u->d_c2.p, 96, 64, d1[0], d1[1], d1[2], u->d_f3.p, 64, 0, s));
  LMR_TRY(mask(u, 2, u->d_f3, u->f3, 64));
  LMR_TRY(conv_bwd(u, 9, u->f3a, u->d_f3, u->d_f3a, acc));
  LMR_TRY(mask(u, 2, u->d_f3a, u->f3a, 64));
  LMR_TRY(conv_bwd(u, 8, u->c3, u->d_f3a, u->d_c3, acc));
  LMR_TRY(unet_up2_back(u->d_c3.p, 192, 128, d2[0], d2[1], d2[2], u->d_e4.p, 128, 0, s));
  // bottom level
  LMR_TRY(mask(u, 3, u->d_e4, u->e4, 128));
  LMR_TRY(conv_bwd(u, 7, u->e4a, u->d_e4, u->d_e4a, acc));
  LMR_TRY(mask(u, 3, u->d_e4a, u->e4a, 128));
  LMR_TRY(conv_bwd(u, 6, u->p3, u->d_e4a, u->d_p3, acc));
  // encoder: d e3 = skip part of d_c3 + pooling gradient
  LMR_TRY(unet_pool2_back(u->d_p3.p, 64, 64, d2[0], d2[1], d2[2], u->d_c3.p + 128, 192, 1, s));
  LMR_TRY(mask(u, 2, u->d_c3.at(128), u->c3.at(128), 64));
  LMR_TRY(conv_bwd(u, 5, u->e3a, u->d_c3.at(128), u->d_e3a, acc));
  LMR_TRY(mask(u, 2, u->d_e3a, u->e3a, 64));
  LMR_TRY(conv_bwd(u, 4, u->p2, u->d_e3a, u->d_p2, acc));
  LMR_TRY(unet_pool2_back(u->d_p2.p, 32, 32, d1[0], d1[1], d1[2], u->d_c2.p + 64, 96, 1, s));
  LMR_TRY(mask(u, 1, u->d_c2.at(64), u->c2.at(64), 32));
  LMR_TRY(conv_bwd(u, 3, u->e2a, u->d_c2.at(64), u->d_e2a, acc));
  LMR_TRY(mask(u, 1, u->d_e2a, u->e2a, 32));
  LMR_TRY(conv_bwd(u, 2, u->p1, u->d_e2a, u->d_p1, acc));
  LMR_TRY(unet_pool2_back(u->d_p1.p, 16, 16, d0[0], d0[1], d0[2], u->d_c1.p + 32, 48, 1, s));
  LMR_TRY(mask(u, 0, u->d_c1.at(32), u->c1.at(32), 16));
  LMR_TRY(conv_bwd(u, 1, u->e1a, u->d_c1.at(32), u->d_e1a, acc));
  LMR_TRY(mask(u, 0, u->d_e1a, u->e1a, 16));
  LMR_TRY(conv_bwd(u, 0, u->x, u->d_e1a, none, acc));
  return LMR_OK;
}

lmr_status lmr_unet_layer_probe(lmr_unet* u, int l, const uint16_t* x, int ldx, float* y,
                                int ldy, const uint16_t* dz, int ldz, uint16_t* dx, int lddx,
                                float* dW, float* db) {
  if (!u || l < 0 || l >= LMR_UNET_LAYERS || !x) return LMR_EINVAL;
  const LayerDef& L = kLayers[l];
  if (ldx < L.cin || ldx % 4 || (reinterpret_cast<uintptr_t>(x) % 8)) return LMR_EINVAL;
  if (y && ldy < L.cout) return LMR_EINVAL;
  if (dz && (ldz < L.cout || ldz % 4 || (reinterpret_cast<uintptr_t>(dz) % 8) || !dW || !db))
    return LMR_EINVAL;
  if (dx && (!dz || lddx < L.cin)) return LMR_EINVAL;
  const T xt{const_cast<uint16_t*>(x), ldx};
  if (y) LMR_TRY(conv_fwd(u, l, xt, L.cin, T{nullptr, 0}, y, ldy));
  if (dz) {
    const int* d = u->dims[L.level];
    LMR_TRY(unet_wgrad(x, ldx, L.cin, pad16(L.cin), dz, ldz, L.cout, pad16(L.cout), d[0],
                       d[1], d[2], u->part, u->partb, dW, db, 0, u->stream));
    if (dx) {
      ConvArgs a{};
      a.X = dz;
      a.ldx = ldz;
      a.cin_valid = L.cout;
      a.cin_p = pad16(L.cout);
      a.W = u->Wb[l];
      a.cout = L.cin;
      a.cout_p = pad16(L.cin);
      a.Y = dx;
      a.ldy = lddx;
      a.nz = d[0];
      a.ny = d[1];
      a.nx = d[2];
      LMR_TRY(unet_conv(a, u->stream));
    }
  }
  return LMR_OK;
}

lmr_status lmr_unet_adam(lmr_unet* u, double lr, double beta1, double beta2, double eps,
                         double grad_scale) {
  if (!u || !(lr > 0) || !(beta1 >= 0 && beta1 < 1) || !(beta2 >= 0 && beta2 < 1) ||
      !(eps > 0) || !isfinite(grad_scale))
    return LMR_EINVAL;
  ++u->step;
  const double c1 = 1.0 - pow(beta1, static_cast<double>(u->step));
  const double c2 = 1.0 - pow(beta2, static_cast<double>(u->step));
  LMR_TRY(unet_adam(u->params, u->m1, u->m2, u->grads, param_count(),
                    static_cast<float>(lr), static_cast<float>(beta1),
                    static_cast<float>(beta2), static_cast<float>(eps),
                    static_cast<float>(c1), static_cast<float>(c2),
                    static_cast<float>(grad_scale), u->stream));
  LMR_TRY(pack_all(u));
  return LMR_OK;
}

}  // extern "C"
