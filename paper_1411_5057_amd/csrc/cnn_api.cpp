// Host side of the warm-start network: parameters, Adam state, activation
// buffers, and the forward / training entry points of the C ABI.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "cnn_types.h"
#include "firls.h"

using namespace firls;
using namespace firls::cnn;

namespace firls {
int set_error(int code, const std::string& msg);
}

namespace {

#define CHK(expr)                                                                             \
  do {                                                                                        \
    hipError_t e_ = (expr);                                                                   \
    if (e_ != hipSuccess) return set_error(FIRLS_E_HIP, std::string(#expr) + ": " + hipGetErrorString(e_)); \
  } while (0)

constexpr int TILES_PER_WG = 16;

}  // namespace

struct firls_cnn {
  int n = 0, max_batch = 0;
  float* master = nullptr;
  float* m = nullptr;
  float* v = nullptr;
  float* grad = nullptr;
  unsigned short* wf = nullptr;
  unsigned short* wb = nullptr;
  float* bias = nullptr;
  LayerGeo geo[LAYERS]{};
  void* act[LAYERS] = {};   // act0 [B,n,n,16], act1..4 [B,n,n,32] (bf16)
  void* g5 = nullptr;       // [B,n,n,16] bf16
  void* gbuf[2] = {};       // [B,n,n,32] bf16
  void* x0 = nullptr;       // complex float [B,n,n]
  float* part = nullptr;
  float* partb = nullptr;
  int max_chunks = 0;
  double* lpart = nullptr;
  double* h_lpart = nullptr;
  int max_lblocks = 0;
  int64_t step = 0;
  bool have_params = false;
};

namespace {

void cnn_free(firls_cnn* c) {
  void* ptrs[] = {c->master, c->m, c->v, c->grad, c->wf, c->wb, c->bias, c->act[0], c->act[1], c->act[2],
                  c->act[3], c->act[4], c->g5, c->gbuf[0], c->gbuf[1], c->x0, c->part, c->partb, c->lpart};
  for (void* p : ptrs)
    if (p) (void)hipFree(p);
  if (c->h_lpart) (void)hipHostFree(c->h_lpart);
}

int pack(firls_cnn* c, hipStream_t st) {
  PackArgs a{};
  a.master = c->master;
  a.wf = c->wf;
  a.wb = c->wb;
  a.bias = c->bias;
  for (int l = 0; l < LAYERS; ++l) a.geo[l] = c->geo[l];
  CHK(launch_pack(a, st));
  return FIRLS_OK;
}

int forward(firls_cnn* c, hipStream_t st, int batch, const void* zf, void* x0) {
  InputArgs ia{zf, c->act[0], c->n, batch};
  CHK(launch_input(ia, st));
  for (int l = 0; l < LAYERS; ++l) {
    const LayerGeo& g = c->geo[l];
    ConvArgs a{};
    a.in = c->act[l];
    a.w = c->wf + g.wfoff;
    a.bias = c->bias + g.boff_pad;
    a.n = c->n;
    a.batch = batch;
    if (l < LAYERS - 1) {
      a.out = c->act[l + 1];
      CHK(launch_conv(g.cin_pad, g.cout_pad, 0, a, st));
    } else {
      a.zf = zf;
      a.out = x0;
      CHK(launch_conv(g.cin_pad, g.cout_pad, 1, a, st));
    }
  }
  return FIRLS_OK;
}

// Inference: the whole network in one kernel (activations stay on chip),
// one persistent workgroup per compute unit looping over the image blocks
// it streams down row by row.
int forward_fused(firls_cnn* c, hipStream_t st, int batch, const void* zf, void* x0) {
  static int cus = 0;
  if (!cus) {
    int dev = 0;
    CHK(hipGetDevice(&dev));
    CHK(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
  }
  NetArgs a{};
  a.zf = zf;
  a.x0 = x0;
  for (int l = 0; l < LAYERS; ++l) {
    a.w[l] = c->wf + c->geo[l].wfoff;
    a.b[l] = c->bias + c->geo[l].boff_pad;
  }
  a.n = c->n;
  a.batch = batch;
  CHK(launch_net_fwd(a, std::min(net_fwd_items(c->n, batch), cus), st));
  return FIRLS_OK;
}

// Forward, loss, backward; leaves the master-layout gradient in c->grad.
int gradients(firls_cnn* c, hipStream_t st, int batch, const void* zf, const void* label, double* loss) {
  int rc = forward(c, st, batch, zf, c->x0);
  if (rc) return rc;
  const size_t pix = (size_t)batch * c->n * c->n;
  const int lblocks = (int)((pix + 255) / 256);
  LossArgs la{c->x0, label, c->g5, c->lpart, c->n, batch};
  CHK(launch_loss(la, lblocks, st));
  const int tiles = (c->n / 32) * (c->n / 8) * batch;
  const int chunks = (tiles + TILES_PER_WG - 1) / TILES_PER_WG;
  const void* gy = c->g5;
  for (int l = LAYERS - 1; l >= 0; --l) {
    const LayerGeo& g = c->geo[l];
    WgradArgs wa{c->act[l], gy, c->part, c->partb, c->n, batch, TILES_PER_WG};
    CHK(launch_wgrad(g.cin_pad, g.cout_pad, wa, chunks, st));
    ReduceArgs ra{c->part, c->partb, c->grad + g.woff, g.cin, g.cout, g.cin_pad, g.cout_pad, chunks};
    CHK(launch_reduce(ra, st));
    if (l > 0) {
      // input gradient through the flipped, transposed weights, times the
      // ReLU mask of the layer input
      ConvArgs a{};
      a.in = gy;
      a.w = c->wb + g.wfoff;
      a.mask = c->act[l];
      a.n = c->n;
      a.batch = batch;
      void* out = c->gbuf[l & 1];
      a.out = out;
      CHK(launch_conv(g.cout_pad, g.cin_pad, 2, a, st));
      gy = out;
    }
  }
  CHK(hipMemcpyAsync(c->h_lpart, c->lpart, sizeof(double) * lblocks, hipMemcpyDeviceToHost, st));
  CHK(hipStreamSynchronize(st));
  double s = 0.0;
  for (int i = 0; i < lblocks; ++i) s += c->h_lpart[i];
  if (loss) *loss = s;
  return FIRLS_OK;
}

}  // namespace

namespace firls {

int cnn_forward(firls_cnn* c, hipStream_t st, int batch, const void* zf, void* x0) {
  return forward_fused(c, st, batch, zf, x0);
}
int cnn_image_side(const firls_cnn* c) { return c->n; }
int cnn_max_batch(const firls_cnn* c) { return c->max_batch; }
bool cnn_ready(const firls_cnn* c) { return c->have_params; }

}  // namespace firls

extern "C" {

int32_t firls_cnn_param_count(void) { return PARAMS; }

int firls_cnn_create(int32_t n, int32_t max_batch, firls_cnn** out) {
  if (!out) return set_error(FIRLS_E_INVALID, "out must be non-null");
  *out = nullptr;
  if (n <= 0 || n % 32 != 0) return set_error(FIRLS_E_UNSUPPORTED, "the network needs n to be a multiple of 32");
  if (max_batch <= 0) return set_error(FIRLS_E_INVALID, "max_batch must be positive");
  firls_cnn* c = new firls_cnn();
  c->n = n;
  c->max_batch = max_batch;
  int woff = 0, wf = 0, bp = 0;
  for (int l = 0; l < LAYERS; ++l) {
    LayerGeo& g = c->geo[l];
    g.cin = CIN[l];
    g.cout = COUT[l];
    g.cin_pad = CIN_PAD[l];
    g.cout_pad = COUT_PAD[l];
    g.woff = woff;
    g.boff = woff + 9 * g.cin * g.cout;
    woff = g.boff + g.cout;
    g.wfoff = wf;
    wf += 9 * g.cin_pad * g.cout_pad;
    g.boff_pad = bp;
    bp += g.cout_pad;
  }
  const size_t pix = (size_t)max_batch * n * n;
  const int tiles = (n / 32) * (n / 8) * max_batch;
  c->max_chunks = (tiles + TILES_PER_WG - 1) / TILES_PER_WG;
  c->max_lblocks = (int)((pix + 255) / 256);
  bool ok = hipMalloc(&c->master, PARAMS * 4) == hipSuccess && hipMalloc(&c->m, PARAMS * 4) == hipSuccess &&
            hipMalloc(&c->v, PARAMS * 4) == hipSuccess && hipMalloc(&c->grad, PARAMS * 4) == hipSuccess &&
            hipMalloc(&c->wf, wf * 2) == hipSuccess && hipMalloc(&c->wb, wf * 2) == hipSuccess &&
            hipMalloc(&c->bias, bp * 4) == hipSuccess && hipMalloc(&c->act[0], pix * 16 * 2) == hipSuccess &&
            hipMalloc(&c->g5, pix * 16 * 2) == hipSuccess && hipMalloc(&c->x0, pix * 8) == hipSuccess &&
            hipMalloc(&c->part, (size_t)c->max_chunks * 9 * 32 * 32 * 4) == hipSuccess &&
            hipMalloc(&c->partb, (size_t)c->max_chunks * 32 * 4) == hipSuccess &&
            hipMalloc(&c->lpart, (size_t)c->max_lblocks * 8) == hipSuccess &&
            hipHostMalloc(&c->h_lpart, (size_t)c->max_lblocks * 8, hipHostMallocDefault) == hipSuccess;
  for (int l = 1; l < LAYERS && ok; ++l) ok = hipMalloc(&c->act[l], pix * 32 * 2) == hipSuccess;
  for (int k = 0; k < 2 && ok; ++k) ok = hipMalloc(&c->gbuf[k], pix * 32 * 2) == hipSuccess;
  if (!ok) {
    (void)hipGetLastError();
    cnn_free(c);
    delete c;
    return set_error(FIRLS_E_NOMEM, "network buffer allocation failed");
  }
  *out = c;
  return FIRLS_OK;
}

int firls_cnn_destroy(firls_cnn* c) {
  if (!c) return FIRLS_OK;
  (void)hipDeviceSynchronize();
  cnn_free(c);
  delete c;
  return FIRLS_OK;
}

int firls_cnn_set_params(firls_cnn* c, const float* host) {
  if (!c || !host) return set_error(FIRLS_E_INVALID, "null argument");
  for (int i = 0; i < PARAMS; ++i)
    if (!std::isfinite(host[i])) return set_error(FIRLS_E_NONFINITE, "non-finite parameter");
  CHK(hipMemcpy(c->master, host, PARAMS * 4, hipMemcpyHostToDevice));
  CHK(hipMemset(c->m, 0, PARAMS * 4));
  CHK(hipMemset(c->v, 0, PARAMS * 4));
  c->step = 0;
  int rc = pack(c, nullptr);
  if (rc) return rc;
  CHK(hipDeviceSynchronize());
  c->have_params = true;
  return FIRLS_OK;
}

int firls_cnn_get_params(const firls_cnn* c, float* host) {
  if (!c || !host) return set_error(FIRLS_E_INVALID, "null argument");
  CHK(hipDeviceSynchronize());
  CHK(hipMemcpy(host, c->master, PARAMS * 4, hipMemcpyDeviceToHost));
  return FIRLS_OK;
}

int firls_cnn_forward(firls_cnn* c, void* stream, int32_t batch, const void* zf, void* x0) {
  if (!c || !zf || !x0) return set_error(FIRLS_E_INVALID, "null argument");
  if (batch <= 0 || batch > c->max_batch) return set_error(FIRLS_E_INVALID, "batch out of range");
  if (!c->have_params) return set_error(FIRLS_E_INVALID, "parameters not set");
  hipStream_t st = (hipStream_t)stream;
  int rc = forward_fused(c, st, batch, zf, x0);
  if (rc) return rc;
  CHK(hipStreamSynchronize(st));
  return FIRLS_OK;
}

int firls_cnn_gradients(firls_cnn* c, void* stream, int32_t batch, const void* zf, const void* label,
                        float* host_grad, double* loss) {
  if (!c || !zf || !label) return set_error(FIRLS_E_INVALID, "null argument");
  if (batch <= 0 || batch > c->max_batch) return set_error(FIRLS_E_INVALID, "batch out of range");
  if (!c->have_params) return set_error(FIRLS_E_INVALID, "parameters not set");
  hipStream_t st = (hipStream_t)stream;
  int rc = gradients(c, st, batch, zf, label, loss);
  if (rc) return rc;
  if (host_grad) {
    CHK(hipMemcpyAsync(host_grad, c->grad, PARAMS * 4, hipMemcpyDeviceToHost, st));
    CHK(hipStreamSynchronize(st));
  }
  return FIRLS_OK;
}

int firls_cnn_train_step(firls_cnn* c, void* stream, int32_t batch, const void* zf, const void* label, float lr,
                         double* loss) {
  if (!c || !zf || !label) return set_error(FIRLS_E_INVALID, "null argument");
  if (batch <= 0 || batch > c->max_batch) return set_error(FIRLS_E_INVALID, "batch out of range");
  if (!c->have_params) return set_error(FIRLS_E_INVALID, "parameters not set");
  if (!(lr > 0.f)) return set_error(FIRLS_E_INVALID, "lr must be positive");
  hipStream_t st = (hipStream_t)stream;
  int rc = gradients(c, st, batch, zf, label, loss);
  if (rc) return rc;
  if (loss && !std::isfinite(*loss)) return set_error(FIRLS_E_NONFINITE, "loss is not finite");
  c->step += 1;
  AdamArgs a{};
  a.master = c->master;
  a.m = c->m;
  a.v = c->v;
  a.grad = c->grad;
  a.lr = lr;
  a.b1 = 0.9f;
  a.b2 = 0.999f;
  a.eps = 1e-8f;
  a.bc1 = (float)(1.0 - std::pow(0.9, (double)c->step));
  a.bc2 = (float)(1.0 - std::pow(0.999, (double)c->step));
  a.count = PARAMS;
  CHK(launch_adam(a, st));
  rc = pack(c, st);
  if (rc) return rc;
  CHK(hipStreamSynchronize(st));
  return FIRLS_OK;
}

}  // extern "C"
