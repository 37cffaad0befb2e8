// Argument structs of the warm-start network kernels (internal).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "firls_types.h"

namespace firls {
namespace cnn {

constexpr int LAYERS = 5;
constexpr int PARAMS = 28930;
// master-parameter layout per layer: W[dy][dx][cin][cout] then b[cout]
constexpr int CIN[LAYERS] = {2, 32, 32, 32, 32};
constexpr int COUT[LAYERS] = {32, 32, 32, 32, 2};
constexpr int CIN_PAD[LAYERS] = {16, 32, 32, 32, 32};
constexpr int COUT_PAD[LAYERS] = {32, 32, 32, 32, 16};

struct LayerGeo {
  int cin, cout, cin_pad, cout_pad;
  int woff, boff;       // offsets in the master array
  int wfoff;            // offset in the packed bf16 weight arrays
  int boff_pad;         // offset in the padded bias array
};

struct ConvArgs {
  const void* in;       // bf16 [B, n, n, CIN]
  const void* w;        // bf16 [9][COUT][CIN]
  const float* bias;    // [COUT]
  const void* mask;     // EPI_BWD: bf16 [B, n, n, COUT] activations (ReLU mask)
  const void* zf;       // EPI_RESID: complex float [B, n, n]
  void* out;
  int n, batch;
};

// Fused inference of the whole network (packed bf16 weights and padded FP32
// biases per layer, as the per-layer kernels use them).
struct NetArgs {
  const void* zf;       // complex float [B, n, n]
  void* x0;             // complex float [B, n, n] = zf + f(zf)
  const void* w[LAYERS];
  const float* b[LAYERS];
  int n, batch;
};

struct WgradArgs {
  const void* x;        // bf16 [B, n, n, CIN] layer input
  const void* gy;       // bf16 [B, n, n, COUT] output gradient
  float* part;          // [chunks][9][COUT][CIN]
  float* partb;         // [chunks][COUT]
  int n, batch, tiles_per_wg;
};

struct ReduceArgs {
  const float* part;
  const float* partb;
  float* grad;          // master layout of the layer (W then b)
  int cin, cout, cin_pad, cout_pad, chunks;
};

struct PackArgs {
  const float* master;
  unsigned short* wf;
  unsigned short* wb;
  float* bias;
  LayerGeo geo[LAYERS];
};

struct InputArgs {
  const void* zf;
  void* out;
  int n, batch;
};

struct LossArgs {
  const void* x0;
  const void* label;
  void* g;
  double* part;
  int n, batch;
};

struct AdamArgs {
  float* master;
  float* m;
  float* v;
  const float* grad;
  float lr, b1, b2, eps, bc1, bc2;
  int count;
};

struct ChooseArgs {
  const SliceState* st_zero;      // objective of the zero-filled starts
  const SliceState* st_learned;   // objective of the learned starts
  const void* zf;                 // complex float [S, n, n]
  const void* x0;                 // complex float [S, n, n]
  void* const* outs;              // per-slice destination x
  int n;
};

hipError_t launch_conv(int cin, int cout, int epi, const ConvArgs& a, hipStream_t st);
hipError_t launch_net_fwd(const NetArgs& a, int grid, hipStream_t st);
int net_fwd_items(int n, int batch);
hipError_t launch_wgrad(int cin, int cout, const WgradArgs& a, int chunks, hipStream_t st);
hipError_t launch_reduce(const ReduceArgs& a, hipStream_t st);
hipError_t launch_pack(const PackArgs& a, hipStream_t st);
hipError_t launch_input(const InputArgs& a, hipStream_t st);
hipError_t launch_loss(const LossArgs& a, int blocks, hipStream_t st);
hipError_t launch_adam(const AdamArgs& a, hipStream_t st);
hipError_t launch_choose(const ChooseArgs& a, int slices, hipStream_t st);

}  // namespace cnn
}  // namespace firls
