// Warm-start network kernels: 3x3 "same" convolutions on bf16 NHWC
// activations with bf16 MFMA (FP32 accumulate), the MSE loss gradient, the
// weight gradient (split over pixel chunks, reduced in a fixed order) and
// Adam on FP32 master weights.
//
// Network: x0 = zf + f(zf), f = conv(2->32) ReLU conv(32->32) ReLU
// conv(32->32) ReLU conv(32->32) ReLU conv(32->2) on [Re zf, Im zf].
// Channel counts are padded to multiples of 16 on the device (2 -> 16).
//
// Convolution as a product per tap t = (dy, dx):
//   Y[p][o] = b[o] + sum_t sum_i W_t[o][i] X[p + t - (1,1)][i],
// computed as D[o][p] = A[o][i] B[i][p] with the 16x16x16 bf16 MFMA
// (A = W_t, B = the input patch), so a lane's four results are four
// consecutive output channels of one pixel.  The input gradient is the
// same product with W'_t[i][o] = W_{flip t}[o][i] on the output gradient.
#include <hip/hip_runtime.h>

#include "cnn_types.h"
#include "firls_dev.h"

namespace firls {
namespace cnn {

typedef short s4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ unsigned short f2bf(float f) {
  // round to nearest even (finite values)
  unsigned int u = __float_as_uint(f);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return (unsigned short)(u >> 16);
}
__device__ __forceinline__ float bf2f(unsigned short h) { return __uint_as_float(((unsigned int)h) << 16); }

constexpr int TH = 8, TW = 32;              // output tile of a workgroup
constexpr int HH = TH + 2, HW = TW + 2;     // input tile with halo

enum Epi : int { EPI_RELU = 0, EPI_RESID = 1, EPI_BWD = 2 };

// One 3x3 convolution over a batch of n x n images.
//   in   : bf16 [B, n, n, CIN]
//   w    : bf16 [9][COUT][CIN]   (tap-major, then output channel)
//   EPI_RELU : out bf16 [B,n,n,COUT] = bf16(max(Y + bias, 0))
//   EPI_RESID: out complex float [B,n,n] = zf + (Y[0] + b[0], Y[1] + b[1])
//   EPI_BWD  : out bf16 [B,n,n,COUT] = bf16(Y * (mask_act > 0)) (no bias)
template <int CIN, int COUT, int EPI>
__global__ __launch_bounds__(256) void k_conv(ConvArgs A) {
  constexpr int PS = CIN + 8;               // LDS pixel stride (bf16), breaks bank aliasing
  constexpr int WS = CIN + 8;               // LDS weight row stride
  __shared__ __align__(16) unsigned short xs[HH * HW * PS];
  __shared__ __align__(16) unsigned short ws[9 * COUT * WS];
  const int n = A.n;
  const int tiles_x = n / TW;
  const int tx = blockIdx.x % tiles_x, ty = blockIdx.x / tiles_x;
  const int img = blockIdx.y;
  const int r0 = ty * TH, c0 = tx * TW;
  const unsigned short* in = static_cast<const unsigned short*>(A.in) + (size_t)img * n * n * CIN;
  const unsigned short* w = static_cast<const unsigned short*>(A.w);
  // input tile with zero halo: 8 channels (16 B) per load
  constexpr int CH8 = CIN / 8;
  for (int i = threadIdx.x; i < HH * HW * CH8; i += 256) {
    const int pix = i / CH8, c8 = i - pix * CH8;
    const int hr = pix / HW, hc = pix - hr * HW;
    const int gr = r0 + hr - 1, gc = c0 + hc - 1;
    uint4 v = make_uint4(0, 0, 0, 0);
    if (gr >= 0 && gr < n && gc >= 0 && gc < n)
      v = *reinterpret_cast<const uint4*>(in + ((size_t)gr * n + gc) * CIN + c8 * 8);
    *reinterpret_cast<uint4*>(xs + pix * PS + c8 * 8) = v;
  }
  for (int i = threadIdx.x; i < 9 * COUT * CH8; i += 256) {
    const int row = i / CH8, c8 = i - row * CH8;
    *reinterpret_cast<uint4*>(ws + row * WS + c8 * 8) = *reinterpret_cast<const uint4*>(w + row * CIN + c8 * 8);
  }
  __syncthreads();

  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int l16 = lane & 15, q = lane >> 4;
  constexpr int MB = COUT / 16;            // output-channel blocks
  constexpr int NB = 4;                    // pixel blocks per wave (2 rows x 32)
  f4 acc[MB][NB];
#pragma unroll
  for (int a = 0; a < MB; ++a)
#pragma unroll
    for (int b = 0; b < NB; ++b) acc[a][b] = f4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
  for (int t = 0; t < 9; ++t) {
    const int dy = t / 3, dx = t - dy * 3;
#pragma unroll
    for (int cb = 0; cb < CIN / 16; ++cb) {
      s4 af[MB], bfr[NB];
#pragma unroll
      for (int a = 0; a < MB; ++a)
        af[a] = *reinterpret_cast<const s4*>(ws + (t * COUT + a * 16 + l16) * WS + cb * 16 + q * 4);
#pragma unroll
      for (int b = 0; b < NB; ++b) {
        const int orow = wave * 2 + (b >> 1), ocol = (b & 1) * 16 + l16;
        const int hp = (orow + dy) * HW + ocol + dx;
        bfr[b] = *reinterpret_cast<const s4*>(xs + hp * PS + cb * 16 + q * 4);
      }
#pragma unroll
      for (int a = 0; a < MB; ++a)
#pragma unroll
        for (int b = 0; b < NB; ++b) acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(af[a], bfr[b], acc[a][b], 0, 0, 0);
    }
  }
  // epilogue: lane holds channels a*16 + 4q .. +3 of pixel (b-block, l16)
#pragma unroll
  for (int b = 0; b < NB; ++b) {
    const int orow = r0 + wave * 2 + (b >> 1), ocol = c0 + (b & 1) * 16 + l16;
    const size_t pix = (size_t)img * n * n + (size_t)orow * n + ocol;
#pragma unroll
    for (int a = 0; a < MB; ++a) {
      const int o = a * 16 + q * 4;
      if constexpr (EPI == EPI_RESID) {
        if (a == 0 && q == 0) {
          const float2 z = static_cast<const float2*>(A.zf)[pix];
          float2 r;
          r.x = z.x + acc[a][b][0] + A.bias[0];
          r.y = z.y + acc[a][b][1] + A.bias[1];
          static_cast<float2*>(A.out)[pix] = r;
        }
      } else {
        unsigned short h[4];
        if constexpr (EPI == EPI_RELU) {
#pragma unroll
          for (int j = 0; j < 4; ++j) h[j] = f2bf(fmaxf(acc[a][b][j] + A.bias[o + j], 0.f));
        } else {
          const unsigned short* m = static_cast<const unsigned short*>(A.mask) + pix * COUT + o;
#pragma unroll
          for (int j = 0; j < 4; ++j) h[j] = bf2f(m[j]) > 0.f ? f2bf(acc[a][b][j]) : (unsigned short)0;
        }
        uint2 pk;
        pk.x = (unsigned int)h[0] | ((unsigned int)h[1] << 16);
        pk.y = (unsigned int)h[2] | ((unsigned int)h[3] << 16);
        *reinterpret_cast<uint2*>(static_cast<unsigned short*>(A.out) + pix * COUT + o) = pk;
      }
    }
  }
}

// Weight gradient partials: for each workgroup's pixel chunk,
//   dW_t[o][i] = sum_p dY[p][o] X[p + t - (1,1)][i],  db[o] = sum_p dY[p][o],
// as D[o][i] = A[o][p] B[p][i] (K = pixels).  Tiles are staged channel-major
// in LDS so a lane's four K values (four consecutive pixels) are adjacent.
// Three waves, three taps each.  Output: part[chunk][9][COUT][CIN] and
// partb[chunk][COUT] (FP32).
template <int CIN, int COUT>
__global__ __launch_bounds__(192) void k_wgrad(WgradArgs A) {
  constexpr int TP = TH * TW;               // 256 output pixels per tile
  constexpr int XP = HH * HW + 4;           // halo pixels (+ pad)
  constexpr int YP = TP + 4;
  __shared__ __align__(16) unsigned short xt[CIN * XP];
  __shared__ __align__(16) unsigned short yt[COUT * YP];
  const int n = A.n;
  const int tiles_x = n / TW, tiles_img = tiles_x * (n / TH);
  const int total = tiles_img * A.batch;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int l16 = lane & 15, q = lane >> 4;
  constexpr int MB = COUT / 16, NBI = CIN / 16;
  f4 acc[3][MB][NBI];
#pragma unroll
  for (int u = 0; u < 3; ++u)
#pragma unroll
    for (int a = 0; a < MB; ++a)
#pragma unroll
      for (int b = 0; b < NBI; ++b) acc[u][a][b] = f4{0.f, 0.f, 0.f, 0.f};
  float bacc = 0.f;   // db partial: thread owns channel threadIdx.x % COUT rows
  const int t_begin = blockIdx.x * A.tiles_per_wg;
  const int t_end = min(total, t_begin + A.tiles_per_wg);
  for (int tile = t_begin; tile < t_end; ++tile) {
    const int img = tile / tiles_img, tl = tile - img * tiles_img;
    const int ty = tl / tiles_x, tx = tl - ty * tiles_x;
    const int r0 = ty * TH, c0 = tx * TW;
    const unsigned short* X = static_cast<const unsigned short*>(A.x) + (size_t)img * n * n * CIN;
    const unsigned short* G = static_cast<const unsigned short*>(A.gy) + (size_t)img * n * n * COUT;
    __syncthreads();
    for (int i = threadIdx.x; i < HH * HW * (CIN / 8); i += 192) {
      const int pix = i / (CIN / 8), c8 = i - pix * (CIN / 8);
      const int hr = pix / HW, hc = pix - hr * HW;
      const int gr = r0 + hr - 1, gc = c0 + hc - 1;
      uint4 v = make_uint4(0, 0, 0, 0);
      if (gr >= 0 && gr < n && gc >= 0 && gc < n)
        v = *reinterpret_cast<const uint4*>(X + ((size_t)gr * n + gc) * CIN + c8 * 8);
      const unsigned short* e = reinterpret_cast<const unsigned short*>(&v);
#pragma unroll
      for (int j = 0; j < 8; ++j) xt[(c8 * 8 + j) * XP + pix] = e[j];
    }
    for (int i = threadIdx.x; i < TP * (COUT / 8); i += 192) {
      const int pix = i / (COUT / 8), c8 = i - pix * (COUT / 8);
      const int rr = pix / TW, cc = pix - rr * TW;
      const uint4 v = *reinterpret_cast<const uint4*>(G + ((size_t)(r0 + rr) * n + c0 + cc) * COUT + c8 * 8);
      const unsigned short* e = reinterpret_cast<const unsigned short*>(&v);
#pragma unroll
      for (int j = 0; j < 8; ++j) yt[(c8 * 8 + j) * YP + pix] = e[j];
    }
    __syncthreads();
    if (threadIdx.x < COUT) {
      float s = 0.f;
      for (int p = 0; p < TP; ++p) s += bf2f(yt[threadIdx.x * YP + p]);
      bacc += s;
    }
#pragma unroll
    for (int kb = 0; kb < TP / 16; ++kb) {
      const int rr = kb >> 1, cc = (kb & 1) * 16;       // 16 pixels of one row
      s4 af[MB];
#pragma unroll
      for (int a = 0; a < MB; ++a)
        af[a] = *reinterpret_cast<const s4*>(yt + (a * 16 + l16) * YP + rr * TW + cc + q * 4);
#pragma unroll
      for (int u = 0; u < 3; ++u) {
        const int t = wave * 3 + u, dy = t / 3, dx = t - dy * 3;
        const int hp = (rr + dy) * HW + cc + dx + q * 4;
#pragma unroll
        for (int b = 0; b < NBI; ++b) {
          const unsigned short* src = xt + (b * 16 + l16) * XP + hp;
          s4 bv;
          bv[0] = (short)src[0];
          bv[1] = (short)src[1];
          bv[2] = (short)src[2];
          bv[3] = (short)src[3];
#pragma unroll
          for (int a = 0; a < MB; ++a) acc[u][a][b] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(af[a], bv, acc[u][a][b], 0, 0, 0);
        }
      }
    }
  }
  // D[o][i]: lane holds o = a*16 + 4q + j, i = b*16 + l16
  float* part = A.part + (size_t)blockIdx.x * 9 * COUT * CIN;
#pragma unroll
  for (int u = 0; u < 3; ++u) {
    const int t = wave * 3 + u;
#pragma unroll
    for (int a = 0; a < MB; ++a)
#pragma unroll
      for (int b = 0; b < NBI; ++b)
#pragma unroll
        for (int j = 0; j < 4; ++j) part[(t * COUT + a * 16 + q * 4 + j) * CIN + b * 16 + l16] = acc[u][a][b][j];
  }
  if (threadIdx.x < COUT) A.partb[(size_t)blockIdx.x * COUT + threadIdx.x] = bacc;
}

// Sum the chunk partials in chunk order (FP64) into the FP32 master-layout
// gradient of one layer: gW[dy][dx][i][o] (i < cin, o < cout), then gb[o].
__global__ __launch_bounds__(256) void k_wgrad_reduce(ReduceArgs A) {
  const int nw = 9 * A.cin * A.cout;
  const int e = blockIdx.x * 256 + threadIdx.x;
  if (e < nw) {
    const int o = e % A.cout, i = (e / A.cout) % A.cin, t = e / (A.cout * A.cin);
    const size_t src = ((size_t)t * A.cout_pad + o) * A.cin_pad + i;
    const size_t stride = (size_t)9 * A.cout_pad * A.cin_pad;
    double s = 0.0;
    for (int c = 0; c < A.chunks; ++c) s += (double)A.part[c * stride + src];
    A.grad[e] = (float)s;
  } else if (e < nw + A.cout) {
    const int o = e - nw;
    double s = 0.0;
    for (int c = 0; c < A.chunks; ++c) s += (double)A.partb[(size_t)c * A.cout_pad + o];
    A.grad[e] = (float)s;
  }
}

// Master FP32 parameters -> padded bf16 forward weights [9][COUT][CIN] and
// backward weights [9][CIN][COUT] (taps flipped), all five layers.
__global__ __launch_bounds__(256) void k_pack(PackArgs A) {
  const int layer = blockIdx.y;
  const LayerGeo g = A.geo[layer];
  const int tot = 9 * g.cout_pad * g.cin_pad;
  for (int e = blockIdx.x * 256 + threadIdx.x; e < tot; e += gridDim.x * 256) {
    // forward layout
    {
      const int i = e % g.cin_pad, o = (e / g.cin_pad) % g.cout_pad, t = e / (g.cin_pad * g.cout_pad);
      float v = 0.f;
      if (i < g.cin && o < g.cout) v = A.master[g.woff + (t * g.cin + i) * g.cout + o];
      A.wf[g.wfoff + e] = f2bf(v);
    }
    // backward-data layout: W'[t'][i][o] = W[8 - t'][o][i]
    {
      const int o = e % g.cout_pad, i = (e / g.cout_pad) % g.cin_pad, tp = e / (g.cin_pad * g.cout_pad);
      const int t = 8 - tp;
      float v = 0.f;
      if (i < g.cin && o < g.cout) v = A.master[g.woff + (t * g.cin + i) * g.cout + o];
      A.wb[g.wfoff + e] = f2bf(v);
    }
  }
  if (blockIdx.x == 0)
    for (int o = threadIdx.x; o < g.cout_pad; o += 256) A.bias[g.boff_pad + o] = o < g.cout ? A.master[g.boff + o] : 0.f;
}

// Complex zero-filled images -> bf16 [B, n, n, 16] (channels 0, 1 = Re, Im).
__global__ __launch_bounds__(256) void k_input(InputArgs A) {
  const size_t tot = (size_t)A.batch * A.n * A.n;
  const size_t p = (size_t)blockIdx.x * 256 + threadIdx.x;
  if (p >= tot) return;
  const float2 z = static_cast<const float2*>(A.zf)[p];
  uint4 v0 = make_uint4((unsigned int)f2bf(z.x) | ((unsigned int)f2bf(z.y) << 16), 0, 0, 0);
  uint4* o = reinterpret_cast<uint4*>(static_cast<unsigned short*>(A.out) + p * 16);
  o[0] = v0;
  o[1] = make_uint4(0, 0, 0, 0);
}

// Loss 1/(2 B n^2) sum |x0 - label|^2 over the two channels (mean over
// pixels and channels) and its gradient 2 (x0 - label) / count as bf16
// [B, n, n, 16]; one FP64 partial per workgroup.
__global__ __launch_bounds__(256) void k_loss(LossArgs A) {
  __shared__ double red[4];
  const size_t tot = (size_t)A.batch * A.n * A.n;
  const double count = 2.0 * (double)tot;
  const size_t p = (size_t)blockIdx.x * 256 + threadIdx.x;
  double s = 0.0;
  if (p < tot) {
    const float2 x = static_cast<const float2*>(A.x0)[p];
    const float2 l = static_cast<const float2*>(A.label)[p];
    const double dr = (double)x.x - (double)l.x, di = (double)x.y - (double)l.y;
    s = dr * dr + di * di;
    const float gr = (float)(2.0 * dr / count), gi = (float)(2.0 * di / count);
    uint4* o = reinterpret_cast<uint4*>(static_cast<unsigned short*>(A.g) + p * 16);
    o[0] = make_uint4((unsigned int)f2bf(gr) | ((unsigned int)f2bf(gi) << 16), 0, 0, 0);
    o[1] = make_uint4(0, 0, 0, 0);
  }
  s = block_sum(s, red);
  if (threadIdx.x == 0) A.part[blockIdx.x] = s / count;
}

// Adam on the FP32 master parameters (bias-corrected).
__global__ __launch_bounds__(256) void k_adam(AdamArgs A) {
  const int e = blockIdx.x * 256 + threadIdx.x;
  if (e >= A.count) return;
  const float g = A.grad[e];
  const float m = A.b1 * A.m[e] + (1.f - A.b1) * g;
  const float v = A.b2 * A.v[e] + (1.f - A.b2) * g * g;
  A.m[e] = m;
  A.v[e] = v;
  const float mh = m / A.bc1, vh = v / A.bc2;
  A.master[e] -= A.lr * mh / (sqrtf(vh) + A.eps);
}

// Keep the learned start only where its objective is not worse:
// x = (F_eps(x0) <= F_eps(zf)) ? x0 : zf, per slice.
__global__ __launch_bounds__(256) void k_choose(ChooseArgs A) {
  const int s = blockIdx.y;
  const bool keep = A.st_learned[s].Fe <= A.st_zero[s].Fe;
  const size_t np = (size_t)A.n * A.n;
  const size_t p = (size_t)blockIdx.x * 256 + threadIdx.x;
  if (p >= np) return;
  const float2* src = static_cast<const float2*>(keep ? A.x0 : A.zf) + s * np;
  static_cast<float2*>(A.outs[s])[p] = src[p];
}

// ---------------------------------------------------------------------------
template <int CIN, int COUT, int EPI>
hipError_t conv_launch(const ConvArgs& a, hipStream_t st) {
  dim3 g((a.n / TW) * (a.n / TH), a.batch);
  hipLaunchKernelGGL((k_conv<CIN, COUT, EPI>), g, dim3(256), 0, st, a);
  return hipGetLastError();
}

hipError_t launch_conv(int cin, int cout, int epi, const ConvArgs& a, hipStream_t st) {
#define C(CI, CO, E) if (cin == CI && cout == CO && epi == E) return conv_launch<CI, CO, E>(a, st);
  C(16, 32, EPI_RELU) C(32, 32, EPI_RELU) C(32, 16, EPI_RESID)
  C(16, 32, EPI_BWD) C(32, 32, EPI_BWD)
#undef C
  return hipErrorInvalidValue;
}

template <int CIN, int COUT>
hipError_t wgrad_launch(const WgradArgs& a, int chunks, hipStream_t st) {
  hipLaunchKernelGGL((k_wgrad<CIN, COUT>), dim3(chunks), dim3(192), 0, st, a);
  return hipGetLastError();
}

hipError_t launch_wgrad(int cin, int cout, const WgradArgs& a, int chunks, hipStream_t st) {
  if (cin == 16 && cout == 32) return wgrad_launch<16, 32>(a, chunks, st);
  if (cin == 32 && cout == 32) return wgrad_launch<32, 32>(a, chunks, st);
  if (cin == 32 && cout == 16) return wgrad_launch<32, 16>(a, chunks, st);
  return hipErrorInvalidValue;
}

hipError_t launch_reduce(const ReduceArgs& a, hipStream_t st) {
  const int tot = 9 * a.cin * a.cout + a.cout;
  hipLaunchKernelGGL(k_wgrad_reduce, dim3((tot + 255) / 256), dim3(256), 0, st, a);
  return hipGetLastError();
}

hipError_t launch_pack(const PackArgs& a, hipStream_t st) {
  hipLaunchKernelGGL(k_pack, dim3(8, 5), dim3(256), 0, st, a);
  return hipGetLastError();
}

hipError_t launch_input(const InputArgs& a, hipStream_t st) {
  const size_t tot = (size_t)a.batch * a.n * a.n;
  hipLaunchKernelGGL(k_input, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, st, a);
  return hipGetLastError();
}

hipError_t launch_loss(const LossArgs& a, int blocks, hipStream_t st) {
  hipLaunchKernelGGL(k_loss, dim3(blocks), dim3(256), 0, st, a);
  return hipGetLastError();
}

hipError_t launch_adam(const AdamArgs& a, hipStream_t st) {
  hipLaunchKernelGGL(k_adam, dim3((a.count + 255) / 256), dim3(256), 0, st, a);
  return hipGetLastError();
}

hipError_t launch_choose(const ChooseArgs& a, int slices, hipStream_t st) {
  const size_t np = (size_t)a.n * a.n;
  hipLaunchKernelGGL(k_choose, dim3((unsigned)((np + 255) / 256), slices), dim3(256), 0, st, a);
  return hipGetLastError();
}

}  // namespace cnn
}  // namespace firls
