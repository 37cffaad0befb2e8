// Inference of the whole warm-start network in one kernel.
//
// The five 3x3 layers run back to back on a 16 x 16 output tile with the
// intermediate activations kept in LDS: layer l (1..5) produces a tile of
// side 16 + 2 (5 - l) around the output tile, so every layer reads only
// what the previous one left on chip, and the image is read once (zf) and
// written once (x0).  Outside the image every activation is zero, exactly
// the "same" zero padding of the layer-by-layer network.  bf16 activations
// and weights, FP32 accumulation on v_mfma_f32_16x16x32_bf16: lane l holds
// A[l%16][8(l/16) .. +7] (weights: out channel, 8 in channels), B[8(l/16)
// .. +7][l%16] (8 channels of one pixel) and D[4(l/16)+j][l%16] (four out
// channels of that pixel).  The first layer stacks its 9 taps x 2 channels
// into one K = 32 product.  Workgroups loop over tiles, so the weights are
// staged in LDS once per workgroup.
#include <hip/hip_runtime.h>

#include "cnn_types.h"

namespace firls {
namespace cnn {

namespace {

typedef __bf16 bf8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf2 __attribute__((ext_vector_type(2)));
typedef float f4 __attribute__((ext_vector_type(4)));
typedef float f2v __attribute__((ext_vector_type(2)));

constexpr int FT = 16;            // output tile side
constexpr int FPS = 40;           // LDS pixel stride (bf16) of 32-channel activations
constexpr int NW = 8;             // waves per workgroup
constexpr int UB = 2;             // 16-pixel blocks per wave and pass
constexpr int IN_W = FT + 10;     // input tile side (5-pixel halo)
constexpr int A_PIX = (FT + 8) * (FT + 8);   // layer-1 output tile (24 x 24)
constexpr int B_PIX = (FT + 6) * (FT + 6);   // layer-2 output tile (22 x 22)
constexpr int W32 = 9 * 32 * 32;              // bf16 weights of a 32 -> 32 layer
constexpr int W5 = 9 * 16 * 32;               // last layer (16 padded outputs)

constexpr size_t OFF_IN = 0;                                   // uint32 [IN_W^2]
constexpr size_t OFF_A = (OFF_IN + IN_W * IN_W * 4 + 15) / 16 * 16;
constexpr size_t OFF_B = OFF_A + (size_t)A_PIX * FPS * 2;
constexpr size_t OFF_W = OFF_B + (size_t)B_PIX * FPS * 2;     // 3 x W32 then W5
constexpr size_t LDS_BYTES = OFF_W + (size_t)(3 * W32 + W5) * 2;

// Weights sit in LDS as rows of 32 in-channels (four 16-byte chunks); chunk
// c of row r is stored at position c ^ ((r >> 1) & 3), so the eight rows a
// group of lanes reads at once fall into distinct banks.
__device__ __forceinline__ int wswz(int row, int chunk) { return row * 4 + (chunk ^ ((row >> 1) & 3)); }

// ReLU of a float through its bit pattern: every negative value (sign bit
// set) maps to +0 by a signed integer max
__device__ __forceinline__ float relu(float v) { return __int_as_float(max(__float_as_int(v), 0)); }

// ReLU (zero outside the image) of four consecutive channels (bias already
// in the accumulator) as bf16
__device__ __forceinline__ void put4(unsigned short* dst, const f4& v, bool inside) {
  const f2v lo = {relu(v[0]), relu(v[1])};
  const f2v hi = {relu(v[2]), relu(v[3])};
  uint2 pk;
  pk.x = inside ? __builtin_bit_cast(unsigned int, __builtin_convertvector(lo, bf2)) : 0u;
  pk.y = inside ? __builtin_bit_cast(unsigned int, __builtin_convertvector(hi, bf2)) : 0u;
  *reinterpret_cast<uint2*>(dst) = pk;
}

// (r, c) inside the n x n image
__device__ __forceinline__ bool in_image(int r, int c, int n) { return (unsigned)r < (unsigned)n && (unsigned)c < (unsigned)n; }

// One 32 -> 32 layer from an LDS tile of side WIN to one of side WIN - 2,
// whose top-left pixel is (gr0, gc0) in the image.
template <int WIN>
__device__ __forceinline__ void layer32(const unsigned short* in, unsigned short* out, const uint4* w,
                                        const float* bias, int gr0, int gc0, int n) {
  constexpr int WOUT = WIN - 2, NPIX = WOUT * WOUT, NBLK = (NPIX + 15) / 16;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, l16 = lane & 15, q = lane >> 4;
  bf8 wf[9][2];
#pragma unroll
  for (int t = 0; t < 9; ++t)
#pragma unroll
    for (int a = 0; a < 2; ++a) wf[t][a] = __builtin_bit_cast(bf8, w[wswz(t * 32 + a * 16 + l16, q)]);
  f4 bo[2];
#pragma unroll
  for (int a = 0; a < 2; ++a) bo[a] = *reinterpret_cast<const f4*>(bias + 16 * a + 4 * q);
  for (int blk = UB * wave; blk < NBLK; blk += UB * NW) {
    int p[UB], base[UB];
    bool inside[UB];
#pragma unroll
    for (int u = 0; u < UB; ++u) {
      p[u] = blk + u < NBLK ? (blk + u) * 16 + l16 : NPIX;
      const int pc = p[u] < NPIX ? p[u] : NPIX - 1;
      const int i = pc / WOUT, j = pc - i * WOUT;
      base[u] = (i * WIN + j) * FPS + 8 * q;
      inside[u] = in_image(gr0 + i, gc0 + j, n);
    }
    f4 acc[UB][2];
#pragma unroll
    for (int u = 0; u < UB; ++u)
#pragma unroll
      for (int a = 0; a < 2; ++a) acc[u][a] = bo[a];
#pragma unroll
    for (int t = 0; t < 9; ++t) {
      bf8 bop[UB];
#pragma unroll
      for (int u = 0; u < UB; ++u)
        bop[u] = *reinterpret_cast<const bf8*>(in + base[u] + ((t / 3) * WIN + t % 3) * FPS);
#pragma unroll
      for (int u = 0; u < UB; ++u)
#pragma unroll
        for (int a = 0; a < 2; ++a) acc[u][a] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(wf[t][a], bop[u], acc[u][a], 0, 0, 0);
    }
#pragma unroll
    for (int u = 0; u < UB; ++u) {
      if (p[u] < NPIX)
#pragma unroll
        for (int a = 0; a < 2; ++a) put4(out + p[u] * FPS + 16 * a + 4 * q, acc[u][a], inside[u]);
    }
  }
}

}  // namespace

__global__ __launch_bounds__(NW * 64) void k_net_fwd(NetArgs A) {
  extern __shared__ __align__(16) unsigned char smem[];
  unsigned int* xin = reinterpret_cast<unsigned int*>(smem + OFF_IN);
  unsigned short* bufA = reinterpret_cast<unsigned short*>(smem + OFF_A);
  unsigned short* bufB = reinterpret_cast<unsigned short*>(smem + OFF_B);
  uint4* wl = reinterpret_cast<uint4*>(smem + OFF_W);
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, l16 = lane & 15, q = lane >> 4;
  const int n = A.n, tpr = n / FT, tpi = tpr * tpr;
  const int ntiles = tpi * A.batch;

  // weights of layers 2..5 into LDS, once per workgroup (16 B per thread)
  for (int l = 0; l < 4; ++l) {
    const int rows = l < 3 ? 9 * 32 : 9 * 16;
    const uint4* src = static_cast<const uint4*>(A.w[l + 1]);
    for (int i = tid; i < rows * 4; i += NW * 64) wl[l * (W32 / 8) + wswz(i >> 2, i & 3)] = src[i];
  }
  // first layer: taps x channels stacked, k = 2 t + c < 18 (the rest zero);
  // lane group q holds the taps 4q .. 4q + 3, one input pixel (2 channels,
  // one uint32 of the input tile) each
  bf8 w1f[2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      const int k = 8 * q + e, t = k >> 1, c = k & 1;
      const unsigned short* w1 = static_cast<const unsigned short*>(A.w[0]);
      w1f[a][e] = __builtin_bit_cast(__bf16, k < 18 ? w1[(t * 32 + a * 16 + l16) * 16 + c] : (unsigned short)0);
    }
  int toff[4];
  bool tok[4];
#pragma unroll
  for (int m = 0; m < 4; ++m) {
    const int t = 4 * q + m;
    tok[m] = t < 9;
    toff[m] = tok[m] ? (t / 3) * IN_W + t % 3 : 0;
  }
  f4 b1[2];
#pragma unroll
  for (int a = 0; a < 2; ++a) b1[a] = *reinterpret_cast<const f4*>(A.b[0] + 16 * a + 4 * q);
  const f4 b5 = *reinterpret_cast<const f4*>(A.b[4] + 4 * q);

  // The input tile of the next tile is fetched into registers while the
  // current one is computed (IN_PER values per thread, zero outside).
  constexpr int IN_PER = (IN_W * IN_W + NW * 64 - 1) / (NW * 64);
  unsigned int pre[IN_PER];
  auto fetch = [&](int tile) {
    const int img = tile / tpi, tl = tile - img * tpi;
    const int r0 = (tl / tpr) * FT, c0 = (tl - (tl / tpr) * tpr) * FT;
    const float2* zf = static_cast<const float2*>(A.zf) + (size_t)img * n * n;
#pragma unroll
    for (int e = 0; e < IN_PER; ++e) {
      const int i = tid + e * NW * 64;
      const int gr = r0 - 5 + i / IN_W, gc = c0 - 5 + i % IN_W;
      unsigned int v = 0;
      if (i < IN_W * IN_W && gr >= 0 && gr < n && gc >= 0 && gc < n) {
        const float2 z = zf[(size_t)gr * n + gc];
        v = __builtin_bit_cast(unsigned int, __builtin_convertvector(f2v{z.x, z.y}, bf2));
      }
      pre[e] = v;
    }
  };
  if (blockIdx.x < ntiles) fetch(blockIdx.x);
  for (int tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
    const int img = tile / tpi, tl = tile - img * tpi;
    const int r0 = (tl / tpr) * FT, c0 = (tl - (tl / tpr) * tpr) * FT;
    const float2* zf = static_cast<const float2*>(A.zf) + (size_t)img * n * n;
    __syncthreads();   // the previous tile's last reads of the LDS are done
#pragma unroll
    for (int e = 0; e < IN_PER; ++e) {
      const int i = tid + e * NW * 64;
      if (i < IN_W * IN_W) xin[i] = pre[e];
    }
    if (tile + (int)gridDim.x < ntiles) fetch(tile + gridDim.x);
    __syncthreads();
    // layer 1: 2 -> 32 on the 24 x 24 tile at (r0 - 4, c0 - 4)
    {
      constexpr int WOUT = FT + 8, NPIX = WOUT * WOUT;
      for (int blk = wave; blk < NPIX / 16; blk += NW) {
        const int p = blk * 16 + l16, i = p / WOUT, j = p % WOUT;
        uint4 raw;
        raw.x = tok[0] ? xin[i * IN_W + j + toff[0]] : 0u;
        raw.y = tok[1] ? xin[i * IN_W + j + toff[1]] : 0u;
        raw.z = tok[2] ? xin[i * IN_W + j + toff[2]] : 0u;
        raw.w = tok[3] ? xin[i * IN_W + j + toff[3]] : 0u;
        const bf8 bop = __builtin_bit_cast(bf8, raw);
        const bool inside = in_image(r0 - 4 + i, c0 - 4 + j, n);
#pragma unroll
        for (int a = 0; a < 2; ++a)
          put4(bufA + p * FPS + 16 * a + 4 * q, __builtin_amdgcn_mfma_f32_16x16x32_bf16(w1f[a], bop, b1[a], 0, 0, 0),
               inside);
      }
    }
    __syncthreads();
    layer32<FT + 8>(bufA, bufB, wl, A.b[1], r0 - 3, c0 - 3, n);
    __syncthreads();
    layer32<FT + 6>(bufB, bufA, wl + W32 / 8, A.b[2], r0 - 2, c0 - 2, n);
    __syncthreads();
    layer32<FT + 4>(bufA, bufB, wl + 2 * (W32 / 8), A.b[3], r0 - 1, c0 - 1, n);
    __syncthreads();
    // layer 5: 32 -> 2 (outputs padded to 16) on the 16 x 16 tile, plus zf
    {
      constexpr int WIN = FT + 2;
      const uint4* w5 = wl + 3 * (W32 / 8);
      float2* x0 = static_cast<float2*>(A.x0) + (size_t)img * n * n;
      for (int blk = wave; blk < FT * FT / 16; blk += NW) {
        const int p = blk * 16 + l16, i = p / FT, j = p % FT;
        f4 acc = b5;
#pragma unroll
        for (int t = 0; t < 9; ++t) {
          const bf8 wv = __builtin_bit_cast(bf8, w5[wswz(t * 16 + l16, q)]);
          const bf8 bop = *reinterpret_cast<const bf8*>(bufB + ((i + t / 3) * WIN + j + t % 3) * FPS + 8 * q);
          acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(wv, bop, acc, 0, 0, 0);
        }
        if (q == 0) {
          const size_t g = (size_t)(r0 + i) * n + c0 + j;
          const float2 z = zf[g];
          x0[g] = make_float2(z.x + acc[0], z.y + acc[1]);
        }
      }
    }
  }
}

size_t net_fwd_lds_bytes() { return LDS_BYTES; }

hipError_t launch_net_fwd(const NetArgs& a, int grid, hipStream_t st) {
  static bool attr = false;
  if (!attr) {
    hipError_t e = hipFuncSetAttribute((const void*)k_net_fwd, hipFuncAttributeMaxDynamicSharedMemorySize, (int)LDS_BYTES);
    if (e != hipSuccess) return e;
    attr = true;
  }
  hipLaunchKernelGGL(k_net_fwd, dim3(grid), dim3(NW * 64), LDS_BYTES, st, a);
  return hipGetLastError();
}

}  // namespace cnn
}  // namespace firls
