// Inference of the whole warm-start network in one kernel, streamed down
// the image row by row.
//
// A workgroup owns an output block of BH rows by SW columns of one image
// (BH, SW in {32, 64, 128}, the largest that divide n) and walks it from top
// to bottom.  Every layer keeps the last four rows it produced in an LDS
// ring buffer: at step t layer l (1..5) computes row R0 - 4 + t - 2 (l - 1)
// of its output from rows r - 1 .. r + 1 of the layer below, written at the
// three steps before, while that layer writes its fourth ring row, so one
// barrier per step orders everything.  Rows are computed once (no vertical
// recomputation between neighbouring tiles); only 5 columns on each side are
// recomputed (layer widths SW + 8, +6, +4, +2, SW).  Outside the image every
// activation is zero, the "same" zero padding of the layer-by-layer network.
//
// Sixteen waves: four per 32 -> 32 layer (2, 3, 4) and four for layers 1
// and 5 (and the input rows).  Each wave keeps its layers' weights in
// registers for the whole kernel and takes every fourth 16-pixel block of
// its layer's row.  Waves w and w + 4k share a SIMD (w mod 4), so each SIMD
// runs one wave of every role, with the block offsets rotated by role so the
// rows' odd ninth blocks land on different SIMDs.  Each role runs its own
// step loop (same barrier count), so registers are allocated per role.
// bf16 activations and weights, FP32 accumulation on
// v_mfma_f32_16x16x32_bf16: lane (q = l / 16, m = l % 16) holds
// A[m][8q .. 8q + 7] (weights: output channel m of the block, 8 input
// channels), B[8q .. 8q + 7][m] (8 input channels of pixel m) and
// D[4q + j][m] (four output channels of pixel m).
//
// An activation pixel is 64 bytes: 32 channels in the order
// 16a + 4q + j -> 8q + 4a + j, so lane (q, m) of a layer's output writes its
// two blocks' four channels (a = 0, 1) as one 16-byte chunk, and chunk q of
// pixel p sits at chunk position q ^ ((p >> 1) & 3): the eight lanes that
// read or write at once (eight consecutive pixels, one chunk each) cover all
// eight 16-byte bank groups of a 128-byte bank row.  The weights are loaded
// in the same input-channel order.
#include <hip/hip_runtime.h>

#include "cnn_types.h"

namespace firls {
namespace cnn {

namespace {

typedef __bf16 bf8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf2 __attribute__((ext_vector_type(2)));
typedef float f4 __attribute__((ext_vector_type(4)));
typedef float f2v __attribute__((ext_vector_type(2)));

constexpr int SNW = 16;                 // waves per workgroup
constexpr int SNT = SNW * 64;
constexpr int WPL = 4;                  // waves per layer role
constexpr int RING = 4;                 // rows kept per layer
constexpr int HALO = 5;                 // columns recomputed on each side of the strip (input)
constexpr int MAXSW = 128;              // widest strip
constexpr int MAXB = (MAXSW + 2 * 4 + 15) / 16;   // 16-pixel blocks of the widest layer row (9)
constexpr int ROWPX = MAXB * 16;        // pixel slots of a ring row (144)
constexpr int PXB = 64;                 // bytes of a 32-channel bf16 pixel
constexpr size_t OFF_IN = 0;                                   // input ring: RING x ROWPX x (re, im) bf16
constexpr size_t OFF_ACT = (size_t)RING * ROWPX * 4;            // layer l ring: OFF_ACT + (l - 1) * ACT_RING
constexpr size_t ACT_RING = (size_t)RING * ROWPX * PXB;
// A row's last block reads up to two pixels past the row's ROWPX slots (its
// lanes beyond the row width are discarded); the tail keeps those reads of
// the last ring row inside the allocation.
constexpr size_t LDS_TAIL = 2 * PXB;
constexpr size_t LDS_BYTES = OFF_ACT + 4 * ACT_RING + LDS_TAIL;

// ring slot of row r (r > -64)
__device__ __forceinline__ int slot(int r) { return (r + 64) & (RING - 1); }

// byte offset of 16-byte chunk q of pixel p within a ring row
__device__ __forceinline__ int chunk_off(int p, int q) { return p * PXB + ((q ^ ((p >> 1) & 3)) << 4); }

// ReLU of a float through its bit pattern: every negative value (sign bit
// set) maps to +0 by a signed integer max
__device__ __forceinline__ float relu(float v) { return __int_as_float(max(__float_as_int(v), 0)); }

__device__ __forceinline__ unsigned int pack2(float a, float b) {
  return __builtin_bit_cast(unsigned int, __builtin_convertvector(f2v{a, b}, bf2));
}

// (r, c) inside the n x n image
__device__ __forceinline__ bool in_image(int r, int c, int n) { return (unsigned)r < (unsigned)n && (unsigned)c < (unsigned)n; }

// A-operand fragment of a 32 -> COUT_PAD layer: output channel o, input
// channels 16 (e / 4) + 4 q + e % 4 for e = 0..7 (packed [9][COUT_PAD][32])
__device__ __forceinline__ bf8 load_w32(const unsigned short* w, int cout_pad, int t, int o, int q) {
  const unsigned short* row = w + ((size_t)t * cout_pad + o) * 32;
  const uint2 lo = *reinterpret_cast<const uint2*>(row + 4 * q);
  const uint2 hi = *reinterpret_cast<const uint2*>(row + 16 + 4 * q);
  return __builtin_bit_cast(bf8, make_uint4(lo.x, lo.y, hi.x, hi.y));
}

// Lane offsets of tap column dx (0..2) within a 16-pixel block: pixel
// 16 b + m + dx of a ring row sits at 1024 b + sw[dx] (the swizzle depends
// only on the pixel's position in its block), so a block's nine reads are a
// row offset plus one of three per-lane offsets plus a constant.
struct TapOffsets {
  int sw[3];
  __device__ __forceinline__ TapOffsets(int m, int q) {
#pragma unroll
    for (int dx = 0; dx < 3; ++dx) sw[dx] = chunk_off(m + dx, q);
  }
};

// One row of a 32 -> 32 layer (2, 3 or 4): blocks b0, b0 + WPL, ... of the
// row's nblk blocks, one at a time (both output blocks of 16 channels share
// each activation read; the next tap's read is issued before this tap's
// products).  in_row[dy] is the LDS offset of input row r - 1 + dy.
__device__ __forceinline__ void conv_row(const unsigned char* lds, const int (&in_row)[3], const bf8 (&wf)[9][2],
                                         const f4 (&bo)[2], const TapOffsets& to, int b0, int nblk, int width, int m,
                                         unsigned char* out_row, int gr, int gc0, int n, bool row_inside) {
#pragma unroll
  for (int u = 0; u < 3; ++u) {
    const int b = b0 + u * WPL;
    if (b >= nblk) break;
    const int j = b * 16 + m;
    const unsigned char* blk = lds + b * 16 * PXB;
    f4 acc[2] = {bo[0], bo[1]};
    if (row_inside) {
      bf8 cur = *reinterpret_cast<const bf8*>(blk + in_row[0] + to.sw[0]);
#pragma unroll
      for (int t = 0; t < 9; ++t) {
        bf8 nxt = cur;
        if (t < 8) {
          const int tn = t + 1;
          nxt = *reinterpret_cast<const bf8*>(blk + in_row[tn / 3] + to.sw[tn % 3]);
        }
#pragma unroll
        for (int a = 0; a < 2; ++a) acc[a] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(wf[t][a], cur, acc[a], 0, 0, 0);
        cur = nxt;
      }
    }
    if (j >= width) continue;
    const bool inside = row_inside && in_image(gr, gc0 + j, n);
    uint4 v;
    v.x = inside ? pack2(relu(acc[0][0]), relu(acc[0][1])) : 0u;
    v.y = inside ? pack2(relu(acc[0][2]), relu(acc[0][3])) : 0u;
    v.z = inside ? pack2(relu(acc[1][0]), relu(acc[1][1])) : 0u;
    v.w = inside ? pack2(relu(acc[1][2]), relu(acc[1][3])) : 0u;
    *reinterpret_cast<uint4*>(out_row + b * 16 * PXB + to.sw[0]) = v;
  }
}

// Layer 5 (32 -> 2, outputs padded to 16: one output block): the wave's
// blocks one at a time, the next tap's activation read issued before this
// tap's product; then x0 = zf + f(zf) (channels 0, 1 in rows 0, 1 of D,
// lanes q = 0).  (Three interleaved chains measured 40% slower: the other
// waves on the SIMD already hide the chain's latency.)
__device__ __forceinline__ void conv_row_last(const unsigned char* lds, const int (&in_row)[3], const bf8 (&wf)[9],
                                              const f4& bo, const TapOffsets& to, int b0, int nblk, int width, int q,
                                              int m, const float2 (&zf)[3], float2* x0_row) {
#pragma unroll
  for (int u = 0; u < 3; ++u) {
    const int b = b0 + u * WPL;
    if (b >= nblk) break;
    const unsigned char* blk = lds + b * 16 * PXB;
    f4 acc = bo;
    bf8 cur = *reinterpret_cast<const bf8*>(blk + in_row[0] + to.sw[0]);
#pragma unroll
    for (int t = 0; t < 9; ++t) {
      bf8 nxt = cur;
      if (t < 8) nxt = *reinterpret_cast<const bf8*>(blk + in_row[(t + 1) / 3] + to.sw[(t + 1) % 3]);
      acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(wf[t], cur, acc, 0, 0, 0);
      cur = nxt;
    }
    const int j = b * 16 + m;
    if (j < width && q == 0) x0_row[j] = make_float2(zf[u].x + acc[0], zf[u].y + acc[1]);
  }
}

}  // namespace

// Geometry of one launch: strips of SW columns, bands of BH = SW rows.
struct NetGeo {
  int n, SW, BH, strips, bands, items;
  __device__ __forceinline__ int width(int l) const { return SW + 2 * (5 - l); }   // layer l's row
  __device__ __forceinline__ int nblocks(int l) const { return (width(l) + 15) / 16; }
  __device__ __forceinline__ void item(int it, int& img, int& R0, int& c0) const {
    img = it / (strips * bands);
    const int rest = it - img * strips * bands, band = rest / strips;
    R0 = band * BH;
    c0 = (rest - band * strips) * SW;
  }
};

__device__ __forceinline__ int ring_row(int l, int r) {   // LDS offset of row r of layer l's ring (l = 1..4)
  return (int)(OFF_ACT + (size_t)(l - 1) * ACT_RING + (size_t)slot(r) * ROWPX * PXB);
}

// Waves 0-3: the input rows, layer 1 (2 -> 32, the 9 taps x 2 channels
// stacked into K = 32) and layer 5 (32 -> 2) with x0 = zf + f(zf).
__device__ __forceinline__ void net_role_io(const NetArgs& A, const NetGeo& G, unsigned char* smem, int sub, int q,
                                            int m) {
  const int tid = threadIdx.x, n = G.n;
  unsigned int* in_ring = reinterpret_cast<unsigned int*>(smem + OFF_IN);
  bf8 w1f[2];
  {
    const unsigned short* w1 = static_cast<const unsigned short*>(A.w[0]);
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        const int k = 8 * q + e, t = k >> 1, c = k & 1;
        w1f[a][e] = __builtin_bit_cast(__bf16, k < 18 ? w1[(t * 32 + a * 16 + m) * 16 + c] : (unsigned short)0);
      }
  }
  const f4 b1[2] = {*reinterpret_cast<const f4*>(A.b[0] + 4 * q), *reinterpret_cast<const f4*>(A.b[0] + 16 + 4 * q)};
  bf8 w5[9];
  {
    const unsigned short* w = static_cast<const unsigned short*>(A.w[4]);
#pragma unroll
    for (int t = 0; t < 9; ++t) w5[t] = load_w32(w, 16, t, m, q);
  }
  const TapOffsets to(m, q);
  const f4 b5 = *reinterpret_cast<const f4*>(A.b[4] + 4 * q);
  // layer-1 taps of this lane group: taps 4q .. 4q + 3 (those below 9)
  int dyo[4], dxo[4];
  bool tok[4];
#pragma unroll
  for (int mm = 0; mm < 4; ++mm) {
    const int tt = 4 * q + mm;
    tok[mm] = tt < 9;
    dyo[mm] = tok[mm] ? tt / 3 - 1 : 0;
    dxo[mm] = tok[mm] ? tt % 3 : 0;
  }
  for (int it = blockIdx.x; it < G.items; it += gridDim.x) {
    int img, R0, c0;
    G.item(it, img, R0, c0);
    const float2* zf = static_cast<const float2*>(A.zf) + (size_t)img * n * n;
    float2* x0 = static_cast<float2*>(A.x0) + (size_t)img * n * n;
    // Input rows (columns c0 - 5 .. c0 + SW + 4; thread tid owns column
    // tid) go through registers: the row a step needs is fetched two steps
    // ahead and written to its ring slot one step ahead, so the global
    // load's latency overlaps a step of work.  zf of the layer-5 row is
    // fetched a step ahead as well.  Zero outside the image.
    const int gcol = c0 - HALO + tid;
    const bool in_col = tid < G.width(0);
    auto fetch_in = [&](int r) -> float2 {
      return in_col && in_image(r, gcol, n) ? zf[(size_t)r * n + gcol] : make_float2(0.f, 0.f);
    };
    auto put_in = [&](int r, float2 z) {
      if (in_col) in_ring[slot(r) * ROWPX + tid] = pack2(z.x, z.y);
    };
    float2 z5[3] = {};
    auto fetch_z5 = [&](int r) {
      if (q != 0 || (unsigned)r >= (unsigned)n) return;
#pragma unroll
      for (int u = 0; u < 3; ++u) {
        const int j = (sub + u * WPL) * 16 + m;
        if (j < G.width(5)) z5[u] = zf[(size_t)r * n + c0 + j];
      }
    };
    __syncthreads();   // the previous item's last reads of the rings are done
    put_in(R0 - 5, fetch_in(R0 - 5));
    put_in(R0 - 4, fetch_in(R0 - 4));
    put_in(R0 - 3, fetch_in(R0 - 3));
    float2 next_in = fetch_in(R0 - 2);
    __syncthreads();
    const int steps = G.BH + 12;
    for (int t = 0; t < steps; ++t) {
      if (t <= G.BH + 6) {   // the next step's layer-1 row needs input row R0 - 2 + t
        put_in(R0 - 2 + t, next_in);
        next_in = fetch_in(R0 - 1 + t);
      }
      if (t == 11) fetch_z5(R0);
      const int r1 = R0 - 4 + t;
      if (t <= G.BH + 7) {
        const int nb = G.nblocks(1), w1w = G.width(1);
        unsigned char* out = smem + ring_row(1, r1);
        const bool row_in = (unsigned)r1 < (unsigned)n;
        for (int b = sub; b < nb; b += WPL) {
          const int j = b * 16 + m;
          f4 acc[2] = {b1[0], b1[1]};
          if (row_in) {
            unsigned int raw[4];
#pragma unroll
            for (int mm = 0; mm < 4; ++mm)
              raw[mm] = tok[mm] ? in_ring[slot(r1 + dyo[mm]) * ROWPX + j + dxo[mm]] : 0u;
            const bf8 bop = __builtin_bit_cast(bf8, make_uint4(raw[0], raw[1], raw[2], raw[3]));
#pragma unroll
            for (int a = 0; a < 2; ++a) acc[a] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(w1f[a], bop, acc[a], 0, 0, 0);
          }
          if (j < w1w) {
            const bool inside = row_in && in_image(r1, c0 - 4 + j, n);
            uint4 v;
            v.x = inside ? pack2(relu(acc[0][0]), relu(acc[0][1])) : 0u;
            v.y = inside ? pack2(relu(acc[0][2]), relu(acc[0][3])) : 0u;
            v.z = inside ? pack2(relu(acc[1][0]), relu(acc[1][1])) : 0u;
            v.w = inside ? pack2(relu(acc[1][2]), relu(acc[1][3])) : 0u;
            *reinterpret_cast<uint4*>(out + b * 16 * PXB + to.sw[0]) = v;
          }
        }
      }
      const int r5 = R0 - 12 + t;
      if (t >= 12) {
        const int in_row[3] = {ring_row(4, r5 - 1), ring_row(4, r5), ring_row(4, r5 + 1)};
        conv_row_last(smem, in_row, w5, b5, to, sub, G.nblocks(5), G.width(5), q, m, z5, x0 + (size_t)r5 * n + c0);
        fetch_z5(r5 + 1);   // for the next step (past the last row: nothing)
      }
      __syncthreads();
    }
  }
}

// Waves 4-15: layer l = 2, 3 or 4 (32 -> 32), row r = R0 - 4 + t - 2 (l - 1)
// at step t.
__device__ __forceinline__ void net_role_conv(const NetArgs& A, const NetGeo& G, unsigned char* smem, int l, int sub,
                                              int q, int m) {
  bf8 wf[9][2];
  f4 bo[2];
  {
    const unsigned short* w = static_cast<const unsigned short*>(A.w[l - 1]);
#pragma unroll
    for (int t = 0; t < 9; ++t)
#pragma unroll
      for (int a = 0; a < 2; ++a) wf[t][a] = load_w32(w, 32, t, 16 * a + m, q);
#pragma unroll
    for (int a = 0; a < 2; ++a) bo[a] = *reinterpret_cast<const f4*>(A.b[l - 1] + 16 * a + 4 * q);
  }
  const TapOffsets to(m, q);
  const int first = 3 * l - 3, last = first + G.BH - 1 + 2 * (5 - l);
  for (int it = blockIdx.x; it < G.items; it += gridDim.x) {
    int img, R0, c0;
    G.item(it, img, R0, c0);
    __syncthreads();
    __syncthreads();
    const int steps = G.BH + 12;
    for (int t = 0; t < steps; ++t) {
      const int r = R0 - 4 + t - 2 * (l - 1);
      if (t >= first && t <= last) {
        const int in_row[3] = {ring_row(l - 1, r - 1), ring_row(l - 1, r), ring_row(l - 1, r + 1)};
        conv_row(smem, in_row, wf, bo, to, sub, G.nblocks(l), G.width(l), m, smem + ring_row(l, r), r,
                 c0 - (5 - l), G.n, (unsigned)r < (unsigned)G.n);
      }
      __syncthreads();
    }
  }
}

__global__ __launch_bounds__(SNT) void k_net_fwd(NetArgs A) {
  extern __shared__ __align__(16) unsigned char smem[];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, m = lane & 15, q = lane >> 4;
  NetGeo G;
  G.n = A.n;
  G.SW = A.n % 128 == 0 ? 128 : (A.n % 64 == 0 ? 64 : 32);
  G.BH = G.SW;
  G.strips = A.n / G.SW;
  G.bands = A.n / G.BH;
  G.items = A.batch * G.strips * G.bands;
  // roles by wave (uniform per wave): waves 0-3 input rows and layers 1, 5;
  // waves 4k .. 4k + 3 layer k + 1.  Both paths pass the same number of
  // barriers per work item (two, then one per step).
  const int simd = wave & 3, k = wave >> 2, sub = (simd + k) & 3;
  if (k == 0) net_role_io(A, G, smem, sub, q, m);
  else net_role_conv(A, G, smem, k + 1, sub, q, m);
}

size_t net_fwd_lds_bytes() { return LDS_BYTES; }

hipError_t launch_net_fwd(const NetArgs& a, int grid, hipStream_t st) {
  static bool attr = false;
  if (!attr) {
    hipError_t e = hipFuncSetAttribute((const void*)k_net_fwd, hipFuncAttributeMaxDynamicSharedMemorySize, (int)LDS_BYTES);
    if (e != hipSuccess) return e;
    attr = true;
  }
  hipLaunchKernelGGL(k_net_fwd, dim3(grid), dim3(SNT), LDS_BYTES, st, a);
  return hipGetLastError();
}

// Work items of one launch (one per output block of BH x SW pixels).
int net_fwd_items(int n, int batch) {
  const int SW = n % 128 == 0 ? 128 : (n % 64 == 0 ? 64 : 32);
  return batch * (n / SW) * (n / SW);
}

}  // namespace cnn
}  // namespace firls
