// Precision-only kernels, per-slice bookkeeping kernels and the launcher
// registry.
#include <mutex>

#include "firls_inst.h"

namespace firls {

// rho = (number of sampled entries) / n^2, the mean (indeed every entry) of
// diag(A^H A) for the unitary F (Section 5.4), and a fresh outer-loop state.
// One workgroup per slice; ``mask`` is the slice's mask (D.mask).
// A TV solve needs the DC entry of every contrast's mask: the differences
// annihilate constants, so without it A 1 = 0 and the minimiser is not
// unique.  Such a slice is not started: status FIRLS_E_INVALID, and its
// stop word (``flag``, host-mapped, if given) reads stopped at once.
__device__ void init_slice(const SliceDesc& D, const uint8_t* mask, SliceState& S, double* red, int32_t* flag) {
  // the paired PCG pass's barrier counters count from zero for each slice
  uint32_t* sync = reinterpret_cast<uint32_t*>(slot_wptr(D, SLOT_SYNC));
  for (int k = threadIdx.x; k < KMAX; k += NT) sync[k] = 0u;
  if (D.rho_fixed > 0.0) {
    // dense sensing matrix: rho = mean diag(A^T A), set by the host; no mask
    if (threadIdx.x == 0) {
      S.rho = D.rho_fixed;
      S.Fe = S.F = S.data = S.Fe_prev = S.rel = 0.0;
      S.active = 1;
      S.outer = S.pcg = S.status = S.converged = S.evals = S.pend = S.pcg_stop = 0;
    }
    return;
  }
  const int n = D.n, rows = D.C * n, total = rows * n;
  // count the samples and pack the mask: word [c16][row] holds columns
  // 16 c16 .. 16 c16 + 15 of the row, bit c = column 16 c16 + c; rows run
  // over all contrasts
  double cnt = 0.0;
  const int words = total / 16;
  for (int w = threadIdx.x; w < words; w += NT) {
    const int c16 = w / rows, row = w - c16 * rows;
    const uint8_t* src = mask + (size_t)row * n + c16 * 16;
    unsigned int bits = 0;
#pragma unroll
    for (int c = 0; c < 16; ++c) bits |= (src[c] != 0 ? 1u : 0u) << c;
    D.mbits[w] = (uint16_t)bits;
    cnt += (double)__popc(bits);
  }
  cnt = block_sum(cnt, red);
  if (threadIdx.x == 0) {
    S.rho = cnt / (double)total;
    S.Fe = S.F = S.data = S.Fe_prev = S.rel = 0.0;
    S.active = 1;
    S.outer = S.pcg = S.status = S.converged = S.evals = S.pend = S.pcg_stop = 0;
    bool dc = true;
    for (int c = 0; D.need_dc && c < D.C; ++c) dc = dc && mask[(size_t)c * n * n] != 0;
    if (!dc) {
      S.status = ST_E_INVALID;
      S.active = 0;
      if (flag) __hip_atomic_store(flag, 0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
    }
  }
}

__global__ __launch_bounds__(NT) void k_slice_init(Params P) {
  __shared__ double red[NT / 64];
  const int s = P.list[blockIdx.x];
  init_slice(P.desc[s], P.desc[s].mask, P.state[s], red, P.stop_flags ? P.stop_flags + s : nullptr);
}

// Slot refills of a streamed batch, one workgroup per record: save the
// stopped slice's final state, give the slot the new slice's inputs (the
// slot's workspace pointers stay) and start the new slice's outer loop.
__global__ __launch_bounds__(NT) void k_refill(RefillArgs A) {
  __shared__ double red[NT / 64];
  const RefillRec r = A.rec[blockIdx.x];
  SliceDesc& D = A.desc[r.slot];
  SliceState& S = A.state[r.slot];
  if (threadIdx.x == 0) {
    if (r.old >= 0) A.state[A.final_base + r.old] = S;
    D.b = r.b;
    D.mask = r.mask;
    D.x = r.x;
    D.lambda = r.lambda;
    A.list[blockIdx.x] = r.slot;
  }
  init_slice(D, r.mask, S, red, A.stop_flags ? A.stop_flags + r.slot : nullptr);
}

hipError_t launch_refill(const RefillArgs& A, hipStream_t st) {
  const LaunchTiming& t = launch_timing();
  launch_kernel(k_refill, dim3(A.count), dim3(NT), 0, st, t.start, t.stop, A);
  return hipGetLastError();
}

// Objective of the current x and the outer stopping rule.  F_eps = data +
// lambda sum sqrt(s_g + eps); stop when (F_eps^{prev} - F_eps) <= tau F_eps
// after the first evaluation, or once Tmax solves are done; otherwise count
// the solve that follows.
__global__ __launch_bounds__(NT) void k_outer_check(Params P) {
  const int s = P.list[blockIdx.x];
  if (!P.state[s].active) return;
  outer_check_wg(P, s);
}

// d in the caller's coefficient order: out[u] = d[perm[u]].
template <typename T>
__global__ __launch_bounds__(NT) void k_export_d(Params P) {
  const int s = P.list[blockIdx.y];
  const SliceDesc& D = P.desc[s];
  const T* d = static_cast<const T*>(D.d);
  T* out = static_cast<T*>(P.out);
  const int u = blockIdx.x * NT + threadIdx.x;
  if (u < P.shape.n_coef) out[u] = d[P.shape.perm[u]];
}

LaunchTiming& launch_timing() {
  thread_local LaunchTiming t{nullptr, nullptr};
  return t;
}

template <class K>
hipError_t launch_static(K kern, const Params& P, dim3 g, hipStream_t st) {
  const LaunchTiming& t = launch_timing();
  launch_kernel(kern, g, dim3(NT), 0, st, t.start, t.stop, P);
  return hipGetLastError();
}

template <typename T> hipError_t L_psi_sq_tv(const Params& P, dim3 g, hipStream_t st) { return launch_static(k_psi_sq_tv<T>, P, g, st); }
template <typename T> hipError_t L_group_w(const Params& P, dim3 g, hipStream_t st) { return launch_static(k_group_w<T>, P, g, st); }
template <typename T> hipError_t L_group_d(const Params& P, dim3 g, hipStream_t st) { return launch_static(k_group_d<T>, P, g, st); }
template <typename T, int M> hipError_t L_update_tv(const Params& P, dim3 g, hipStream_t st) { return launch_static(k_update_tv<T, M>, P, g, st); }
template <typename T> hipError_t L_export_d(const Params& P, dim3 g, hipStream_t st) { return launch_static(k_export_d<T>, P, g, st); }
hipError_t L_slice_init(const Params& P, dim3 g, hipStream_t st) { return launch_static(k_slice_init, P, g, st); }
hipError_t L_outer_check(const Params& P, dim3 g, hipStream_t st) { return launch_static(k_outer_check, P, g, st); }

template <typename T>
PrecKernels make_prec() {
  PrecKernels k{};
  k.psi_sq_tv = L_psi_sq_tv<T>;
  k.group_w = L_group_w<T>;
  k.group_d = L_group_d<T>;
  k.update_tv[UP_INIT] = L_update_tv<T, UP_INIT>;
  k.update_tv[UP_STEP] = L_update_tv<T, UP_STEP>;
  k.export_d = L_export_d<T>;
  k.slice_init = L_slice_init;
  k.outer_check = L_outer_check;
  return k;
}

#define FIRLS_DECL(N) SizeKernels make_size_f32_##N(); SizeKernels make_size_f64_##N();
FIRLS_SIZES(FIRLS_DECL)
#undef FIRLS_DECL

namespace {
struct Tables {
  SizeKernels f32[10], f64[10];
  PrecKernels p32, p64;
};
constexpr int kSizes[10] = {16, 32, 48, 64, 96, 128, 192, 256, 384, 512};
std::once_flag g_once;
Tables* g_tables = nullptr;

void build_tables() {
  static Tables t;
  int i = 0;
#define FIRLS_FILL(N)                  \
  t.f32[i] = make_size_f32_##N();      \
  t.f64[i] = make_size_f64_##N();      \
  ++i;
  FIRLS_SIZES(FIRLS_FILL)
#undef FIRLS_FILL
  t.p32 = make_prec<float>();
  t.p64 = make_prec<double>();
  g_tables = &t;
}

int size_index(int n) {
  for (int i = 0; i < 10; ++i)
    if (kSizes[i] == n) return i;
  return -1;
}
}  // namespace

bool size_supported(int n) { return size_index(n) >= 0; }

const SizeKernels* size_kernels(bool fp64, int n) {
  std::call_once(g_once, build_tables);
  const int i = size_index(n);
  if (i < 0) return nullptr;
  return fp64 ? &g_tables->f64[i] : &g_tables->f32[i];
}

const PrecKernels* prec_kernels(bool fp64) {
  std::call_once(g_once, build_tables);
  return fp64 ? &g_tables->p64 : &g_tables->p32;
}

}  // namespace firls
