// Host side of the C ABI: validation, group-map preparation, workspace,
// and the outer loop of Algorithms 2 / 3 driving the device kernels.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cstdio>
#include <cstdlib>
#include <fstream>
#include <mutex>
#include <sstream>
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "firls.h"
#include "firls_registry.h"
#include "cnn_types.h"

using namespace firls;

namespace {

thread_local std::string g_err;

int fail(int code, const std::string& msg) {
  g_err = msg;
  return code;
}

#define HIPCHK(expr)                                                                   \
  do {                                                                                 \
    hipError_t e_ = (expr);                                                            \
    if (e_ != hipSuccess) return fail(FIRLS_E_HIP, std::string(#expr) + ": " + hipGetErrorString(e_)); \
  } while (0)

size_t align256(size_t v) { return (v + 255) & ~size_t(255); }


struct Shape {
  int n = 0, psi = 0, L = 0, n_groups = 0, n_coef = 0;
  int tvb = 0;   // TV boundary: 0 periodic, 1 the paper's non-periodic D
  int C = 1;     // contrasts, stacked as C blocks of n rows
  bool dense = false;   // dense sensing matrix instead of the masked FFT
  int M = 0, Mp = 0;    // its rows, and rows padded to the GEMM tile
  void* d_A = nullptr;  // Mp x n^2 in the working precision
  double rho_A = 0.0;   // mean diag(A^T A)
  int32_t* d_bgptr = nullptr;   // band-local group map: first group of every row band
  uint16_t* d_gell = nullptr;   // and its padded member / membership lists (ShapeDev)
  uint16_t* d_tell = nullptr;
  int ell_gw = 0, ell_tw = 0;
  size_t pixels() const { return (size_t)C * n * n; }
  int row_wgs() const { return C * n / band_rows(n); }                  // row-pass workgroups
  int col_wgs(bool fp64) const { return C * (n / strip_cols(fp64, n)); }  // column-pass workgroups
  int64_t n_members = 0;
  int32_t* d_gptr = nullptr;
  int32_t* d_gidx = nullptr;
  int32_t* d_tptr = nullptr;
  int32_t* d_tidx = nullptr;
  int32_t* d_perm = nullptr;
  const SizeKernels* sk = nullptr;
  void* tw = nullptr;
};

// Position of Mallat coefficient (gr, gc) of an n x n, L-level Haar
// transform in the library's in-place layout: a level-l detail sits in the
// tile of side 2^L its support lies in, at the pixel where the in-place
// transform leaves it (row offset 2^(l-1) for a vertical detail, column
// offset 2^(l-1) for a horizontal one, within the 2^l block it summarises);
// the coarsest approximation sits at the tile's top-left pixel.
int32_t haar_internal_index(int n, int L, int gr, int gc) {
  const int hL = n >> L;
  if (gr < hL && gc < hL) return (gr << L) * n + (gc << L);
  int lev = 1;
  while (lev < L && std::max(gr, gc) < (n >> lev)) ++lev;
  const int hg = n >> lev;
  const bool vert = gr >= hg, horz = gc >= hg;
  const int i = vert ? gr - hg : gr;
  const int j = horz ? gc - hg : gc;
  const int sh = L - lev;
  const int I = i >> sh, J = j >> sh;
  const int s = ((i & ((1 << sh) - 1)) << lev) + (vert ? 1 << (lev - 1) : 0);
  const int c = ((j & ((1 << sh) - 1)) << lev) + (horz ? 1 << (lev - 1) : 0);
  return ((I << L) + s) * n + (J << L) + c;
}

// Device memory of firls_solve_batched_noalloc: one array per GPU, held
// until the process ends.  Host code never uses the array's name as an
// address (on the host it is only a stand-in): the device address comes
// from hipGetSymbolAddress, taken once per device at handle creation with
// that device current.
constexpr size_t kNoallocBytes = FIRLS_NOALLOC_SCRATCH_BYTES;
__device__ __align__(256) unsigned char g_noalloc_scratch[kNoallocBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// The array's address on ``device`` (the current device), looked up once.
int noalloc_scratch(int device, void** out) {
  *out = nullptr;
  if (device < 0 || device >= kMaxDevices) return fail(FIRLS_E_UNSUPPORTED, "device index too large");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[device]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(g_noalloc_scratch));
    if (e != hipSuccess || !p) {
      (void)hipGetLastError();
      return fail(FIRLS_E_HIP, std::string("hipGetSymbolAddress of the allocation-free scratch: ") +
                                   hipGetErrorString(e));
    }
    g_scratch_ptr[device] = p;
  }
  *out = g_scratch_ptr[device];
  return FIRLS_OK;
}

}  // namespace

namespace firls {
int set_error(int code, const std::string& msg) { return fail(code, msg); }
int cnn_forward(firls_cnn* c, hipStream_t st, int batch, const void* zf, void* x0);
int cnn_image_side(const firls_cnn* c);
int cnn_max_batch(const firls_cnn* c);
bool cnn_ready(const firls_cnn* c);
}  // namespace firls

struct firls_handle {
  firls_config cfg{};
  std::vector<Shape> shapes;
  bool fp64 = false;
  size_t elt = 8;    // bytes per complex
  size_t relt = 4;   // bytes per real
  std::vector<std::pair<int, void*>> tw;
  int device = 0;

  void* ws = nullptr;
  size_t ws_cap = 0;
  int cap_slices = 0;
  SliceDesc* d_desc = nullptr;
  SliceState* d_state = nullptr;
  int32_t* d_list = nullptr;
  SliceDesc* h_desc = nullptr;
  SliceState* h_state = nullptr;
  int32_t* h_list = nullptr;
  // stop-test words, (evaluations << 1) | active per slice, in host memory
  // the kernels write to directly (coherent, mapped)
  int32_t* h_flags = nullptr;
  int32_t* d_flags = nullptr;
  // slot refills of a streamed batch, read by k_refill (coherent, mapped)
  RefillRec* h_refill = nullptr;
  RefillRec* d_refill = nullptr;
  hipEvent_t ev = nullptr;

  // graph replay of one outer iteration's launches
  bool use_graphs = true;
  // the paired PCG pass (row inverse of k - 1 and step of k in one launch)
  bool use_pair = true;
  int test_flags = 0;       // firls_test_hooks (TEST_*)
  hipStream_t own = nullptr;          // work stream when the caller passes the null stream
  hipEvent_t ev_in = nullptr;
  struct GraphKey {
    std::vector<int> counts;
    int Tmax = -1;
    double tau = -1.0;
    void* ws = nullptr;
    void* desc = nullptr;
    hipStream_t stream = nullptr;
    int multi = 0;   // schedule of launches across shapes (0: per shape)
    bool operator==(const GraphKey& o) const {
      return counts == o.counts && Tmax == o.Tmax && tau == o.tau && ws == o.ws && desc == o.desc &&
             stream == o.stream && multi == o.multi;
    }
  } gkey;
  hipGraphExec_t g_iter = nullptr;
  // sub-batch size chosen by firls_autotune (0: the whole batch at once)
  int chunk = 0;
  // set while firls_solve_batched_noalloc runs: buffers must already fit
  bool noalloc = false;
  // how a batch of several shapes is launched: FIRLS_SCHED_PER_SHAPE, or
  // one launch per kernel class and position across shapes
  // (FIRLS_SCHED_ACROSS in batch order, FIRLS_SCHED_ACROSS_LARGEST_FIRST)
  int schedule = FIRLS_SCHED_PER_SHAPE;
  // while set, launch_prep / launch_pcg record their launches here
  struct LaunchRec {
    Launcher fn;
    Params P;
    dim3 grid;
    int cls;
  };
  std::vector<LaunchRec>* rec_seq = nullptr;
  // device work tables of the launches across shapes
  Params* d_mparams = nullptr;
  size_t mparams_cap = 0;
  MultiItem* d_mitems = nullptr;
  size_t mitems_cap = 0;
  void* scratch = nullptr;   // this device's g_noalloc_scratch (null if the lookup failed)
  std::string scratch_err;

  // learned-start staging: zero-filled and network starts [S, n, n] complex,
  // per-slice output pointers and a copy of the slice states
  void* ws_learn = nullptr;
  size_t ws_learn_cap = 0;
  void* gscr = nullptr;     // split-K partial tiles of the dense-matrix GEMMs
  size_t gscr_cap = 0;

  // Opt-in per-launch timing (firls_profile): one event pair per launch.
  struct ProfRec {
    int cls, group, it, phase, count;
    hipEvent_t a, b;
  };
  bool profiling = false;
  std::vector<hipEvent_t> ev_pool;
  size_t ev_used = 0;
  std::vector<ProfRec> recs;
  int ctx_group = 0, ctx_it = 0, ctx_phase = 0, ctx_count = 0;
  double prof_ms[FIRLS_PROF_CLASSES] = {};
  int64_t prof_launches[FIRLS_PROF_CLASSES] = {};
  int64_t prof_units[FIRLS_PROF_CLASSES] = {};
  // the same per shape (index shape * FIRLS_PROF_CLASSES + class)
  std::vector<double> prof_ms_shape;
  std::vector<int64_t> prof_launches_shape, prof_units_shape;

  size_t slice_bytes(const Shape& s) const {
    return slice_bytes_of(s.pixels(), s.psi == PSI_TV, (size_t)s.n_coef, (size_t)s.n_groups, s.dense ? s.Mp : 0,
                          elt, relt);
  }
  // Workspace of one slice (fill_desc carves it in this order): r, p, q, t
  // (and for TV a second r and z), d and |Psi x|^2 per coefficient, W per
  // group, the packed mask, the partial sums, and A v for a dense matrix.
  static size_t slice_bytes_of(size_t pixels, bool tv, size_t n_coef, size_t n_groups, int Mp, size_t elt,
                               size_t relt) {
    const size_t vec = align256(pixels * elt);
    const size_t nvec = tv ? 6 : 4;
    return nvec * vec + 2 * align256(n_coef * relt) + align256(n_groups * relt) + align256(pixels / 8) +
           align256((size_t)SLOT_COUNT * PMAX * sizeof(double)) + (Mp ? align256((size_t)Mp * elt) : 0);
  }
  bool ws_owned = true;   // false: the workspace is the caller's (firls_config.workspace)
};

namespace {

void drop_graphs(firls_handle* h) {
  if (h->g_iter) (void)hipGraphExecDestroy(h->g_iter);
  h->g_iter = nullptr;
  h->gkey = firls_handle::GraphKey{};
}

void free_batch(firls_handle* h) {
  drop_graphs(h);
  if (h->d_mparams) (void)hipFree(h->d_mparams);
  if (h->d_mitems) (void)hipFree(h->d_mitems);
  h->d_mparams = nullptr;
  h->d_mitems = nullptr;
  h->mparams_cap = h->mitems_cap = 0;
  if (h->ws_learn) (void)hipFree(h->ws_learn);
  h->ws_learn = nullptr;
  h->ws_learn_cap = 0;
  if (h->gscr) (void)hipFree(h->gscr);
  h->gscr = nullptr;
  h->gscr_cap = 0;
  if (h->ws && h->ws_owned) (void)hipFree(h->ws);
  if (h->d_desc) (void)hipFree(h->d_desc);
  if (h->d_state) (void)hipFree(h->d_state);
  if (h->d_list) (void)hipFree(h->d_list);
  if (h->h_desc) (void)hipHostFree(h->h_desc);
  if (h->h_state) (void)hipHostFree(h->h_state);
  if (h->h_list) (void)hipHostFree(h->h_list);
  if (h->h_flags) (void)hipHostFree(h->h_flags);
  if (h->h_refill) (void)hipHostFree(h->h_refill);
  if (h->ws_owned) {
    h->ws = nullptr;
    h->ws_cap = 0;
  }
  h->d_desc = nullptr;
  h->d_state = nullptr;
  h->d_list = nullptr;
  h->h_desc = nullptr;
  h->h_state = nullptr;
  h->h_list = nullptr;
  h->h_flags = h->d_flags = nullptr;
  h->h_refill = h->d_refill = nullptr;
  h->cap_slices = 0;
}

int ensure_capacity(firls_handle* h, hipStream_t st, size_t bytes, int slices) {
  if (h->noalloc && (bytes > h->ws_cap || std::max(slices, 2) > h->cap_slices))
    return fail(FIRLS_E_INVALID, "internal: the allocation-free solve needs more memory than it checked for");
  if (!h->ws_owned && bytes > h->ws_cap)
    return fail(FIRLS_E_INVALID, "the caller's workspace holds " + std::to_string(h->ws_cap) + " bytes; this call needs " +
                                     std::to_string(bytes));
  if (bytes > h->ws_cap || std::max(slices, 2) > h->cap_slices) drop_graphs(h);
  if (bytes > h->ws_cap) {
    HIPCHK(hipStreamSynchronize(st));
    if (h->ws) HIPCHK(hipFree(h->ws));
    h->ws = nullptr;
    h->ws_cap = 0;
    if (hipMalloc(&h->ws, bytes) != hipSuccess) {
      (void)hipGetLastError();
      return fail(FIRLS_E_NOMEM, "workspace allocation of " + std::to_string(bytes) + " bytes failed");
    }
    h->ws_cap = bytes;
  }
  // two list copies (all slices, then the zero-filled subset) need 2x
  const int want = std::max(slices, 2);
  if (want > h->cap_slices) {
    HIPCHK(hipStreamSynchronize(st));
    if (h->d_desc) HIPCHK(hipFree(h->d_desc));
    if (h->d_state) HIPCHK(hipFree(h->d_state));
    if (h->d_list) HIPCHK(hipFree(h->d_list));
    if (h->h_desc) HIPCHK(hipHostFree(h->h_desc));
    if (h->h_state) HIPCHK(hipHostFree(h->h_state));
    if (h->h_list) HIPCHK(hipHostFree(h->h_list));
    if (h->h_flags) HIPCHK(hipHostFree(h->h_flags));
    if (h->h_refill) HIPCHK(hipHostFree(h->h_refill));
    h->h_desc = nullptr;
    h->h_state = nullptr;
    h->h_list = nullptr;
    h->h_flags = h->d_flags = nullptr;
    h->h_refill = h->d_refill = nullptr;
    h->cap_slices = 0;
    HIPCHK(hipMalloc(&h->d_desc, sizeof(SliceDesc) * want));
    HIPCHK(hipMalloc(&h->d_state, sizeof(SliceState) * want));
    HIPCHK(hipMalloc(&h->d_list, sizeof(int32_t) * 2 * want));
    HIPCHK(hipHostMalloc(&h->h_desc, sizeof(SliceDesc) * want, hipHostMallocDefault));
    HIPCHK(hipHostMalloc(&h->h_state, sizeof(SliceState) * want, hipHostMallocDefault));
    HIPCHK(hipHostMalloc(&h->h_list, sizeof(int32_t) * 2 * want, hipHostMallocDefault));
    HIPCHK(hipHostMalloc(&h->h_flags, sizeof(int32_t) * want, hipHostMallocMapped | hipHostMallocCoherent));
    HIPCHK(hipHostGetDevicePointer(reinterpret_cast<void**>(&h->d_flags), h->h_flags, 0));
    HIPCHK(hipHostMalloc(&h->h_refill, sizeof(RefillRec) * want, hipHostMallocMapped | hipHostMallocCoherent));
    HIPCHK(hipHostGetDevicePointer(reinterpret_cast<void**>(&h->d_refill), h->h_refill, 0));
    h->cap_slices = want;
  }
  return FIRLS_OK;
}

// Carve slice i's workspace at byte offset ``off``.
void fill_desc(firls_handle* h, SliceDesc& D, const Shape& s, size_t off, const firls_slice* sl) {
  char* base = static_cast<char*>(h->ws) + off;
  const size_t vec = align256(s.pixels() * h->elt);
  std::memset(&D, 0, sizeof(D));
  D.r[0] = base;
  D.p = base + vec;
  D.q = base + 2 * vec;
  D.t = base + 3 * vec;
  size_t o = 4 * vec;
  if (s.psi == PSI_TV) {
    D.r[1] = base + o;
    D.z = base + o + vec;
    o += 2 * vec;
  } else {
    D.r[1] = D.r[0];
  }
  D.d = base + o;
  o += align256((size_t)s.n_coef * h->relt);
  D.sq = base + o;
  o += align256((size_t)s.n_coef * h->relt);
  D.W = base + o;
  o += align256((size_t)s.n_groups * h->relt);
  D.mbits = reinterpret_cast<uint16_t*>(base + o);
  o += align256(s.pixels() / 8);
  D.parts = reinterpret_cast<double*>(base + o);
  o += align256((size_t)SLOT_COUNT * PMAX * sizeof(double));
  if (s.dense) D.y = base + o;
  D.rho_fixed = s.dense ? s.rho_A : 0.0;
  D.n = s.n;
  D.C = s.C;
  D.shape = 0;
  D.need_dc = sl && s.psi == PSI_TV && !s.dense ? 1 : 0;
  if (sl) {
    D.b = sl->b;
    D.mask = sl->mask;
    D.x = sl->x;
    D.lambda = sl->lambda;
  }
}

Params base_params(const firls_handle* h, const Shape& s, int shape_id, const int32_t* list) {
  Params P{};
  P.desc = h->d_desc;
  P.state = h->d_state;
  P.list = list;
  P.tw = s.tw;
  P.shape.gptr = s.d_gptr;
  P.shape.gidx = s.d_gidx;
  P.shape.tptr = s.d_tptr;
  P.shape.tidx = s.d_tidx;
  P.shape.perm = s.d_perm;
  P.shape.A = s.d_A;
  P.shape.bgptr = s.d_bgptr;
  P.shape.gell = s.d_gell;
  P.shape.tell = s.d_tell;
  P.shape.gw = s.ell_gw;
  P.shape.tw = s.ell_tw;
  P.shape.M = s.M;
  P.shape.Mp = s.Mp;
  P.nofft = s.dense ? 1 : 0;
  P.tvb = s.tvb;
  P.shape.n_groups = s.n_groups;
  P.shape.n_coef = s.n_coef;
  P.n = s.n;
  P.C = s.C;
  P.L = s.L;
  P.K = h->cfg.pcg_iters;
  P.Tmax = h->cfg.max_outer;
  P.precond = h->cfg.precond;
  P.eps = h->cfg.eps;
  P.tau = h->cfg.outer_tol;
  P.eta2 = h->cfg.pcg_rtol * h->cfg.pcg_rtol;
  P.test_flags = h->test_flags;
  // rounding slack of the monotone-objective check: F_eps is summed in FP64
  // from FP32 (or FP64) terms
  P.mono_slack = (h->test_flags & TEST_NONMONOTONE) ? -1.0 : (h->fp64 ? 1e-12 : 1e-6);
  const int R = band_rows(s.n);
  // partials per slot: one per workgroup, over the rows of every contrast
  P.npq = s.C * (s.n / R + (s.psi == PSI_HAAR ? s.n / strip_cols(h->fp64, s.n) : 0));
  P.ndata = s.C * (s.n / strip_cols(h->fp64, s.n));
  P.nrz = s.C * (s.psi == PSI_HAAR ? s.n / R : (s.n / TV_TR) * (s.n / TV_TC));
  if (s.dense) {
    // the A x / A p products write one partial per row tile
    P.ndata = s.Mp / GEMM_BM;
    P.npq = s.n / R + (s.psi == PSI_HAAR ? s.Mp / GEMM_BM : 0);
    P.pq_gemm = s.psi == PSI_HAAR ? 1 : 0;
  }
  P.nreg = (s.n_groups + GROUPS_PER_WG - 1) / GROUPS_PER_WG;
  (void)shape_id;
  return P;
}

#define LAUNCH(fn, P, grid, st)                                                         \
  do {                                                                                  \
    hipError_t e_ = (fn)((P), (grid), (st));                                            \
    if (e_ != hipSuccess) return fail(FIRLS_E_HIP, std::string("launch ") + #fn + ": " + hipGetErrorString(e_)); \
  } while (0)

hipEvent_t prof_event(firls_handle* h) {
  if (h->ev_used == h->ev_pool.size()) {
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    h->ev_pool.push_back(e);
  }
  return h->ev_pool[h->ev_used++];
}

struct TimingScope {   // launch_timing() set for one launcher call
  TimingScope(hipEvent_t a, hipEvent_t b) { launch_timing() = {a, b}; }
  ~TimingScope() { launch_timing() = {nullptr, nullptr}; }
};

// Launch with optional timing (the kernel's own start and end);
// ``cls`` is a FIRLS_PROF_* class.
#define KLAUNCH(h, cls, fn, P, grid, st)                                                \
  do {                                                                                  \
    if ((h)->rec_seq) {                                                                 \
      (h)->rec_seq->push_back({(fn), (P), (grid), (cls)});                              \
      break;                                                                            \
    }                                                                                   \
    hipEvent_t a_ = nullptr, b_ = nullptr;                                              \
    if ((h)->profiling) {                                                               \
      a_ = prof_event(h);                                                               \
      b_ = prof_event(h);                                                               \
      if (!a_ || !b_) a_ = b_ = nullptr;                                                \
    }                                                                                   \
    {                                                                                   \
      TimingScope ts_(a_, b_);                                                          \
      LAUNCH(fn, P, grid, st);                                                          \
    }                                                                                   \
    if (a_ && b_)                                                                       \
      (h)->recs.push_back({(cls), (h)->ctx_group, (h)->ctx_it, (h)->ctx_phase, (h)->ctx_count, a_, b_}); \
  } while (0)

// Weights of the current x: |Psi x|^2, W per group (+ penalty partials), d.
// ``penalty_only``: the penalty partials without d (enough for F_eps); with
// band-local groups one pass from x (the callers then read s.row_wgs()
// partials, P.nreg).
int launch_weights(firls_handle* h, const Shape& s, const Params& P, int c, hipStream_t st,
                   bool penalty_only = false) {
  const PrecKernels* pk = prec_kernels(h->fp64);
  if (penalty_only && s.psi == PSI_HAAR && s.d_bgptr && !s.dense) {
    KLAUNCH(h, FIRLS_PROF_GROUP_W, s.sk->rowfwd[RF_PEN_HAAR], P, dim3(s.row_wgs(), c), st);
    return FIRLS_OK;
  }
  if (s.psi == PSI_HAAR) KLAUNCH(h, FIRLS_PROF_PSI_SQ, s.sk->psi_sq_haar, P, dim3(s.row_wgs(), c), st);
  else KLAUNCH(h, FIRLS_PROF_PSI_SQ, pk->psi_sq_tv, P, dim3(((int)s.pixels() + 4 * NT - 1) / (4 * NT), c), st);
  KLAUNCH(h, FIRLS_PROF_GROUP_W, pk->group_w, P, dim3(P.nreg, c), st);
  if (!penalty_only)
    KLAUNCH(h, FIRLS_PROF_GROUP_D, pk->group_d, P, dim3((s.n_coef + 4 * NT - 1) / (4 * NT), c), st);
  return FIRLS_OK;
}

// Weights and residual of the current x, then the objective check (one
// outer iteration's preparation).  Haar: the row FFT of x also writes
// |Phi x|^2, and the row-inverse pass of r0 = A^H b - S x also sums
// <r0, z0>; TV: |D x|^2, weights, the residual passes and z0 = M^{-1} r0.
// Split-K factor of a dense-matrix GEMM: enough workgroups to fill the
// device (about 1024), a power of two dividing the K steps, at most 8.
struct GemmPlan {
  int rows, K, ct, split;
  size_t scratch;   // bytes of partial tiles (0 without a split)
};
GemmPlan gemm_plan(const firls_handle* h, const Shape& s, int mode, int c) {
  GemmPlan g{};
  const bool trans = mode == G_ATB || mode == G_ATY;
  g.rows = trans ? s.n * s.n : s.Mp;
  g.K = trans ? s.Mp : s.n * s.n;
  g.ct = (c + GEMM_BS - 1) / GEMM_BS;
  const int tiles = g.rows / GEMM_BM * g.ct, steps = g.K / GEMM_BK;
  g.split = 1;
  while (g.split < 8 && tiles * g.split < 1024 && steps % (2 * g.split) == 0) g.split *= 2;
  g.scratch = g.split > 1 ? (size_t)g.split * g.rows * g.ct * 2 * GEMM_BS * h->relt : 0;
  return g;
}

// Scratch for every GEMM of c slices of a dense shape (before any capture).
int ensure_gemm_scratch(firls_handle* h, hipStream_t st, const Shape& s, int c) {
  size_t need = 0;
  for (int m = 0; m < 4; ++m) need = std::max(need, gemm_plan(h, s, m, c).scratch);
  if (need <= h->gscr_cap) return FIRLS_OK;
  drop_graphs(h);
  HIPCHK(hipStreamSynchronize(st));
  if (h->gscr) HIPCHK(hipFree(h->gscr));
  h->gscr = nullptr;
  h->gscr_cap = 0;
  if (hipMalloc(&h->gscr, need) != hipSuccess) {
    (void)hipGetLastError();
    return fail(FIRLS_E_NOMEM, "GEMM scratch allocation failed");
  }
  h->gscr_cap = need;
  return FIRLS_OK;
}

int launch_gemm(firls_handle* h, const Shape& s, Params P, int mode, int c, hipStream_t st, int cls) {
  const GemmPlan g = gemm_plan(h, s, mode, c);
  if (g.scratch > h->gscr_cap) return fail(FIRLS_E_INVALID, "GEMM scratch not prepared");
  P.count = c;
  P.gsplit = g.split;
  P.gscr = h->gscr;
  KLAUNCH(h, cls, gemm_kernels(h->fp64)->g[mode], P, dim3(g.rows / GEMM_BM, g.ct), st);
  return FIRLS_OK;
}

// A x - b and A^T (b - A x) for a dense sensing matrix (the data term and
// the A^H part of r0), in place of the row FFT and column pass.
int launch_dense_residual(firls_handle* h, const Shape& s, Params P, int c, hipStream_t st) {
  int rc = launch_gemm(h, s, P, G_AX_R0, c, st, FIRLS_PROF_R0_COL);
  return rc ? rc : launch_gemm(h, s, P, G_ATY, c, st, FIRLS_PROF_R0_COL);
}

// q's A^T A p part for a dense sensing matrix: y = A p, t = A^T y.
int launch_dense_normal(firls_handle* h, const Shape& s, Params P, int c, hipStream_t st) {
  int rc = launch_gemm(h, s, P, G_AP, c, st, FIRLS_PROF_COL);
  return rc ? rc : launch_gemm(h, s, P, G_ATY, c, st, FIRLS_PROF_COL);
}

// The fused Haar PCG's closing x += alpha p rides in the next residual row
// pass when that pass is the band-local weights pass (every PCG is followed
// by a preparation: the stop test comes after the residual).
bool fold_last_x(const firls_handle* h, const Shape& s) {
  return s.psi == PSI_HAAR && h->cfg.precond == FIRLS_PC_PAPER && s.d_bgptr && !s.dense;
}

// With the paper's preconditioner and the FFT operator, the residual's
// row-inverse pass also forms z0, p0 = z0 and the row FFTs of p0, which is
// all the first PCG iteration's row pass would do.
bool p0_in_prep(const firls_handle* h, const Shape& s) {
  return s.psi == PSI_HAAR && h->cfg.precond == FIRLS_PC_PAPER && !s.dense;
}

// Weights, residual and data term of the current x, then the objective
// check (one outer iteration's preparation).
int launch_prep(firls_handle* h, const Shape& s, const Params& P0, int c, hipStream_t st) {
  const PrecKernels* pk = prec_kernels(h->fp64);
  const dim3 rows(s.row_wgs(), c);
  Params P = P0;
  P.p0_prep = p0_in_prep(h, s) ? 1 : 0;
  // Haar: the residual's row-inverse pass, the last of the preparation,
  // also runs the stop test (TV keeps its own launch after the z0 pass)
  P.check_r0 = s.psi == PSI_HAAR ? 1 : 0;
  if (s.dense) {
    int rc = launch_weights(h, s, P, c, st);
    if (rc || (rc = launch_dense_residual(h, s, P, c, st))) return rc;
    if (s.psi == PSI_HAAR) {
      KLAUNCH(h, FIRLS_PROF_R0_ROWINV, s.sk->rowinv[P.p0_prep ? RI_R0_HAAR_P0 : RI_R0_HAAR], P, rows, st);
    } else {
      KLAUNCH(h, FIRLS_PROF_R0_ROWINV, s.sk->rowinv[RI_R0_TV], P, rows, st);
      KLAUNCH(h, FIRLS_PROF_R0_UPDATE, pk->update_tv[UP_INIT], P, dim3(P.nrz, c), st);
    }
  } else if (s.psi == PSI_HAAR && s.d_bgptr) {
    // band-local groups: weights inside the residual's row pass, which also
    // applies the last PCG step's x update
    P.nreg = s.row_wgs();
    P.fold_x = fold_last_x(h, s) ? 1 : 0;
    P.k = h->cfg.pcg_iters - 1;
    KLAUNCH(h, FIRLS_PROF_R0_ROWFWD, s.sk->rowfwd[RF_SQW_HAAR], P, rows, st);
    KLAUNCH(h, FIRLS_PROF_R0_COL, s.sk->col[COL_R0], P, dim3(s.col_wgs(h->fp64), c), st);
    KLAUNCH(h, FIRLS_PROF_R0_ROWINV, s.sk->rowinv[P.p0_prep ? RI_R0_HAAR_P0 : RI_R0_HAAR], P, rows, st);
  } else if (s.psi == PSI_HAAR) {
    KLAUNCH(h, FIRLS_PROF_R0_ROWFWD, s.sk->rowfwd[RF_SQ_HAAR], P, rows, st);
    KLAUNCH(h, FIRLS_PROF_GROUP_W, pk->group_w, P, dim3(P.nreg, c), st);
    KLAUNCH(h, FIRLS_PROF_GROUP_D, pk->group_d, P, dim3((s.n_coef + 4 * NT - 1) / (4 * NT), c), st);
    KLAUNCH(h, FIRLS_PROF_R0_COL, s.sk->col[COL_R0], P, dim3(s.col_wgs(h->fp64), c), st);
    KLAUNCH(h, FIRLS_PROF_R0_ROWINV, s.sk->rowinv[P.p0_prep ? RI_R0_HAAR_P0 : RI_R0_HAAR], P, rows, st);
  } else {
    int rc = launch_weights(h, s, P, c, st);
    if (rc) return rc;
    KLAUNCH(h, FIRLS_PROF_R0_ROWFWD, s.sk->rowfwd[RF_PLAIN], P, rows, st);
    KLAUNCH(h, FIRLS_PROF_R0_COL, s.sk->col[COL_R0], P, dim3(s.col_wgs(h->fp64), c), st);
    KLAUNCH(h, FIRLS_PROF_R0_ROWINV, s.sk->rowinv[RI_R0_TV], P, rows, st);
    KLAUNCH(h, FIRLS_PROF_R0_UPDATE, pk->update_tv[UP_INIT], P, dim3(P.nrz, c), st);
  }
  if (!P.check_r0) KLAUNCH(h, FIRLS_PROF_CHECK, pk->outer_check, P, dim3(c), st);
  return FIRLS_OK;
}

// K PCG iterations.  Haar with the paper's preconditioner: 3 launches per
// iteration (the update of one iteration rides in the row pass of the
// next) and x += alpha p at the end; with the paired pass 2 (the row
// inverse rides in the next step's launch, and the last iteration's
// <p, S p> share in its own): 2K - 1 in all when the residual pass has
// prepared p0.  Haar with the Jacobi or identity preconditioner, and TV:
// 4 launches per iteration in the textbook order.
int launch_pcg(firls_handle* h, const Shape& s, Params P, int c, hipStream_t st) {
  const PrecKernels* pk = prec_kernels(h->fp64);
  const bool haar = s.psi == PSI_HAAR;
  const bool fused = haar && h->cfg.precond == FIRLS_PC_PAPER;
  const dim3 rows(s.row_wgs(), c);
  const int K = h->cfg.pcg_iters;
  // the row inverse of iteration k - 1 rides in the launch of step k
  const bool pair = fused && !s.dense && s.sk->pcg_pair && h->use_pair;
  for (int k = 0; k < K; ++k) {
    P.k = k;
    if (fused) {
      if (k > 0 && pair) KLAUNCH(h, FIRLS_PROF_UPDATE, s.sk->pcg_pair, P, rows, st);
      else if (k > 0) KLAUNCH(h, FIRLS_PROF_UPDATE, s.sk->rowfwd[RF_STEP_HAAR], P, rows, st);
      else if (!p0_in_prep(h, s)) KLAUNCH(h, FIRLS_PROF_ROWFWD, s.sk->rowfwd[RF_PCG_HAAR], P, rows, st);
    } else if (haar) {
      KLAUNCH(h, FIRLS_PROF_ROWFWD, s.sk->rowfwd[RF_PCG_HAAR], P, rows, st);
    } else {
      KLAUNCH(h, FIRLS_PROF_ROWFWD, s.sk->rowfwd[RF_PCG_Z], P, rows, st);
    }
    if (s.dense) {
      int rc = launch_dense_normal(h, s, P, c, st);
      if (rc) return rc;
    } else {
      KLAUNCH(h, FIRLS_PROF_COL, s.sk->col[haar ? COL_SP_PQ : COL_SP], P, dim3(s.col_wgs(h->fp64), c), st);
    }
    // the fused step reads q of iterations 0 .. K-2 only; the paired pass
    // of the last iteration also forms that iteration's <p, S p> partials,
    // so with K >= 2 no row-inverse launch is left, except in a sequence
    // recorded for launches across shapes, whose paired kernel leaves that
    // sum to the row inverse
    if (!pair || (k == K - 1 && (K == 1 || h->rec_seq))) {
      P.q_dead = fused && k == K - 1 ? 1 : 0;
      KLAUNCH(h, FIRLS_PROF_ROWINV, s.sk->rowinv[haar ? RI_SP_HAAR : RI_SP_TV], P, rows, st);
      P.q_dead = 0;
    }
    if (haar && !fused) KLAUNCH(h, FIRLS_PROF_UPDATE, s.sk->update_haar, P, rows, st);
    if (!haar) KLAUNCH(h, FIRLS_PROF_UPDATE, pk->update_tv[UP_STEP], P, dim3(P.nrz, c), st);
  }
  if (fused && !fold_last_x(h, s)) {
    P.k = K - 1;
    KLAUNCH(h, FIRLS_PROF_LAST_X, s.sk->last_x, P, rows, st);
  }
  return FIRLS_OK;
}

// Fold the timed launches of one run_batch into the per-class totals.
// Units are active slices: a launch at outer iteration ``it`` counts the
// slices of its group still active when it ran.
// act_prep[it]: slots of each shape active entering iteration it's
// residual pass (it >= 1); act_pcg[it]: active in its PCG iterations.
int prof_collect(firls_handle* h, const std::vector<std::vector<int>>& act_pcg,
                 const std::vector<std::vector<int>>& act_prep) {
  for (const auto& r : h->recs) {
    float ms = 0.f;   // records without events: the other shapes of a launch across shapes
    if (r.a && r.b) HIPCHK(hipEventElapsedTime(&ms, r.a, r.b));
    int units = r.count;
    if (r.phase == 1 && r.it > 0) units = act_prep[r.it][r.group];
    if (r.phase == 2) units = act_pcg[r.it][r.group];
    // a launch across shapes has one record per shape; the first carries
    // its time and counts the launch
    const int launches = r.a ? 1 : 0;
    h->prof_ms[r.cls] += ms;
    h->prof_launches[r.cls] += launches;
    h->prof_units[r.cls] += units;
    const size_t k = (size_t)r.group * FIRLS_PROF_CLASSES + r.cls;
    if (r.group >= 0 && k < h->prof_ms_shape.size()) {
      h->prof_ms_shape[k] += ms;
      h->prof_launches_shape[k] += launches;
      h->prof_units_shape[k] += units;
    }
  }
  h->recs.clear();
  h->ev_used = 0;
  return FIRLS_OK;
}

int check_slice(const firls_handle* h, const firls_slice& sl) {
  if (sl.shape_id < 0 || sl.shape_id >= (int)h->shapes.size()) return fail(FIRLS_E_INVALID, "shape_id out of range");
  if (!(sl.lambda > 0.0) || !std::isfinite(sl.lambda)) return fail(FIRLS_E_INVALID, "lambda must be positive and finite");
  if (!sl.b || !sl.x) return fail(FIRLS_E_INVALID, "b and x must be device pointers");
  if (!sl.mask && !h->shapes[sl.shape_id].dense) return fail(FIRLS_E_INVALID, "mask must be a device pointer");
  return FIRLS_OK;
}

// ---- launches across shapes ------------------------------------------------
// A batch of several shapes runs each position of its outer iteration (the
// k-th launch of the weights and residual passes, the k-th launch of the
// PCG iterations) as one launch per kernel class and mode covering every
// shape: the per-shape launch sequences are recorded, then merged position
// by position.  Within a shape the order is unchanged, and shapes never
// depend on each other, so only the launch count changes (a batch of ten
// shapes needs about a tenth of the launches).

// Which kernel class and mode a recorded per-shape launcher is.
bool multi_class_of(const firls_handle* h, const Shape& S, Launcher fn, int& cls, int& mode) {
  const SizeKernels* sk = S.sk;
  const PrecKernels* pk = prec_kernels(h->fp64);
  auto hit = [&](Launcher cand, int c, int m) {
    if (!cand || cand != fn) return false;
    cls = c;
    mode = m;
    return true;
  };
  for (int m = 0; m < 7; ++m)
    if (hit(sk->rowfwd[m], MC_ROWFWD, m)) return true;
  for (int m = 0; m < 5; ++m)
    if (hit(sk->col[m], MC_COL, m)) return true;
  for (int m = 0; m < 6; ++m)
    if (hit(sk->rowinv[m], MC_ROWINV, m)) return true;
  // the paired pass of sides above 256 (two tile columns per thread) has a
  // kernel of its own across shapes
  return hit(sk->pcg_pair, MC_PAIR, S.n > 256 ? 1 : 0) || hit(sk->psi_sq_haar, MC_PSI_SQ_HAAR, 0) ||
         hit(sk->update_haar, MC_UPDATE_HAAR, 0) || hit(sk->last_x, MC_LAST_X, 0) ||
         hit(pk->psi_sq_tv, MC_PSI_SQ_TV, 0) || hit(pk->group_w, MC_GROUP_W, 0) || hit(pk->group_d, MC_GROUP_D, 0) ||
         hit(pk->update_tv[UP_INIT], MC_UPDATE_TV, UP_INIT) || hit(pk->update_tv[UP_STEP], MC_UPDATE_TV, UP_STEP) ||
         hit(pk->outer_check, MC_OUTER_CHECK, 0);
}

struct MultiLaunch {
  int cls, mode, prof_cls;
  int item0, items;
  size_t lds;
  std::vector<std::pair<int, int>> groups;   // (shape, slices) it covers
};
struct MultiPlan {
  std::vector<MultiLaunch> prep, pcg;
};

// Records the per-shape sequences of one outer iteration, merges them
// position by position and uploads the Params table and the work items.
// Returns 1 (plan built), 0 (some launch has no cross-shape kernel: the
// caller launches per shape) or an error.
int build_multi_plan(firls_handle* h, hipStream_t st, const std::vector<std::vector<int>>& by_shape,
                     const std::vector<int>& lo, int Tmax, double tau, MultiPlan& plan) {
  const int nsh = (int)h->shapes.size();
  std::vector<std::vector<firls_handle::LaunchRec>> seq[2];
  seq[0].resize(nsh);
  seq[1].resize(nsh);
  for (int sh = 0; sh < nsh; ++sh) {
    const int c = (int)by_shape[sh].size();
    if (!c) continue;
    const Shape& S = h->shapes[sh];
    Params P = base_params(h, S, sh, h->d_list + lo[sh]);
    P.Tmax = Tmax;
    P.tau = tau;
    P.stop_flags = h->d_flags;
    h->rec_seq = &seq[0][sh];
    int rc = launch_prep(h, S, P, c, st);
    if (!rc) {
      h->rec_seq = &seq[1][sh];
      rc = launch_pcg(h, S, base_params(h, S, sh, h->d_list + lo[sh]), c, st);
    }
    h->rec_seq = nullptr;
    if (rc) return rc;
  }
  // the order of the shapes' items within every launch
  std::vector<int> order;
  for (int sh = 0; sh < nsh; ++sh)
    if (!by_shape[sh].empty()) order.push_back(sh);
  if (h->schedule == FIRLS_SCHED_ACROSS_LARGEST_FIRST)
    std::stable_sort(order.begin(), order.end(),
                     [&](int a, int b) { return h->shapes[a].pixels() > h->shapes[b].pixels(); });
  const MultiKernels* mk = multi_kernels(h->fp64);
  std::vector<Params> params;
  std::vector<MultiItem> items;
  for (int ph = 0; ph < 2; ++ph) {
    std::vector<MultiLaunch>& out = ph == 0 ? plan.prep : plan.pcg;
    out.clear();
    size_t len = 0;
    for (int sh : order) len = std::max(len, seq[ph][sh].size());
    for (size_t pos = 0; pos < len; ++pos) {
      std::vector<MultiLaunch> bucket;
      std::vector<std::vector<MultiItem>> bucket_items;
      for (int sh : order) {
        if (pos >= seq[ph][sh].size()) continue;
        const firls_handle::LaunchRec& r = seq[ph][sh][pos];
        int cls = 0, mode = 0;
        if (!multi_class_of(h, h->shapes[sh], r.fn, cls, mode) || !mk->fn[cls][mode]) return 0;
        size_t b = 0;
        while (b < bucket.size() && !(bucket[b].cls == cls && bucket[b].mode == mode)) ++b;
        if (b == bucket.size()) {
          bucket.push_back(MultiLaunch{cls, mode, r.cls, 0, 0, 0, {}});
          bucket_items.emplace_back();
        }
        const int pidx = (int)params.size();
        params.push_back(r.P);
        const int32_t* list = h->h_list + lo[sh];
        std::vector<MultiItem>& mine = bucket_items[b];
        if (cls == MC_OUTER_CHECK) {   // one workgroup per slice, indexed by x
          for (unsigned x = 0; x < r.grid.x; ++x) mine.push_back(MultiItem{list[x], 0, pidx});
        } else {                       // grid (blocks of a slice, slices)
          for (unsigned y = 0; y < r.grid.y; ++y)
            for (unsigned x = 0; x < r.grid.x; ++x) mine.push_back(MultiItem{list[y], (int32_t)x, pidx});
        }
        bucket[b].groups.push_back({sh, (int)by_shape[sh].size()});
        bucket[b].lds = std::max(bucket[b].lds, multi_lds_bytes(h->fp64, cls, h->shapes[sh].n));
      }
      for (size_t b = 0; b < bucket.size(); ++b) {
        bucket[b].item0 = (int)items.size();
        bucket[b].items = (int)bucket_items[b].size();
        items.insert(items.end(), bucket_items[b].begin(), bucket_items[b].end());
        out.push_back(bucket[b]);
      }
    }
  }
  // device copies (grown as needed; a graph captured on the old ones is dropped)
  auto grow = [&](void** ptr, size_t& cap, size_t bytes) -> int {
    if (bytes <= cap) return FIRLS_OK;
    drop_graphs(h);
    HIPCHK(hipStreamSynchronize(st));
    if (*ptr) HIPCHK(hipFree(*ptr));
    *ptr = nullptr;
    cap = 0;
    if (hipMalloc(ptr, bytes) != hipSuccess) {
      (void)hipGetLastError();
      return fail(FIRLS_E_NOMEM, "work table allocation failed");
    }
    cap = bytes;
    return FIRLS_OK;
  };
  int rc = grow(reinterpret_cast<void**>(&h->d_mparams), h->mparams_cap, params.size() * sizeof(Params));
  if (!rc) rc = grow(reinterpret_cast<void**>(&h->d_mitems), h->mitems_cap, items.size() * sizeof(MultiItem));
  if (rc) return rc;
  HIPCHK(hipMemcpyAsync(h->d_mparams, params.data(), params.size() * sizeof(Params), hipMemcpyHostToDevice, st));
  HIPCHK(hipMemcpyAsync(h->d_mitems, items.data(), items.size() * sizeof(MultiItem), hipMemcpyHostToDevice, st));
  // the copies come from host vectors that end here
  HIPCHK(hipStreamSynchronize(st));
  return 1;
}

// One merged launch list (timed per launch like KLAUNCH; the time goes to
// the first shape it covers, the others get their slice counts).
int launch_multi_list(firls_handle* h, const std::vector<MultiLaunch>& L, hipStream_t st) {
  const MultiKernels* mk = multi_kernels(h->fp64);
  for (const MultiLaunch& m : L) {
    hipEvent_t a_ = nullptr, b_ = nullptr;
    if (h->profiling) {
      a_ = prof_event(h);
      b_ = prof_event(h);
      if (!a_ || !b_) a_ = b_ = nullptr;
    }
    const MultiArgs A{h->d_mparams, h->d_mitems + m.item0};
    {
      TimingScope ts_(a_, b_);
      const hipError_t e = mk->fn[m.cls][m.mode](A, m.items, m.lds, st);
      if (e != hipSuccess) return fail(FIRLS_E_HIP, std::string("launch across shapes: ") + hipGetErrorString(e));
    }
    if (a_ && b_) {
      for (size_t g = 0; g < m.groups.size(); ++g)
        h->recs.push_back({m.prof_cls, m.groups[g].first, h->ctx_it, h->ctx_phase, m.groups[g].second,
                           g == 0 ? a_ : nullptr, g == 0 ? b_ : nullptr});
    }
  }
  return FIRLS_OK;
}

// The batched outer loop shared by every solve entry point.  The first
// ``slots`` slices start at once.  With slots < ns (a streamed batch: one
// masked-FFT shape) each slot takes the next queued slice as soon as its
// own slice stops, so a sub-batch never idles behind its slowest slice;
// the final states of finished slices are kept behind the slot states.
int run_chunk(firls_handle* h, hipStream_t st, int slots, int ns, const firls_slice* sl, firls_report* rep, int Tmax,
              double tau) {
  if (ns <= 0 || slots <= 0 || slots > ns) return fail(FIRLS_E_INVALID, "n_slices must be positive");
  if (slots > h->cfg.max_slices) return fail(FIRLS_E_INVALID, "n_slices exceeds max_slices");
  if (!sl || !rep) return fail(FIRLS_E_INVALID, "slices and reports must be non-null");
  for (int i = 0; i < ns; ++i) {
    int rc = check_slice(h, sl[i]);
    if (rc) return rc;
  }
  const bool streamed = slots < ns;
  if (streamed) {
    for (int i = 1; i < ns; ++i)
      if (sl[i].shape_id != sl[0].shape_id) return fail(FIRLS_E_INVALID, "a streamed batch needs one shape");
    if (h->shapes[sl[0].shape_id].dense) return fail(FIRLS_E_INVALID, "a streamed batch needs a masked-FFT shape");
  }
  std::vector<size_t> off(slots);
  size_t need = 0;
  for (int i = 0; i < slots; ++i) {
    off[i] = need;
    need += h->slice_bytes(h->shapes[sl[i].shape_id]);
  }
  int rc = ensure_capacity(h, st, need, streamed ? slots + ns : slots);
  if (rc) return rc;
  HIPCHK(hipStreamSynchronize(st));  // pinned staging below may still feed an earlier copy
  const int nsh = (int)h->shapes.size();
  std::vector<std::vector<int>> by_shape(nsh), zf_by_shape(nsh);
  for (int i = 0; i < slots; ++i) {
    fill_desc(h, h->h_desc[i], h->shapes[sl[i].shape_id], off[i], &sl[i]);
    h->h_desc[i].shape = sl[i].shape_id;
    by_shape[sl[i].shape_id].push_back(i);
    if (!sl[i].x_is_init) zf_by_shape[sl[i].shape_id].push_back(i);
  }
  std::vector<int> lo(nsh), zlo(nsh);
  int pos = 0;
  for (int s = 0; s < nsh; ++s) {
    lo[s] = pos;
    for (int i : by_shape[s]) h->h_list[pos++] = i;
  }
  for (int s = 0; s < nsh; ++s) {
    zlo[s] = pos;
    for (int i : zf_by_shape[s]) h->h_list[pos++] = i;
  }
  for (int s = 0; s < nsh; ++s)
    if (h->shapes[s].dense && !by_shape[s].empty() &&
        (rc = ensure_gemm_scratch(h, st, h->shapes[s], (int)by_shape[s].size())))
      return rc;
  HIPCHK(hipMemcpyAsync(h->d_desc, h->h_desc, sizeof(SliceDesc) * slots, hipMemcpyHostToDevice, st));
  HIPCHK(hipMemcpyAsync(h->d_list, h->h_list, sizeof(int32_t) * pos, hipMemcpyHostToDevice, st));

  const PrecKernels* pk = prec_kernels(h->fp64);
  std::vector<std::vector<int>> act_pcg, act_prep(1);
  h->ctx_phase = 0;
  h->ctx_it = 0;
  h->ctx_group = 0;
  // x^1 = A^H b for slices without a warm start (Section 3.3); ``list``
  // holds the c descs of shape s that need it
  auto launch_ahb = [&](int s, const int32_t* list, int c) -> int {
    const Shape& S = h->shapes[s];
    Params P = base_params(h, S, s, list);
    h->ctx_group = s;
    h->ctx_count = c;
    if (S.dense) return launch_gemm(h, S, P, G_ATB, c, st, FIRLS_PROF_AHB);
    KLAUNCH(h, FIRLS_PROF_AHB, S.sk->col[COL_AHB], P, dim3(S.col_wgs(h->fp64), c), st);
    KLAUNCH(h, FIRLS_PROF_AHB, S.sk->rowinv[RI_PLAIN], P, dim3(S.row_wgs(), c), st);
    return FIRLS_OK;
  };
  // Streamed batches: A^H b of every queued zero-filled slice up front, in
  // groups of ``slots`` that borrow the slots' workspaces before the loop
  // starts (descs behind the slots' ones, the list behind the refill list),
  // as a few full launches instead of a small pair at each refill; those
  // slices then enter their slots with x already set.
  std::vector<char> x_ready(ns, 0);
  if (streamed) {
    const int s0 = sl[0].shape_id;
    const Shape& S = h->shapes[s0];
    int32_t* hl = h->h_list + 3 * slots;
    int nq = 0;
    for (int i = slots; i < ns; ++i) {
      if (sl[i].x_is_init) continue;
      fill_desc(h, h->h_desc[i], S, off[nq % slots], &sl[i]);
      h->h_desc[i].shape = s0;
      hl[nq++] = i;
      x_ready[i] = 1;
    }
    if (nq) {
      HIPCHK(hipMemcpyAsync(h->d_desc + slots, h->h_desc + slots, sizeof(SliceDesc) * (ns - slots),
                            hipMemcpyHostToDevice, st));
      HIPCHK(hipMemcpyAsync(h->d_list + 3 * slots, hl, sizeof(int32_t) * nq, hipMemcpyHostToDevice, st));
      for (int g0 = 0; g0 < nq; g0 += slots) {
        const int c = std::min(slots, nq - g0);
        const int32_t* list = h->d_list + 3 * slots + g0;
        h->ctx_group = s0;
        h->ctx_count = c;
        Params P = base_params(h, S, s0, list);   // states of these descs: the final-state area, unused yet
        KLAUNCH(h, FIRLS_PROF_INIT, pk->slice_init, P, dim3(c), st);
        if ((rc = launch_ahb(s0, list, c))) return rc;
      }
    }
  }
  h->ctx_group = 0;
  h->ctx_count = slots;
  // Stop words start as active; a slice rejected at its start (a TV mask
  // without DC) writes its word as stopped.  The host's own stores must
  // come first, so they happen before the launch.
  for (int i = 0; i < slots; ++i) __atomic_store_n(h->h_flags + i, 1, __ATOMIC_RELAXED);
  {
    Params P = base_params(h, h->shapes[0], 0, h->d_list);
    P.stop_flags = h->d_flags;
    KLAUNCH(h, FIRLS_PROF_INIT, pk->slice_init, P, dim3(slots), st);
  }
  for (int s = 0; s < nsh; ++s)
    if (!zf_by_shape[s].empty() && (rc = launch_ahb(s, h->d_list + zlo[s], (int)zf_by_shape[s].size()))) return rc;
  // several masked-FFT shapes at once: one launch per class and position
  // across the shapes (the schedule chosen by firls_set_schedule or the
  // autotuner)
  MultiPlan mplan;
  bool multi = false;
  {
    int present = 0;
    bool dense = false;
    for (int s = 0; s < nsh; ++s)
      if (!by_shape[s].empty()) {
        ++present;
        dense = dense || h->shapes[s].dense;
      }
    if (h->schedule != FIRLS_SCHED_PER_SHAPE && present >= 2 && !dense && !streamed && !h->noalloc) {
      rc = build_multi_plan(h, st, by_shape, lo, Tmax, tau, mplan);
      if (rc < 0) return rc;
      multi = rc == 1;
    }
  }
  auto enqueue_prep = [&]() -> int {
    if (multi) return launch_multi_list(h, mplan.prep, st);
    for (int s = 0; s < nsh; ++s) {
      const int c = (int)by_shape[s].size();
      if (!c) continue;
      const Shape& S = h->shapes[s];
      Params P = base_params(h, S, s, h->d_list + lo[s]);
      P.Tmax = Tmax;
      P.tau = tau;
      P.stop_flags = h->d_flags;
      h->ctx_group = s;
      h->ctx_count = c;
      int r2;
      if ((r2 = launch_prep(h, S, P, c, st))) return r2;
    }
    return FIRLS_OK;
  };
  auto enqueue_pcg = [&]() -> int {
    if (multi) return launch_multi_list(h, mplan.pcg, st);
    for (int s = 0; s < nsh; ++s) {
      const int c = (int)by_shape[s].size();
      if (!c) continue;
      const Shape& S = h->shapes[s];
      Params P = base_params(h, S, s, h->d_list + lo[s]);
      h->ctx_group = s;
      h->ctx_count = c;
      int r2;
      if ((r2 = launch_pcg(h, S, P, c, st))) return r2;
    }
    return FIRLS_OK;
  };
  // Every outer iteration launches the same kernels with the same arguments,
  // so one iteration is captured once as a graph and replayed.
  const bool graphs = h->use_graphs && !h->profiling && st != nullptr;
  if (graphs) {
    firls_handle::GraphKey key;
    for (int s = 0; s < nsh; ++s) key.counts.push_back((int)by_shape[s].size());
    key.Tmax = Tmax;
    key.tau = tau;
    key.ws = h->ws;
    key.desc = h->d_desc;
    key.stream = st;
    key.multi = multi ? h->schedule : 0;
    if (!(key == h->gkey) || !h->g_iter) {
      drop_graphs(h);
      hipGraph_t g = nullptr;
      HIPCHK(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
      rc = enqueue_prep();
      if (!rc) rc = enqueue_pcg();
      hipError_t e = hipStreamEndCapture(st, &g);
      if (rc) {
        if (g) (void)hipGraphDestroy(g);
        return rc;
      }
      HIPCHK(e);
      e = hipGraphInstantiate(&h->g_iter, g, nullptr, nullptr, 0);
      (void)hipGraphDestroy(g);
      HIPCHK(e);
      h->gkey = key;
    }
  }
  // The outer check of each slot writes (evaluations << 1) | active to host
  // memory at the start of every iteration.  Before launching iteration it
  // the host polls for iteration it - 1's words, so the GPU works through
  // that iteration's PCG launches meanwhile; once no slot is active (and no
  // slice is queued) nothing more is launched, and only the PCG launches of
  // the last iteration run empty (kernels of stopped slices exit at once).
  // A slot refilled at iteration k has made it - k evaluations by then.
  std::vector<int> slot_slice(slots), start_it(slots, 0), fin(ns, -1);
  std::vector<char> settled(slots, 0);   // stopped, queue empty: its slice's state stays in the slot
  for (int i = 0; i < slots; ++i) slot_slice[i] = i;
  int next = slots;   // next queued slice
  auto read_active = [&](int j, bool& done) {
    done = true;
    for (int i = 0; i < slots && done; ++i) {
      const int32_t w = __atomic_load_n(h->h_flags + i, __ATOMIC_ACQUIRE);
      if ((w & 1) && (w >> 1) <= j - start_it[i]) done = false;
    }
    if (!done) return 0;
    std::vector<int> cnt(nsh, 0);
    int active = 0;
    for (int i = 0; i < slots; ++i) {
      const int32_t w = __atomic_load_n(h->h_flags + i, __ATOMIC_ACQUIRE) & 1;
      active += w;
      cnt[sl[slot_slice[i]].shape_id] += w;
    }
    act_pcg.push_back(cnt);
    return active;
  };
  // Polls until iteration j's outer checks have all reported.  The event
  // recorded after iteration j's launches bounds the wait: once it has
  // completed, every word is final.
  auto wait_checks = [&](int j, int& active) -> int {
    bool done = false;
    for (unsigned spin = 1;; ++spin) {
      active = read_active(j, done);
      if (done) return FIRLS_OK;
      if (spin % 64) continue;
      const hipError_t e = hipEventQuery(h->ev);
      if (e == hipErrorNotReady) continue;
      HIPCHK(e);
      active = read_active(j, done);
      if (done) return FIRLS_OK;
      return fail(FIRLS_E_HIP, "an outer check did not report");
    }
  };
  // Streamed batches: slots whose slice stopped take the next queued slices
  // at once (zero-filled starts first, so they form a prefix of the refill
  // list).  Waiting to refill several slots together measured slower: an
  // iteration's time does not shrink in proportion to its idle slots.
  int32_t* d_refill_list = h->d_list + 2 * slots;
  auto refill = [&](int it, int& count) -> int {
    count = 0;
    std::vector<RefillRec> zf, given;
    for (int i = 0; i < slots; ++i) {
      if (settled[i] || (__atomic_load_n(h->h_flags + i, __ATOMIC_ACQUIRE) & 1)) continue;
      const int old = slot_slice[i];
      if (next >= ns) {
        settled[i] = 1;
        fin[old] = i;
        continue;
      }
      const firls_slice& q = sl[next];
      RefillRec r{q.b, q.mask, q.x, q.lambda, i, old};
      (q.x_is_init || x_ready[next] ? given : zf).push_back(r);
      fin[old] = slots + old;
      slot_slice[i] = next++;
      start_it[i] = it;
      __atomic_store_n(h->h_flags + i, 1, __ATOMIC_RELAXED);
    }
    count = (int)(zf.size() + given.size());
    if (!count) return FIRLS_OK;
    std::copy(zf.begin(), zf.end(), h->h_refill);
    std::copy(given.begin(), given.end(), h->h_refill + zf.size());
    RefillArgs A{h->d_refill, count, slots, h->d_desc, h->d_state, d_refill_list, h->d_flags};
    HIPCHK(launch_refill(A, st));
    h->ctx_phase = 0;
    int r2;
    if (!zf.empty() && (r2 = launch_ahb(sl[0].shape_id, d_refill_list, (int)zf.size()))) return r2;
    return FIRLS_OK;
  };
  const long max_it = (long)ns * (Tmax + 1) + 1;
  for (int it = 0;; ++it) {
    if (it > max_it) return fail(FIRLS_E_HIP, "the outer loop did not end");
    if (it >= 1) {
      int active = 0, added = 0;
      if ((rc = wait_checks(it - 1, active))) return rc;
      if (streamed && (rc = refill(it, added))) return rc;
      if (!active && !added) break;
      std::vector<int> cnt = act_pcg.back();
      cnt[sl[0].shape_id] += added;
      act_prep.push_back(cnt);
    }
    h->ctx_it = it;
    if (graphs) {
      HIPCHK(hipGraphLaunch(h->g_iter, st));
    } else {
      h->ctx_phase = 1;
      if ((rc = enqueue_prep())) return rc;
      h->ctx_phase = 2;
      if ((rc = enqueue_pcg())) return rc;
    }
    HIPCHK(hipEventRecord(h->ev, st));
  }
  HIPCHK(hipStreamSynchronize(st));
  if (h->profiling && (rc = prof_collect(h, act_pcg, act_prep))) return rc;
  for (int i = 0; i < slots; ++i)
    if (!settled[i]) fin[slot_slice[i]] = i;
  const int nstate = streamed ? slots + ns : slots;
  HIPCHK(hipMemcpy(h->h_state, h->d_state, sizeof(SliceState) * nstate, hipMemcpyDeviceToHost));
  int worst = FIRLS_OK;
  for (int i = 0; i < ns; ++i) {
    const SliceState& S = h->h_state[fin[i]];
    firls_report& r = rep[i];
    r.status = S.status;
    r.outer_iters = S.outer;
    r.pcg_iters = S.pcg;
    r.converged = S.converged;
    r.F = S.F;
    r.F_eps = S.Fe;
    r.data = S.data;
    r.rel_change = S.rel;
    if (S.status < 0 && (worst >= 0 || S.status < worst)) worst = S.status;
    else if (worst >= 0 && S.status > worst) worst = S.status;
  }
  if (worst == FIRLS_E_SYNC) g_err = "workgroups of a slice missed a barrier (internal error)";
  else if (worst == FIRLS_E_BREAKDOWN) g_err = "PCG breakdown: <p, S p> <= 0 with a nonzero residual";
  else if (worst == FIRLS_E_INVALID)
    g_err = "a TV slice's mask does not sample the DC entry (its minimiser would not be unique)";
  else if (worst < 0) g_err = "a slice's objective became non-finite";
  return worst;
}

// Runs the slices on the caller's stream, or on the library's own stream
// ordered after the null stream when the caller passes the null stream
// (graphs need a capturable stream).  With a sub-batch size h->chunk below
// the batch size, a batch of one masked-FFT shape is streamed through
// h->chunk slots; other batches run in sub-batches of h->chunk one after
// the other (all at once when 0).
int run_batch(firls_handle* h, hipStream_t st, int ns, const firls_slice* sl, firls_report* rep, int Tmax, double tau) {
  hipStream_t ws = st;
  if (!st && h->use_graphs) {
    if (!h->own) {
      HIPCHK(hipStreamCreateWithFlags(&h->own, hipStreamNonBlocking));
      HIPCHK(hipEventCreateWithFlags(&h->ev_in, hipEventDisableTiming));
    }
    HIPCHK(hipEventRecord(h->ev_in, nullptr));
    HIPCHK(hipStreamWaitEvent(h->own, h->ev_in, 0));
    ws = h->own;
  }
  const int chunk = h->chunk > 0 ? std::min(h->chunk, ns) : ns;
  bool one_shape = ns > 0 && sl != nullptr;
  for (int i = 1; one_shape && i < ns; ++i) one_shape = sl[i].shape_id == sl[0].shape_id;
  int worst = FIRLS_OK;
  if (chunk < ns && one_shape && sl[0].shape_id >= 0 && sl[0].shape_id < (int)h->shapes.size() &&
      !h->shapes[sl[0].shape_id].dense) {
    worst = run_chunk(h, ws, chunk, ns, sl, rep, Tmax, tau);
    if (worst < 0) return worst;
  } else {
    for (int c0 = 0; c0 < ns; c0 += chunk) {
      const int cn = std::min(chunk, ns - c0);
      int rc = run_chunk(h, ws, cn, cn, sl + c0, rep + c0, Tmax, tau);
      if (rc < 0) return rc;
      worst = std::max(worst, rc);
    }
  }
  if (ws != st) HIPCHK(hipStreamSynchronize(ws));
  return worst;
}

int upload_shape(firls_handle* h, const firls_shape& in, Shape& s) {
  const int n = in.n;
  if (!size_supported(n)) return fail(FIRLS_E_UNSUPPORTED, "image side " + std::to_string(n) + " is not built");
  s.n = n;
  s.psi = in.psi;
  s.C = in.channels <= 0 ? 1 : in.channels;
  if (s.C > 64) return fail(FIRLS_E_UNSUPPORTED, "at most 64 contrasts");
  if (in.op == FIRLS_OP_DENSE) {
    // dense sensing matrix: copied, converted to the working precision and
    // padded with zero rows to the GEMM row tile
    if (s.C != 1) return fail(FIRLS_E_UNSUPPORTED, "a dense sensing matrix needs channels = 1");
    if (in.m < 1 || !in.A) return fail(FIRLS_E_INVALID, "a dense sensing matrix needs m >= 1 and A");
    const size_t N = (size_t)n * n;
    s.dense = true;
    s.M = in.m;
    s.Mp = (in.m + GEMM_BM - 1) / GEMM_BM * GEMM_BM;
    if (s.Mp / GEMM_BM > PMAX) return fail(FIRLS_E_UNSUPPORTED, "too many measurements (m > 32768)");
    if (N % GEMM_BM) return fail(FIRLS_E_UNSUPPORTED, "n^2 must be a multiple of " + std::to_string(GEMM_BM));
    double fro = 0.0;
    for (size_t i = 0; i < (size_t)s.M * N; ++i) fro += in.A[i] * in.A[i];
    s.rho_A = fro / (double)N;
    if (!(s.rho_A > 0.0) || !std::isfinite(s.rho_A)) return fail(FIRLS_E_INVALID, "A must be finite and nonzero");
    const size_t bytes = (size_t)s.Mp * N * h->relt;   // real entries
    HIPCHK(hipMalloc(&s.d_A, bytes));
    if (h->fp64) {
      std::vector<double> a((size_t)s.Mp * N, 0.0);
      std::copy(in.A, in.A + (size_t)s.M * N, a.begin());
      HIPCHK(hipMemcpy(s.d_A, a.data(), bytes, hipMemcpyHostToDevice));
    } else {
      std::vector<float> a((size_t)s.Mp * N, 0.f);
      for (size_t i = 0; i < (size_t)s.M * N; ++i) a[i] = (float)in.A[i];
      HIPCHK(hipMemcpy(s.d_A, a.data(), bytes, hipMemcpyHostToDevice));
    }
  } else if (in.op != FIRLS_OP_FOURIER) {
    return fail(FIRLS_E_INVALID, "unknown measurement operator");
  }
  if (in.psi == FIRLS_PSI_HAAR) {
    const int maxL = 4;
    if (in.levels < 1) return fail(FIRLS_E_INVALID, "Haar levels must be >= 1");
    if (in.levels > maxL) return fail(FIRLS_E_UNSUPPORTED, "Haar levels above " + std::to_string(maxL) + " are not built for this precision");
    if (n % (1 << in.levels)) return fail(FIRLS_E_INVALID, "n must be a multiple of 2^levels");
    s.L = in.levels;
    s.n_coef = s.C * n * n;
  } else if (in.psi == FIRLS_PSI_TV || in.psi == FIRLS_PSI_TV_PAPER) {
    if (n % TV_TC || n % TV_TR) return fail(FIRLS_E_UNSUPPORTED, "TV needs n to be a multiple of 32");
    s.psi = PSI_TV;
    s.tvb = in.psi == FIRLS_PSI_TV_PAPER ? 1 : 0;
    s.L = 0;
    s.n_coef = 2 * s.C * n * n;
  } else {
    return fail(FIRLS_E_INVALID, "unknown psi");
  }
  // group map (caller order) -> internal order
  std::vector<int32_t> ptr, idx;
  if (in.n_groups == 0 && !in.group_ptr && !in.group_idx) {
    // default: coefficient j of every contrast (Haar: standard / joint
    // sparsity), or rows p of D1 and D2 of every contrast (isotropic / joint TV)
    const int N = n * n, C = s.C;
    const int per = (s.psi == PSI_HAAR ? 1 : 2) * C;
    ptr.resize(N + 1);
    idx.resize((size_t)N * per);
    for (int i = 0; i <= N; ++i) ptr[i] = i * per;
    for (int i = 0; i < N; ++i)
      for (int c = 0; c < C; ++c) {
        idx[(size_t)i * per + c] = c * N + i;
        if (s.psi != PSI_HAAR) idx[(size_t)i * per + C + c] = (C + c) * N + i;
      }
  } else {
    if (in.n_groups <= 0 || !in.group_ptr || !in.group_idx) return fail(FIRLS_E_INVALID, "group map needs n_groups > 0 and both arrays");
    if (in.group_ptr[0] != 0) return fail(FIRLS_E_INVALID, "group_ptr[0] must be 0");
    ptr.assign(in.group_ptr, in.group_ptr + in.n_groups + 1);
    for (int g = 0; g < in.n_groups; ++g)
      if (ptr[g + 1] < ptr[g]) return fail(FIRLS_E_INVALID, "group_ptr must be non-decreasing");
    idx.assign(in.group_idx, in.group_idx + ptr[in.n_groups]);
    for (int32_t v : idx)
      if (v < 0 || v >= s.n_coef) return fail(FIRLS_E_INVALID, "group_idx entry out of range");
  }
  s.n_groups = (int)ptr.size() - 1;
  s.n_members = (int64_t)idx.size();
  if ((s.n_groups + GROUPS_PER_WG - 1) / GROUPS_PER_WG > PMAX) return fail(FIRLS_E_UNSUPPORTED, "too many groups");
  {
    // every partial-sum slot holds one value per workgroup of a pass
    const int R = band_rows(n), sc = strip_cols(h->fp64, n);
    const int most = std::max({s.C * (n / R + n / sc), s.C * (n / TV_TR) * (n / TV_TC) * (s.psi == PSI_TV)});
    if (most > PMAX) return fail(FIRLS_E_UNSUPPORTED, "too many contrasts for this image size");
  }
  std::vector<int32_t> perm(s.n_coef);
  const int N = n * n, C = s.C;
  if (s.psi == FIRLS_PSI_HAAR) {
    // contrast c's coefficients: block c, in-place layout within it
    for (int ch = 0; ch < C; ++ch)
      for (int r = 0; r < n; ++r)
        for (int c = 0; c < n; ++c) perm[ch * N + r * n + c] = ch * N + haar_internal_index(n, s.L, r, c);
  } else if (s.tvb) {
    // the paper's coefficient of pixel (r, c) lives in forward slot (r-1, c)
    // of D1 and (r, c-1) of D2 (indices mod n), contrast by contrast
    for (int ch = 0; ch < C; ++ch)
      for (int r = 0; r < n; ++r)
        for (int c = 0; c < n; ++c) {
          perm[ch * N + r * n + c] = ch * N + ((r + n - 1) % n) * n + c;
          perm[(C + ch) * N + r * n + c] = (C + ch) * N + r * n + (c + n - 1) % n;
        }
  } else {
    for (int i = 0; i < s.n_coef; ++i) perm[i] = i;
  }
  for (auto& v : idx) v = perm[v];
  // Haar maps whose groups each lie inside one row band of the row passes
  // (tree groups do) get their weights inside the residual's row pass:
  // groups are ordered by band, and the band's |Psi x|^2 and W must fit in
  // that pass's LDS
  std::vector<int32_t> bgptr;
  if (s.psi == PSI_HAAR && !s.dense) {
    const int R = band_rows(n), nb = s.C * n / R;
    const int64_t per = (int64_t)R * n;
    std::vector<int> band(s.n_groups, -1);
    bool local = true;
    for (int g = 0; g < s.n_groups && local; ++g)
      for (int j = ptr[g]; j < ptr[g + 1]; ++j) {
        const int b = (int)(idx[j] / per);
        if (band[g] < 0) band[g] = b;
        else if (band[g] != b) { local = false; break; }
      }
    std::vector<int32_t> cnt(nb + 1, 0);
    for (int g = 0; g < s.n_groups && local; ++g)
      if (band[g] >= 0) cnt[band[g] + 1]++;
      else local = false;                      // an empty group
    if (local) {
      for (int b = 0; b < nb; ++b) cnt[b + 1] += cnt[b];
      const size_t lds = (size_t)R * (n + n / 16 + 1) * h->elt;
      int most = 0;
      for (int b = 0; b < nb; ++b) most = std::max(most, cnt[b + 1] - cnt[b]);
      if ((size_t)(per + most) * h->relt <= lds) {
        // stable reorder by band
        std::vector<int32_t> order(s.n_groups), fill(cnt.begin(), cnt.end() - 1);
        for (int g = 0; g < s.n_groups; ++g) order[fill[band[g]]++] = g;
        std::vector<int32_t> p2(s.n_groups + 1, 0), i2;
        i2.reserve(idx.size());
        for (int k = 0; k < s.n_groups; ++k) {
          const int g = order[k];
          for (int j = ptr[g]; j < ptr[g + 1]; ++j) i2.push_back(idx[j]);
          p2[k + 1] = (int32_t)i2.size();
        }
        ptr.swap(p2);
        idx.swap(i2);
        bgptr = cnt;
      }
    }
  }
  std::vector<int32_t> tptr(s.n_coef + 1, 0), tidx(idx.size());
  for (int32_t v : idx) tptr[v + 1]++;
  for (int i = 0; i < s.n_coef; ++i) tptr[i + 1] += tptr[i];
  std::vector<int32_t> fillp(tptr.begin(), tptr.end() - 1);
  for (int g = 0; g < s.n_groups; ++g)
    for (int j = ptr[g]; j < ptr[g + 1]; ++j) tidx[fillp[idx[j]]++] = g;
  auto up = [&](int32_t** dst, const std::vector<int32_t>& v) -> int {
    HIPCHK(hipMalloc(dst, std::max<size_t>(1, v.size()) * sizeof(int32_t)));
    if (!v.empty()) HIPCHK(hipMemcpy(*dst, v.data(), v.size() * sizeof(int32_t), hipMemcpyHostToDevice));
    return FIRLS_OK;
  };
  int rc;
  if ((rc = up(&s.d_gptr, ptr)) || (rc = up(&s.d_gidx, idx)) || (rc = up(&s.d_tptr, tptr)) ||
      (rc = up(&s.d_tidx, tidx)) || (rc = up(&s.d_perm, perm)) ||
      (!bgptr.empty() && (rc = up(&s.d_bgptr, bgptr))))
    return rc;
  // small band-local groups also get the padded lists: one coalesced load
  // per member instead of a pointer chase through the CSR arrays
  if (!bgptr.empty()) {
    const int64_t per = (int64_t)band_rows(n) * n;
    int gw = 0, tw = 0;
    for (int g = 0; g < s.n_groups; ++g) gw = std::max(gw, ptr[g + 1] - ptr[g]);
    for (int i = 0; i < s.n_coef; ++i) tw = std::max(tw, tptr[i + 1] - tptr[i]);
    auto pow2 = [](int v) { int w = 1; while (w < v) w *= 2; return w; };
    gw = pow2(gw);
    tw = pow2(tw);
    if (gw <= ELL_MAX && tw <= ELL_MAX && per <= 0xFFFF) {
      std::vector<uint16_t> gell((size_t)gw * s.n_groups, 0xFFFF), tell((size_t)tw * s.n_coef, 0xFFFF);
      const int nb = (int)bgptr.size() - 1;
      for (int b = 0; b < nb; ++b)
        for (int g = bgptr[b]; g < bgptr[b + 1]; ++g)
          for (int j = ptr[g]; j < ptr[g + 1]; ++j)
            gell[(size_t)g * gw + (j - ptr[g])] = (uint16_t)(idx[j] - b * per);
      for (int i = 0; i < s.n_coef; ++i) {
        const int b = (int)(i / per);
        for (int t = tptr[i]; t < tptr[i + 1]; ++t)
          tell[(size_t)i * tw + (t - tptr[i])] = (uint16_t)(tidx[t] - bgptr[b]);
      }
      auto up16 = [&](uint16_t** dst, const std::vector<uint16_t>& v) -> int {
        HIPCHK(hipMalloc(dst, std::max<size_t>(1, v.size()) * sizeof(uint16_t)));
        if (!v.empty()) HIPCHK(hipMemcpy(*dst, v.data(), v.size() * sizeof(uint16_t), hipMemcpyHostToDevice));
        return FIRLS_OK;
      };
      if ((rc = up16(&s.d_gell, gell)) || (rc = up16(&s.d_tell, tell))) return rc;
      s.ell_gw = gw;
      s.ell_tw = tw;
    }
  }
  s.sk = size_kernels(h->fp64, n);
  if (!s.sk) return fail(FIRLS_E_UNSUPPORTED, "no kernels for this size");
  // twiddles exp(-2 pi i k / n), computed in FP64
  for (auto& e : h->tw)
    if (e.first == n) s.tw = e.second;
  if (!s.tw) {
    std::vector<double> w(2 * n);
    for (int k = 0; k < n; ++k) {
      const double a = 2.0 * M_PI * (double)k / (double)n;
      w[2 * k] = std::cos(a);
      w[2 * k + 1] = -std::sin(a);
    }
    void* d = nullptr;
    HIPCHK(hipMalloc(&d, n * h->elt));
    if (h->fp64) {
      HIPCHK(hipMemcpy(d, w.data(), n * h->elt, hipMemcpyHostToDevice));
    } else {
      std::vector<float> f(w.begin(), w.end());
      HIPCHK(hipMemcpy(d, f.data(), n * h->elt, hipMemcpyHostToDevice));
    }
    h->tw.push_back({n, d});
    s.tw = d;
  }
  return FIRLS_OK;
}

void destroy_shapes(firls_handle* h) {
  for (auto& s : h->shapes) {
    for (int32_t* p : {s.d_gptr, s.d_gidx, s.d_tptr, s.d_tidx, s.d_perm, s.d_bgptr})
      if (p) (void)hipFree(p);
    for (uint16_t* p : {s.d_gell, s.d_tell})
      if (p) (void)hipFree(p);
    if (s.d_A) (void)hipFree(s.d_A);
  }
  h->shapes.clear();
  for (auto& e : h->tw) (void)hipFree(e.second);
  h->tw.clear();
}

// Single-slice operator set-up: slot 0 (and 1) of the batch arrays.
int op_begin(firls_handle* h, hipStream_t st, int shape_id, int slots) {
  if (shape_id < 0 || shape_id >= (int)h->shapes.size()) return fail(FIRLS_E_INVALID, "shape_id out of range");
  const Shape& s = h->shapes[shape_id];
  int rc = ensure_capacity(h, st, slots * h->slice_bytes(s), slots);
  if (rc) return rc;
  HIPCHK(hipStreamSynchronize(st));
  for (int i = 0; i < slots; ++i) {
    fill_desc(h, h->h_desc[i], s, i * h->slice_bytes(s), nullptr);
    h->h_list[i] = i;
  }
  return FIRLS_OK;
}

int op_upload(firls_handle* h, hipStream_t st, int slots) {
  HIPCHK(hipMemcpyAsync(h->d_desc, h->h_desc, sizeof(SliceDesc) * slots, hipMemcpyHostToDevice, st));
  HIPCHK(hipMemcpyAsync(h->d_list, h->h_list, sizeof(int32_t) * slots, hipMemcpyHostToDevice, st));
  return FIRLS_OK;
}

}  // namespace

extern "C" {

const char* firls_last_error(void) { return g_err.c_str(); }

int firls_create(const firls_config* cfg, firls_handle** out) {
  g_err.clear();
  if (!cfg || !out) return fail(FIRLS_E_INVALID, "cfg and out must be non-null");
  *out = nullptr;
  if (cfg->n_shapes <= 0 || !cfg->shapes) return fail(FIRLS_E_INVALID, "need at least one shape");
  if (cfg->max_slices <= 0) return fail(FIRLS_E_INVALID, "max_slices must be positive");
  if (cfg->prec != FIRLS_FP32 && cfg->prec != FIRLS_FP64) return fail(FIRLS_E_INVALID, "prec must be FIRLS_FP32 or FIRLS_FP64");
  if (!(cfg->eps > 0.0) || !std::isfinite(cfg->eps)) return fail(FIRLS_E_INVALID, "eps must be positive");
  if (cfg->max_outer < 0) return fail(FIRLS_E_INVALID, "max_outer must be >= 0");
  if (cfg->pcg_iters < 1 || cfg->pcg_iters > KMAX) return fail(FIRLS_E_INVALID, "pcg_iters must be in 1..64");
  if (!(cfg->outer_tol >= 0.0)) return fail(FIRLS_E_INVALID, "outer_tol must be >= 0");
  if (!(cfg->pcg_rtol >= 0.0 && cfg->pcg_rtol < 1.0)) return fail(FIRLS_E_INVALID, "pcg_rtol must be in [0, 1)");
  if (cfg->precond != FIRLS_PC_PAPER && cfg->precond != FIRLS_PC_JACOBI && cfg->precond != FIRLS_PC_NONE)
    return fail(FIRLS_E_INVALID, "precond must be FIRLS_PC_PAPER, FIRLS_PC_JACOBI or FIRLS_PC_NONE");
  if (cfg->workspace && (reinterpret_cast<uintptr_t>(cfg->workspace) & 255))
    return fail(FIRLS_E_INVALID, "workspace must be 256-byte aligned");
  if (cfg->workspace && cfg->workspace_bytes < firls_workspace_bytes(cfg))
    return fail(FIRLS_E_INVALID, "workspace_bytes is smaller than firls_workspace_bytes(cfg) = " +
                                     std::to_string(firls_workspace_bytes(cfg)));
  firls_handle* h = new firls_handle();
  h->cfg = *cfg;
  h->cfg.shapes = nullptr;
  if (cfg->workspace) {
    h->ws = cfg->workspace;
    h->ws_cap = cfg->workspace_bytes;
    h->ws_owned = false;
  }
  h->fp64 = cfg->prec == FIRLS_FP64;
  h->elt = h->fp64 ? 16 : 8;
  h->relt = h->fp64 ? 8 : 4;
  if (hipGetDevice(&h->device) != hipSuccess) {
    delete h;
    return fail(FIRLS_E_HIP, "no HIP device");
  }
  h->shapes.resize(cfg->n_shapes);
  for (int i = 0; i < cfg->n_shapes; ++i) {
    int rc = upload_shape(h, cfg->shapes[i], h->shapes[i]);
    if (rc) {
      std::string msg = "shape " + std::to_string(i) + ": " + g_err;
      destroy_shapes(h);
      delete h;
      return fail(rc, msg);
    }
  }
  if (hipEventCreateWithFlags(&h->ev, hipEventDisableTiming) != hipSuccess) {
    destroy_shapes(h);
    delete h;
    return fail(FIRLS_E_HIP, "event creation failed");
  }
  // slice tables and pinned staging for max_slices up front (the
  // allocation-free solve relies on them), and this device's scratch
  int rc = ensure_capacity(h, nullptr, 0, cfg->max_slices);
  if (rc) {
    const std::string msg = g_err;
    firls_destroy(h);
    return fail(rc, msg);
  }
  if (noalloc_scratch(h->device, &h->scratch)) h->scratch_err = g_err;
  g_err.clear();
  *out = h;
  return FIRLS_OK;
}

int firls_destroy(firls_handle* h) {
  if (!h) return FIRLS_OK;
  (void)hipDeviceSynchronize();
  free_batch(h);
  destroy_shapes(h);
  if (h->ev) (void)hipEventDestroy(h->ev);
  if (h->ev_in) (void)hipEventDestroy(h->ev_in);
  if (h->own) (void)hipStreamDestroy(h->own);
  for (hipEvent_t e : h->ev_pool) (void)hipEventDestroy(e);
  delete h;
  return FIRLS_OK;
}

size_t firls_slice_workspace_bytes(const firls_handle* h, int32_t shape_id, int32_t n) {
  if (!h || shape_id < 0 || shape_id >= (int)h->shapes.size() || n < 0) return 0;
  return (size_t)n * h->slice_bytes(h->shapes[shape_id]);
}

size_t firls_workspace_bytes(const firls_config* cfg) {
  if (!cfg || cfg->n_shapes <= 0 || !cfg->shapes || cfg->max_slices <= 0) return 0;
  const bool fp64 = cfg->prec == FIRLS_FP64;
  const size_t elt = fp64 ? 16 : 8, relt = fp64 ? 8 : 4;
  size_t most = 0;
  for (int i = 0; i < cfg->n_shapes; ++i) {
    const firls_shape& in = cfg->shapes[i];
    const bool tv = in.psi == FIRLS_PSI_TV || in.psi == FIRLS_PSI_TV_PAPER;
    const size_t C = in.channels <= 0 ? 1 : (size_t)in.channels;
    const size_t pixels = C * (size_t)in.n * (size_t)in.n;
    const size_t n_coef = tv ? 2 * pixels : pixels;
    const size_t n_groups = in.n_groups > 0 ? (size_t)in.n_groups : (size_t)in.n * (size_t)in.n;
    const int Mp = in.op == FIRLS_OP_DENSE ? (in.m + GEMM_BM - 1) / GEMM_BM * GEMM_BM : 0;
    most = std::max(most, firls_handle::slice_bytes_of(pixels, tv, n_coef, n_groups, Mp, elt, relt));
  }
  return most * (size_t)cfg->max_slices;
}

int firls_solve(firls_handle* h, void* stream, const firls_slice* slice, firls_report* report) {
  if (!h) return fail(FIRLS_E_INVALID, "null handle");
  g_err.clear();
  return run_batch(h, (hipStream_t)stream, 1, slice, report, h->cfg.max_outer, h->cfg.outer_tol);
}

int firls_solve_batched(firls_handle* h, void* stream, int32_t n_slices, const firls_slice* slices,
                        firls_report* reports) {
  if (!h) return fail(FIRLS_E_INVALID, "null handle");
  if (n_slices <= 0) return fail(FIRLS_E_INVALID, "n_slices must be positive");
  if (!slices || !reports) return fail(FIRLS_E_INVALID, "slices and reports must be non-null");
  g_err.clear();
  return run_batch(h, (hipStream_t)stream, n_slices, slices, reports, h->cfg.max_outer, h->cfg.outer_tol);
}

int firls_solve_batched_noalloc(firls_handle* h, void* stream, int32_t n_slices, const firls_slice* slices,
                                firls_report* reports) {
  if (!h) return fail(FIRLS_E_INVALID, "null handle");
  if (n_slices <= 0) return fail(FIRLS_E_INVALID, "n_slices must be positive");
  if (n_slices > h->cfg.max_slices) return fail(FIRLS_E_INVALID, "n_slices exceeds max_slices");
  if (!slices || !reports) return fail(FIRLS_E_INVALID, "slices and reports must be non-null");
  g_err.clear();
  if (!h->scratch) return fail(FIRLS_E_HIP, "no allocation-free scratch on this device: " + h->scratch_err);
  int dev = -1;
  HIPCHK(hipGetDevice(&dev));
  if (dev != h->device) return fail(FIRLS_E_INVALID, "the handle belongs to another device");
  for (int i = 0; i < n_slices; ++i) {
    int rc = check_slice(h, slices[i]);
    if (rc) return rc;
    if (h->shapes[slices[i].shape_id].dense)
      return fail(FIRLS_E_UNSUPPORTED, "the allocation-free solve is for masked-FFT shapes");
  }
  // scratch layout: slice descs, slice states, the two slice lists, then
  // each slice's workspace in call order (as run_chunk carves it)
  const size_t ns = (size_t)n_slices;
  const size_t o_state = align256(ns * sizeof(SliceDesc));
  const size_t o_list = o_state + align256(ns * sizeof(SliceState));
  const size_t o_ws = o_list + align256(2 * ns * sizeof(int32_t));
  size_t need = 0;
  for (int i = 0; i < n_slices; ++i) need += h->slice_bytes(h->shapes[slices[i].shape_id]);
  if (o_ws + need > kNoallocBytes)
    return fail(FIRLS_E_INVALID, "the batch needs " + std::to_string(o_ws + need) + " bytes of scratch; the "
                "allocation-free solve has " + std::to_string(kNoallocBytes) + " (FIRLS_NOALLOC_SCRATCH_BYTES)");
  if (std::max(n_slices, 2) > h->cap_slices) return fail(FIRLS_E_INVALID, "slice tables smaller than max_slices");
  // Run the ordinary batched loop on the scratch: direct launches (no graph
  // is captured or instantiated), all slices at once, no profiling events.
  // The handle's own buffers and settings come back on every return path.
  struct Swap {
    firls_handle* h;
    void* ws;
    size_t ws_cap;
    SliceDesc* desc;
    SliceState* state;
    int32_t* list;
    bool graphs, prof;
    int chunk;
    ~Swap() {
      h->ws = ws;
      h->ws_cap = ws_cap;
      h->d_desc = desc;
      h->d_state = state;
      h->d_list = list;
      h->use_graphs = graphs;
      h->profiling = prof;
      h->chunk = chunk;
      h->noalloc = false;
    }
  } keep{h, h->ws, h->ws_cap, h->d_desc, h->d_state, h->d_list, h->use_graphs, h->profiling, h->chunk};
  char* base = static_cast<char*>(h->scratch);
  h->d_desc = reinterpret_cast<SliceDesc*>(base);
  h->d_state = reinterpret_cast<SliceState*>(base + o_state);
  h->d_list = reinterpret_cast<int32_t*>(base + o_list);
  h->ws = base + o_ws;
  h->ws_cap = kNoallocBytes - o_ws;
  h->use_graphs = false;
  h->profiling = false;
  h->chunk = 0;
  h->noalloc = true;
  return run_batch(h, (hipStream_t)stream, n_slices, slices, reports, h->cfg.max_outer, h->cfg.outer_tol);
}

int firls_profile(firls_handle* h, int32_t enable) {
  if (!h) return fail(FIRLS_E_INVALID, "null handle");
  h->profiling = enable != 0;
  h->recs.clear();
  h->ev_used = 0;
  if (!enable) return FIRLS_OK;   // the totals stay readable until the next enable
  for (int c = 0; c < FIRLS_PROF_CLASSES; ++c) {
    h->prof_ms[c] = 0.0;
    h->prof_launches[c] = 0;
    h->prof_units[c] = 0;
  }
  const size_t ks = h->shapes.size() * FIRLS_PROF_CLASSES;
  h->prof_ms_shape.assign(ks, 0.0);
  h->prof_launches_shape.assign(ks, 0);
  h->prof_units_shape.assign(ks, 0);
  return FIRLS_OK;
}

namespace {
const char* const kProfNames[FIRLS_PROF_CLASSES] = {
    "init", "adjoint", "psi_sq", "group_w", "group_d", "r0_rowfwd", "r0_col", "r0_rowinv",
    "r0_update", "check", "rowfwd", "col", "rowinv", "update", "last_x"};
}  // namespace

int firls_profile_read(const firls_handle* h, int32_t n, firls_kernel_stat* out) {
  if (!h || !out || n < 0) return fail(FIRLS_E_INVALID, "null argument");
  const int m = std::min<int>(n, FIRLS_PROF_CLASSES);
  for (int c = 0; c < m; ++c) {
    std::memset(&out[c], 0, sizeof(out[c]));
    std::strncpy(out[c].name, kProfNames[c], sizeof(out[c].name) - 1);
    out[c].launches = h->prof_launches[c];
    out[c].slice_launches = h->prof_units[c];
    out[c].ms = h->prof_ms[c];
  }
  return m;
}

int firls_profile_read_shape(const firls_handle* h, int32_t shape_id, int32_t n, firls_kernel_stat* out) {
  if (!h || !out || n < 0) return fail(FIRLS_E_INVALID, "null argument");
  if (shape_id < 0 || shape_id >= (int)h->shapes.size()) return fail(FIRLS_E_INVALID, "shape_id out of range");
  const int m = std::min<int>(n, FIRLS_PROF_CLASSES);
  for (int c = 0; c < m; ++c) {
    const size_t k = (size_t)shape_id * FIRLS_PROF_CLASSES + c;
    std::memset(&out[c], 0, sizeof(out[c]));
    std::strncpy(out[c].name, kProfNames[c], sizeof(out[c].name) - 1);
    if (k < h->prof_ms_shape.size()) {
      out[c].launches = h->prof_launches_shape[k];
      out[c].slice_launches = h->prof_units_shape[k];
      out[c].ms = h->prof_ms_shape[k];
    }
  }
  return m;
}

int firls_op_adjoint(firls_handle* h, void* stream, int32_t shape_id, const void* b, const uint8_t* mask, void* x) {
  if (!h || !b || !x) return fail(FIRLS_E_INVALID, "null argument");
  hipStream_t st = (hipStream_t)stream;
  int rc = op_begin(h, st, shape_id, 1);
  if (rc) return rc;
  const Shape& s = h->shapes[shape_id];
  if (!mask && !s.dense) return fail(FIRLS_E_INVALID, "null argument");
  h->h_desc[0].b = b;
  h->h_desc[0].mask = mask;
  h->h_desc[0].x = x;
  h->h_desc[0].lambda = 1.0;
  if ((rc = op_upload(h, st, 1))) return rc;
  Params P = base_params(h, s, shape_id, h->d_list);
  P.count = 1;
  LAUNCH(prec_kernels(h->fp64)->slice_init, P, dim3(1), st);
  if (s.dense) {
    if ((rc = ensure_gemm_scratch(h, st, s, 1)) || (rc = launch_gemm(h, s, P, G_ATB, 1, st, FIRLS_PROF_AHB))) return rc;
  } else {
    LAUNCH(s.sk->col[COL_AHB], P, dim3(s.col_wgs(h->fp64), 1), st);
    LAUNCH(s.sk->rowinv[RI_PLAIN], P, dim3(s.row_wgs(), 1), st);
  }
  HIPCHK(hipStreamSynchronize(st));
  return FIRLS_OK;
}

int firls_op_weights(firls_handle* h, void* stream, int32_t shape_id, const void* x, void* d_out) {
  if (!h || !x || !d_out) return fail(FIRLS_E_INVALID, "null argument");
  hipStream_t st = (hipStream_t)stream;
  int rc = op_begin(h, st, shape_id, 1);
  if (rc) return rc;
  h->h_desc[0].x = const_cast<void*>(x);
  h->h_desc[0].mask = static_cast<const uint8_t*>(x);  // any readable bytes: only rho uses it
  h->h_desc[0].lambda = 1.0;
  if ((rc = op_upload(h, st, 1))) return rc;
  const Shape& s = h->shapes[shape_id];
  Params P = base_params(h, s, shape_id, h->d_list);
  P.out = d_out;
  LAUNCH(prec_kernels(h->fp64)->slice_init, P, dim3(1), st);
  if ((rc = launch_weights(h, s, P, 1, st))) return rc;
  LAUNCH(prec_kernels(h->fp64)->export_d, P, dim3((s.n_coef + NT - 1) / NT, 1), st);
  HIPCHK(hipStreamSynchronize(st));
  return FIRLS_OK;
}

int firls_op_system(firls_handle* h, void* stream, int32_t shape_id, const uint8_t* mask, double lambda,
                    const void* x_w, const void* p, void* q) {
  if (!h || !x_w || !p || !q) return fail(FIRLS_E_INVALID, "null argument");
  if (!(lambda > 0.0)) return fail(FIRLS_E_INVALID, "lambda must be positive");
  hipStream_t st = (hipStream_t)stream;
  int rc = op_begin(h, st, shape_id, 2);
  if (rc) return rc;
  if (!mask && !h->shapes[shape_id].dense) return fail(FIRLS_E_INVALID, "null argument");
  SliceDesc& A = h->h_desc[0];
  SliceDesc& B = h->h_desc[1];
  A.x = const_cast<void*>(x_w);
  A.mask = mask;
  A.lambda = lambda;
  B.d = A.d;
  B.x = const_cast<void*>(p);
  B.p = const_cast<void*>(p);
  B.q = q;
  B.mask = mask;
  B.lambda = lambda;
  if ((rc = op_upload(h, st, 2))) return rc;
  const Shape& s = h->shapes[shape_id];
  Params PA = base_params(h, s, shape_id, h->d_list);
  Params PB = base_params(h, s, shape_id, h->d_list + 1);
  LAUNCH(prec_kernels(h->fp64)->slice_init, PA, dim3(2), st);
  if ((rc = launch_weights(h, s, PA, 1, st))) return rc;
  PB.k = 0;
  PB.count = 1;
  if (s.dense) {
    if ((rc = ensure_gemm_scratch(h, st, s, 1)) || (rc = launch_dense_normal(h, s, PB, 1, st))) return rc;
  } else {
    LAUNCH(s.sk->rowfwd[RF_PLAIN], PB, dim3(s.row_wgs(), 1), st);
    LAUNCH(s.sk->col[COL_SP], PB, dim3(s.col_wgs(h->fp64), 1), st);
  }
  LAUNCH(s.sk->rowinv[s.psi == PSI_HAAR ? RI_SP_HAAR : RI_SP_TV], PB, dim3(s.row_wgs(), 1), st);
  HIPCHK(hipStreamSynchronize(st));
  return FIRLS_OK;
}

int firls_op_precond(firls_handle* h, void* stream, int32_t shape_id, const uint8_t* mask, double lambda,
                     const void* x_w, const void* r, void* z) {
  if (!h || !x_w || !r || !z) return fail(FIRLS_E_INVALID, "null argument");
  if (!(lambda > 0.0)) return fail(FIRLS_E_INVALID, "lambda must be positive");
  hipStream_t st = (hipStream_t)stream;
  int rc = op_begin(h, st, shape_id, 2);
  if (rc) return rc;
  if (!mask && !h->shapes[shape_id].dense) return fail(FIRLS_E_INVALID, "null argument");
  SliceDesc& A = h->h_desc[0];
  SliceDesc& B = h->h_desc[1];
  A.x = const_cast<void*>(x_w);
  A.mask = mask;
  A.lambda = lambda;
  B.d = A.d;
  B.r[0] = const_cast<void*>(r);
  B.r[1] = const_cast<void*>(r);
  B.p = z;
  B.z = z;
  B.mask = mask;
  B.lambda = lambda;
  if ((rc = op_upload(h, st, 2))) return rc;
  const Shape& s = h->shapes[shape_id];
  Params PA = base_params(h, s, shape_id, h->d_list);
  Params PB = base_params(h, s, shape_id, h->d_list + 1);
  LAUNCH(prec_kernels(h->fp64)->slice_init, PA, dim3(2), st);
  if ((rc = launch_weights(h, s, PA, 1, st))) return rc;
  PB.k = 0;
  if (s.psi == PSI_HAAR) LAUNCH(s.sk->rowfwd[RF_PCG_HAAR], PB, dim3(s.row_wgs(), 1), st);
  else LAUNCH(prec_kernels(h->fp64)->update_tv[UP_INIT], PB, dim3(PB.nrz, 1), st);
  HIPCHK(hipStreamSynchronize(st));
  return FIRLS_OK;
}

int firls_op_objective(firls_handle* h, void* stream, int32_t shape_id, const void* b, const uint8_t* mask,
                       double lambda, const void* x, double* out3) {
  if (!h || !b || !x || !out3) return fail(FIRLS_E_INVALID, "null argument");
  if (!(lambda > 0.0)) return fail(FIRLS_E_INVALID, "lambda must be positive");
  hipStream_t st = (hipStream_t)stream;
  int rc = op_begin(h, st, shape_id, 1);
  if (rc) return rc;
  if (!mask && !h->shapes[shape_id].dense) return fail(FIRLS_E_INVALID, "null argument");
  SliceDesc& A = h->h_desc[0];
  A.x = const_cast<void*>(x);
  A.b = b;
  A.mask = mask;
  A.lambda = lambda;
  if ((rc = op_upload(h, st, 1))) return rc;
  const Shape& s = h->shapes[shape_id];
  Params P = base_params(h, s, shape_id, h->d_list);
  P.Tmax = 0;
  P.tau = 0.0;
  LAUNCH(prec_kernels(h->fp64)->slice_init, P, dim3(1), st);
  if ((rc = launch_weights(h, s, P, 1, st))) return rc;
  if (s.dense) {
    if ((rc = ensure_gemm_scratch(h, st, s, 1)) || (rc = launch_gemm(h, s, P, G_AX_R0, 1, st, FIRLS_PROF_R0_COL))) return rc;
  } else {
    LAUNCH(s.sk->rowfwd[RF_PLAIN], P, dim3(s.row_wgs(), 1), st);
    LAUNCH(s.sk->col[COL_R0], P, dim3(s.col_wgs(h->fp64), 1), st);
  }
  LAUNCH(prec_kernels(h->fp64)->outer_check, P, dim3(1), st);
  HIPCHK(hipMemcpyAsync(h->h_state, h->d_state, sizeof(SliceState), hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  out3[0] = h->h_state[0].Fe;
  out3[1] = h->h_state[0].F;
  out3[2] = h->h_state[0].data;
  return FIRLS_OK;
}

int firls_solve_batched_learned(firls_handle* h, firls_cnn* net, void* stream, int32_t n_slices,
                                const firls_slice* slices, firls_report* reports, int32_t* used_learned) {
  if (!h || !net) return fail(FIRLS_E_INVALID, "null handle or network");
  g_err.clear();
  if (h->fp64) return fail(FIRLS_E_UNSUPPORTED, "the learned start is built for FIRLS_FP32");
  if (!cnn_ready(net)) return fail(FIRLS_E_INVALID, "network parameters not set");
  if (n_slices <= 0 || n_slices > h->cfg.max_slices) return fail(FIRLS_E_INVALID, "n_slices out of range");
  if (!slices || !reports) return fail(FIRLS_E_INVALID, "slices and reports must be non-null");
  const int n = cnn_image_side(net);
  for (int i = 0; i < n_slices; ++i) {
    int rc = check_slice(h, slices[i]);
    if (rc) return rc;
    if (h->shapes[slices[i].shape_id].n != n) return fail(FIRLS_E_INVALID, "every slice must have the network's image size");
    if (h->shapes[slices[i].shape_id].C != 1 || h->shapes[slices[i].shape_id].dense)
      return fail(FIRLS_E_UNSUPPORTED, "the learned start is built for single-contrast masked-FFT shapes");
  }
  hipStream_t st = (hipStream_t)stream;
  const int ns = n_slices;
  const size_t np = (size_t)n * n;
  const size_t stage = align256(np * 8 * ns);
  const size_t need = 2 * stage + align256(sizeof(void*) * ns) + align256(sizeof(SliceState) * ns);
  if (need > h->ws_learn_cap) {
    HIPCHK(hipStreamSynchronize(st));
    if (h->ws_learn) HIPCHK(hipFree(h->ws_learn));
    h->ws_learn = nullptr;
    h->ws_learn_cap = 0;
    if (hipMalloc(&h->ws_learn, need) != hipSuccess) {
      (void)hipGetLastError();
      return fail(FIRLS_E_NOMEM, "staging allocation failed");
    }
    h->ws_learn_cap = need;
  }
  char* base = static_cast<char*>(h->ws_learn);
  char* zf = base;
  char* x0 = base + stage;
  void** outs = reinterpret_cast<void**>(base + 2 * stage);
  SliceState* st_zero = reinterpret_cast<SliceState*>(base + 2 * stage + align256(sizeof(void*) * ns));
  // candidates evaluated through the batch machinery: descs whose x points
  // into a staging buffer
  std::vector<firls_slice> tmp(slices, slices + ns);
  std::vector<size_t> off(ns);
  size_t wneed = 0;
  for (int i = 0; i < ns; ++i) {
    off[i] = wneed;
    wneed += h->slice_bytes(h->shapes[slices[i].shape_id]);
  }
  int rc = ensure_capacity(h, st, wneed, 2 * ns);   // room for two staged desc sets
  if (rc) return rc;
  HIPCHK(hipStreamSynchronize(st));   // an earlier copy may still read the pinned staging
  const int nsh = (int)h->shapes.size();
  std::vector<std::vector<int>> by_shape(nsh);
  for (int i = 0; i < ns; ++i) by_shape[slices[i].shape_id].push_back(i);
  std::vector<int> lo(nsh);
  int pos = 0;
  for (int s = 0; s < nsh; ++s) {
    lo[s] = pos;
    for (int i : by_shape[s]) h->h_list[pos++] = i;
  }
  // the descs of both candidate sets (x in the zero-filled or the network
  // staging) sit in two regions of the pinned staging from the start, so
  // switching the device descs between them is a plain ordered copy
  SliceDesc* const staged[2] = {h->h_desc, h->h_desc + ns};
  char* const xbuf[2] = {zf, x0};
  for (int v = 0; v < 2; ++v)
    for (int i = 0; i < ns; ++i) {
      tmp[i].x = xbuf[v] + (size_t)i * np * 8;
      fill_desc(h, staged[v][i], h->shapes[slices[i].shape_id], off[i], &tmp[i]);
    }
  HIPCHK(hipMemcpyAsync(h->d_list, h->h_list, sizeof(int32_t) * pos, hipMemcpyHostToDevice, st));
  enum { ZF = 0, X0 = 1 };
  auto upload = [&](int v) -> int {
    HIPCHK(hipMemcpyAsync(h->d_desc, staged[v], sizeof(SliceDesc) * ns, hipMemcpyHostToDevice, st));
    return FIRLS_OK;
  };
  auto evaluate = [&]() -> int {   // F_eps of every slice's x into the states
    for (int s = 0; s < nsh; ++s) {
      const int c = (int)by_shape[s].size();
      if (!c) continue;
      const Shape& S = h->shapes[s];
      Params P = base_params(h, S, s, h->d_list + lo[s]);
      P.Tmax = 0;
      P.tau = 0.0;
      // Both candidates reproduce the measurements exactly (A A^H b = b, and
      // the data-consistency step sets m F x0 = b), so F_eps is lambda times
      // the penalty: no Fourier pass is needed.
      P.no_data = 1;
      if (S.psi == PSI_HAAR && S.d_bgptr && !S.dense) P.nreg = S.row_wgs();   // one partial per band
      LAUNCH(prec_kernels(false)->slice_init, P, dim3(c), st);
      int r2 = launch_weights(h, S, P, c, st, true);
      if (r2) return r2;
      LAUNCH(prec_kernels(false)->outer_check, P, dim3(c), st);
    }
    return FIRLS_OK;
  };
  // the prelude's launches are not profiled; the setting comes back on
  // every return path
  struct ProfilingOff {
    firls_handle* h;
    bool was;
    ~ProfilingOff() { h->profiling = was; }
  } prof_off{h, h->profiling};
  h->profiling = false;
  // 1. zero-filled starts A^H b
  if ((rc = upload(ZF))) return rc;
  for (int s = 0; s < nsh; ++s) {
    const int c = (int)by_shape[s].size();
    if (!c) continue;
    const Shape& S = h->shapes[s];
    Params P = base_params(h, S, s, h->d_list + lo[s]);
    LAUNCH(prec_kernels(false)->slice_init, P, dim3(c), st);
    LAUNCH(S.sk->col[COL_AHB], P, dim3(S.col_wgs(false), c), st);
    LAUNCH(S.sk->rowinv[RI_PLAIN], P, dim3(S.row_wgs(), c), st);
  }
  // 2. network starts x0 = zf + f(zf), in network batches
  const int mb = cnn_max_batch(net);
  for (int b0 = 0; b0 < ns; b0 += mb) {
    const int bn = std::min(mb, ns - b0);
    if ((rc = cnn_forward(net, st, bn, zf + (size_t)b0 * np * 8, x0 + (size_t)b0 * np * 8))) return rc;
  }
  // 3. data consistency on the network starts: x0 <- F^H (m b + (1 - m) F x0)
  if ((rc = upload(X0))) return rc;
  for (int s = 0; s < nsh; ++s) {
    const int c = (int)by_shape[s].size();
    if (!c) continue;
    const Shape& S = h->shapes[s];
    Params P = base_params(h, S, s, h->d_list + lo[s]);
    LAUNCH(S.sk->rowfwd[RF_PLAIN], P, dim3(S.row_wgs(), c), st);
    LAUNCH(S.sk->col[COL_DC], P, dim3(S.col_wgs(false), c), st);
    LAUNCH(S.sk->rowinv[RI_PLAIN], P, dim3(S.row_wgs(), c), st);
  }
  if ((rc = upload(ZF))) return rc;
  // 4. objectives of both candidates, 5. keep the better one in each x
  if ((rc = evaluate())) return rc;
  HIPCHK(hipMemcpyAsync(st_zero, h->d_state, sizeof(SliceState) * ns, hipMemcpyDeviceToDevice, st));
  if ((rc = upload(X0))) return rc;
  if ((rc = evaluate())) return rc;
  std::vector<void*> hx(ns);
  for (int i = 0; i < ns; ++i) hx[i] = slices[i].x;
  HIPCHK(hipMemcpyAsync(outs, hx.data(), sizeof(void*) * ns, hipMemcpyHostToDevice, st));
  cnn::ChooseArgs ca{st_zero, h->d_state, zf, x0, outs, n};
  HIPCHK(cnn::launch_choose(ca, ns, st));
  std::vector<SliceState> s0(ns), s1(ns);
  HIPCHK(hipMemcpyAsync(s0.data(), st_zero, sizeof(SliceState) * ns, hipMemcpyDeviceToHost, st));
  HIPCHK(hipMemcpyAsync(s1.data(), h->d_state, sizeof(SliceState) * ns, hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  if (used_learned)
    for (int i = 0; i < ns; ++i) used_learned[i] = s1[i].Fe <= s0[i].Fe ? 1 : 0;
  h->profiling = prof_off.was;
  // 6. FIRLS from the chosen starts
  for (int i = 0; i < ns; ++i) tmp[i] = slices[i], tmp[i].x_is_init = 1;
  return run_batch(h, st, ns, tmp.data(), reports, h->cfg.max_outer, h->cfg.outer_tol);
}

int firls_set_graphs(firls_handle* h, int32_t enable) {
  if (!h) return fail(FIRLS_E_INVALID, "null handle");
  h->use_graphs = enable != 0;
  drop_graphs(h);
  return FIRLS_OK;
}

int firls_set_paired(firls_handle* h, int32_t enable) {
  if (!h) return fail(FIRLS_E_INVALID, "null handle");
  h->use_pair = enable != 0;
  drop_graphs(h);
  return FIRLS_OK;
}

int firls_test_sync_timeout(firls_handle* h, int32_t enable) {
  if (!h) return fail(FIRLS_E_INVALID, "null handle");
  h->test_flags = enable ? (h->test_flags | TEST_SYNC_TIMEOUT) : (h->test_flags & ~TEST_SYNC_TIMEOUT);
  drop_graphs(h);
  return FIRLS_OK;
}

int firls_test_hooks(firls_handle* h, int32_t flags) {
  if (!h) return fail(FIRLS_E_INVALID, "null handle");
  if (flags & ~(FIRLS_TEST_SYNC_TIMEOUT | FIRLS_TEST_BREAKDOWN | FIRLS_TEST_NONMONOTONE))
    return fail(FIRLS_E_INVALID, "unknown test hook");
  h->test_flags = flags;
  drop_graphs(h);
  return FIRLS_OK;
}

int firls_set_schedule(firls_handle* h, int32_t schedule) {
  if (!h || schedule < FIRLS_SCHED_PER_SHAPE || schedule > FIRLS_SCHED_ACROSS_LARGEST_FIRST)
    return fail(FIRLS_E_INVALID, "bad argument");
  h->schedule = schedule;
  drop_graphs(h);
  return FIRLS_OK;
}

int firls_get_schedule(const firls_handle* h) { return h ? h->schedule : FIRLS_E_INVALID; }

int firls_get_paired(const firls_handle* h) { return h ? (h->use_pair ? 1 : 0) : FIRLS_E_INVALID; }

int firls_set_chunk(firls_handle* h, int32_t chunk) {
  if (!h || chunk < 0) return fail(FIRLS_E_INVALID, "bad argument");
  h->chunk = chunk;
  return FIRLS_OK;
}

int firls_autotune(firls_handle* h, void* stream, int32_t n_slices, const firls_slice* slices, int32_t* chosen,
                   int32_t* graphs) {
  if (!h || !slices || n_slices <= 0) return fail(FIRLS_E_INVALID, "bad argument");
  if (n_slices > h->cfg.max_slices) return fail(FIRLS_E_INVALID, "n_slices exceeds max_slices");
  g_err.clear();
  hipStream_t st = (hipStream_t)stream;
  for (int i = 0; i < n_slices; ++i) {
    int rc = check_slice(h, slices[i]);
    if (rc) return rc;
  }
  // cache key: the batch's shape mix, precision, PCG length and batch size
  std::ostringstream ks;
  ks << "v2 prec=" << (h->fp64 ? 64 : 32) << " K=" << h->cfg.pcg_iters << " slices=" << n_slices;
  {
    std::vector<int> cnt(h->shapes.size(), 0);
    for (int i = 0; i < n_slices; ++i) cnt[slices[i].shape_id]++;
    for (size_t s = 0; s < cnt.size(); ++s)
      if (cnt[s]) ks << " n" << h->shapes[s].n << "psi" << h->shapes[s].psi << "L" << h->shapes[s].L << "x" << cnt[s];
  }
  const std::string key = ks.str();
  const char* cache = std::getenv("FIRLS_TUNE_CACHE");
  if (cache) {
    std::ifstream in(cache);
    std::string line;
    while (std::getline(in, line)) {
      // key|chunk|graphs|schedule|paired
      const size_t b4 = line.rfind('|');
      const size_t b3 = b4 == std::string::npos || b4 == 0 ? std::string::npos : line.rfind('|', b4 - 1);
      const size_t b2 = b3 == std::string::npos || b3 == 0 ? std::string::npos : line.rfind('|', b3 - 1);
      const size_t b1 = b2 == std::string::npos || b2 == 0 ? std::string::npos : line.rfind('|', b2 - 1);
      if (b1 != std::string::npos && line.substr(0, b1) == key) {
        h->chunk = std::atoi(line.c_str() + b1 + 1);
        h->use_graphs = std::atoi(line.c_str() + b2 + 1) != 0;
        h->schedule = std::atoi(line.c_str() + b3 + 1);
        h->use_pair = std::atoi(line.c_str() + b4 + 1) != 0;
        drop_graphs(h);
        if (chosen) *chosen = h->chunk;
        if (graphs) *graphs = h->use_graphs ? 1 : 0;
        return FIRLS_OK;
      }
    }
  }
  // snapshot every x (trials overwrite it) and time a few outer iterations
  // per candidate sub-batch size and launch mode (graph replay or direct
  // launches); each candidate runs twice, the second run (graphs already
  // captured) is timed
  size_t bytes = 0;
  std::vector<size_t> xb(n_slices);
  for (int i = 0; i < n_slices; ++i) {
    xb[i] = h->shapes[slices[i].shape_id].pixels() * h->elt;
    bytes += xb[i];
  }
  void* snap = nullptr;
  if (hipMalloc(&snap, bytes) != hipSuccess) {
    (void)hipGetLastError();
    return fail(FIRLS_E_NOMEM, "autotune snapshot allocation failed");
  }
  auto copy_all = [&](bool save) -> int {
    size_t o = 0;
    for (int i = 0; i < n_slices; ++i) {
      char* sp = static_cast<char*>(snap) + o;
      if (save) HIPCHK(hipMemcpyAsync(sp, slices[i].x, xb[i], hipMemcpyDeviceToDevice, st));
      else HIPCHK(hipMemcpyAsync(slices[i].x, sp, xb[i], hipMemcpyDeviceToDevice, st));
      o += xb[i];
    }
    return FIRLS_OK;
  };
  int rc = copy_all(true);
  // schedules of batches that mix masked-FFT shapes
  std::vector<int> scheds = {FIRLS_SCHED_PER_SHAPE};
  {
    std::vector<int> seen(h->shapes.size(), 0);
    int present = 0;
    bool dense = false;
    for (int i = 0; i < n_slices; ++i) {
      present += seen[slices[i].shape_id]++ == 0;
      dense = dense || h->shapes[slices[i].shape_id].dense;
    }
    if (present >= 2 && !dense) scheds = {FIRLS_SCHED_PER_SHAPE, FIRLS_SCHED_ACROSS, FIRLS_SCHED_ACROSS_LARGEST_FIRST};
  }
  // the paired PCG pass (row inverse of one iteration and the step of the
  // next in one launch) against the two launches, where a shape has it
  std::vector<int> pairs = {h->use_pair ? 1 : 0};
  for (int i = 0; i < n_slices; ++i) {
    const Shape& S = h->shapes[slices[i].shape_id];
    if (S.psi == PSI_HAAR && !S.dense && S.sk->pcg_pair && h->cfg.precond == FIRLS_PC_PAPER) {
      pairs = {1, 0};
      break;
    }
  }
  std::vector<int> cands = {0};
  for (int c : {256, 128, 64, 32})
    if (c < n_slices) cands.push_back(c);
  std::vector<firls_report> rep(n_slices);
  const int T = std::max(1, std::min(3, h->cfg.max_outer));
  double best = 1e300;
  int best_c = 0, best_s = FIRLS_SCHED_PER_SHAPE;
  bool best_g = true, best_p = h->use_pair;
  const int chunk0 = h->chunk, sched0 = h->schedule;
  const bool graphs0 = h->use_graphs, pair0 = h->use_pair;
  const bool prof = h->profiling;
  h->profiling = false;
  const int per_p = 2 * (int)scheds.size(), per_c = per_p * (int)pairs.size();
  for (int trial = 0; trial < per_c * (int)cands.size(); ++trial) {
    if (rc) break;
    const int c = cands[trial / per_c];
    const bool pr = pairs[(trial % per_c) / per_p] != 0;
    const bool g = trial % 2 == 0;
    const int sc = scheds[(trial % per_p) / 2];
    h->chunk = c;
    h->use_graphs = g;
    if (h->schedule != sc || h->use_pair != pr) {
      h->schedule = sc;
      h->use_pair = pr;
      drop_graphs(h);
    }
    double t = 0.0;
    for (int rep_i = 0; rep_i < 2 && !rc; ++rep_i) {
      if ((rc = copy_all(false))) break;
      if (hipStreamSynchronize(st) != hipSuccess) { rc = fail(FIRLS_E_HIP, "sync failed"); break; }
      const auto t0 = std::chrono::steady_clock::now();
      rc = run_batch(h, st, n_slices, slices, rep.data(), T, 0.0);
      if (rc > 0) rc = 0;
      if (hipStreamSynchronize(st) != hipSuccess) rc = fail(FIRLS_E_HIP, "sync failed");
      t = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    }
    if (!rc && t < best) {
      best = t;
      best_c = c;
      best_g = g;
      best_s = sc;
      best_p = pr;
    }
  }
  h->profiling = prof;
  // the caller's x comes back from the snapshot also when a trial failed
  const int rc_restore = copy_all(false);
  if (!rc) rc = rc_restore;
  (void)hipStreamSynchronize(st);
  (void)hipFree(snap);
  if (rc) {
    h->chunk = chunk0;
    h->use_graphs = graphs0;
    h->schedule = sched0;
    h->use_pair = pair0;
    drop_graphs(h);
    return rc;
  }
  h->chunk = best_c;
  h->use_graphs = best_g;
  if (h->schedule != best_s || h->use_pair != best_p) {
    h->schedule = best_s;
    h->use_pair = best_p;
    drop_graphs(h);
  }
  if (chosen) *chosen = best_c;
  if (graphs) *graphs = best_g ? 1 : 0;
  if (cache) {
    std::ofstream out(cache, std::ios::app);
    out << key << "|" << best_c << "|" << (best_g ? 1 : 0) << "|" << best_s << "|" << (best_p ? 1 : 0) << "\n";
  }
  return FIRLS_OK;
}

int firls_op_outer_step(firls_handle* h, void* stream, int32_t shape_id, const void* b, const uint8_t* mask,
                        double lambda, void* x) {
  if (!h) return fail(FIRLS_E_INVALID, "null handle");
  firls_slice sl{};
  sl.shape_id = shape_id;
  sl.x_is_init = 1;
  sl.lambda = lambda;
  sl.b = b;
  sl.mask = mask;
  sl.x = x;
  firls_report rep{};
  int rc = run_batch(h, (hipStream_t)stream, 1, &sl, &rep, 1, 0.0);
  return rc < 0 ? rc : FIRLS_OK;
}

}  // extern "C"
