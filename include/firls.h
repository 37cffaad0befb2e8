/*
 * firls.h - C ABI of the MI355X FIRLS library (libfirls.so).
 *
 * FIRLS (Chen, Huang, He, Li: "Fast Iteratively Reweighted Least Squares
 * Algorithms for Analysis-Based Sparsity Reconstruction") reconstructs an
 * n x n complex image x from undersampled k-space data b by minimising
 *
 *     F(x) = 1/2 ||A x - b||^2 + lambda ||Psi x||_{2,1}        (Section 1, eq. 3)
 *
 * with A = R F the masked unitary 2D Fourier transform (Section 5.4) and Psi
 * either an L-level orthonormal Haar transform Phi with (possibly
 * overlapping) groups given by a replication matrix G (Section 3.1, eq. 8),
 * or the periodic forward differences [D1; D2] of total variation
 * (Section 4.1, eqs. 32-35).  Each outer iteration refreshes the group
 * weights W (eq. 12 / eq. 37) and runs PCG on the normal equations
 * (A^H A + lambda Psi^T G^T W G Psi) x = A^H b (eq. 15 / eq. 39) with the
 * pseudo-diagonal preconditioner (eq. 17) or, for TV, the triangular
 * factors of the penta-diagonal preconditioner (eqs. 40-43) in red-black
 * order.  Algorithms 2 and 3 give the loop.
 *
 * Conventions for every entry point
 * ---------------------------------
 *  - Device pointers are HIP device memory on the current device; host
 *    pointers are ordinary host memory.  The caller owns every buffer it
 *    passes; the library owns its handle and its workspace.
 *  - Images and k-space arrays are n x n, row-major, complex interleaved
 *    (re, im): float2 in FIRLS_FP32 mode, double2 in FIRLS_FP64 mode.
 *    k-space is unshifted (DC at [0, 0]); F is unitary (1/n both ways).
 *  - Masks are uint8 n x n (nonzero = sampled).  b is read as mask * b.
 *  - ``stream`` is a hipStream_t passed as void*; NULL is the null stream.
 *    Every call enqueues its work on it and returns once that work is done.
 *  - Return codes: 0 = success, negative = error (nothing useful was
 *    written), positive = warning.  firls_last_error() gives a message
 *    for the calling thread.
 *  - A handle is not thread-safe: one caller at a time.
 */
#ifndef FIRLS_H
#define FIRLS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct firls_handle firls_handle;

enum {
  FIRLS_OK = 0,
  FIRLS_E_INVALID = -1,      /* bad argument (message says which) */
  FIRLS_E_UNSUPPORTED = -2,  /* valid but not built (size, levels) */
  FIRLS_E_HIP = -3,          /* a HIP runtime call failed */
  FIRLS_E_NOMEM = -4,        /* device allocation failed */
  FIRLS_E_NONFINITE = -5,    /* objective became NaN or Inf */
  FIRLS_E_SYNC = -6,         /* workgroups of a slice did not meet at a barrier
                                within its time limit (internal error) */
  FIRLS_E_BREAKDOWN = -7,    /* PCG: <p, S p> <= 0 with <r, z> > 0, impossible for
                                the Hermitian positive definite S of eq. (15) /
                                eq. (39) in exact arithmetic (Section 3.2) */
  FIRLS_W_MAXITER = 1,       /* stopped at max_outer before the tolerance */
  FIRLS_W_NONMONOTONE = 2    /* F_eps rose between outer iterations by more than
                                rounding (1e-6 relative in FP32, 1e-12 in FP64),
                                against Theorem 2 (Section 3.3) */
};
/* Per-slice statuses (firls_report.status) use the same codes; FIRLS_E_INVALID
 * there means a TV slice whose mask leaves out the DC entry of some contrast:
 * the difference operators annihilate constant images, so without that
 * sample the minimiser is not unique.  Such a slice is not solved (its x is
 * left as given). */

/* Sparsifying transform Psi.  HAAR: orthonormal L-level 2D Haar (Section
 * 3, eq. 17).  TV: first-order differences with a periodic boundary,
 * (D1 x)[r,c] = x[r+1,c] - x[r,c], (D2 x)[r,c] = x[r,c+1] - x[r,c] mod n.
 * TV_PAPER: the difference matrices printed in Section 4.1 (ones on the
 * diagonal, minus ones one pixel above for D1 / to the left for D2, no
 * wrap), so (D1 x)[r,c] = x[r,c] - x[r-1,c] with (D1 x)[0,c] = x[0,c], and
 * likewise along rows. */
enum { FIRLS_PSI_HAAR = 0, FIRLS_PSI_TV = 1, FIRLS_PSI_TV_PAPER = 2 };

/* Measurement operator A.  FOURIER: A = R F, the masked unitary 2D DFT of
 * CS-MRI (Section 5.4).  DENSE: a real M x N matrix on the row-major image
 * vector (the random projections of Section 5.2); products with it run on
 * MFMA. */
enum { FIRLS_OP_FOURIER = 0, FIRLS_OP_DENSE = 1 };
enum { FIRLS_FP64 = 0, FIRLS_FP32 = 1 };

/* Preconditioner of the inner PCG.  PAPER is the paper's choice: eq. (17)
 * for Haar, the triangular factors of eq. (40) for TV.  JACOBI uses
 * diag(S)^{-1} and NONE is plain CG (the comparisons of Section 5.2). */
enum { FIRLS_PC_PAPER = 0, FIRLS_PC_JACOBI = 1, FIRLS_PC_NONE = 2 };

/* One image geometry and regulariser.
 *   n           image side; n in {16, 32, 48, 64, 96, 128, 192, 256, 384, 512}.
 *   psi         FIRLS_PSI_HAAR, FIRLS_PSI_TV or FIRLS_PSI_TV_PAPER.
 *   levels      Haar levels, 1 <= L <= 4, n % 2^L == 0.  Ignored for TV.
 *   n_groups    number of groups s; 0 with NULL pointers selects the
 *               default map: singletons for Haar (standard sparsity), pixel
 *               pairs {D1 row p, D2 row p} for TV (isotropic TV, eq. 35).
 *   group_ptr   host int32[n_groups + 1], CSR offsets (group_ptr[0] = 0).
 *   group_idx   host int32[group_ptr[n_groups]]: members of each group as
 *               rows of the transform output.  Haar: Mallat index r * n + c
 *               of the coefficient (top-left block = coarsest approximation,
 *               level-l details in [0,h)x[h,2h), [h,2h)x[0,h), [h,2h)^2
 *               with h = n / 2^l).  TV, TV_PAPER: p for (D1 x)[p],
 *               N + p for (D2 x)[p], N = n^2, p = r * n + c.  A coefficient may sit in several groups
 *               (overlap through G, Section 3.1, Fig. 1); a coefficient in
 *               no group is not penalised.
 *   channels    C contrasts reconstructed jointly (Section 5.6: FIRLS_MT
 *               with groups across contrasts, FIRLS_JTV); 0 or 1 for a single
 *               image.  The C images are one problem: b, mask and x of a
 *               slice are C contiguous n x n images, A and Psi act on each,
 *               one PCG solves each reweighted system and rho is the sampled
 *               fraction over all C masks.  Transform rows are numbered
 *               contrast by contrast: Haar c * N + j; TV D1 rows of every
 *               contrast (c * N + p), then D2 rows (C * N + c * N + p).  The
 *               default map (n_groups = 0) groups row j (Haar) or the D1 and
 *               D2 rows of pixel p (TV) across all contrasts.  Requires
 *               C * (n / 16 + n / 16) <= 512 (and C * n^2 / 512 <= 512 for
 *               TV); the learned start needs C = 1.
 *   op          FIRLS_OP_FOURIER (default, 0) or FIRLS_OP_DENSE.
 *   m, A        DENSE only: m measurements (1 <= m <= 32768) and the host
 *               matrix A, double[m * n^2], row-major (row i is measurement
 *               i on the row-major image).  rho = ||A||_F^2 / n^2, the mean
 *               of diag(A^T A) (eq. 17).  A slice's b then holds m complex
 *               values and its mask is not read (may be NULL).  Needs
 *               channels = 1 and n^2 % 64 == 0; not for the learned start.
 * The arrays are copied at create; the caller keeps ownership. */
typedef struct {
  int32_t n;
  int32_t psi;
  int32_t levels;
  int32_t n_groups;
  const int32_t* group_ptr;
  const int32_t* group_idx;
  int32_t channels;
  int32_t op;
  int32_t m;
  const double* A;
} firls_shape;

/* Solver configuration.
 *   max_slices  largest batch a solve call may pass (>= 1).
 *   prec        FIRLS_FP32 (vectors float2, PCG scalars and every reduction
 *               in FP64) or FIRLS_FP64 (everything double).
 *   eps         smoothing of the weights, eq. (12); > 0 (paper: 1e-10).
 *   max_outer   T_max: largest number of reweighted solves (>= 0).
 *   pcg_iters   K: PCG iterations per outer iteration, 1..64 (Section 3.2
 *               reports 10 to 30 sufficient).
 *   outer_tol   tau: stop once (F_eps^{k-1} - F_eps^k) <= tau F_eps^k; 0
 *               runs max_outer solves.
 *   pcg_rtol    eta in [0, 1): the PCG stopping criterion of Algorithms 2
 *               and 3, which the paper leaves open, read as a relative
 *               preconditioned-residual test: a solve stops after iteration
 *               j once <r_j, P^{-1} r_j> <= eta^2 <r_0, P^{-1} r_0>
 *               (x keeps that iterate; the report counts the iterations
 *               taken); the launches of the remaining iterations return at
 *               once for that slice.  0 runs exactly pcg_iters iterations
 *               per solve.
 *   precond     FIRLS_PC_*.
 *   workspace   optional caller-owned device buffer (256-byte aligned) of
 *               workspace_bytes >= firls_workspace_bytes(cfg) bytes for the
 *               per-slice vectors, weights and partial sums of every solve
 *               (a torch tensor, say); NULL lets the library allocate and
 *               grow its own on demand.  It must stay valid until
 *               firls_destroy and is used by one call at a time.  The
 *               learned start's staging and the split-K scratch of dense
 *               sensing matrices are still the library's. */
typedef struct {
  int32_t n_shapes;
  const firls_shape* shapes;
  int32_t max_slices;
  int32_t prec;
  double eps;
  int32_t max_outer;
  int32_t pcg_iters;
  double outer_tol;
  double pcg_rtol;
  int32_t precond;
  void* workspace;
  size_t workspace_bytes;
} firls_config;

/* One image to reconstruct.  b, mask and x are device pointers of the
 * layouts above; x is read (when x_is_init != 0, the warm start x^1) and
 * overwritten with the result.  With x_is_init == 0 the solve starts from
 * x^1 = A^H b (Section 3.3). lambda > 0. */
typedef struct {
  int32_t shape_id;
  int32_t x_is_init;
  double lambda;
  const void* b;
  const uint8_t* mask;
  void* x;
} firls_slice;

/* Per-slice result.  F_eps = 1/2||Ax-b||^2 + lambda sum sqrt(||(Psi x)_g||^2
 * + eps) and F (eps = 0) of the returned x; rel_change = (F_eps^{prev} -
 * F_eps) / F_eps at the last evaluation (0 if only one). */
typedef struct {
  int32_t status;
  int32_t outer_iters;
  int32_t pcg_iters;
  int32_t converged;
  double F;
  double F_eps;
  double data;
  double rel_change;
} firls_report;

/* Build a handle: validates the shapes, copies the group maps to the
 * device (remapped to the library's tile-major coefficient layout) and
 * uploads twiddle tables.  Allocates device memory; the per-slice
 * workspace is allocated on the first solve that needs it. */
int firls_create(const firls_config* cfg, firls_handle** out);

/* Release the handle and all device memory it owns (NULL is a no-op). */
int firls_destroy(firls_handle* h);

/* Device bytes of the workspace a handle for this configuration needs to
 * solve any batch of up to max_slices slices of its shapes at once:
 * max_slices times the largest per-slice workspace (about 3.6 MB for a
 * 256^2 FP32 Haar slice).  0 for an invalid configuration.  Computed from
 * the configuration alone (no device calls), so a caller can allocate the
 * buffer before firls_create. */
size_t firls_workspace_bytes(const firls_config* cfg);

/* Device bytes of the workspace of ``n`` slices of shape ``shape_id`` (a
 * streamed batch needs only its slots' worth). */
size_t firls_slice_workspace_bytes(const firls_handle* h, int32_t shape_id, int32_t n);

/* FIRLS_OG (Algorithm 2) or FIRLS_TV (Algorithm 3) on one slice.  Blocks
 * until the report is written. */
int firls_solve(firls_handle* h, void* stream, const firls_slice* slice, firls_report* report);

/* Many independent slices of any configured shapes in one call; slices of
 * the same shape share every launch, converged slices drop out at outer
 * iteration boundaries.  reports[i] belongs to slices[i].  Returns the
 * worst status (error < 0 first, else the largest warning);
 * FIRLS_E_INVALID for n_slices <= 0 or more than the handle's max_slices
 * in one sub-batch, before any work. */
int firls_solve_batched(firls_handle* h, void* stream, int32_t n_slices,
                        const firls_slice* slices, firls_report* reports);

/* For callers that cannot allocate device memory during a solve: code
 * running under HIP graph capture, tight serving loops, harnesses that
 * forbid allocation.  Same as firls_solve_batched (same kernels, bitwise the
 * same reports and x), but it allocates nothing: the slice tables, states
 * and per-slice workspace live in a fixed array of
 * FIRLS_NOALLOC_SCRATCH_BYTES (64 MiB) of device memory per GPU, which the
 * library holds from its load until the process ends (the host-side slice
 * tables were reserved for max_slices by firls_create).  All slices run at
 * once with direct launches (the firls_set_chunk and firls_set_graphs
 * settings do not apply); masked-FFT shapes only.  A batch whose tables and
 * workspace do not fit (about 3.6 MB per 256^2 FP32 Haar slice, 17 such
 * slices) is rejected with FIRLS_E_INVALID before any work.  Every call on
 * a GPU shares that GPU's array, so calls that overlap in time on one GPU
 * (from several threads, handles or streams) race and must not be made;
 * each call initialises what it reads, so nothing carries over. */
#define FIRLS_NOALLOC_SCRATCH_BYTES ((size_t)64 << 20)
int firls_solve_batched_noalloc(firls_handle* h, void* stream, int32_t n_slices,
                                const firls_slice* slices, firls_report* reports);

/* ---- single-operator entry points (one slice; each blocks until done) -- */

/* x = A^H b = F^H (mask * b)  (the zero-filled start, Section 3.3). */
int firls_op_adjoint(firls_handle* h, void* stream, int32_t shape_id,
                     const void* b, const uint8_t* mask, void* x);

/* d = diag(G^T W G) for W = W(x) (eq. 12-13 / eq. 37-38), written to the
 * device array d_out (float or double per prec) in the caller's
 * transform-row order (Mallat for Haar, [D1; D2] rows for TV); length n^2
 * (Haar) or 2 n^2 (TV). */
int firls_op_weights(firls_handle* h, void* stream, int32_t shape_id,
                     const void* x, void* d_out);

/* q = S p = A^H A p + lambda Psi^T diag(d) Psi p with d = d(x_w)
 * (eq. 15 / eq. 39). */
int firls_op_system(firls_handle* h, void* stream, int32_t shape_id,
                    const uint8_t* mask, double lambda, const void* x_w,
                    const void* p, void* q);

/* z = P^{-1} r for the configured preconditioner at the weights of x_w
 * (FIRLS_PC_PAPER: eq. 17 exactly for Haar, SGS factors of eq. 40 for TV;
 * FIRLS_PC_JACOBI: r / diag(S); FIRLS_PC_NONE: z = r). */
int firls_op_precond(firls_handle* h, void* stream, int32_t shape_id,
                     const uint8_t* mask, double lambda, const void* x_w,
                     const void* r, void* z);

/* Host double[3] = {F_eps(x), F(x), 1/2||Ax - b||^2}; blocks. */
int firls_op_objective(firls_handle* h, void* stream, int32_t shape_id,
                       const void* b, const uint8_t* mask, double lambda,
                       const void* x, double* out3);

/* One reweighted solve: weights from x, then pcg_iters PCG iterations on
 * eq. (15) / (39) started at x; x is updated in place (one outer
 * iteration of Algorithm 2 / 3).  Blocks. */
int firls_op_outer_step(firls_handle* h, void* stream, int32_t shape_id,
                        const void* b, const uint8_t* mask, double lambda, void* x);

/* ---- learned warm start -------------------------------------------------- */

/* A small convolutional network gives the start x0 = A^H b + f(A^H b) of
 * FIRLS (the paper starts from A^H b, Section 3.3; any start keeps
 * Theorems 1-3).  f: five 3x3 "same" convolutions, channels 2 -> 32 -> 32 ->
 * 32 -> 32 -> 2, ReLU after the first four, on the real and imaginary parts
 * (bfloat16 weights and activations, FP32 accumulation on MFMA).  Parameter
 * order (28930 floats): for each layer W[dy][dx][cin][cout] then b[cout]. */
typedef struct firls_cnn firls_cnn;

int32_t firls_cnn_param_count(void);

/* Network for n x n images (n % 32 == 0) and batches up to max_batch. */
int firls_cnn_create(int32_t n, int32_t max_batch, firls_cnn** out);
int firls_cnn_destroy(firls_cnn* net);

/* Copy host float[28930] parameters in (resets the Adam state) / out. */
int firls_cnn_set_params(firls_cnn* net, const float* params);
int firls_cnn_get_params(const firls_cnn* net, float* params);

/* x0 = zf + f(zf) for a batch: zf, x0 device complex64 [batch, n, n]. */
int firls_cnn_forward(firls_cnn* net, void* stream, int32_t batch, const void* zf, void* x0);

/* Loss mean |x0 - label|^2 over pixels and real/imaginary parts, and its
 * gradient with respect to the parameters (host float[28930], may be NULL);
 * label device complex64 [batch, n, n].  Parameters unchanged. */
int firls_cnn_gradients(firls_cnn* net, void* stream, int32_t batch, const void* zf, const void* label,
                        float* grad, double* loss);

/* One Adam step (beta 0.9 / 0.999, eps 1e-8, bias-corrected) on the FP32
 * master parameters with learning rate lr; *loss gets the pre-step loss. */
int firls_cnn_train_step(firls_cnn* net, void* stream, int32_t batch, const void* zf, const void* label,
                         float lr, double* loss);

/* firls_solve_batched started from the network: every slice (FP32 handle,
 * image side = the network's) gets z = A^H b and x0 = z + f(z), then the
 * measured samples are put back into x0 (x0 <- F^H (m b + (1 - m) F x0));
 * x0 is kept where F_eps(x0) <= F_eps(z), else z (used_learned[i] = 1 / 0,
 * may be NULL); FIRLS then runs from there with the handle's tolerance. */
int firls_solve_batched_learned(firls_handle* h, firls_cnn* net, void* stream, int32_t n_slices,
                                const firls_slice* slices, firls_report* reports, int32_t* used_learned);

/* ---- execution tuning --------------------------------------------------- */

/* Each outer iteration launches the same kernels (reweighting, residual
 * and stop test, then the PCG iterations); by default they are captured
 * once as a HIP graph and replayed (enable = 0 launches them directly).
 * Either way the host launches iteration k + 1 once the stop test of
 * iteration k has reported, through host-mapped memory, while the GPU runs
 * iteration k's PCG launches (the calling thread busy-waits for it).  With the null stream the library works on its
 * own stream, ordered after the null stream's earlier work. */
int firls_set_graphs(firls_handle* h, int32_t enable);

/* Haar with the paper's preconditioner (FP32: every side; FP64: sides up
 * to 256): the row inverse pass of PCG iteration k - 1 and the step of
 * iteration k run in one launch, the workgroups of a slice meeting at a
 * barrier in between, so q stays on chip (default).  enable = 0 runs them
 * as two launches; results are bitwise the same. */
int firls_set_paired(firls_handle* h, int32_t enable);
/* 1 if the paired pass is enabled (firls_set_paired, firls_autotune), else 0;
 * FIRLS_E_INVALID for a null handle. */
int firls_get_paired(const firls_handle* h);

/* Test hook for the paired pass's error path: while enabled, its barrier
 * waits for one workgroup more than the slice has and gives up after a few
 * polls, so every slice that runs a paired launch ends with FIRLS_E_SYNC
 * (its results are then meaningless).  Every kernel still exits normally.
 * For tests only; off by default. */
int firls_test_sync_timeout(firls_handle* h, int32_t enable);

/* How a batch of several shapes is launched.  PER_SHAPE: every kernel of an
 * outer iteration once per shape.  ACROSS, ACROSS_LARGEST_FIRST: the k-th
 * launch of every shape's sequence becomes one launch per kernel class and
 * mode covering all shapes (a work table gives each workgroup its slice,
 * block and parameters), with the shapes' workgroups in shape order or
 * largest images first.  Batches
 * of one shape, streamed batches, dense sensing matrices and the
 * allocation-free solve always launch per shape.  firls_autotune chooses it
 * together with the sub-batch size and launch mode.  Each shape's kernels
 * are the same code either way; results agree to rounding (the compiler
 * may fuse multiply-adds differently in the two kernels). */
enum { FIRLS_SCHED_PER_SHAPE = 0, FIRLS_SCHED_ACROSS = 1, FIRLS_SCHED_ACROSS_LARGEST_FIRST = 2 };
int firls_set_schedule(firls_handle* h, int32_t schedule);
int firls_get_schedule(const firls_handle* h);

/* Test hooks: conditions forced from the host so the error paths run with
 * every kernel still exiting normally.  flags is a bit set (0 clears all):
 *   FIRLS_TEST_SYNC_TIMEOUT  as firls_test_sync_timeout;
 *   FIRLS_TEST_BREAKDOWN     every <p, S p> is taken as negative, so the first
 *                            PCG step of each slice records FIRLS_E_BREAKDOWN;
 *   FIRLS_TEST_NONMONOTONE   the monotonicity check's rounding slack becomes
 *                            -100%, so every evaluation after the first counts
 *                            as a rise and records FIRLS_W_NONMONOTONE.
 * For tests only; off by default. */
enum { FIRLS_TEST_SYNC_TIMEOUT = 1, FIRLS_TEST_BREAKDOWN = 2, FIRLS_TEST_NONMONOTONE = 4 };
int firls_test_hooks(firls_handle* h, int32_t flags);

/* Solve at most ``chunk`` slices at a time (0: the whole batch at once);
 * a smaller working set stays in the device's last-level cache.  A batch
 * of one masked-FFT shape is streamed: ``chunk`` slots start with the
 * first slices, and a slot whose slice has stopped takes the next one in
 * batch order at the following outer iteration, so slow slices do not hold
 * up the rest.  Other batches run in sub-batches of ``chunk`` slices, one
 * after the other.  Results do not depend on the setting. */
int firls_set_chunk(firls_handle* h, int32_t chunk);

/* Time a few outer iterations of these slices for candidate sub-batch sizes
 * (whole batch, 256, 128, 64, 32), each with graph replay and with direct
 * launches, for a batch of several masked-FFT shapes each schedule
 * (FIRLS_SCHED_*), and where a shape can use it with and without the paired
 * PCG pass, and keep the fastest: the sub-batch size is written to *chosen
 * and the launch mode (1 graphs, 0 direct) to *graphs (either may be NULL),
 * and all four stay set on the handle as firls_set_chunk, firls_set_graphs,
 * firls_set_schedule and firls_set_paired would set them
 * (firls_get_schedule and firls_get_paired read the last two).  Every x
 * is restored afterwards; on an error the handle keeps its earlier
 * settings.  With the environment variable FIRLS_TUNE_CACHE naming a file,
 * a previous choice for the same shape mix and batch size is reused, and
 * new choices are appended (one line each: key|chunk|graphs|schedule|paired). */
int firls_autotune(firls_handle* h, void* stream, int32_t n_slices, const firls_slice* slices, int32_t* chosen,
                   int32_t* graphs);

/* ---- instrumentation -------------------------------------------------- */

/* Kernel classes timed by firls_profile (index into the stats array). */
enum {
  FIRLS_PROF_INIT = 0,      /* per-slice state and rho */
  FIRLS_PROF_AHB = 1,       /* zero-filled start A^H b (two passes) */
  FIRLS_PROF_PSI_SQ = 2,    /* |Psi x|^2 */
  FIRLS_PROF_GROUP_W = 3,   /* group weights W and penalty partials */
  FIRLS_PROF_GROUP_D = 4,   /* d = diag(G^T W G) */
  FIRLS_PROF_R0_ROWFWD = 5, /* residual A^H b - S x: row FFT (Haar: and |Psi x|^2) */
  FIRLS_PROF_R0_COL = 6,    /*   column pass with the data term (dense A: b - A x, A^T y) */
  FIRLS_PROF_R0_ROWINV = 7, /*   row inverse FFT + regulariser (Haar: and <r0, z0>) */
  FIRLS_PROF_R0_UPDATE = 8, /*   TV: z0 and <r0, z0> */
  FIRLS_PROF_CHECK = 9,     /* objective and stop rule */
  FIRLS_PROF_ROWFWD = 10,   /* PCG: first p and row FFT (Haar), or p = z + beta p and row FFT (TV) */
  FIRLS_PROF_COL = 11,      /* PCG: column FFT, mask, column inverse FFT (dense A: A p, A^T y) */
  FIRLS_PROF_ROWINV = 12,   /* PCG: row inverse FFT + regulariser, <p, q> (Haar: and <q, P^{-1} q>) */
  FIRLS_PROF_UPDATE = 13,   /* PCG: x, r update, z and <r, z> (Haar: and the next p and row FFT) */
  FIRLS_PROF_LAST_X = 14,   /* PCG, Haar: x += alpha p after the last iteration */
  FIRLS_PROF_CLASSES = 15
};

typedef struct {
  char name[32];
  int64_t launches;        /* launches timed */
  int64_t slice_launches;  /* sum over those launches of the active slices */
  double ms;               /* sum of HIP-event durations */
} firls_kernel_stat;

/* enable != 0: time every kernel launch of the solve entry points with a
 * HIP event pair on the solve's stream and accumulate per class (resets
 * the totals).  enable == 0 stops timing (totals are kept until the next
 * enable).  Timing adds two event records per launch. */
int firls_profile(firls_handle* h, int32_t enable);

/* Copy up to n class totals into out; returns the number written. */
int firls_profile_read(const firls_handle* h, int32_t n, firls_kernel_stat* out);

/* The same totals restricted to the launches of one shape (a batch mixing
 * shapes launches every kernel once per shape present). */
int firls_profile_read_shape(const firls_handle* h, int32_t shape_id, int32_t n, firls_kernel_stat* out);

/* Thread-local text of the last error (empty string if none). */
const char* firls_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* FIRLS_H */
