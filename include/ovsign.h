/*
 * ovsign -- sgn(gamma5 Dw(mu)) b for the overlap operator at nonzero chemical
 * potential, on one AMD Instinct MI355X (gfx950).
 *
 * The operation follows Bloch, Breu and Wettig, "Comparing iterative methods
 * to compute the overlap Dirac operator at nonzero chemical potential"
 * (Lattice 2008):
 *   - Section 1: Dw(mu) = 1 - kappa sum_i (T_i^+ + T_i^-)
 *                         - kappa (e^mu T_4^+ + e^-mu T_4^-),
 *     (T_nu^{+-})_{yx} = (1 +- gamma_nu) U_{x,+-nu} delta_{y,x+-nu},
 *     kappa = 1/(8 + 2 m_w), and D_ov(mu) = 1 + gamma5 sgn(gamma5 Dw(mu)).
 *   - Section 1, eq. for sgn(z): sgn(z) = sgn(Re z) on eigenvalues.
 *   - Section 3: LR deflation with left/right critical eigenvectors,
 *     L^dagger R = I, computed once for all sources.
 *   - Section 4: two-sided Lanczos, f(A) b ~ R f(Lambda) L^dagger b
 *                + |b_R| V_k f(G_k) e_1 (eq. 2sLapp).
 *   - Section 2: Arnoldi, the same with the Hessenberg H_k (eq. Arnapp).
 *
 * Conventions (shared with the caller):
 *   - Site index s = x + Lx*(y + Ly*(z + Lz*t)).
 *   - Links: complex128 (re, im interleaved) [V][4][3][3], direction 0..3 with
 *     3 = time; U_{x,-nu} is taken as U_{x-nu,nu}^dagger.
 *   - Spinor fields: complex128 [nrhs][V][4][3]  (N = 12 V per source).
 *   - Euclidean chiral gamma basis, gamma5 = diag(1, 1, -1, -1) in spin.
 *   - bc[nu] = +1 periodic, -1 antiperiodic; the sign sits on the link that
 *     leaves the last slice in direction nu.
 *
 * Ownership: the caller owns every buffer it passes.  Pointers documented as
 * "device" must be device memory of the current HIP device; "host" pointers
 * are ordinary host memory.  The library copies links and eigentriples into
 * its own storage and never frees caller memory.  All work is enqueued on the
 * stream given at lattice creation; calls that return results to the host
 * (sign_apply, the timing calls) synchronise that stream before returning.
 *
 * Errors: every call returns an ovs_status; nothing throws or aborts across
 * this boundary.  Negative values are errors (outputs undefined), positive
 * values are warnings (outputs valid, see ovs_rhs_info).  A handle must not be
 * used from two host threads at once.
 */
#ifndef OVSIGN_H
#define OVSIGN_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t ovs_status;
#define OVS_OK                   0
#define OVS_WARN_NOT_CONVERGED   1  /* tolerance not reached within k_max        */
#define OVS_WARN_BREAKDOWN       2  /* serious Lanczos breakdown (delta ~ 0)      */
#define OVS_WARN_SIGN_AMBIGUOUS  3  /* inner quadrature error above its target:   */
                                     /* a Ritz value near the imaginary axis, where */
                                     /* sgn(z) = sgn(Re z) jumps (Section 1)        */
#define OVS_ERR_ARG             -1  /* invalid argument                           */
#define OVS_ERR_HIP             -2  /* HIP runtime error                          */
#define OVS_ERR_ALLOC           -3  /* device allocation failed                   */
#define OVS_ERR_STATE           -4  /* handle not ready (e.g. links not set)      */

typedef enum { OVS_F64 = 0, OVS_F32_STORE = 1 } ovs_precision;
typedef enum { OVS_OP_DW = 0, OVS_OP_DW_DAG = 1, OVS_OP_A = 2, OVS_OP_A_DAG = 3 } ovs_op;
typedef enum { OVS_2SL = 0, OVS_ARNOLDI = 1 } ovs_method;

enum {
  OVS_FLAG_TWO_PASS = 1,  /* 2sL: do not store V_k; replay the recurrence (end of Section 5) */
  OVS_FLAG_GRAPH    = 4,  /* replay the Lanczos iterations as captured HIP graphs             */
  OVS_FLAG_OVERLAP  = 8,  /* return D_ov b = b + gamma5 sgn(A) b instead of sgn(A) b         */
  OVS_FLAG_NO_SPLIT = 16, /* run a batch of 8 or more sources as one batch, not two halves    */
  OVS_FLAG_PERSISTENT = 32 /* 2sL: run the iterations in persistent cooperative launches      */
};
enum {
  OVS_VJP_STORE_BASIS = 1 /* ovs_sign_apply_vjp: keep both bases instead of recomputing them */
};

typedef struct ovs_lattice_s* ovs_lattice;
typedef struct ovs_deflation_s* ovs_deflation;
typedef struct ovs_field_s* ovs_field;

/* Per-source result record of ovs_sign_apply. */
typedef struct {
  int32_t k_used;        /* Krylov size actually used                                  */
  int32_t status;        /* OVS_OK or a warning code for this source                   */
  double est_rel_err;    /* convergence estimate: relative change of y on 512 sampled
                            entries over the last 25 iterations (0 without tol)        */
  double quad_err;       /* estimated relative error of x = sgn(G_k) e_1: the coarse/fine
                            difference of the quadrature at the step that met its target
                            (3e-7, or tol/10 if smaller but at least 1e-12, the FP64
                            rounding level of the difference) or at the finest step, 1/64;
                            above the target the status is OVS_WARN_SIGN_AMBIGUOUS     */
  double n_b;            /* |b_R|, norm of the deflated source                         */
  double t_defl_ms, t_krylov_ms, t_inner_ms, t_combine_ms; /* phase times (whole batch) */
  int32_t fp64;          /* 1: y was computed with FP64 vector storage                 */
  int32_t escalated;     /* 1: FP32 storage stalled (below) and the source was solved
                            again with FP64 storage                                    */
  double min_abs_delta;  /* 2sL: smallest |delta_i| / (|v~_i| |w~_i|) over the
                            iterations (Section 4: delta = w~^dagger v~; a serious
                            breakdown below 1e-13); -1 for Arnoldi or k < 2          */
  double biorth_err;     /* OVS_DEBUG_CHECKS, 2sL one-pass: largest |w_j^dagger v_i -
                            delta_ij| of the rows j checked every 25 iterations and at
                            the end (Section 4 keeps W^dagger V = I only in exact
                            arithmetic); else -1                                       */
  double ritz_min_re;    /* OVS_DEBUG_CHECKS: smallest |Re theta| / |theta| over the
                            eigenvalues theta of G_k (H_k) by a dense eigensolve; else -1 */
  double inner_check_err;/* OVS_DEBUG_CHECKS: relative difference of the quadrature's
                            x from the spectral sgn(G_k) e_1 of that eigensolve; else -1 */
} ovs_rhs_info;

/* Debug flags of ovs_set_debug. */
#define OVS_DEBUG_CHECKS 1
#define OVS_DEBUG_PROGRESS 2   /* ovs_deflation_compute prints its progress (subspace passes,
                                  inner solves, restarts) to stderr */
#define OVS_DEBUG_RANGES 4     /* roctx ranges around each call and its phases (deflation,
                                  Lanczos, inner sign, combination; the gradient's and the
                                  eigensolver's phases), for rocprofv3 --marker-trace */

/* ---- lattice ------------------------------------------------------------ */

/* Create a lattice handle.  dims = {Lx, Ly, Lz, Lt}, each >= 2 and Lx*Ly*Lz*Lt
 * <= 2^24 (the kernels address one source field with 32-bit byte offsets);
 * bc = {+-1, +-1, +-1, +-1}; prec selects the storage type of links
 * and Krylov vectors (coefficients, dots and deflation are always FP64);
 * hip_stream is a hipStream_t (NULL = default stream).  Section 1 defines the
 * lattice operator this handle applies.  Errors: OVS_ERR_ARG for bad
 * dims/bc/prec, OVS_ERR_ALLOC. */
ovs_status ovs_lattice_create(const int32_t dims[4], const int32_t bc[4], ovs_precision prec,
                              void* hip_stream, ovs_lattice* out);
ovs_status ovs_lattice_destroy(ovs_lattice lat);

/* Copy gauge links U_{x,nu} in SU(3) (Section 1) into the handle.  U:
 * complex128 [V][4][3][3], device memory if on_device != 0, else host memory
 * (copied to the device through a temporary buffer the call allocates and
 * frees; the call then returns after the copy).  The library keeps its own
 * packed copy (FP64 or FP32 per prec) with the boundary signs folded in. */
ovs_status ovs_set_links(ovs_lattice lat, const void* U, int32_t on_device);

/* Set m_w and mu (Section 1): kappa = 1/(8 + 2 m_w).  OVS_ERR_ARG if
 * 8 + 2 m_w <= 0 or a value is not finite. */
ovs_status ovs_set_params(ovs_lattice lat, double m_w, double mu);

/* Diagnostics of later ovs_sign_apply calls on this handle.
 *   flags        : OVS_DEBUG_CHECKS and/or OVS_DEBUG_PROGRESS.  With
 *                  OVS_DEBUG_CHECKS the 2sL
 *                  biorthogonality w_j^dagger V_j (Section 4: W^dagger V = I,
 *                  which short recurrences keep only in exact arithmetic) is
 *                  measured every 25 iterations and at the end against the
 *                  stored basis (one-pass only), and the inner sign is checked
 *                  against a dense eigendecomposition of G_k (H_k) on the host,
 *                  O(k^3) per source (Section 1, eq. for f(A)); results in
 *                  ovs_rhs_info.  A Ritz value with |Re theta| <= 1e-12 |theta|
 *                  then also returns OVS_WARN_SIGN_AMBIGUOUS.
 *   breakdown_at : >= 0: the 2sL beta step of that iteration (0-based) takes
 *                  delta = 0, the serious breakdown of Section 4 (the source
 *                  stops with k = breakdown_at + 1 and OVS_WARN_BREAKDOWN; y
 *                  is the result of that k); -1: none.  For testing the
 *                  breakdown path; applies to every source of a call.
 * OVS_ERR_ARG for unknown flags or breakdown_at < -1. */
ovs_status ovs_set_debug(ovs_lattice lat, int32_t flags, int32_t breakdown_at);

/* y = op x for nrhs sources (Section 1).  x, y: device complex128
 * [nrhs][V][4][3], must not alias.  OVS_OP_A is gamma5 Dw(mu), OVS_OP_A_DAG its
 * adjoint (= gamma5 Dw(-mu)), OVS_OP_DW_DAG = gamma5 Dw(-mu) gamma5.  In
 * OVS_F32_STORE mode the stencil runs in FP32 (inputs rounded to FP32). */
ovs_status ovs_apply(ovs_lattice lat, ovs_op op, const void* x, void* y, int32_t nrhs);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): ovs_apply
 * with the same arguments, stream semantics and results (the same kernels),
 * but its two staging fields (the packed input and output) live in a fixed
 * per-device scratch array of OVS_APPLY_NOALLOC_MAX_BYTES held by the library
 * until the process ends, so the call allocates and frees nothing.
 * 2 * nrhs * 12 * Vs * (16 for OVS_F64, 8 for OVS_F32_STORE) bytes must fit,
 * Vs = V rounded up to a multiple of 64, plus 64 (each field rounded up to 256
 * bytes): OVS_ERR_ARG otherwise (e.g. 16^3 x 32 FP64: one source; 16^4 FP32:
 * up to five).  Every call on one GPU shares that GPU's scratch and leaves its
 * contents behind: calls that overlap on one GPU (two streams, two host
 * threads) race and must be serialised by the caller. */
#define OVS_APPLY_NOALLOC_MAX_BYTES (64ull << 20)
ovs_status ovs_apply_noalloc(ovs_lattice lat, ovs_op op, const void* x, void* y, int32_t nrhs);

/* ---- resident fields (library layout, for repeated stencil application) -- */

/* A field of nrhs sources in the library's private layout and storage type. */
ovs_status ovs_field_create(ovs_lattice lat, int32_t nrhs, ovs_field* out);
ovs_status ovs_field_destroy(ovs_field f);
/* Import from / export to device complex128 [nrhs][V][4][3]. */
ovs_status ovs_field_import(ovs_field f, const void* x);
ovs_status ovs_field_export(ovs_field f, void* x);
/* out = op in, both resident (same nrhs, distinct fields).  Enqueues one
 * stencil kernel launch on the lattice stream and does not synchronise. */
ovs_status ovs_field_apply(ovs_lattice lat, ovs_op op, ovs_field in, ovs_field out);
/* Launch ovs_field_apply `iters` times back to back and return the average
 * kernel time in milliseconds measured with HIP events on the lattice stream. */
ovs_status ovs_field_apply_timed(ovs_lattice lat, ovs_op op, ovs_field in, ovs_field out,
                                 int32_t iters, double* ms_per_apply);
/* Launch the tuned dual stencil of the two-sided Lanczos step (Section 4:
 * A v~ and A^dag w~ with the partial sums of w~^dagger A v~ and |A v~|^2) for
 * all nrhs sources of v, with v~ = v and w~ = a copy of v in library
 * workspace (distinct memory, as in a solve), `iters` times back to back into
 * library workspace, and return the average kernel time in milliseconds
 * measured with HIP events on the lattice stream.  v is only read.  For
 * measurement; OVS_ERR_ARG for a field of another lattice or iters < 1. */
ovs_status ovs_dual_apply_timed(ovs_lattice lat, ovs_field v, int32_t iters, double* ms_per_apply);
/* Choose the RHS block and launch shape of the stencil for this nrhs by timing
 * the candidates (the choice is kept in the lattice handle). */
ovs_status ovs_autotune(ovs_lattice lat, int32_t nrhs);
/* Current tuned stencil configuration: rhs block and workgroup size. */
ovs_status ovs_get_tuning(ovs_lattice lat, int32_t nrhs, int32_t* rhs_block, int32_t* wg_size);
/* Full tuned configuration for nrhs sources, host int32 [8]:
 * {stencil shape = 1000*staged tile + 100*rhs block + 10*lanes per site +
 *  streaming stores (staged tile: the workgroup's own input spinors copied to
 *  LDS, lanes per site 1 and rhs block <= 4 in FP32, <= 2 in FP64),
 *  stencil workgroup size, stencil LDS cap KiB, stencil block order,
 *  Lanczos dual-stencil shape = 100*rhs block + 10*variant + streaming stores
 *  (bit 0: the dual stencil's outputs, bit 1: the new Lanczos vectors of the
 *  update)
 *  (variant 1: one thread computes A v and A^dag w; 2: a lane pair splits the two
 *  operators; 3: as 2 with the tile's spinors staged in LDS, rhs block <= 2 in
 *  FP32, 1 in FP64; 4: one operator per workgroup, the two workgroups of a tile
 *  adjacent on one XCD; 5: as 4 with the tile's spinors staged in LDS; 6: one
 *  operator and one source per workgroup, marching along t through the XCD's
 *  time chunk with the time neighbours in registers and the plane in LDS, FP32
 *  storage, rhs block 1, Lx Ly = 256 and Lt a multiple of 8, block order 0 (sources of a
 *  column adjacent) or 1 (columns of a source adjacent)), its workgroup size
 *  (512 for variants 2 and 3, else 256), its LDS cap KiB, its block order}.  Block order: 0 = the source blocks of a tile adjacent; 1 =
 *  source block slowest; 2 to 7 = each XCD sweeps its chunk of time slices
 *  once per window of 1, 2, 3, 4, 6 or all source blocks (lattices whose Lx Ly
 *  is a multiple of the tile and Lt of 8; otherwise as 0). */
ovs_status ovs_get_tuning_ex(ovs_lattice lat, int32_t nrhs, int32_t out[8]);
/* Install a configuration in the encoding of ovs_get_tuning_ex (e.g. one saved
 * from an earlier ovs_autotune).  OVS_ERR_ARG for values the kernels do not
 * provide. */
ovs_status ovs_set_tuning_ex(ovs_lattice lat, int32_t nrhs, const int32_t cfg[8]);

/* ---- deflation (Section 3) -------------------------------------------- */

/* Supply m critical eigentriples: lambda host complex128 [m]; R, L device
 * complex128 [m][V][4][3] (column j of R_m / L_m is row j).  The library
 * copies them (FP64) and checks |L^dagger R - I|_max <= 1e-8 and
 * |A r_j - lambda_j r_j| <= 1e-6 |lambda_j| (OVS_ERR_ARG otherwise). */
ovs_status ovs_deflation_set(ovs_lattice lat, int32_t m, const double* lambda, const void* R,
                             const void* L, ovs_deflation* out);
/* Compute the m critical eigentriples on the GPU (Section 5 obtains them with
 * ARPACK; here shift-and-invert Krylov-Schur on A^{-1} and on A^dagger^{-1},
 * each inverse applied by conjugate gradients on the normal equations started
 * from a deflation space of small singular vectors, then Rayleigh-Ritz on A,
 * pairing lambda_L = conj(lambda_R) and L <- L (L^dagger R)^{-dagger}; FP64
 * throughout, also on FP32 lattices).  tol: target relative residual
 * |A r - lambda r| / |lambda| (and the same for the left vectors), 1e-10
 * typical; max_iter: Krylov-Schur restarts per side (30 is ample).  Returns
 * OVS_WARN_NOT_CONVERGED (handle still created) if tol or |L^dagger R - I| <=
 * 1e-6 was not reached.  Cost grows with the condition number of A (an inner
 * CG solve per Krylov vector). */
ovs_status ovs_deflation_compute(ovs_lattice lat, int32_t m, double tol, int32_t max_iter,
                                 ovs_deflation* out);
/* Copy out eigenvalues (host complex128 [m]), R and L (device complex128
 * [m][V][4][3]) and info (host double [3]: max relative residual of right
 * and left vectors, max |L^dagger R - I|, Krylov-Schur restarts of both
 * sides; for supplied triples the checked values).  Any pointer may be NULL. */
ovs_status ovs_deflation_get(ovs_deflation d, double* lambda, void* R, void* L, double* info);
ovs_status ovs_deflation_destroy(ovs_deflation d);

/* ---- sign function ------------------------------------------------------ */

/* Bytes of caller workspace an ovs_sign_apply call with these arguments
 * needs (its `workspace` argument): both halves of a batch that is split, with
 * convergence checks, and the one-pass basis for k_max vectors (at 16^3 x 32
 * with 12 sources and k_max = 1000, about 150 GB in FP32 storage;
 * OVS_FLAG_TWO_PASS keeps three vectors: 2.6 GB).  No device work, and links
 * need not be set; OVS_ERR_ARG as for ovs_sign_apply. */
ovs_status ovs_workspace_size(ovs_lattice lat, ovs_deflation defl, int32_t n_defl, int32_t nrhs,
                              int32_t k_max, ovs_method method, int32_t flags, size_t* bytes);

/* Device memory (bytes) the handle holds for ovs_sign_apply calls without a
 * caller workspace: its cached workspace, the one-pass basis (grown in
 * doubling steps from 256 vectors as the iteration needs them, so a solve that
 * stops at k holds at most 2k of them, not k_max) and the gather buffer, plus
 * those of its internal second-half and FP64 handles.  Kept until
 * ovs_lattice_destroy. */
ovs_status ovs_workspace_held(ovs_lattice lat, size_t* bytes);

/* y = sgn(A) b (or D_ov b with OVS_FLAG_OVERLAP) for nrhs sources, A = gamma5
 * Dw(mu): LR-deflated two-sided Lanczos (eq. 2sLapp) or Arnoldi (eq. Arnapp).
 *   defl   : NULL for no deflation, else the first n_defl triples are used.
 *   b, y   : device complex128 [nrhs][V][4][3].
 *   k_max  : maximal Krylov size (1 <= k_max <= N).
 *   tol    : host [nrhs] target relative errors, or NULL to run exactly k_max
 *            steps.  With tol, a source stops when its estimate falls below
 *            tol/10, checked every 25 iterations (2sL and Arnoldi alike).  On an OVS_F32_STORE lattice
 *            the sources with tol < 1e-6 (below what FP32 storage attains) run
 *            as an FP64 group on the FP64 copy of the links; the rest in FP32.
 *            A source whose FP32-storage estimate has not halved over 6 checks
 *            (150 iterations) while above its target is stopped there and solved
 *            again with FP64 storage (info.escalated); FP32 rounding of the
 *            stored vectors can stall the recurrence for an individual source.
 *   workspace, ws_bytes : device memory the caller owns for this call
 *            (e.g. from torch's caching allocator), at least
 *            ovs_workspace_size bytes (OVS_ERR_ARG otherwise), used only
 *            during the call; or NULL for the handle's cached workspace
 *            (ovs_workspace_held).  On an OVS_F32_STORE lattice with tol, the
 *            caller's workspace serves the FP32 group; the FP64 group and the
 *            gather of a partial group use the handle's own memory.
 *   info   : host [nrhs] result records, or NULL.
 * Batches of 8 or more sources run as two halves at the same time, on the
 * handle's stream and on a second internal stream (each half with the whole
 * batch's tuned kernels); OVS_FLAG_NO_SPLIT runs them as one batch.
 * OVS_FLAG_PERSISTENT (2sL; ignored by Arnoldi): the iterations between
 * convergence checks run in cooperative launches of at most 25 iterations,
 * each iteration's phases (dual stencil, alpha, update, beta) separated by
 * grid barriers, with the one-operator-per-workgroup dual stencil at the
 * tuned source block (at most 2 in FP32, 1 in FP64) and LDS staging; the
 * batch is never split.  Results equal those of the per-step kernels with
 * the same dual-stencil configuration bit for bit.  OVS_ERR_HIP when the
 * device has no cooperative launch.
 * The inner function sgn(G_k) e_1 (or sgn(H_k) e_1) is evaluated on the GPU
 * in FP64 by a quadrature whose step is halved per source (from 1/4 down to
 * 1/64) until its error estimate meets 3e-7 and tol/10; a source that misses
 * it at the finest step has a Ritz value within a few degrees of the
 * imaginary axis and returns OVS_WARN_SIGN_AMBIGUOUS (y still written).
 * Returns the most severe per-source warning, or an error. */
ovs_status ovs_sign_apply(ovs_lattice lat, ovs_deflation defl, int32_t n_defl, const void* b,
                          void* y, int32_t nrhs, int32_t k_max, const double* tol,
                          ovs_method method, int32_t flags, void* workspace, size_t ws_bytes,
                          ovs_rhs_info* info);

/* Gradient of L = sum_r Re <chi_r, y_r>, where y_r = |b_r| V_k sgn(G_k) e_1 is
 * the two-sided Lanczos approximation of sgn(gamma5 Dw(mu)) b_r (Section 4,
 * eq. 2sLapp) at exactly k iterations, with respect to the sources, mu and
 * the links.  Without deflation: the exact derivative of that algorithm
 * (reverse sweep of its recurrences; the inner sign and its Jacobian by the
 * tau = e^u trapezoid rule).  With n_defl LR-deflation eigentriples (Section
 * 3), y_r = R S L^dagger b_r + the run from the deflated starts, and the
 * gradient is that of sgn(A) b_r through the eigentriples as well: the
 * Daleckii-Krein terms that couple the deflated eigenvalues with the rest
 * are formed from the eigentriples and from a second k-step two-sided
 * Lanczos run on A^dagger started from (1 - L R^dagger) chi (about twice the
 * undeflated cost).  The eigentriples must be those of A at the lattice's
 * current mu and links.  Complex gradients follow dL = Re <zbar, dz> with
 * zbar = dL/dRe z + i dL/dIm z; link matrices are differentiated entry by
 * entry (no projection on su(3)).
 *   defl, n_defl : as for ovs_sign_apply (n_defl = 0: no deflation).
 *   b, chi   : device complex128 [nrhs][V][4][3] (canonical layout).
 *   k        : Krylov size, 1 <= k <= 65535; every source must complete k
 *              iterations.
 *   flags    : 0: the Lanczos vectors are recomputed in the reverse sweep from
 *              checkpoints every ceil(sqrt k) steps (bitwise the forward ones);
 *              OVS_VJP_STORE_BASIS: both bases are kept instead (no replay,
 *              2k fields per source).
 *   y        : device complex128 [nrhs][V][4][3], or NULL: the forward result.
 *   grad_b   : device complex128 [nrhs][V][4][3].
 *   grad_mu  : host double [1], summed over sources.
 *   grad_U   : device complex128 [V][4][3][3] (link layout), summed over sources.
 *   quad_err : host double [nrhs], or NULL: relative change of the quadrature
 *              (x and the Jacobian band) between its last two step sizes.
 *   workspace, ws_bytes : caller device memory for this call, at least
 *              ovs_vjp_workspace_size bytes (OVS_ERR_ARG otherwise), or NULL for
 *              the handle's cached workspace.
 * Needs an OVS_F64 lattice (OVS_ERR_ARG otherwise) and FP64 workspace of about
 * (4k/c + 4c + 22) nrhs fields with c = ceil(sqrt k), or (2k + 2c + 18) nrhs
 * with OVS_VJP_STORE_BASIS, plus (k + 11) nrhs fields with deflation
 * (OVS_ERR_ALLOC if the handle's cache cannot grow to it).
 * Returns OVS_WARN_BREAKDOWN, writing no output, when a source (or the
 * second run) breaks down before k iterations, when with deflation a source
 * lies in span R (|b_R| <= 1e-12 |b|) or chi in span L, or when a deflated
 * eigenvalue is an eigenvalue of G_k; OVS_WARN_SIGN_AMBIGUOUS, with all outputs written, when
 * the quadrature changed by more than 1e-6 between its two finest steps. */
ovs_status ovs_sign_apply_vjp(ovs_lattice lat, ovs_deflation defl, int32_t n_defl, const void* b,
                              const void* chi, int32_t nrhs, int32_t k, int32_t flags, void* y,
                              void* grad_b, double* grad_mu, void* grad_U, double* quad_err,
                              void* workspace, size_t ws_bytes);

/* Bytes of caller workspace an ovs_sign_apply_vjp call with these arguments
 * needs.  No device work; OVS_ERR_ARG as for ovs_sign_apply_vjp. */
ovs_status ovs_vjp_workspace_size(ovs_lattice lat, ovs_deflation defl, int32_t n_defl,
                                  int32_t nrhs, int32_t k, int32_t flags, size_t* bytes);

/* Krylov coefficients of the last ovs_sign_apply on this handle (2sL only):
 * alpha, gamma host complex128 [nrhs][k_max], beta host double [nrhs][k_max],
 * x host complex128 [nrhs][k_max] (sgn(G_k) e_1, zero beyond k_used).  Any
 * pointer may be NULL.  For testing and diagnostics. */
ovs_status ovs_last_coefficients(ovs_lattice lat, double* alpha, double* beta, double* gamma,
                                 double* x);

/* x = sgn(T) e_1 for a batch of tridiagonal T (Section 4: G_k), on the GPU,
 * by the library's inner-sign quadrature (the same refinement as
 * ovs_sign_apply without tol: target 3e-7).  Host inputs: diag, super (gamma)
 * complex128 [batch][k]; sub (beta) complex128 [batch][k] (entry k-1 unused,
 * imaginary parts zero, else OVS_ERR_ARG).  Output x host complex128
 * [batch][k]; err host double [batch] (may be NULL): the estimate of each
 * x's relative error.  Returns OVS_WARN_SIGN_AMBIGUOUS (outputs written) if
 * an estimate is above the target: T has an eigenvalue near the imaginary
 * axis, where sgn(Re z) is ill-defined (Section 1). */
ovs_status ovs_inner_sign_tridiag(ovs_lattice lat, int32_t batch, int32_t k, const double* diag,
                                  const double* sub, const double* super, double* x, double* err);

/* x = sgn(H) e_1 for a batch of upper Hessenberg H (Section 2: H_k), column
 * major complex128 [batch][k][k] host; x host complex128 [batch][k]; err and
 * the returned status as for ovs_inner_sign_tridiag. */
ovs_status ovs_inner_sign_hessenberg(ovs_lattice lat, int32_t batch, int32_t k, const double* H,
                                     double* x, double* err);

/* su(3) force of a real function L of the links, from its link gradient (for
 * molecular-dynamics updates of the gauge field; the paper computes no forces):
 * for U -> exp(eps X) U with X traceless anti-Hermitian, dL/deps = sum over
 * links of Re tr(F^dagger X) with F = -TA(U G^dagger), TA(M) = (M - M^dagger)/2
 * - tr(M - M^dagger)/6 * 1, where G = dL/dRe U + i dL/dIm U is the gradient
 * ovs_sign_apply_vjp returns.
 *   U      : device complex128 [V][4][3][3], the links as given to ovs_set_links.
 *   grad_U : device complex128 [V][4][3][3].
 *   force  : device complex128 [V][4][3][3] (traceless anti-Hermitian), written.
 * Runs on the handle's stream.  OVS_ERR_ARG for NULL pointers. */
ovs_status ovs_link_force(ovs_lattice lat, const void* U, const void* grad_U, void* force);

/* ---- eigenvalues of the overlap operator (Sections 1 and 5) ------------- */

/* The nev eigenvalues of smallest magnitude of D_ov(mu) = 1 + gamma5 sgn(A)
 * (Section 1), with sgn(A) applied by the two-sided Lanczos driver (Section
 * 4; the closing outlook of Section 5 applies these methods to the overlap
 * operator's eigenvalues).  Block Arnoldi with thick restarts in Krylov-Schur
 * form: a basis of ncv vectors grown by one block of `block` vectors per step,
 * each step one batched sign solve of `block` sources (ovs_sign_apply,
 * OVS_FLAG_OVERLAP, deflated by the first n_defl triples of defl if not NULL),
 * classical Gram-Schmidt twice against the basis and Cholesky QR twice within
 * the block.  Harmonic Ritz pairs for the target 0 (ordinary Ritz pairs in a
 * cycle where the projected matrix is singular) are ordered by |theta|; each
 * is reported with the Rayleigh quotient of its vector.  At a restart the
 * vectors of about nev + (ncv - nev)/2 smallest |theta| are kept (rounded so
 * that whole blocks are added), with the block their residuals lie in.
 *   nev, ncv    : 1 <= nev, nev + 2 block <= ncv <= 256, ncv + block < N.
 *   block       : 1..16, ncv a multiple of it (1: plain Arnoldi).  The
 *                 wanted eigenvalues lie inside the spectrum; a cycle of
 *                 ncv/block steps builds a polynomial of that degree, and
 *                 fewer than ~20 steps can converge to other eigenvalues than
 *                 the smallest ones (measured at 8^4: block 4 with ncv 40 did).
 *   k_inner, tol_inner : k_max and target relative error of each sign solve.
 *   inner_flags : further flags of each sign solve: OVS_FLAG_GRAPH,
 *                 OVS_FLAG_TWO_PASS, OVS_FLAG_PERSISTENT (others: OVS_ERR_ARG).
 *   tol         : stop when every wanted Ritz pair (unit x) has the residual
 *                 estimate |D_ov x - theta x| <= tol; the inner solves' error
 *                 limits what tol can reach.
 *   max_restarts: restarts at most (0: one Arnoldi pass of ncv steps).
 *   lambda      : host complex128 [nev], ordered by increasing magnitude.
 *   vecs        : device complex128 [nev][V][4][3] unit Ritz vectors, or NULL.
 *   info        : host double [4] or NULL: largest residual estimate of the
 *                 wanted pairs, restarts, sources solved, sources whose sign
 *                 solve returned a warning.
 * The library allocates (ncv + block) + ncv FP64 fields of device memory for
 * the call and frees them on return.  OVS_WARN_NOT_CONVERGED if tol was not met
 * within max_restarts or an inner solve returned a warning (outputs still
 * written); OVS_WARN_BREAKDOWN if the basis could not be extended (an
 * invariant subspace or dependent Ritz vectors).  Errors: OVS_ERR_ARG,
 * OVS_ERR_STATE (links or parameters not set), OVS_ERR_ALLOC, OVS_ERR_HIP. */
ovs_status ovs_overlap_eigs(ovs_lattice lat, ovs_deflation defl, int32_t n_defl, int32_t nev,
                           int32_t ncv, int32_t block, int32_t k_inner, double tol_inner,
                           int32_t inner_flags, double tol, int32_t max_restarts,
                           double* lambda, void* vecs, double* info);

/* Eigen-decomposition of a small general complex matrix on the host (the
 * Rayleigh-Ritz step of ovs_deflation_compute): A host complex128 n x n,
 * column major; lambda host complex128 [n]; V host complex128 n x n, unit-norm
 * right eigenvectors as columns.  No GPU is used.  OVS_ERR_ARG if the QR
 * iteration does not converge. */
ovs_status ovs_small_eig(int32_t n, const double* A, double* lambda, double* V);

const char* ovs_status_string(ovs_status s);
/* Description of the last failing runtime call on this host thread (for
 * OVS_ERR_HIP); empty if none. */
const char* ovs_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* OVSIGN_H */
