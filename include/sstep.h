/*
 * sstep.h -- C ABI of libsstep.so: preconditioned s-step conjugate gradient
 * (Chronopoulos-Gear) on one AMD Instinct MI355X (gfx950).
 *
 * Method: Bernaschi, Carrozzo, Celestini, Piperno, D'Ambra, "Communication-
 * reduced Conjugate Gradient Variants for GPU-accelerated Clusters",
 * Euromicro PDP 2025 (arXiv 2501.03743):
 *   Alg. 3 (PCGs), Alg. 4 (pMPK), Alg. 5 (cvm), Alg. 6 (SW), Sec. II-A;
 *   Alg. 1 (PCG-HS) as the standard-CG comparator.
 *
 * Conventions for every entry point:
 *   - Return value: SSP_OK (0), a positive solver outcome (SSP_NOT_CONVERGED,
 *     SSP_BREAKDOWN) or a negative error code.  No C++ exception crosses the
 *     ABI.  After a negative return, ssp_last_error() describes the problem.
 *   - "device" pointers are HIP device allocations on the handle's device;
 *     "host" pointers are ordinary host memory.  The library never frees
 *     caller memory.
 *   - All device work is ordered on the handle's stream.  Calls that return
 *     results to the host (ssp_solve, the query functions) synchronise that
 *     stream; the others only enqueue work.
 *   - A handle is not thread-safe: use one handle per host thread.
 *   - Vectors are dense FP64 arrays of n entries; unknowns of grid operators
 *     are numbered lexicographically, index = x + nx*(y + ny*z).
 */
#ifndef SSTEP_H
#define SSTEP_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct ssp_handle ssp_handle;
typedef struct ssp_matrix ssp_matrix;

/* ---- status codes -------------------------------------------------------- */
#define SSP_OK 0              /* converged: ||r||_2 <= rtol ||b||_2            */
#define SSP_NOT_CONVERGED 1   /* iteration limit reached; x = last iterate
                                 (Alg. 1 and Alg. 3 "did not converge")         */
#define SSP_BREAKDOWN 2       /* non-SPD s x s Gram matrix, alpha_{i-1}(s) ~ 0 or
                                 a non-finite value; x = last good iterate      */
#define SSP_EINVAL (-1)       /* invalid argument                               */
#define SSP_ENOMEM (-2)       /* device allocation failed                       */
#define SSP_EHIP (-3)         /* HIP runtime error                              */
#define SSP_EUNSUPPORTED (-4) /* valid but not implemented combination          */

/* Largest block size s (the moment matrices are s x s). */
#define SSP_SMAX 16

/* ---- operator kinds (ssp_matrix_stencil) --------------------------------- */
#define SSP_STENCIL_2D5 1     /* 2D 5-point; default coef {4, -1}; nz must be 1 */
#define SSP_STENCIL_3D7 2     /* 3D 7-point; default coef {6, -1}               */
#define SSP_STENCIL_3D27 3    /* 3D 27-point; default coef {26, -1}             */
#define SSP_STENCIL_3D7_VARK 4/* -div(k grad u), 7-point: face weight
                                 2 k_p k_q / (k_p + k_q), weight k_p on faces to
                                 the boundary, diagonal = sum of the 6 weights   */

/* ---- flags of ssp_matrix_csr ---------------------------------------------- */
#define SSP_BORROW 0u         /* library keeps the caller's device arrays; they
                                 must outlive the matrix (default)              */
#define SSP_COPY 1u           /* library copies the arrays into its own memory  */
#define SSP_VALIDATE 2u       /* O(nnz) check: rowptr monotone from 0, column
                                 indices in range and ascending in each row, a
                                 positive diagonal entry in each row            */

/* ---- preconditioners ----------------------------------------------------- */
#define SSP_PREC_NONE 0       /* B = I (Sec. V-A "no preconditioning")          */
#define SSP_PREC_JACOBI 1     /* B = diag(A) (the weighted-Jacobi building block
                                 of the paper's AMG smoother, Sec. III-A)       */
#define SSP_PREC_AMG 2        /* B^-1 = one V-cycle of the aggregation AMG that
                                 ssp_set_amg builds (Sec. III-A)                */

/* ---- solver options ------------------------------------------------------ */
#define SSP_METHOD_SSTEP 0    /* Alg. 3 with Alg. 4-6                           */
#define SSP_METHOD_PCG 1      /* Alg. 1                                         */
#define SSP_METHOD_PFCG 2     /* Alg. 2: flexible PCG with one reduction per
                                 step (the paper's comparator); s is ignored    */

#define SSP_BASIS_MONOMIAL 0   /* Alg. 4's basis [z, Kz, ..., K^{s-1} z] with
                                 Alg. 5's 2s moments and Alg. 6                 */
#define SSP_BASIS_CHEBYSHEV 1  /* z_{j+1} = T_j((K - cI)/h) z over an interval
                                 [lo, hi] = [c - h, c + h] enclosing the
                                 spectrum of K = B^-1 A (the stabilised bases of
                                 the related work, Sec. IV); the s x (2s+1)
                                 inner products Z^T [AZ | AP_{i-1} | r] are
                                 formed in one pass on the FP64 matrix cores    */

#define SSP_PRECISION_FP64 0
#define SSP_PRECISION_MIXED_IR 1  /* FP32 inner s-step (matrix powers and block
                                     updates in FP32, moments and s x s solves
                                     in FP64) inside FP64 iterative refinement */

typedef struct ssp_opts {
  int method;          /* SSP_METHOD_*                                          */
  int precision;       /* SSP_PRECISION_*                                       */
  double inner_rtol;   /* MIXED_IR: relative tolerance of each inner solve      */
  int max_refine;      /* MIXED_IR: limit on refinement steps                   */
  int check_every;     /* outer iterations enqueued between host polls of the
                          device status word; 0 = library default               */
  int fixed_outer;     /* > 0: run exactly this many outer iterations with no
                          stopping test (stops early only on breakdown); the
                          result is SSP_OK if the residual test holds at the end */
  int profile;         /* 1: time every kernel class with HIP events on the
                          handle's stream (see ssp_get_profile)                 */
  int trace_cap;       /* > 0 with the trace_* host buffers: record per outer
                          iteration the moments vm(1..2s), alpha (s), beta (s*s,
                          beta(l,j) at [l*s+j]) and W (s*s, row-major), for up
                          to trace_cap iterations (synchronises every iteration;
                          for testing)                                          */
  double *trace_vm;    /* host, trace_cap * 2s                                  */
  double *trace_alpha; /* host, trace_cap * s                                   */
  double *trace_beta;  /* host, trace_cap * s * s                               */
  double *trace_W;     /* host, trace_cap * s * s                               */
  int warm_start;      /* 1: x holds a predicted initial guess (e.g. the warm-
                          start network's); it is judged by its true residual
                          before the solve and replaced by x = 0 when
                          ||b - A x|| >= ||b|| or not finite (see
                          ssp_get_warm_start)                                   */
  int warm_sweeps;     /* warm start only: damped Jacobi sweeps
                          x += omega B^-1 (b - A x) applied to the guess before
                          it is judged (removes its rough, high-residual part);
                          0 = none                                              */
  double warm_omega;   /* damping of those sweeps; 0 = 2/3                      */
  int restarts;        /* FP64 solves: when the recursive test holds but the
                          true residual ||b - A x|| exceeds rtol ||b|| (the
                          recurrences drift from it by rounding, most at large
                          s), start the method again from the current x, at
                          most this many times, within the budget of maxit
                          CG-equivalent steps; 0 = never.  Iteration counts add
                          up and the residual histories are concatenated (each
                          run starts with its true residual); see
                          ssp_get_restarts.  MIXED_IR ignores it: its
                          refinement loop already ends on the true residual   */
  int basis;           /* SSP_BASIS_* (s-step method, FP64 and MIXED_IR)         */
  double basis_lo;     /* Chebyshev basis interval; basis_hi <= basis_lo selects
                          the default [0, 2] with the Jacobi preconditioner and
                          [0, 2 max_i a_ii] without one (Gershgorin, for a
                          weakly diagonally dominant SPD matrix)               */
  double basis_hi;
} ssp_opts;

/* ---- handle ---------------------------------------------------------------- */

/* Creates a handle bound to HIP device `device` and to the caller's stream
 * `hip_stream` (a hipStream_t; NULL = the legacy default stream).  Allocates
 * only small control blocks; solve workspaces are allocated on first use and
 * cached.  *h is set to NULL on failure. */
int ssp_create(ssp_handle **h, int device, void *hip_stream);

/* Frees every library-owned allocation of the handle.  Matrices created with
 * it must be destroyed first.  NULL is accepted. */
int ssp_destroy(ssp_handle *h);

/* ---- matrices -------------------------------------------------------------- */

/* Sparse SPD matrix in CSR form (Sec. III: local CSR storage).  rowptr
 * (n+1 int32), colind (nnz int32, ascending in each row) and val (nnz FP64)
 * are DEVICE pointers.  flags: SSP_BORROW or SSP_COPY, optionally or-ed with
 * SSP_VALIDATE.  Builds D^-1 = 1/diag(A) for the Jacobi preconditioner.
 * The default preconditioner is SSP_PREC_JACOBI.  Errors: SSP_EINVAL for
 * n < 1, nnz < n, nnz >= 2^31, NULL pointers or a failed validation. */
int ssp_matrix_csr(ssp_handle *h, int64_t n, int64_t nnz, const int32_t *rowptr,
                   const int32_t *colind, const double *val, unsigned flags,
                   ssp_matrix **A);

/* Matrix-free grid operator (Dirichlet zero outside the grid, unscaled).
 * For the constant-coefficient kinds `coef` is a HOST pointer to {diag, off}
 * or NULL for the defaults above.  For SSP_STENCIL_3D7_VARK `coef` is a DEVICE
 * pointer to the n cell coefficients k (borrowed: it must outlive the matrix).
 * Default preconditioner SSP_PREC_JACOBI. */
int ssp_matrix_stencil(ssp_handle *h, int kind, int nx, int ny, int nz,
                       const double *coef, ssp_matrix **A);

/* The same grid operator materialised on the device in CSR form (library-
 * owned arrays, ascending columns), so that the CSR kernels can run on it
 * without a host build or upload.  Arguments as for ssp_matrix_stencil. */
int ssp_matrix_csr_from_stencil(ssp_handle *h, int kind, int nx, int ny, int nz,
                                const double *coef, ssp_matrix **A);

/* Size of a matrix (nnz = stored entries of its CSR form). */
int ssp_matrix_info(const ssp_matrix *A, int64_t *n, int64_t *nnz);

/* Device pointers of a CSR matrix (borrowed, copied or library-built);
 * SSP_EINVAL for a matrix-free operator. */
int ssp_matrix_csr_arrays(const ssp_matrix *A, const int32_t **rowptr,
                          const int32_t **colind, const double **val);

/* The CSR kernel form chosen for A at creation by timing (0 = LDS-staged row
 * blocks, 1 = one row per thread, 2 = sliced ELL copy, slices of 64 rows);
 * -1 for matrix-free operators. */
int ssp_matrix_csr_form(const ssp_matrix *A, int *form);

int ssp_matrix_destroy(ssp_matrix *A);

/* SSP_PREC_NONE, SSP_PREC_JACOBI, or SSP_PREC_AMG once ssp_set_amg has built
 * the matrix's hierarchy (SSP_EINVAL otherwise). */
int ssp_set_preconditioner(ssp_matrix *A, int kind);

/* ---- AMG preconditioner -------------------------------------------------- */

/* The paper's weak-scaling preconditioner (Sec. III-A, Sec. V-B) is an
 * algebraic multigrid whose B^-1 is weighted-Jacobi sweeps on each level of a
 * hierarchy of coarser matrices built from A.  This one is smoothed
 * aggregation: strength a_ij^2 >= theta^2 |a_ii a_jj|; three-pass greedy
 * aggregation in row order; P = (I - 4/(3 rho_G) D^-1 A) P_t with rho_G the
 * Gershgorin bound of rho(D^-1 A); A_c = P^T A P, R = P^T; the coarsest level
 * is solved with its dense inverse.  B^-1 y is one V-cycle: `sweeps` Jacobi
 * sweeps with weight omega before (the first from zero) and after the coarse
 * correction, so B^-1 is symmetric.  The strength threshold halves from one
 * level to the next (theta 2^-l on level l).  All fields 0 = default. */
#define SSP_AMG_MAX_LEVELS 16
#define SSP_AMG_DENSE_MAX 4096   /* rows of the coarsest level at most */
typedef struct ssp_amg_opts {
  double theta;     /* strength threshold of level 0 (default 0.08)             */
  double omega;     /* Jacobi weight of the smoother (default 2/3)              */
  int sweeps;       /* sweeps before and after the coarse correction (1)        */
  int max_coarse;   /* coarsening stops at this many rows (64)                  */
  int max_levels;   /* at most this many levels (10)                            */
} ssp_amg_opts;

/* Builds A's hierarchy (on the host, once; the level matrices, prolongators,
 * restrictions and the coarse inverse then live on the device with the
 * matrix) and makes SSP_PREC_AMG A's preconditioner.  CSR matrices with a
 * positive diagonal only (SSP_EUNSUPPORTED for grid operators: build their
 * CSR form with ssp_matrix_csr_from_stencil).  SSP_EUNSUPPORTED also when the
 * coarsest level would exceed SSP_AMG_DENSE_MAX rows.  The s-step method
 * (FP64, monomial basis) and ssp_mpk use it; other methods and precisions
 * return SSP_EUNSUPPORTED with it.  A later call rebuilds the hierarchy. */
int ssp_set_amg(ssp_handle *h, ssp_matrix *A, const ssp_amg_opts *opts);

/* Number of levels of A's hierarchy (0: none) and, if rows is not NULL, the
 * rows of each level (HOST array of at least SSP_AMG_MAX_LEVELS entries). */
int ssp_amg_levels(const ssp_matrix *A, int *levels, int64_t *rows);

/* z = B^-1 y: one V-cycle (DEVICE vectors of length n, distinct), enqueued on
 * the handle's stream. */
int ssp_amg_apply(ssp_handle *h, const ssp_matrix *A, const double *y, double *z);

/* ---- building blocks ------------------------------------------------------- */

/* y = A x (DEVICE vectors of n entries).  Enqueues only. */
int ssp_spmv(ssp_handle *h, const ssp_matrix *A, const double *x, double *y);

/* Alg. 4 and Alg. 5 on their own: fills the DEVICE block P (column-major,
 * leading dimension ld >= n, 2s columns) with P(:,1:s) = [z, Kz, ..., K^{s-1}z],
 * z = B^-1 r, K = B^-1 A, and P(:,s+1:2s) = A P(:,1:s); and, if vm is a
 * non-NULL HOST pointer, returns vm(1:s) = P(:,1:s)^T r and
 * vm(s+1:2s) = P(:,1:s)^T P(:,2s) (synchronises). */
int ssp_mpk(ssp_handle *h, const ssp_matrix *A, const double *r, int s, double *P,
            int64_t ld, double *vm);

/* The Chebyshev basis of one outer iteration (SSP_BASIS_CHEBYSHEV; the
 * stabilised bases of the related work, Sec. IV) on its own: fills the DEVICE
 * block P (column-major, leading dimension ld >= n, even; P and r 16-byte
 * aligned; 2s columns) with Z = [z_1 .. z_s], z_1 = B^-1 r, z_2 = (K z_1 - c z_1)/h,
 * z_{j+1} = 2 (K z_j - c z_j)/h - z_{j-1} (K = B^-1 A, c = (hi + lo)/2,
 * h = (hi - lo)/2; hi <= lo selects the default interval of ssp_opts), and
 * P(:,s+1:2s) = A Z; and, if gram is a non-NULL HOST pointer, the block Gram
 * product of the matrix cores, gram = Z^T [AZ | r] (s x (s+1), row-major)
 * (synchronises). */
int ssp_cheb_basis(ssp_handle *h, const ssp_matrix *A, const double *r, int s, double lo,
                   double hi, double *P, int64_t ld, double *gram);

/* ssp_mpk without any device allocation, for callers that cannot allocate
 * (code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc).  Same arguments, kernels and results (bit for bit) as ssp_mpk.
 * Its control block and per-workgroup partial sums live in one static
 * device array per GPU of 7 KB + 512 KiB (room for 2048 workgroups x 2s
 * partial sums at s <= SSP_SMAX; a call needing more is rejected with
 * SSP_EINVAL), set up once per device by ssp_create and held until the
 * process ends.  Every call on a GPU shares that array: calls that overlap
 * on one GPU (other streams, other handles, other host threads) race and
 * must be serialised by the caller.  The caller still owns r, P and vm;
 * the matrix must have been created beforehand (creation allocates). */
int ssp_mpk_noalloc(ssp_handle *h, const ssp_matrix *A, const double *r, int s, double *P,
                    int64_t ld, double *vm);

/* ---- solve ------------------------------------------------------------------ */

/* Solves A x = b.  b (n) and x (n, in: x0, out: solution) are DEVICE pointers
 * owned by the caller.  s in 1..SSP_SMAX (and s <= n) is the block size of
 * the s-step method (ignored by SSP_METHOD_PCG and SSP_METHOD_PFCG).  Stops
 * when the recursive residual satisfies ||r||_2 <= rtol ||b||_2, tested once
 * per outer iteration; maxit counts CG-equivalent steps (outer limit
 * ceil(maxit/s); for PFCG every step counts, the one before the loop of
 * Alg. 2 included).  Mixed precision is implemented for the s-step method
 * only (SSP_EUNSUPPORTED otherwise).
 * opts may be NULL (defaults: s-step, FP64).  b = 0 gives x = 0 and SSP_OK.
 * Returns SSP_OK, SSP_NOT_CONVERGED, SSP_BREAKDOWN or an error.  Blocks until
 * the result is in x. */
int ssp_solve(ssp_handle *h, const ssp_matrix *A, const double *b, double *x, int s,
              double rtol, int maxit, const ssp_opts *opts);

/* Outer iterations and CG-equivalent steps (s * outer) of the last solve
 * (summed over its restarts). */
int ssp_get_iterations(const ssp_handle *h, int *outer, int *cg_equiv);

/* Restarts the last solve made (opts.restarts; 0 if none). */
int ssp_get_restarts(const ssp_handle *h, int *restarts);

/* Outcome of the last solve's warm-start judge (opts.warm_start = 1):
 * *kept = 1 if the given x was used, 0 if it fell back to x = 0, -1 if the
 * last solve had no warm start; *rel0 = ||b - A x0|| / ||b|| of the guess as
 * judged (after the smoothing sweeps). */
int ssp_get_warm_start(const ssp_handle *h, int *kept, double *rel0);

/* ||r_i||_2/||b||_2 of the last solve, i = 0 (initial) .. outer; copies at most
 * cap entries into the HOST buffer and sets *len to the full length. */
int ssp_get_residual_history(const ssp_handle *h, double *buf, int cap, int *len);

/* ||b - A x||_2/||b||_2 computed from the returned x at the end of the last
 * solve (for MIXED_IR: of the final FP64 iterate). */
int ssp_get_true_residual(const ssp_handle *h, double *rel);

/* Kernel-class timings of the last solve run with opts.profile = 1, measured
 * with HIP events on the handle's stream: for each class the number of
 * launches and the summed duration in milliseconds (HOST arrays of
 * SSP_PROFILE_CLASSES).  Classes: 0 = matrix powers j < s (Alg. 4; SpMV of
 * standard CG), 1 = last power fused with the moments (Alg. 5) and the s x s
 * solve (Alg. 6; on the Chebyshev basis the last power and the s x s
 * algebra), 2 = block update (Alg. 3; vector updates of standard CG),
 * 3 = other (initial and true residual), 4 = the block Gram pass of the
 * Chebyshev basis. */
#define SSP_PROFILE_CLASSES 5
int ssp_get_profile(const ssp_handle *h, int *launches, double *ms);

/* ---- batched solves ---------------------------------------------------------- */

/* Tuning of the batched persistent solver (all fields 0 = default). */
typedef struct ssp_tune {
  int tile_rows;       /* rows per work item; 0 = the row partition of a single
                          solve, so that every system's result equals its
                          ssp_solve (MIXED_IR) result bit for bit           */
  int grid;            /* persistent workgroups (default 512)                 */
  int order;           /* 0 = idle workgroups look at the largest systems
                          first; 1 = round-robin start per workgroup          */
  int spin_limit;      /* consecutive empty polls without global progress
                          after which the launch gives up (default 2^20)      */
  int schedule;        /* 0 = one persistent launch (workgroups claim tiles);
                          1 = stepped: one launch pair per phase step of all
                          systems together (no in-kernel synchronisation;
                          grid, order and spin_limit unused).  Both give the
                          same results bit for bit                             */
  int run;             /* persistent schedule: tiles a workgroup claims at once
                          (one acquire and one release fence per run instead
                          of per tile); 0 = 1                                  */
} ssp_tune;

/* Solves nsys independent systems A[i] x[i] = b[i] in ONE persistent launch
 * (the batch extension of the method): each system runs the mixed-precision
 * form of the s-step method (FP32 matrix powers and block updates, FP64
 * moments, s x s solves, residuals and refinement; opts->inner_rtol and
 * opts->max_refine as for ssp_solve, opts->precision is ignored), with its
 * own phase state machine; workgroups take tiles of rows from any system
 * with work ready.  A, b, x are HOST arrays of nsys matrix handles / DEVICE
 * vector pointers (x in: x0, out: solution).  1 <= s <= 8, s <= every n.
 * Per-system outcome codes, inner outer-iteration counts and true relative
 * residuals go to the optional HOST arrays status_out, outer_out,
 * true_rel_out.  Returns the worst per-system outcome (SSP_OK,
 * SSP_NOT_CONVERGED, SSP_BREAKDOWN) or a negative error (SSP_EHIP if the
 * scheduler stalled). */
int ssp_solve_batch(ssp_handle *h, int nsys, const ssp_matrix *const *A,
                    const double *const *b, double *const *x, int s, double rtol,
                    int maxit, const ssp_opts *opts, const ssp_tune *tune,
                    int *status_out, int *outer_out, double *true_rel_out);

/* Chooses the schedule, tile size, grid size and scan order for a batch by
 * timing short runs of ssp_solve_batch on scratch iterates; with a non-NULL cache_path the
 * choice is read from / appended to that text file, keyed by architecture,
 * batch size, total rows (log2), s and operator kinds. */
int ssp_autotune_batch(ssp_handle *h, int nsys, const ssp_matrix *const *A,
                       const double *const *b, int s, const char *cache_path,
                       ssp_tune *out);

/* ---- learned warm start --------------------------------------------------- */

/* A 3-level U-shaped 3D conv net (about 246k parameters) that maps the pair
 * (log k, f) of a variable-coefficient Poisson problem on a D x H x W grid
 * to an initial guess x0 (the learned-warm-start extension).  Convolutions
 * run on the BF16 matrix cores with FP32 accumulation; master weights, Adam
 * moments and gradients are FP32.  The levels are 4x apart (two stride-2
 * convolutions down, nearest upsampling by 4 up), so the coarsest level's
 * receptive field covers the grid.  Layers: 3x3x3 convolutions 8->16,
 * 16->16 | 16->16 /2, 16->32 /2 | 32->32 | 32->32 /2, 32->48 /2 | 48->32 |
 * 64->32 (after upsampling and concatenation with the 32-channel level),
 * 48->16 (likewise with the 16-channel level), then a 1x1 head 16->1; ReLU
 * after every 3x3x3 convolution; zero padding of one cell.  Weights are
 * He-normal from `seed`, biases zero. */
typedef struct ssp_net ssp_net;

int ssp_net_create(ssp_handle *h, int D, int H, int W, int max_batch, uint64_t seed,
                   ssp_net **net);
int ssp_net_destroy(ssp_net *net);

/* DEVICE pointers to the flat FP32 parameters and gradients (layout: per
 * layer W[27][Ci][Co] then b[Co], then the head's w[16] and b[1]) and their
 * count. */
int ssp_net_params(ssp_net *net, float **params, float **grads, int64_t *count);

/* Forward pass.  in: DEVICE FP32 [batch][D][H][W][2] (log k and f, already
 * normalised), out: DEVICE FP32 [batch][D][H][W].  Keeps the activations for
 * ssp_net_backward. */
int ssp_net_forward(ssp_net *net, const float *in, int batch, float *out);

/* Inference for one problem, every step on the device: the input channels
 * log k and f / rms(f), with rms(f) = sqrt(sum f^2 / n) in FP64 (1 when f is
 * zero), the forward pass (the decoder reads its upsampled and concatenated
 * inputs straight from the two levels instead of building them), and the
 * FP64 output x0 = y rms(f) out_scale.  logk, f: DEVICE FP64 [D][H][W];
 * x0: DEVICE FP64 [D][H][W], not aliasing them.  The result equals
 * ssp_net_forward on the FP32 pair (log k, f / rms(f)) followed by that
 * scaling.  Asynchronous on the handle's stream; SSP_EINVAL for a null
 * pointer or a non-finite out_scale.  The activations it leaves are not a
 * training forward's: ssp_net_backward afterwards returns SSP_EINVAL. */
int ssp_net_predict(ssp_net *net, const double *logk, const double *f, double out_scale,
                    double *x0);

/* Squared-error loss of the last forward's output y against target (DEVICE
 * FP32, batch*D*H*W): writes dy = 2 (y - t) / N (DEVICE) and, if loss is a
 * HOST pointer, the mean squared error (synchronises). */
int ssp_net_loss(ssp_net *net, const float *y, const float *target, float *dy, double *loss);

/* Energy-type loss of the last forward's output y against target (DEVICE,
 * FP32, [batch][D][H][W]): with e = y - target and L the 7-point Laplacian
 * of each sample's grid (zero outside it), loss = e^T (L + lambda I) e / N
 * and dy = 2 (L e + lambda e) / N, N = batch * D * H * W.  It weighs the
 * error as CG started from y does (energy norm of a constant-coefficient
 * operator), rather than by its mean square.  lambda >= 0. */
int ssp_net_loss_h1(ssp_net *net, const float *y, const float *target, float lambda, float *dy,
                    double *loss);

/* Accumulates the parameter gradients of the last forward for the output
 * gradient dy (DEVICE FP32); ssp_net_zero_grad clears them. */
int ssp_net_backward(ssp_net *net, const float *dy);
int ssp_net_zero_grad(ssp_net *net);

/* One Adam step with bias correction (step counts from 1). */
int ssp_net_adam_step(ssp_net *net, float lr, float beta1, float beta2, float eps, int step);

/* Checkpoint: parameters, then Adam first and second moments (3 * count
 * floats, HOST buffer).  set_state accepts count (parameters only) or
 * 3 * count floats. */
int ssp_net_get_state(ssp_net *net, float *host, int64_t cap);
int ssp_net_set_state(ssp_net *net, const float *host, int64_t len);

/* One 3x3x3 convolution (zero padding 1, stride 1 or 2) on its own, with the
 * network's kernels; inputs are rounded to BF16, results are FP32.  mode 0:
 * out = conv(in, w) for in [B][D][H][W][ci] (ci % 8 == 0, co % 16 == 0);
 * mode 1: out = the input gradient for the output gradient `in`
 * ([B][Do][Ho][Wo][co]; ci % 16 == 0, co % 8 == 0).  w: FP32 [27][ci][co]
 * with tap (dz+1)*9 + (dy+1)*3 + (dx+1).  DEVICE pointers; synchronises. */
int ssp_conv3d(ssp_handle *h, int mode, const float *in, int B, int D, int H, int W, int ci,
               const float *w, int co, int stride, float *out);

/* Weight and bias gradients of that convolution for input x and output
 * gradient dz (DEVICE, FP32, rounded to BF16): dw [27][ci][co], db [co].
 * Grids of 2^31 points or more (batch included) return SSP_EINVAL. */
int ssp_conv3d_wgrad(ssp_handle *h, const float *x, int B, int D, int H, int W, int ci,
                     const float *dz, int co, int stride, float *dw, float *db);

/* One 16x16x32 BF16 matrix-core product D = A B with the operand layout the
 * convolutions use (DEVICE FP32 row-major A 16x32, B 32x16, D 16x16). */
int ssp_net_mfma_selftest(ssp_handle *h, const float *A, const float *B, float *D);

/* Roofline reference: the mean duration (*ms, milliseconds, HIP events on
 * the handle's stream, after one warm-up launch) of `reps` launches of a
 * plain streaming read of the n doubles at src (mode 0) or a copy src -> dst
 * (mode 1), 16-byte accesses over the library's largest launch grid.  DEVICE
 * pointers, 16-byte aligned; n even.  Synchronises. */
int ssp_stream_probe(ssp_handle *h, int mode, const double *src, double *dst, int64_t n,
                     int reps, double *ms);

/* Text for a status code (static storage). */
const char *ssp_status_string(int status);

/* Last error message of the handle (static per handle, never NULL). */
const char *ssp_last_error(const ssp_handle *h);

#ifdef __cplusplus
}
#endif

#endif /* SSTEP_H */
