/*
 * libhelm — compact 4th/6th-order 3D Helmholtz solver with the EigT / PFFT preconditioner on one MI355X GPU.
 *
 * Method: arXiv 2602.07711 (Gryazin, Gonzales, Li), "High-Resolution Solvers for 3D Helmholtz Scattering
 * Problems Using PFFT and Eigenvector-Based Preconditioning".
 *
 *   PDE        nabla^2 u + k^2(x) u = f on a box, absorbing condition du/dn - i k0 u = 0 (Sec. 1, Sec. 2.1).
 *   Grid       N_nu unknowns per axis at spacing h_nu; the absorbing condition sits half a cell outside the
 *              first and last node and eliminates the ghosts as U_0 = gamma U_1, U_{N+1} = gamma U_N with
 *              gamma = (2 + i k0 h)/(2 - i k0 h) (Sec. 2.3, eq. D_bc). Dirichlet uses gamma = 0.
 *   Operator   A = compact 4th-order scheme (Sec. 2.2, eq. scheme4; 19 points, any h) or 6th-order scheme
 *              (Sec. 2.3, eq. scheme6; 27 points, uniform h), or the plain 7-point 2nd-order operator.
 *   Precond.   M = Delta_2 + k0^2 I, the 7-point operator with the same absorbing closure and the background
 *              k0 (Sec. 4: A_p / h_z^2). Applied by EigT (Sec. 4.1, eq. EIG_SOLVER) or PFFT (Sec. 4.2, eq.
 *              PFFT_SOLVER), in complex FP64 or complex FP32.
 *   Krylov     restarted right-preconditioned GMRES(m) (Sec. 3.1 eq. Preconditioned_System, Sec. 5) or
 *              flexible GMRES(m) (needed when the preconditioner runs in FP32 or changes between calls).
 *
 * Data layout.  Every vector is an array of complex128 (interleaved re, im; 16 bytes) in device memory with
 * index i + Nx*(j + Ny*l): x fastest, then y, then z (the slice ordering of Sec. 4.1). Fields sampled with a
 * two-cell halo have (Nx+4)*(Ny+4)*(Nz+4) entries in the same order, node (i,j,l) at (i+2, j+2, l+2).
 *
 * Ownership.  All pointers passed in are caller-owned device memory. The library reads them during the
 * call (k^2 during helm_setup only) and keeps no reference afterwards. The context owns every buffer it
 * allocates (eigen-data, derived fields, Krylov workspace) and helm_destroy frees them.
 *
 * Streams.  Every call enqueues its kernels on the stream given to helm_setup (NULL = the default stream)
 * of the device that was current at helm_setup. helm_rhs, helm_matvec and helm_precond_apply return
 * without waiting; helm_gmres_solve returns after the solve with `info` filled in. One context must not be
 * used by two host threads at once.
 *
 * Errors.  Functions return a helm_status and never throw. The message of the last failure on a context is
 * available from helm_last_error(ctx); helm_setup failures before a context exists are reported through
 * helm_last_setup_error().
 */
#ifndef HELM_H
#define HELM_H

#ifdef __cplusplus
extern "C" {
#endif

typedef struct helm_ctx helm_ctx;

typedef enum {
    HELM_OK = 0,
    HELM_EINVAL = 1,       /* invalid argument: shape, order, h, halo, NULL pointer, NaN/Inf in k^2        */
    HELM_ENOMEM = 2,       /* device allocation failed                                                     */
    HELM_EDEVICE = 3,      /* a HIP runtime call failed                                                    */
    HELM_ENOCONV = 4,      /* GMRES hit maxit; x holds the last iterate                                    */
    HELM_EBREAKDOWN = 5,   /* Arnoldi breakdown with a residual above tolerance                            */
    HELM_ENUMERIC = 6,     /* NaN/Inf appeared in a reduction, or the 1D eigen-decomposition failed checks */
    HELM_EUNSUPPORTED = 7  /* a valid request that the library does not implement                          */
} helm_status;

typedef struct { int nx, ny, nz; } helm_grid;   /* unknowns per axis, each >= 3 */

typedef enum {
    HELM_BC_ABC2 = 0,      /* two-point absorbing closure, gamma = (2 + i k0 h)/(2 - i k0 h), zeta = 1 (Sec. 2.3) */
    HELM_BC_DIRICHLET = 1, /* gamma = 0: zero ghost values                                                     */
    HELM_BC_ABC3 = 2       /* the three-point closure of collocated grids (Sec. 4.1, zeta = 2): the boundary
                              nodes are unknowns and the central difference of u_n + i k0 u = 0 eliminates the
                              ghost, so Lambda-bar has gamma = 2 i k0 h and zeta = 2 in its corners. Direct
                              solves of the second-order system only (helm_precond_apply with HELM_PREC_EIGT or
                              HELM_PREC_PFFT, the EigT3 and PFFT3 of Table 2); the paper does not give the
                              high-order closures of its collocated runs, so helm_rhs, helm_matvec,
                              helm_gmres_solve, helm_scale_guess and batches return HELM_EUNSUPPORTED for such
                              contexts                                                                        */
} helm_bc_kind;

typedef struct {
    int kind;              /* helm_bc_kind                                                                  */
    double k0;             /* background wavenumber on the boundary (Sec. 2.1 eq. background); also the
                              constant k0 of the preconditioner M                                           */
} helm_bc;

typedef enum {
    HELM_PREC_EIGT = 0,    /* eigenvector transforms in x and y + z-tridiagonal solves (Sec. 4.1)            */
    HELM_PREC_PFFT = 1,    /* sine transforms + boundary correction on the x/y faces (Sec. 4.2; two layers per
                              face with the collocated closure)                                               */
    HELM_PREC_NONE = 2,    /* identity (unpreconditioned GMRES)                                              */
    HELM_PREC_FFT2 = 3,    /* the comparison preconditioner FFT2 of Sec. 5.1 (the earlier FFT-type approach
                              recalled at the start of Sec. 4): the same 7-point operator with constant k0 but
                              zero Dirichlet closures on all six faces (gamma = 0 on every axis), inverted by
                              sine transforms in x and y and z-tridiagonal solves                            */
    HELM_PREC_FFT4 = 4,    /* FFT4 of Sec. 5.1: the fourth-order compact operator (Sec. 2.2 eq. scheme4) with
                              the constant k0 and zero Dirichlet closures, inverted by the 3D sine transform
                              (sine-matrix GEMMs along x, y and z) and division by the scheme's symbol         */
    HELM_PREC_FFT6 = 5     /* FFT6 of Sec. 5.1: the same with the sixth-order scheme (Sec. 2.3 eq. scheme6;
                              needs h_x = h_y = h_z, HELM_EINVAL otherwise)                                   */
} helm_prec_kind;

typedef struct {
    int m;                 /* restart length, 1..256                                                         */
    int maxit;             /* total iteration cap (> 0)                                                      */
    double rtol;           /* stop when ||F - A x||_2 <= rtol * ||F||_2 (Sec. 5.1 rel-res with U^0 = 0)      */
    int flexible;          /* 0: right-preconditioned GMRES, x = x0 + M^{-1} V y; 1: FGMRES, x = x0 + Z y    */
    int prec_fp32;         /* 1: run the preconditioner in complex FP32 (requires flexible = 1)              */
    int prec;              /* helm_prec_kind                                                                 */
    int x0_given;          /* 1: x holds the initial guess on entry; 0: start from x = 0; 2 (flexible only):
                              x holds a guess p that the first cycle takes as its first search direction
                              z_0 = p, starting from x = 0 (then z_1 = M^{-1} v_0 and z_j = M^{-1} v_j for
                              j >= 2), so the minimal residual over x in span{p, M^{-1} v_0, M^{-1} v_2, ...}
                              decides how much of p is used                                                   */
    double *resid_hist;    /* optional host array receiving relative residual estimates, one per iteration
                              plus one per restart (true residual); may be NULL                              */
    int hist_len;          /* capacity of resid_hist                                                         */
} helm_solve_opts;

typedef struct {
    int iters;             /* Arnoldi steps taken (= preconditioner applications inside cycles)             */
    int restarts;          /* completed cycles                                                               */
    int converged;         /* 1 if the true residual met rtol                                                */
    int hist_used;         /* entries written to resid_hist                                                  */
    int reorths;           /* Arnoldi steps that took a second Gram-Schmidt pass: those whose orthogonalised
                              vector keeps at most 1e-2 of the squared norm (||y - V h||^2 <= 1e-2 ||y||^2); the
                              environment variable HELM_CGS_REORTH (a number in (0, 1)) replaces 1e-2          */
    double relres_est;     /* last Givens residual estimate / ||F||                                          */
    double relres_true;    /* ||F - A x|| / ||F|| at exit                                                    */
    double t_ms[6];        /* device time per phase: matvec, preconditioner, Arnoldi (dots + update),
                              end-of-cycle update, host work (Givens, sync), total wall                      */
} helm_solve_info;

/* Create a context: validates the grid, computes gamma per axis, runs the 1D eigen-decompositions of
 * Lambda-bar_x and Lambda-bar_y on the host (Sec. 4.1 EigT Step 1), uploads V, V^{-1}, D, and derives the
 * per-node fields of the operator from k^2 (Sec. 2.3: grad k^2 and lap k^2 by 4th-order central differences).
 *   g        unknowns per axis (each >= 3).
 *   h        grid steps h_x, h_y, h_z (> 0). order 6 requires h_x = h_y = h_z (Sec. 2.3).
 *   k2_dev   real k^2 samples (float64) in device memory, with a two-cell halo (k2_halo = 2) or on the
 *            interior only (k2_halo = 0; allowed for order 2 and 4, which need no derivatives of k^2).
 *   order    2, 4 or 6.
 *   bc       closure kind and background k0 (k0 >= 0 and finite).
 *   stream   hipStream_t to enqueue on, or NULL.
 * On success *ctx owns its device buffers. Returns HELM_EINVAL for bad arguments or non-finite k^2,
 * HELM_ENOMEM / HELM_EDEVICE on runtime failures, HELM_ENUMERIC if the eigen-decomposition fails its
 * residual checks. */
helm_status helm_setup(helm_ctx **ctx, helm_grid g, const double h[3], const double *k2_dev, int k2_halo,
                       int order, helm_bc bc, void *stream);

/* The same with a complex k^2 (attenuating media, e.g. the inclusion k^2 = 1050 + 2.26i of the scattering
 * experiment of Sec. 5.1): k2_dev holds complex128 samples in the layout above. The scheme is unchanged
 * (Sec. 2.2 eq. scheme4, Sec. 2.3 eq. scheme6 with complex k^2 and complex derived fields); the preconditioner
 * keeps the real constant k0 of `bc`. Batched solves do not accept such contexts (HELM_EUNSUPPORTED). */
helm_status helm_setup_complex(helm_ctx **ctx, helm_grid g, const double h[3], const void *k2_dev, int k2_halo,
                               int order, helm_bc bc, void *stream);

/* F = R_h f, the modified right-hand side of the scheme (Sec. 2.2 f^(IV), Sec. 2.3 f^(VI) together with the
 * k^2 f and f_nu terms of Delta_h(k^2 U)). f_dev: complex128 samples of f with a two-cell halo.
 * F_dev: n complex128. f is data: its halo samples are used as they are. */
helm_status helm_rhs(helm_ctx *ctx, const void *f_dev, void *F_dev);

/* y = A x: the compact operator of Sec. 2.2 (eq. scheme4, order 4) or Sec. 2.3 (eq. scheme6, order 6; order 2 is the
 * 7-point operator) with the variable k^2 of the context and the ghost values eliminated by the absorbing closure
 * (Sec. 2.3, eq. D_bc). x_dev, y_dev: n complex128, must not overlap. */
helm_status helm_matvec(helm_ctx *ctx, const void *x_dev, void *y_dev);

/* z = M^{-1} y with M = Delta_2 + k0^2 I (Sec. 4). kind: HELM_PREC_EIGT or HELM_PREC_PFFT (M with the
 * operator's absorbing closure), HELM_PREC_FFT2 (M with zero Dirichlet closures), HELM_PREC_FFT4 / FFT6 (the
 * compact operators with constant k0 and zero Dirichlet closures), HELM_PREC_NONE (z = y);
 * fp32: 1 runs the transforms and tridiagonal solves in complex FP32 (input read as FP64, output written as
 * FP64). y_dev, z_dev: n complex128; they may be the same buffer. PFFT requires N_x, N_y <= 832
 * (HELM_EUNSUPPORTED otherwise). */
helm_status helm_precond_apply(helm_ctx *ctx, const void *y_dev, void *z_dev, int kind, int fp32);

/* For callers that cannot allocate device memory (code under stream capture, tight serving loops, harnesses that
 * forbid allocation): the FP32 EigT preconditioner of helm_precond_apply(ctx, y_dev, z_dev, HELM_PREC_EIGT, 1)
 * (same kernels, same results) without any allocation inside the call. Its two complex64 staging vectors live in one
 * static device array of the library (32 MiB, held by every device the library runs on until the process ends), so
 * n = Nx*Ny*Nz must not exceed 2^21 (HELM_EINVAL otherwise). Every call on a device shares that device's array:
 * calls that overlap on one device (two streams or two host threads) race. y_dev, z_dev: n complex128 each,
 * caller-owned; they may be the same buffer. Its launches are not counted by the per-kernel timing. HELM_EDEVICE if
 * the array's device address cannot be resolved. */
helm_status helm_precond_apply_noalloc(helm_ctx *ctx, const void *y_dev, void *z_dev);

/* Solve A x = F by restarted (F)GMRES preconditioned on the right by M (Sec. 3.1, Sec. 4, Sec. 5).
 * F_dev: n complex128. x_dev: n complex128, initial guess on entry when opts->x0_given, solution on exit.
 * The Krylov workspace ((m+1) + (flexible ? m : 0) vectors of n complex128) is allocated on the first solve
 * with a given (m, flexible) and kept by the context. Returns HELM_OK when converged, HELM_ENOCONV at maxit
 * (x holds the last iterate), HELM_EBREAKDOWN, HELM_ENUMERIC on NaN/Inf, HELM_EINVAL for bad options. */
helm_status helm_gmres_solve(helm_ctx *ctx, const void *F_dev, void *x_dev, const helm_solve_opts *opts,
                             helm_solve_info *info);

/* Kernel classes for per-kernel timing. */
typedef enum {
    HELM_K_MATVEC = 0,     /* compact-stencil y = A x (also r = F - A x)                                     */
    HELM_K_GEMM_X64 = 1,   /* EigT x-transform, complex FP64 MFMA (forward and inverse)                      */
    HELM_K_GEMM_Y64 = 2,   /* EigT y-transform, complex FP64 MFMA, batched over slices                       */
    HELM_K_GEMM_X32 = 3,   /* EigT x-transform, complex FP32 MFMA                                            */
    HELM_K_GEMM_Y32 = 4,   /* EigT y-transform, complex FP32 MFMA                                            */
    HELM_K_TRIDIAG64 = 5,  /* z-tridiagonal solves, FP64                                                     */
    HELM_K_TRIDIAG32 = 6,  /* z-tridiagonal solves, FP32                                                     */
    HELM_K_DOTS = 7,       /* Krylov block inner products + norm (both reduction stages)                     */
    HELM_K_LINCOMB = 8,    /* Krylov linear combinations (orthogonalisation update, x += Z y, restart)       */
    HELM_K_PFFT = 9,       /* PFFT sine transforms (MFMA GEMMs against the real sine matrix)                 */
    HELM_K_RING = 10,      /* PFFT face-only transforms (restricted inverse, sparse forward)                  */
    HELM_K_COUNT = 11
} helm_kernel_class;

/* Per-kernel device timing. With on = 1 every launch of the classes above is bracketed by HIP events on the
 * context stream and its duration is accumulated by class (counters reset); on = 0 stops recording.
 * Launches that follow each other on the stream share an event (the end of one is the start of the next), so
 * a launch's time includes the few microseconds of launch gap before it. Idle time after a host
 * synchronisation, untimed library work and work the caller enqueues between library calls are not counted.
 * Pending events are resolved at the end of a solve and in helm_profile_read. */
helm_status helm_profile_enable(helm_ctx *ctx, int on);

/* Accumulated device milliseconds, launch count and algorithmic work of one kernel class since the last
 * enable. Work is the method's minimum per launch, summed: HBM bytes for the memory-bound classes (matvec:
 * x, k^2 and the order-6 field block read once, y written once; tridiagonal: transformed data read and
 * written once; Krylov kernels: every vector read or written once) and real flops for the GEMMs
 * (8 M N K per complex product). Any output pointer may be NULL. Waits for the context stream. */
helm_status helm_profile_read(helm_ctx *ctx, int kernel_class, double *ms_total, long long *launches,
                              double *work);

/* Short name of a kernel class ("matvec", "gemm_x64", ...), or "" for an unknown class. */
const char *helm_profile_name(int kernel_class);

/* GEMM tile autotuner for the EigT transforms of a context. For each of the four transform GEMMs (x and y,
 * FP64 and FP32) it times every tile configuration (BM, BN, BK) = (64,64,16), (64,64,32), (128,64,16),
 * (64,128,16) with the launches the preconditioner makes (the FP32 x-transform as its FP64-input forward and
 * FP64-output inverse pair), best of three trials of `reps` launches on the context stream, and keeps the
 * fastest for this context, separately for the forward and the inverse transform of each kind. If the environment
 * variable HELM_TUNE_CACHE names a file, choices are read from it by (transform, direction, axis length, lines,
 * slices) and new ones appended to it. chosen: NULL or 8 ints, the forward choices of (x64, y64, x32, y32) then the
 * inverse ones; ms: NULL or 32 doubles, the per-launch time of configuration c of transform t in direction d
 * (0 forward, 1 inverse) at ms[16 d + 4 t + c] (not written for cached choices).
 * Batches created afterwards use the tuned choices of their first context. */
helm_status helm_autotune(helm_ctx *ctx, int reps, int *chosen, double *ms);

/* Set the tile configuration (0..3) of transform kind (0 x64, 1 y64, 2 x32, 3 y32), forward and inverse, by hand. */
helm_status helm_gemm_config(helm_ctx *ctx, int kind, int cfg);

/* Scale an initial guess known up to its amplitude: x <- alpha x with the complex alpha minimising
 * ||F - alpha A x||_2, i.e. alpha = (A x)^H F / ||A x||^2 (the one-dimensional minimal-residual step of GMRES,
 * Sec. 3.1, taken over span{x}; alpha = 0 when A x = 0). Afterwards ||F - A x|| <= ||F||. F, x: device complex128
 * vectors of n entries (x overwritten). alpha_re, alpha_im: NULL or host doubles receiving alpha. Uses one matvec
 * and two inner products on the context stream and returns when alpha is known (the scaling is queued). The
 * first call allocates one vector of work in the context. */
helm_status helm_scale_guess(helm_ctx *ctx, const void *F, void *x, double *alpha_re, double *alpha_im);

/* ---- Batched solves (many right-hand sides and/or many independent problems) ----
 *
 * A batch groups P FGMRES(m) solves with the EigT preconditioner. Problem p uses the operator and the
 * eigen-data of contexts[p]; one context may appear several times (several right-hand sides, e.g. incident
 * directions, on one medium), and different contexts may have different grid sizes and k0 (uneven problems).
 * Every phase of an iteration (preconditioner transforms, z-solves, matvec, inner products, Givens updates,
 * linear combinations) is one grouped launch over all problems, the GEMMs as one persistent launch striding
 * over the tiles of every problem, and the Arnoldi/Givens/least-squares updates run on the device, so one
 * whole restart cycle is a fixed launch sequence that is captured once in a hipGraph and replayed. Problems
 * that have converged are skipped by every kernel. */
typedef struct helm_batch helm_batch;

/* Create a batch. All contexts must live on the current device, share the same order, and stay alive until
 * helm_batch_destroy. m: restart length (1..128). prec_fp32: 1 = complex FP32 preconditioner.
 * Allocates per problem (m+1) + m vectors (V, Z) of its size plus preconditioner work buffers, on a private
 * stream of the batch. */
helm_status helm_batch_create(helm_batch **batch, helm_ctx *const *contexts, int nprob, int m, int prec_fp32);

/* Solve A_p x_p = F_p for every problem to ||F_p - A_p x_p|| <= rtol ||F_p|| or maxit iterations.
 * F[p], x[p]: device vectors of problem p (complex128, n_p entries). x0_given = 1 starts from the x[p]
 * contents, else from 0. use_graph = 1 captures one restart cycle in a hipGraph on the first call and replays
 * it; 0 launches the same sequence directly. infos: NULL or an array of nprob. Work is ordered after prior
 * work on the stream of contexts[0] and the call returns when the batch is done. Returns HELM_ENOCONV if any
 * problem stopped at maxit. */
helm_status helm_batch_solve(helm_batch *batch, const void *const *F, void *const *x, int x0_given, double rtol,
                             int maxit, int use_graph, helm_solve_info *infos);

/* Free the batch (not the contexts). NULL is allowed. */
void helm_batch_destroy(helm_batch *batch);

/* Message of the last failure of a batch, or of the last helm_batch_create failure when batch is NULL. */
const char *helm_batch_last_error(const helm_batch *batch);

/* Number of unknowns n = Nx*Ny*Nz of a context. */
long long helm_size(const helm_ctx *ctx);

/* Message of the last failure on ctx (never NULL; "" if none). */
const char *helm_last_error(const helm_ctx *ctx);

/* Message of the last helm_setup failure in this process (never NULL). */
const char *helm_last_setup_error(void);

/* Free every buffer owned by ctx. NULL is allowed. */
void helm_destroy(helm_ctx *ctx);

/* Host-side 1D eigen-decomposition of Lambda-bar (Sec. 4.1, eq. lambda_mat_definition with zeta = 1):
 * Lambda-bar = V diag(d) V^{-1}. n >= 2; gamma as (re, im). Outputs are host arrays of complex128 (re, im):
 * d[n], V[n*n] and Vinv[n*n] in row-major order. Returns HELM_ENUMERIC if the residual checks fail. */
helm_status helm_eig1d(int n, double gamma_re, double gamma_im, double *d, double *V, double *Vinv);

/* The same with a corner off-diagonal zeta > 0 (eq. lambda_mat_definition; zeta = 2 for the collocated
 * three-point closure): Lambda-bar has zeta at (1, 2) and (N, N-1). Exported for tests. */
helm_status helm_eig1d_zeta(int n, double gamma_re, double gamma_im, double zeta, double *d, double *V,
                            double *Vinv);

/* ---------------------------------------------------------------------------------------------------------
 * Learned warm start: a 3D encoder-decoder CNN that maps (contrast, source) sampled on an S^3 grid to an
 * initial guess (Re u, Im u) on the same grid, trained and run on the GPU. It only supplies x0: the solver
 * (helm_gmres_solve with x0_given = 1) still converges to the caller's tolerance relative to ||F||, so a poor
 * prediction costs iterations, never accuracy.
 *
 * Network (channels 16/32/64/64 on levels S, S/2, S/4, S/8): per level two 3x3x3 convolutions with bias and
 * ReLU, 2x average pooling between levels; decoder: nearest 2x upsampling, concatenation [upsampled | skip],
 * one 3x3x3 convolution with ReLU per level; a linear 1x1x1 head to 2 channels. Convolutions have zero
 * padding and are cross-correlations, out[co][v] = b[co] + sum_{ci, tap} W[co][ci][tap] in[ci][v + off(tap)],
 * tap = 9 (dz+1) + 3 (dy+1) + (dx+1). Parameters are one FP32 array: per layer in the order above, W[co][ci][tap]
 * then b[co] (helm_cnn_num_params entries). MFMA operands are BF16 (bf16 = 1) or FP32, accumulation is FP32,
 * activations are stored in FP32. Tensors: device FP32, [batch][channel][z][y][x], x fastest.
 * All calls are ordered on the stream given at creation and return once the work is queued, except those that
 * copy to or from host memory, which return when the copy is done.
 * --------------------------------------------------------------------------------------------------------- */
typedef struct helm_cnn helm_cnn;

/* Create a network for S^3 volumes (size S: multiple of 8, >= 8) and batches up to max_batch, with He-uniform
 * initial weights drawn from `seed` and zero biases. stream: a hipStream_t or NULL (default stream).
 * Allocates all activations and their gradients (about 0.9 KiB per voxel of S^3 per sample) and the Adam moments.
 * Returns HELM_EINVAL on bad sizes, HELM_ENOMEM / HELM_EDEVICE on allocation or copy failure. */
helm_status helm_cnn_create(helm_cnn **net, int size, int max_batch, int bf16, unsigned long long seed, void *stream);

/* Number of FP32 parameters. */
long long helm_cnn_num_params(const helm_cnn *net);

/* Copy all parameters to / from host memory (helm_cnn_num_params floats, layout above). Setting them also
 * refreshes the packed MFMA operands. */
helm_status helm_cnn_get_params(helm_cnn *net, float *host_params);
helm_status helm_cnn_set_params(helm_cnn *net, const float *host_params);

/* Copy the gradient of the last helm_cnn_loss_grad call to host memory (same layout as the parameters). */
helm_status helm_cnn_get_grads(helm_cnn *net, float *host_grads);

/* Inference: x [B][2][S^3] (device) -> y [B][2][S^3] (device, may be NULL to keep the result internal).
 * 1 <= B <= max_batch. */
helm_status helm_cnn_forward(helm_cnn *net, const float *x, float *y, int B);

/* Forward, mean-squared-error loss L = mean((y - t)^2) over all B*2*S^3 outputs, and backward: dL/dparams into
 * the gradient buffer. t: device targets [B][2][S^3]. loss: NULL or host double receiving L (then the call
 * waits for it). */
helm_status helm_cnn_loss_grad(helm_cnn *net, const float *x, const float *t, int B, double *loss);

/* One Adam step (beta1 0.9, beta2 0.999, eps 1e-8, bias-corrected) on the FP32 master parameters with the
 * current gradient, learning rate lr > 0. */
helm_status helm_cnn_adam_step(helm_cnn *net, double lr);

/* helm_cnn_loss_grad followed by helm_cnn_adam_step. */
helm_status helm_cnn_train_step(helm_cnn *net, const float *x, const float *t, int B, double lr, double *loss);

/* Trilinear prolongation of a 2-channel prediction (Re, Im) on nc^3 nodes (i+1)/(nc+1) to the nf^3 nodes
 * (I+1)/(nf+1) of the unit cube, times `scale`, written as complex128 into `fine` (device, nf^3 entries).
 * Beyond the outermost coarse nodes the field follows the coarse grid's ghost rule, one factor
 * gamma = gamma_re + i gamma_im per axis crossed: U(-1) = gamma U(0), U(nc) = gamma U(nc-1) (Sec. 2.3, eq.
 * D_bc; gamma = (2 + i k0 h_c)/(2 - i k0 h_c) with h_c = 1/(nc+1) for the absorbing closure, 0 for Dirichlet).
 * cubic = 1 replaces the trilinear weights by Keys' cubic convolution (a = -1/2, coarse indices i0-1..i0+2 per
 * axis), the second ghost layer taking gamma^2 U(0) (the closure applied twice), computed as three 1-D passes;
 * it keeps a work buffer of (nf nc^2 + nf^2 nc) complex128 values in the network, allocated on first use and
 * grown for larger grids (HELM_EDEVICE if that allocation fails). */
helm_status helm_cnn_prolong(helm_cnn *net, const float *coarse, int nc, double scale, double gamma_re,
                             double gamma_im, int cubic, void *fine, int nf);

/* Network input for a solver problem on nf^3 unknowns: k2_halo (FP64) and f_halo (complex128) are the device
 * arrays given to helm_setup and helm_rhs, with `halo` >= 1 cells per side, nf >= S. Node (i, j, l) of the S^3
 * network grid is the point ((i, j, l) + 1)/(S + 1) of the unit cube; k^2 and f there are interpolated
 * trilinearly from the solver nodes (I + 1)/(nf + 1) (exact injection when nf + 1 is a multiple of S + 1).
 * Writes x [2][S^3] (device FP32): channel 0 = c_scale (k^2/k0^2 - 1), channel 1 = f_scale Re f.
 * Returns HELM_EINVAL on a halo below 1 or nf < S. */
helm_status helm_cnn_features(helm_cnn *net, const double *k2_halo, const void *f_halo, int halo, int nf, double k0,
                              double c_scale, double f_scale, float *x);

/* Message of the last failure of `net`, or of the last helm_cnn_create failure when net is NULL. */
const char *helm_cnn_last_error(const helm_cnn *net);

/* Free the network. NULL is allowed. */
void helm_cnn_destroy(helm_cnn *net);

#ifdef __cplusplus
}
#endif
#endif /* HELM_H */
