/*
 * phx: mixed-variational phononic band structures and adjoint design
 * sensitivities on one AMD Instinct MI355X (gfx950).
 *
 * Method (Lu, Yang, Guest, Srivastava, "3-D phononic crystals with ultra-wide
 * band gaps"):
 *   - a periodic two-phase unit cell, voxelized into nv^3 elements laid along
 *     the primitive vectors of an SC, BCC or FCC lattice (Methods, "Study of
 *     cubic unit cells");
 *   - displacement and stress expanded in the Bloch plane waves
 *     exp[i 2 pi K.x], K = T^T (Q + n), n in [-M, M]^3 (Results, "Phononic band
 *     structure calculation"), giving the mixed-variational eigenproblem
 *     H Phi^{-1} H^* U = lambda Omega U, lambda = omega^2 (Eq. 4) with the
 *     matrices of Eqs. (5)-(7) evaluated by the element-centroid rule
 *     (Eqs. 16-19);
 *   - design sensitivities d omega / d rho_e from the adjoint form of Eq. (15)
 *     with the element derivative matrices of Eqs. (20)-(21).
 *
 * Conventions shared by every call:
 *   - All arrays are owned by the caller.  Host-pointer calls copy in and out
 *     and return only after the results are in the caller's arrays; the
 *     library keeps no caller pointer after a call returns.
 *   - Units: SI in (m, kg/m^3, Pa); omega out in rad/s; derivatives of omega
 *     in rad/s per unit of rho_e.
 *   - Design fields rho are nv^3 doubles in C order [i1][i2][i3], i_j along
 *     primitive vector a_j; voxel e = (i1, i2, i3) has centroid
 *     sum_j (i_j + 1/2)/nv a_j.  rho_e = 0 is phase0, rho_e = 1 is phase1;
 *     density and compliance are affine in w_e = rho_e^simp_p.
 *   - Bloch vectors are given in reciprocal coordinates Q (3 doubles per
 *     k-point): K = sum_j (Q_j + n_j) b_j with a_i . b_j = delta_ij.
 *   - Bands are numbered from 1 in ascending omega.
 *   - Every call returns PHX_OK (0), a negative error or a positive warning;
 *     phx_last_error() then describes it.  One context per host thread; calls
 *     on a context are serialised on its HIP stream.
 */
#ifndef PHX_H
#define PHX_H

#ifdef __cplusplus
extern "C" {
#endif

#define PHX_OK 0
#define PHX_EINVAL (-1)  /* invalid argument (checked on the host before any device work) */
#define PHX_ENOMEM (-2)  /* device allocation failed */
#define PHX_EHIP (-3)    /* a HIP runtime call failed, or no device */
#define PHX_ENOCONV (-4) /* eigensolver hit its iteration cap; outputs hold the last iterate */
#define PHX_ENOTPD (-5)  /* a matrix that must be positive definite failed its Cholesky */
/* Warning (outputs complete and valid): a band whose sensitivity was requested lies in a
 * degenerate cluster (see phx_sens).  Eq. (15) defines d lambda / d rho_e for a simple
 * eigenvalue only; the paper does not discuss repeated eigenvalues. */
#define PHX_WDEGEN 1

typedef struct phx_ctx phx_ctx;

typedef enum { PHX_SC = 0, PHX_BCC = 1, PHX_FCC = 2 } phx_lattice;

/* PHX_FP64: every factorisation and solve in FP64.
 * PHX_MIXED: the per-k pencil factorisation and the preconditioner solves in
 * FP32 on the matrix cores; residuals, Rayleigh-Ritz and the material
 * operators in FP64, so converged eigenvalues carry FP64 residuals. */
typedef enum { PHX_FP64 = 0, PHX_MIXED = 1 } phx_precision;

typedef struct {
  double density; /* kg/m^3, > 0 */
  double youngs;  /* Pa, > 0 */
  double poisson; /* in (-1, 1/2) */
} phx_material;

typedef struct {
  phx_lattice lattice;
  double a;            /* conventional cube edge (m), > 0 */
  int nv;              /* voxels per primitive axis; must satisfy nv >= 2M+1 */
  int M;               /* plane-wave order, 1 <= M <= 8; N = (2M+1)^3 waves */
  phx_material phase0; /* rho_e = 0 */
  phx_material phase1; /* rho_e = 1 */
  double simp_p;       /* w = rho^p, p >= 1 */
} phx_cell;

/* ------------------------------------------------------------------ context */

/* Creates a context on HIP device `hip_device` with its own stream.
 * Returns PHX_EHIP if the device is missing. */
int phx_create(phx_ctx** out, int hip_device);
int phx_destroy(phx_ctx* ctx);
/* Message of the last call on ctx that did not return PHX_OK (valid until the next call). */
const char* phx_last_error(const phx_ctx* ctx);

/* Solver options.  Keys: "tol_fp64", "tol_mixed" (relative residual
 * |K x - lambda Omega x| / ((lambda + sigma)|Omega x|) at which a band counts as
 * converged; defaults 1e-8 and 1e-6), "maxit" (default 60), "block" (search
 * block size s, 0 = automatic, else nbands < s <= 21), "shift" (preconditioner
 * shift relative to the lowest shear-wave eigenvalue scale, default 0.02),
 * "drop" (Omega-orthonormalisation drops a search column whose orthogonal part
 * has squared norm below drop times its own, default 1e-8),
 * "sbinv" (1, default: the preconditioner's triangular solves use explicit
 * inverses of the factor's 256-wide (FP64: 128-wide) diagonal blocks, computed
 * once per factorisation, so every solve step is a matrix product; 0: blocked
 * substitution inside each diagonal block),
 * "kshare" (1..8, default 2), "kshare_dist" (default 0.15) and "kshare_rel"
 * (default 0.5): consecutive k-points of a chunk that lie within kshare_dist
 * (Cartesian, cycles per a) of a group's first k-point, and within kshare_rel
 * times the shorter of the two wave vectors, share that k-point's
 * preconditioner factor, at most kshare of them (needs "sbinv"; 1: every
 * k-point has its own factor; Gamma never shares).  Wider sharing (e.g. 4
 * within 0.5) saves factorisations on smooth designs but costs iterations on
 * sharp high-contrast inclusions,
 * "kskip" (1, default: a k-point whose wanted bands all meet the tolerance is
 * frozen, its vectors, eigenvalues and residuals kept, and the remaining
 * iterations of its chunk skip it; 0: every k-point of a chunk iterates until the
 * slowest converges; every per-k decision of the eigensolver is taken per k-point,
 * so with kshare = 1 a k-point's results depend neither on the other k-points of its
 * chunk nor on the chunk size),
 * "rr_fused" (2, default: both Omega-orthonormalisations of the search basis folded
 * into the Rayleigh-Ritz step in the small m x m space, so an iteration makes one Gram
 * product and one basis update; 1: one explicit Omega-orthonormalisation of the basis,
 * the second folded; with 1 and 2 a k-point whose residual is below 1e-13/tolerance (the
 * last iterations of an FP64 solve) has its basis orthonormalised twice explicitly; 0:
 * always two explicit orthonormalisations of the basis before Rayleigh-Ritz),
 * "small_eig" (1, default: the eigenproblem of the folded Rayleigh-Ritz step, order
 * m = 3s, by Householder reduction to real tridiagonal form, multisection on Sturm
 * counts and inverse iteration, with exactly zero rows of the projected matrix (null
 * vectors of K in the basis) deflated as eigenvalue 0; eigenvalues accurate to a small
 * multiple of eps times the projected matrix's norm; 0: cyclic Jacobi, accurate relative
 * to each eigenvalue and several times slower; more than 24 wanted pairs always take
 * Jacobi; also selects the solver of phx_small_rr),
 * "mem_gb" (device memory budget that sets the k-chunk size, default 64; per worker
 * context of phx_sens_batch_dev), "mem_limit_gb" (hard cap on the device workspace one
 * context, or each worker context of a batched call, may hold; 0, default: none; a
 * workspace that would exceed it fails like a failed allocation), "streams" (1..16, see
 * phx_sens_batch_dev),
 * "coarse" (1:
 * for M >= 4 every k-chunk is first solved at order M-2 to the residual
 * "coarse_tol", default 1e-3, and its Ritz vectors, embedded in the order-M
 * plane-wave set, start the order-M solve; 0: start from plane-wave unit
 * vectors; default 1), "coarse_drop" (1..3, default 2: the coarse start's order is
 * M - coarse_drop, at least 1),
 * "profile" (0, default: off; 1: every kernel class is timed with HIP events,
 * stage intervals on the library stream and, for the classes herk, op_gemm,
 * op_conv, solve_upd and solve_diag, events that each launch records at its kernel's
 * start and end; 2: only the latter, which disturbs concurrent streams least),
 * "profile_reset" (any value: clears the class timers),
 * "kstreams" (1..16, default 1): phx_bands_dev, phx_sens_dev and phx_adjoint_dev
 * split the k-points into this many consecutive ranges solved concurrently on worker
 * streams (one design alone leaves most of the GPU idle); each range has its own
 * preconditioner factors and coarse start,
 * "gram_split" (0..16; 0, default: min(16, 3Np / 256)): the eigensolver's Gram
 * products S^H [K S | Omega S] are split over this many parts of their long
 * dimension (partial products summed by a second kernel; 1: one kernel),
 * "spin_wait" (0, default: the eigensolver's once-per-iteration host wait sleeps on a
 * blocking-sync event, leaving the core to the threads of concurrent design
 * streams; 1: it spins in hipStreamSynchronize),
 * "guard_lock" (1..1e4, default 1000: the eigensolver's guard vectors, the block columns
 * beyond the wanted bands, are soft locked once their relative residual is below
 * guard_lock x the tolerance, the wanted bands' at the tolerance itself; the guards are
 * not results, and a wanted band still counts as converged only at the tolerance; 1: every
 * column locks at the tolerance),
 * "zskip" (1, default: the Gram product and the basis update of the eigensolver's
 * Rayleigh-Ritz step do not load the basis columns known to be zero, the search and
 * previous directions of soft-locked columns and their images; 0: they load every
 * column; the results are identical),
 * "omega_conv" (1, default: for orders M <= 5 the eigensolver's products Omega_s X are
 * exact convolutions of the density's Fourier coefficients with the columns, by DFTs of
 * length 4M+1 (Omega_s is Toeplitz in the wave index, Eqs. (6)-(7)); 0: products with the dense
 * N x N matrix; both give the same result up to rounding),
 * "precond" (the eigensolver's preconditioner; 0: the Cholesky factor of the shifted
 * pencil K(k) + sigma Omega, assembled per k-point (or per group of k-points, see
 * "kshare"); 1: block Jacobi, the 3 x 3 diagonal block of that pencil for each plane wave,
 * built from the diagonals of the k-independent operators and the wave vectors, so K(k)
 * is never formed or factored; converges as fast as the pencil on smooth designs and far
 * slower on sharp high-contrast inclusions; 2, default: block Jacobi first, and a
 * k-point whose residual has not fallen tenfold over the last "stall_its" iterations
 * (default 8, 2..30), or that reaches iteration 30, gets its own pencil factor (shared
 * with k-points that stall in the same iteration, as "kshare" allows) from then on),
 * "degen_tol" (default 1e-8; 0 disables): consecutive frequencies of one k-point whose
 * relative gap (omega_{i+1} - omega_i) / omega_{i+1} is below this form a degenerate
 * cluster (see phx_sens).
 * A k-chunk whose workspaces cannot be allocated (or would exceed mem_limit_gb) is
 * freed and solved again with half as many k-points, down to one, before PHX_ENOMEM is
 * returned.
 * Returns PHX_EINVAL for an unknown key or an out-of-range value. */
int phx_set_option(phx_ctx* ctx, const char* key, double value);
/* Statistics of the last solve: "iters" (eigensolver iterations of the
 * slowest chunk), "chunks", "block", "kchunk", "rr_sweeps" (most Jacobi sweeps
 * one Rayleigh-Ritz step needed at any k), "coarse_iters" (iterations of the
 * coarse start), "iters_mean_k" (mean over k-points of the iteration at which
 * each met the tolerance), "factors" (preconditioner factorisations of the
 * order-M solves), "degen" (requested (k, band) entries inside a degenerate cluster),
 * "precond_switches" (solves that went from block Jacobi to the pencil factors),
 * "enomem_retries" (k-chunks solved again with fewer k-points), "mem_bytes" (device
 * workspace the context holds).  "prof.<class>.<ms|flops|bytes|count>"
 * reads the kernel-class timers (enabled with the option "profile"); the classes:
 * potrf_diag, panel, herk, trsm_diag, trsm_update, solve_upd, solve_diag, sbinv,
 * assemble, apply, op_gemm, gram, small, update, residual, adjoint, op_conv. */
int phx_get_stat(const phx_ctx* ctx, const char* key, double* value);

/* ------------------------------------------------------------------ helpers */

/* k-points along the edges of the irreducible Brillouin zone (Results, "A note
 * on normalized band gaps"; Methods, "Study of cubic unit cells"), as
 * reciprocal coordinates q_out[3*nk].  `path` names high-symmetry points (G for
 * Gamma; SC: X M R; BCC: H N P; FCC: X W K L U) with "|" for a break; NULL
 * selects G-X-M-G-R-X|M-R (SC), G-H-N-G-P-H|P-N (BCC), G-X-W-K-G-L-U-W-L-K|U-X
 * (FCC).  Every vertex is included and the other points are spread over the
 * segments in proportion to their length (largest remainder), evenly inside a
 * segment.  Host-only; needs no context.  PHX_EINVAL if nk is smaller than the
 * number of vertices or the path names an unknown point. */
int phx_kpath(phx_lattice lattice, const char* path, int nk, double* q_out);

/* Host-only argument check shared by every solver call: the cell (lattice,
 * a > 0, 1 <= M <= 8, 2M+1 <= nv <= 256, materials, simp_p >= 1), rho (if not
 * NULL: nv^3 finite non-negative values), q (if nk or q given: nk >= 1 finite
 * triples), bands (if nbands or nsens given: 1 <= nbands <= min(16, 3N), band_no
 * entries in [1, nbands]).  Writes a message into msg (msglen bytes, may be
 * NULL).  Needs no device. */
int phx_validate(const phx_cell* cell, const double* rho, int nk, const double* q, int nbands, int nsens,
                 const int* band_no, char* msg, int msglen);

/* ------------------------------------------------------------------ stages */

/* Centroid-rule Fourier coefficients of the density and of the two Mandel
 * compliance channels (1/(3K) and 1/(2G)) of the interpolated design, the
 * building blocks of Eqs. (6)-(7) through Eqs. (16)-(19):
 *   ghat(m) = v sum_e g_e exp(i 2 pi m . s_e),  m in [-2M, 2M]^3, v = V / nv^3.
 * out: 3 * (4M+1)^3 complex values as (re, im) double pairs, order
 * [field][m1+2M][m2+2M][m3+2M], fields (density, c_vol, c_dev), SI units
 * (kg and m^3/Pa). */
int phx_fourier(phx_ctx* ctx, const phx_cell* cell, const double* rho, double* out);

/* The stress-eliminated operator of Eq. (4), K(Q) = H Phi^{-1} H^*, at one Bloch
 * vector q (3 doubles), as a dense 3N x 3N complex matrix, column-major, rows
 * and columns ordered (plane wave p, component c) -> 3p + c, plane waves in
 * lexicographic order of (n1, n2, n3) with n1 slowest; SI units (N/m).
 * out: 2 * (3N)^2 doubles. */
int phx_schur(phx_ctx* ctx, const phx_cell* cell, const double* rho, const double* q, double* out);

/* ------------------------------------------------------------------ band structure */

/* Lowest `nbands` eigenfrequencies of Eq. (4) at nk Bloch vectors.
 * omega: nk * nbands (rad/s, ascending per k).  err_bound (may be NULL):
 * nk * nbands residual-based bounds on |omega - omega_exact| for the
 * discretised problem.  1 <= nbands <= 16.  PHX_ENOCONV if a band did not reach
 * the tolerance (outputs hold the last iterate). */
int phx_bands(phx_ctx* ctx, const phx_cell* cell, const double* rho, int nk, const double* q, int nbands,
              phx_precision prec, double* omega, double* err_bound);

/* Bands plus d omega_b / d rho_e (Eq. 15 with Eqs. 20-21) for the nsens bands
 * band_no[0..nsens) (1-based, each <= nbands), at every k-point.
 * domega_drho: nk * nsens * nv^3, order [k][sens][e].  A band with omega = 0
 * (acoustic bands at Gamma) gets a zero derivative.
 * Degenerate clusters: Eq. (15) needs a simple eigenvalue.  Where the requested band b
 * and its neighbours form a cluster (option "degen_tol"; clusters are formed among the
 * solver's Ritz pairs, which extend past nbands by its guard vectors), the per-vector
 * derivatives depend on which orthonormal basis of the cluster's eigenspace the solver
 * returned, but their sum over the cluster does not; band b then receives the mean of
 * d omega_i / d rho_e over every member i of its cluster (basis-independent, and equal to
 * the derivative of the cluster's mean frequency), and the call returns PHX_WDEGEN
 * (after PHX_ENOCONV in precedence) with the outputs complete. */
int phx_sens(phx_ctx* ctx, const phx_cell* cell, const double* rho, int nk, const double* q, int nbands,
             phx_precision prec, int nsens, const int* band_no, double* omega, double* domega_drho);

/* Weighted adjoint: grad_e = sum_{k, j} weight[k * nsens + j] d omega_{band_no[j]}(k) / d rho_e,
 * i.e. the gradient of any objective of the band frequencies given its
 * partial derivatives (Eq. 15 followed by the chain rule through Eq. 10).
 * omega: nk * nbands (may be NULL); grad: nv^3.  Derivatives inside degenerate
 * clusters follow phx_sens (cluster means; PHX_WDEGEN). */
int phx_adjoint(phx_ctx* ctx, const phx_cell* cell, const double* rho, int nk, const double* q, int nbands,
                phx_precision prec, int nsens, const int* band_no, const double* weight, double* omega,
                double* grad);

/* Several designs (cells may differ in lattice, nv and M) through one call:
 * omega[d] receives nk * nbands values for design d; if band_no is given,
 * domega[d] (if not NULL) receives nk * nsens * nv_d^3 sensitivities. */
int phx_bands_batch(phx_ctx* ctx, int ndesign, const phx_cell* cells, const double* const* rho, int nk,
                    const double* q, int nbands, phx_precision prec, int nsens, const int* band_no,
                    double* const* omega, double* const* domega);

/* Device-pointer variants, used by the PyTorch binding.  rho_dev (nv^3),
 * omega_dev (nk * nbands), domega_dev (nk * nsens * nv^3), weight_dev
 * (nk * nsens) and grad_dev (nv^3) are device arrays; q_host and band_no stay
 * on the host.  Work already queued on `stream` (a hipStream_t, may be NULL)
 * is waited for first; the call then runs on the context's stream and returns
 * after its results are in place.  Same errors as the host calls; a non-finite
 * or negative rho is detected after copying the design to the host. */
int phx_bands_dev(phx_ctx* ctx, const phx_cell* cell, const double* rho_dev, int nk, const double* q_host,
                  int nbands, phx_precision prec, double* omega_dev, void* stream);
int phx_sens_dev(phx_ctx* ctx, const phx_cell* cell, const double* rho_dev, int nk, const double* q_host,
                 int nbands, phx_precision prec, int nsens, const int* band_no, double* omega_dev,
                 double* domega_dev, void* stream);
/* Several designs (cells may differ in lattice, nv and M) at the same k-points:
 * rho_dev[d] (nv_d^3), omega_dev[d] (nk * nbands), domega_dev[d]
 * (nk * nsens * nv_d^3, only if nsens > 0; domega_dev may be NULL otherwise)
 * are device arrays.  The designs are spread over up to "streams" (option,
 * default 4) worker contexts, each with its own HIP stream and workspaces, so
 * the latency-bound steps of one design overlap the matrix-core work of
 * another; the highest M goes first.  HIP maps streams onto GPU_MAX_HW_QUEUES
 * hardware queues (environment, read when the HIP runtime starts; 4 by
 * default): streams sharing a queue run their kernels in turn, so set it to at
 * least "streams".  Statistics and kernel-class timers of
 * the workers are merged into ctx.  Returns the first error (naming the
 * design), else PHX_ENOCONV if any design did not converge. */
int phx_sens_batch_dev(phx_ctx* ctx, int ndesign, const phx_cell* cells, const double* const* rho_dev, int nk,
                       const double* q_host, int nbands, phx_precision prec, int nsens, const int* band_no,
                       double* const* omega_dev, double* const* domega_dev, void* stream);
/* grad_dev = sum_{k, j} weight_dev[k * nsens + j] d omega_{band_no[j]}(k) / d rho_e
 * (the backward of any objective of the band frequencies); omega_dev may be NULL. */
int phx_adjoint_dev(phx_ctx* ctx, const phx_cell* cell, const double* rho_dev, int nk, const double* q_host,
                    int nbands, phx_precision prec, int nsens, const int* band_no, const double* weight_dev,
                    double* omega_dev, double* grad_dev, void* stream);

/* ------------------------------------------------------------------ dense building blocks */

/* Batched complex GEMM on the matrix cores: C_b = alpha op(A_b) op(B_b) + beta C_b,
 * column-major, op 'N' or 'C' (conjugate transpose); A_b = A + b*strideA etc.
 * (element strides; 0 shares an operand).  prec selects FP64 or FP32
 * arithmetic (FP32 operands are rounded from the FP64 host arrays).  Host
 * arrays of (re, im) doubles. */
int phx_zgemm(phx_ctx* ctx, phx_precision prec, char opa, char opb, int m, int n, int k, const double* alpha,
              const double* A, long lda, long strideA, const double* B, long ldb, long strideB, const double* beta,
              double* C, long ldc, long strideC, int batch);

/* Batched Hermitian positive definite solve A_b X_b = B_b by Cholesky: A is
 * batch x n x n (lower triangle read), B is batch x n x nrhs; X overwrites B.
 * n must be a multiple of 64.  PHX_ENOTPD if a pivot is not positive.  With the
 * option "sbinv" set, solves with at most 32 right-hand sides go through the
 * diagonal super-block inverses, as in the eigensolver. */
int phx_zposv(phx_ctx* ctx, phx_precision prec, int n, int nrhs, int batch, const double* A, double* B);

/* Small dense kernels of the block eigensolver (one workgroup per batch item,
 * order m <= 64, FP64, column-major (re, im) pairs).
 * phx_small_orth: from a Hermitian Gram matrix G = S^H W S of a basis S, the
 * coefficients C0 (m x m, upper triangular) with (S C0)^H W (S C0) = I on the
 * kept columns; columns are first scaled to unit norm and a column whose
 * Cholesky pivot falls below `drop` is dropped (keep = 0, its C0 column zero).
 * phx_small_eig: the s lowest eigenpairs of the Hermitian G (m x m) restricted
 * to the columns with keep != 0, by cyclic Jacobi: C (m x s) eigenvectors,
 * theta (s) ascending. */
int phx_small_orth(phx_ctx* ctx, int m, int batch, const double* G, double drop, double* C0, int* keep);
int phx_small_eig(phx_ctx* ctx, int m, int s, int batch, const double* G, const int* keep, double* C,
                  double* theta);
/* phx_small_rr: Rayleigh-Ritz on a basis S that is only approximately
 * Omega-orthonormal, from G2 = S^H [K S | Omega S] (m x 2m per batch item):
 * Omega-Cholesky with scaling and dropping as phx_small_orth, then the s lowest
 * eigenpairs of the projected K (by the solver the option "small_eig" selects).
 * Cx (m x s): Ritz-vector coefficients in S
 * ((S Cx)^H Omega (S Cx) = I, G_K Cx = G_Omega Cx diag(theta)); Cp (m x s): the
 * same with only the contributions of columns s.. of the orthonormalised basis
 * (the previous-direction update); keep (m): columns kept by the Cholesky. */
int phx_small_rr(phx_ctx* ctx, int m, int s, int batch, const double* G2, double drop, double* Cx, double* Cp,
                 double* theta, int* keep);

/* ------------------------------------------------------------ design projection */

/* The design parameterisation of the topology optimisation (section "Topology
 * optimization formulation": the Heaviside projection method with a reduced design
 * variable field and continuation on the Heaviside parameter; section "Study of cubic
 * unit cells": the SC design optimised on one eighth of the cell, mirrored about the
 * cell's mid-planes).  Elements are the nv^3 voxels (centroids at i + 1/2 element
 * widths along each primitive axis).  Design nodes sit every `spacing` elements, node j
 * at the centre of elements spacing*j .. spacing*j + spacing - 1; nn = nv / spacing per
 * axis.  With `octant` the design array holds nodes j < nn/2 per axis and node j >= nn/2
 * takes the value of node nn - 1 - j.  Per element, with w_en = max(0, radius - |x_e -
 * x_n|) (periodic minimum image, element widths, index space):
 *   mu_e  = sum_n w_en x_n / sum_n w_en,
 *   rho_e = 1 - exp(-beta mu_e) + mu_e exp(-beta)          (beta = 0: rho = mu).   */
typedef struct {
  int nv;        /* elements per primitive axis */
  int spacing;   /* 1 or 2 elements between design nodes; nv % spacing == 0 */
  double radius; /* projection radius in element widths: > sqrt(3)/2 for spacing 2,
                    > 0 for spacing 1, and 2 radius + spacing < nv */
  double beta;   /* Heaviside parameter, 0 <= beta <= 1000 */
  int octant;    /* 1: mirrored octant design (nn even) */
} phx_projection;

/* Number of design variables: nn^3, or (nn/2)^3 with the octant.  Host only. */
int phx_projection_size(const phx_projection* p, long* ndesign);
/* rho (nv^3, C order [i1][i2][i3]) from the design variables x (C order over the design
 * nodes).  Host arrays (copied in and out) or device arrays (the _dev form, ordered after
 * the caller's `stream`, complete on return).  PHX_EINVAL for an invalid projection. */
int phx_project(phx_ctx* ctx, const phx_projection* p, const double* x, double* rho);
int phx_project_dev(phx_ctx* ctx, const phx_projection* p, const double* x_dev, double* rho_dev, void* stream);
/* grad_x = (d rho / d x)^T grad_rho: the backward of phx_project (chain rule through the
 * Heaviside, the filter and the mirror images). */
int phx_project_adjoint(phx_ctx* ctx, const phx_projection* p, const double* x, const double* grad_rho,
                        double* grad_x);
int phx_project_adjoint_dev(phx_ctx* ctx, const phx_projection* p, const double* x_dev, const double* grad_rho_dev,
                            double* grad_x_dev, void* stream);
/* The same backward for callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving or optimisation loops, harnesses that forbid hipMalloc): the
 * per-element scratch of the computation lives in a fixed device array of the library
 * (nv^3 doubles, nv <= 64; one per GPU, held until the process ends), so this call makes
 * no hipMalloc, hipFree or other allocating call.  x_dev, grad_rho_dev and grad_x_dev are
 * the caller's device arrays as for phx_project_adjoint_dev.  The work is queued on
 * `stream` (the context's stream if NULL) and the call returns without waiting for it.
 * Every call on one GPU uses that GPU's one scratch array: calls that can run at the same
 * time on one GPU (on different streams, or from different contexts) race and give wrong
 * results; calls ordered on one stream do not.  PHX_EINVAL for an invalid projection or
 * nv > 64. */
int phx_project_adjoint_dev_noalloc(phx_ctx* ctx, const phx_projection* p, const double* x_dev,
                                    const double* grad_rho_dev, double* grad_x_dev, void* stream);

#ifdef __cplusplus
}
#endif
#endif /* PHX_H */
