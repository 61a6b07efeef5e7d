/*
 * rbcg.h -- C ABI of the MI355X (gfx950) randomized block-CG library.
 *
 * The library solves regularized symmetric positive definite systems
 *     (A + mu I) x = b,      A in R^{d x d} SPD, mu >= 0
 * (paper: Sec. 1, eq. regularized_ls) with block-CG on the block Krylov space
 * K_t(A, [b Omega]) of the augmented start block [b Omega], Omega a d x k
 * Gaussian block (Sec. 3, def. BCG; Thm. main).  It is implemented with
 * block-Lanczos and full reorthogonalisation, after which the iterate for any
 * shift is ||b|| Q_t (T_t + mu I)^{-1} e_1 (Sec. 3.2, eq. bcg_alg).
 *
 * Three entry points follow the paper's three problem statements:
 *   rbcg_solve       one shift per system, many independent systems per call
 *                    (Sec. 1, eq. regularized_ls)
 *   rbcg_path        one operator, L shifts from one Krylov space: the whole
 *                    ridge-regression path when A = Z^T Z (Sec. 1,
 *                    eq. ridge_regression; Sec. 3.2, eq. bcg_alg)
 *   rbcg_sqrt_apply  Gaussian sampling A^{1/2} B by the block-Lanczos square
 *                    root with a quadrature over the shifts z^2 (Sec. 1,
 *                    eq. sqrt_rational; Sec. 5, def. blansq); rbcg_invsqrt_apply
 *                    is the inverse square root A^{-1/2} B (whitening) from the
 *                    same Lanczos data and rule (Sec. 5.1, def. blanisq)
 *
 * Conventions for every call
 *   - Memory: every matrix or vector argument documented as "device" is a
 *     pointer into GPU memory of the device current when the context was
 *     created; "host" arguments are ordinary host memory.  The caller owns
 *     all of them.  The library reads inputs, writes outputs, never frees or
 *     retains caller pointers after the call returns, and never modifies
 *     inputs.  Internal workspace belongs to the context (rbcg_ctx) or to an
 *     operator handle (rbcg_op) and is released by the matching destroy call.
 *   - Layout: matrices are row-major.  A set of r vectors of length d is an
 *     r x d row-major array (vector i at offset i*ld), i.e. what a
 *     contiguous torch tensor of shape (r, d) holds.
 *   - Streams: work is enqueued on the stream bound to the context.  Every
 *     solver call returns only after its results are complete (it
 *     synchronises that stream), because the iteration count and the status
 *     are decided on the device.
 *   - Errors: functions return an rbcg_status code.  Argument validation
 *     happens before any device work; on RBCG_ERR_INVALID_ARG nothing has
 *     been enqueued and outputs are untouched.  rbcg_status_string gives a
 *     static description.
 *   - Threads: a context must not be used by two threads at once.  Distinct
 *     contexts are independent.
 */
#ifndef RBCG_H
#define RBCG_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  RBCG_OK = 0,
  RBCG_ERR_INVALID_ARG = -1,    /* bad size, pointer, tolerance or option */
  RBCG_ERR_NOT_SPD = -2,        /* a non-positive pivot in T_t + mu I or in a start block; with
                                   refinement (rtol > 0) only when the final FP64 residual also
                                   misses rtol (a later sweep can repair a spoiled one) */
  RBCG_ERR_BREAKDOWN = -3,      /* the whole block deflated before convergence */
  RBCG_ERR_NO_CONVERGENCE = -4, /* budget exhausted; best iterate written, info.relres set */
  RBCG_ERR_HIP = -5,            /* a HIP runtime call failed */
  RBCG_ERR_OOM = -6,            /* device workspace allocation failed */
  RBCG_ERR_UNSUPPORTED = -7,    /* device is not gfx950, or an unsupported option combination */
  RBCG_ERR_TOO_LARGE = -8       /* rbcg_op_apply_noalloc: the call needs more device scratch than
                                   the fixed buffer holds (see rbcg_noalloc_scratch_bytes) */
} rbcg_status;

typedef enum { RBCG_F64 = 0, RBCG_F32 = 1, RBCG_BF16 = 2 } rbcg_dtype;
typedef enum { RBCG_OP_DENSE = 0, RBCG_OP_GRAM = 1 } rbcg_op_kind;

typedef struct rbcg_ctx rbcg_ctx;
typedef struct rbcg_op rbcg_op;

/* Static description of a status code (never NULL). */
const char* rbcg_status_string(int status);

/* Library version as major*10000 + minor*100 + patch. */
int rbcg_version(void);

/* Create a context bound to `hip_stream` (a hipStream_t; NULL = the null
 * stream) on the current device.  Fails with RBCG_ERR_UNSUPPORTED when the
 * current device is not gfx950. */
int rbcg_create(rbcg_ctx** ctx, void* hip_stream);
int rbcg_destroy(rbcg_ctx* ctx);

/* ------------------------------------------------------------------ operators
 * An operator handle describes A and holds the low-precision copies used by
 * mixed-precision block products.  The caller's master data must stay alive
 * and unchanged while the handle is used.
 *
 * Dense:  A is d x d, row-major, FP64, leading dimension lda >= d, symmetric
 *         positive semi-definite (Sec. 1).  `lo` chooses which low-precision
 *         copy to build now: RBCG_F64 = none, RBCG_F32 = FP32 copy (RNE).
 * Gram:   A = Z^T Z with Z n x d row-major FP32, ldz >= d, 1 <= n < 2^31,
 *         1 <= d <= 2^21 (Sec. 1, ridge regression).  The block product is
 *         Z^T (Z X) (two passes over Z).  The handle always holds an FP32
 *         copy of Z^T (4 n d bytes), which the second pass of the FP64
 *         products and residuals streams; `lo` = RBCG_BF16 also builds BF16
 *         copies of Z and of Z^T (RNE); RBCG_F64 builds no further copy
 *         (FP64 arithmetic on the FP32 values).
 */
int rbcg_op_create_dense(rbcg_ctx* ctx, rbcg_op** op, int64_t d, const double* A /*device*/,
                         int64_t lda, int lo);
int rbcg_op_create_gram(rbcg_ctx* ctx, rbcg_op** op, int64_t n, int64_t d, const float* Z /*device*/,
                        int64_t ldz, int lo);

/* Dense operator whose A stays in host memory: the out-of-core setting of the
 * paper's wall-clock experiment (Sec. 7.1.1, intro figure: A is held in row
 * chunks and every block product loads each chunk once, so run time follows
 * the number of matrix-loads).  A_host is d x d, row-major, FP64, leading
 * dimension lda >= d, in page-locked host memory (hipHostMalloc, or a pinned
 * torch tensor); pageable memory is rejected with RBCG_ERR_INVALID_ARG.
 * chunk_rows (1 <= chunk_rows <= d) rows are copied per chunk, on a copy
 * stream the handle owns, into one of two device staging buffers of
 * chunk_rows * lda doubles; the block-product kernel then forms those rows of
 * A X while the next chunk copies.  `lo` = RBCG_F32 also builds an FP32 copy
 * (RNE, rows padded to 64 values) in page-locked host memory the handle
 * allocates, which low-precision products stream (half the bytes per load);
 * FP64 residuals always stream A itself.  Everything the handle allocates is
 * freed by rbcg_op_destroy.  Every call that takes an operator accepts it;
 * FP32 products without the FP32 copy return RBCG_ERR_UNSUPPORTED.  rbcg_solve
 * learns each step's convergence before it streams the next product;
 * rbcg_path, rbcg_sqrt_apply and rbcg_invsqrt_apply keep their step loop,
 * which may stream one product past convergence.  The staging buffers belong to the handle: calls
 * that use one streamed handle at the same time (from several contexts or
 * threads) race. */
int rbcg_op_create_dense_host(rbcg_ctx* ctx, rbcg_op** op, int64_t d, const double* A_host /*host, pinned*/,
                              int64_t lda, int64_t chunk_rows, int lo);
int rbcg_op_destroy(rbcg_op* op);

/* ---------------------------------------------------------------------- options */
typedef struct {
  int32_t t_max;       /* max block products (matrix-loads) per Krylov space; >= 1 */
  double rtol;         /* stop when ||b - A_mu x|| / ||b|| <= rtol (FP64 residual);
                          0 = run exactly t_max products, no refinement */
  int32_t matvec;      /* rbcg_dtype of the block products: F64 = plain; F32 (dense) or
                          BF16 (Gram) = low precision with FP32 accumulation and FP64
                          iterative refinement */
  int32_t refine_max;  /* max Krylov spaces (refinement sweeps) when rtol > 0; >= 1 */
  int32_t nquad;       /* rbcg_sqrt_apply: quadrature nodes (default 32 when 0) */
  int32_t group;       /* rbcg_sqrt_apply: samples per Krylov block (default 32 when 0) */
  double eta;          /* deflation threshold relative to a block's pre-projection norm
                          (default 1e-10 when 0) */
  double sweep_tol;    /* low-precision products with rtol > 0: reduction of the residual
                          that one Krylov space aims for before the next FP64 residual
                          (0 = default: 1e-4 for FP32, 1e-6 for BF16); never below what
                          the remaining rtol needs */
  uint64_t seed;       /* start blocks passed as NULL (omega, or omega[s] of rbcg_solve) with
                          k > 0 are drawn on the device from this seed: the layout of
                          rbcg_omega_fill with stream = s (system index) for rbcg_solve and
                          stream = 0 for rbcg_path */
  int32_t reorth;      /* rbcg_reorth: how each new block is orthogonalised against the basis
                          (Sec. 3.2 uses full reorthogonalisation; the numerical appendix also
                          runs none and a partial scheme).  One policy per rbcg_solve call. */
  int32_t reorth_blocks; /* RBCG_REORTH_PARTIAL: leading blocks kept (default 3 when 0) */
} rbcg_opts;

typedef enum {
  RBCG_REORTH_FULL = 0,     /* against every previous block, two passes (BCGS2); the default */
  RBCG_REORTH_NONE = 1,     /* against the last two blocks only: the block three-term
                               recurrence of block Lanczos, two passes */
  RBCG_REORTH_PARTIAL = 2   /* full while the basis has reorth_blocks blocks, then against
                               those leading blocks and the last two only */
} rbcg_reorth;

/* Per-result report. */
typedef struct {
  int32_t status;          /* rbcg_status of this result */
  int32_t iters;           /* block products in the last Krylov space */
  int32_t matrix_loads;    /* all block products, plus one per FP64 residual evaluation */
  int32_t refine_sweeps;   /* Krylov spaces built */
  int32_t deflated;        /* basis directions dropped as rank-deficient */
  int32_t precision_used;  /* rbcg_dtype used for the block products */
  double relres;           /* ||b - A_mu x|| / ||b|| in FP64 (-1 if not evaluated) */
} rbcg_info;

/* ----------------------------------------------------------------- solvers */

/* Gaussian start block drawn on the device (the Omega of def. BCG, i.i.d.
 * N(0, 1) entries): out[r][c], r < rows, c < cols, row stride ld (device,
 * FP64, caller-owned).  Element e = r cols + c is standard normal number
 * e mod 2 of Philox4x32-10 (Salmon et al., SC 2011) called with counter
 * (lo32(e / 2), hi32(e / 2), stream, 0) and key (lo32(seed), hi32(seed)); a
 * call's words x0..x3 give u1 = ((x0 2^32 + x1) >> 11 + 1/2) 2^-53 and
 * u2 = ((x2 2^32 + x3) >> 11 + 1/2) 2^-53, and the Box-Muller pair
 * sqrt(-2 ln u1) (cos, sin)(2 pi u2).  The solvers use this layout for start
 * blocks passed as NULL.  Blocking; RBCG_ERR_INVALID_ARG for rows < 0,
 * cols < 1, ld < cols or sizes above 2^31 - 1. */
int rbcg_omega_fill(rbcg_ctx* ctx, uint64_t seed, uint32_t stream, int64_t rows, int64_t cols,
                    double* out /*device*/, int64_t ld);

/* Independent systems (A_s + mu_s I) x_s = b_s, s = 0..nsys-1, advanced
 * together (one launch per kernel for all systems).
 *   ops[s]    operator of system s (host array of nsys handles); d_s = its dimension
 *   mu        host[nsys], mu_s >= 0
 *   b         host[nsys] of device pointers to b_s (length d_s, FP64)
 *   omega     host[nsys] of device pointers to Omega_s (k_s x d_s row-major FP64),
 *             or NULL (the array or an entry): Omega_s is drawn on the device
 *             from opts[s].seed, stream s (see rbcg_omega_fill); unused for k_s = 0
 *   k         host[nsys], 0 <= k_s < d_s; block width m_s = k_s + 1
 *   x         host[nsys] of device pointers to x_s (length d_s, FP64), written
 *   opts      host[nsys] options per system
 *   info      host[nsys] reports, written
 * Returns RBCG_OK when every system reached its tolerance (or ran t_max
 * products with rtol = 0), else the first failing status (per-system status
 * is in info). */
int rbcg_solve(rbcg_ctx* ctx, int64_t nsys, const rbcg_op* const* ops, const double* mu,
               const double* const* b, const double* const* omega, const int32_t* k,
               double* const* x, const rbcg_opts* opts, rbcg_info* info);

/* Regularization path: one Krylov space K_t(A, [b Omega]) serves all L
 * shifts (eq. bcg_alg).
 *   b      device, length d (FP64)
 *   omega  device, k x d row-major (FP64), or NULL: drawn on the device from
 *          opts.seed, stream 0 (see rbcg_omega_fill); unused when k = 0
 *   mu     host[L], each >= 0
 *   X      device, L x d row-major (FP64), row l = solution for mu[l]
 *   info   host[L]
 * With opts.matvec low-precision and rtol > 0, each refinement sweep builds
 * a new space on [R Omega] where R holds the FP64 residuals of the shifts not
 * yet at rtol; only those shifts are corrected.  When t_max m >= d (and
 * L <= 144, refine_max > 1), the first space is built out to the whole of
 * R^d instead and the refinement steps reuse it: x_l += Q (T + mu_l I)^{-1}
 * Q^T r_l with the factors of the first solve, one FP64 residual per step;
 * a step that contracts by less than 3x hands over to fresh sweeps.
 * info.refine_sweeps counts spaces and reuse steps.  With the environment
 * variable RBCG_DEBUG set, each sweep prints one line (its Krylov steps and
 * the range of relative residuals) to stderr. */
int rbcg_path(rbcg_ctx* ctx, const rbcg_op* op, const double* b, const double* omega, int32_t k,
              int64_t L, const double* mu, double* X, const rbcg_opts* opts, rbcg_info* info);

/* Nystrom-preconditioned CG, the comparison method of the paper, built from
 * the same Gaussian block Omega (Sec. 2.2.2, eq. nystromBKI_def; def. PCG,
 * Sec. 2.1; theta as in Sec. 7):
 *   1. Q = orthonormal basis of K_s(A, Omega) (s - 1 block products of k
 *      vectors; directions below 1e-14 of a block's largest are dropped),
 *   2. Y = A Q (the s-th product) and the Nystrom approximation
 *      A<K_s> = Y (Q^T Y)^+ Y^T = U^T diag(D) U (U: r orthonormal rows,
 *      r <= s k, eigenvalues below 1e-13 of the largest dropped),
 *   3. theta = the smallest kept D, or `theta` when > 0,
 *   4. preconditioned CG on (A + mu I) x = b from x = 0 with
 *      P^{-1} = (theta + mu) U^T (D + mu I)^{-1} U + (I - U^T U), until the
 *      recursive residual reaches opts.rtol (checked every 4 iterations) or
 *      opts.t_max iterations (rtol = 0: exactly t_max).
 *   op       FP64 products only (opts.matvec = RBCG_F64, else UNSUPPORTED)
 *   b, x     device, length d (FP64); x written
 *   omega    device, k x d row-major (FP64), or NULL: drawn from opts.seed
 *            (stream 0, see rbcg_omega_fill); 1 <= k < d, 1 <= s, s k <= 128
 *   eig_out  host[s k] or NULL: the Nystrom eigenvalues D, descending, 0 for
 *            dropped directions; rank_out, theta_out: host or NULL
 *   info     one report: iters = PCG iterations, matrix_loads = s + iters + 1
 *            (the construction, one single-vector product per iteration, the
 *            final FP64 residual), deflated = s k - rank, relres = FP64
 *            ||b - A_mu x|| / ||b||; status NO_CONVERGENCE when rtol > 0 and
 *            relres misses it, NOT_SPD when a search direction has
 *            p^T A_mu p <= 0. */
int rbcg_nystrom_pcg(rbcg_ctx* ctx, const rbcg_op* op, const double* b, const double* omega, int32_t k,
                     int32_t s, double mu, double theta, double* x, const rbcg_opts* opts, rbcg_info* info,
                     double* eig_out, int32_t* rank_out, double* theta_out);

/* Block-Lanczos square root Y ~ A^{1/2} B (def. blansq).  The m_s samples
 * (rows of B) are split into groups of opts.group; each group's samples form
 * one Krylov start block (every sample is augmented by the others in its
 * group).  All groups share each block product (one pass over A for up to
 * 144 fused vectors; wider products run as column chunks of at most 144, one
 * pass each).  The z-integral uses an
 * opts.nquad-node conformal-map rule on the Ritz-value interval of each
 * group's T_t, evaluated exactly through the Lanczos relation
 * A Q_t = Q_t T_t + Q_{t+1} B_t E_t^T.
 *   B   device, m_s x d row-major (FP64)
 *   Y   device, m_s x d row-major (FP64), written
 *   info host[m_s]; relres holds -1 (no residual is defined)
 * opts.rtol is ignored; exactly opts.t_max products are run.  All groups share
 * one block product, so ceil(m_s / g) * g <= 256 with g = min(opts.group, m_s),
 * else RBCG_ERR_UNSUPPORTED before any device work. */
int rbcg_sqrt_apply(rbcg_ctx* ctx, const rbcg_op* op, int64_t m_s, const double* B, double* Y,
                    const rbcg_opts* opts, rbcg_info* info);

/* Block-Lanczos inverse square root Y ~ A^{-1/2} B (def. blanisq): the same
 * groups, Krylov spaces, Ritz-value interval and quadrature rule as
 * rbcg_sqrt_apply, with the leading A dropped from the integrand:
 * A^{-1/2} = (2/pi) int_0^inf (A + z^2 I)^{-1} dz, so Y = Q_t sum_i w_i
 * (T_t + s_i I)^{-1} Q_t^T B (t blocks of the basis, where the square root
 * uses t + 1).  Arguments, layout, ownership and errors as rbcg_sqrt_apply;
 * RBCG_ERR_NOT_SPD when a shifted block-tridiagonal factorization fails.
 * A must be positive definite: for a singular A the Ritz values approach 0,
 * the quadrature interval's lower end falls to rounding level and the result
 * is not meaningful (the square root has no such restriction). */
int rbcg_invsqrt_apply(rbcg_ctx* ctx, const rbcg_op* op, int64_t m_s, const double* B, double* Y,
                       const rbcg_opts* opts, rbcg_info* info);

/* The block product the solvers use (one matrix-load, Sec. 1.2):
 * W = A X for N vectors (rows of X, N x d row-major FP64, device), written to W
 * (N x d row-major FP64, device).  matvec selects the arithmetic exactly as in
 * rbcg_opts.matvec (F64; F32 for a dense operator with an FP32 copy; BF16 for
 * a Gram operator with BF16 copies, where X and Z X are carried as three BF16
 * parts).  1 <= N <= 256.  Returns after W is complete. */
int rbcg_op_apply(rbcg_ctx* ctx, const rbcg_op* op, int64_t N, const double* X, double* W, int matvec);

/* The same block product as rbcg_op_apply, for callers that cannot allocate device memory
 * (code under HIP graph capture, tight serving loops, harnesses that forbid allocation): it calls
 * no hipMalloc, hipFree, hipHostMalloc or other allocating routine.  Its device buffers (the
 * padded copy of X, the low-precision copy of the block, the split-K partials and the kernel
 * descriptors) are carved from one fixed array of rbcg_noalloc_scratch_bytes() bytes per GPU,
 * which the library holds from the first rbcg_create on that device until the process ends.
 * Arguments, layout, ownership and result as rbcg_op_apply (the operator handle and its
 * low-precision copies must already exist).  A call whose buffers do not fit returns
 * RBCG_ERR_TOO_LARGE before any device work; the FP64 and FP32 dense products fit for
 * N * round_up(d, 64) up to about 600000 (e.g. d = 8192 with N = 65).  Gram operators with BF16
 * products need n-sized staging and fit only for small n.  Every call on a GPU shares that GPU's
 * array and leaves its contents behind (nothing in it is assumed to start at zero): calls that
 * overlap on one GPU (two host threads, or two contexts on different streams) race and must be
 * serialised by the caller.  Returns after W is complete. */
int rbcg_op_apply_noalloc(rbcg_ctx* ctx, const rbcg_op* op, int64_t N, const double* X, double* W, int matvec);

/* Size in bytes of the fixed per-GPU scratch array used by rbcg_op_apply_noalloc (host-only). */
int64_t rbcg_noalloc_scratch_bytes(void);

/* Bytes of device memory currently held by the context's workspace. */
int64_t rbcg_workspace_bytes(const rbcg_ctx* ctx);

/* Measurement hook.  rbcg_profile(ctx, n) with n >= 1 clears the counters and
 * starts timing every n-th block-product GEMM launch (the A X or Z^T (Z X)
 * products that the paper counts as matrix-loads, Sec. 1.2; n = 1: all of
 * them) with a pair of HIP events on the context's stream; each pair adds a
 * marker to the stream, which n > 1 keeps off most launches.  rbcg_profile(ctx,
 * 0) stops; n < 0 is RBCG_ERR_INVALID_ARG.  rbcg_profile_read reports the
 * number of timed launches, their summed GPU time in milliseconds, and their
 * summed algorithmic flops (2 * rows * cols * block width per GEMM) and HBM
 * bytes (one read of the operator per GEMM).  All pointers are host
 * pointers. */
int rbcg_profile(rbcg_ctx* ctx, int enable);
int rbcg_profile_read(const rbcg_ctx* ctx, int64_t* launches, double* ms_total, double* flops_total,
                      double* bytes_total);

/* Host-only, no device needed: the n-node quadrature rule rbcg_sqrt_apply
 * uses for the integral sqrt(l) = (2/pi) int_0^inf l / (l + z^2) dz on
 * spectra inside [lo, hi] (eq. sqrt_rational): the conformal-map rule of
 * Hale, Higham and Trefethen (2008).  Writes shifts[i] = z_i^2 and weights[i]
 * (host arrays of length n) so that sqrt(l) ~ sum_i weights[i] l / (l + shifts[i]).
 * Requires 0 < lo <= hi and n >= 1, else RBCG_ERR_INVALID_ARG. */
int rbcg_sqrt_rule(double lo, double hi, int32_t n, double* shifts, double* weights);

#ifdef __cplusplus
}
#endif
#endif /* RBCG_H */
