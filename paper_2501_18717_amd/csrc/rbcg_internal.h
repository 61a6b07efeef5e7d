// Internal declarations shared by the device kernels (kernels.hip) and the
// host runtime (rbcg.cpp).  Not part of the public ABI.
#pragma once
#include <hip/hip_runtime.h>
#include <cstdint>

namespace rbcg {

// Largest block width a single-workgroup factorization keeps in LDS:
// a 129 x 129 FP64 matrix is 133 KB of the 160 KB per CU.
constexpr int kMaxBlock = 129;

// A set of "rows": vectors stored contiguously, row a at
//   p + (a / rb) * bs + (a % rb) * ld      (elements)
// The two-level form lets several Krylov bases be interleaved block by block.
struct RowOp {
  const void* p;
  int64_t ld;
  int64_t bs;
  int32_t rb;
  int32_t pad_;
};

inline RowOp plain_rows(const void* p, int64_t ld) { return RowOp{p, ld, 0, 0x3fffffff, 0}; }

// C[i][c] = sum_k P[i][k] * X[c][k] for i < M, c < N, k < K.
// Partial sums of split s go to part[(s * M + i) * N + c] (FP64).
struct NtDesc {
  RowOp P;
  RowOp X;
  int32_t M, N, K, active;   // active: index into the active-flag array, -1 = always
  double* part;              // split-K partials (when splits > 1), in output orientation; the FP32
                             // 32x32x2 product stores them as FP32 (its accumulators' precision)
  RowOp O;                   // direct transposed output: row c, element i (when out == null)
  double* out;               // direct row-major output out[i * ldo + c]
  int64_t ldo;
  int32_t out_t, pad_;       // element type of O: DType, or 3 = three BF16 parts (rows 3c, 3c+1, 3c+2)
};

// Reduction of the split-K partials with an epilogue.
enum FinMode : int32_t {
  FIN_ROWMAJOR = 0,   // out[i * ldo + c] = alpha * sum
  FIN_TRANS = 1,      // row c of `O` (a RowOp), element i:  = alpha * sum
  FIN_RESID = 2,      // row c of O, element i: rhs[c][i] - sum - mu[c] * xin[c][i]
  FIN_T2R = 3,        // partials in (c, i) order, out[i * ldo + c] = alpha * sum
  FIN_AXPBY = 4,      // row c of O, element i: beta * rhs[c][i] + alpha * sum
};
struct FinDesc {
  const double* part;
  int32_t M, N, splits, mode;
  double* out;            // FIN_ROWMAJOR target
  int64_t ldo;
  RowOp O;                // FIN_TRANS / FIN_RESID target rows (p is writable)
  RowOp rhs;              // FIN_RESID: right-hand sides
  RowOp xin;              // FIN_RESID: current iterates
  const double* mu;       // FIN_RESID: shift of each row c
  double alpha;
  int32_t active;
  int32_t part_f32;       // partials stored as FP32 (the FP32 32x32x2 product's accumulators)
  double beta;            // FIN_AXPBY
};

// O[b][i] = beta * Y[b][i] + alpha * sum_a C[a][b] * P[a][i]
// for b < Mo, i < N, a < Ka.  O may alias Y.
struct NnDesc {
  RowOp P;
  const double* C;
  int64_t ldc;
  RowOp Y;
  RowOp O;
  double alpha, beta;
  int32_t Ka, Mo, N, active;
  double* part;            // split partials of the tall variant ([s][b][i]) when splits > 1
  RowOp O32;               // k_gemm_nn: FP32 copy of the output rows as well (p == null: none)
  // k_gemm_nn only: also acc_out[e] = acc_a[e] + acc_b[e] for e < acc_n (acc_out == null: none),
  // spread over the launch's threads (the off-band projection coefficients of a Lanczos step)
  const double* acc_a;
  const double* acc_b;
  double* acc_out;
  int64_t acc_n;
};

// Symmetrised diagonal block of T from the two projection passes.
struct DiagDesc {
  const double* C1; const double* C2;  // rows of Q_j^T W from each pass (m x m, ld = ldc)
  int64_t ldc;
  double* D;                           // T diagonal block j (m x m)
  const int32_t* mask;                 // deflated columns of Q_j
  int32_t m, has_c2, active, pad_;
};

// Factorization of a small Gram matrix G = W^T W (m x m) for Cholesky QR
// with rank-revealing pivoting and deflation.
//   Mout[a][s]  : Q = W * Mout  (m x m, zero columns for deflated s)
//   Bout[s][c]  : W = Q * Bout  (m x m, zero rows for deflated s)
//   mask[s]     : 1 if basis column s is deflated
// With prevB != null the reported coefficient is Bout * prevB.
struct QrDesc {
  const double* G;
  int64_t ldg;
  const double* pre;       // pre-projection squared norms (stride pre_stride) or null
  int64_t pre_stride;
  double* Mout;
  double* Bout;
  const double* prevB;
  int32_t* mask;
  int32_t* rank_out;
  int32_t m, pivot, force_first, active;
  double eta2;             // deflation threshold (relative, squared) vs pre-projection norm
  double tau;              // deflation threshold (relative, squared) vs the block's own norm
  double floor2;           // absolute floor on the squared Schur pivot (second pass: columns are
                           // nominally unit, so a pivot below it came from a rounding-dominated
                           // first-pass Schur complement); 0 = none
  DiagDesc dg;             // also form this diagonal block of T (dg.D == null: none)
};


// Shifted block-tridiagonal solve (T_t + sigma I) Y = RHS with RHS nonzero
// only in the first block row.  Blocks: D[j] (diagonal, m x m), Bsub[j]
// (T[j+1][j], m x m), masks per block.  Workspace per block: Lw = S_j^{-1}
// (inverse Schur complement), Xw = U_j = B_j S_j^{-1}, Zw = eliminated
// right-hand side (t + 1 blocks of m x r).
struct TriDesc {
  const double* D;         // t blocks of m*m
  const double* Bsub;      // t blocks of m*m (block j couples j+1 to j)
  const int32_t* mask;     // t*m deflation flags
  const double* rhs;       // m x r (first block of the right-hand side), row stride ld_rhs
  int64_t ld_rhs;
  double* Lw;              // workspace: t blocks of m*m (inverse Schur complements)
  double* Xw;              // workspace: t blocks of m*m (B_j S_j^{-1})
  double* Zw;              // workspace: t+1 blocks of m*r (eliminated right-hand sides)
  double* Y;               // output rows (block j row i at Y[(j*m + i) * ldy + c])
  int64_t ldy;
  double* est;             // residual estimate output (monitor) or null
  int32_t* fail;           // set to 1 on a non-positive pivot
  double sigma;
  int32_t m, r, active;
  int32_t nblk;            // backward sweep: blocks of this descriptor (0: the launch's t)
  // projection coefficients Q_i^T A Q_j of block column j for i < j (the full-reorthogonalisation
  // coefficients of Lanczos step j), used by the refinement step: block column j >= 1 holds j
  // m x m blocks, rows i m .. i m + m - 1 for block i, at Hoff + hoff_offset(j, m); null: band only
  const double* Hoff;
  int32_t refine;          // k_tri_refine: 0 = leave Y as the sweeps left it, 1 = one refinement
                           // step, 2 = apply the stored factors to a right-hand side over all t
                           // blocks (rhs[e * ld_rhs], e < t m), Y = (T + sigma I)^{-1} rhs
  int32_t pad2_;
};

// Offset (elements) of block column j (>= 1) in the coefficient store; hoff_offset(t, m) is the
// size of the store for t blocks.
__host__ __device__ inline int64_t hoff_offset(int j, int m) { return j < 1 ? 0 : (int64_t)m * m * j * (j - 1) / 2; }

// Conversion of rows between precisions (RNE).
enum DType : int32_t { DT_F64 = 0, DT_F32 = 1, DT_BF16 = 2 };
struct CvtDesc {
  RowOp src;  // FP64 or FP32 rows
  RowOp dst;
  int32_t rows, cols, src_t, dst_t;
  int32_t active, split_lo, pad0, pad1;   // split_lo: write three BF16 parts (dst rows 3r, 3r+1, 3r+2)
};

// ---------------------------------------------------------------- launchers
// Each launcher enqueues on `st` for `nz` problems whose descriptors already
// live in device memory.  They return hipSuccess or the launch error.
// dtype: DType or 3 = FP32 P values with FP64 arithmetic; out_t: 0 = row-major (i, c),
// 1 = transposed (row c); xsplit: X rows hold BF16 hi/lo pairs.
hipError_t launch_gemm_nt_ex(int dtype, int out_t, bool xsplit, const NtDesc* d_desc, int nz, int maxM,
                             int maxN, int splits, const int32_t* active, hipStream_t st);
// Gram matrix W^T W of one block per descriptor (P = the block, M = N = m <= 80, K = d), split
// over k into part (splits x m x m, FIN_T2R order).
bool gram_supported(int m);
hipError_t launch_gram(const NtDesc* d_desc, int nz, int maxm, int splits, const int32_t* active, hipStream_t st);
// BF16 products of the Gram operator with the right operand as three BF16 parts (rows 3c, 3c + 1,
// 3c + 2 of X), N <= 144, FP32 MFMA accumulation over `splits` ranges of k, each written as FP32
// partials part[s][c][i] (reduced in FP64 by k_finish with part_f32, or by launch_gram_combine).
hipError_t launch_gram_bf16(const NtDesc* d_desc, int nz, int maxM, int maxN, int splits, const int32_t* active,
                            hipStream_t st);
// Sum of those partials in FP64, stored as three BF16 parts in rows 3c .. 3c + 2 of O.
hipError_t launch_gram_combine(const NtDesc* d_desc, int nz, int maxM, int maxN, int splits, const int32_t* active,
                               hipStream_t st);
// Split count of a BF16 Gram pass over K values of k (about 1024 values per split).
int gram_bf16_splits(int K);
int gram_bf16_rows_per_workgroup();
hipError_t launch_finish(const FinDesc* d_desc, int nz, int maxM, int maxN, const int32_t* active,
                         hipStream_t st, int lanes_per_output = 1);
hipError_t launch_gemm_nn_ex(bool p_f32, const NnDesc* d_desc, int nz, int maxMo, int maxN,
                             const int32_t* active, hipStream_t st);
// uniform: every problem of the launch has block width maxm (enables the exact-width kernels).
hipError_t launch_qr_factor(const QrDesc* d_desc, int nz, int maxm, bool uniform, const int32_t* active,
                            hipStream_t st);
// One lane per column, compiled for an exact block width (m = 9, 17, 33, 65, 129).
bool qr_m_supported(int m);
hipError_t launch_qr_m(const QrDesc* d_desc, int nz, int m, const int32_t* active, hipStream_t st);
hipError_t launch_diag(const DiagDesc* d_desc, int nz, int maxm, const int32_t* active, hipStream_t st);
// Forward sweep for one exact block width m in {9, 17, 33, 65, 129} (every descriptor of the
// launch has that width); hipErrorNotSupported for other widths or when the LDS image does not
// fit, in which case launch_tri_forward serves.
hipError_t launch_tri_exact(const TriDesc* d_desc, int nz, int m, int r, int j0, int j1, const int32_t* active,
                            hipStream_t st);
hipError_t launch_tri_forward(const TriDesc* d_desc, int nz, int maxm, int maxr, int j0, int j1,
                              const int32_t* active, hipStream_t st);
hipError_t launch_tri_backward(const TriDesc* d_desc, int nz, int maxm, int maxr, int t,
                               const int32_t* active, hipStream_t st);
// One step of FP64 refinement of Y (one right-hand side per descriptor) after the forward and
// backward sweeps: R = RHS - (T + sigma I) Y with the band and, where Hoff is set, the off-band
// coefficients; then the stored factors solve for the correction and Y += correction.  With
// refine = 2 the descriptor's right-hand side spans all t blocks and Y = (T + sigma I)^{-1} rhs
// with the stored factors (band T, as the forward sweep factored it).
// hipErrorNotSupported when r > 1 or the t m solution values do not fit in LDS.
hipError_t launch_tri_refine(const TriDesc* d_desc, int nz, int maxm, int maxr, int t, const int32_t* active,
                             hipStream_t st);
// LDS bytes the two sweeps need for block width m and r right-hand sides.
inline size_t tri_forward_lds(int m, int r) { return ((size_t)m * m + 19 * (size_t)m + 2 * (size_t)m * r) * 8; }
inline size_t tri_backward_lds(int m, int r) { return ((size_t)m * m + 2 * (size_t)m * r) * 8; }
constexpr size_t kLdsCap = 160 * 1024 - 4096;
hipError_t launch_convert(const CvtDesc* d_desc, int nz, int maxRows, int maxCols,
                          const int32_t* active, hipStream_t st);
// Column sums of squares: out[z * ldout + r] = sum_i rows[r][i]^2 for r < rows_z.
struct NormDesc { RowOp x; double* out; int32_t rows, n, active, pad_; };
hipError_t launch_sqnorms(const NormDesc* d_desc, int nz, int maxRows, const int32_t* active,
                          hipStream_t st);
// Copy rows (FP64): dst[r][i] = alpha * src[r][i]; zero-fills rows [rows, rows_total).
struct CopyDesc { RowOp src; RowOp dst; double alpha; int32_t rows, rows_total, n, active; };
hipError_t launch_copy(const CopyDesc* d_desc, int nz, int maxRows, int maxN, const int32_t* active,
                       hipStream_t st);

// Refill of deflated start-block columns: the j-th deflated position s (mask[s] != 0, in
// position order) gets src row (src_first + j) when j < src_avail; other rows are untouched.
struct FillDesc { RowOp dst; const int32_t* mask; RowOp src; int32_t src_first, src_avail, m, n, active, pad_; };
hipError_t launch_fill(const FillDesc* d_desc, int nz, int maxN, const int32_t* active, hipStream_t st);

// Nystrom-PCG helpers (nystrom.hip).  Symmetric eigendecomposition of an n x n matrix, n <=
// kEighMax, in one workgroup (cyclic Jacobi): w[i] eigenvalues (unsorted), V[k][i] eigenvectors.
constexpr int kEighMax = 128;
hipError_t launch_sym_eigh(const double* S, int64_t lds_, int n, double* w, double* V, hipStream_t st);
// M[a][i] = V[a][i] / sqrt(w_i) for w_i > cut max w, else 0; mode 1 also writes the kept
// eigenvalues D, theta (smallest kept, unless theta_in > 0), coef_i = (theta + mu)/(D_i + mu) - 1
// and the kept count.
hipError_t launch_nys_factor(const double* w, const double* V, int r, double cut, int mode, double mu,
                             double theta_in, double* M, double* D, double* coef, double* theta_out, int32_t* count,
                             hipStream_t st);
// PCG updates with device scalars sc[0] = r.z, sc[1] = r.r: step A after qneg = -(A + mu I) p,
// scale cw = coef .* w, step B after z = P^{-1} r.
hipError_t launch_pcg_step_a(double* x, double* r, const double* p, const double* qneg, int64_t n, double* sc,
                             int32_t* fail, hipStream_t st);
hipError_t launch_pcg_scale(const double* coef, const double* wv, double* cw, int r, hipStream_t st);
hipError_t launch_pcg_step_b(const double* r, const double* z, double* p, int64_t n, double* sc, int first,
                             hipStream_t st);

// Seeded Gaussian block out[r][c] (rows x cols, row stride ld): Philox4x32-10 counter (lo32, hi32
// of e / 2, stream, 0) with e = r cols + c, key = seed, two 53-bit uniforms per call, Box-Muller.
hipError_t launch_gaussian(double* out, int64_t ld, int rows, int cols, uint64_t seed, uint32_t stream,
                           hipStream_t st);

// dst (cols x ldt) = src^T for a rows x cols FP32 matrix (row-major, leading dimension ld), as
// BF16 or FP32
hipError_t launch_transpose_bf16(const float* src, int64_t ld, int rows, int cols, unsigned short* dst,
                                 int64_t ldt, hipStream_t st);
hipError_t launch_transpose_f32(const float* src, int64_t ld, int rows, int cols, float* dst, int64_t ldt,
                                hipStream_t st);

// Quadrature-node sum and block-tridiagonal product for the square root.
struct WsumDesc { const double* Y; int64_t node_stride; const double* w; int32_t nq, n, r, active; double* out; };
struct TmulDesc { const double* D; const double* Bsub; const double* Y; double* out; int32_t t, m, r, active; };
hipError_t launch_wsum(const WsumDesc* d_desc, int nz, int64_t maxTotal, const int32_t* active, hipStream_t st);
hipError_t launch_tmul(const TmulDesc* d_desc, int nz, int64_t maxTotal, const int32_t* active, hipStream_t st);

// Device-side convergence: clears *active_flag once *est <= tol * *scale, recording the step.
// Convergence test of one problem after step `step`; a converged problem clears its device
// flag and, when host_flag is set, its mirror in pinned host memory (read by the host loop).
struct ConvDesc {
  const double* est; const double* scale; const double* tol; int32_t* active_flag; int32_t* done_at; int32_t step, pad_;
  int32_t* host_flag;
};
hipError_t launch_converge(const ConvDesc* d_desc, int nz, hipStream_t st);

}  // namespace rbcg
