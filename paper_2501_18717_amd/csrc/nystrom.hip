// Small dense steps of the Nystrom-preconditioned CG comparison method (Sec. 2.2.2,
// eq. nystromBKI_def; def. PCG, Sec. 2.1): the eigendecompositions of the r x r matrices that
// turn the block-Krylov Nystrom approximation into its factors, and the PCG vector updates with
// their scalars kept on the device.  The d-long products (A p, U r, U^T w, Q^T Y) run on the
// library's tall block-product kernels; these kernels are one workgroup each.
#include "device_common.inc"

namespace rbcg {

namespace {

// Sum over the workgroup (1024 threads); every thread gets the total.
__device__ double wg_sum(double v, double* red) {
  const int tid = threadIdx.x;
  red[tid] = v;
  __syncthreads();
  for (int off = 512; off > 0; off >>= 1) {
    if (tid < off) red[tid] += red[tid + off];
    __syncthreads();
  }
  const double s = red[0];
  __syncthreads();
  return s;
}

}  // namespace

// Eigendecomposition of a symmetric n x n matrix (n <= kEighMax), cyclic Jacobi with the
// round-robin ordering: each round rotates n/2 disjoint index pairs at once (the 2 x 2 symmetric
// Schur rotation that zeroes A[p][q]: tau = (a_qq - a_pp) / (2 a_pq), t = sign(tau) / (|tau| +
// sqrt(1 + tau^2)), c = 1 / sqrt(1 + t^2), s = t c), first on rows, then on columns and on the
// eigenvector matrix.  The pairs of round r come from the circle method on N = n rounded up to
// even (index N - 1 fixed): (r, N - 1) and ((r + i) mod (N - 1), (r - i) mod (N - 1)) for
// 1 <= i < N / 2; N - 1 rounds meet every pair once (for odd n the pairs with index n idle).
// Sweeps until the off-diagonal part is below 1e-15 of the diagonal in Frobenius norm.  S is read
// as (S + S^T) / 2.  Out: w[i] = eigenvalue i (unsorted), V[k][i] = component k of eigenvector i.
// VL: the eigenvector matrix is accumulated in LDS (when 2 n^2 doubles fit) and written out once.
template <bool VL>
__global__ __launch_bounds__(1024) void k_sym_eigh(const double* __restrict__ S, int64_t lds_, int n,
                                                   double* __restrict__ Vout, double* __restrict__ w, int max_sweeps) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  double* A = (double*)smem_raw;                    // n x n
  double* red = A + (size_t)n * n;                  // 1024
  double* V = VL ? red + 1024 + 2 * (kEighMax / 2 + 1) + kEighMax + 2 : Vout;   // n x n (LDS or global)
  double* cs = red + 1024;                          // pairs
  double* sn = cs + kEighMax / 2 + 1;
  int* pp = (int*)(sn + kEighMax / 2 + 1);
  int* qq = pp + kEighMax / 2 + 1;   // ints: 2 (kEighMax / 2 + 1) <= (kEighMax + 2) doubles of room
  const int tid = threadIdx.x;
  const int npad = n + (n & 1);
  const int npairs = npad / 2;
  for (int e = tid; e < n * n; e += 1024) {
    const int i = e / n, j = e - i * n;
    A[e] = 0.5 * (S[(int64_t)i * lds_ + j] + S[(int64_t)j * lds_ + i]);
    V[e] = i == j ? 1.0 : 0.0;
  }
  __syncthreads();
  for (int sweep = 0; sweep < max_sweeps; ++sweep) {
    double off = 0.0, dia = 0.0;
    for (int e = tid; e < n * n; e += 1024) {
      const int i = e / n, j = e - i * n;
      const double a2 = A[e] * A[e];
      if (i == j) dia += a2;
      else off += a2;
    }
    off = wg_sum(off, red);
    dia = wg_sum(dia, red);
    if (!(off > 1e-30 * dia)) break;
    for (int round = 0; round < npad - 1; ++round) {
      if (tid < npairs) {
        const int L = npad - 1;
        const int p = tid == 0 ? round : (round + tid) % L;
        const int q = tid == 0 ? L : (round - tid + L) % L;
        double c = 1.0, s = 0.0;
        if (p < n && q < n) {
          const double apq = A[p * n + q];
          if (apq != 0.0) {
            const double tau = (A[q * n + q] - A[p * n + p]) / (2.0 * apq);
            const double t = (tau >= 0.0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1.0 + tau * tau));
            c = 1.0 / sqrt(1.0 + t * t);
            s = t * c;
          }
        }
        cs[tid] = c;
        sn[tid] = s;
        pp[tid] = p;
        qq[tid] = q;
      }
      __syncthreads();
      // rows: A <- J^T A
      for (int e = tid; e < npairs * n; e += 1024) {
        const int i = e / n, k = e - i * n;
        const int p = pp[i], q = qq[i];
        if (p >= n || q >= n) continue;
        const double c = cs[i], s = sn[i];
        const double ap = A[p * n + k], aq = A[q * n + k];
        A[p * n + k] = c * ap - s * aq;
        A[q * n + k] = s * ap + c * aq;
      }
      __syncthreads();
      // columns: A <- A J, V <- V J (consecutive threads take different pairs of one row); the
      // thread's eigenvector elements are all loaded before any is updated, so their global loads
      // are in flight together
      {
        constexpr int QM = (kEighMax / 2 * kEighMax + 1023) / 1024;
        double vpv[QM], vqv[QM];
#pragma unroll
        for (int qi = 0; qi < QM; ++qi) {
          const int e = tid + 1024 * qi;
          vpv[qi] = 0.0;
          vqv[qi] = 0.0;
          if (e < npairs * n) {
            const int k = e / npairs, i = e - k * npairs;
            const int p = pp[i], q = qq[i];
            if (p < n && q < n) {
              vpv[qi] = V[(int64_t)k * n + p];
              vqv[qi] = V[(int64_t)k * n + q];
            }
          }
        }
#pragma unroll
        for (int qi = 0; qi < QM; ++qi) {
          const int e = tid + 1024 * qi;
          if (e >= npairs * n) continue;
          const int k = e / npairs, i = e - k * npairs;
          const int p = pp[i], q = qq[i];
          if (p >= n || q >= n) continue;
          const double c = cs[i], s = sn[i];
          const double ap = A[k * n + p], aq = A[k * n + q];
          A[k * n + p] = c * ap - s * aq;
          A[k * n + q] = s * ap + c * aq;
          V[(int64_t)k * n + p] = c * vpv[qi] - s * vqv[qi];
          V[(int64_t)k * n + q] = s * vpv[qi] + c * vqv[qi];
        }
      }
      __syncthreads();
    }
  }
  for (int i = tid; i < n; i += 1024) w[i] = A[i * n + i];
  if constexpr (VL)
    for (int e = tid; e < n * n; e += 1024) Vout[e] = V[e];
}

size_t sym_eigh_lds(int n, bool vl) {
  return ((size_t)n * n + 1024 + 2 * (kEighMax / 2 + 1) + kEighMax + 2 + (vl ? (size_t)n * n : 0)) * 8;
}

hipError_t launch_sym_eigh(const double* S, int64_t lds_, int n, double* w, double* V, hipStream_t st) {
  if (n < 1 || n > kEighMax) return hipErrorInvalidValue;
  const bool vl = sym_eigh_lds(n, true) <= kLdsCap;
  const size_t lds = sym_eigh_lds(n, vl);
  if (lds > kLdsCap) return hipErrorInvalidValue;
  static const hipError_t attr0 =
      hipFuncSetAttribute((const void*)k_sym_eigh<false>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)kLdsCap);
  static const hipError_t attr1 =
      hipFuncSetAttribute((const void*)k_sym_eigh<true>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)kLdsCap);
  if (attr0 != hipSuccess) return attr0;
  if (attr1 != hipSuccess) return attr1;
  if (vl)
    hipLaunchKernelGGL(k_sym_eigh<true>, dim3(1), dim3(1024), lds, st, S, lds_, n, V, w, 30);
  else
    hipLaunchKernelGGL(k_sym_eigh<false>, dim3(1), dim3(1024), lds, st, S, lds_, n, V, w, 30);
  return hipGetLastError();
}

// Factors from an eigendecomposition (w, V) of an r x r positive semi-definite matrix: eigenvalue
// i is kept when w_i > cut * max_j w_j; M[a][i] = V[a][i] / sqrt(w_i) for kept i, else 0.
// mode 1 (the Nystrom eigenvalues D = w): D_i = w_i for kept i, else 0; theta = the smallest
// kept w_i unless theta_in > 0; coef_i = (theta + mu) / (D_i + mu) - 1 for kept i, else 0 (the
// preconditioner P_mu^{-1} = I + U^T diag(coef) U); count = number kept.
__global__ __launch_bounds__(1024) void k_nys_factor(const double* __restrict__ w, const double* __restrict__ V,
                                                     int r, double cut, int mode, double mu, double theta_in,
                                                     double* __restrict__ M, double* __restrict__ D,
                                                     double* __restrict__ coef, double* __restrict__ theta_out,
                                                     int32_t* __restrict__ count) {
  __shared__ double red[1024];
  const int tid = threadIdx.x;
  double mx = -1e300;
  for (int i = tid; i < r; i += 1024) mx = fmax(mx, w[i]);
  red[tid] = mx;
  __syncthreads();
  for (int off = 512; off > 0; off >>= 1) {
    if (tid < off) red[tid] = fmax(red[tid], red[tid + off]);
    __syncthreads();
  }
  const double wmax = red[0];
  __syncthreads();
  const double thr = wmax > 0.0 ? cut * wmax : 1e300;
  double mn = 1e300;
  for (int i = tid; i < r; i += 1024)
    if (w[i] > thr) mn = fmin(mn, w[i]);
  red[tid] = mn;
  __syncthreads();
  for (int off = 512; off > 0; off >>= 1) {
    if (tid < off) red[tid] = fmin(red[tid], red[tid + off]);
    __syncthreads();
  }
  const double wmin = red[0];
  __syncthreads();
  const double theta = theta_in > 0.0 ? theta_in : wmin;
  for (int e = tid; e < r * r; e += 1024) {
    const int a = e / r, i = e - a * r;
    M[e] = w[i] > thr ? V[e] / sqrt(w[i]) : 0.0;
  }
  if (mode == 1) {
    for (int i = tid; i < r; i += 1024) {
      const bool keep = w[i] > thr;
      D[i] = keep ? w[i] : 0.0;
      coef[i] = keep ? (theta + mu) / (w[i] + mu) - 1.0 : 0.0;
    }
    int cnt = 0;
    for (int i = tid; i < r; i += 1024) cnt += w[i] > thr ? 1 : 0;
    red[tid] = (double)cnt;
    __syncthreads();
    for (int off = 512; off > 0; off >>= 1) {
      if (tid < off) red[tid] += red[tid + off];
      __syncthreads();
    }
    if (tid == 0) {
      *count = (int32_t)red[0];
      *theta_out = theta;
    }
  }
}

hipError_t launch_nys_factor(const double* w, const double* V, int r, double cut, int mode, double mu,
                             double theta_in, double* M, double* D, double* coef, double* theta_out, int32_t* count,
                             hipStream_t st) {
  hipLaunchKernelGGL(k_nys_factor, dim3(1), dim3(1024), 0, st, w, V, r, cut, mode, mu, theta_in, M, D, coef,
                     theta_out, count);
  return hipGetLastError();
}

// PCG scalars on the device: sc[0] = r.z, sc[1] = r.r (after the last update).
// Step A (after q_neg = -(A + mu I) p):  alpha = (r.z) / (p.q);  x += alpha p;  r -= alpha q;
// sc[1] = r.r.  A non-positive p.q (A_mu not positive definite in floating point) sets *fail.
__global__ __launch_bounds__(1024) void k_pcg_step_a(double* __restrict__ x, double* __restrict__ r,
                                                     const double* __restrict__ p, const double* __restrict__ qneg,
                                                     int64_t n, double* __restrict__ sc, int32_t* __restrict__ fail) {
  __shared__ double red[1024];
  const int tid = threadIdx.x;
  double pq = 0.0;
  for (int64_t i = tid; i < n; i += 1024) pq -= p[i] * qneg[i];
  pq = wg_sum(pq, red);
  const double rz = sc[0];
  const bool ok = pq > 0.0 && rz >= 0.0;
  const double alpha = ok ? rz / pq : 0.0;
  double rr = 0.0;
  for (int64_t i = tid; i < n; i += 1024) {
    x[i] += alpha * p[i];
    const double ri = r[i] + alpha * qneg[i];
    r[i] = ri;
    rr += ri * ri;
  }
  rr = wg_sum(rr, red);
  if (tid == 0) {
    sc[1] = rr;
    if (!ok && fail) *fail = 1;
  }
}

// cw = coef .* w (the preconditioner's diagonal on the r Nystrom coordinates of the residual)
__global__ __launch_bounds__(256) void k_pcg_scale(const double* __restrict__ coef, const double* __restrict__ wv,
                                                   double* __restrict__ cw, int r) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i < r) cw[i] = coef[i] * wv[i];
}

// Step B (after z = P^{-1} r):  beta = (r.z)_new / (r.z)_old;  p = z + beta p  (first = true:
// p = z);  sc[0] = (r.z)_new.
__global__ __launch_bounds__(1024) void k_pcg_step_b(const double* __restrict__ r, const double* __restrict__ z,
                                                     double* __restrict__ p, int64_t n, double* __restrict__ sc,
                                                     int first) {
  __shared__ double red[1024];
  const int tid = threadIdx.x;
  double rz = 0.0;
  for (int64_t i = tid; i < n; i += 1024) rz += r[i] * z[i];
  rz = wg_sum(rz, red);
  const double beta = first ? 0.0 : (sc[0] != 0.0 ? rz / sc[0] : 0.0);
  for (int64_t i = tid; i < n; i += 1024) p[i] = z[i] + beta * p[i];
  if (tid == 0) sc[0] = rz;
}

hipError_t launch_pcg_step_a(double* x, double* r, const double* p, const double* qneg, int64_t n, double* sc,
                             int32_t* fail, hipStream_t st) {
  hipLaunchKernelGGL(k_pcg_step_a, dim3(1), dim3(1024), 0, st, x, r, p, qneg, n, sc, fail);
  return hipGetLastError();
}

hipError_t launch_pcg_scale(const double* coef, const double* wv, double* cw, int r, hipStream_t st) {
  hipLaunchKernelGGL(k_pcg_scale, dim3((r + 255) / 256), dim3(256), 0, st, coef, wv, cw, r);
  return hipGetLastError();
}

hipError_t launch_pcg_step_b(const double* r, const double* z, double* p, int64_t n, double* sc, int first,
                             hipStream_t st) {
  hipLaunchKernelGGL(k_pcg_step_b, dim3(1), dim3(1024), 0, st, r, z, p, n, sc, first);
  return hipGetLastError();
}

}  // namespace rbcg
