// Device kernels of the randomized block-CG library (gfx950 / CDNA4), except the MFMA "NT"
// products which live in gemm_nt_*.hip (see device_common.inc for the shared template).
//
// Every kernel is batched: blockIdx.z selects a problem descriptor, so one launch serves many
// systems, shifts, quadrature nodes or sample groups.  A problem whose `active` flag is cleared
// on the device returns at once.  The small dense work (Cholesky QR of a block, shifted
// block-tridiagonal solves) runs in one workgroup per problem with the block held in LDS.
#include "device_common.inc"

namespace rbcg {

hipError_t nt_f64_o1(int, const NtDesc*, int, int, int, const int32_t*, hipStream_t);
hipError_t nt_f64_o0(int, const NtDesc*, int, int, int, const int32_t*, hipStream_t);
hipError_t nt_f32_o1(int, const NtDesc*, int, int, int, const int32_t*, hipStream_t);
hipError_t nt_f32_o0(int, const NtDesc*, int, int, int, const int32_t*, hipStream_t);
hipError_t nt_f32f64_o1(int, const NtDesc*, int, int, int, const int32_t*, hipStream_t);
hipError_t nt_f32f64_o0(int, const NtDesc*, int, int, int, const int32_t*, hipStream_t);
hipError_t nt_bf16_o1_split(int, const NtDesc*, int, int, int, const int32_t*, hipStream_t);
hipError_t nt_bf16_o1(int, const NtDesc*, int, int, int, const int32_t*, hipStream_t);
hipError_t nt_bf16_o0(int, const NtDesc*, int, int, int, const int32_t*, hipStream_t);

hipError_t launch_gemm_nt_ex(int dtype, int out_t, bool xsplit, const NtDesc* dd, int nz, int maxM, int maxN,
                             int splits, const int32_t* act, hipStream_t st) {
  const int tn = (maxN + 15) / 16;
  if (tn < 1 || tn > 16 || splits < 1) return hipErrorInvalidValue;
  switch (dtype) {
    case DT_F64: return out_t ? nt_f64_o1(tn, dd, nz, maxM, splits, act, st) : nt_f64_o0(tn, dd, nz, maxM, splits, act, st);
    case DT_F32: return out_t ? nt_f32_o1(tn, dd, nz, maxM, splits, act, st) : nt_f32_o0(tn, dd, nz, maxM, splits, act, st);
    case DT_F32F64:
      return out_t ? nt_f32f64_o1(tn, dd, nz, maxM, splits, act, st) : nt_f32f64_o0(tn, dd, nz, maxM, splits, act, st);
    case DT_BF16:
      if (xsplit) return nt_bf16_o1_split(tn, dd, nz, maxM, splits, act, st);
      return out_t ? nt_bf16_o1(tn, dd, nz, maxM, splits, act, st) : nt_bf16_o0(tn, dd, nz, maxM, splits, act, st);
    default: return hipErrorInvalidValue;
  }
}

// Allow the largest dynamic LDS the kernel can take next to its static __shared__ data.
static hipError_t set_big_lds(const void* k) {
  hipFuncAttributes fa;
  hipError_t e = hipFuncGetAttributes(&fa, k);
  if (e != hipSuccess) return e;
  const int dyn = 160 * 1024 - (int)fa.sharedSizeBytes;
  return hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, dyn);
}

// ---------------------------------------------------------------------------------------------
// Split-K reduction and epilogues.  Partials are in output orientation:
//   FIN_ROWMAJOR: part[s][i][c] -> out[i*ldo + c]
//   FIN_TRANS / FIN_RESID: part[s][c][i] -> row c of O, element i
// ---------------------------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_finish(const FinDesc* __restrict__ descs, const int32_t* __restrict__ act) {
  const FinDesc f = descs[blockIdx.z];
  if (!is_active(act, f.active)) return;
  const bool rowmajor = f.mode == FIN_ROWMAJOR;
  const int rows = rowmajor ? f.M : f.N;   // outer index of the partial layout
  const int cols = rowmajor ? f.N : f.M;
  const int64_t total = (int64_t)rows * cols;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += stride) {
    const int o = (int)(e / cols), in = (int)(e % cols);
    double v = 0.0;
    for (int s = 0; s < f.splits; ++s) v += f.part[(int64_t)s * total + e];
    v *= f.alpha;
    if (rowmajor) {
      f.out[(int64_t)o * f.ldo + in] = v;
    } else if (f.mode == FIN_TRANS) {
      ((double*)f.O.p)[row_off(f.O, o) + in] = v;
    } else {
      const double rv = ((const double*)f.rhs.p)[row_off(f.rhs, o) + in];
      const double xv = ((const double*)f.xin.p)[row_off(f.xin, o) + in];
      ((double*)f.O.p)[row_off(f.O, o) + in] = rv - v - f.mu[o] * xv;
    }
  }
}

hipError_t launch_finish(const FinDesc* dd, int nz, int maxM, int maxN, const int32_t* act, hipStream_t st) {
  const int64_t tot = (int64_t)maxM * maxN;
  int blocks = (int)std::min<int64_t>((tot + 255) / 256, 2048);
  if (blocks < 1) blocks = 1;
  hipLaunchKernelGGL(k_finish, dim3(blocks, 1, nz), dim3(256), 0, st, dd, act);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------------------------
// GEMM "NN" update: O[b][i] = beta * Y[b][i] + alpha * sum_a C[a][b] P[a][i]
//   One workgroup = 16 columns i, all Mo rows b (TB tiles), the 4 waves split the a range.
//   MFMA A operand = C^T (b x a), B operand = P (a x i); D rows = b, columns = i.
// ---------------------------------------------------------------------------------------------
template <typename PT, int TB>
__global__ __launch_bounds__(256) void k_gemm_nn(const NnDesc* __restrict__ descs, const int32_t* __restrict__ act) {
  const NnDesc d = descs[blockIdx.z];
  if (!is_active(act, d.active)) return;
  const int i0 = blockIdx.x * 16;
  if (i0 >= d.N) return;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int q = lane >> 4, r16 = lane & 15;
  const int i = i0 + r16;
  const bool ival = i < d.N;
  v4d acc[TB];
#pragma unroll
  for (int tb = 0; tb < TB; ++tb) acc[tb] = v4d{0, 0, 0, 0};
  // wave w takes a-chunks of 16 starting at 16 w, stepping 64
  for (int ac = 16 * wave; ac < d.Ka; ac += 64) {
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int a = ac + 4 * e + q;
      const bool aval = a < d.Ka;
      const double pv = (aval && ival) ? (double)((const PT*)d.P.p)[row_off(d.P, a) + i] : 0.0;
#pragma unroll
      for (int tb = 0; tb < TB; ++tb) {
        const int b = 16 * tb + r16;
        const double cv = (aval && b < d.Mo) ? d.C[(int64_t)a * d.ldc + b] : 0.0;
        acc[tb] = __builtin_amdgcn_mfma_f64_16x16x4f64(cv, pv, acc[tb], 0, 0, 0);
      }
    }
  }
  extern __shared__ __align__(16) unsigned char smem_raw[];
  double* red = (double*)smem_raw;   // [3][TB][4][64]
  if (wave > 0) {
#pragma unroll
    for (int tb = 0; tb < TB; ++tb)
#pragma unroll
      for (int r = 0; r < 4; ++r) red[(((wave - 1) * TB + tb) * 4 + r) * 64 + lane] = acc[tb][r];
  }
  __syncthreads();
  if (wave != 0 || !ival) return;
#pragma unroll
  for (int tb = 0; tb < TB; ++tb) {
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int b = 16 * tb + (lane >> 4) + 4 * r;
      if (b >= d.Mo) continue;
      double v = acc[tb][r];
#pragma unroll
      for (int w = 0; w < 3; ++w) v += red[((w * TB + tb) * 4 + r) * 64 + lane];
      double out = d.alpha * v;
      if (d.beta != 0.0) out += d.beta * ((const double*)d.Y.p)[row_off(d.Y, b) + i];
      ((double*)d.O.p)[row_off(d.O, b) + i] = out;
    }
  }
}

template <typename PT, int TB>
static hipError_t launch_nn_t(const NnDesc* dd, int nz, int maxN, const int32_t* act, hipStream_t st) {
  const size_t lds = (size_t)3 * TB * 4 * 64 * 8;
  auto kern = k_gemm_nn<PT, TB>;
  static bool attr_set = false;
  if (!attr_set && lds > 64 * 1024) {
    hipError_t e = hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
  }
  attr_set = true;
  hipLaunchKernelGGL(kern, dim3((maxN + 15) / 16, 1, nz), dim3(256), lds, st, dd, act);
  return hipGetLastError();
}

template <typename PT>
static hipError_t dispatch_tb(int tb, const NnDesc* dd, int nz, int maxN, const int32_t* act, hipStream_t st) {
  switch (tb) {
    case 1: return launch_nn_t<PT, 1>(dd, nz, maxN, act, st);
    case 2: return launch_nn_t<PT, 2>(dd, nz, maxN, act, st);
    case 3: return launch_nn_t<PT, 3>(dd, nz, maxN, act, st);
    case 4: return launch_nn_t<PT, 4>(dd, nz, maxN, act, st);
    case 5: return launch_nn_t<PT, 5>(dd, nz, maxN, act, st);
    case 6: return launch_nn_t<PT, 6>(dd, nz, maxN, act, st);
    case 7: case 8: return launch_nn_t<PT, 8>(dd, nz, maxN, act, st);
    case 9: return launch_nn_t<PT, 9>(dd, nz, maxN, act, st);
    case 10: case 11: case 12: return launch_nn_t<PT, 12>(dd, nz, maxN, act, st);
    case 13: case 14: case 15: case 16: return launch_nn_t<PT, 16>(dd, nz, maxN, act, st);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_gemm_nn_ex(bool p_f32, const NnDesc* dd, int nz, int maxMo, int maxN, const int32_t* act,
                             hipStream_t st) {
  const int tb = (maxMo + 15) / 16;
  if (tb < 1 || tb > 16) return hipErrorInvalidValue;
  return p_f32 ? dispatch_tb<float>(tb, dd, nz, maxN, act, st) : dispatch_tb<double>(tb, dd, nz, maxN, act, st);
}

// ---------------------------------------------------------------------------------------------
// Cholesky QR factor of a small Gram matrix with rank-revealing pivoting (one workgroup per
// problem).  See QrDesc.  The pivot at each step is the column with the largest remaining
// Schur-complement diagonal relative to its own squared norm, so the factor is rank revealing;
// a column is deflated when that ratio falls below tau, or its remaining norm falls below
// sqrt(eta2) of its norm before the projections against the basis.
// ---------------------------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_qr_factor(const QrDesc* __restrict__ descs, const int32_t* __restrict__ act) {
  const QrDesc d = descs[blockIdx.z];
  if (!is_active(act, d.active)) return;
  const int m = d.m;
  const int tid = threadIdx.x;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  double* S = (double*)smem_raw;             // m*m: Schur complement; row perm[s] becomes R row s
  double* row = S + m * m;                   // m
  double* dref = row + m;                    // m
  double* pre = dref + m;                    // m
  double* redv = pre + m;                    // 256
  int* redi = (int*)(redv + 256);            // 256
  int* perm = redi + 256;                    // m: pivot position s -> column of W
  int* chosen = perm + m;                    // m: per column of W
  int* kept = chosen + m;                    // m: per pivot position, 1 = basis vector kept
  __shared__ int s_p, s_rank;

  for (int e = tid; e < m * m; e += 256) S[e] = d.G[(int64_t)(e / m) * d.ldg + (e % m)];
  __syncthreads();
  for (int e = tid; e < m; e += 256) {
    dref[e] = S[e * m + e];
    pre[e] = d.pre ? d.pre[(int64_t)e * d.pre_stride] : -1.0;
    chosen[e] = 0;
    kept[e] = 0;
    perm[e] = e;
  }
  if (tid == 0) s_rank = 0;
  __syncthreads();

  for (int s = 0; s < m; ++s) {
    // ---- choose the pivot column
    if (d.pivot && !(d.force_first && s == 0)) {
      double best = -2.0;
      int bi = m;
      for (int c = tid; c < m; c += 256) {
        if (chosen[c]) continue;
        const double rel = dref[c] > 0.0 ? S[c * m + c] / dref[c] : -1.0;
        if (rel > best || (rel == best && c < bi)) { best = rel; bi = c; }
      }
      redv[tid] = best;
      redi[tid] = bi;
      __syncthreads();
      for (int off = 128; off > 0; off >>= 1) {
        if (tid < off) {
          const double ov = redv[tid + off];
          const int oi = redi[tid + off];
          if (ov > redv[tid] || (ov == redv[tid] && oi < redi[tid])) { redv[tid] = ov; redi[tid] = oi; }
        }
        __syncthreads();
      }
      if (tid == 0) s_p = redi[0];
    } else if (tid == 0) {
      s_p = s;
    }
    __syncthreads();
    const int p = s_p;
    const double piv2 = S[p * m + p];
    bool defl;
    if (d.force_first && s == 0) defl = !(piv2 > 0.0);
    else defl = !(dref[p] > 0.0) || !(piv2 > d.tau * dref[p]) || (pre[p] >= 0.0 && !(piv2 > d.eta2 * pre[p]));
    if (defl && d.pivot) {
      // every remaining column is at least as deficient: list them in index order and stop
      __syncthreads();
      if (tid == 0) {
        int pos = s;
        for (int c = 0; c < m; ++c)
          if (!chosen[c]) { perm[pos++] = c; chosen[c] = 1; }
      }
      __syncthreads();
      break;
    }
    if (defl) {
      __syncthreads();
      if (tid == 0) { perm[s] = p; chosen[p] = 1; }
      __syncthreads();
      continue;
    }
    const double rp = sqrt(piv2);
    for (int c = tid; c < m; c += 256) {
      double v = 0.0;
      if (c == p) v = rp;
      else if (!chosen[c]) v = S[p * m + c] / rp;
      row[c] = v;
    }
    __syncthreads();
    // row p of S is retired: it now stores R row s
    for (int c = tid; c < m; c += 256) S[p * m + c] = row[c];
    if (tid == 0) { perm[s] = p; chosen[p] = 1; kept[s] = 1; s_rank = s_rank + 1; }
    __syncthreads();
    // Schur complement update of the remaining columns
    for (int e = tid; e < m * m; e += 256) {
      const int a = e / m, c = e % m;
      if (chosen[a] || chosen[c]) continue;
      S[e] -= row[a] * row[c];
    }
    __syncthreads();
  }
  __syncthreads();
  // ---- reported coefficient block: Bout[s][c] = R[s][c] (times prevB when given)
  for (int e = tid; e < m * m; e += 256) {
    const int s = e / m, c = e % m;
    double v = 0.0;
    if (kept[s]) {
      const double* Rs = S + perm[s] * m;
      if (d.prevB) {
        for (int u = 0; u < m; ++u) v += Rs[u] * d.prevB[u * m + c];
      } else {
        v = Rs[c];
      }
    }
    d.Bout[e] = v;
  }
  for (int e = tid; e < m; e += 256) d.mask[e] = kept[e] ? 0 : 1;
  if (tid == 0 && d.rank_out) *d.rank_out = s_rank;
  __syncthreads();
  int* iperm = chosen;   // no longer needed: reuse as the inverse permutation
  for (int s = tid; s < m; s += 256) iperm[perm[s]] = s;
  __syncthreads();
  // ---- X = Rhat^{-1}, Rhat[s][u] = R[s][perm[u]] upper triangular over kept positions.
  //      Row s of X overwrites row perm[s] of S (rows u > s already hold X, rows < s hold R):
  //      X[s][c] stored at S[perm[s]][perm[c]].
  for (int s = m - 1; s >= 0; --s) {
    if (!kept[s]) continue;   // uniform (LDS)
    const int ps = perm[s];
    for (int u = tid; u < m; u += 256) row[u] = kept[u] ? S[ps * m + perm[u]] : 0.0;
    __syncthreads();
    const double rss = row[s];
    for (int c = tid; c < m; c += 256) {
      double v = 0.0;
      if (c >= s && kept[c]) {
        double acc = (c == s) ? 1.0 : 0.0;
        for (int u = s + 1; u <= c; ++u)
          if (kept[u]) acc -= row[u] * S[perm[u] * m + perm[c]];
        v = acc / rss;
      }
      S[ps * m + perm[c]] = v;
    }
    __syncthreads();
  }
  // ---- Mout[perm[s']][s] = X[s'][s]: Q column s = sum_s' W column perm[s'] * X[s'][s]
  for (int e = tid; e < m * m; e += 256) {
    const int a = e / m, s = e % m;   // a = column of W
    const int sp = iperm[a];
    double v = 0.0;
    if (kept[sp] && kept[s] && sp <= s) v = S[a * m + perm[s]];
    d.Mout[e] = v;
  }
}

hipError_t launch_qr_factor(const QrDesc* dd, int nz, int maxm, const int32_t* act, hipStream_t st) {
  const size_t lds = (size_t)maxm * maxm * 8 + (size_t)maxm * 3 * 8 + 256 * 8 + 256 * 4 + (size_t)maxm * 3 * 4 + 64;
  static bool attr_set = false;
  if (!attr_set) {
    hipError_t e = set_big_lds((const void*)k_qr_factor);
    if (e != hipSuccess) return e;
    attr_set = true;
  }
  if (lds > kLdsCap) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_qr_factor, dim3(1, 1, nz), dim3(256), lds, st, dd, act);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------------------------
// Diagonal block of T: D = sym(C1 + C2); deflated columns become decoupled unit rows.
// ---------------------------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_diag(const DiagDesc* __restrict__ descs, const int32_t* __restrict__ act) {
  const DiagDesc d = descs[blockIdx.z];
  if (!is_active(act, d.active)) return;
  const int m = d.m;
  for (int e = threadIdx.x; e < m * m; e += 256) {
    const int a = e / m, b = e % m;
    double v = d.C1[(int64_t)a * d.ldc + b] + d.C1[(int64_t)b * d.ldc + a];
    if (d.has_c2) v += d.C2[(int64_t)a * d.ldc + b] + d.C2[(int64_t)b * d.ldc + a];
    v *= 0.5;
    if (d.mask && (d.mask[a] || d.mask[b])) v = (a == b) ? 1.0 : 0.0;
    d.D[e] = v;
  }
}

hipError_t launch_diag(const DiagDesc* dd, int nz, int maxm, const int32_t* act, hipStream_t st) {
  (void)maxm;
  hipLaunchKernelGGL(k_diag, dim3(1, 1, nz), dim3(256), 0, st, dd, act);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------------------------
// Shifted block-tridiagonal solve, one workgroup per (shift, system).
// Forward sweep over blocks j in [j0, j1):
//   S_j = D_j + sigma I - V_{j-1}^T V_{j-1},  L_j L_j^T = S_j,
//   z_j = L_j^{-1} (rhs_j - V_{j-1}^T z_{j-1}),  V_j = L_j^{-1} B_j^T
// (B_j = T[j+1][j]; V_j^T = L_{j+1,j}), and optionally the residual estimate
// || B_j y_j || = || V_j^T z_j || of the truncated solve (y_j = last block of the solution).
// Backward sweep: y_j = L_j^{-T} (z_j - V_j y_{j+1}).
// LDS: S (m*m) + panel (16*m) + z (m*r).
// ---------------------------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_tri_forward(const TriDesc* __restrict__ descs, int j0, int j1,
                                                     const int32_t* __restrict__ act) {
  const TriDesc d = descs[blockIdx.z];
  if (!is_active(act, d.active)) return;
  const int m = d.m, r = d.r, tid = threadIdx.x;
  const int64_t mm = (int64_t)m * m;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  double* S = (double*)smem_raw;      // m*m
  double* pan = S + mm;               // 16*m
  double* zb = pan + 16 * m;          // m*r
  __shared__ int s_fail;
  __shared__ double s_red[256];
  if (tid == 0) s_fail = 0;
  for (int j = j0; j < j1; ++j) {
    const double* Dj = d.D + j * mm;
    const int32_t* mk = d.mask + (int64_t)j * m;
    for (int e = tid; e < mm; e += 256) {
      const int a = (int)(e / m), b = (int)(e % m);
      double v = Dj[e];
      if (mk[a] || mk[b]) v = (a == b) ? 1.0 : 0.0;
      else if (a == b) v += d.sigma;
      S[e] = v;
    }
    __syncthreads();
    if (j > 0) {
      // S -= V_{j-1}^T V_{j-1}, V rows staged 16 at a time
      const double* V = d.Xw + (j - 1) * mm;
      for (int p0 = 0; p0 < m; p0 += 16) {
        const int np = min(16, m - p0);
        for (int e = tid; e < np * m; e += 256) pan[e] = V[(int64_t)p0 * m + e];
        __syncthreads();
        for (int e = tid; e < mm; e += 256) {
          const int a = (int)(e / m), b = (int)(e % m);
          if (b > a) continue;
          double acc = 0.0;
          for (int u = 0; u < np; ++u) acc += pan[u * m + a] * pan[u * m + b];
          S[e] -= acc;
        }
        __syncthreads();
      }
      for (int e = tid; e < mm; e += 256) {
        const int a = (int)(e / m), b = (int)(e % m);
        if (b > a) S[e] = S[(int64_t)b * m + a];
      }
      __syncthreads();
    }
    // Cholesky (lower) in place
    for (int s = 0; s < m; ++s) {
      const double piv = S[s * m + s];
      if (!(piv > 0.0)) {
        if (tid == 0) s_fail = 1;
      }
      const double ls = sqrt(piv > 0.0 ? piv : 1.0);
      __syncthreads();
      for (int i = s + 1 + tid; i < m; i += 256) S[i * m + s] /= ls;
      if (tid == 0) S[s * m + s] = ls;
      __syncthreads();
      const int rem = m - s - 1;
      for (int e = tid; e < rem * rem; e += 256) {
        const int i = s + 1 + e / rem, c = s + 1 + e % rem;
        if (c <= i) S[i * m + c] -= S[i * m + s] * S[c * m + s];
      }
      __syncthreads();
    }
    double* Lj = d.Lw + j * mm;
    for (int e = tid; e < mm; e += 256) Lj[e] = S[e];
    // right-hand side of block j
    if (j == 0) {
      for (int e = tid; e < m * r; e += 256) zb[e] = d.rhs[(int64_t)(e / r) * d.ld_rhs + (e % r)];
    } else {
      const double* V = d.Xw + (j - 1) * mm;
      const double* zp = d.Zw + (int64_t)(j - 1) * m * r;
      for (int e = tid; e < m * r; e += 256) {
        const int a = e / r, c = e % r;
        double acc = 0.0;
        for (int u = 0; u < m; ++u) acc += V[(int64_t)u * m + a] * zp[u * r + c];
        zb[e] = -acc;
      }
    }
    __syncthreads();
    // z_j = L^{-1} zb (column-oriented forward substitution)
    for (int s = 0; s < m; ++s) {
      for (int c = tid; c < r; c += 256) zb[s * r + c] /= S[s * m + s];
      __syncthreads();
      const int rem = m - s - 1;
      for (int e = tid; e < rem * r; e += 256) {
        const int i = s + 1 + e / r, c = e % r;
        zb[i * r + c] -= S[i * m + s] * zb[s * r + c];
      }
      __syncthreads();
    }
    double* zj = d.Zw + (int64_t)j * m * r;
    for (int e = tid; e < m * r; e += 256) zj[e] = zb[e];
    // V_j = L^{-1} B_j^T, 16 columns of B_j^T (= rows of B_j) at a time
    const double* Bj = d.Bsub + j * mm;
    double* Vj = d.Xw + j * mm;
    double est2 = 0.0;
    for (int p0 = 0; p0 < m; p0 += 16) {
      const int np = min(16, m - p0);
      // pan[i][c] = B_j[p0 + c][i]
      for (int e = tid; e < m * 16; e += 256) {
        const int i = e / 16, c = e % 16;
        pan[e] = c < np ? Bj[(int64_t)(p0 + c) * m + i] : 0.0;
      }
      __syncthreads();
      for (int s = 0; s < m; ++s) {
        for (int c = tid; c < 16; c += 256) pan[s * 16 + c] /= S[s * m + s];
        __syncthreads();
        const int rem = m - s - 1;
        for (int e = tid; e < rem * 16; e += 256) {
          const int i = s + 1 + e / 16, c = e % 16;
          pan[i * 16 + c] -= S[i * m + s] * pan[s * 16 + c];
        }
        __syncthreads();
      }
      for (int e = tid; e < m * 16; e += 256) {
        const int i = e / 16, c = e % 16;
        if (c < np) Vj[(int64_t)i * m + p0 + c] = pan[e];
      }
      if (d.est) {
        // (V_j^T z_j)[p0 + c][col] = sum_i pan[i][c] z[i][col]
        for (int e = tid; e < np * r; e += 256) {
          const int c = e / r, col = e % r;
          double acc = 0.0;
          for (int i = 0; i < m; ++i) acc += pan[i * 16 + c] * zb[i * r + col];
          est2 += acc * acc;
        }
      }
      __syncthreads();
    }
    if (d.est) {
      s_red[tid] = est2;
      __syncthreads();
      for (int off = 128; off > 0; off >>= 1) {
        if (tid < off) s_red[tid] += s_red[tid + off];
        __syncthreads();
      }
      if (tid == 0) d.est[j] = sqrt(s_red[0]);
    }
    __syncthreads();
  }
  if (tid == 0 && s_fail && d.fail) *d.fail = 1;
}

__global__ __launch_bounds__(256) void k_tri_backward(const TriDesc* __restrict__ descs, int t,
                                                      const int32_t* __restrict__ act) {
  const TriDesc d = descs[blockIdx.z];
  if (!is_active(act, d.active)) return;
  const int m = d.m, r = d.r, tid = threadIdx.x;
  const int64_t mm = (int64_t)m * m;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  double* S = (double*)smem_raw;   // L_j
  double* yb = S + mm;             // current block (m*r)
  double* yn = yb + m * r;         // next block y_{j+1} (m*r)
  for (int j = t - 1; j >= 0; --j) {
    const double* Lj = d.Lw + j * mm;
    for (int e = tid; e < mm; e += 256) S[e] = Lj[e];
    const double* zj = d.Zw + (int64_t)j * m * r;
    if (j == t - 1) {
      for (int e = tid; e < m * r; e += 256) yb[e] = zj[e];
    } else {
      const double* V = d.Xw + j * mm;
      for (int e = tid; e < m * r; e += 256) {
        const int a = e / r, c = e % r;
        double acc = 0.0;
        for (int u = 0; u < m; ++u) acc += V[(int64_t)a * m + u] * yn[u * r + c];
        yb[e] = zj[e] - acc;
      }
    }
    __syncthreads();
    // solve L^T y = yb (backward, column oriented)
    for (int s = m - 1; s >= 0; --s) {
      for (int c = tid; c < r; c += 256) yb[s * r + c] /= S[s * m + s];
      __syncthreads();
      for (int e = tid; e < s * r; e += 256) {
        const int i = e / r, c = e % r;
        yb[i * r + c] -= S[s * m + i] * yb[s * r + c];
      }
      __syncthreads();
    }
    for (int e = tid; e < m * r; e += 256) {
      const int i = e / r, c = e % r;
      d.Y[(int64_t)(j * m + i) * d.ldy + c] = yb[e];
      yn[e] = yb[e];
    }
    __syncthreads();
  }
}



hipError_t launch_tri_forward(const TriDesc* dd, int nz, int maxm, int maxr, int j0, int j1, const int32_t* act,
                              hipStream_t st) {
  static bool attr = false;
  if (!attr) { hipError_t e = set_big_lds((const void*)k_tri_forward); if (e != hipSuccess) return e; attr = true; }
  const size_t lds = tri_forward_lds(maxm, maxr);
  if (lds > kLdsCap) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_tri_forward, dim3(1, 1, nz), dim3(256), lds, st, dd, j0, j1, act);
  return hipGetLastError();
}

hipError_t launch_tri_backward(const TriDesc* dd, int nz, int maxm, int maxr, int t, const int32_t* act,
                               hipStream_t st) {
  static bool attr = false;
  if (!attr) { hipError_t e = set_big_lds((const void*)k_tri_backward); if (e != hipSuccess) return e; attr = true; }
  const size_t lds = tri_backward_lds(maxm, maxr);
  if (lds > kLdsCap) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_tri_backward, dim3(1, 1, nz), dim3(256), lds, st, dd, t, act);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------------------------
// Precision conversion of rows (RNE), optional BF16 hi/lo split.
// ---------------------------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_convert(const CvtDesc* __restrict__ descs, const int32_t* __restrict__ act) {
  const CvtDesc d = descs[blockIdx.z];
  if (!is_active(act, d.active)) return;
  const int64_t total = (int64_t)d.rows * d.cols;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += stride) {
    const int rr = (int)(e / d.cols), c = (int)(e % d.cols);
    double v = d.src_t == DT_F64 ? ((const double*)d.src.p)[row_off(d.src, rr) + c]
                                 : (double)((const float*)d.src.p)[row_off(d.src, rr) + c];
    if (d.dst_t == DT_F32) {
      ((float*)d.dst.p)[row_off(d.dst, rr) + c] = (float)v;
    } else if (d.dst_t == DT_F64) {
      ((double*)d.dst.p)[row_off(d.dst, rr) + c] = v;
    } else if (!d.split_lo) {
      ((unsigned short*)d.dst.p)[row_off(d.dst, rr) + c] = f32_to_bf16((float)v);
    } else {
      const float f = (float)v;
      const unsigned short hi = f32_to_bf16(f);
      const unsigned short lo = f32_to_bf16((float)(v - (double)bf16_to_f32(hi)));
      ((unsigned short*)d.dst.p)[row_off(d.dst, 2 * rr) + c] = hi;
      ((unsigned short*)d.dst.p)[row_off(d.dst, 2 * rr + 1) + c] = lo;
    }
  }
}

hipError_t launch_convert(const CvtDesc* dd, int nz, int maxRows, int maxCols, const int32_t* act, hipStream_t st) {
  const int64_t tot = (int64_t)maxRows * maxCols;
  int blocks = (int)std::min<int64_t>((tot + 255) / 256, 4096);
  if (blocks < 1) blocks = 1;
  hipLaunchKernelGGL(k_convert, dim3(blocks, 1, nz), dim3(256), 0, st, dd, act);
  return hipGetLastError();
}

// Transpose-convert an FP32 matrix (rows x cols, ld) into BF16 (cols x rows, ldt).
__global__ __launch_bounds__(256) void k_transpose_bf16(const float* __restrict__ src, int64_t ld, int rows, int cols,
                                                        unsigned short* __restrict__ dst, int64_t ldt) {
  __shared__ float tile[32][33];
  const int r0 = blockIdx.y * 32, c0 = blockIdx.x * 32;
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
  for (int y = ty; y < 32; y += 8) {
    const int rr = r0 + y, cc = c0 + tx;
    tile[y][tx] = (rr < rows && cc < cols) ? src[(int64_t)rr * ld + cc] : 0.f;
  }
  __syncthreads();
  for (int y = ty; y < 32; y += 8) {
    const int cc = c0 + y, rr = r0 + tx;
    if (cc < cols && rr < rows) dst[(int64_t)cc * ldt + rr] = f32_to_bf16(tile[tx][y]);
  }
}

hipError_t launch_transpose_bf16(const float* src, int64_t ld, int rows, int cols, unsigned short* dst, int64_t ldt,
                                 hipStream_t st) {
  dim3 grid((cols + 31) / 32, (rows + 31) / 32);
  hipLaunchKernelGGL(k_transpose_bf16, grid, dim3(256), 0, st, src, ld, rows, cols, dst, ldt);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------------------------
// Squared norms of rows; FP64 copies with scaling and zero fill.
// ---------------------------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_sqnorms(const NormDesc* __restrict__ descs, const int32_t* __restrict__ act) {
  const NormDesc d = descs[blockIdx.z];
  if (!is_active(act, d.active)) return;
  const int rr = blockIdx.x;
  if (rr >= d.rows) return;
  const double* x = (const double*)d.x.p + row_off(d.x, rr);
  double acc = 0.0;
  for (int i = threadIdx.x; i < d.n; i += 256) acc += x[i] * x[i];
  __shared__ double red[256];
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int off = 128; off > 0; off >>= 1) {
    if (threadIdx.x < off) red[threadIdx.x] += red[threadIdx.x + off];
    __syncthreads();
  }
  if (threadIdx.x == 0) d.out[rr] = red[0];
}

hipError_t launch_sqnorms(const NormDesc* dd, int nz, int maxRows, const int32_t* act, hipStream_t st) {
  hipLaunchKernelGGL(k_sqnorms, dim3(maxRows, 1, nz), dim3(256), 0, st, dd, act);
  return hipGetLastError();
}

__global__ __launch_bounds__(256) void k_copy(const CopyDesc* __restrict__ descs, const int32_t* __restrict__ act) {
  const CopyDesc d = descs[blockIdx.z];
  if (!is_active(act, d.active)) return;
  const int64_t total = (int64_t)d.rows_total * d.n;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += stride) {
    const int rr = (int)(e / d.n), c = (int)(e % d.n);
    const double v = rr < d.rows ? d.alpha * ((const double*)d.src.p)[row_off(d.src, rr) + c] : 0.0;
    ((double*)d.dst.p)[row_off(d.dst, rr) + c] = v;
  }
}

hipError_t launch_copy(const CopyDesc* dd, int nz, int maxRows, int maxN, const int32_t* act, hipStream_t st) {
  const int64_t tot = (int64_t)maxRows * maxN;
  int blocks = (int)std::min<int64_t>((tot + 255) / 256, 4096);
  if (blocks < 1) blocks = 1;
  hipLaunchKernelGGL(k_copy, dim3(blocks, 1, nz), dim3(256), 0, st, dd, act);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------------------------
// Square-root assembly helpers (def. blansq).
//   k_wsum:   Ybar = sum_j w_j Y_j              (nodes j, n x r blocks)
//   k_tmul:   C = [T Ybar ; B_t Ybar_last]      (block tridiagonal times dense)
// ---------------------------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_wsum(const WsumDesc* __restrict__ descs, const int32_t* __restrict__ act) {
  const WsumDesc d = descs[blockIdx.z];
  if (!is_active(act, d.active)) return;
  const int64_t total = (int64_t)d.n * d.r;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
    double acc = 0.0;
    for (int j = 0; j < d.nq; ++j) acc += d.w[j] * d.Y[j * d.node_stride + e];
    d.out[e] = acc;
  }
}

__global__ __launch_bounds__(256) void k_tmul(const TmulDesc* __restrict__ descs, const int32_t* __restrict__ act) {
  const TmulDesc d = descs[blockIdx.z];
  if (!is_active(act, d.active)) return;
  const int m = d.m, r = d.r, t = d.t;
  const int64_t mm = (int64_t)m * m;
  const int64_t total = (int64_t)(t + 1) * m * r;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
    const int row = (int)(e / r), c = (int)(e % r);
    const int j = row / m, a = row % m;
    double acc = 0.0;
    if (j < t) {
      // D_j Y_j (the true T entries: deflated rows/cols of D are zero, their Y entries are zero)
      for (int u = 0; u < m; ++u) acc += d.D[j * mm + (int64_t)a * m + u] * d.Y[(int64_t)(j * m + u) * r + c];
      if (j > 0)  // B_{j-1} Y_{j-1}
        for (int u = 0; u < m; ++u) acc += d.Bsub[(j - 1) * mm + (int64_t)a * m + u] * d.Y[(int64_t)((j - 1) * m + u) * r + c];
      if (j + 1 < t)  // B_j^T Y_{j+1}
        for (int u = 0; u < m; ++u) acc += d.Bsub[j * mm + (int64_t)u * m + a] * d.Y[(int64_t)((j + 1) * m + u) * r + c];
    } else {
      // B_t Y_t (coupling to the next basis block)
      for (int u = 0; u < m; ++u) acc += d.Bsub[(t - 1) * mm + (int64_t)a * m + u] * d.Y[(int64_t)((t - 1) * m + u) * r + c];
    }
    d.out[e] = acc;
  }
}

hipError_t launch_wsum(const WsumDesc* dd, int nz, int64_t maxTotal, const int32_t* act, hipStream_t st) {
  int blocks = (int)std::min<int64_t>((maxTotal + 255) / 256, 2048);
  if (blocks < 1) blocks = 1;
  hipLaunchKernelGGL(k_wsum, dim3(blocks, 1, nz), dim3(256), 0, st, dd, act);
  return hipGetLastError();
}
hipError_t launch_tmul(const TmulDesc* dd, int nz, int64_t maxTotal, const int32_t* act, hipStream_t st) {
  int blocks = (int)std::min<int64_t>((maxTotal + 255) / 256, 2048);
  if (blocks < 1) blocks = 1;
  hipLaunchKernelGGL(k_tmul, dim3(blocks, 1, nz), dim3(256), 0, st, dd, act);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------------------------
// Convergence bookkeeping on the device: active[z] = 0 once est[z] <= tol[z] * scale[z].
// ---------------------------------------------------------------------------------------------
__global__ void k_converge(const ConvDesc* __restrict__ descs, int nz) {
  const int z = blockIdx.x * blockDim.x + threadIdx.x;
  if (z >= nz) return;
  const ConvDesc c = descs[z];
  if (*c.active_flag == 0) return;
  if (*c.est <= c.tol * (*c.scale)) {
    *c.active_flag = 0;
    *c.done_at = c.step;
  }
}
hipError_t launch_converge(const ConvDesc* dd, int nz, hipStream_t st) {
  hipLaunchKernelGGL(k_converge, dim3((nz + 63) / 64), dim3(64), 0, st, dd, nz);
  return hipGetLastError();
}

}  // namespace rbcg
