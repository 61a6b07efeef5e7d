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

hipError_t launch_gemm_nt_ex(int dtype, int out_t, bool xsplit, const NtDesc* dd, int nz, int maxM, int maxN,
                             int splits, const int32_t* act, hipStream_t st) {
  const int tn = (maxN + 15) / 16;
  if (tn < 1 || tn > 16 || splits < 1) return hipErrorInvalidValue;
  switch (dtype) {
    case DT_F64: return out_t ? nt_f64_o1(tn, dd, nz, maxM, splits, act, st) : nt_f64_o0(tn, dd, nz, maxM, splits, act, st);
    case DT_F32: return out_t ? nt_f32_o1(tn, dd, nz, maxM, splits, act, st) : nt_f32_o0(tn, dd, nz, maxM, splits, act, st);
    case DT_F32F64:
      return out_t ? nt_f32f64_o1(tn, dd, nz, maxM, splits, act, st) : nt_f32f64_o0(tn, dd, nz, maxM, splits, act, st);
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
// sum over s = first, first + step, ... < splits of p[s * stride], in that order; the loads of
// four splits are issued together.
template <typename T>
__device__ __forceinline__ double split_sum(gmem_t<const T> p, int64_t stride, int splits, int first = 0,
                                            int step = 1) {
  double v = 0.0;
  int s = first;
  for (; s + 3 * step < splits; s += 4 * step) {
    const double a = (double)p[(int64_t)s * stride], b = (double)p[(int64_t)(s + step) * stride];
    const double c = (double)p[(int64_t)(s + 2 * step) * stride], d = (double)p[(int64_t)(s + 3 * step) * stride];
    v = (((v + a) + b) + c) + d;
  }
  for (; s < splits; s += step) v += (double)p[(int64_t)s * stride];
  return v;
}

// tpo (a power of two up to 64, FIN_T2R only): lanes per output; lane u of a group sums splits
// u, u + tpo, ... and the group combines by a fixed butterfly, so the result does not depend on
// the launch shape beyond tpo.  Small outputs with many splits (the Gram and projection
// reductions) get the extra parallelism.
__global__ __launch_bounds__(256) void k_finish(const FinDesc* __restrict__ descs, const int32_t* __restrict__ act,
                                                int tpo) {
  const FinDesc f = descs[blockIdx.z];
  if (!is_active(act, f.active)) return;
  const bool rowmajor = f.mode == FIN_ROWMAJOR;
  const int rows = rowmajor ? f.M : f.N;   // outer index of the partial layout
  const int cols = rowmajor ? f.N : f.M;
  if (f.mode == FIN_T2R) {
    const int64_t total = (int64_t)f.N * f.M;
    const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int sub = (int)(gid & (tpo - 1));
    const int64_t stride = (int64_t)gridDim.x * blockDim.x / tpo;
    // every lane of a group sees the same e, so whole groups enter and leave the loop together
    for (int64_t e = gid / tpo; e < total; e += stride) {
      double v = split_sum(gmem(f.part) + e, total, f.splits, sub, tpo);
      for (int off = 1; off < tpo; off <<= 1) v += __shfl_xor(v, off, 64);
      if (sub == 0) {
        const int c = (int)(e / f.M), i = (int)(e % f.M);
        gmem(f.out)[(int64_t)i * f.ldo + c] = f.alpha * v;
      }
    }
    return;
  }
  const int64_t total = (int64_t)rows * cols;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += stride) {
    const int o = (int)(e / cols), in = (int)(e % cols);
    double v = (f.part_f32 ? split_sum(gmem((const float*)f.part) + e, total, f.splits)
                           : split_sum(gmem(f.part) + e, total, f.splits)) * f.alpha;
    if (rowmajor) {
      gmem(f.out)[(int64_t)o * f.ldo + in] = v;
    } else if (f.mode == FIN_TRANS) {
      gmem((double*)f.O.p)[row_off(f.O, o) + in] = v;
    } else if (f.mode == FIN_AXPBY) {
      double y = v;
      if (f.beta != 0.0) y += f.beta * gmem((const double*)f.rhs.p)[row_off(f.rhs, o) + in];
      gmem((double*)f.O.p)[row_off(f.O, o) + in] = y;
    } else {
      const double rv = gmem((const double*)f.rhs.p)[row_off(f.rhs, o) + in];
      const double xv = gmem((const double*)f.xin.p)[row_off(f.xin, o) + in];
      gmem((double*)f.O.p)[row_off(f.O, o) + in] = rv - v - gmem(f.mu)[o] * xv;
    }
  }
}

hipError_t launch_finish(const FinDesc* dd, int nz, int maxM, int maxN, const int32_t* act, hipStream_t st,
                         int tpo) {
  if (tpo < 1 || tpo > 64 || (tpo & (tpo - 1))) return hipErrorInvalidValue;
  const int64_t tot = (int64_t)maxM * maxN * tpo;
  int blocks = (int)std::min<int64_t>((tot + 255) / 256, 2048);
  if (blocks < 1) blocks = 1;
  hipLaunchKernelGGL(k_finish, dim3(blocks, 1, nz), dim3(256), 0, st, dd, act, tpo);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------------------------
// GEMM "NN" update: O[b][i] = beta * Y[b][i] + alpha * sum_a C[a][b] P[a][i]
//   One workgroup = 16 columns i, all Mo rows b (TB tiles), the 4 waves split the a range.
//   MFMA A operand = C^T (b x a), B operand = P (a x i); D rows = b, columns = i.
// ---------------------------------------------------------------------------------------------
template <typename PT, int TB, int NW>
__global__ __launch_bounds__(64 * NW) void k_gemm_nn(const NnDesc* __restrict__ descs, const int32_t* __restrict__ act) {
  const NnDesc d = descs[blockIdx.z];
  if (!is_active(act, d.active)) return;
  if (d.acc_out) {
    const int64_t nthr = (int64_t)gridDim.x * blockDim.x;
    const gmem_t<const double> xa = gmem(d.acc_a), xb = gmem(d.acc_b);
    const gmem_t<double> xo = gmem(d.acc_out);
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < d.acc_n; e += nthr) xo[e] = xa[e] + xb[e];
  }
  const int i0 = blockIdx.x * 16;
  if (i0 >= d.N) return;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int q = lane >> 4, r16 = lane & 15;
  const int i = i0 + r16;
  const bool ival = i < d.N;
  v4d acc[TB];
#pragma unroll
  for (int tb = 0; tb < TB; ++tb) acc[tb] = v4d{0, 0, 0, 0};
  // wave w takes a-chunks of 16 starting at 16 w, stepping 16 NW (deeper register pipelining of
  // the operands measured slower: it costs occupancy)
  const gmem_t<const PT> P = gmem((const PT*)d.P.p);
  const gmem_t<const double> C = gmem(d.C);
  for (int ac = 16 * wave; ac < d.Ka; ac += 16 * NW) {
    double pv[4], cv[4][TB];
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int a = ac + 4 * e + q;
      const bool aval = a < d.Ka;
      pv[e] = (aval && ival) ? (double)P[row_off(d.P, a) + i] : 0.0;
#pragma unroll
      for (int tb = 0; tb < TB; ++tb) {
        const int b = 16 * tb + r16;
        cv[e][tb] = (aval && b < d.Mo) ? C[(int64_t)a * d.ldc + b] : 0.0;
      }
    }
#pragma unroll
    for (int e = 0; e < 4; ++e)
#pragma unroll
      for (int tb = 0; tb < TB; ++tb)
        acc[tb] = __builtin_amdgcn_mfma_f64_16x16x4f64(cv[e][tb], pv[e], acc[tb], 0, 0, 0);
  }
  extern __shared__ __align__(16) unsigned char smem_raw[];
  double* red = (double*)smem_raw;   // [NW - 1][TB][4][64]
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
      for (int w = 0; w < NW - 1; ++w) v += red[((w * TB + tb) * 4 + r) * 64 + lane];
      double out = d.alpha * v;
      if (d.beta != 0.0) out += d.beta * gmem((const double*)d.Y.p)[row_off(d.Y, b) + i];
      gmem((double*)d.O.p)[row_off(d.O, b) + i] = out;
      if (d.O32.p) gmem((float*)d.O32.p)[row_off(d.O32, b) + i] = (float)out;   // RNE, as k_convert
    }
  }
}

template <typename PT, int TB, int NW>
static hipError_t launch_nn_w(const NnDesc* dd, int nz, int maxN, const int32_t* act, hipStream_t st) {
  const size_t lds = (size_t)(NW - 1) * TB * 4 * 64 * 8;
  auto kern = k_gemm_nn<PT, TB, NW>;
  // raised once per process; function-local static initialisation is thread-safe
  static const hipError_t attr =
      lds > 64 * 1024 ? hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds)
                      : hipSuccess;
  if (attr != hipSuccess) return attr;
  hipLaunchKernelGGL(kern, dim3((maxN + 15) / 16, 1, nz), dim3(64 * NW), lds, st, dd, act);
  return hipGetLastError();
}

template <typename PT, int TB>
static hipError_t launch_nn_t(const NnDesc* dd, int nz, int maxN, const int32_t* act, hipStream_t st) {
  return launch_nn_w<PT, TB, 4>(dd, nz, maxN, act, st);
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
__device__ __forceinline__ void wave_argmax(double& v, int& i) {
  // maximum value, smallest index on ties, across the 64 lanes of a wave
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    const double ov = __shfl_xor(v, off, 64);
    const int oi = __shfl_xor(i, off, 64);
    if (ov > v || (ov == v && oi < i)) { v = ov; i = oi; }
  }
}

// Register-resident pivoted Cholesky QR factor.  Thread t owns column c = t % m and rows
// a = stripe + stripes*q (stripe = t / m, stripes = 1024 / m) of the Gram matrix, slot q.
// Per pivot step: wave argmax over the published diagonal, publish the pivot row (zeros on
// retired columns), one FMA per owned element.  Three barriers per step.
template <int NS>
__global__ __launch_bounds__(1024) void k_qr_factor(const QrDesc* __restrict__ descs, const int32_t* __restrict__ act,
                                                    int lds_bytes) {
  const QrDesc d = descs[blockIdx.z];
  if (!is_active(act, d.active)) return;
  const int m = d.m;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int stripes = 1024 / m;
  const int c = tid % m, stripe = tid / m;
  const bool owner = stripe < stripes;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  double* Rl = (double*)smem_raw;            // m*m: R rows by pivot position
  double* rowb = Rl + m * m;                 // m: published row
  double* diag = rowb + m;                   // m: current Schur diagonal
  double* dref = diag + m;                   // m
  double* pre = dref + m;                    // m
  double* pan = pre + m;                     // 16*m: prevB panel
  double* wv = pan + 16 * m;                 // 16
  int* wi = (int*)(wv + 16);                 // 16
  int* perm = wi + 16;                       // m: pivot position -> column of W
  int* chosen = perm + m;                    // m: per column of W (later: inverse permutation)
  int* kept = chosen + m;                    // m: per pivot position
  __shared__ int s_rank;

  // ---- second pass on a near-identity Gram: G = I + E over the non-zero columns with
  //      max |E| <= 1e-8 gives R = I + F (F = upper part of E, halved diagonal) and
  //      R^{-1} = I - F, both exact to O(|E|^2) = rounding level; no sequential factorization.
  if (!d.pivot && d.prevB) {
    __shared__ int s_small, s_kept;
    __shared__ double s_wmax[16];
    __shared__ int s_wcnt[16];
    // G into LDS (Rl) and prevB behind the other arrays when the launch reserved room: one pass
    // over global memory, everything after it reads LDS
    const size_t pb_off = ((size_t)((unsigned char*)(kept + m) - smem_raw) + 15) & ~(size_t)15;
    double* pb = (double*)(smem_raw + pb_off);
    const bool whole = (int64_t)((unsigned char*)(pb + m * m) - smem_raw) <= lds_bytes;
    {
      const gmem_t<const double> G = gmem(d.G), PB = gmem(d.prevB);
      for (int e = tid; e < m * m; e += 1024) {
        const int a = e / m, cc = e - a * m;
        Rl[e] = G[(int64_t)a * d.ldg + cc];
        if (whole) pb[e] = PB[e];
      }
    }
    if (d.dg.D) diag_block(d.dg, threadIdx.x, 1024);   // independent work while the loads land
    __syncthreads();
    double emax = 0.0;
    for (int e = tid; e < m * m; e += 1024) {
      const int a = e / m, cc = e - a * m;
      if (Rl[a * m + a] == 0.0 || Rl[cc * m + cc] == 0.0) continue;   // deflated (zero) columns
      emax = fmax(emax, fabs(Rl[e] - (a == cc ? 1.0 : 0.0)));
    }
    int cnt = (tid < m && Rl[tid * m + tid] != 0.0) ? 1 : 0;   // m <= 1024
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
      emax = fmax(emax, __shfl_xor(emax, off, 64));
      cnt += __shfl_xor(cnt, off, 64);
    }
    if (lane == 0) {
      s_wmax[wave] = emax;
      s_wcnt[wave] = cnt;
    }
    __syncthreads();
    if (tid == 0) {
      double mx = 0.0;
      int kc = 0;
      for (int w = 0; w < 16; ++w) {
        mx = fmax(mx, s_wmax[w]);
        kc += s_wcnt[w];
      }
      s_small = mx <= 1e-8;
      s_kept = kc;
    }
    __syncthreads();
    if (s_small) {
      // kept[i] = column i non-zero; F in Rl (upper), Bout = (I + F) prevB, Mout = I - F
      for (int i = tid; i < m; i += 1024) {
        kept[i] = Rl[i * m + i] != 0.0;
        gmem(d.mask)[i] = kept[i] ? 0 : 1;
      }
      __syncthreads();
      for (int e = tid; e < m * m; e += 1024) {   // in place: each element read and written by one thread
        const int a = e / m, cc = e - a * m;
        double f = 0.0;
        if (kept[a] && kept[cc] && cc >= a) {
          const double g = Rl[e];
          f = (a == cc) ? 0.5 * (g - 1.0) : g;
        }
        Rl[e] = f;
        gmem(d.Mout)[e] = (kept[a] && kept[cc]) ? ((a == cc ? 1.0 : 0.0) - f) : 0.0;
      }
      if (tid == 0 && d.rank_out) *gmem(d.rank_out) = s_kept;
      __syncthreads();
      if (whole) {
        // F prevB on the FP64 16x16x4 MFMA from LDS: 16 x 16 output tiles dealt to the 16
        // waves; F is upper triangular, so tile row ti starts its reduction at u = 16 ti
        const int MT = (m + 15) / 16;
        const int r16 = lane & 15, kq = lane >> 4;
        for (int tile = wave; tile < MT * MT; tile += 16) {
          const int ti = tile / MT, tj = tile - ti * MT;
          const int s0 = 16 * ti + r16, cc = 16 * tj + r16;
          v4d acc = {0.0, 0.0, 0.0, 0.0};
          for (int u0 = 16 * ti; u0 < m; u0 += 4) {
            const int u = u0 + kq;
            const double a = (s0 < m && u < m) ? Rl[s0 * m + u] : 0.0;
            const double b = (u < m && cc < m) ? pb[u * m + cc] : 0.0;
            acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc, 0, 0, 0);
          }
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const int row = 16 * ti + kq + 4 * r, col = 16 * tj + r16;
            if (row < m && col < m) gmem(d.Bout)[row * m + col] = kept[row] ? pb[row * m + col] + acc[r] : 0.0;
          }
        }
        return;
      }
      for (int c0 = 0; c0 < m; c0 += 16) {
        const int nc = min(16, m - c0);
        for (int e = tid; e < m * 16; e += 1024) {
          const int u = e >> 4, cc = e & 15;
          pan[e] = cc < nc ? gmem(d.prevB)[u * m + c0 + cc] : 0.0;
        }
        __syncthreads();
        for (int e = tid; e < m * 16; e += 1024) {
          const int s0 = e >> 4, cc = e & 15;
          if (cc >= nc) continue;
          double acc = 0.0;
          if (kept[s0]) {
            acc = pan[s0 * 16 + cc];
            const double* Fs = Rl + s0 * m;
            for (int u = s0; u < m; ++u) acc += Fs[u] * pan[u * 16 + cc];
          }
          gmem(d.Bout)[s0 * m + c0 + cc] = acc;
        }
        __syncthreads();
      }
      return;
    }
    __syncthreads();   // Rl is reused below
  } else if (d.dg.D) {
    diag_block(d.dg, threadIdx.x, 1024);
  }

  // ---- unpivoted attempt (the common case) with the inverse factor carried along: thread
  //      (stripe, c) holds the Schur entries (a, c) and the entries E[a][c] of E = L^{-1}
  //      (G = L D L^T, L unit lower triangular), i.e. the elimination's row operations applied to
  //      the identity.  Rhat^{-1} = E^T D^{-1/2}, so no triangular inversion follows.  One barrier
  //      per step (publication double-buffered), the row slot of the pivot a compile-time
  //      constant.  A pivot failing any test ends the attempt and the general path below redoes
  //      the factorization (pivoting where asked; a pivoted factorization attempts with the
  //      stricter relative threshold max(tau, 1e-8)).
  bool fast_ok = false;
  double ev[NS];
  if constexpr (NS <= 9) {   // (wider slot counts would spill the extra registers)
    const double tau_a = d.pivot ? fmax(d.tau, 1e-8) : d.tau;
    const gmem_t<const double> G = gmem(d.G);
    double va[NS];
    for (int i = tid; i < m; i += 1024) {
      dref[i] = G[(int64_t)i * d.ldg + i];
      pre[i] = d.pre ? gmem(d.pre)[(int64_t)i * d.pre_stride] : -1.0;
    }
#pragma unroll
    for (int q = 0; q < NS; ++q) {
      const int a = stripe + stripes * q;
      va[q] = (owner && a < m) ? G[(int64_t)a * d.ldg + c] : 0.0;
      ev[q] = (owner && a == c) ? 1.0 : 0.0;
    }
    __syncthreads();
    bool ok = true;
    static_for<NS>([&](auto qc) {
      constexpr int qs = decltype(qc)::value;
      for (int ps = 0; ps < stripes; ++ps) {
        const int s = qs * stripes + ps;
        if (s >= m || !ok) break;   // uniform
        double* rb = pan + (s & 1) * 2 * m;   // Schur row s (= column s)
        double* eb = rb + m;                  // row s of E (final: last updated at step s - 1)
        if (owner && stripe == ps) {
          rb[c] = va[qs];
          eb[c] = ev[qs];
        }
        __syncthreads();
        const double piv2 = rb[s], drp = dref[s], prp = pre[s];
        const double rcv = owner ? rb[c] : 0.0, ecv = owner ? eb[c] : 0.0;
        double ra[NS];
#pragma unroll
        for (int q = qs; q < NS; ++q) {
          const int a = stripe + stripes * q;
          ra[q] = a < m ? rb[a] : 0.0;
        }
        bool bad;
        if (d.force_first && s == 0) bad = !(piv2 > 0.0);
        else
          bad = !(drp > 0.0) | !(piv2 > tau_a * drp) | ((prp >= 0.0) & !(piv2 > d.eta2 * prp)) |
                !(piv2 > d.floor2);
        if (bad) {
          ok = false;
          break;
        }
        const bool fast = pos_in_range(piv2);
        const double f = fast ? recip_pos(piv2) : 1.0 / piv2;
#pragma unroll
        for (int q = qs; q < NS; ++q) {
          double li = ra[q] * f;
          if (q == qs && stripe <= ps) li = 0.0;   // rows up to the pivot are final
          va[q] = fma(-li, rcv, va[q]);
          ev[q] = fma(-li, ecv, ev[q]);
        }
        const double irp = fast ? rsqrt_pos(piv2) : 1.0 / sqrt(piv2);
        if (tid < m) Rl[s * m + tid] = tid >= s ? rcv * irp : 0.0;   // row s of R
        if (tid == 0) diag[s] = irp;                                 // 1 / Rhat[s][s]
      }
    });
    fast_ok = ok;
  }

  double v[NS];
  if (!fast_ok) {
    __syncthreads();
#pragma unroll
    for (int q = 0; q < NS; ++q) {
      const int a = stripe + stripes * q;
      v[q] = (owner && a < m) ? gmem(d.G)[(int64_t)a * d.ldg + c] : 0.0;
    }
    for (int e = tid; e < m * m; e += 1024) Rl[e] = 0.0;
    for (int i = tid; i < m; i += 1024) {
      const double g = gmem(d.G)[(int64_t)i * d.ldg + i];
      dref[i] = g;
      diag[i] = g;
      pre[i] = d.pre ? gmem(d.pre)[(int64_t)i * d.pre_stride] : -1.0;
      chosen[i] = 0;
      kept[i] = 0;
      perm[i] = i;
    }
    if (tid == 0) s_rank = 0;
    __syncthreads();

    int s = 0;
    for (; s < m; ++s) {
      int p = s;
      if (d.pivot && !(d.force_first && s == 0)) {
        if (wave == 0) {
          double best = -2.0;
          int bi = 0x7fffffff;
          for (int cc = lane; cc < m; cc += 64) {
            if (chosen[cc]) continue;
            const double rel = dref[cc] > 0.0 ? diag[cc] / dref[cc] : -1.0;
            if (rel > best || (rel == best && cc < bi)) { best = rel; bi = cc; }
          }
          wave_argmax(best, bi);
          if (lane == 0) wi[0] = bi;
        }
        __syncthreads();
        p = wi[0];
      }
      const double piv2 = diag[p];
      bool defl;
      if (d.force_first && s == 0) defl = !(piv2 > 0.0);
      else defl = !(dref[p] > 0.0) || !(piv2 > d.tau * dref[p]) || (pre[p] >= 0.0 && !(piv2 > d.eta2 * pre[p])) ||
                  !(piv2 > d.floor2);
      if (defl && d.pivot) break;   // every remaining column is at least as deficient
      if (defl) {
        __syncthreads();
        if (tid == 0) { perm[s] = p; chosen[p] = 1; }
        __syncthreads();
        continue;
      }
      const double rp = sqrt(piv2);
      const double irp = 1.0 / rp;
      // publish row p of R: the owner of (p, c) for every column c
      if (owner && stripe == p % stripes) {
        const int qp = p / stripes;
        double x = 0.0;
#pragma unroll
        for (int q = 0; q < NS; ++q)
          if (q == qp) x = v[q];
        rowb[c] = (c == p) ? rp : (chosen[c] ? 0.0 : x * irp);
      }
      __syncthreads();
      // Schur update of owned elements; retired and chosen rows/columns see a zero factor
      if (owner) {
        const double rc = rowb[c];
#pragma unroll
        for (int q = 0; q < NS; ++q) {
          const int a = stripe + stripes * q;
          if (a < m) {
            v[q] -= rowb[a] * rc;
            if (a == c) diag[a] = v[q];
          }
        }
      }
      for (int i = tid; i < m; i += 1024) Rl[s * m + i] = rowb[i];
      if (tid == 0) { perm[s] = p; chosen[p] = 1; kept[s] = 1; s_rank = s_rank + 1; }
      __syncthreads();
    }
    if (tid == 0) {
      int pos = s;
      for (int i = 0; i < m && pos < m; ++i)
        if (!chosen[i]) { perm[pos++] = i; chosen[i] = 1; }
    }
  } else {
    for (int i = tid; i < m; i += 1024) {
      kept[i] = 1;
      perm[i] = i;
    }
    if (tid == 0) s_rank = m;
  }
  __syncthreads();
  // ---- reported coefficient block Bout = R (times prevB, staged 16 columns at a time)
  if (d.prevB) {
    for (int c0 = 0; c0 < m; c0 += 16) {
      const int nc = min(16, m - c0);
      for (int e = tid; e < m * 16; e += 1024) {
        const int u = e >> 4, cc = e & 15;
        pan[e] = cc < nc ? gmem(d.prevB)[u * m + c0 + cc] : 0.0;
      }
      __syncthreads();
      for (int e = tid; e < m * 16; e += 1024) {
        const int s0 = e >> 4, cc = e & 15;
        if (cc >= nc) continue;
        double acc = 0.0;
        if (kept[s0]) {
          const double* Rs = Rl + s0 * m;
          for (int u = 0; u < m; ++u) acc += Rs[u] * pan[u * 16 + cc];
        }
        gmem(d.Bout)[s0 * m + c0 + cc] = acc;
      }
      __syncthreads();
    }
  } else {
    for (int e = tid; e < m * m; e += 1024) gmem(d.Bout)[e] = kept[e / m] ? Rl[e] : 0.0;
  }
  for (int i = tid; i < m; i += 1024) gmem(d.mask)[i] = kept[i] ? 0 : 1;
  if (tid == 0 && d.rank_out) *gmem(d.rank_out) = s_rank;
  if (fast_ok) {   // Mout[c][a] = E[a][c] / sqrt(D[a]) (zero for c > a)
    if (owner) {
#pragma unroll
      for (int q = 0; q < NS; ++q) {
        const int a = stripe + stripes * q;
        if (a < m) gmem(d.Mout)[(int64_t)c * m + a] = ev[q] * diag[a];
      }
    }
    return;
  }
  // ---- X = Rhat^{-1} in registers (pivot positions), Rhat[i][u] = R[i][perm[u]]:
  //      X = I; for q descending: X[q][:] /= Rhat[q][q]; X[i][:] -= Rhat[i][q] X[q][:], i < q.
  __syncthreads();
#pragma unroll
  for (int q = 0; q < NS; ++q) {
    const int a = stripe + stripes * q;
    v[q] = (owner && a < m && a == c && kept[a]) ? 1.0 : 0.0;
  }
  const int qtop = d.pivot ? s_rank - 1 : m - 1;
  for (int qq = qtop; qq >= 0; --qq) {
    if (!kept[qq]) continue;                        // uniform (LDS)
    const double rqq = Rl[qq * m + perm[qq]];
    if (owner && stripe == qq % stripes) {
      const int qs = qq / stripes;
#pragma unroll
      for (int q = 0; q < NS; ++q)
        if (q == qs) {
          v[q] /= rqq;
          rowb[c] = v[q];
        }
    }
    __syncthreads();
    if (owner) {
      const double xc = rowb[c];
      const int pq = perm[qq];
#pragma unroll
      for (int q = 0; q < NS; ++q) {
        const int a = stripe + stripes * q;
        if (a < qq && kept[a]) v[q] -= Rl[a * m + pq] * xc;
      }
    }
    __syncthreads();
  }
  // ---- Mout[perm[i]][c] = X[i][c] for kept i <= c (Q column c = sum_a W column a * Mout[a][c])
  if (owner) {
#pragma unroll
    for (int q = 0; q < NS; ++q) {
      const int a = stripe + stripes * q;
      if (a >= m) continue;
      const double x = (kept[a] && kept[c] && a <= c) ? v[q] : 0.0;
      gmem(d.Mout)[perm[a] * m + c] = x;
    }
  }
}

hipError_t launch_qr_factor(const QrDesc* dd, int nz, int maxm, bool uniform, const int32_t* act,
                            hipStream_t st) {
  if (uniform && qr_m_supported(maxm)) return launch_qr_m(dd, nz, maxm, act, st);
  size_t lds = ((size_t)maxm * maxm + 4 * (size_t)maxm + 16 * (size_t)maxm + 16) * 8 + 16 * 4 +
               (size_t)maxm * 3 * 4 + 64;
  if (lds > kLdsCap) return hipErrorInvalidValue;
  // room for the whole previous factor behind the other arrays (first-order second pass)
  if (lds + (size_t)maxm * maxm * 8 + 16 <= kLdsCap) lds += (size_t)maxm * maxm * 8 + 16;
  const int ns = (maxm + (1024 / maxm) - 1) / (1024 / maxm);   // rows per thread
  const void* kern;
  int slot;
  if (ns <= 1) { kern = (const void*)k_qr_factor<1>; slot = 0; }
  else if (ns <= 2) { kern = (const void*)k_qr_factor<2>; slot = 1; }
  else if (ns <= 5) { kern = (const void*)k_qr_factor<5>; slot = 2; }
  else if (ns <= 9) { kern = (const void*)k_qr_factor<9>; slot = 3; }
  else if (ns <= 14) { kern = (const void*)k_qr_factor<14>; slot = 4; }
  else if (ns <= 19) { kern = (const void*)k_qr_factor<19>; slot = 5; }
  else return hipErrorInvalidValue;
  static const hipError_t attr[6] = {
      set_big_lds((const void*)k_qr_factor<1>), set_big_lds((const void*)k_qr_factor<2>),
      set_big_lds((const void*)k_qr_factor<5>), set_big_lds((const void*)k_qr_factor<9>),
      set_big_lds((const void*)k_qr_factor<14>), set_big_lds((const void*)k_qr_factor<19>)};
  if (attr[slot] != hipSuccess) return attr[slot];
  int lb = (int)lds;
  void* args[] = {(void*)&dd, (void*)&act, (void*)&lb};
  return hipLaunchKernel(kern, dim3(1, 1, nz), dim3(1024), args, lds, st);
}

// ---------------------------------------------------------------------------------------------
// Diagonal block of T: D = sym(C1 + C2); deflated columns become decoupled unit rows.
// ---------------------------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_diag(const DiagDesc* __restrict__ descs, const int32_t* __restrict__ act) {
  const DiagDesc d = descs[blockIdx.z];
  if (!is_active(act, d.active)) return;
  diag_block(d, threadIdx.x, 256);
}

hipError_t launch_diag(const DiagDesc* dd, int nz, int maxm, const int32_t* act, hipStream_t st) {
  (void)maxm;
  hipLaunchKernelGGL(k_diag, dim3(1, 1, nz), dim3(256), 0, st, dd, act);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------------------------
// Shifted block-tridiagonal solve, one workgroup per (shift, system): block Thomas elimination
// with explicit inverses of the SPD Schur complements (Gauss-Jordan in LDS, no pivoting).
// Forward sweep over blocks j in [j0, j1):
//   S_j = D_j + sigma I - U_{j-1} B_{j-1}^T,   Sinv_j = S_j^{-1},   U_j = B_j Sinv_j,
//   rhs'_0 = rhs,  rhs'_{j+1} = -U_j rhs'_j
// with B_j = T[j+1][j].  The truncated solve over blocks 0..j has last block y_j = Sinv_j rhs'_j
// and residual norm || B_j y_j || = || rhs'_{j+1} || (Lanczos relation), reported in est[j].
// Backward sweep: y_{t-1} = Sinv_{t-1} rhs'_{t-1},  y_j = Sinv_j (rhs'_j - B_j^T y_{j+1}).
// Storage: Lw[j] = Sinv_j, Xw[j] = U_j, Zw[j] = rhs'_j (block j+1 also written by block j).
// LDS: S (m*m) always; B_j and U_j too when 3 m^2 + 2 m r doubles fit ("resident" mode).
// ---------------------------------------------------------------------------------------------
// S[a][b] -= sum_u U[a][u] B[b][u] with U, B in global memory, through 8-row LDS panels.
__device__ __forceinline__ void schur_update_paneled(double* S, int m, const double* U, const double* B, double* pa,
                                                     double* pb, int tid) {
  for (int a0 = 0; a0 < m; a0 += 8) {
    const int na = min(8, m - a0);
    for (int e = tid; e < 8 * m; e += 1024) pa[e] = (e / m) < na ? U[(int64_t)a0 * m + e] : 0.0;
    for (int b0 = 0; b0 < m; b0 += 8) {
      const int nb = min(8, m - b0);
      for (int e = tid; e < 8 * m; e += 1024) pb[e] = (e / m) < nb ? B[(int64_t)b0 * m + e] : 0.0;
      __syncthreads();
      // 64 outputs, 16 lanes each over a sixteenth of u, reduced with shuffles
      const int o = tid >> 4, part = tid & 15;
      const int a = o >> 3, b = o & 7;
      double acc = 0.0;
#pragma unroll 2
      for (int u = part; u < m; u += 16) acc += pa[a * m + u] * pb[b * m + u];
#pragma unroll
      for (int off = 1; off < 16; off <<= 1) acc += __shfl_xor(acc, off, 64);
      if (part == 0 && a < na && b < nb) S[(a0 + a) * m + b0 + b] -= acc;
      __syncthreads();
    }
  }
}

// U[a][c] = sum_u B[a][u] Sinv[u][c] with B in global memory (8-row panels), Sinv in LDS.
__device__ __forceinline__ void left_mul_paneled(double* Uout, int m, const double* B, const double* Sinv,
                                                 double* pa, int tid) {
  for (int a0 = 0; a0 < m; a0 += 8) {
    const int na = min(8, m - a0);
    for (int e = tid; e < 8 * m; e += 1024) pa[e] = (e / m) < na ? B[(int64_t)a0 * m + e] : 0.0;
    __syncthreads();
    for (int e = tid; e < na * m; e += 1024) {
      const int a = e / m, c = e - a * m;
      double acc = 0.0;
#pragma unroll 2
      for (int u = 0; u < m; ++u) acc += pa[a * m + u] * Sinv[u * m + c];
      Uout[(int64_t)(a0 + a) * m + c] = acc;
    }
    __syncthreads();
  }
}

// Block-Thomas forward sweep (see the comment above).  1024 threads; the Schur complement is
// inverted register-resident by Gauss-Jordan: thread t owns column c = t % m and rows
// stripe + stripes*q (stripe = t / m, stripes = 1024 / m); two barriers per pivot.  Products
// run from LDS.
template <int NS>
__global__ __launch_bounds__(1024) void k_tri_forward(const TriDesc* __restrict__ descs, int j0, int j1, int lds_bytes,
                                                      const int32_t* __restrict__ act) {
  const TriDesc d = descs[blockIdx.z];
  if (!is_active(act, d.active)) return;
  const int m = d.m, r = d.r, tid = threadIdx.x;
  const int64_t mm = (int64_t)m * m;
  const int stripes = 1024 / m;
  const int c = tid % m, stripe = tid / m;
  const bool owner = stripe < stripes;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const bool resident = (int64_t)(3 * mm + 2 * m * r + 3 * m) * 8 <= lds_bytes;
  double* S = (double*)smem_raw;                 // m*m: LDS image of S / S^-1
  double* col = S + mm;                          // m
  double* prow = col + m;                        // m
  double* diag = prow + m;                       // m
  double* zb = diag + m;                         // m*r: rhs'_j
  double* zn = zb + m * r;                       // m*r: rhs'_{j+1}
  double* Bl = zn + m * r;                       // resident: m*m (B_j); else 8*m panel
  double* Ul = Bl + (resident ? mm : 8 * m);     // resident: m*m (U_j);  else 8*m panel
  __shared__ int s_fail;
  __shared__ double s_red[16];
  double v[NS];
  if (tid == 0) s_fail = 0;
  for (int j = j0; j < j1; ++j) {
    const double* Dj = d.D + j * mm;
    const int32_t* mk = d.mask + (int64_t)j * m;
    if (j > 0 && resident && j == j0) {
      for (int e = tid; e < mm; e += 1024) {
        Ul[e] = d.Xw[(j - 1) * mm + e];
        Bl[e] = d.Bsub[(j - 1) * mm + e];
      }
    }
    for (int e = tid; e < mm; e += 1024) S[e] = Dj[e];
    if (j == j0) {
      if (j == 0) {
        for (int e = tid; e < m * r; e += 1024) zb[e] = d.rhs[(int64_t)(e / r) * d.ld_rhs + (e % r)];
      } else {
        for (int e = tid; e < m * r; e += 1024) zb[e] = d.Zw[(int64_t)j * m * r + e];
      }
    }
    __syncthreads();
    // S = D_j - U_{j-1} B_{j-1}^T
    if (j > 0) {
      if (resident) {
        for (int e = tid; e < mm; e += 1024) {
          const int a = (int)(e / m), b = (int)(e % m);
          double acc = 0.0;
#pragma unroll 2
          for (int u = 0; u < m; ++u) acc += Ul[a * m + u] * Bl[b * m + u];
          S[e] -= acc;
        }
      } else {
        schur_update_paneled(S, m, d.Xw + (j - 1) * mm, d.Bsub + (j - 1) * mm, Bl, Ul, tid);
      }
    }
    __syncthreads();
    // registers: + sigma I, symmetrised, deflated indices decoupled with a unit diagonal
    const bool mc = owner ? (mk[c] != 0) : false;
#pragma unroll
    for (int q = 0; q < NS; ++q) {
      const int a = stripe + stripes * q;
      double x = 0.0;
      if (owner && a < m) {
        x = (a == c) ? S[a * m + c] + d.sigma : 0.5 * (S[a * m + c] + S[c * m + a]);
        if (mc || mk[a]) x = (a == c) ? 1.0 : 0.0;
        if (a == c) diag[a] = x;
      }
      v[q] = x;
    }
    __syncthreads();
    // Gauss-Jordan inverse in registers
    for (int p = 0; p < m; ++p) {
      const double piv = diag[p];
      const bool bad = !(piv > 0.0);
      const double ipv = bad ? 0.0 : 1.0 / piv;
      if (bad && tid == 0) s_fail = 1;
      if (owner) {
        const int ps = p % stripes, pq = p / stripes;
        if (c == p) {
#pragma unroll
          for (int q = 0; q < NS; ++q) {
            const int a = stripe + stripes * q;
            if (a < m) col[a] = v[q];
          }
        }
        if (stripe == ps) {
#pragma unroll
          for (int q = 0; q < NS; ++q)
            if (q == pq) {
              v[q] = (c == p) ? ipv : v[q] * ipv;
              prow[c] = v[q];
            }
        }
      }
      __syncthreads();
      if (owner) {
        const double pc = prow[c];
#pragma unroll
        for (int q = 0; q < NS; ++q) {
          const int a = stripe + stripes * q;
          if (a >= m || a == p) continue;
          v[q] = ((c == p) ? 0.0 : v[q]) - col[a] * pc;
          if (a == c) diag[a] = v[q];
        }
      }
      __syncthreads();
    }
    double* Lj = d.Lw + j * mm;
    if (owner) {
#pragma unroll
      for (int q = 0; q < NS; ++q) {
        const int a = stripe + stripes * q;
        if (a < m) {
          S[a * m + c] = v[q];
          Lj[a * m + c] = v[q];
        }
      }
    }
    for (int e = tid; e < m * r; e += 1024) d.Zw[(int64_t)j * m * r + e] = zb[e];
    const double* Bj = d.Bsub + j * mm;
    double* Uj = d.Xw + j * mm;
    if (resident) {
      for (int e = tid; e < mm; e += 1024) Bl[e] = Bj[e];
    }
    __syncthreads();
    // U_j = B_j Sinv_j
    if (resident) {
      for (int e = tid; e < mm; e += 1024) {
        const int a = (int)(e / m), cc = (int)(e % m);
        double acc = 0.0;
#pragma unroll 2
        for (int u = 0; u < m; ++u) acc += Bl[a * m + u] * S[u * m + cc];
        Ul[e] = acc;
        Uj[e] = acc;
      }
      __syncthreads();
    } else {
      left_mul_paneled(Uj, m, Bj, S, Bl, tid);
      __threadfence();   // U_j is read back from global memory below and by the next block
      __syncthreads();
    }
    // rhs'_{j+1} = -U_j rhs'_j and its norm (the residual estimate of the truncated solve)
    double sq = 0.0;
    const double* Us = resident ? Ul : Uj;
    for (int e = tid; e < m * r; e += 1024) {
      const int a = e / r, cc = e % r;
      double acc = 0.0;
#pragma unroll 2
      for (int u = 0; u < m; ++u) acc += Us[(int64_t)a * m + u] * zb[u * r + cc];
      zn[e] = -acc;
      sq += acc * acc;
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) sq += __shfl_xor(sq, off, 64);
    if ((tid & 63) == 0) s_red[tid >> 6] = sq;
    __syncthreads();
    if (d.est && tid == 0) {
      double t2 = 0.0;
      for (int w = 0; w < 16; ++w) t2 += s_red[w];
      d.est[j] = sqrt(t2);
    }
    for (int e = tid; e < m * r; e += 1024) {
      zb[e] = zn[e];
      d.Zw[(int64_t)(j + 1) * m * r + e] = zn[e];
    }
    __syncthreads();
  }
  if (tid == 0 && s_fail && d.fail) *d.fail = 1;
}

__global__ __launch_bounds__(1024) void k_tri_backward(const TriDesc* __restrict__ descs, int t,
                                                       const int32_t* __restrict__ act) {
  const TriDesc d = descs[blockIdx.z];
  if (!is_active(act, d.active)) return;
  const int m = d.m, r = d.r, tid = threadIdx.x;
  const int64_t mm = (int64_t)m * m;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  double* S = (double*)smem_raw;   // B_j, then Sinv_j
  double* yb = S + mm;             // rhs'_j - B_j^T y_{j+1}
  double* yn = yb + m * r;         // y_{j+1}
  const int tt = d.nblk > 0 ? d.nblk : t;
  for (int j = tt - 1; j >= 0; --j) {
    const double* zj = d.Zw + (int64_t)j * m * r;
    if (j == tt - 1) {
      for (int e = tid; e < m * r; e += 1024) yb[e] = zj[e];
    } else {
      const double* Bj = d.Bsub + j * mm;
      for (int e = tid; e < mm; e += 1024) S[e] = Bj[e];
      __syncthreads();
      for (int e = tid; e < m * r; e += 1024) {
        const int a = e / r, c = e % r;
        double acc = 0.0;
        for (int u = 0; u < m; ++u) acc += S[u * m + a] * yn[u * r + c];
        yb[e] = zj[e] - acc;
      }
    }
    __syncthreads();
    const double* Lj = d.Lw + j * mm;
    for (int e = tid; e < mm; e += 1024) S[e] = Lj[e];
    __syncthreads();
    for (int e = tid; e < m * r; e += 1024) {
      const int a = e / r, c = e % r;
      double acc = 0.0;
      for (int u = 0; u < m; ++u) acc += S[a * m + u] * yb[u * r + c];
      d.Y[(int64_t)(j * m + a) * d.ldy + c] = acc;
      yn[e] = acc;
    }
    __syncthreads();
  }
}

// One refinement step of the projected solve (see the declaration).  One workgroup per
// descriptor; y and the residual live in LDS.  Residual, row a of block i:
//   R_i[a] = rhs_i[a] - sum_c S_i[a][c] y_i[c] - (K_{i-1} y_{i-1})[a] - (K_i^T y_{i+1})[a]
//            - sum_{j >= i+2} (H_j[i] y_j)[a] - sum_{j <= i-2} (H_i[j]^T y_j)[a]
// with S_i = sym(D_i) + sigma I and unit rows for deflated indices (as in the forward sweep).
// The coupling K_i of blocks i and i+1 has two FP64 estimates: B_i from the Cholesky QR of the
// projected block (Q_{i+1}^T A Q_i) and H_{i+1}[i]^T from the next step's projection
// (Q_i^T A Q_{i+1}, transposed); with the coefficients present K_i is their mean, the
// symmetric part of Q^T A Q, else B_i.  Then z_0 = R_0, z_{i+1} = R_{i+1} - U_i z_i,
// delta_{t-1} = Sinv_{t-1} z_{t-1}, delta_i = Sinv_i (z_i - B_i^T delta_{i+1}), y += delta.
__global__ __launch_bounds__(1024) void k_tri_refine(const TriDesc* __restrict__ descs, int t_launch,
                                                     const int32_t* __restrict__ act) {
  const TriDesc d = descs[blockIdx.z];
  if (!is_active(act, d.active) || !d.refine) return;
  const int m = d.m, tid = threadIdx.x;
  const int t = d.nblk > 0 ? d.nblk : t_launch;
  const int n = t * m;
  const int64_t mm = (int64_t)m * m;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  double* y = (double*)smem_raw;   // n
  double* R = y + n;               // n: residual, eliminated right-hand side, correction
  double* tmp = R + n;             // 1024 + m
  const bool apply = d.refine == 2;   // Y = (T + sigma I)^{-1} rhs for a right-hand side over all t blocks
  for (int e = tid; e < n; e += 1024) {
    y[e] = apply ? 0.0 : d.Y[(int64_t)e * d.ldy];
    if (apply) R[e] = d.mask[e] ? 0.0 : d.rhs[(int64_t)e * d.ld_rhs];
  }
  __syncthreads();
  // band part
  for (int e = tid; e < n && !apply; e += 1024) {
    const int i = e / m, a = e - i * m;
    const int32_t* mk = d.mask + (int64_t)i * m;
    if (mk[a]) {
      R[e] = 0.0;
      continue;
    }
    const double* Di = d.D + i * mm;
    double s = d.sigma * y[e];
    for (int c = 0; c < m; ++c) {
      if (mk[c]) continue;
      const double tac = (c == a) ? Di[a * m + a] : 0.5 * (Di[a * m + c] + Di[c * m + a]);
      s += tac * y[i * m + c];
    }
    if (i > 0) {   // T[i][i-1] = K_{i-1}: B_{i-1}[a][c], H_i[i-1][c][a]
      const double* Bp = d.Bsub + (i - 1) * mm;
      if (d.Hoff) {
        const double* Hp = d.Hoff + hoff_offset(i, m) + (i - 1) * mm;
        for (int c = 0; c < m; ++c) s += 0.5 * (Bp[a * m + c] + Hp[c * m + a]) * y[(i - 1) * m + c];
      } else {
        for (int c = 0; c < m; ++c) s += Bp[a * m + c] * y[(i - 1) * m + c];
      }
    }
    if (i + 1 < t) {   // T[i][i+1] = K_i^T: B_i[c][a], H_{i+1}[i][a][c]
      const double* Bi = d.Bsub + i * mm;
      if (d.Hoff) {
        const double* Hn = d.Hoff + hoff_offset(i + 1, m) + i * mm;
        for (int c = 0; c < m; ++c) s += 0.5 * (Bi[c * m + a] + Hn[a * m + c]) * y[(i + 1) * m + c];
      } else {
        for (int c = 0; c < m; ++c) s += Bi[c * m + a] * y[(i + 1) * m + c];
      }
    }
    R[e] = (i == 0 ? d.rhs[(int64_t)a * d.ld_rhs] : 0.0) - s;
  }
  __syncthreads();
  // off-band part, one block column j at a time
  if (d.Hoff && !apply) {
    const int slices = 1024 / m;
    for (int j = 2; j < t; ++j) {
      const double* H = d.Hoff + hoff_offset(j, m);   // rows of blocks 0 .. j - 2 (x m columns)
      const int rows = (j - 1) * m;
      const int32_t* mkj = d.mask + (int64_t)j * m;
      for (int rr = tid; rr < rows; rr += 1024) {
        if (d.mask[rr]) continue;   // masks of blocks 0 .. j - 2 are contiguous
        double s = 0.0;
        // four independent partial sums keep several loads in flight
        double s1 = 0.0, s2 = 0.0, s3 = 0.0;
        const double* hr = H + (int64_t)rr * m;
        const double* yj = y + j * m;
        int b = 0;
        for (; b + 3 < m; b += 4) {
          s += hr[b] * yj[b];
          s1 += hr[b + 1] * yj[b + 1];
          s2 += hr[b + 2] * yj[b + 2];
          s3 += hr[b + 3] * yj[b + 3];
        }
        for (; b < m; ++b) s += hr[b] * yj[b];
        s += (s1 + s2) + s3;
        R[rr] -= s;
      }
      const int b = tid % m, sl = tid / m;
      double s = 0.0;
      if (sl < slices)
      {
        double s1 = 0.0, s2 = 0.0, s3 = 0.0;
        int rr = sl;
        for (; rr + 3 * slices < rows; rr += 4 * slices) {
          s += H[(int64_t)rr * m + b] * y[rr];
          s1 += H[(int64_t)(rr + slices) * m + b] * y[rr + slices];
          s2 += H[(int64_t)(rr + 2 * slices) * m + b] * y[rr + 2 * slices];
          s3 += H[(int64_t)(rr + 3 * slices) * m + b] * y[rr + 3 * slices];
        }
        for (; rr < rows; rr += slices) s += H[(int64_t)rr * m + b] * y[rr];
        s += (s1 + s2) + s3;
      }
      tmp[tid] = s;
      __syncthreads();
      if (tid < m && !mkj[tid]) {
        double acc = 0.0;
        for (int q = 0; q < slices; ++q) acc += tmp[q * m + tid];
        R[j * m + tid] -= acc;
      }
      __syncthreads();
    }
  }
  // forward elimination with the stored factors U_i = B_i Sinv_i, then backward substitution
  // with Sinv_i.  Each m x m matrix-vector product spreads a row over tpr = 1024 / m threads
  // (each takes every tpr-th column, so consecutive threads read consecutive elements of the
  // row), and the row's tpr partial sums are combined through LDS.
  double* red = tmp + 1024 + m;   // 1024 partial sums
  const int tpr = 1024 / m;
  const int ra = tid / tpr, rj = tid - ra * tpr;
  auto mv_part = [&](const double* mat, bool trans, const double* xv) {
    double acc = 0.0;
    if (ra < m) {
      if (trans) {
        for (int u = rj; u < m; u += tpr) acc += mat[u * m + ra] * xv[u];
      } else {
        for (int u = rj; u < m; u += tpr) acc += mat[ra * m + u] * xv[u];
      }
    }
    red[tid] = acc;
    __syncthreads();
  };
  auto row_sum = [&](int a) {
    double acc = 0.0;
    for (int q = 0; q < tpr; ++q) acc += red[a * tpr + q];
    return acc;
  };
  for (int i = 0; i + 1 < t; ++i) {
    mv_part(d.Xw + i * mm, false, R + i * m);
    if (tid < m) R[(i + 1) * m + tid] -= row_sum(tid);
    __syncthreads();
  }
  for (int i = t - 1; i >= 0; --i) {
    if (i + 1 < t) {
      mv_part(d.Bsub + i * mm, true, R + (i + 1) * m);
      if (tid < m) tmp[tid] = R[i * m + tid] - row_sum(tid);
    } else if (tid < m) {
      tmp[tid] = R[i * m + tid];
    }
    __syncthreads();
    mv_part(d.Lw + i * mm, false, tmp);
    if (tid < m) R[i * m + tid] = row_sum(tid);
    __syncthreads();
  }
  for (int e = tid; e < n; e += 1024) d.Y[(int64_t)e * d.ldy] = y[e] + R[e];
}

hipError_t launch_tri_refine(const TriDesc* dd, int nz, int maxm, int maxr, int t, const int32_t* act,
                             hipStream_t st) {
  if (maxr != 1 || maxm < 1 || maxm > 1024) return hipErrorNotSupported;
  const size_t lds = ((size_t)2 * t * maxm + 2048 + maxm) * 8;
  if (lds > kLdsCap) return hipErrorNotSupported;
  static const hipError_t attr = set_big_lds((const void*)k_tri_refine);
  if (attr != hipSuccess) return attr;
  hipLaunchKernelGGL(k_tri_refine, dim3(1, 1, nz), dim3(1024), lds, st, dd, t, act);
  return hipGetLastError();
}

hipError_t launch_tri_forward(const TriDesc* dd, int nz, int maxm, int maxr, int j0, int j1, const int32_t* act,
                              hipStream_t st) {
  size_t lds = tri_forward_lds(maxm, maxr);
  if (lds > kLdsCap) return hipErrorInvalidValue;
  const size_t resident = ((size_t)3 * maxm * maxm + 2 * (size_t)maxm * maxr + 3 * (size_t)maxm) * 8;
  if (resident <= kLdsCap) lds = std::max(lds, resident);
  const int ns = (maxm + (1024 / maxm) - 1) / (1024 / maxm);   // rows per thread
  const void* kern;
  int slot;
  if (ns <= 1) { kern = (const void*)k_tri_forward<1>; slot = 0; }
  else if (ns <= 2) { kern = (const void*)k_tri_forward<2>; slot = 1; }
  else if (ns <= 5) { kern = (const void*)k_tri_forward<5>; slot = 2; }
  else if (ns <= 9) { kern = (const void*)k_tri_forward<9>; slot = 3; }
  else if (ns <= 14) { kern = (const void*)k_tri_forward<14>; slot = 4; }
  else if (ns <= 19) { kern = (const void*)k_tri_forward<19>; slot = 5; }
  else return hipErrorInvalidValue;
  static const hipError_t attr[6] = {
      set_big_lds((const void*)k_tri_forward<1>), set_big_lds((const void*)k_tri_forward<2>),
      set_big_lds((const void*)k_tri_forward<5>), set_big_lds((const void*)k_tri_forward<9>),
      set_big_lds((const void*)k_tri_forward<14>), set_big_lds((const void*)k_tri_forward<19>)};
  if (attr[slot] != hipSuccess) return attr[slot];
  int lb = (int)lds;
  void* args[] = {(void*)&dd, (void*)&j0, (void*)&j1, (void*)&lb, (void*)&act};
  return hipLaunchKernel(kern, dim3(1, 1, nz), dim3(1024), args, lds, st);
}

hipError_t launch_tri_backward(const TriDesc* dd, int nz, int maxm, int maxr, int t, const int32_t* act,
                               hipStream_t st) {
  static const hipError_t attr = set_big_lds((const void*)k_tri_backward);
  if (attr != hipSuccess) return attr;
  const size_t lds = tri_backward_lds(maxm, maxr);
  if (lds > kLdsCap) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_tri_backward, dim3(1, 1, nz), dim3(1024), lds, st, dd, t, act);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------------------------
// Gram matrix G = W^T W of one block of m <= 16 MT rows (W's rows are the block's vectors):
// workgroup s takes one range of k, stages it for all m rows in LDS in chunks of 32 and
// accumulates the whole m x m result on the FP64 16x16x4 MFMA (16 x 16 tiles dealt to the 4
// waves); partials part[s][c][i] = sum over the range of W[i][k] W[c][k] (reduced by k_finish,
// FIN_T2R).  Both operands of a tile come from the same LDS rows, so every value of W is read
// from memory once per launch.
// ---------------------------------------------------------------------------------------------
template <int MT>
__global__ __launch_bounds__(256) void k_gram(const NtDesc* __restrict__ descs, int splits,
                                              const int32_t* __restrict__ act) {
  constexpr int KC = 32, WS = KC + 1;
  constexpr int NTL = MT * MT, TPW = (NTL + 3) / 4;
  const NtDesc d = descs[blockIdx.z];
  if (!is_active(act, d.active)) return;
  const int m = d.M, s = blockIdx.x;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int r16 = lane & 15, kq = lane >> 4;
  const int kper = ((d.K + splits - 1) / splits + KC - 1) / KC * KC;
  const int kb = s * kper, ke = min(d.K, kb + kper);
  extern __shared__ __align__(16) unsigned char smem_raw[];
  double* ws = (double*)smem_raw;   // [16 MT][WS]
  const gmem_t<const double> W = gmem((const double*)d.P.p);
  v4d acc[TPW];
#pragma unroll
  for (int t = 0; t < TPW; ++t) acc[t] = v4d{0.0, 0.0, 0.0, 0.0};
  for (int kc = kb; kc < ke; kc += KC) {
    for (int e = tid; e < 16 * MT * KC; e += 256) {
      const int a = e / KC, kk = e - a * KC;
      ws[a * WS + kk] = (a < m && kc + kk < ke) ? W[row_off(d.P, a) + kc + kk] : 0.0;
    }
    __syncthreads();
#pragma unroll
    for (int k4 = 0; k4 < KC; k4 += 4) {
#pragma unroll
      for (int t = 0; t < TPW; ++t) {
        const int tile = wave + 4 * t;
        if (tile < NTL) {
          const int ti = tile / MT, tj = tile - ti * MT;
          const double x = ws[(16 * ti + r16) * WS + k4 + kq];
          const double y = ws[(16 * tj + r16) * WS + k4 + kq];
          acc[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(x, y, acc[t], 0, 0, 0);
        }
      }
    }
    __syncthreads();
  }
  const gmem_t<double> part = gmem(d.part);
#pragma unroll
  for (int t = 0; t < TPW; ++t) {
    const int tile = wave + 4 * t;
    if (tile >= NTL) continue;
    const int ti = tile / MT, tj = tile - ti * MT;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int i = 16 * ti + kq + 4 * r, c = 16 * tj + r16;
      if (i < m && c < m) part[((int64_t)s * m + c) * m + i] = acc[t][r];
    }
  }
}

bool gram_supported(int m) { return m >= 1 && m <= 80; }

hipError_t launch_gram(const NtDesc* dd, int nz, int maxm, int splits, const int32_t* act, hipStream_t st) {
  const int mt = (maxm + 15) / 16;
  if (maxm < 1 || mt > 5 || splits < 1) return hipErrorInvalidValue;
  const size_t lds = (size_t)16 * mt * (32 + 1) * 8;
  const dim3 grid(splits, 1, nz);
  switch (mt) {
    case 1: hipLaunchKernelGGL(k_gram<1>, grid, dim3(256), lds, st, dd, splits, act); break;
    case 2: hipLaunchKernelGGL(k_gram<2>, grid, dim3(256), lds, st, dd, splits, act); break;
    case 3: hipLaunchKernelGGL(k_gram<3>, grid, dim3(256), lds, st, dd, splits, act); break;
    case 4: hipLaunchKernelGGL(k_gram<4>, grid, dim3(256), lds, st, dd, splits, act); break;
    default: hipLaunchKernelGGL(k_gram<5>, grid, dim3(256), lds, st, dd, splits, act); break;
  }
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
    double v = d.src_t == DT_F64 ? gmem((const double*)d.src.p)[row_off(d.src, rr) + c]
                                 : (double)gmem((const float*)d.src.p)[row_off(d.src, rr) + c];
    if (d.dst_t == DT_F32) {
      gmem((float*)d.dst.p)[row_off(d.dst, rr) + c] = (float)v;
    } else if (d.dst_t == DT_F64) {
      gmem((double*)d.dst.p)[row_off(d.dst, rr) + c] = v;
    } else if (!d.split_lo) {
      gmem((unsigned short*)d.dst.p)[row_off(d.dst, rr) + c] = f32_to_bf16((float)v);
    } else {
      // three BF16 parts of the FP64 value (about 24 significant bits)
      const unsigned short hi = f32_to_bf16((float)v);
      const double r1 = v - (double)bf16_to_f32(hi);
      const unsigned short mid = f32_to_bf16((float)r1);
      const unsigned short lo = f32_to_bf16((float)(r1 - (double)bf16_to_f32(mid)));
      gmem((unsigned short*)d.dst.p)[row_off(d.dst, 3 * rr) + c] = hi;
      gmem((unsigned short*)d.dst.p)[row_off(d.dst, 3 * rr + 1) + c] = mid;
      gmem((unsigned short*)d.dst.p)[row_off(d.dst, 3 * rr + 2) + c] = lo;
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
// dst[c][r] = src[r][c] for a rows x cols FP32 matrix, stored as BF16 (OutBf16) or FP32; 32 x 32
// tiles through LDS, row tiles on grid x (up to 2^31 rows), column tiles on grid y.
template <bool OutBf16>
__global__ __launch_bounds__(256) void k_transpose(const float* __restrict__ src, int64_t ld, int rows, int cols,
                                                   void* __restrict__ dstv, int64_t ldt) {
  __shared__ float tile[32][33];
  const int64_t r0 = (int64_t)blockIdx.x * 32;
  const int c0 = blockIdx.y * 32;
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
  for (int y = ty; y < 32; y += 8) {
    const int64_t rr = r0 + y;
    const int cc = c0 + tx;
    tile[y][tx] = (rr < rows && cc < cols) ? src[rr * ld + cc] : 0.f;
  }
  __syncthreads();
  for (int y = ty; y < 32; y += 8) {
    const int cc = c0 + y;
    const int64_t rr = r0 + tx;
    if (cc >= cols || rr >= rows) continue;
    if constexpr (OutBf16)
      ((unsigned short*)dstv)[(int64_t)cc * ldt + rr] = f32_to_bf16(tile[tx][y]);
    else
      ((float*)dstv)[(int64_t)cc * ldt + rr] = tile[tx][y];
  }
}

static hipError_t launch_transpose(bool bf16, const float* src, int64_t ld, int rows, int cols, void* dst, int64_t ldt,
                                   hipStream_t st) {
  if (rows < 1 || cols < 1 || (cols + 31) / 32 > 65535) return hipErrorInvalidValue;
  dim3 grid((rows + 31) / 32, (cols + 31) / 32);
  if (bf16)
    hipLaunchKernelGGL(k_transpose<true>, grid, dim3(256), 0, st, src, ld, rows, cols, dst, ldt);
  else
    hipLaunchKernelGGL(k_transpose<false>, grid, dim3(256), 0, st, src, ld, rows, cols, dst, ldt);
  return hipGetLastError();
}

hipError_t launch_transpose_bf16(const float* src, int64_t ld, int rows, int cols, unsigned short* dst, int64_t ldt,
                                 hipStream_t st) {
  return launch_transpose(true, src, ld, rows, cols, dst, ldt, st);
}

hipError_t launch_transpose_f32(const float* src, int64_t ld, int rows, int cols, float* dst, int64_t ldt,
                                hipStream_t st) {
  return launch_transpose(false, src, ld, rows, cols, dst, ldt, st);
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
    const double v = rr < d.rows ? d.alpha * gmem((const double*)d.src.p)[row_off(d.src, rr) + c] : 0.0;
    gmem((double*)d.dst.p)[row_off(d.dst, rr) + c] = v;
  }
}

hipError_t launch_copy(const CopyDesc* dd, int nz, int maxRows, int maxN, const int32_t* act, hipStream_t st) {
  const int64_t tot = (int64_t)maxRows * maxN;
  int blocks = (int)std::min<int64_t>((tot + 255) / 256, 4096);
  if (blocks < 1) blocks = 1;
  hipLaunchKernelGGL(k_copy, dim3(blocks, 1, nz), dim3(256), 0, st, dd, act);
  return hipGetLastError();
}

__global__ __launch_bounds__(256) void k_fill(const FillDesc* __restrict__ descs, const int32_t* __restrict__ act) {
  const FillDesc d = descs[blockIdx.z];
  if (!is_active(act, d.active)) return;
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i >= d.n) return;
  int j = 0;
  for (int s = 0; s < d.m && j < d.src_avail; ++s) {
    if (!d.mask[s]) continue;
    gmem((double*)d.dst.p)[row_off(d.dst, s) + i] = gmem((const double*)d.src.p)[row_off(d.src, d.src_first + j) + i];
    ++j;
  }
}

hipError_t launch_fill(const FillDesc* dd, int nz, int maxN, const int32_t* act, hipStream_t st) {
  hipLaunchKernelGGL(k_fill, dim3((maxN + 255) / 256, 1, nz), dim3(256), 0, st, dd, act);
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
  if (*c.est <= (*c.tol) * (*c.scale)) {
    *c.active_flag = 0;
    *c.done_at = c.step;
    if (c.host_flag) __hip_atomic_store(c.host_flag, 0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
  }
}
hipError_t launch_converge(const ConvDesc* dd, int nz, hipStream_t st) {
  hipLaunchKernelGGL(k_converge, dim3((nz + 63) / 64), dim3(64), 0, st, dd, nz);
  return hipGetLastError();
}

}  // namespace rbcg

namespace rbcg {

// ---------------------------------------------------------------------------------------------
// Seeded Gaussian block: out[r][c] (r < rows, c < cols, row stride ld) = standard normal number
// e mod 2 of Philox4x32-10 call e / 2 (e = r cols + c), counter (lo32, hi32 of e / 2, stream, 0),
// key (lo32, hi32 of seed); the call's four words give two 53-bit uniforms in (0, 1) and the
// Box-Muller pair.  Philox4x32-10 as published (Salmon et al., SC 2011): ten rounds of
// multiply-high/low by 0xD2511F53 and 0xCD9E8D57 with the key bumped by 0x9E3779B9, 0xBB67AE85.
// ---------------------------------------------------------------------------------------------
__device__ __forceinline__ void philox4x32_10(uint32_t c[4], uint32_t k0, uint32_t k1) {
#pragma unroll
  for (int rnd = 0; rnd < 10; ++rnd) {
    if (rnd) {
      k0 += 0x9E3779B9u;
      k1 += 0xBB67AE85u;
    }
    const uint64_t p0 = (uint64_t)0xD2511F53u * c[0];
    const uint64_t p1 = (uint64_t)0xCD9E8D57u * c[2];
    const uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
    const uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
    const uint32_t n0 = hi1 ^ c[1] ^ k0, n2 = hi0 ^ c[3] ^ k1;
    c[0] = n0;
    c[1] = lo1;
    c[2] = n2;
    c[3] = lo0;
  }
}

__global__ __launch_bounds__(256) void k_gaussian(double* __restrict__ out, int64_t ld, int rows, int cols,
                                                  uint64_t seed, uint32_t stream) {
  const int64_t n = (int64_t)rows * cols;
  const int64_t ncall = (n + 1) / 2;
  for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < ncall; p += (int64_t)gridDim.x * blockDim.x) {
    uint32_t c[4] = {(uint32_t)p, (uint32_t)((uint64_t)p >> 32), stream, 0u};
    philox4x32_10(c, (uint32_t)seed, (uint32_t)(seed >> 32));
    const uint64_t a = (((uint64_t)c[0] << 32) | c[1]) >> 11;
    const uint64_t b = (((uint64_t)c[2] << 32) | c[3]) >> 11;
    const double u1 = ((double)a + 0.5) * 0x1p-53;
    const double u2 = ((double)b + 0.5) * 0x1p-53;
    const double r = sqrt(-2.0 * log(u1));
    const double th = 2.0 * 3.141592653589793 * u2;
    const double g[2] = {r * cos(th), r * sin(th)};
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int64_t e = 2 * p + h;
      if (e >= n) break;
      const int64_t rr = e / cols, cc = e - rr * cols;
      out[rr * ld + cc] = g[h];
    }
  }
}

hipError_t launch_gaussian(double* out, int64_t ld, int rows, int cols, uint64_t seed, uint32_t stream,
                           hipStream_t st) {
  const int64_t ncall = ((int64_t)rows * cols + 1) / 2;
  const int blocks = (int)std::max<int64_t>(1, std::min<int64_t>((ncall + 255) / 256, 8192));
  hipLaunchKernelGGL(k_gaussian, dim3(blocks), dim3(256), 0, st, out, ld, rows, cols, seed, stream);
  return hipGetLastError();
}

}  // namespace rbcg
