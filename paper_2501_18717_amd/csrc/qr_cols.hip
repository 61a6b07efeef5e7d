// Pivoted Cholesky QR factor of a small Gram matrix, one lane per column.
//
// Contract (QrDesc): G = W^T W (m x m).  Outputs Mout (Q = W Mout), Bout (W = Q Bout, times
// prevB when given), the deflation mask per pivot position and the rank.  Pivot rule: the
// column with the largest remaining Schur diagonal relative to its own squared norm (rank
// revealing); a column is deflated when that ratio falls below tau, when its remaining norm is
// below sqrt(eta2) of its pre-projection norm, or when its Schur pivot is below floor2.
//
// Lane c owns column c of the Schur complement in registers (MMAX rows).  Per pivot step the
// owner of the pivot column publishes it to LDS (double-buffered, so one barrier per step
// suffices; two when several waves exchange their argmax), and every lane applies the rank-1
// update to its own column.  The triangular inverse and the coefficient product run from LDS
// with runtime loops, which keeps the code size independent of m.  R and the inverse both sit
// in LDS (2 m^2 doubles), so the kernel takes m <= 96; wider blocks use k_qr_factor.
#include "device_common.inc"

namespace rbcg {

__device__ __forceinline__ void argmax_wave(double& v, int& i) {
  // maximum value, smallest index on ties, across the 64 lanes of a wave
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    const double ov = __shfl_xor(v, off, 64);
    const int oi = __shfl_xor(i, off, 64);
    if (ov > v || (ov == v && oi < i)) { v = ov; i = oi; }
  }
}

__device__ __forceinline__ double max_wave(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_xor(v, off, 64));
  return v;
}

// LDS layout (doubles first, then ints), for block width m and row capacity MMAX:
//   Rl    m*m         R rows by pivot position, columns in W's order (later: in pivot order)
//   Xl    m*m         columns of Rhat^{-1} (lane-private slots Xl[a*m + c])
//   prow  2*(MMAX+2)  published pivot column, its reference norm and pre-projection norm
//   wv    8           per-wave argmax values (double-buffered) / reductions
//   wi    8           per-wave argmax indices
//   perm  m           pivot position -> column of W
//   kept  m           per pivot position
inline size_t qr_cols_lds(int m, int mmax) {
  return ((size_t)2 * m * m + 2 * ((size_t)mmax + 2) + 8) * 8 + (8 + 2 * (size_t)m) * 4 + 16;
}

template <int MMAX>
__global__ __launch_bounds__(192) void k_qr_cols(const QrDesc* __restrict__ descs, const int32_t* __restrict__ act) {
  const QrDesc d = descs[blockIdx.z];
  if (!is_active(act, d.active)) return;
  const int m = d.m;
  const int nt = blockDim.x;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, nw = nt >> 6;
  const int c = tid;
  const bool own = c < m;
  constexpr int PB = MMAX + 2;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  double* Rl = (double*)smem_raw;
  double* Xl = Rl + m * m;
  double* prow = Xl + m * m;
  double* wv = prow + 2 * PB;
  int* wi = (int*)(wv + 8);
  int* perm = wi + 8;
  int* kept = perm + m;

  // ---- second pass on a near-identity Gram: G = I + E over the non-zero columns with
  //      max |E| <= 1e-8 gives R = I + F (F = upper part of E, halved diagonal) and
  //      R^{-1} = I - F, both exact to O(|E|^2) = rounding level; no sequential factorization.
  if (!d.pivot && d.prevB) {
    double emax = 0.0;
    for (int e = tid; e < m * m; e += nt) {
      const int a = e / m, cc = e - a * m;
      const double ga = d.G[(int64_t)a * d.ldg + a], gc = d.G[(int64_t)cc * d.ldg + cc];
      if (ga == 0.0 || gc == 0.0) continue;   // deflated (zero) columns
      const double g = d.G[(int64_t)a * d.ldg + cc];
      emax = fmax(emax, fabs(g - (a == cc ? 1.0 : 0.0)));
    }
    emax = max_wave(emax);
    if (lane == 0) wv[wave] = emax;
    __syncthreads();
    double mx = 0.0;
    for (int w = 0; w < nw; ++w) mx = fmax(mx, wv[w]);
    if (mx <= 1e-8) {
      for (int i = tid; i < m; i += nt) kept[i] = d.G[(int64_t)i * d.ldg + i] != 0.0;
      __syncthreads();
      for (int e = tid; e < m * m; e += nt) {
        const int a = e / m, cc = e - a * m;
        double f = 0.0;
        if (kept[a] && kept[cc] && cc >= a) {
          const double g = d.G[(int64_t)a * d.ldg + cc];
          f = (a == cc) ? 0.5 * (g - 1.0) : g;
        }
        Rl[e] = f;
        d.Mout[e] = (kept[a] && kept[cc]) ? ((a == cc ? 1.0 : 0.0) - f) : 0.0;
      }
      for (int i = tid; i < m; i += nt) d.mask[i] = kept[i] ? 0 : 1;
      if (tid == 0 && d.rank_out) {
        int rk = 0;
        for (int i = 0; i < m; ++i) rk += kept[i];
        *d.rank_out = rk;
      }
      __syncthreads();
      // Bout column c = (I + F) prevB column c, rows of deflated positions zero
      if (own) {
        double acc[MMAX];
#pragma unroll
        for (int s0 = 0; s0 < MMAX; ++s0) acc[s0] = 0.0;
        for (int u = 0; u < m; ++u) {
          const double pb = d.prevB[(int64_t)u * m + c];
#pragma unroll
          for (int s0 = 0; s0 < MMAX; ++s0)
            if (s0 < m && s0 <= u) acc[s0] += (s0 == u ? 1.0 + Rl[s0 * m + u] : Rl[s0 * m + u]) * pb;
        }
#pragma unroll
        for (int s0 = 0; s0 < MMAX; ++s0)
          if (s0 < m) d.Bout[(int64_t)s0 * m + c] = kept[s0] ? acc[s0] : 0.0;
      }
      return;
    }
    __syncthreads();
  }

  // ---- pivoted (or in-order) Cholesky with deflation
  double v[MMAX];
#pragma unroll
  for (int a = 0; a < MMAX; ++a) v[a] = (own && a < m) ? d.G[(int64_t)a * d.ldg + c] : 0.0;
  double diag = own ? d.G[(int64_t)c * d.ldg + c] : 0.0;
  const double dref = diag;
  const double pre = (own && d.pre) ? d.pre[(int64_t)c * d.pre_stride] : -1.0;
  bool chosen = !own;
  for (int e = tid; e < m * m; e += nt) Rl[e] = 0.0;
  for (int i = tid; i < m; i += nt) {
    perm[i] = i;
    kept[i] = 0;
  }
  // chosen columns as a uniform bitmask (identical in every lane)
  uint64_t ch0 = 0, ch1 = 0, ch2 = 0;
  __syncthreads();

  int s = 0, rank = 0;
  for (; s < m; ++s) {
    const int buf = s & 1;
    double* pr = prow + buf * PB;
    int p = s;
    if (d.pivot && !(d.force_first && s == 0)) {
      double rel = chosen ? -2.0 : (dref > 0.0 ? diag / dref : -1.0);
      int bi = chosen ? 0x7fffffff : c;
      argmax_wave(rel, bi);
      if (nw > 1) {
        if (lane == 0) {
          wv[buf * 4 + wave] = rel;
          wi[buf * 4 + wave] = bi;
        }
        __syncthreads();
        rel = wv[buf * 4];
        bi = wi[buf * 4];
        for (int w = 1; w < nw; ++w) {
          const double ov = wv[buf * 4 + w];
          const int oi = wi[buf * 4 + w];
          if (ov > rel || (ov == rel && oi < bi)) { rel = ov; bi = oi; }
        }
      }
      p = __builtin_amdgcn_readfirstlane(bi);
    }
    // the owner of column p publishes it (the Schur row p, by symmetry), zero on chosen rows
    if (c == p) {
#pragma unroll
      for (int a = 0; a < MMAX; ++a) {
        const uint64_t w = a < 64 ? ch0 : (a < 128 ? ch1 : ch2);
        if (a < m) pr[a] = ((w >> (a & 63)) & 1) ? 0.0 : v[a];
      }
      pr[MMAX] = dref;
      pr[MMAX + 1] = pre;
    }
    __syncthreads();
    const double piv2 = pr[p];
    const double drp = pr[MMAX], prp = pr[MMAX + 1];
    bool defl;
    if (d.force_first && s == 0) defl = !(piv2 > 0.0);
    else
      defl = !(drp > 0.0) || !(piv2 > d.tau * drp) || (prp >= 0.0 && !(piv2 > d.eta2 * prp)) ||
             !(piv2 > d.floor2);
    if (defl && d.pivot) break;   // every remaining column is at least as deficient
    const uint64_t bit = 1ull << (p & 63);
    if (p < 64) ch0 |= bit; else if (p < 128) ch1 |= bit; else ch2 |= bit;
    if (c == p) chosen = true;
    if (tid == 0) perm[s] = p;
    if (defl) continue;
    if (tid == 0) kept[s] = 1;
    ++rank;
    const double rp = sqrt(piv2);
    const double irp = 1.0 / rp;
    // my factor: R[s][c] (zero for columns chosen before this step)
    double rc = 0.0;
    if (own) {
      if (c == p) rc = rp;
      else if (!chosen) rc = pr[c] * irp;
      Rl[s * m + c] = rc;
    }
    // rank-1 update of my column; pr[a] is zero on chosen rows, and row p of column p
    // becomes rp^2 - rp^2
    if (rc != 0.0) {
#pragma unroll
      for (int a = 0; a < MMAX; a += 2) {
        if (a < m) {
          const double2 q = *(const double2*)(pr + a);
          const double r0 = (a == p) ? rp : q.x * irp;
          const double r1 = (a + 1 == p) ? rp : q.y * irp;
          v[a] -= r0 * rc;
          v[a + 1] -= r1 * rc;
        }
      }
      diag -= rc * rc;
    }
  }
  __syncthreads();
  if (tid == 0) {
    // positions after the break take the remaining columns, in order, as deflated
    int pos = s;
    uint64_t c0 = ch0, c1 = ch1, c2 = ch2;
    for (int i = 0; i < m && pos < m; ++i) {
      const uint64_t w = i < 64 ? c0 : (i < 128 ? c1 : c2);
      if (!((w >> (i & 63)) & 1)) perm[pos++] = i;
    }
  }
  __syncthreads();

  // ---- reported coefficient block Bout = R (times prevB); rows of deflated positions zero
  if (own) {
    if (d.prevB) {
      double acc[MMAX];
#pragma unroll
      for (int s0 = 0; s0 < MMAX; ++s0) acc[s0] = 0.0;
      for (int u = 0; u < m; ++u) {
        const double pb = d.prevB[(int64_t)u * m + c];
#pragma unroll
        for (int s0 = 0; s0 < MMAX; ++s0)
          if (s0 < m) acc[s0] += Rl[s0 * m + u] * pb;   // rows of deflated positions are zero
      }
#pragma unroll
      for (int s0 = 0; s0 < MMAX; ++s0)
        if (s0 < m) d.Bout[(int64_t)s0 * m + c] = kept[s0] ? acc[s0] : 0.0;
    } else {
      for (int s0 = 0; s0 < m; ++s0) d.Bout[(int64_t)s0 * m + c] = kept[s0] ? Rl[s0 * m + c] : 0.0;
    }
  }
  for (int i = tid; i < m; i += nt) d.mask[i] = kept[i] ? 0 : 1;
  if (tid == 0 && d.rank_out) *d.rank_out = rank;

  // ---- Rl columns into pivot order (Rhat[s][u] = R[s][perm[u]]), in place
  double col[MMAX];
  if (own) {
    const int pc = perm[c];
#pragma unroll
    for (int s0 = 0; s0 < MMAX; ++s0) col[s0] = s0 < m ? Rl[s0 * m + pc] : 0.0;
  }
  __syncthreads();
  if (own) {
#pragma unroll
    for (int s0 = 0; s0 < MMAX; ++s0)
      if (s0 < m) Rl[s0 * m + c] = col[s0];
  }
  __syncthreads();

  // ---- X = Rhat^{-1}, lane c computes column c (pivot positions), kept positions only:
  //      X[q][c] = (delta_qc - sum_{q < u <= c} Rhat[q][u] X[u][c]) / Rhat[q][q], q = c .. 0
  if (own) {
    const bool kc = kept[c];
    for (int q = m - 1; q >= 0; --q) {
      double x = 0.0;
      if (kc && q <= c && kept[q]) {
        const double* Rq = Rl + q * m;
        double a0 = (q == c) ? 1.0 : 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
        int u = q + 1;
        for (; u + 3 <= c; u += 4) {
          a0 -= Rq[u] * Xl[u * m + c];
          a1 -= Rq[u + 1] * Xl[(u + 1) * m + c];
          a2 -= Rq[u + 2] * Xl[(u + 2) * m + c];
          a3 -= Rq[u + 3] * Xl[(u + 3) * m + c];
        }
        for (; u <= c; ++u) a0 -= Rq[u] * Xl[u * m + c];
        x = ((a0 + a1) + (a2 + a3)) / Rq[q];
      }
      Xl[q * m + c] = x;
    }
    // Mout[perm[a]][c] = X[a][c]  (Q column c = sum_a W column a * Mout[a][c])
    for (int a = 0; a < m; ++a) d.Mout[(int64_t)perm[a] * m + c] = Xl[a * m + c];
  }
}

hipError_t launch_qr_cols(const QrDesc* dd, int nz, int maxm, const int32_t* act, hipStream_t st) {
  if (maxm < 1 || maxm > kQrColsMax) return hipErrorInvalidValue;
  const int mmax = (maxm + 15) / 16 * 16;
  const size_t lds = qr_cols_lds(maxm, mmax);
  if (lds > kLdsCap) return hipErrorInvalidValue;
  const void* kern;
  int slot;
  switch (mmax) {
    case 16: kern = (const void*)k_qr_cols<16>; slot = 0; break;
    case 32: kern = (const void*)k_qr_cols<32>; slot = 1; break;
    case 48: kern = (const void*)k_qr_cols<48>; slot = 2; break;
    case 64: kern = (const void*)k_qr_cols<64>; slot = 3; break;
    case 80: kern = (const void*)k_qr_cols<80>; slot = 4; break;
    default: kern = (const void*)k_qr_cols<96>; slot = 5; break;
  }
  static bool attr[6] = {false, false, false, false, false, false};
  if (!attr[slot]) {
    hipFuncAttributes fa;
    hipError_t e = hipFuncGetAttributes(&fa, kern);
    if (e != hipSuccess) return e;
    e = hipFuncSetAttribute(kern, hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024 - (int)fa.sharedSizeBytes);
    if (e != hipSuccess) return e;
    attr[slot] = true;
  }
  const int threads = 64 * ((maxm + 63) / 64);
  void* args[] = {(void*)&dd, (void*)&act};
  return hipLaunchKernel(kern, dim3(1, 1, nz), dim3(threads), args, lds, st);
}

}  // namespace rbcg
