// Pivoted Cholesky QR factor of a small Gram matrix, one lane per column, for the block
// widths m = k + 1 with k a power of two (9, 17, 33, 65, 129), compiled for that exact m.
//
// Contract (QrDesc): G = W^T W (m x m).  Outputs Mout (Q = W Mout), Bout (W = Q Bout, times
// prevB when given), the deflation mask per pivot position and the rank.  Pivot rule: the
// column with the largest remaining Schur diagonal relative to its own squared norm (rank
// revealing); a column is deflated when that ratio falls below tau, when its remaining norm is
// below sqrt(eta2) of its pre-projection norm, or when its Schur pivot is below floor2.
//
// Lane c owns column c of the Schur complement in registers.  Per pivot step the owner of the
// pivot column publishes it to LDS (double-buffered, so one barrier per step suffices; two when
// several waves exchange their argmax), and every lane applies the rank-1 update to its own
// column from 16-byte LDS broadcast reads.  With m fixed at compile time every loop over rows
// is unrolled without guards.
#include "device_common.inc"

namespace rbcg {

// Maximum of a 32-bit key over the 64 lanes of a wave: four DPP stages give every lane the
// maximum of its row of 16, then the four row maxima are read out (uniform result).
__device__ __forceinline__ unsigned wave_max_key(unsigned v) {
  v = max(v, (unsigned)__builtin_amdgcn_update_dpp(0, (int)v, 0xB1, 0xF, 0xF, false));    // quad_perm 1,0,3,2
  v = max(v, (unsigned)__builtin_amdgcn_update_dpp(0, (int)v, 0x4E, 0xF, 0xF, false));    // quad_perm 2,3,0,1
  v = max(v, (unsigned)__builtin_amdgcn_update_dpp(0, (int)v, 0x141, 0xF, 0xF, false));   // row_half_mirror
  v = max(v, (unsigned)__builtin_amdgcn_update_dpp(0, (int)v, 0x140, 0xF, 0xF, false));   // row_mirror
  const unsigned r0 = __builtin_amdgcn_readlane(v, 0), r1 = __builtin_amdgcn_readlane(v, 16);
  const unsigned r2 = __builtin_amdgcn_readlane(v, 32), r3 = __builtin_amdgcn_readlane(v, 48);
  return max(max(r0, r1), max(r2, r3));
}

// Pivot key of column c: priority class in the top bits (candidate with a non-negative relative
// Schur diagonal > candidate with a negative one (rounding) > column with no norm > chosen),
// then the relative diagonal as a float truncated to 16 mantissa bits, then 255 - c so that
// near-ties go to the smallest column index.
__device__ __forceinline__ unsigned pivot_key(bool chosen, double diag, double idref, bool has_norm, int c) {
  if (chosen) return 0u;
  const unsigned idx = 255u - (unsigned)c;
  if (!has_norm) return 0x20000000u | idx;
  const float rel = (float)(diag * idref);
  if (!(rel >= 0.0f)) return 0x40000000u | idx;
  return 0x80000000u | (((unsigned)__float_as_uint(rel) >> 1) & ~0xFFu) | idx;
}

__device__ __forceinline__ double max_wave(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_xor(v, off, 64));
  return v;
}

// LDS layout for block width M (row stride MP = M rounded up to even):
//   Rl    M*MP       R rows by pivot position (columns in W's order); later the transpose of
//                    Rhat (row u = column u of Rhat, in pivot order); fast path: F rows
//   prow  2*(MP+2)   published pivot column + its reference and pre-projection norms
//   wv    8, wi 8    per-wave argmax (double-buffered) and reductions
//   perm  M, kept M  pivot position -> column of W; kept flag per pivot position
inline size_t qr_m_lds(int M) {
  const int MP = (M + 1) & ~1;
  return ((size_t)M * MP + 2 * ((size_t)MP + 2) + 8) * 8 + (8 + 2 * (size_t)M) * 4 + 16;
}

template <int M>
__global__ __launch_bounds__(64 * ((M + 63) / 64)) void k_qr_m(const QrDesc* __restrict__ descs,
                                                               const int32_t* __restrict__ act) {
  constexpr int NW = (M + 63) / 64;
  constexpr int NT = 64 * NW;
  constexpr int MP = (M + 1) & ~1;
  constexpr int PB = MP + 2;
  const QrDesc d = descs[blockIdx.z];
  if (!is_active(act, d.active)) return;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int c = tid;
  const bool own = c < M;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  double* Rl = (double*)smem_raw;
  double* prow = Rl + M * MP;
  double* wv = prow + 2 * PB;
  int* wi = (int*)(wv + 8);
  int* perm = wi + 8;
  int* kept = perm + M;
  const double* __restrict__ G = d.G;
  const int64_t ldg = d.ldg;

  // ---- second pass on a near-identity Gram: G = I + E over the non-zero columns with
  //      max |E| <= 1e-8 gives R = I + F (F = upper part of E, halved diagonal) and
  //      R^{-1} = I - F, both exact to O(|E|^2) = rounding level; no sequential factorization.
  if (!d.pivot && d.prevB) {
    double emax = 0.0;
    for (int e = tid; e < M * M; e += NT) {
      const int a = e / M, cc = e - a * M;
      const double ga = G[(int64_t)a * ldg + a], gc = G[(int64_t)cc * ldg + cc];
      if (ga == 0.0 || gc == 0.0) continue;   // deflated (zero) columns
      emax = fmax(emax, fabs(G[(int64_t)a * ldg + cc] - (a == cc ? 1.0 : 0.0)));
    }
    emax = max_wave(emax);
    if (lane == 0) wv[wave] = emax;
    __syncthreads();
    double mx = wv[0];
#pragma unroll
    for (int w = 1; w < NW; ++w) mx = fmax(mx, wv[w]);
    if (mx <= 1e-8) {
      for (int i = tid; i < M; i += NT) kept[i] = G[(int64_t)i * ldg + i] != 0.0;
      __syncthreads();
      for (int e = tid; e < M * MP; e += NT) {
        const int a = e / MP, cc = e - a * MP;
        double f = 0.0;
        if (cc < M && kept[a] && kept[cc] && cc >= a) {
          const double g = G[(int64_t)a * ldg + cc];
          f = (a == cc) ? 0.5 * (g - 1.0) : g;
        }
        Rl[e] = (a == cc) ? 1.0 + f : f;   // rows of R = I + F
        if (cc < M) d.Mout[a * M + cc] = (kept[a] && kept[cc]) ? ((a == cc ? 1.0 : 0.0) - f) : 0.0;
      }
      for (int i = tid; i < M; i += NT) d.mask[i] = kept[i] ? 0 : 1;
      if (tid == 0 && d.rank_out) {
        int rk = 0;
        for (int i = 0; i < M; ++i) rk += kept[i];
        *d.rank_out = rk;
      }
      __syncthreads();
      // Bout column c = (I + F) prevB column c; rows of deflated positions zero (their row of
      // I + F is a unit row, masked here)
      if (own) {
        double pb[MP];
#pragma unroll
        for (int u = 0; u < MP; ++u) pb[u] = u < M ? d.prevB[u * M + c] : 0.0;
        for (int s0 = 0; s0 < M; ++s0) {
          const double* Fs = Rl + s0 * MP;
          double a0 = 0.0, a1 = 0.0;
#pragma unroll
          for (int u = 0; u < MP; u += 2) {
            const double2 f2 = *(const double2*)(Fs + u);
            a0 = fma(f2.x, pb[u], a0);
            a1 = fma(f2.y, pb[u + 1], a1);
          }
          d.Bout[s0 * M + c] = kept[s0] ? a0 + a1 : 0.0;
        }
      }
      return;
    }
    __syncthreads();
  }

  // ---- pivoted (or in-order) Cholesky with deflation
  double v[MP];
#pragma unroll
  for (int a = 0; a < MP; ++a) v[a] = (own && a < M) ? G[(int64_t)a * ldg + c] : 0.0;
  double diag = own ? G[(int64_t)c * ldg + c] : 0.0;
  const double dref = diag;
  const double idref = dref > 0.0 ? 1.0 / dref : 0.0;
  const double pre = (own && d.pre) ? d.pre[(int64_t)c * d.pre_stride] : -1.0;
  bool chosen = !own;
  for (int e = tid; e < M * MP; e += NT) Rl[e] = 0.0;
  for (int i = tid; i < M; i += NT) {
    perm[i] = i;
    kept[i] = 0;
  }
  uint64_t ch[NW];   // chosen columns as a uniform bitmask (identical in every lane)
#pragma unroll
  for (int w = 0; w < NW; ++w) ch[w] = 0;
  __syncthreads();

  int s = 0, rank = 0;
  for (; s < M; ++s) {
    const int buf = s & 1;
    double* pr = prow + buf * PB;
    int p = s;
    if (d.pivot && !(d.force_first && s == 0)) {
      unsigned key = wave_max_key(pivot_key(chosen, diag, idref, dref > 0.0, c));
      if constexpr (NW > 1) {
        if (lane == 0) wi[buf * 4 + wave] = (int)key;
        __syncthreads();
        key = (unsigned)wi[buf * 4];
#pragma unroll
        for (int w = 1; w < NW; ++w) key = max(key, (unsigned)wi[buf * 4 + w]);
      }
      p = (int)(255u - (key & 0xFFu));
    }
    // The owner of column p publishes it (the Schur row p, by symmetry); entry p is the pivot
    // itself, so r_a = pr[a] / sqrt(pivot) for every row a.  Entries in rows chosen earlier are
    // rounding leftovers: they only ever update other chosen rows, which nothing reads.
    if (c == p) {
#pragma unroll
      for (int a = 0; a < MP; a += 2) *(double2*)(pr + a) = double2{v[a], v[a + 1]};
      pr[MP] = dref;
      pr[MP + 1] = pre;
    }
    __syncthreads();
    const double piv2 = pr[p];
    const double drp = pr[MP], prp = pr[MP + 1];
    bool defl;
    if (d.force_first && s == 0) defl = !(piv2 > 0.0);
    else
      defl = !(drp > 0.0) || !(piv2 > d.tau * drp) || (prp >= 0.0 && !(piv2 > d.eta2 * prp)) ||
             !(piv2 > d.floor2);
    if (defl && d.pivot) break;   // every remaining column is at least as deficient
    const bool was_chosen = chosen;
#pragma unroll
    for (int w = 0; w < NW; ++w)
      if ((p >> 6) == w) ch[w] |= 1ull << (p & 63);
    if (c == p) chosen = true;
    if (tid == 0) perm[s] = p;
    if (defl) continue;
    if (tid == 0) kept[s] = 1;
    ++rank;
    const double irp = 1.0 / sqrt(piv2);
    // my factor R[s][c] (zero for columns chosen before this step; rp for the pivot column)
    const double rc = (own && !was_chosen) ? pr[c] * irp : 0.0;
    if (own) Rl[s * MP + c] = rc;
    const double f = rc * irp;
#pragma unroll
    for (int a = 0; a < MP; a += 2) {
      const double2 q = *(const double2*)(pr + a);
      v[a] = fma(-q.x, f, v[a]);
      v[a + 1] = fma(-q.y, f, v[a + 1]);
    }
    diag -= rc * rc;
  }
  __syncthreads();
  if (tid == 0) {
    // positions after the break take the remaining columns, in order, as deflated
    int pos = s;
#pragma unroll
    for (int w = 0; w < NW; ++w)
      for (int i = 64 * w; i < M && i < 64 * w + 64; ++i)
        if (!((ch[w] >> (i & 63)) & 1)) perm[pos++] = i;
  }
  __syncthreads();

  // ---- reported coefficient block Bout = R (times prevB); rows of deflated positions zero
  if (own) {
    if (d.prevB) {
      double pb[MP];
#pragma unroll
      for (int u = 0; u < MP; ++u) pb[u] = u < M ? d.prevB[u * M + c] : 0.0;
      for (int s0 = 0; s0 < M; ++s0) {
        const double* Rs = Rl + s0 * MP;
        double a0 = 0.0, a1 = 0.0;
#pragma unroll
        for (int u = 0; u < MP; u += 2) {
          const double2 r2 = *(const double2*)(Rs + u);
          a0 = fma(r2.x, pb[u], a0);
          a1 = fma(r2.y, pb[u + 1], a1);
        }
        d.Bout[s0 * M + c] = kept[s0] ? a0 + a1 : 0.0;
      }
    } else {
      for (int s0 = 0; s0 < M; ++s0) d.Bout[s0 * M + c] = kept[s0] ? Rl[s0 * MP + c] : 0.0;
    }
    d.mask[c] = kept[c] ? 0 : 1;
  }
  if (tid == 0 && d.rank_out) *d.rank_out = rank;

  // ---- transpose of Rhat into Rl: row u = column u of Rhat = column perm[u] of R
  double col[MP];
  if (own) {
    const int pc = perm[c];
#pragma unroll
    for (int s0 = 0; s0 < MP; ++s0) col[s0] = s0 < M ? Rl[s0 * MP + pc] : 0.0;
  }
  __syncthreads();
  if (own) {
#pragma unroll
    for (int s0 = 0; s0 < MP; s0 += 2) *(double2*)(Rl + c * MP + s0) = double2{col[s0], col[s0 + 1]};
  }
  __syncthreads();

  // ---- X = Rhat^{-1} by a right-looking sweep; lane c holds column c (pivot positions):
  //      for q = M-1 .. 0 (kept): X[q][c] /= Rhat[q][q]; X[a][c] -= Rhat[a][q] X[q][c], a < q
  if (own) {
    double x[MP];
#pragma unroll
    for (int a = 0; a < MP; ++a) x[a] = (a == c) ? 1.0 : 0.0;
#pragma unroll
    for (int q = M - 1; q >= 0; --q) {
      if (kept[q]) {
        const double* Rq = Rl + q * MP;   // column q of Rhat
        const double xq = x[q] / Rq[q];
        x[q] = xq;
#pragma unroll
        for (int a = 0; a + 1 < q; a += 2) {
          const double2 r2 = *(const double2*)(Rq + a);
          x[a] = fma(-r2.x, xq, x[a]);
          x[a + 1] = fma(-r2.y, xq, x[a + 1]);
        }
        if (q & 1) x[q - 1] = fma(-Rq[q - 1], xq, x[q - 1]);
      }
    }
    // Mout[perm[a]][c] = X[a][c] for kept a <= c (Q column c = sum_a W column a * Mout[a][c])
    const bool kc = kept[c];
#pragma unroll
    for (int a = 0; a < M; ++a) d.Mout[perm[a] * M + c] = (kc && kept[a] && a <= c) ? x[a] : 0.0;
  }
}

template <int M>
static hipError_t launch_qr_m_t(const QrDesc* dd, int nz, const int32_t* act, hipStream_t st) {
  const size_t lds = qr_m_lds(M);
  if (lds > kLdsCap) return hipErrorInvalidValue;
  const void* kern = (const void*)k_qr_m<M>;
  static bool attr = false;
  if (!attr) {
    hipFuncAttributes fa;
    hipError_t e = hipFuncGetAttributes(&fa, kern);
    if (e != hipSuccess) return e;
    e = hipFuncSetAttribute(kern, hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024 - (int)fa.sharedSizeBytes);
    if (e != hipSuccess) return e;
    attr = true;
  }
  void* args[] = {(void*)&dd, (void*)&act};
  return hipLaunchKernel(kern, dim3(1, 1, nz), dim3(64 * ((M + 63) / 64)), args, lds, st);
}

bool qr_m_supported(int m) { return m == 9 || m == 17 || m == 33 || m == 65 || m == 129; }

hipError_t launch_qr_m(const QrDesc* dd, int nz, int m, const int32_t* act, hipStream_t st) {
  switch (m) {
    case 9: return launch_qr_m_t<9>(dd, nz, act, st);
    case 17: return launch_qr_m_t<17>(dd, nz, act, st);
    case 33: return launch_qr_m_t<33>(dd, nz, act, st);
    case 65: return launch_qr_m_t<65>(dd, nz, act, st);
    case 129: return launch_qr_m_t<129>(dd, nz, act, st);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace rbcg
