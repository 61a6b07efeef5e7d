// Pivoted Cholesky QR factor of a small Gram matrix for the block widths m = k + 1 with k a
// power of two (9, 17, 33, 65, 129), compiled for that exact m.
//
// Contract (QrDesc): G = W^T W (m x m).  Outputs Mout (Q = W Mout), Bout (W = Q Bout, times
// prevB when given), the deflation mask per pivot position and the rank.  Pivot rule: the
// column with the largest remaining Schur diagonal relative to its own squared norm (rank
// revealing); a column is deflated when that ratio falls below tau, when its remaining norm is
// below sqrt(eta2) of its pre-projection norm, or when its Schur pivot is below floor2.
//
// The factorization runs in a 2D block-cyclic register layout (one wave for m <= 33, four
// waves for m = 65 and 129), the pivot column published through double-buffered LDS.  The
// common case is an unpivoted attempt that carries the inverse factor along (k_qr_np); the
// pivoted redo forms the triangular inverse and the outputs one lane per column.  With m fixed
// at compile time every loop over rows is unrolled.
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


// LDS layout for block width M (row stride MP = M rounded up to even):
//   Rl    M*MP       R rows by pivot position (columns in W's order); later the transpose of
//                    Rhat (row u = column u of Rhat, in pivot order)
//   prow  2*(MP+2)   published pivot column + its reference and pre-projection norms
//   wi    8 (+8)     per-wave argmax keys (double-buffered); s and rank after the loop
//   perm  M, kept M  pivot position -> column of W; kept flag per pivot position
//   rinv  M          1 / Rhat[s][s] of kept positions
//   erow  2*MP       (unpivoted attempt) published row of the inverse factor, double-buffered
template <int M>
struct QrLds {   // byte offsets (compile-time, so every access stays an LDS access)
  static constexpr size_t MP = (M + 1) & ~1;
  static constexpr size_t prow = (size_t)M * MP * 8;
  static constexpr size_t wi = prow + 2 * (MP + 2) * 8;
  static constexpr size_t perm = wi + 16 * 4;
  static constexpr size_t kept = perm + (size_t)M * 4;
  static constexpr size_t rinv = (kept + (size_t)M * 4 + 15) & ~(size_t)15;
  static constexpr size_t erow = rinv + MP * 8;
  static constexpr size_t bytes = erow + 2 * MP * 8;
};

// Outputs of a factorization whose R rows (by pivot position, columns in W's order) are in Rl:
// Bout, mask, rank, and Mout = the columns of Rhat^{-1} placed by perm.  One lane per column.
template <int M>
__device__ __forceinline__ void qr_epilogue(const QrDesc& d, double* Rl, const int* perm, const int* kept,
                                            const double* rinv, int rank, int tid) {
  constexpr int MP = (M + 1) & ~1;
  const int c = tid;
  const bool own = c < M;

  // ---- reported coefficient block Bout = R (times prevB); rows of deflated positions zero
  if (own) {
    if (d.prevB) {
      double pb[MP];
#pragma unroll
      for (int u = 0; u < MP; ++u) pb[u] = u < M ? gmem(d.prevB)[u * M + c] : 0.0;
      for (int s0 = 0; s0 < M; ++s0) {
        const double* Rs = Rl + s0 * MP;
        double a0 = 0.0, a1 = 0.0;
#pragma unroll
        for (int u = 0; u < MP; u += 2) {
          const double2 r2 = *(const double2*)(Rs + u);
          a0 = fma(r2.x, pb[u], a0);
          a1 = fma(r2.y, pb[u + 1], a1);
        }
        gmem(d.Bout)[s0 * M + c] = kept[s0] ? a0 + a1 : 0.0;
      }
    } else {
      for (int s0 = 0; s0 < M; ++s0) gmem(d.Bout)[s0 * M + c] = kept[s0] ? Rl[s0 * MP + c] : 0.0;
    }
    gmem(d.mask)[c] = kept[c] ? 0 : 1;
  }
  if (tid == 0 && d.rank_out) *gmem(d.rank_out) = rank;

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
        const double xq = x[q] * rinv[q];
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
    for (int a = 0; a < M; ++a) gmem(d.Mout)[perm[a] * M + c] = (kc && kept[a] && a <= c) ? x[a] : 0.0;
  }
}

// Factorization in a 2D block-cyclic layout: the GR x GR lanes of the first NWF waves own
// element (a, c) of the Schur complement in register slot (a / GR, c / GR) when a % GR and
// c % GR are the lane's row and column index.  Per pivot step a lane needs only the S = M / GR
// pivot-column values of its rows and of its columns, and applies S x S register FMAs.  The
// triangular inverse and the outputs then run one lane per column.
template <int M, int GR, int NWF>
__device__ __forceinline__ void qr_pivoted(const QrDesc& d) {
  constexpr int NWC = (M + 63) / 64;               // waves for the one-lane-per-column phases
  constexpr int NT = 64 * (NWC > NWF ? NWC : NWF);
  static_assert(GR * GR == 64 * NWF, "lane grid must fill the factorization waves");
  static_assert(NWF == 1 || NWF == NT / 64, "either one factorization wave or all waves");
  constexpr int S = (M + GR - 1) / GR;             // register slots per dimension
  constexpr int MP = (M + 1) & ~1;
  constexpr int PB = MP + 2;
  constexpr int NCH = (M + 63) / 64;               // 64-bit words of the chosen-column mask
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  using L = QrLds<M>;
  double* Rl = (double*)smem_raw;
  double* prow = (double*)(smem_raw + L::prow);
  int* wi = (int*)(smem_raw + L::wi);
  int* perm = (int*)(smem_raw + L::perm);
  int* kept = (int*)(smem_raw + L::kept);
  double* rinv = (double*)(smem_raw + L::rinv);   // 1 / Rhat[s][s]
  const gmem_t<const double> G = gmem(d.G);
  const int64_t ldg = d.ldg;

  for (int e = tid; e < M * MP; e += NT) Rl[e] = 0.0;
  for (int i = tid; i < M; i += NT) {
    perm[i] = i;
    kept[i] = 0;
  }
  __syncthreads();

  if (wave < NWF) {
    const int rl = tid % GR, cl = tid / GR;
    const bool dl = rl == cl;                       // holds diagonal elements (slot (i, i))
    double v[S][S];
#pragma unroll
    for (int i = 0; i < S; ++i)
#pragma unroll
      for (int j = 0; j < S; ++j) {
        const int a = rl + GR * i, c = cl + GR * j;
        v[i][j] = (a < M && c < M) ? G[(int64_t)a * ldg + c] : 0.0;
      }
    double dref[S], idref[S], pre[S];
#pragma unroll
    for (int i = 0; i < S; ++i) {
      const int a = rl + GR * i;
      dref[i] = (dl && a < M) ? v[i][i] : 0.0;
      idref[i] = dref[i] > 0.0 ? 1.0 / dref[i] : 0.0;
      pre[i] = (dl && a < M && d.pre) ? gmem(d.pre)[(int64_t)a * d.pre_stride] : -1.0;
    }
    uint64_t ch[NCH];
#pragma unroll
    for (int w = 0; w < NCH; ++w) ch[w] = 0;
    // chosen flags of this lane's diagonal slots (slot i <-> column rl + GR i); slots beyond M
    // count as chosen
    unsigned mych = 0u;
#pragma unroll
    for (int i = 0; i < S; ++i)
      if (rl + GR * i >= M) mych |= 1u << i;
    auto chosen = [&](int a) -> bool {
      uint64_t w = ch[0];
#pragma unroll
      for (int k = 1; k < NCH; ++k)
        if ((a >> 6) == k) w = ch[k];
      return (w >> (a & 63)) & 1;
    };
    auto sync = [&]() {
      if constexpr (NWF > 1) __syncthreads();
      else __builtin_amdgcn_wave_barrier();
    };
    int s = 0, rank = 0;
    for (; s < M; ++s) {
      const int buf = s & 1;
      double* pr = prow + buf * PB;
      int p = s;
      if (d.pivot && !(d.force_first && s == 0)) {
        unsigned key = 0u;
        if (dl) {
#pragma unroll
          for (int i = 0; i < S; ++i)
            if (!((mych >> i) & 1u)) key = max(key, pivot_key(false, v[i][i], idref[i], dref[i] > 0.0, rl + GR * i));
        }
        if constexpr (NWF == 1) {
          // only the GR diagonal lanes (lane rl + GR rl) hold candidates
          unsigned k2 = (unsigned)__builtin_amdgcn_readlane((int)key, 0);
#pragma unroll
          for (int r = 1; r < GR; ++r) k2 = max(k2, (unsigned)__builtin_amdgcn_readlane((int)key, r * (GR + 1)));
          key = k2;
        } else {
          key = wave_max_key(key);
        }
        if constexpr (NWF > 1) {
          if (lane == 0) wi[buf * 4 + wave] = (int)key;
          __syncthreads();
          key = (unsigned)wi[buf * 4];
#pragma unroll
          for (int w = 1; w < NWF; ++w) key = max(key, (unsigned)wi[buf * 4 + w]);
        }
        p = (int)(255u - (key & 0xFFu));
      }
      // publish column p (the Schur row p, by symmetry) from its owners; entry p is the pivot
      // itself.  Entries in rows chosen earlier are rounding leftovers that only ever update
      // other chosen rows, which nothing reads.
      const int jp = __builtin_amdgcn_readfirstlane(p / GR);
      // slot column jp is uniform: one scalar branch per candidate slot (the scheduling barrier
      // keeps the compiler from turning the cases into per-element selects)
#pragma unroll
      for (int j = 0; j < S; ++j) {
        if (j == jp) {
          __builtin_amdgcn_sched_barrier(0);
          if (cl == p % GR) {
#pragma unroll
            for (int i = 0; i < S; ++i) {
              const int a = rl + GR * i;
              if (a < M) pr[a] = v[i][j];
            }
            if (dl) {
              pr[MP] = dref[j];
              pr[MP + 1] = pre[j];
            }
          }
        }
      }
      sync();
      const double piv2 = pr[p];
      const double drp = pr[MP], prp = pr[MP + 1];
      bool defl;
      if (d.force_first && s == 0) defl = !(piv2 > 0.0);
      else
        defl = !(drp > 0.0) || !(piv2 > d.tau * drp) || (prp >= 0.0 && !(piv2 > d.eta2 * prp)) ||
               !(piv2 > d.floor2);
      if (defl && d.pivot) break;   // every remaining column is at least as deficient
      double ra[S], rc[S];
      bool cb[S];                     // column chosen before this step
#pragma unroll
      for (int i = 0; i < S; ++i) {
        const int a = rl + GR * i, c = cl + GR * i;
        ra[i] = a < M ? pr[a] : 0.0;
        rc[i] = c < M ? pr[c] : 0.0;
        cb[i] = c < M ? chosen(c) : true;
      }
#pragma unroll
      for (int w = 0; w < NCH; ++w)
        if ((p >> 6) == w) ch[w] |= 1ull << (p & 63);
      if (dl && rl == p % GR) mych |= 1u << (p / GR);
      if (tid == 0) perm[s] = p;
      if (defl) continue;
      ++rank;
      const double irp = 1.0 / sqrt(piv2);
      if (tid == 0) {
        kept[s] = 1;
        rinv[s] = irp;
      }
      const double f = irp * irp;
      if (rl == 0) {
#pragma unroll
        for (int j = 0; j < S; ++j) {
          const int c = cl + GR * j;
          if (c < M) Rl[s * MP + c] = cb[j] ? 0.0 : rc[j] * irp;
        }
      }
#pragma unroll
      for (int i = 0; i < S; ++i) {
        const double ri = ra[i] * f;
#pragma unroll
        for (int j = 0; j < S; ++j) v[i][j] = fma(-ri, rc[j], v[i][j]);
      }
      // no barrier here: step s + 1 publishes into the other buffer, and step s + 2 reuses this
      // one only after every wave has passed step s + 1's publication barrier
    }
    if (tid == 0) {
      // positions after the break take the remaining columns, in order, as deflated
      int pos = s;
      for (int i = 0; i < M && pos < M; ++i)
        if (!chosen(i)) perm[pos++] = i;
      wi[8] = rank;
    }
  }
  __syncthreads();
  qr_epilogue<M>(d, Rl, perm, kept, rinv, wi[8], tid);
}

// Unpivoted attempt at the same factorization, for the common case of a well-conditioned block:
// the pivot of step s is column s, so the loop over s runs by register-slot column and the pivot
// column's slot is a compile-time constant (no argmax, no slot selection).  The inverse factor is
// carried in the same lane grid: the row operations that reduce G = L D L^T (L unit lower
// triangular) to upper triangular form turn the identity into E = L^{-1}, and Rhat^{-1} =
// E^T D^{-1/2}, so Mout leaves the registers without a separate triangular inversion.  Slots
// that no later step reads (Schur entries left of or above the pivot block, E entries right of
// it) are never touched, E slot columns start as identity columns when their block begins, and
// finished E slot rows are written out at the end of their block.  Any relative Schur pivot
// below max(tau, 1e-8), or any deflation test that fires, aborts the attempt, and the same
// workgroup redoes the factorization with pivoting (whose outputs overwrite the attempt's).
template <int M, int GR, int NWF>
__global__ __launch_bounds__(64 * ((M + 63) / 64 > NWF ? (M + 63) / 64 : NWF))
void k_qr_np(const QrDesc* __restrict__ descs, const int32_t* __restrict__ act) {
  constexpr int NWC = (M + 63) / 64;
  constexpr int NT = 64 * (NWC > NWF ? NWC : NWF);
  static_assert(GR * GR == 64 * NWF, "lane grid must fill the factorization waves");
  static_assert(NWF == 1 || NWF == NT / 64, "either one factorization wave or all waves");
  constexpr int S = (M + GR - 1) / GR;
  constexpr int MP = (M + 1) & ~1;
  constexpr int PB = MP + 2;
  const QrDesc d = descs[blockIdx.z];
  if (!is_active(act, d.active)) return;
  // the diagonal block of T: by the waves the factorization leaves idle, else up front
  if (NWF == NT / 64 && d.dg.D) diag_block(d.dg, threadIdx.x, NT);
  const int tid = threadIdx.x, wave = tid >> 6;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  using L = QrLds<M>;
  double* Rl = (double*)smem_raw;
  double* prow = (double*)(smem_raw + L::prow);
  int* wi = (int*)(smem_raw + L::wi);
  double* erow = (double*)(smem_raw + L::erow);   // 2 x MP: published row of E (double-buffered)
  const gmem_t<const double> G = gmem(d.G);
  const int64_t ldg = d.ldg;
  const double tau = fmax(d.tau, 1e-8);
  // rows of R go to LDS as they are formed (Bout leaves after the loop, or as R prevB); the pad
  // column is read by the R prevB product
  const bool keepR = d.prevB != nullptr;
  if (keepR && (M & 1))
    for (int e = tid; e < M; e += NT) Rl[e * MP + M] = 0.0;

  if (wave < NWF) {
    const int rl = tid % GR, cl = tid / GR;
    const bool dl = rl == cl;
    double v[S][S], e[S][S];
#pragma unroll
    for (int i = 0; i < S; ++i)
#pragma unroll
      for (int j = 0; j < S; ++j) {
        const int a = rl + GR * i, c = cl + GR * j;
        v[i][j] = (a < M && c < M) ? G[(int64_t)a * ldg + c] : 0.0;
      }
    // per column the bound its Schur pivot must exceed (every deflation test in one number):
    // max(tau dref, eta2 pre (when known), floor2), +inf when the column has no norm; only 0 for
    // a forced first column
    double thr[S], rv[S];
#pragma unroll
    for (int i = 0; i < S; ++i) {
      const int a = rl + GR * i;
      const double dref = (dl && a < M) ? v[i][i] : 0.0;
      const double pre = (dl && a < M && d.pre) ? gmem(d.pre)[(int64_t)a * d.pre_stride] : -1.0;
      double t = fmax(tau * dref, d.floor2);
      if (pre >= 0.0) t = fmax(t, d.eta2 * pre);
      if (!(dref > 0.0)) t = INFINITY;
      if (d.force_first && a == 0) t = 0.0;
      thr[i] = t;
      rv[i] = 0.0;
    }
    bool ok = true;
    static_for<S>([&](auto jc) {
      constexpr int js = decltype(jc)::value;
      // E slot column js enters as identity columns
#pragma unroll
      for (int i = js; i < S; ++i) e[i][js] = (rl + GR * i == cl + GR * js) ? 1.0 : 0.0;
#pragma nounroll
      for (int r = 0; r < GR; ++r) {
        const int s = GR * js + r;
        if (s >= M || !ok) break;   // uniform
        double* pr = prow + (s & 1) * PB;
        double* pq = erow + (s & 1) * MP;
        if (cl == r) {   // Schur column s (rows of later pivots; earlier rows are never read)
#pragma unroll
          for (int i = js; i < S; ++i) {
            const int a = rl + GR * i;
            if (a < M) pr[a] = v[i][js];
          }
          if (dl) pr[MP] = thr[js];
        }
        if (rl == r) {   // row s of E (final: its last update was step s - 1)
#pragma unroll
          for (int j = 0; j <= js; ++j) {
            const int c = cl + GR * j;
            if (c < M) pq[c] = e[js][j];
          }
        }
        if constexpr (NWF > 1) __syncthreads();
        else __builtin_amdgcn_wave_barrier();
        // every value this step needs, read at once
        const double piv2 = pr[s];
        const double thp = pr[MP];
        double ra[S], rc[S], re[S];
#pragma unroll
        for (int i = js; i < S; ++i) {
          const int a = rl + GR * i, c = cl + GR * i;
          ra[i] = a < M ? pr[a] : 0.0;
          rc[i] = c < M ? pr[c] : 0.0;
        }
#pragma unroll
        for (int j = 0; j <= js; ++j) {
          const int c = cl + GR * j;
          re[j] = c < M ? pq[c] : 0.0;
        }
        if (!(piv2 > thp)) {
          ok = false;
          break;
        }
        const bool fast = pos_in_range(piv2);
        const double f = fast ? recip_pos(piv2) : 1.0 / piv2;
#pragma unroll
        for (int i = js; i < S; ++i) {
          const double li = ra[i] * f;
#pragma unroll
          for (int j = js; j < S; ++j) v[i][j] = fma(-li, rc[j], v[i][j]);
        }
#pragma unroll
        for (int i = js; i < S; ++i) {
          double li = ra[i] * f;
          if (i == js && rl <= r) li = 0.0;   // rows up to the pivot are final
#pragma unroll
          for (int j = 0; j <= js; ++j) e[i][j] = fma(-li, re[j], e[i][j]);
        }
        const double irp = fast ? rsqrt_pos(piv2) : 1.0 / sqrt(piv2);
        if (rl == r) rv[js] = irp;
        if (rl == 0) {   // row s of R: zero left of the pivot
#pragma unroll
          for (int j = 0; j < S; ++j) {
            const int c = cl + GR * j;
            if (c < M) Rl[s * MP + c] = (j >= js && c >= s) ? rc[j] * irp : 0.0;
          }
        }
      }
      // E slot row js is final: Mout[b][a] = E[a][b] / sqrt(D[a]) (zero for b > a)
      if (ok) {
        const int a = rl + GR * js;
        if (a < M) {
#pragma unroll
          for (int j = 0; j < S; ++j) {
            const int b = cl + GR * j;
            if (b < M) gmem(d.Mout)[(int64_t)b * M + a] = j <= js ? e[js][j] * rv[js] : 0.0;
          }
        }
      }
    });
    if (tid == 0) wi[8] = ok ? M : -1;
  } else if (d.dg.D) {
    diag_block(d.dg, tid - 64 * NWF, NT - 64 * NWF);
  }
  __syncthreads();
  if (wi[8] < 0) {   // uniform: redo the factorization with pivoting
    // the attempt already stored rows of Mout; those stores must be complete before the redo
    // stores the same addresses from other lanes
    __threadfence();
    __syncthreads();
    qr_pivoted<M, GR, NWF>(d);
    return;
  }
  for (int c = tid; c < M; c += NT) gmem(d.mask)[c] = 0;
  if (tid == 0 && d.rank_out) *gmem(d.rank_out) = M;
  if (!keepR)
    for (int e = tid; e < M * M; e += NT) gmem(d.Bout)[e] = Rl[(e / M) * MP + e % M];
  if (keepR) {   // Bout = R prevB, one lane per column
    const int c = tid;
    if (c < M) {
      double pb[MP];
#pragma unroll
      for (int u = 0; u < MP; ++u) pb[u] = u < M ? gmem(d.prevB)[u * M + c] : 0.0;
      for (int s0 = 0; s0 < M; ++s0) {
        const double* Rs = Rl + s0 * MP;
        double a0 = 0.0, a1 = 0.0;
#pragma unroll
        for (int u = 0; u < MP; u += 2) {
          const double2 r2 = *(const double2*)(Rs + u);
          a0 = fma(r2.x, pb[u], a0);
          a1 = fma(r2.y, pb[u + 1], a1);
        }
        gmem(d.Bout)[s0 * M + c] = a0 + a1;
      }
    }
  }
}

template <int M, int GR, int NWF>
static hipError_t launch_qr_m_t(const QrDesc* dd, int nz, const int32_t* act, hipStream_t st) {
  constexpr size_t lds = QrLds<M>::bytes;
  if (lds > kLdsCap) return hipErrorInvalidValue;
  const void* kern = (const void*)k_qr_np<M, GR, NWF>;
  static const hipError_t attr = [&] {   // once per process, thread-safe
    hipFuncAttributes fa;
    hipError_t e = hipFuncGetAttributes(&fa, kern);
    if (e == hipSuccess)
      e = hipFuncSetAttribute(kern, hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024 - (int)fa.sharedSizeBytes);
    return e;
  }();
  if (attr != hipSuccess) return attr;
  void* args[] = {(void*)&dd, (void*)&act};
  constexpr int NWC = (M + 63) / 64;
  const dim3 block(64 * (NWC > NWF ? NWC : NWF));
  return hipLaunchKernel(kern, dim3(1, 1, nz), block, args, lds, st);
}

bool qr_m_supported(int m) { return m == 9 || m == 17 || m == 33 || m == 65 || m == 129; }

hipError_t launch_qr_m(const QrDesc* dd, int nz, int m, const int32_t* act, hipStream_t st) {
  switch (m) {
    case 9: return launch_qr_m_t<9, 8, 1>(dd, nz, act, st);
    case 17: return launch_qr_m_t<17, 8, 1>(dd, nz, act, st);
    case 33: return launch_qr_m_t<33, 8, 1>(dd, nz, act, st);
    case 65: return launch_qr_m_t<65, 16, 4>(dd, nz, act, st);
    case 129: return launch_qr_m_t<129, 16, 4>(dd, nz, act, st);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace rbcg
