// Block product of the Gram operator A = Z^T Z with BF16 operands (the ridge-regression
// matrix-load, paper Sec. 1, eq. ridge_regression; one matrix-load per Krylov block, Sec. 1.2).
//
// Both passes are "NT" products with the right operand carried as three BF16 parts (hi + mid +
// lo, about 24 significant bits):
//     out(i, c) = sum_k P[i][k] * (X[3c][k] + X[3c+1][k] + X[3c+2][k])
//   pass 1: P = Z   (n x d), X = the Krylov block,  out = Y = Z X
//   pass 2: P = Z^T (d x n), X = Y,                 out = Z^T Y
// on the 16x16x32 BF16 MFMA with FP32 accumulation.  Both passes split k into ranges of about
// 1024 values and write FP32 partial sums; the partials are summed in FP64 (k_gram_combine forms
// the three BF16 parts of Y, k_finish the FP64 product).  Short FP32 chains matter: refinement at
// the small shifts of a ridge path contracts by about the rounding of Z itself (1e-3 per sweep)
// only when the accumulation error stays well below it along the small singular directions,
// whose sums cancel heavily.
//
// Workgroup: 8 waves (512 threads), one workgroup per CU (its double-buffered X image takes 111 KB
// of LDS) and two waves per SIMD.  Wave w owns 32 rows of P (RT = 2 tiles of 16) and every column
// tile of X, so a workgroup covers 256 rows; with 4 waves of 64 rows each the accumulators filled
// the accumulation registers and one wave per SIMD streamed Z (measured 1.03 ms per pass at the
// ridge workload's 129 columns, against 0.89 ms with 8 waves).  Per chunk of 64 values of k,
// each lane streams 32 bytes of each of its RT rows of P (row r16 of the tile, k = 16 q .. 16 q +
// 15, q = lane / 16) into registers, and the workgroup stages the X chunk (3 parts x 16 NT
// columns x 64 k, BF16) into a double-buffered LDS image; both are loaded one chunk ahead, their
// loads in flight while the MFMAs of the current chunk run.  The image is laid out [part][k-group
// g of 8][column][8 values] with one padding column per (part, g) so the stores of eight
// consecutive groups and the fragment reads of 16 consecutive columns both spread over the
// banks.  MFMA half h takes values 16 q + 8 h .. 16 q + 8 h + 7 of both operands (the k index is
// relabelled identically on both sides, which keeps every lane's loads contiguous).  D rows are
// columns c of X, D columns rows i of P, so stores run along i.
//
// The grid is laid out so that consecutive logical workgroups (the row tiles of one split of k,
// which read the same X chunk) land on the same XCD: workgroup b runs on XCD b % 8, and the
// logical index is (b % 8) * ceil(total / 8) + b / 8.
#include "device_common.inc"

namespace rbcg {

namespace {

constexpr int kGramW = 8;                    // waves per workgroup
constexpr int kGramThreads = 64 * kGramW;
constexpr int kGramRT = 16 / kGramW;         // row tiles of 16 per wave
constexpr int kGramRows = 16 * kGramRT * kGramW;  // rows of P per workgroup (256)
constexpr int kGramKC = 64;                  // k values per chunk
constexpr int kGramSplitK = 512;             // target k values per split (FP32 chain length)
constexpr int kParts = 3;

template <int NT>
struct GramLds {
  static constexpr int NR = 16 * NT;             // staged columns (zero beyond N)
  static constexpr int CS = NR + 1;              // column slots per (part, group), one of padding
  static constexpr int BUF = kParts * 8 * CS;    // 16-byte slots of one buffer
  static constexpr int ITEMS = kParts * 8 * NR;  // 16-byte items staged per chunk
  static constexpr int XP = (ITEMS + kGramThreads - 1) / kGramThreads;
  static constexpr size_t BYTES = (size_t)2 * BUF * 16;
  static_assert((size_t)kGramW * 16 * NR * 4 <= BYTES, "epilogue image must fit");
};

}  // namespace

template <int NT>
__global__ __launch_bounds__(kGramThreads, 1) void k_gram_bf16(const NtDesc* __restrict__ descs, int splits,
                                                      const int32_t* __restrict__ act) {
  typedef GramLds<NT> L;
  const NtDesc d = descs[blockIdx.z];
  if (!is_active(act, d.active)) return;
  const int ntiles = (d.M + kGramRows - 1) / kGramRows;
  const int total = ntiles * splits;
  const int per = (total + 7) / 8;
  const int logical = (int)(blockIdx.x % 8) * per + (int)(blockIdx.x / 8);
  if (logical >= total) return;
  const int s = logical / ntiles, tile = logical - s * ntiles;
  const int i0 = tile * kGramRows;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int q = lane >> 4, r16 = lane & 15;
  const int kper = ((d.K + splits - 1) / splits + kGramKC - 1) / kGramKC * kGramKC;
  const int kb = s * kper;
  const int ke = min(d.K, kb + kper);
  const int N = d.N;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  v8u* xs = (v8u*)smem_raw;   // [2][3][8][CS]

  // X staging: item it = (p * NR + c) * 8 + g, so eight consecutive threads read the 128 bytes
  // of one row's chunk
  const gmem_t<const unsigned short> xbase = gmem((const unsigned short*)d.X.p);
  v8u xreg[L::XP];
  auto load_x = [&](int kc) {
#pragma unroll
    for (int t = 0; t < L::XP; ++t) {
      const int it = tid + kGramThreads * t;
      v8u v = v8u{0, 0, 0, 0, 0, 0, 0, 0};
      if (it < L::ITEMS) {
        const int g = it & 7, pc = it >> 3;
        const int p = pc / L::NR, c = pc - p * L::NR;
        const int k = kc + 8 * g;
        if (c < N) {
          const gmem_t<const unsigned short> src = xbase + row_off(d.X, kParts * c + p);
          if (k + 8 <= ke) {
            v = *(gmem_t<const v8u>)(src + k);
          } else {
#pragma unroll
            for (int e = 0; e < 8; ++e) v[e] = k + e < ke ? src[k + e] : (unsigned short)0;
          }
        }
      }
      xreg[t] = v;
    }
  };
  auto store_x = [&](int buf) {
#pragma unroll
    for (int t = 0; t < L::XP; ++t) {
      const int it = tid + kGramThreads * t;
      if (it < L::ITEMS) {
        const int g = it & 7, pc = it >> 3;
        const int p = pc / L::NR, c = pc - p * L::NR;
        xs[buf * L::BUF + (p * 8 + g) * L::CS + c] = xreg[t];
      }
    }
  };

  // rows of P of this lane
  const gmem_t<const unsigned short> pbase = gmem((const unsigned short*)d.P.p);
  int64_t poff[kGramRT];
  bool pval[kGramRT];
#pragma unroll
  for (int rt = 0; rt < kGramRT; ++rt) {
    const int row = i0 + wave * 16 * kGramRT + rt * 16 + r16;
    pval[rt] = row < d.M;
    poff[rt] = pval[rt] ? row_off(d.P, row) : 0;
  }
  v8u an[kGramRT][2];
  auto load_a = [&](int kc, v8u (&dst)[kGramRT][2]) {
    const int k = kc + 16 * q;
#pragma unroll
    for (int rt = 0; rt < kGramRT; ++rt) {
      const gmem_t<const unsigned short> src = pbase + poff[rt];
      if (pval[rt] && k + 16 <= ke) {
        const gmem_t<const v8u> v = (gmem_t<const v8u>)(src + k);
        dst[rt][0] = v[0];
        dst[rt][1] = v[1];
      } else {
#pragma unroll
        for (int e = 0; e < 8; ++e) {
          dst[rt][0][e] = (pval[rt] && k + e < ke) ? src[k + e] : (unsigned short)0;
          dst[rt][1][e] = (pval[rt] && k + 8 + e < ke) ? src[k + 8 + e] : (unsigned short)0;
        }
      }
    }
  };

  v4f acc[kGramRT][NT];
#pragma unroll
  for (int rt = 0; rt < kGramRT; ++rt)
#pragma unroll
    for (int ct = 0; ct < NT; ++ct) acc[rt][ct] = v4f{0, 0, 0, 0};

  if (kb < ke) {
    load_a(kb, an);
    load_x(kb);
    store_x(0);
  }
  __syncthreads();
  int buf = 0;
  for (int kc = kb; kc < ke; kc += kGramKC) {
    const bool more = kc + kGramKC < ke;
    v8u anext[kGramRT][2];
    if (more) {   // the next chunk's loads fly while this chunk's MFMAs run
      load_a(kc + kGramKC, anext);
      load_x(kc + kGramKC);
    }
    const v8u* xb = xs + buf * L::BUF;
    // 2 NT groups (half h, column tile ct), each 3 fragment reads and 12 MFMAs; the next group's
    // fragments are read ahead of this group's MFMAs, and scheduling barriers keep the compiler
    // from hoisting every read of the chunk
    v8u bf[2][kParts];
#pragma unroll
    for (int p = 0; p < kParts; ++p) bf[0][p] = xb[(p * 8 + 2 * q) * L::CS + r16];
#pragma unroll
    for (int g = 0; g < 2 * NT; ++g) {
      const int h = g / NT, ct = g - h * NT;
      if (g + 1 < 2 * NT) {
        const int h1 = (g + 1) / NT, ct1 = (g + 1) - h1 * NT;
#pragma unroll
        for (int p = 0; p < kParts; ++p) bf[(g + 1) & 1][p] = xb[(p * 8 + 2 * q + h1) * L::CS + 16 * ct1 + r16];
      }
      __builtin_amdgcn_sched_barrier(0);
#pragma unroll
      for (int p = 0; p < kParts; ++p) {
        const v8bf b = __builtin_bit_cast(v8bf, bf[g & 1][p]);
#pragma unroll
        for (int rt = 0; rt < kGramRT; ++rt)
          acc[rt][ct] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(b, __builtin_bit_cast(v8bf, an[rt][h]), acc[rt][ct],
                                                                0, 0, 0);
      }
      __builtin_amdgcn_sched_barrier(0);
    }
    if (more) {
      store_x(buf ^ 1);
#pragma unroll
      for (int rt = 0; rt < kGramRT; ++rt) {
        an[rt][0] = anext[rt][0];
        an[rt][1] = anext[rt][1];
      }
    }
    __syncthreads();
    buf ^= 1;
  }

  // epilogue, one row tile at a time through LDS (the X image is free now): each wave dumps its
  // 16 x 16 NT tile as vals[c][16], then its lanes store the FP32 partials part[s][c][i] along i
  // (16 consecutive rows) for columns c = lane / 16 + 4 j; a runtime loop keeps the registers of
  // the stores few
  float* vals = (float*)smem_raw + wave * (16 * L::NR);
  const int ii = lane & 15, c0 = lane >> 4;
  const gmem_t<float> pb = gmem((float*)d.part);
#pragma unroll
  for (int rt = 0; rt < kGramRT; ++rt) {
    __syncthreads();
#pragma unroll
    for (int ct = 0; ct < NT; ++ct)
#pragma unroll
      for (int r = 0; r < 4; ++r) vals[(16 * ct + 4 * q + r) * 16 + r16] = acc[rt][ct][r];
    __syncthreads();
    const int i = i0 + wave * 16 * kGramRT + rt * 16 + ii;
    if (i >= d.M) continue;
#pragma unroll 1
    for (int c = c0; c < N; c += 4) pb[((int64_t)s * N + c) * d.M + i] = vals[c * 16 + ii];
  }
}

// Y = sum over splits of the FP32 partials part[s][c][i] (in FP64), stored as three BF16 parts
// in rows 3c, 3c + 1, 3c + 2 of O (element i).
__global__ __launch_bounds__(256) void k_gram_combine(const NtDesc* __restrict__ descs, int splits,
                                                      const int32_t* __restrict__ act) {
  const NtDesc d = descs[blockIdx.z];
  if (!is_active(act, d.active)) return;
  const int64_t total = (int64_t)d.N * d.M;
  const gmem_t<const float> pb = gmem((const float*)d.part);
  const gmem_t<unsigned short> ob = gmem((unsigned short*)d.O.p);
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
    const int c = (int)(e / d.M), i = (int)(e - (int64_t)c * d.M);
    double v = 0.0;
    for (int s = 0; s < splits; ++s) v += (double)pb[(int64_t)s * total + e];
    const unsigned short hi = f32_to_bf16((float)v);
    const double r1 = v - (double)bf16_to_f32(hi);
    const unsigned short mid = f32_to_bf16((float)r1);
    const unsigned short lo = f32_to_bf16((float)(r1 - (double)bf16_to_f32(mid)));
    ob[row_off(d.O, 3 * c) + i] = hi;
    ob[row_off(d.O, 3 * c + 1) + i] = mid;
    ob[row_off(d.O, 3 * c + 2) + i] = lo;
  }
}

template <int NT>
static hipError_t launch_gram_bf16_t(const NtDesc* dd, int nz, int maxM, int splits, const int32_t* act,
                                     hipStream_t st) {
  const size_t lds = GramLds<NT>::BYTES;
  auto kern = k_gram_bf16<NT>;
  static const hipError_t attr = hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize,
                                                     (int)lds);
  if (attr != hipSuccess) return attr;
  const int ntiles = (maxM + kGramRows - 1) / kGramRows;
  const int total = ntiles * splits;
  const int per = (total + 7) / 8;
  hipLaunchKernelGGL(kern, dim3(8 * per, 1, nz), dim3(kGramThreads), lds, st, dd, splits, act);
  return hipGetLastError();
}

int gram_bf16_splits(int K) { return std::max(1, (K + kGramSplitK - 1) / kGramSplitK); }

hipError_t launch_gram_bf16(const NtDesc* dd, int nz, int maxM, int maxN, int splits, const int32_t* act,
                            hipStream_t st) {
  switch ((maxN + 15) / 16) {
    case 1: return launch_gram_bf16_t<1>(dd, nz, maxM, splits, act, st);
    case 2: return launch_gram_bf16_t<2>(dd, nz, maxM, splits, act, st);
    case 3: return launch_gram_bf16_t<3>(dd, nz, maxM, splits, act, st);
    case 4: return launch_gram_bf16_t<4>(dd, nz, maxM, splits, act, st);
    case 5: return launch_gram_bf16_t<5>(dd, nz, maxM, splits, act, st);
    case 6: return launch_gram_bf16_t<6>(dd, nz, maxM, splits, act, st);
    case 7: return launch_gram_bf16_t<7>(dd, nz, maxM, splits, act, st);
    case 8: return launch_gram_bf16_t<8>(dd, nz, maxM, splits, act, st);
    case 9: return launch_gram_bf16_t<9>(dd, nz, maxM, splits, act, st);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_gram_combine(const NtDesc* dd, int nz, int maxM, int maxN, int splits, const int32_t* act,
                               hipStream_t st) {
  const int64_t tot = (int64_t)maxM * maxN;
  const int blocks = (int)std::min<int64_t>((tot + 255) / 256, 4096);
  hipLaunchKernelGGL(k_gram_combine, dim3(std::max(1, blocks), 1, nz), dim3(256), 0, st, dd, splits, act);
  return hipGetLastError();
}

}  // namespace rbcg
