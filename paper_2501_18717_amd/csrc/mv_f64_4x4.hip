// FP64 tall block product on the 4x4x4 FP64 MFMA (four independent 4x4x4 blocks per
// instruction): out(i, c) = sum_k P[i][k] X[c][k] for many rows i and 33 <= N <= 144 vectors c,
// P in FP64, or in FP32 widened to FP64 in registers (the Gram operator's FP64 products).
// On gfx950 this instruction issues FP64 multiply-adds at the rate of the 16x16x4 one, and its
// 4-column granularity wastes less of a width such as 65 (68 columns instead of 80).
//
// Lane layout of the instruction (measured on the device): lane l = 16 q + 4 b + x belongs to
// block b; block b's A element (row m, depth k) is at lane 16 k + 4 b + m, its B element (depth
// k, column n) at lane 16 k + 4 b + n, its D element (m, n) at lane 16 m + 4 b + n.
//
// Tiling.  A workgroup owns 64 rows with 4 waves (the row tiling of the 16x16x4 tall kernel, so
// split counts and partial buffers carry over); wave w owns rows 16 w .. 16 w + 15 and lane
// (q, b, x) supplies the A element of row 16 w + 4 b + x.  Every lane holds the B elements of
// all CG column groups (columns 4 j + x), the same for the four blocks, so one instruction per
// column group j forms block b's 4 x 4 tile (rows 16 w + 4 b + m, columns 4 j + n).  Per chunk of
// KC values of k the depth index is relabelled identically for both operands: at step s
// (0..KC/4-1) lane quarter q takes k = kc + (KC/4) q + s, so each lane streams KC/4 consecutive
// values of its row of P, one chunk ahead in registers, and reads its B values of a column group
// as contiguous bytes of the chunk of X staged in LDS (double-buffered, rows padded by 4 doubles).
// D element (m, n) of tile j at lane (q = m, b, x = n) is out(16 w + 4 b + m, 4 j + n).
// KC = 32 (the launches below) halves the barriers and staging rounds of KC = 16; measured on
// gfx950 it is as fast or faster at every shape of the solvers (widths 33-129, d 2000-16384).
#include "device_common.inc"

namespace rbcg {

template <int CG, int KC, bool PVEC, typename PT>
__global__ __launch_bounds__(256) void k_mv_tall44(const NtDesc* __restrict__ descs, int splits,
                                                   const int32_t* __restrict__ act) {
  static_assert(KC == 16 || KC == 32, "chunk of 4 or 8 values of k per lane");
  constexpr int KPL = KC / 4;                // consecutive values of k per lane and chunk
  constexpr int VPR = KC / 2;                // 16-byte items per staged row and chunk
  constexpr int XS = KC + 4;                 // LDS row stride (doubles; 16-byte aligned rows)
  constexpr int NR = 4 * CG;                 // staged X rows (zero beyond N)
  constexpr int XIT = NR * VPR;              // 16-byte items staged per chunk
  constexpr int XP = (XIT + 255) / 256;
  const NtDesc d = descs[blockIdx.z];
  if (!is_active(act, d.active)) return;
  const int i0 = blockIdx.x * 64;
  if (i0 >= d.M) return;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int q = lane >> 4, b = (lane >> 2) & 3, x = lane & 3;
  const int s = blockIdx.y;
  const int kper = ((d.K + splits - 1) / splits + KC - 1) / KC * KC;
  const int kb = s * kper;
  const int ke = min(d.K, kb + kper);
  const int N = d.N;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  double* xs = (double*)smem_raw;            // [2][NR][XS]

  // X staging: item it = r * VPR + v (row r, pair v of the chunk)
  const gmem_t<const double> xbase = gmem((const double*)d.X.p);
  v2d xreg[XP];
  auto load_x = [&](int kc) {
#pragma unroll
    for (int t = 0; t < XP; ++t) {
      const int it = tid + 256 * t;
      v2d v = v2d{0.0, 0.0};
      if (it < XIT) {
        const int r = it / VPR, k = kc + 2 * (it % VPR);
        if (r < N) {
          const gmem_t<const double> src = xbase + row_off(d.X, r);
          if (k + 2 <= ke && ((uintptr_t)(src + k) & 15) == 0) {
            v = *(gmem_t<const v2d>)(src + k);
          } else {
            v[0] = k < ke ? src[k] : 0.0;
            v[1] = k + 1 < ke ? src[k + 1] : 0.0;
          }
        }
      }
      xreg[t] = v;
    }
  };
  auto store_x = [&](int buf) {
#pragma unroll
    for (int t = 0; t < XP; ++t) {
      const int it = tid + 256 * t;
      if (it < XIT) *(v2d*)(xs + buf * (NR * XS) + (it / VPR) * XS + 2 * (it % VPR)) = xreg[t];
    }
  };

  // this lane's row of P (A operand; FP32 values are widened to FP64 in registers)
  const int prow = i0 + wave * 16 + 4 * b + x;
  const bool pval = prow < d.M;
  const gmem_t<const PT> pp = gmem((const PT*)d.P.p) + (pval ? row_off(d.P, prow) : 0);
  double ar[KPL];
  auto load_a = [&](int kc) {
    const int k = kc + KPL * q;
    if (pval && k + KPL <= ke) {   // whole run in range: no per-element checks
      if constexpr (PVEC && sizeof(PT) == 8) {
#pragma unroll
        for (int t = 0; t < KPL / 2; ++t) {
          const v2d u = *(gmem_t<const v2d>)(pp + k + 2 * t);
          ar[2 * t] = u[0];
          ar[2 * t + 1] = u[1];
        }
      } else if constexpr (PVEC) {
#pragma unroll
        for (int t = 0; t < KPL / 4; ++t) {
          const v4f u = *(gmem_t<const v4f>)(pp + k + 4 * t);
#pragma unroll
          for (int e = 0; e < 4; ++e) ar[4 * t + e] = (double)u[e];
        }
      } else {
#pragma unroll
        for (int e = 0; e < KPL; ++e) ar[e] = (double)pp[k + e];
      }
    } else {
#pragma unroll
      for (int e = 0; e < KPL; ++e) ar[e] = (pval && k + e < ke) ? (double)pp[k + e] : 0.0;
    }
  };

  double acc[CG];
#pragma unroll
  for (int j = 0; j < CG; ++j) acc[j] = 0.0;

  int buf = 0;
  if (kb < ke) {
    load_x(kb);
    load_a(kb);
    store_x(0);
  }
  __syncthreads();
  for (int kc = kb; kc < ke; kc += KC) {
    double cur[KPL];
#pragma unroll
    for (int e = 0; e < KPL; ++e) cur[e] = ar[e];
    const bool more = kc + KC < ke;
    if (more) {   // the next chunk's loads fly while this chunk's MFMAs run
      load_x(kc + KC);
      load_a(kc + KC);
    }
    // column group j: the lane's B values for the KPL steps are X[4 j + x][kc + KPL q + 0..KPL-1]
    const double* xb = xs + buf * (NR * XS) + x * XS + KPL * q;
#pragma unroll
    for (int j = 0; j < CG; ++j) {
#pragma unroll
      for (int t = 0; t < KPL / 2; ++t) {
        const v2d bb = *(const v2d*)(xb + 4 * j * XS + 2 * t);
        acc[j] = __builtin_amdgcn_mfma_f64_4x4x4f64(cur[2 * t], bb[0], acc[j], 0, 0, 0);
        acc[j] = __builtin_amdgcn_mfma_f64_4x4x4f64(cur[2 * t + 1], bb[1], acc[j], 0, 0, 0);
      }
    }
    if (more) store_x(buf ^ 1);
    __syncthreads();
    buf ^= 1;
  }
  // D element of tile j at this lane: row 16 w + 4 b + q, column 4 j + x
  const int row = i0 + wave * 16 + 4 * b + q;
  if (row >= d.M) return;
#pragma unroll
  for (int j = 0; j < CG; ++j) {
    const int c = 4 * j + x;
    if (c >= N) continue;
    if (splits > 1) gmem(d.part)[((int64_t)s * N + c) * d.M + row] = acc[j];
    else store_out(d, d.out_t, row, c, acc[j]);
  }
}

template <int CG, bool PVEC, typename PT, int KC = 32>
static hipError_t launch_44(const NtDesc* dd, int nz, int maxM, int splits, const int32_t* act, hipStream_t st) {
  const size_t lds = (size_t)2 * 4 * CG * (KC + 4) * sizeof(double);
  auto kern = k_mv_tall44<CG, KC, PVEC, PT>;
  static const hipError_t attr =
      lds > 64 * 1024 ? hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds)
                      : hipSuccess;
  if (attr != hipSuccess) return attr;
  dim3 grid((maxM + 63) / 64, splits, nz);
  hipLaunchKernelGGL(kern, grid, dim3(256), lds, st, dd, splits, act);
  return hipGetLastError();
}

template <bool PVEC, typename PT>
static hipError_t dispatch_44(int maxN, const NtDesc* dd, int nz, int maxM, int splits, const int32_t* act,
                              hipStream_t st) {
  if (maxN <= 36) return launch_44<9, PVEC, PT>(dd, nz, maxM, splits, act, st);
  if (maxN <= 48) return launch_44<12, PVEC, PT>(dd, nz, maxM, splits, act, st);
  if (maxN <= 68) return launch_44<17, PVEC, PT>(dd, nz, maxM, splits, act, st);
  if (maxN <= 100) return launch_44<25, PVEC, PT>(dd, nz, maxM, splits, act, st);
  if (maxN <= 132) return launch_44<33, PVEC, PT>(dd, nz, maxM, splits, act, st);
  if (maxN <= 144) return launch_44<36, PVEC, PT>(dd, nz, maxM, splits, act, st);
  return hipErrorInvalidValue;
}

hipError_t mv_f64_44(int maxN, bool pvec, const NtDesc* dd, int nz, int maxM, int splits, const int32_t* act,
                     hipStream_t st) {
  return pvec ? dispatch_44<true, double>(maxN, dd, nz, maxM, splits, act, st)
              : dispatch_44<false, double>(maxN, dd, nz, maxM, splits, act, st);
}

// P in FP32 (Z or its transposed copy for the Gram operator's FP64 products), FP64 arithmetic.
hipError_t mv_f32f64_44(int maxN, bool pvec, const NtDesc* dd, int nz, int maxM, int splits, const int32_t* act,
                        hipStream_t st) {
  return pvec ? dispatch_44<true, float>(maxN, dd, nz, maxM, splits, act, st)
              : dispatch_44<false, float>(maxN, dd, nz, maxM, splits, act, st);
}

}  // namespace rbcg
