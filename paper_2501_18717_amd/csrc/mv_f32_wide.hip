// FP32 block product on the 32x32x2 MFMA: out(i, c) = sum_k P[i][k] X[c][k] with P (the
// operator, FP32) streamed from HBM once and N = 32 T2 + NE vectors c.  Block widths of the
// method are 2^p + 1 (the right-hand side plus a power-of-two Gaussian block), so the last
// column (NE = 1) runs on the vector ALU beside the matrix cores instead of padding a whole
// 32-wide tile.
//
// Workgroup = W waves = 32 W rows i, all N columns, one split of k.  Per chunk of BK = 64 values
// of k the X rows are staged in LDS (double-buffered, next chunk's global loads in flight while
// this chunk computes) and each lane streams 32 consecutive values of its own row of P straight
// into registers.  Inside a chunk the k index is relabelled identically for both operands: lane
// half h (lane / 32) takes the run kc + 32 h + [0, 32), and MFMA step s pairs the two halves'
// values s.  D rows = c (X side), D columns = i (P side), so stores run along i.  Split-K
// partials are stored as FP32, the precision they were accumulated in (half the bytes of FP64;
// the reduction converts each exactly before adding in FP64).
#include "device_common.inc"

namespace rbcg {

typedef float v16f __attribute__((ext_vector_type(16)));

template <int T2, int NE, int W>
__global__ __launch_bounds__(64 * W) void k_mv_wide(const NtDesc* __restrict__ descs, int splits,
                                                    const int32_t* __restrict__ act) {
  constexpr int BK = 64;
  constexpr int XS = BK + 4;                 // LDS row stride (floats), 16-byte aligned rows
  constexpr int NC = 32 * T2 + NE;           // staged X rows
  constexpr int NT = 64 * W;
  constexpr int VPR = BK / 4;                // float4 per staged row and chunk
  constexpr int XP = (NC * VPR + NT - 1) / NT;
  const NtDesc d = descs[blockIdx.z];
  if (!is_active(act, d.active)) return;
  const int i0 = blockIdx.x * 32 * W;
  if (i0 >= d.M) return;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int rr = lane & 31, h = lane >> 5;
  const int s = blockIdx.y;
  const int kper = ((d.K + splits - 1) / splits + BK - 1) / BK * BK;
  const int kb = s * kper;
  const int ke = min(d.K, kb + kper);
  const int N = d.N;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  float* xs = (float*)smem_raw;              // [2][NC][XS]
  __shared__ gmem_t<const float> xrow_ptr[NC];
  for (int r = tid; r < NC; r += NT) xrow_ptr[r] = r < N ? gmem((const float*)d.X.p) + row_off(d.X, r) : nullptr;
  __syncthreads();

  const int row = i0 + wave * 32 + rr;
  const bool rval = row < d.M;
  const gmem_t<const float> pp = gmem((const float*)d.P.p) + (rval ? row_off(d.P, row) : 0);

  v4f xreg[XP];
  auto load_x = [&](int kc) {
    const bool full = kc + BK <= ke;
#pragma unroll
    for (int p = 0; p < XP; ++p) {
      const int e = tid + NT * p;
      const int r = e / VPR, k = kc + 4 * (e % VPR);
      v4f v = (v4f)(0.f);
      const gmem_t<const float> src = r < NC ? xrow_ptr[r] : nullptr;
      if (src) {
        if (full) {
          v = *(gmem_t<const v4f>)(src + k);
        } else {
#pragma unroll
          for (int t = 0; t < 4; ++t) v[t] = k + t < ke ? src[k + t] : 0.f;
        }
      }
      xreg[p] = v;
    }
  };
  auto store_x = [&](int buf) {
    float* dst = xs + buf * (NC * XS);
#pragma unroll
    for (int p = 0; p < XP; ++p) {
      const int e = tid + NT * p;
      const int r = e / VPR;
      if (r < NC) *(v4f*)(dst + r * XS + 4 * (e % VPR)) = xreg[p];
    }
  };
  float ar[32];
  auto load_a = [&](int kc) {
    const int k = kc + 32 * h;
    if (rval && k + 32 <= ke) {
      const gmem_t<const v4f> src = (gmem_t<const v4f>)(pp + k);
#pragma unroll
      for (int t = 0; t < 8; ++t) {
        const v4f u = src[t];
#pragma unroll
        for (int e = 0; e < 4; ++e) ar[4 * t + e] = u[e];
      }
    } else {
#pragma unroll
      for (int t = 0; t < 32; ++t) ar[t] = (rval && k + t < ke) ? pp[k + t] : 0.f;
    }
  };

  v16f acc[T2];
  static_for<T2>([&](auto tc) { acc[decltype(tc)::value] = (v16f)(0.f); });
  float ex = 0.f;

  int buf = 0;
  if (kb < ke) {
    load_x(kb);
    load_a(kb);
    store_x(0);
  }
  __syncthreads();
  for (int kc = kb; kc < ke; kc += BK) {
    float cur[32];
#pragma unroll
    for (int t = 0; t < 32; ++t) cur[t] = ar[t];
    const bool more = kc + BK < ke;
    if (more) {
      load_x(kc + BK);
      load_a(kc + BK);
    }
    const float* xb = xs + buf * (NC * XS) + rr * XS + 32 * h;
    const float* eb = xs + buf * (NC * XS) + (32 * T2) * XS + 32 * h;
    float4 xg[2][T2 + NE];
#pragma unroll
    for (int t = 0; t < T2; ++t) xg[0][t] = *(const float4*)(xb + 32 * t * XS);
    if constexpr (NE) xg[0][T2] = *(const float4*)eb;
    static_for<8>([&](auto gc) {
      constexpr int g = decltype(gc)::value;
      if constexpr (g + 1 < 8) {
#pragma unroll
        for (int t = 0; t < T2; ++t) xg[(g + 1) & 1][t] = *(const float4*)(xb + 32 * t * XS + 4 * (g + 1));
        if constexpr (NE) xg[(g + 1) & 1][T2] = *(const float4*)(eb + 4 * (g + 1));
      }
      __builtin_amdgcn_sched_barrier(0);
      static_for<4>([&](auto uc) {
        constexpr int u = decltype(uc)::value;
        static_for<T2>([&](auto tc) {
          constexpr int t = decltype(tc)::value;
          acc[t] = __builtin_amdgcn_mfma_f32_32x32x2f32(xg[g & 1][t][u], cur[4 * g + u], acc[t], 0, 0, 0);
        });
        if constexpr (NE) ex = fmaf(cur[4 * g + u], xg[g & 1][T2][u], ex);
      });
      __builtin_amdgcn_sched_barrier(0);
    });
    if (more) store_x(buf ^ 1);
    __syncthreads();
    buf ^= 1;
  }
  const int i = i0 + wave * 32 + rr;
  const bool iv = i < d.M;
  static_for<T2>([&](auto tc) {
    constexpr int t = decltype(tc)::value;
    const v16f a = acc[t];
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      const int c = 32 * t + 8 * (r >> 2) + 4 * h + (r & 3);
      if (!iv || c >= N) continue;
      if (splits > 1) gmem((float*)d.part)[((int64_t)s * N + c) * d.M + i] = a[r];   // FP32 partials
      else store_out(d, d.out_t, i, c, (double)a[r]);
    }
  });
  if constexpr (NE) {
    const float tot = ex + __shfl_xor(ex, 32);
    const int c = 32 * T2;
    if (h == 0 && iv && c < N) {
      if (splits > 1) gmem((float*)d.part)[((int64_t)s * N + c) * d.M + i] = tot;
      else store_out(d, d.out_t, i, c, (double)tot);
    }
  }
}

size_t mv_wide_lds(int t2, int ne) { return (size_t)2 * (32 * t2 + ne) * (64 + 4) * sizeof(float); }

template <int T2, int NE, int W>
static hipError_t launch_wide_t(const NtDesc* dd, int nz, int maxM, int splits, const int32_t* act, hipStream_t st) {
  const size_t lds = mv_wide_lds(T2, NE);
  auto kern = k_mv_wide<T2, NE, W>;
  // raised once per process; function-local static initialisation is thread-safe
  static const hipError_t attr =
      lds > 64 * 1024 ? hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds)
                      : hipSuccess;
  if (attr != hipSuccess) return attr;
  dim3 grid((maxM + 32 * W - 1) / (32 * W), splits, nz);
  hipLaunchKernelGGL(kern, grid, dim3(64 * W), lds, st, dd, splits, act);
  return hipGetLastError();
}

// N = 32 t2 + ne columns; w = waves per workgroup (2 or 4).
hipError_t mv_f32_wide(int t2, int ne, int w, const NtDesc* dd, int nz, int maxM, int splits, const int32_t* act,
                       hipStream_t st) {
  const int key = t2 * 100 + ne * 10 + w;
  switch (key) {
    case 112: return launch_wide_t<1, 1, 2>(dd, nz, maxM, splits, act, st);
    case 114: return launch_wide_t<1, 1, 4>(dd, nz, maxM, splits, act, st);
    case 212: return launch_wide_t<2, 1, 2>(dd, nz, maxM, splits, act, st);
    case 214: return launch_wide_t<2, 1, 4>(dd, nz, maxM, splits, act, st);
    case 202: return launch_wide_t<2, 0, 2>(dd, nz, maxM, splits, act, st);
    case 204: return launch_wide_t<2, 0, 4>(dd, nz, maxM, splits, act, st);
    case 412: return launch_wide_t<4, 1, 2>(dd, nz, maxM, splits, act, st);
    case 414: return launch_wide_t<4, 1, 4>(dd, nz, maxM, splits, act, st);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace rbcg
