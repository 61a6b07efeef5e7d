// Block-Thomas forward step for one exact block width M (the widths 2^p + 1 of the method),
// one workgroup of 4 waves per (shift, system).  Same recurrence and outputs as the generic
// k_tri_forward (kernels.hip):
//   S_j = D_j + sigma I - U_{j-1} B_{j-1}^T,  Sinv_j = S_j^{-1},  U_j = B_j Sinv_j,
//   rhs'_{j+1} = -B_j Sinv_j rhs'_j,  est[j] = || rhs'_{j+1} ||
// with a different division of the work:
//  * the two M x M x M products run on the FP64 16x16x4 MFMA, all four waves, operands read
//    straight from global memory (L2) or from the LDS image of Sinv_j;
//  * S_j is inverted by M symmetric sweeps (Gauss-Jordan on an SPD matrix without pivoting)
//    held in a GR x GR lane grid, block-cyclic, GR = 8 (one wave, no barriers) for M <= 33
//    and GR = 16 (four waves) for M = 65 and 129: each sweep publishes one column through LDS and
//    applies a rank-one update to the lane's registers.  After all M sweeps the registers hold
//    -S^{-1};
//  * rhs'_{j+1} is formed as -B_j (Sinv_j rhs'_j), which needs only Sinv_j (in LDS) and B_j.
// Global data written inside the kernel (U_j, Zw) is read back with agent-scope loads, which
// bypass the per-CU vector cache.
#include "device_common.inc"

namespace rbcg {

__device__ __forceinline__ double ld_agent(const double* p) {
  return __hip_atomic_load(gmem(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Panels: 16 values of u in the Schur product (P and Q panels, placed in the region of S when
// they fit there, S being written only after the product), 8 in the Sinv_j product (P panel
// only, beside S).
constexpr int kPanelA = 16, kPanelC = 8;
__host__ __device__ constexpr int tri_mt16(int m) { return (m + 15) / 16 * 16; }
__host__ __device__ constexpr bool tri_a_in_s(int m) { return 2 * tri_mt16(m) * (kPanelA + 1) <= m * (m + 1); }
__host__ __device__ constexpr int tri_pan_elems(int m) {
  return tri_a_in_s(m) ? tri_mt16(m) * (kPanelC + 1)
                       : (2 * (kPanelA + 1) > kPanelC + 1 ? 2 * (kPanelA + 1) : kPanelC + 1) * tri_mt16(m);
}
size_t tri_exact_lds(int m, int r) {
  return ((size_t)m * (m + 1) + 2 * (size_t)(m + 3) + 2 * (size_t)m * r + (size_t)tri_pan_elems(m)) * 8;
}

// out(a, b) = sum_u P(a, u) Q(b, u) for a, b < M on the FP64 16x16x4 MFMA, the 16 x 16 output
// tiles dealt round-robin to the 4 waves (tile = wave + 4 tw).  The reduction runs over panels of
// KP values of u: each panel of P (global, row-major M x M) is staged in LDS by all threads; Q is
// either staged the same way (QS == nullptr: from global Qg) or read in place from an LDS image
// QS (row stride MP).  E(a, b, value) stores each result.
template <int M, int KP, int TG, typename FE>
__device__ __forceinline__ void panel_gemm_nt(int tid, const double* Pg, bool p_agent, const double* Qg,
                                              const double* QS, double* panP, double* panQ, FE E) {
  constexpr int MT = (M + 15) / 16;
  constexpr int NTW = (MT * MT + 3) / 4;             // tiles per wave
  constexpr int KPS = KP + 1;
  constexpr int MP = M + 1;
  constexpr int PE = (MT * 16 * KP + 255) / 256;     // panel elements per thread
  const int lane = tid & 63, wave = tid >> 6, r16 = lane & 15, kq = lane >> 4;
  const bool stage_q = QS == nullptr;
  double rp[PE], rq[PE];
  // next panel into registers (issued before the current panel's products)
  auto fetch = [&](int u0) {
#pragma unroll
    for (int t = 0; t < PE; ++t) {
      const int e = tid + 256 * t;
      const int a = e / KP, u = u0 + e % KP;
      const bool in = e < MT * 16 * KP && a < M && u < M;
      rp[t] = in ? (p_agent ? ld_agent(Pg + a * M + u) : gmem(Pg)[a * M + u]) : 0.0;
      rq[t] = (in && stage_q) ? gmem(Qg)[a * M + u] : 0.0;
    }
  };
  auto put = [&]() {
#pragma unroll
    for (int t = 0; t < PE; ++t) {
      const int e = tid + 256 * t;
      if (e < MT * 16 * KP) {
        panP[(e / KP) * KPS + e % KP] = rp[t];
        if (stage_q) panQ[(e / KP) * KPS + e % KP] = rq[t];
      }
    }
  };
  for (int g0 = 0; g0 < NTW; g0 += TG) {
    v4d acc[TG];
    static_for<TG>([&](auto tc) { acc[decltype(tc)::value] = v4d{0.0, 0.0, 0.0, 0.0}; });
    fetch(0);
    for (int u0 = 0; u0 < M; u0 += KP) {
      put();
      __syncthreads();
      if (u0 + KP < M) fetch(u0 + KP);
#pragma unroll
      for (int k4 = 0; k4 < KP; k4 += 4) {
        const int uk = k4 + kq;
        static_for<TG>([&](auto tc) {
          constexpr int tw = decltype(tc)::value;
          const int tile = wave + 4 * (g0 + tw);
          if (g0 + tw < NTW && tile < MT * MT) {
            const int a = (tile / MT) * 16 + r16, b = (tile % MT) * 16 + r16;
            const double x = panP[a * KPS + uk];
            double y;
            if (stage_q) y = panQ[b * KPS + uk];
            else y = (b < M && u0 + uk < M) ? QS[b * MP + u0 + uk] : 0.0;
            acc[tw] = __builtin_amdgcn_mfma_f64_16x16x4f64(x, y, acc[tw], 0, 0, 0);
          }
        });
      }
      __syncthreads();
    }
    static_for<TG>([&](auto tc) {
      constexpr int tw = decltype(tc)::value;
      const int tile = wave + 4 * (g0 + tw);
      if (g0 + tw < NTW && tile < MT * MT) {
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const int a = (tile / MT) * 16 + kq + 4 * q, b = (tile % MT) * 16 + r16;
          if (a < M && b < M) E(a, b, acc[tw][q]);
        }
      }
    });
  }
}

template <int M, int GR, int NWF>
__global__ __launch_bounds__(256) void k_tri_exact(const TriDesc* __restrict__ descs, int j0, int j1,
                                                   const int32_t* __restrict__ act) {
  constexpr int MP = M + 1;
  constexpr int PB = M + 3;
  constexpr int SL = (M + GR - 1) / GR;
  static_assert(GR * GR == 64 * NWF, "lane grid must fill the sweep waves");
  const TriDesc d = descs[blockIdx.z];
  if (!is_active(act, d.active)) return;
  const int r = d.r, tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  constexpr int64_t mm = (int64_t)M * M;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  double* S = (double*)smem_raw;   // M x MP: S_j, then Sinv_j
  double* prow = S + M * MP;       // 2 x PB: published sweep columns
  double* zb = prow + 2 * PB;      // M x r: rhs'_j, then rhs'_{j+1}
  double* zy = zb + M * r;         // M x r: Sinv_j rhs'_j
  double* pan = zy + M * r;        // panel region
  constexpr int MT16 = tri_mt16(M);
  __shared__ double s_red[4];
  __shared__ int s_fail;
  if (tid == 0) s_fail = 0;
  for (int e = tid; e < 2 * PB; e += 256) prow[e] = 0.0;
  for (int j = j0; j < j1; ++j) {
    const double* Dj = d.D + j * mm;
    const double* Bj = d.Bsub + j * mm;
    const int32_t* mk = d.mask + (int64_t)j * M;
    if (j == j0) {
      if (j == 0) {
        for (int e = tid; e < M * r; e += 256) zb[e] = d.rhs[(int64_t)(e / r) * d.ld_rhs + (e % r)];
      } else {
        for (int e = tid; e < M * r; e += 256) zb[e] = ld_agent(d.Zw + (int64_t)j * M * r + e);
      }
      __syncthreads();
    }
    for (int e = tid; e < M * r; e += 256) gmem(d.Zw)[(int64_t)j * M * r + e] = zb[e];

    // S_j = D_j - U_{j-1} B_{j-1}^T  (the shift and the symmetrisation come with the sweep load)
    if (j == 0) {
      for (int e = tid; e < M * M; e += 256) S[(e / M) * MP + (e % M)] = gmem(Dj)[e];
    } else {
      const double* U = d.Xw + (j - 1) * mm;
      const double* B = d.Bsub + (j - 1) * mm;
      double* panA = tri_a_in_s(M) ? S : pan;   // S is free until the product is done
      double* panB = panA + MT16 * (kPanelA + 1);
      constexpr int NTW = ((M + 15) / 16 * ((M + 15) / 16) + 3) / 4;
      if constexpr (NTW <= 8 || !tri_a_in_s(M)) {
        // every tile of a wave stays in registers until the last panel: S may share its region
        // with the panels, as it is written only after them
        panel_gemm_nt<M, kPanelA, NTW>(tid, U, true, B, nullptr, panA, panB,
                                       [&](int a, int b, double v) { S[a * MP + b] = gmem(Dj)[a * M + b] - v; });
      } else {
        // tiles in groups of 8: results go to Lw[j] (overwritten by Sinv_j later), then to S
        double* Lj = d.Lw + j * mm;
        panel_gemm_nt<M, kPanelA, 8>(tid, U, true, B, nullptr, panA, panB,
                                     [&](int a, int b, double v) { gmem(Lj)[a * M + b] = gmem(Dj)[a * M + b] - v; });
        __threadfence();
        __syncthreads();
        for (int e = tid; e < M * M; e += 256) S[(e / M) * MP + (e % M)] = ld_agent(Lj + e);
      }
    }
    __syncthreads();

    // Sinv_j by M symmetric sweeps in the lane grid
    if (wave < NWF) {
      const int rl = tid % GR, cl = tid / GR;
      double v[SL][SL];
#pragma unroll
      for (int i = 0; i < SL; ++i)
#pragma unroll
        for (int k = 0; k < SL; ++k) {
          const int a = rl + GR * i, c = cl + GR * k;
          double x = 0.0;
          if (a < M && c < M) {
            x = a == c ? S[a * MP + a] + d.sigma : 0.5 * (S[a * MP + c] + S[c * MP + a]);
            if (gmem(mk)[a] || gmem(mk)[c]) x = a == c ? 1.0 : 0.0;
          }
          v[i][k] = x;
        }
      static_for<SL>([&](auto jc) {
        constexpr int js = decltype(jc)::value;
#pragma nounroll
        for (int rr = 0; rr < GR; ++rr) {
          const int p = GR * js + rr;
          if (p >= M) break;   // uniform
          double* pr = prow + (p & 1) * PB;
          if (cl == rr) {
#pragma unroll
            for (int i = 0; i < SL; ++i) {
              const int a = rl + GR * i;
              if (a < M) pr[a] = v[i][js];
            }
          }
          if constexpr (NWF > 1) __syncthreads();
          else __builtin_amdgcn_wave_barrier();
          const double piv = pr[p];
          const bool bad = !(piv > 0.0);
          const double f = bad ? 0.0 : recip_pos(piv);
          if (bad && tid == 0) s_fail = 1;
          double ra[SL], rc[SL];
#pragma unroll
          for (int i = 0; i < SL; ++i) {
            const int a = rl + GR * i, c = cl + GR * i;
            ra[i] = a < M ? pr[a] : 0.0;
            rc[i] = c < M ? pr[c] : 0.0;
          }
#pragma unroll
          for (int i = 0; i < SL; ++i) {
            const double ri = ra[i] * f;
#pragma unroll
            for (int k = 0; k < SL; ++k) v[i][k] = fma(-ri, rc[k], v[i][k]);
          }
          if (rl == rr) {
#pragma unroll
            for (int k = 0; k < SL; ++k) v[js][k] = rc[k] * f;
          }
          if (cl == rr) {
#pragma unroll
            for (int i = 0; i < SL; ++i) v[i][js] = ra[i] * f;
          }
          if (rl == rr && cl == rr) v[js][js] = -f;
        }
      });
      // the registers hold -Sinv_j
      double* Lj = d.Lw + j * mm;
#pragma unroll
      for (int i = 0; i < SL; ++i)
#pragma unroll
        for (int k = 0; k < SL; ++k) {
          const int a = rl + GR * i, c = cl + GR * k;
          if (a < M && c < M) {
            S[a * MP + c] = -v[i][k];
            gmem(Lj)[a * M + c] = -v[i][k];
          }
        }
    }
    __syncthreads();

    // U_j = B_j Sinv_j  (Sinv_j symmetric: Q(b, u) = Sinv_j[b][u])
    {
      double* Uj = d.Xw + j * mm;
      panel_gemm_nt<M, kPanelC, 8>(tid, Bj, false, nullptr, S, pan, nullptr,
                                [&](int a, int b, double v) { gmem(Uj)[a * M + b] = v; });
    }
    // y = Sinv_j rhs'_j
    for (int e = tid; e < M * r; e += 256) {
      const int a = e / r, c = e % r;
      double acc = 0.0;
      for (int u = 0; u < M; ++u) acc += S[a * MP + u] * zb[u * r + c];
      zy[e] = acc;
    }
    __syncthreads();
    // rhs'_{j+1} = -B_j y and its norm
    double sq = 0.0;
    for (int e = tid; e < M * r; e += 256) {
      const int a = e / r, c = e % r;
      double acc = 0.0;
      for (int u = 0; u < M; ++u) acc += gmem(Bj)[a * M + u] * zy[u * r + c];
      zb[e] = -acc;
      gmem(d.Zw)[(int64_t)(j + 1) * M * r + e] = -acc;
      sq += acc * acc;
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) sq += __shfl_xor(sq, off, 64);
    if (lane == 0) s_red[wave] = sq;
    __threadfence();   // U_j and Zw are read back by the next step
    __syncthreads();
    if (d.est && tid == 0) d.est[j] = sqrt(s_red[0] + s_red[1] + s_red[2] + s_red[3]);
  }
  if (tid == 0 && s_fail && d.fail) *d.fail = 1;
}

template <int M, int GR, int NWF>
static hipError_t launch_tri_exact_t(const TriDesc* dd, int nz, int r, int j0, int j1, const int32_t* act,
                                     hipStream_t st) {
  const size_t lds = tri_exact_lds(M, r);
  if (lds > kLdsCap) return hipErrorNotSupported;
  const void* kern = (const void*)k_tri_exact<M, GR, NWF>;
  static const hipError_t attr = [&] {   // once per process, thread-safe
    hipFuncAttributes fa;
    hipError_t e = hipFuncGetAttributes(&fa, kern);
    if (e == hipSuccess)
      e = hipFuncSetAttribute(kern, hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024 - (int)fa.sharedSizeBytes);
    return e;
  }();
  if (attr != hipSuccess) return attr;
  void* args[] = {(void*)&dd, (void*)&j0, (void*)&j1, (void*)&act};
  return hipLaunchKernel(kern, dim3(1, 1, nz), dim3(256), args, lds, st);
}

// Every descriptor of the launch must have d.m == m.  hipErrorNotSupported: use the generic kernel.
hipError_t launch_tri_exact(const TriDesc* dd, int nz, int m, int r, int j0, int j1, const int32_t* act,
                            hipStream_t st) {
  switch (m) {
    case 9: return launch_tri_exact_t<9, 8, 1>(dd, nz, r, j0, j1, act, st);
    case 17: return launch_tri_exact_t<17, 8, 1>(dd, nz, r, j0, j1, act, st);
    case 33: return launch_tri_exact_t<33, 8, 1>(dd, nz, r, j0, j1, act, st);
    case 65: return launch_tri_exact_t<65, 16, 4>(dd, nz, r, j0, j1, act, st);
    case 129: return launch_tri_exact_t<129, 16, 4>(dd, nz, r, j0, j1, act, st);
    default: return hipErrorNotSupported;
  }
}

}  // namespace rbcg
