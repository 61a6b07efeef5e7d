// MFMA "NT" products, one precision per translation unit (parallel build).
#include "device_common.inc"

namespace rbcg {
hipError_t nt_f32f64_o1(int tn, const NtDesc* dd, int nz, int maxM, int splits, const int32_t* act, hipStream_t st) {
  return dispatch_tn<DT_F32F64, 1, false>(tn, dd, nz, maxM, splits, act, st);
}
hipError_t nt_f32f64_o0(int tn, const NtDesc* dd, int nz, int maxM, int splits, const int32_t* act, hipStream_t st) {
  return dispatch_tn<DT_F32F64, 0, false>(tn, dd, nz, maxM, splits, act, st);
}
}  // namespace rbcg

namespace rbcg {
hipError_t mv_f32f64_44(int maxN, bool pvec, const NtDesc* dd, int nz, int maxM, int splits, const int32_t* act,
                        hipStream_t st);

// Tall block product with FP32 P and FP64 arithmetic, up to 144 vectors: the 16x16x4 kernel for at
// most 32 of them, the 4x4x4 kernel above (as for FP64 P).
hipError_t mv_f32f64(int maxN, bool pvec, const NtDesc* dd, int nz, int maxM, int splits, const int32_t* act,
                     hipStream_t st) {
  if (maxN > 32) return mv_f32f64_44(maxN, pvec, dd, nz, maxM, splits, act, st);
  const int tn = (maxN + 15) / 16;
  return pvec ? dispatch_mv<DT_F32F64, true>(tn, dd, nz, maxM, splits, act, st)
              : dispatch_mv<DT_F32F64, false>(tn, dd, nz, maxM, splits, act, st);
}
}  // namespace rbcg
