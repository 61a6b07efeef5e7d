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
hipError_t mv_f32f64(int tn, bool pvec, const NtDesc* dd, int nz, int maxM, int splits, const int32_t* act,
                     hipStream_t st) {
  return pvec ? dispatch_mv<DT_F32F64, true>(tn, dd, nz, maxM, splits, act, st)
              : dispatch_mv<DT_F32F64, false>(tn, dd, nz, maxM, splits, act, st);
}
}  // namespace rbcg
