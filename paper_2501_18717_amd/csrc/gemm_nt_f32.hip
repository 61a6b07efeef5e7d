// MFMA "NT" products, one precision per translation unit (parallel build).
#include "device_common.inc"

namespace rbcg {
hipError_t nt_f32_o1(int tn, const NtDesc* dd, int nz, int maxM, int splits, const int32_t* act, hipStream_t st) {
  return dispatch_tn<DT_F32, 1, false>(tn, dd, nz, maxM, splits, act, st);
}
hipError_t nt_f32_o0(int tn, const NtDesc* dd, int nz, int maxM, int splits, const int32_t* act, hipStream_t st) {
  return dispatch_tn<DT_F32, 0, false>(tn, dd, nz, maxM, splits, act, st);
}
}  // namespace rbcg

namespace rbcg {
hipError_t mv_f32(int tn, bool pvec, const NtDesc* dd, int nz, int maxM, int splits, const int32_t* act, hipStream_t st) {
  return pvec ? dispatch_mv<DT_F32, true>(tn, dd, nz, maxM, splits, act, st)
              : dispatch_mv<DT_F32, false>(tn, dd, nz, maxM, splits, act, st);
}
}  // namespace rbcg
