// MFMA "NT" products, one precision per translation unit (parallel build).
#include "device_common.inc"

namespace rbcg {
hipError_t nt_bf16_o1_split(int tn, const NtDesc* dd, int nz, int maxM, int splits, const int32_t* act, hipStream_t st) {
  return dispatch_tn<DT_BF16, 1, true>(tn, dd, nz, maxM, splits, act, st);
}
hipError_t nt_bf16_o1(int tn, const NtDesc* dd, int nz, int maxM, int splits, const int32_t* act, hipStream_t st) {
  return dispatch_tn<DT_BF16, 1, false>(tn, dd, nz, maxM, splits, act, st);
}
hipError_t nt_bf16_o0(int tn, const NtDesc* dd, int nz, int maxM, int splits, const int32_t* act, hipStream_t st) {
  return dispatch_tn<DT_BF16, 0, false>(tn, dd, nz, maxM, splits, act, st);
}
}  // namespace rbcg
