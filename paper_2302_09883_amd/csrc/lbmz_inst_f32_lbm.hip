// Kernel instantiations: float, scheme S_LBM (D2Q9 BGK), patch sizes [8, 16, 32, 64], Haar and BL5/3, float32 records.
#include "lbmz_patch_kernel.h"

namespace lbmz {

bool dispatch_f32_lbm(LBMZ_DISPATCH_ARGS) {
  if (k.dtype != 0 || k.scheme != S_LBM) return false;
  LBMZ_CASE_T(float, 8, W_HAAR, S_LBM, VF_F32)
  LBMZ_CASE_T(float, 8, W_BL53, S_LBM, VF_F32)
  LBMZ_CASE_T(float, 16, W_HAAR, S_LBM, VF_F32)
  LBMZ_CASE_T(float, 16, W_BL53, S_LBM, VF_F32)
  LBMZ_CASE_T(float, 32, W_HAAR, S_LBM, VF_F32)
  LBMZ_CASE_T(float, 32, W_BL53, S_LBM, VF_F32)
  LBMZ_CASE_T(float, 64, W_HAAR, S_LBM, VF_F32)
  LBMZ_CASE_T(float, 64, W_BL53, S_LBM, VF_F32)
  return false;
}

}  // namespace lbmz

#ifdef LBMZ_PHASE_CLOCK
extern "C" int lbmz_debug_phase_clock(void* dst, size_t bytes) {
  return (int)hipMemcpyFromSymbol(dst, HIP_SYMBOL(lbmz::lbmz_phase_clock), bytes, 0, hipMemcpyDeviceToHost);
}
#endif
