// Kernel instantiations: float, scheme S_EULER (compressible Euler, Rusanov flux),
// patch sizes [32, 64], Haar and BL5/3, value formats float32, binary16 and E4M3.
#include "lbmz_patch_kernel.h"

namespace lbmz {

#define LBMZ_CASE(P_, W_, V_)                                                                  \
  if (k.p == P_ && k.wavelet == W_ && k.vf == V_) {                                            \
    if (op == 0) *err = launch_patch_kernels<float, P_, W_, S_EULER, V_>(true, *a, npatch, s);   \
    else if (op == 1) *err = launch_patch_kernels<float, P_, W_, S_EULER, V_>(false, *a, npatch, s); \
    else *lds = patch_lds_bytes<float, P_, W_, S_EULER, V_>();                                 \
    return true;                                                                               \
  }

bool dispatch_f32_euler(const KernelKey& k, int op, const PatchArgs* a, int npatch, hipStream_t s,
                        hipError_t* err, size_t* lds) {
  if (k.dtype != 0 || k.scheme != S_EULER) return false;
  LBMZ_CASE(32, W_HAAR, VF_F32)
  LBMZ_CASE(32, W_BL53, VF_F32)
  LBMZ_CASE(64, W_HAAR, VF_F32)
  LBMZ_CASE(64, W_BL53, VF_F32)
  LBMZ_CASE(32, W_HAAR, VF_F16)
  LBMZ_CASE(32, W_BL53, VF_F16)
  LBMZ_CASE(64, W_HAAR, VF_F16)
  LBMZ_CASE(64, W_BL53, VF_F16)
  LBMZ_CASE(32, W_HAAR, VF_E4M3)
  LBMZ_CASE(32, W_BL53, VF_E4M3)
  LBMZ_CASE(64, W_HAAR, VF_E4M3)
  LBMZ_CASE(64, W_BL53, VF_E4M3)
  return false;
}

#undef LBMZ_CASE

}  // namespace lbmz
