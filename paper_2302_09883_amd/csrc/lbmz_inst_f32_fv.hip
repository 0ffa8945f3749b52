// Kernel instantiations: float, scheme S_FV, patch sizes [8, 16, 32, 64], Haar and BL5/3.
#include "lbmz_patch_kernel.h"

namespace lbmz {

bool dispatch_f32_fv(const KernelKey& k, int op, const PatchArgs* a, int npatch, hipStream_t s,
                       hipError_t* err, size_t* lds) {
  if (k.dtype != 0 || k.scheme != S_FV || k.vf != VF_F32) return false;
  if (k.p == 8 && k.wavelet == W_HAAR) {
    if (op == 0) *err = launch_patch_kernels<float, 8, W_HAAR, S_FV>(true, *a, npatch, s);
    else if (op == 1) *err = launch_patch_kernels<float, 8, W_HAAR, S_FV>(false, *a, npatch, s);
    else *lds = patch_lds_bytes<float, 8, W_HAAR, S_FV>();
    return true;
  }
  if (k.p == 8 && k.wavelet == W_BL53) {
    if (op == 0) *err = launch_patch_kernels<float, 8, W_BL53, S_FV>(true, *a, npatch, s);
    else if (op == 1) *err = launch_patch_kernels<float, 8, W_BL53, S_FV>(false, *a, npatch, s);
    else *lds = patch_lds_bytes<float, 8, W_BL53, S_FV>();
    return true;
  }
  if (k.p == 16 && k.wavelet == W_HAAR) {
    if (op == 0) *err = launch_patch_kernels<float, 16, W_HAAR, S_FV>(true, *a, npatch, s);
    else if (op == 1) *err = launch_patch_kernels<float, 16, W_HAAR, S_FV>(false, *a, npatch, s);
    else *lds = patch_lds_bytes<float, 16, W_HAAR, S_FV>();
    return true;
  }
  if (k.p == 16 && k.wavelet == W_BL53) {
    if (op == 0) *err = launch_patch_kernels<float, 16, W_BL53, S_FV>(true, *a, npatch, s);
    else if (op == 1) *err = launch_patch_kernels<float, 16, W_BL53, S_FV>(false, *a, npatch, s);
    else *lds = patch_lds_bytes<float, 16, W_BL53, S_FV>();
    return true;
  }
  if (k.p == 32 && k.wavelet == W_HAAR) {
    if (op == 0) *err = launch_patch_kernels<float, 32, W_HAAR, S_FV>(true, *a, npatch, s);
    else if (op == 1) *err = launch_patch_kernels<float, 32, W_HAAR, S_FV>(false, *a, npatch, s);
    else *lds = patch_lds_bytes<float, 32, W_HAAR, S_FV>();
    return true;
  }
  if (k.p == 32 && k.wavelet == W_BL53) {
    if (op == 0) *err = launch_patch_kernels<float, 32, W_BL53, S_FV>(true, *a, npatch, s);
    else if (op == 1) *err = launch_patch_kernels<float, 32, W_BL53, S_FV>(false, *a, npatch, s);
    else *lds = patch_lds_bytes<float, 32, W_BL53, S_FV>();
    return true;
  }
  if (k.p == 64 && k.wavelet == W_HAAR) {
    if (op == 0) *err = launch_patch_kernels<float, 64, W_HAAR, S_FV>(true, *a, npatch, s);
    else if (op == 1) *err = launch_patch_kernels<float, 64, W_HAAR, S_FV>(false, *a, npatch, s);
    else *lds = patch_lds_bytes<float, 64, W_HAAR, S_FV>();
    return true;
  }
  if (k.p == 64 && k.wavelet == W_BL53) {
    if (op == 0) *err = launch_patch_kernels<float, 64, W_BL53, S_FV>(true, *a, npatch, s);
    else if (op == 1) *err = launch_patch_kernels<float, 64, W_BL53, S_FV>(false, *a, npatch, s);
    else *lds = patch_lds_bytes<float, 64, W_BL53, S_FV>();
    return true;
  }
  return false;
}

}  // namespace lbmz
