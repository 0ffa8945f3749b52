// Kernel instantiations: double, scheme S_LBM, patch sizes [8, 16, 32], Haar and BL5/3.
#include "lbmz_patch_kernel.h"

namespace lbmz {

bool dispatch_f64_lbm(const KernelKey& k, int op, const PatchArgs* a, int npatch, hipStream_t s,
                       hipError_t* err, size_t* lds) {
  if (k.dtype != 1 || k.scheme != S_LBM || k.vf != VF_F32) return false;
  if (k.p == 8 && k.wavelet == W_HAAR) {
    if (op == 0) *err = launch_patch_kernels<double, 8, W_HAAR, S_LBM>(true, *a, npatch, s);
    else if (op == 1) *err = launch_patch_kernels<double, 8, W_HAAR, S_LBM>(false, *a, npatch, s);
    else *lds = patch_lds_bytes<double, 8, W_HAAR, S_LBM>();
    return true;
  }
  if (k.p == 8 && k.wavelet == W_BL53) {
    if (op == 0) *err = launch_patch_kernels<double, 8, W_BL53, S_LBM>(true, *a, npatch, s);
    else if (op == 1) *err = launch_patch_kernels<double, 8, W_BL53, S_LBM>(false, *a, npatch, s);
    else *lds = patch_lds_bytes<double, 8, W_BL53, S_LBM>();
    return true;
  }
  if (k.p == 16 && k.wavelet == W_HAAR) {
    if (op == 0) *err = launch_patch_kernels<double, 16, W_HAAR, S_LBM>(true, *a, npatch, s);
    else if (op == 1) *err = launch_patch_kernels<double, 16, W_HAAR, S_LBM>(false, *a, npatch, s);
    else *lds = patch_lds_bytes<double, 16, W_HAAR, S_LBM>();
    return true;
  }
  if (k.p == 16 && k.wavelet == W_BL53) {
    if (op == 0) *err = launch_patch_kernels<double, 16, W_BL53, S_LBM>(true, *a, npatch, s);
    else if (op == 1) *err = launch_patch_kernels<double, 16, W_BL53, S_LBM>(false, *a, npatch, s);
    else *lds = patch_lds_bytes<double, 16, W_BL53, S_LBM>();
    return true;
  }
  if (k.p == 32 && k.wavelet == W_HAAR) {
    if (op == 0) *err = launch_patch_kernels<double, 32, W_HAAR, S_LBM>(true, *a, npatch, s);
    else if (op == 1) *err = launch_patch_kernels<double, 32, W_HAAR, S_LBM>(false, *a, npatch, s);
    else *lds = patch_lds_bytes<double, 32, W_HAAR, S_LBM>();
    return true;
  }
  if (k.p == 32 && k.wavelet == W_BL53) {
    if (op == 0) *err = launch_patch_kernels<double, 32, W_BL53, S_LBM>(true, *a, npatch, s);
    else if (op == 1) *err = launch_patch_kernels<double, 32, W_BL53, S_LBM>(false, *a, npatch, s);
    else *lds = patch_lds_bytes<double, 32, W_BL53, S_LBM>();
    return true;
  }
  return false;
}

}  // namespace lbmz
