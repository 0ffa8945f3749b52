// Internal declarations shared by the host runtime and the HIP kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace lbmz {

enum Wavelet : int { W_HAAR = 0, W_BL53 = 1 };
enum SchemeKind : int { S_FV = 0, S_LBM = 1, S_EULER = 2, S_LBM3 = 3 };   // S_LBM3: D3Q19 on 3-D grids
enum Rule : int { R_CAPPED = 0, R_CONSTANT = 1, R_ACCUM = 2 };
// How the values of a record are stored: float32 (every kept coefficient), or
// float32 samples plus binary16 / OCP E4M3 details with per-subband scales;
// VF_E4M3B chooses per record: E4M3 where its rounding error is bounded by
// half of every occupied subband's threshold, binary16 otherwise.
enum ValueFormat : int { VF_F32 = 0, VF_F16 = 1, VF_E4M3 = 2, VF_E4M3B = 3 };

// Modes of the auxiliary (not time-critical) patch kernel.
enum AuxMode : int {
  AUX_INIT = 0,     // dense state -> forward transform -> threshold -> store
  AUX_COEF = 1,     // given coefficient tiles -> threshold -> store
  AUX_RESTORE = 2,  // store -> inverse transform -> halo strips + totals
  AUX_DECOMP = 3    // store -> inverse transform -> dense state
};

// Control block in device memory, one per context.
struct Ctrl {
  unsigned long long top16[3];   // pool bump counters (16-byte units), rotated by epoch % 3
  unsigned int abort;            // bit 0: pool overflow, bit 1: non-finite coefficient
  unsigned int abort_epoch;      // smallest epoch that raised a flag (0xffffffff = none)
  unsigned int queue[3];         // persistent step: next patch to take, rotated by epoch % 3
  unsigned int pad;
};

constexpr unsigned int ABORT_OVERFLOW = 1u;
constexpr unsigned int ABORT_NONFINITE = 2u;
constexpr uint32_t MASK_BIT = 0x80000000u;

// Parameters of one patch-kernel launch.
struct PatchArgs {
  int n;             // grid cells per side
  int npx;           // patches per side
  int npatch;        // patches in the grid
  int npx_shift;     // log2(npx) when npx is a power of two, else -1
  int levels;        // wavelet levels per dimension
  int rule;          // Rule
  double eps;        // threshold constant
  const double* eps_patch;       // per-patch threshold constants [npatch], or null for eps
  const int8_t* lev_patch;       // per-patch threshold level counts [npatch] (<= levels), or null for levels
  float* features;               // per-patch stride-8 coefficients [npatch][M][8][8], or null
  // scheme
  double dt_over_h;  // FV
  double cp[4];      // FV: max(a.N^k, 0)
  double cm[4];      // FV: min(a.N^k, 0)
  double omega;      // LBM: 1 / tau
  double gamma;      // Euler: ratio of specific heats
  // store, time n
  const uint8_t* pool_in;
  const uint32_t* table_in;
  const void* halo_in;
  // store, time n + 1
  uint8_t* pool_out;
  uint32_t* table_out;
  void* halo_out;
  double* partials_out;          // [npatch][nfields]
  float* scratch;                // 3-D step: per-workgroup population staging [grid][19][S^3]
  unsigned long long cap16;      // pool_out capacity in 16-byte units
  Ctrl* ctrl;
  unsigned int epoch;            // launch counter
  // auxiliary modes
  int mode;
  const void* dense_in;          // AUX_INIT: [nfields][n][n] ([nfields][n][n][n] in 3-D)
  const void* coef_in;           // AUX_COEF: [npatch][nfields][s][s] ([...][s][s][s] in 3-D)
  void* dense_out;               // AUX_DECOMP: same layout as dense_in
  int field_only;                // AUX_DECOMP, 3-D: >= 0 decompresses that field alone into dense_out [n][n][n]
};

// Configuration key of a compiled kernel family.
struct KernelKey {
  int dtype;   // 0 = f32, 1 = f64
  int p;       // cells per patch side
  int wavelet; // Wavelet
  int scheme;  // SchemeKind
  int vf;      // ValueFormat
};

// Flag of the dispatch operations that selects the step kernels with
// per-patch controls (per-patch thresholds or level counts, network input).
constexpr int OP_CTL = 0x100;

// Launch the fused step kernel (time n -> n + 1) or the auxiliary kernel;
// `ctl` selects the step kernel with per-patch controls.  Return
// hipErrorInvalidValue when no kernel is compiled for the key.
hipError_t launch_step(const KernelKey& k, const PatchArgs& a, int npatch, hipStream_t s, bool ctl);
hipError_t launch_step_persistent(const KernelKey& k, const PatchArgs& a, int grid, hipStream_t s, bool ctl);
hipError_t launch_aux(const KernelKey& k, const PatchArgs& a, int npatch, hipStream_t s);
bool have_kernel(const KernelKey& k);
// LDS bytes used by the kernels of a key (0 if not compiled).
size_t kernel_lds_bytes(const KernelKey& k);
// Entry of the step kernel (persistent or one workgroup per patch) and its
// workgroup size, for graph kernel nodes.
const void* step_kernel_entry(const KernelKey& k, bool persistent, bool ctl);
int kernel_threads(const KernelKey& k);

// Dispatch of one compiled kernel family: true when the key is compiled in
// this unit; `out` receives the operation's result (see dispatch_op).
#define LBMZ_DISPATCH_ARGS const KernelKey& k, int op, const PatchArgs* a, int grid, hipStream_t s, \
                           hipError_t* err, size_t* out

// Dense (uncompressed) reference step on a periodic [nfields][n][n] grid.
hipError_t launch_reference_step(int dtype, int scheme, const void* in, void* out, int n,
                                 const PatchArgs& a, hipStream_t s);
// D2Q9 equilibrium populations [9][n][n] from rho, ux, uy [n][n].
hipError_t launch_equilibrium(int dtype, const void* rho, const void* ux, const void* uy,
                              void* f, int n, hipStream_t s);
// Per-field trapezoid-free sums of a dense state of `cells` nodes per field
// into partials [nfields][nblocks] (FP64, fixed reduction order), for the
// reference context.
hipError_t launch_dense_totals(int dtype, const void* in, int nfields, size_t cells, double* partials,
                               int nblocks, hipStream_t s);
// D3Q19 (float32, periodic [19][n][n][n]): uncompressed step and equilibrium.
hipError_t launch_reference_step3(const void* in, void* out, int n, double omega, hipStream_t s);
hipError_t launch_equilibrium3(const void* rho, const void* ux, const void* uy, const void* uz, void* f, int n,
                               hipStream_t s);

}  // namespace lbmz
