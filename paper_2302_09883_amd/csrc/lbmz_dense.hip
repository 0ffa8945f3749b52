// Uncompressed reference kernels: the plain two-buffer time loop of the
// schemes on the periodic global grid, D2Q9 equilibrium set-up, and FP64
// per-field sums of a dense state.
#include <hip/hip_runtime.h>

#include "lbmz_internal.h"
#include "lbmz_patch_kernel.h"

namespace lbmz {

namespace {

template <class T>
__global__ __launch_bounds__(256) void ref_lbm_kernel(const T* __restrict__ fin, T* __restrict__ fout,
                                                      int n, T omega) {
  const int x = blockIdx.x * 16 + (threadIdx.x & 15);
  const int y = blockIdx.y * 16 + (threadIdx.x >> 4);
  if (x >= n || y >= n) return;
  const size_t nn = (size_t)n * n;
  T f[9];
#pragma unroll
  for (int i = 0; i < 9; ++i) {
    const int sx = (x - D2Q9::CX[i] + n) % n;
    const int sy = (y - D2Q9::CY[i] + n) % n;
    f[i] = fin[i * nn + (size_t)sy * n + sx];
  }
  T out[9];
  d2q9_collide<T>(f, omega, out);
#pragma unroll
  for (int i = 0; i < 9; ++i) fout[i * nn + (size_t)y * n + x] = out[i];
}

template <class T>
__global__ __launch_bounds__(256) void ref_fv_kernel(const T* __restrict__ win, T* __restrict__ wout,
                                                     int n, PatchArgs a) {
  const int x = blockIdx.x * 16 + (threadIdx.x & 15);
  const int y = blockIdx.y * 16 + (threadIdx.x >> 4);
  if (x >= n || y >= n) return;
  const T r = T(a.dt_over_h);
  const T w = win[(size_t)y * n + x];
  const T nb[4] = {win[(size_t)y * n + (x + 1) % n], win[(size_t)y * n + (x - 1 + n) % n],
                   win[(size_t)((y + 1) % n) * n + x], win[(size_t)((y - 1 + n) % n) * n + x]};
  T o = w;
#pragma unroll
  for (int k = 0; k < 4; ++k) o = o - r * (w * T(a.cp[k]) + nb[k] * T(a.cm[k]));
  wout[(size_t)y * n + x] = o;
}

template <class T>
__global__ __launch_bounds__(256) void ref_euler_kernel(const T* __restrict__ win, T* __restrict__ wout, int n,
                                                        PatchArgs a) {
  const int x = blockIdx.x * 16 + (threadIdx.x & 15);
  const int y = blockIdx.y * 16 + (threadIdx.x >> 4);
  if (x >= n || y >= n) return;
  const size_t nn = (size_t)n * n;
  const size_t c = (size_t)y * n + x;
  const size_t e = (size_t)y * n + (x + 1) % n, w_ = (size_t)y * n + (x - 1 + n) % n;
  const size_t no = (size_t)((y + 1) % n) * n + x, so = (size_t)((y - 1 + n) % n) * n + x;
  T w[4], we[4], ww[4], wn[4], ws[4];
#pragma unroll
  for (int f = 0; f < 4; ++f) {
    w[f] = win[f * nn + c];
    we[f] = win[f * nn + e];
    ww[f] = win[f * nn + w_];
    wn[f] = win[f * nn + no];
    ws[f] = win[f * nn + so];
  }
  T o[4];
  euler_node<T>(w, we, ww, wn, ws, T(a.gamma), T(a.dt_over_h), o);
#pragma unroll
  for (int f = 0; f < 4; ++f) wout[f * nn + c] = o[f];
}

template <class T>
__global__ __launch_bounds__(256) void equilibrium_kernel(const T* __restrict__ rho, const T* __restrict__ ux,
                                                          const T* __restrict__ uy, T* __restrict__ f, int n) {
  const size_t nn = (size_t)n * n;
  const size_t i0 = (size_t)blockIdx.x * 256 + threadIdx.x;
  if (i0 >= nn) return;
  const T r = rho[i0], u = ux[i0], v = uy[i0];
  const T usq = T(1.5) * (u * u + v * v);
  const T wr[3] = {T(4.0 / 9.0) * r, T(1.0 / 9.0) * r, T(1.0 / 36.0) * r};
  const T cuv[9] = {T(0), u, v, -u, -v, u + v, v - u, -(u + v), u - v};
#pragma unroll
  for (int i = 0; i < 9; ++i) {
    const T cu = cuv[i];
    const T w = wr[i == 0 ? 0 : (i < 5 ? 1 : 2)];
    f[i * nn + i0] = w * ((T(1) + T(3) * cu) + (T(4.5) * cu * cu - usq));
  }
}

// Each block sums a contiguous chunk of one field in FP64 in a fixed order.
template <class T>
__global__ __launch_bounds__(256) void dense_sum_kernel(const T* __restrict__ in, int nfields, size_t nn,
                                                        double* __restrict__ partials) {
  __shared__ double red[4];
  const int f = blockIdx.y;
  const size_t chunk = (nn + gridDim.x - 1) / gridDim.x;
  const size_t lo = (size_t)blockIdx.x * chunk;
  const size_t hi = lo + chunk < nn ? lo + chunk : nn;
  double acc = 0.0;
  for (size_t i = lo + threadIdx.x; i < hi; i += 256) acc += (double)in[(size_t)f * nn + i];
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) acc += __shfl_xor(acc, d, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0)
    partials[(size_t)f * gridDim.x + blockIdx.x] = ((red[0] + red[1]) + red[2]) + red[3];
}

}  // namespace

hipError_t launch_reference_step(int dtype, int scheme, const void* in, void* out, int n,
                                 const PatchArgs& a, hipStream_t s) {
  const dim3 grid((n + 15) / 16, (n + 15) / 16);
  if (scheme == S_LBM) {
    if (dtype == 0)
      hipLaunchKernelGGL(ref_lbm_kernel<float>, grid, dim3(256), 0, s, static_cast<const float*>(in),
                         static_cast<float*>(out), n, (float)a.omega);
    else
      hipLaunchKernelGGL(ref_lbm_kernel<double>, grid, dim3(256), 0, s, static_cast<const double*>(in),
                         static_cast<double*>(out), n, a.omega);
  } else if (scheme == S_EULER) {
    if (dtype == 0)
      hipLaunchKernelGGL(ref_euler_kernel<float>, grid, dim3(256), 0, s, static_cast<const float*>(in),
                         static_cast<float*>(out), n, a);
    else
      hipLaunchKernelGGL(ref_euler_kernel<double>, grid, dim3(256), 0, s, static_cast<const double*>(in),
                         static_cast<double*>(out), n, a);
  } else {
    if (dtype == 0)
      hipLaunchKernelGGL(ref_fv_kernel<float>, grid, dim3(256), 0, s, static_cast<const float*>(in),
                         static_cast<float*>(out), n, a);
    else
      hipLaunchKernelGGL(ref_fv_kernel<double>, grid, dim3(256), 0, s, static_cast<const double*>(in),
                         static_cast<double*>(out), n, a);
  }
  return hipGetLastError();
}

hipError_t launch_equilibrium(int dtype, const void* rho, const void* ux, const void* uy, void* f, int n,
                              hipStream_t s) {
  const size_t nn = (size_t)n * n;
  const dim3 grid((unsigned)((nn + 255) / 256));
  if (dtype == 0)
    hipLaunchKernelGGL(equilibrium_kernel<float>, grid, dim3(256), 0, s, static_cast<const float*>(rho),
                       static_cast<const float*>(ux), static_cast<const float*>(uy), static_cast<float*>(f), n);
  else
    hipLaunchKernelGGL(equilibrium_kernel<double>, grid, dim3(256), 0, s, static_cast<const double*>(rho),
                       static_cast<const double*>(ux), static_cast<const double*>(uy), static_cast<double*>(f),
                       n);
  return hipGetLastError();
}

hipError_t launch_dense_totals(int dtype, const void* in, int nfields, size_t cells, double* partials, int nblocks,
                               hipStream_t s) {
  const size_t nn = cells;
  const dim3 grid((unsigned)nblocks, (unsigned)nfields);
  if (dtype == 0)
    hipLaunchKernelGGL(dense_sum_kernel<float>, grid, dim3(256), 0, s, static_cast<const float*>(in), nfields,
                       nn, partials);
  else
    hipLaunchKernelGGL(dense_sum_kernel<double>, grid, dim3(256), 0, s, static_cast<const double*>(in),
                       nfields, nn, partials);
  return hipGetLastError();
}

}  // namespace lbmz
