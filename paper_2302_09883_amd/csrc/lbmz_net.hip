// Learned per-patch threshold predictor: a small convolutional network with
// bfloat16 weights and float32 accumulation, trained and evaluated by the
// kernels below (one workgroup per sample for the forward pass, one per group
// of samples for the gradients, a fixed-order reduction, an Adam update).
//
//   input  x[36][8][8], the patch features of the step kernel: channels 0..8
//          a patch's stored coefficients at the owned positions of stride 8,
//          channels 9 + 3 f + l - 1 the energy of field f's level-l
//          coefficients (l = 1, 2, 3) in each 8 x 8 block;
//          mapped to 12 channels: asinh(c / 1e-4) of the 9 coefficients and
//          asinh(sqrt(sum over the fields of the level-l energy) / 1e-4)
//   conv1  3x3, pad 1, 12 -> 32, bias, ReLU       (8 x 8)
//   conv2  3x3, pad 1, 32 -> 32, bias, ReLU       (8 x 8)
//   conv3  3x3, pad 1, stride 2, 32 -> 32, ReLU   (4 x 4)
//   pool   mean over the 16 positions
//   head   32 -> K, bias: predicted log10 squared error per candidate threshold
// Loss of a batch: mean of the B x K squared differences to the targets.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "../../include/lbmz.h"

namespace lbmz_net_impl {

constexpr int CF = 9;                      // fields of the patch (coefficient channels)
constexpr int CIN = 4 * CF;                // channels of one input sample (the patch features)
constexpr int CI = CF + 3, CH = 32, KMAX = 32;
constexpr int NT = 256;
constexpr int OW1 = 0, OB1 = OW1 + CH * CI * 9, OW2 = OB1 + CH, OB2 = OW2 + CH * CH * 9, OW3 = OB2 + CH,
              OB3 = OW3 + CH * CH * 9, OWH = OB3 + CH;   // head weights at OWH, head biases at OWH + 32 K
constexpr int NPMAX = OWH + (CH + 1) * KMAX;
constexpr int SPW = 16;                                     // samples per workgroup in the gradient pass
constexpr float FSCALE = 1.0e4f;                            // 1 / feature scale

__host__ __device__ constexpr int nparams(int k) { return OWH + (CH + 1) * k; }

__device__ __forceinline__ float bf(uint16_t w) { return __uint_as_float((uint32_t)w << 16); }

// float32 -> bfloat16, round to nearest even
__device__ __forceinline__ uint16_t to_bf16(float x) {
  const uint32_t u = __float_as_uint(x);
  if ((u & 0x7F800000u) == 0x7F800000u) return (uint16_t)(u >> 16);   // inf / nan kept
  return (uint16_t)((u + 0x7FFFu + ((u >> 16) & 1u)) >> 16);
}

struct Acts {
  float x[CI * 64];
  float a1[CH * 64];
  float a2[CH * 64];
  float a3[CH * 16];
  float g[CH];
  float y[KMAX];
};

// Forward pass of one sample into the activation buffers (pre-ReLU values).
__device__ void forward_sample(const uint16_t* w, const float* xin_raw, int k, Acts& s) {
  const int tid = threadIdx.x;
  for (int i = tid; i < CI * 64; i += NT) {
    const int c = i / 64, pos = i - 64 * c;
    float v;
    if (c < CF) {
      v = xin_raw[i];
    } else {
      float e = 0.0f;   // level c - CF + 1, summed over the fields in field order
      for (int f = 0; f < CF; ++f) e += xin_raw[(CF + 3 * f + (c - CF)) * 64 + pos];
      v = sqrtf(e);
    }
    s.x[i] = asinhf(v * FSCALE);
  }
  __syncthreads();
  for (int idx = tid; idx < CH * 64; idx += NT) {
    const int o = idx >> 6, p = idx & 63, i = p >> 3, j = p & 7;
    float acc = 0.0f;
    for (int c = 0; c < CI; ++c)
#pragma unroll
      for (int di = 0; di < 3; ++di)
#pragma unroll
        for (int dj = 0; dj < 3; ++dj) {
          const int yy = i + di - 1, xx = j + dj - 1;
          if (yy >= 0 && yy < 8 && xx >= 0 && xx < 8)
            acc += bf(w[OW1 + ((o * CI + c) * 3 + di) * 3 + dj]) * s.x[c * 64 + yy * 8 + xx];
        }
    s.a1[idx] = acc + bf(w[OB1 + o]);
  }
  __syncthreads();
  for (int idx = tid; idx < CH * 64; idx += NT) {
    const int o = idx >> 6, p = idx & 63, i = p >> 3, j = p & 7;
    float acc = 0.0f;
    for (int c = 0; c < CH; ++c)
#pragma unroll
      for (int di = 0; di < 3; ++di)
#pragma unroll
        for (int dj = 0; dj < 3; ++dj) {
          const int yy = i + di - 1, xx = j + dj - 1;
          if (yy >= 0 && yy < 8 && xx >= 0 && xx < 8)
            acc += bf(w[OW2 + ((o * CH + c) * 3 + di) * 3 + dj]) * fmaxf(s.a1[c * 64 + yy * 8 + xx], 0.0f);
        }
    s.a2[idx] = acc + bf(w[OB2 + o]);
  }
  __syncthreads();
  for (int idx = tid; idx < CH * 16; idx += NT) {
    const int o = idx >> 4, q = idx & 15, i = q >> 2, j = q & 3;
    float acc = 0.0f;
    for (int c = 0; c < CH; ++c)
#pragma unroll
      for (int di = 0; di < 3; ++di)
#pragma unroll
        for (int dj = 0; dj < 3; ++dj) {
          const int yy = 2 * i + di - 1, xx = 2 * j + dj - 1;
          if (yy >= 0 && yy < 8 && xx >= 0 && xx < 8)
            acc += bf(w[OW3 + ((o * CH + c) * 3 + di) * 3 + dj]) * fmaxf(s.a2[c * 64 + yy * 8 + xx], 0.0f);
        }
    s.a3[idx] = acc + bf(w[OB3 + o]);
  }
  __syncthreads();
  if (tid < CH) {
    float acc = 0.0f;
    for (int q = 0; q < 16; ++q) acc += fmaxf(s.a3[tid * 16 + q], 0.0f);
    s.g[tid] = acc * (1.0f / 16.0f);
  }
  __syncthreads();
  if (tid < k) {
    float acc = 0.0f;
    for (int c = 0; c < CH; ++c) acc += bf(w[OWH + tid * CH + c]) * s.g[c];
    s.y[tid] = acc + bf(w[OWH + CH * k + tid]);
  }
  __syncthreads();
}

__global__ __launch_bounds__(NT) void net_forward_kernel(const uint16_t* __restrict__ wbf,
                                                         const float* __restrict__ x, float* __restrict__ y,
                                                         int k) {
  __shared__ uint16_t w[NPMAX];
  __shared__ Acts s;
  const int np = nparams(k);
  for (int i = threadIdx.x; i < np; i += NT) w[i] = wbf[i];
  __syncthreads();
  forward_sample(w, x + (size_t)blockIdx.x * CIN * 64, k, s);
  if (threadIdx.x < k) y[(size_t)blockIdx.x * k + threadIdx.x] = s.y[threadIdx.x];
}

// Gradients of the batch loss, accumulated over the samples of this
// workgroup: thread t owns parameters t, t + NT, ...; the partial sums go to
// part[blockIdx.x][np] and are reduced in a fixed order afterwards.
__global__ __launch_bounds__(NT) void net_grad_kernel(const uint16_t* __restrict__ wbf,
                                                      const float* __restrict__ x, const float* __restrict__ t,
                                                      int batch, int k, float* __restrict__ part,
                                                      float* __restrict__ loss_part) {
  __shared__ uint16_t w[NPMAX];
  __shared__ Acts s;
  __shared__ float ga1[CH * 64];
  __shared__ float ga2[CH * 64];
  __shared__ float ga3[CH * 16];
  __shared__ float dy[KMAX];
  __shared__ float gg[CH];
  const int tid = threadIdx.x;
  const int np = nparams(k);
  for (int i = tid; i < np; i += NT) w[i] = wbf[i];
  float* acc = part + (size_t)blockIdx.x * np;   // this workgroup's partial sums
  for (int j = tid; j < np; j += NT) acc[j] = 0.0f;
  float lsum = 0.0f;
  const float scale = 2.0f / ((float)batch * (float)k);
  __syncthreads();
  for (int b = blockIdx.x * SPW; b < batch && b < (int)(blockIdx.x + 1) * SPW; ++b) {
    forward_sample(w, x + (size_t)b * CIN * 64, k, s);
    if (tid < k) {
      const float d = s.y[tid] - t[(size_t)b * k + tid];
      dy[tid] = scale * d;
      lsum += d * d;
    }
    __syncthreads();
    if (tid < CH) {
      float a = 0.0f;
      for (int kk = 0; kk < k; ++kk) a += dy[kk] * bf(w[OWH + kk * CH + tid]);
      gg[tid] = a;
    }
    __syncthreads();
    for (int idx = tid; idx < CH * 16; idx += NT) ga3[idx] = s.a3[idx] > 0.0f ? gg[idx >> 4] * (1.0f / 16.0f) : 0.0f;
    __syncthreads();
    // gradient into h2 through conv3 (stride 2), masked by ReLU
    for (int idx = tid; idx < CH * 64; idx += NT) {
      const int c = idx >> 6, p = idx & 63, pi = p >> 3, pj = p & 7;
      float a = 0.0f;
#pragma unroll
      for (int di = 0; di < 3; ++di) {
        const int qi2 = pi - di + 1;
        if (qi2 < 0 || (qi2 & 1) || (qi2 >> 1) >= 4) continue;
#pragma unroll
        for (int dj = 0; dj < 3; ++dj) {
          const int qj2 = pj - dj + 1;
          if (qj2 < 0 || (qj2 & 1) || (qj2 >> 1) >= 4) continue;
          const int q = (qi2 >> 1) * 4 + (qj2 >> 1);
          for (int o = 0; o < CH; ++o) a += ga3[o * 16 + q] * bf(w[OW3 + ((o * CH + c) * 3 + di) * 3 + dj]);
        }
      }
      ga2[idx] = s.a2[idx] > 0.0f ? a : 0.0f;
    }
    __syncthreads();
    // gradient into h1 through conv2 (stride 1), masked by ReLU
    for (int idx = tid; idx < CH * 64; idx += NT) {
      const int c = idx >> 6, p = idx & 63, pi = p >> 3, pj = p & 7;
      float a = 0.0f;
#pragma unroll
      for (int di = 0; di < 3; ++di) {
        const int oi = pi - di + 1;
        if (oi < 0 || oi >= 8) continue;
#pragma unroll
        for (int dj = 0; dj < 3; ++dj) {
          const int oj = pj - dj + 1;
          if (oj < 0 || oj >= 8) continue;
          for (int o = 0; o < CH; ++o) a += ga2[o * 64 + oi * 8 + oj] * bf(w[OW2 + ((o * CH + c) * 3 + di) * 3 + dj]);
        }
      }
      ga1[idx] = s.a1[idx] > 0.0f ? a : 0.0f;
    }
    __syncthreads();
    // parameter gradients of this sample, added to the owned partial sums
    for (int j = tid; j < np; j += NT) {
      float gj = 0.0f;
      if (j >= OWH) {
        const int jj = j - OWH;
        if (jj < CH * k) gj = dy[jj / CH] * s.g[jj % CH];
        else gj = dy[jj - CH * k];
      } else if (j >= OB3) {
        const int o = j - OB3;
        for (int q = 0; q < 16; ++q) gj += ga3[o * 16 + q];
      } else if (j >= OW3) {
        const int jj = j - OW3, dj = jj % 3, di = (jj / 3) % 3, c = (jj / 9) % CH, o = jj / (9 * CH);
        for (int q = 0; q < 16; ++q) {
          const int yy = 2 * (q >> 2) + di - 1, xx = 2 * (q & 3) + dj - 1;
          if (yy >= 0 && yy < 8 && xx >= 0 && xx < 8) gj += ga3[o * 16 + q] * fmaxf(s.a2[c * 64 + yy * 8 + xx], 0.0f);
        }
      } else if (j >= OB2) {
        const int o = j - OB2;
        for (int p = 0; p < 64; ++p) gj += ga2[o * 64 + p];
      } else if (j >= OW2) {
        const int jj = j - OW2, dj = jj % 3, di = (jj / 3) % 3, c = (jj / 9) % CH, o = jj / (9 * CH);
        for (int p = 0; p < 64; ++p) {
          const int yy = (p >> 3) + di - 1, xx = (p & 7) + dj - 1;
          if (yy >= 0 && yy < 8 && xx >= 0 && xx < 8) gj += ga2[o * 64 + p] * fmaxf(s.a1[c * 64 + yy * 8 + xx], 0.0f);
        }
      } else if (j >= OB1) {
        const int o = j - OB1;
        for (int p = 0; p < 64; ++p) gj += ga1[o * 64 + p];
      } else {
        const int jj = j - OW1, dj = jj % 3, di = (jj / 3) % 3, c = (jj / 9) % CI, o = jj / (9 * CI);
        for (int p = 0; p < 64; ++p) {
          const int yy = (p >> 3) + di - 1, xx = (p & 7) + dj - 1;
          if (yy >= 0 && yy < 8 && xx >= 0 && xx < 8) gj += ga1[o * 64 + p] * s.x[c * 64 + yy * 8 + xx];
        }
      }
      acc[j] += gj;
    }
    __syncthreads();
  }
  // loss: the K lanes' sums of squares, in lane order
  __shared__ float lred[KMAX];
  if (tid < k) lred[tid] = lsum;
  __syncthreads();
  if (tid == 0) {
    float l = 0.0f;
    for (int kk = 0; kk < k; ++kk) l += lred[kk];
    loss_part[blockIdx.x] = l;
  }
}

__global__ void net_reduce_kernel(const float* __restrict__ part, int nblocks, int np, float* __restrict__ grad) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= np) return;
  float a = 0.0f;
  for (int b = 0; b < nblocks; ++b) a += part[(size_t)b * np + j];
  grad[j] = a;
}

// Adam (Kingma and Ba) on the float32 master weights, then their bfloat16 copy.
__global__ void net_adam_kernel(float* __restrict__ master, const float* __restrict__ grad, float* __restrict__ m,
                                float* __restrict__ v, uint16_t* __restrict__ wbf, int np, float lr, float b1,
                                float b2, float eps, float c1, float c2) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= np) return;
  const float g = grad[j];
  const float mj = b1 * m[j] + (1.0f - b1) * g;
  const float vj = b2 * v[j] + (1.0f - b2) * g * g;
  m[j] = mj;
  v[j] = vj;
  const float w = master[j] - lr * (mj / c1) / (sqrtf(vj / c2) + eps);
  master[j] = w;
  wbf[j] = to_bf16(w);
}

__global__ void net_round_kernel(const float* __restrict__ master, uint16_t* __restrict__ wbf, int np) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j < np) wbf[j] = to_bf16(master[j]);
}

// Loss of a batch from the per-workgroup sums of squared differences: the
// same double-precision sum in block order as the host reduction of
// lbmz_net_gradients, so that both entry points give the same float.
__global__ void net_loss_kernel(const float* __restrict__ loss_part, int nblocks, double denom,
                                float* __restrict__ loss) {
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    double l = 0.0;
    for (int b = 0; b < nblocks; ++b) l += (double)loss_part[b];
    *loss = (float)(l / denom);
  }
}

}  // namespace lbmz_net_impl

// Workspace of lbmz_net_gradients_noalloc: the per-workgroup partial
// gradient sums [blocks][np] and, from the next 256-byte boundary, the
// per-workgroup loss sums [blocks].  One copy per GPU, for the life of the
// process.  In host code this name is only a stand-in for the symbol: the
// device address of each GPU's copy comes from hipGetSymbolAddress (below)
// and is the only value passed to kernels.
static __device__ __align__(256) unsigned char scratch[LBMZ_NET_SCRATCH_BYTES];

using namespace lbmz_net_impl;

struct lbmz_net {
  int k = 0, np = 0;
  int step = 0;
  int device = 0;               // device current at creation (its parameters live there)
  hipStream_t stream = nullptr;
  float* master = nullptr;
  uint16_t* wbf = nullptr;
  float* m = nullptr;
  float* v = nullptr;
  float* grad = nullptr;
  float* part = nullptr;
  float* loss_part = nullptr;
  float* io = nullptr;          // staging of host inputs, targets and outputs
  size_t io_bytes = 0, part_blocks = 0;
  std::string err;
};

namespace {

// Device address of `scratch` per device ordinal, set once per device by the
// first lbmz_net_create on it (with that device current).
constexpr int MAX_DEVICES = 256;
std::mutex g_scratch_mu;
void* g_scratch_ptr[MAX_DEVICES] = {};

hipError_t scratch_setup(int dev) {
  if (dev < 0 || dev >= MAX_DEVICES) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (g_scratch_ptr[dev]) return hipSuccess;
  void* p = nullptr;
  const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
  if (e != hipSuccess) return e;
  g_scratch_ptr[dev] = p;
  return hipSuccess;
}

void* scratch_of(int dev) {
  if (dev < 0 || dev >= MAX_DEVICES) return nullptr;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  return g_scratch_ptr[dev];
}

int net_fail(lbmz_net* n, int code, const char* msg) {
  if (n) n->err = msg;
  return code;
}

#define NETCHK(n, expr)                                                    \
  do {                                                                     \
    hipError_t e_ = (expr);                                                \
    if (e_ != hipSuccess) return net_fail((n), LBMZ_EDEVICE, hipGetErrorString(e_)); \
  } while (0)

int ensure_io(lbmz_net* n, size_t bytes) {
  if (n->io_bytes >= bytes) return LBMZ_OK;
  if (n->io) NETCHK(n, hipFree(n->io));
  n->io = nullptr;
  n->io_bytes = 0;
  NETCHK(n, hipMalloc(&n->io, bytes));
  n->io_bytes = bytes;
  return LBMZ_OK;
}

int ensure_part(lbmz_net* n, size_t blocks) {
  if (n->part_blocks >= blocks) return LBMZ_OK;
  if (n->part) NETCHK(n, hipFree(n->part));
  if (n->loss_part) NETCHK(n, hipFree(n->loss_part));
  n->part = nullptr;
  n->loss_part = nullptr;
  n->part_blocks = 0;
  NETCHK(n, hipMalloc(&n->part, blocks * (size_t)n->np * sizeof(float)));
  NETCHK(n, hipMalloc(&n->loss_part, blocks * sizeof(float)));
  n->part_blocks = blocks;
  return LBMZ_OK;
}

// Gradients of the batch loss into n->grad; the loss (host) if asked.
int batch_gradients(lbmz_net* n, const float* x, const float* t, int batch, int on_device, float* loss) {
  const float* xd = x;
  const float* td = t;
  const size_t xb = (size_t)batch * CIN * 64 * sizeof(float), tb = (size_t)batch * n->k * sizeof(float);
  if (!on_device) {
    int rc = ensure_io(n, xb + tb);
    if (rc) return rc;
    NETCHK(n, hipMemcpyAsync(n->io, x, xb, hipMemcpyHostToDevice, n->stream));
    NETCHK(n, hipMemcpyAsync(reinterpret_cast<uint8_t*>(n->io) + xb, t, tb, hipMemcpyHostToDevice, n->stream));
    xd = n->io;
    td = reinterpret_cast<const float*>(reinterpret_cast<uint8_t*>(n->io) + xb);
  }
  const int blocks = (batch + SPW - 1) / SPW;
  int rc = ensure_part(n, (size_t)blocks);
  if (rc) return rc;
  hipLaunchKernelGGL(net_grad_kernel, dim3(blocks), dim3(NT), 0, n->stream, n->wbf, xd, td, batch, n->k, n->part,
                     n->loss_part);
  NETCHK(n, hipGetLastError());
  hipLaunchKernelGGL(net_reduce_kernel, dim3((n->np + 255) / 256), dim3(256), 0, n->stream, n->part, blocks, n->np,
                     n->grad);
  NETCHK(n, hipGetLastError());
  if (loss) {
    std::vector<float> lp((size_t)blocks);
    NETCHK(n, hipMemcpyAsync(lp.data(), n->loss_part, lp.size() * sizeof(float), hipMemcpyDeviceToHost, n->stream));
    NETCHK(n, hipStreamSynchronize(n->stream));
    double l = 0.0;
    for (float v : lp) l += v;
    *loss = (float)(l / ((double)batch * n->k));
  } else if (!on_device) {
    NETCHK(n, hipStreamSynchronize(n->stream));
  }
  return LBMZ_OK;
}

}  // namespace

extern "C" {

int lbmz_net_create(int k, lbmz_net** out) {
  if (!out) return LBMZ_EINVAL;
  *out = nullptr;
  if (k < 1 || k > KMAX) return LBMZ_EINVAL;
  lbmz_net* n = new (std::nothrow) lbmz_net();
  if (!n) return LBMZ_ENOMEM;
  n->k = k;
  n->np = nparams(k);
  if (hipGetDevice(&n->device) != hipSuccess || scratch_setup(n->device) != hipSuccess) {
    delete n;
    return LBMZ_EDEVICE;
  }
  const size_t fb = (size_t)n->np * sizeof(float);
  if (hipMalloc(&n->master, fb) != hipSuccess || hipMalloc(&n->wbf, (size_t)n->np * 2) != hipSuccess ||
      hipMalloc(&n->m, fb) != hipSuccess || hipMalloc(&n->v, fb) != hipSuccess ||
      hipMalloc(&n->grad, fb) != hipSuccess) {
    lbmz_net_destroy(n);
    return LBMZ_ENOMEM;
  }
  if (hipMemset(n->master, 0, fb) != hipSuccess || hipMemset(n->wbf, 0, (size_t)n->np * 2) != hipSuccess ||
      hipMemset(n->m, 0, fb) != hipSuccess || hipMemset(n->v, 0, fb) != hipSuccess ||
      hipMemset(n->grad, 0, fb) != hipSuccess || hipDeviceSynchronize() != hipSuccess) {
    lbmz_net_destroy(n);
    return LBMZ_EDEVICE;
  }
  *out = n;
  return LBMZ_OK;
}

int lbmz_net_param_count(const lbmz_net* n) { return n ? n->np : 0; }

int lbmz_net_set_stream(lbmz_net* n, void* stream) {
  if (!n) return LBMZ_EINVAL;
  n->stream = static_cast<hipStream_t>(stream);
  return LBMZ_OK;
}

int lbmz_net_set_params(lbmz_net* n, const float* params, size_t count) {
  if (!n || !params) return LBMZ_EINVAL;
  if (count != (size_t)n->np) return net_fail(n, LBMZ_EINVAL, "wrong parameter count");
  for (size_t j = 0; j < count; ++j)
    if (!std::isfinite(params[j])) return net_fail(n, LBMZ_EINVAL, "non-finite parameter");
  const size_t fb = count * sizeof(float);
  NETCHK(n, hipMemcpyAsync(n->master, params, fb, hipMemcpyHostToDevice, n->stream));
  hipLaunchKernelGGL(net_round_kernel, dim3((n->np + 255) / 256), dim3(256), 0, n->stream, n->master, n->wbf, n->np);
  NETCHK(n, hipGetLastError());
  NETCHK(n, hipMemsetAsync(n->m, 0, fb, n->stream));
  NETCHK(n, hipMemsetAsync(n->v, 0, fb, n->stream));
  NETCHK(n, hipStreamSynchronize(n->stream));
  n->step = 0;
  return LBMZ_OK;
}

int lbmz_net_get_params(lbmz_net* n, float* params, size_t count) {
  if (!n || !params) return LBMZ_EINVAL;
  if (count != (size_t)n->np) return net_fail(n, LBMZ_EINVAL, "wrong parameter count");
  NETCHK(n, hipMemcpyAsync(params, n->master, count * sizeof(float), hipMemcpyDeviceToHost, n->stream));
  NETCHK(n, hipStreamSynchronize(n->stream));
  return LBMZ_OK;
}

int lbmz_net_forward(lbmz_net* n, const float* x, int batch, float* y, int on_device) {
  if (!n || !x || !y || batch < 0) return LBMZ_EINVAL;
  if (batch == 0) return LBMZ_OK;
  const size_t xb = (size_t)batch * CIN * 64 * sizeof(float), yb = (size_t)batch * n->k * sizeof(float);
  const float* xd = x;
  float* yd = y;
  if (!on_device) {
    int rc = ensure_io(n, xb + yb);
    if (rc) return rc;
    NETCHK(n, hipMemcpyAsync(n->io, x, xb, hipMemcpyHostToDevice, n->stream));
    xd = n->io;
    yd = reinterpret_cast<float*>(reinterpret_cast<uint8_t*>(n->io) + xb);
  }
  hipLaunchKernelGGL(net_forward_kernel, dim3(batch), dim3(NT), 0, n->stream, n->wbf, xd, yd, n->k);
  NETCHK(n, hipGetLastError());
  if (!on_device) {
    NETCHK(n, hipMemcpyAsync(y, yd, yb, hipMemcpyDeviceToHost, n->stream));
    NETCHK(n, hipStreamSynchronize(n->stream));
  }
  return LBMZ_OK;
}

int lbmz_net_gradients(lbmz_net* n, const float* x, const float* t, int batch, float* grad_host, float* loss,
                       int on_device) {
  if (!n || !x || !t || !grad_host || batch <= 0) return LBMZ_EINVAL;
  int rc = batch_gradients(n, x, t, batch, on_device, loss);
  if (rc) return rc;
  NETCHK(n, hipMemcpyAsync(grad_host, n->grad, (size_t)n->np * sizeof(float), hipMemcpyDeviceToHost, n->stream));
  NETCHK(n, hipStreamSynchronize(n->stream));
  return LBMZ_OK;
}

int lbmz_net_train_step(lbmz_net* n, const float* x, const float* t, int batch, float lr, float* loss,
                        int on_device) {
  if (!n || !x || !t || batch <= 0 || !(lr > 0.0f)) return LBMZ_EINVAL;
  int rc = batch_gradients(n, x, t, batch, on_device, loss);
  if (rc) return rc;
  n->step += 1;
  const float b1 = 0.9f, b2 = 0.999f;
  const float c1 = 1.0f - powf(b1, (float)n->step), c2 = 1.0f - powf(b2, (float)n->step);
  hipLaunchKernelGGL(net_adam_kernel, dim3((n->np + 255) / 256), dim3(256), 0, n->stream, n->master, n->grad, n->m,
                     n->v, n->wbf, n->np, lr, b1, b2, 1e-8f, c1, c2);
  NETCHK(n, hipGetLastError());
  if (!on_device) NETCHK(n, hipStreamSynchronize(n->stream));
  return LBMZ_OK;
}

int lbmz_net_gradients_noalloc(lbmz_net* n, const float* x, const float* t, int batch, float* grad, float* loss) {
  if (!n) return LBMZ_EINVAL;
  if (!x || !t || !grad || !loss) return net_fail(n, LBMZ_EINVAL, "null device pointer");
  if (batch <= 0) return net_fail(n, LBMZ_EINVAL, "batch must be > 0");
  // workspace bytes of b workgroups: partial sums, 256-byte boundary, loss sums
  auto need_of = [n](long long b) {
    const size_t part_bytes = (size_t)b * (size_t)n->np * sizeof(float);
    return ((part_bytes + 255u) & ~(size_t)255u) + (size_t)b * sizeof(float);
  };
  const int blocks = (batch + SPW - 1) / SPW;
  const size_t need = need_of(blocks);
  if (need > (size_t)LBMZ_NET_SCRATCH_BYTES) {
    long long maxb = (long long)LBMZ_NET_SCRATCH_BYTES / ((long long)n->np * 4);
    while (maxb > 0 && need_of(maxb) > (size_t)LBMZ_NET_SCRATCH_BYTES) --maxb;
    char msg[200];
    snprintf(msg, sizeof msg, "batch %d needs %zu bytes of gradient workspace, above the fixed %d (batch <= %lld)",
             batch, need, (int)LBMZ_NET_SCRATCH_BYTES, maxb * SPW);
    return net_fail(n, LBMZ_EINVAL, msg);
  }
  const size_t lp_off = (((size_t)blocks * (size_t)n->np * sizeof(float)) + 255u) & ~(size_t)255u;
  uint8_t* base = static_cast<uint8_t*>(scratch_of(n->device));
  if (!base) return net_fail(n, LBMZ_ESTATE, "no workspace address for the network's device");
  float* part = reinterpret_cast<float*>(base);
  float* loss_part = reinterpret_cast<float*>(base + lp_off);
  hipLaunchKernelGGL(net_grad_kernel, dim3(blocks), dim3(NT), 0, n->stream, n->wbf, x, t, batch, n->k, part,
                     loss_part);
  NETCHK(n, hipGetLastError());
  hipLaunchKernelGGL(net_reduce_kernel, dim3((n->np + 255) / 256), dim3(256), 0, n->stream, part, blocks, n->np,
                     grad);
  NETCHK(n, hipGetLastError());
  hipLaunchKernelGGL(net_loss_kernel, dim3(1), dim3(64), 0, n->stream, loss_part, blocks,
                     (double)batch * n->k, loss);
  NETCHK(n, hipGetLastError());
  return LBMZ_OK;
}

const char* lbmz_net_last_error(const lbmz_net* n) { return n ? n->err.c_str() : "null network"; }

void lbmz_net_destroy(lbmz_net* n) {
  if (!n) return;
  (void)hipDeviceSynchronize();
  (void)hipFree(n->master);
  (void)hipFree(n->wbf);
  (void)hipFree(n->m);
  (void)hipFree(n->v);
  (void)hipFree(n->grad);
  (void)hipFree(n->part);
  (void)hipFree(n->loss_part);
  (void)hipFree(n->io);
  delete n;
}

}  // extern "C"
