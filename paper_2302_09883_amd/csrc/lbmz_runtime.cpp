// Host runtime and C ABI of liblbmz (see include/lbmz.h).
//
// A context owns two copies of the compressed store (input and output of a
// step: pool, offset table, halo strips, per-patch totals), a control block
// for the pool bump counters and abort flags, and optional dense staging used
// only while the state is being set.  lbmz_step issues one fused kernel per
// time step and reads the control block once per call: a pool overflow is
// absorbed by growing both pools and replaying the remaining steps from the
// last good state; a non-finite coefficient stops at the last good state.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/lbmz.h"
#include "lbmz_internal.h"

namespace lbmz {
bool dispatch_f32_fv(LBMZ_DISPATCH_ARGS);
bool dispatch_f32_lbm(LBMZ_DISPATCH_ARGS);
bool dispatch_f64_fv(LBMZ_DISPATCH_ARGS);
bool dispatch_f64_lbm(LBMZ_DISPATCH_ARGS);
bool dispatch_f32_fv_q(LBMZ_DISPATCH_ARGS);
bool dispatch_f32_lbm_q(LBMZ_DISPATCH_ARGS);
bool dispatch_f32_euler(LBMZ_DISPATCH_ARGS);
bool dispatch_f32_d3q19(LBMZ_DISPATCH_ARGS);
bool dispatch_f32_e4m3b_lbm(LBMZ_DISPATCH_ARGS);
bool dispatch_f32_e4m3b_fv(LBMZ_DISPATCH_ARGS);

static bool dispatch(LBMZ_DISPATCH_ARGS) {
  return dispatch_f32_fv(k, op, a, grid, s, err, out) || dispatch_f32_lbm(k, op, a, grid, s, err, out) ||
         dispatch_f64_fv(k, op, a, grid, s, err, out) || dispatch_f64_lbm(k, op, a, grid, s, err, out) ||
         dispatch_f32_fv_q(k, op, a, grid, s, err, out) || dispatch_f32_lbm_q(k, op, a, grid, s, err, out) ||
         dispatch_f32_euler(k, op, a, grid, s, err, out) || dispatch_f32_d3q19(k, op, a, grid, s, err, out) ||
         dispatch_f32_e4m3b_lbm(k, op, a, grid, s, err, out) || dispatch_f32_e4m3b_fv(k, op, a, grid, s, err, out);
}

static size_t dispatch_op_of(const KernelKey& k, int op, const PatchArgs* a, int grid, hipStream_t s,
                             hipError_t* err) {
  size_t out = 0;
  if (!dispatch(k, op, a, grid, s, err, &out)) *err = hipErrorInvalidValue;
  return out;
}

hipError_t launch_step(const KernelKey& k, const PatchArgs& a, int npatch, hipStream_t s, bool ctl) {
  hipError_t e = hipSuccess;
  dispatch_op_of(k, ctl ? OP_CTL : 0, &a, npatch, s, &e);
  return e;
}

hipError_t launch_step_persistent(const KernelKey& k, const PatchArgs& a, int grid, hipStream_t s, bool ctl) {
  hipError_t e = hipSuccess;
  dispatch_op_of(k, (ctl ? OP_CTL : 0) | 3, &a, grid, s, &e);
  return e;
}

hipError_t launch_aux(const KernelKey& k, const PatchArgs& a, int npatch, hipStream_t s) {
  hipError_t e = hipSuccess;
  dispatch_op_of(k, 1, &a, npatch, s, &e);
  return e;
}

size_t kernel_lds_bytes(const KernelKey& k) {
  hipError_t e = hipSuccess;
  const size_t v = dispatch_op_of(k, 2, nullptr, 0, nullptr, &e);
  return e == hipSuccess ? v : 0;
}

const void* step_kernel_entry(const KernelKey& k, bool persistent, bool ctl) {
  hipError_t e = hipSuccess;
  const size_t v = dispatch_op_of(k, (ctl ? OP_CTL : 0) | (persistent ? 5 : 4), nullptr, 0, nullptr, &e);
  return e == hipSuccess ? reinterpret_cast<const void*>(v) : nullptr;
}

int kernel_threads(const KernelKey& k) {
  hipError_t e = hipSuccess;
  const size_t v = dispatch_op_of(k, 6, nullptr, 0, nullptr, &e);
  return e == hipSuccess ? (int)v : 0;
}

bool have_kernel(const KernelKey& k) { return kernel_lds_bytes(k) != 0; }

// 3-D kernels: halo floats per patch and scratch floats per workgroup.
static size_t kernel_size_op(const KernelKey& k, int op) {
  hipError_t e = hipSuccess;
  const size_t v = dispatch_op_of(k, op, nullptr, 0, nullptr, &e);
  return e == hipSuccess ? v : 0;
}
}  // namespace lbmz

using namespace lbmz;

struct lbmz_ctx {
  bool reference = false;
  int dtype = 0;
  size_t esize = 4;
  int n = 0, p = 0, npx = 0, npatch = 0, s = 0, levels = 0, wavelet = 0, rule = 0, scheme = 0;
  int dim = 2;
  float* scratch = nullptr;   // 3-D step: per-workgroup population staging
  int slots3 = 0;             // 3-D step: resident workgroups (scratch slices)
  int vf = VF_F32;   // ValueFormat of the records
  // execution of the step: persistent work-queue kernel, hipGraph chunks
  int exec_persistent = 0, exec_graph = 0, persist_grid = 0;
  hipGraph_t graph[2] = {nullptr, nullptr};      // GRAPH_STEPS launches from buffer parity 0 / 1
  hipGraphExec_t gexec[2] = {nullptr, nullptr};
  hipGraphNode_t gnode[2][6] = {};
  int graph_mode[2] = {-1, -1};                  // exec_mode() at instantiation
  PatchArgs gargs[6] = {};
  double* eps_patch = nullptr;   // per-patch thresholds (device), or null
  int8_t* lev_patch = nullptr;   // per-patch threshold level counts (device), or null
  float* features = nullptr;     // per-patch network inputs of the last step (device), or null
  bool features_valid = false;
  int nfields = 1, nslot = 1;
  double eps = 0.0;
  KernelKey key{};
  PatchArgs base{};
  int device = 0;
  hipStream_t stream = nullptr;
  void* (*ualloc)(size_t, void*) = nullptr;
  void (*ufree)(void*, void*) = nullptr;
  void* uuser = nullptr;
  bool allocated = false;
  // compressed store, double buffered
  uint8_t* pool[2] = {nullptr, nullptr};
  uint32_t* table[2] = {nullptr, nullptr};
  void* halo[2] = {nullptr, nullptr};
  double* partials[2] = {nullptr, nullptr};
  int64_t cap_bytes = 0;
  Ctrl* ctrl = nullptr;
  Ctrl* ctrl_host = nullptr;   // pinned
  int cur = 0;
  unsigned epoch_next = 1;
  uint64_t used16 = 0;         // store size of the current state, 16-byte units
  // dense buffers: staging (compressed context) or the state (reference context)
  void* dense[2] = {nullptr, nullptr};
  bool staging_dirty = false;
  bool have_state = false;
  int64_t steps = 0, regrows = 0;
  double ms_last = 0.0;
  hipEvent_t ev0 = nullptr, ev1 = nullptr;
  std::string err;
};

namespace {

int fail(lbmz_ctx* c, int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  if (c) c->err = buf;
  return code;
}

#define HIPCHK(c, expr)                                                                   \
  do {                                                                                    \
    hipError_t e_ = (expr);                                                               \
    if (e_ != hipSuccess) return fail((c), LBMZ_EDEVICE, "%s: %s", #expr, hipGetErrorString(e_)); \
  } while (0)

int64_t align_up(int64_t v, int64_t a) { return (v + a - 1) / a * a; }

int64_t ncoef(const lbmz_ctx* c) { return (int64_t)c->s * c->s * (c->dim == 3 ? c->s : 1); }
int64_t nwords(const lbmz_ctx* c) { return (ncoef(c) + 63) / 64; }

// Record bytes for nnz stored coefficients (layout of include/lbmz.h).
int64_t record_bytes(const lbmz_ctx* c, int64_t nnz, bool* is_mask) {
  const int64_t w = nwords(c);
  const bool mask = !(2 * nnz < 8 * w);
  if (is_mask) *is_mask = mask;
  const int64_t vb = align_up(nnz * (int64_t)c->esize, 8);
  return align_up(vb + (mask ? 8 * w : 2 * nnz), 16);
}

// Narrow records: samples per tile, bytes per detail code, and the section
// offsets of a record with ndet kept details and nocc occupied subbands.
int64_t narrow_samples(const lbmz_ctx* c) {
  const int64_t sc = ((c->s - 1) >> c->levels) + 1;
  return sc * sc;
}
// Bytes per detail code: 2 (binary16), 1 (E4M3); the bounded format's
// records use either (bit 63 of OCC), so its worst case is 2.
int64_t narrow_code_bytes(const lbmz_ctx* c) { return c->vf == VF_E4M3 ? 1 : 2; }
struct NarrowLayout {
  bool mask;
  int64_t hb, sb, vb, rb;
};
NarrowLayout narrow_layout(const lbmz_ctx* c, int64_t ndet, int64_t nocc, int64_t code_bytes) {
  NarrowLayout l;
  const int64_t w = nwords(c);
  l.mask = !(2 * ndet < 8 * w);
  l.hb = align_up(8 + 4 * nocc, 8);
  l.sb = l.hb + align_up(4 * narrow_samples(c), 8);
  l.vb = l.sb + align_up(ndet * code_bytes, 8);
  l.rb = align_up(l.vb + (l.mask ? 8 * w : 2 * ndet), 16);
  return l;
}

int64_t worst_store_bytes(const lbmz_ctx* c) {
  if (c->vf != VF_F32) {
    const int64_t nb = (int64_t)(c->levels + 1) * (c->levels + 1);
    return narrow_layout(c, ncoef(c), nb - 1, narrow_code_bytes(c)).rb * c->nfields * c->npatch;
  }
  return record_bytes(c, ncoef(c), nullptr) * c->nfields * c->npatch;
}

void* dalloc(lbmz_ctx* c, size_t bytes) {
  if (bytes == 0) bytes = 256;
  if (c->ualloc) return c->ualloc(bytes, c->uuser);
  void* p = nullptr;
  if (hipMalloc(&p, bytes) != hipSuccess) return nullptr;
  return p;
}

void dfree(lbmz_ctx* c, void* p) {
  if (!p) return;
  if (c->ufree) c->ufree(p, c->uuser);
  else (void)hipFree(p);
}

size_t cells(const lbmz_ctx* c) { return (size_t)c->n * c->n * (c->dim == 3 ? (size_t)c->n : 1); }
size_t dense_bytes(const lbmz_ctx* c) { return cells(c) * c->nfields * c->esize; }
size_t field_bytes(const lbmz_ctx* c) { return cells(c) * c->esize; }
size_t halo_bytes(const lbmz_ctx* c) {
  if (c->dim == 3) return sizeof(float) * kernel_size_op(c->key, 7) * (size_t)c->npatch;
  return c->esize * 4 * (size_t)c->nslot * c->s * c->npatch;
}

int ensure_buffers(lbmz_ctx* c) {
  if (c->allocated) return LBMZ_OK;
  HIPCHK(c, hipSetDevice(c->device));
  if (c->reference) {
    for (int b = 0; b < 2; ++b) {
      c->dense[b] = dalloc(c, dense_bytes(c));
      if (!c->dense[b]) return fail(c, LBMZ_ENOMEM, "dense state allocation failed");
      HIPCHK(c, hipMemsetAsync(c->dense[b], 0, dense_bytes(c), c->stream));
    }
    c->partials[0] = static_cast<double*>(dalloc(c, sizeof(double) * 256 * c->nfields));
    if (!c->partials[0]) return fail(c, LBMZ_ENOMEM, "partials allocation failed");
  } else {
    if (c->cap_bytes <= 0) c->cap_bytes = align_up(std::max<int64_t>(worst_store_bytes(c) / 4, 4096), 256);
    const size_t tb = sizeof(uint32_t) * 2 * (size_t)c->npatch * c->nfields;
    const size_t hb = halo_bytes(c);
    const size_t pb = sizeof(double) * (size_t)c->npatch * c->nfields;
    for (int b = 0; b < 2; ++b) {
      c->pool[b] = static_cast<uint8_t*>(dalloc(c, (size_t)c->cap_bytes));
      c->table[b] = static_cast<uint32_t*>(dalloc(c, tb));
      c->halo[b] = dalloc(c, hb);
      c->partials[b] = static_cast<double*>(dalloc(c, pb));
      if (!c->pool[b] || !c->table[b] || !c->halo[b] || !c->partials[b])
        return fail(c, LBMZ_ENOMEM, "store allocation failed");
      HIPCHK(c, hipMemsetAsync(c->table[b], 0, tb, c->stream));
      HIPCHK(c, hipMemsetAsync(c->halo[b], 0, hb, c->stream));
      HIPCHK(c, hipMemsetAsync(c->partials[b], 0, pb, c->stream));
    }
    if (c->dim == 3) {
      const size_t sb = sizeof(float) * kernel_size_op(c->key, 8) * (size_t)c->slots3;
      c->scratch = static_cast<float*>(dalloc(c, sb));
      if (!c->scratch) return fail(c, LBMZ_ENOMEM, "step scratch allocation failed");
    }
    c->ctrl = static_cast<Ctrl*>(dalloc(c, sizeof(Ctrl)));
    if (!c->ctrl) return fail(c, LBMZ_ENOMEM, "control block allocation failed");
    HIPCHK(c, hipHostMalloc((void**)&c->ctrl_host, sizeof(Ctrl), hipHostMallocDefault));
    Ctrl z{};
    z.abort_epoch = 0xffffffffu;
    *c->ctrl_host = z;
    HIPCHK(c, hipMemcpyAsync(c->ctrl, c->ctrl_host, sizeof(Ctrl), hipMemcpyHostToDevice, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
  }
  HIPCHK(c, hipEventCreate(&c->ev0));
  HIPCHK(c, hipEventCreate(&c->ev1));
  c->allocated = true;
  return LBMZ_OK;
}

int reset_ctrl(lbmz_ctx* c) {
  Ctrl z{};
  z.abort_epoch = 0xffffffffu;
  *c->ctrl_host = z;
  HIPCHK(c, hipMemcpyAsync(c->ctrl, c->ctrl_host, sizeof(Ctrl), hipMemcpyHostToDevice, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  return LBMZ_OK;
}

int read_ctrl(lbmz_ctx* c) {
  HIPCHK(c, hipMemcpyAsync(c->ctrl_host, c->ctrl, sizeof(Ctrl), hipMemcpyDeviceToHost, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  return LBMZ_OK;
}

// Grow both pools to `bytes`, keeping the current store.
int regrow(lbmz_ctx* c, int64_t bytes) {
  bytes = align_up(bytes, 256);
  if (bytes / 16 >= (int64_t)0xffffffffLL) return fail(c, LBMZ_EOVERFLOW, "store larger than 64 GiB");
  uint8_t* np[2] = {nullptr, nullptr};
  for (int b = 0; b < 2; ++b) {
    np[b] = static_cast<uint8_t*>(dalloc(c, (size_t)bytes));
    if (!np[b]) {
      for (int k = 0; k < b; ++k) dfree(c, np[k]);
      return fail(c, LBMZ_EOVERFLOW, "pool regrow to %lld bytes failed", (long long)bytes);
    }
  }
  if (c->used16 > 0)
    HIPCHK(c, hipMemcpyAsync(np[c->cur], c->pool[c->cur], (size_t)c->used16 * 16, hipMemcpyDeviceToDevice,
                             c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  for (int b = 0; b < 2; ++b) {
    dfree(c, c->pool[b]);
    c->pool[b] = np[b];
  }
  c->cap_bytes = bytes;
  return LBMZ_OK;
}

PatchArgs args_for(lbmz_ctx* c, int in, int out, unsigned epoch) {
  PatchArgs a = c->base;
  a.pool_in = c->pool[in];
  a.table_in = c->table[in];
  a.halo_in = c->halo[in];
  a.pool_out = c->pool[out];
  a.table_out = c->table[out];
  a.halo_out = c->halo[out];
  a.partials_out = c->partials[out];
  a.cap16 = (unsigned long long)(c->cap_bytes / 16);
  a.ctrl = c->ctrl;
  a.epoch = epoch;
  a.eps_patch = c->eps_patch;
  a.lev_patch = c->lev_patch;
  a.features = c->features;
  a.scratch = c->scratch;
  return a;
}

// Produce a new state with an auxiliary writing mode (AUX_INIT or AUX_COEF)
// from `src` (dense state or coefficient tiles); retries after a pool overflow.
int produce_state(lbmz_ctx* c, int mode, const void* src) {
  for (int attempt = 0; attempt < 64; ++attempt) {
    int rc = reset_ctrl(c);
    if (rc) return rc;
    const unsigned e = c->epoch_next++;
    PatchArgs a = args_for(c, c->cur, c->cur ^ 1, e);
    a.mode = mode;
    if (mode == AUX_INIT) a.dense_in = src;
    else a.coef_in = src;
    HIPCHK(c, launch_aux(c->key, a, c->npatch, c->stream));
    rc = read_ctrl(c);
    if (rc) return rc;
    const Ctrl& h = *c->ctrl_host;
    if (h.abort & ABORT_NONFINITE) return fail(c, LBMZ_ENAN, "non-finite value in the state being set");
    if (h.abort & ABORT_OVERFLOW) {
      const int64_t need = (int64_t)h.top16[e % 3] * 16;
      rc = regrow(c, std::max<int64_t>(2 * c->cap_bytes, need + need / 4));
      if (rc) return rc;
      c->regrows++;
      continue;
    }
    c->cur ^= 1;
    c->used16 = h.top16[e % 3];
    c->have_state = true;
    c->steps = 0;
    return LBMZ_OK;
  }
  return fail(c, LBMZ_EOVERFLOW, "pool kept overflowing");
}

int commit(lbmz_ctx* c) {
  if (c->reference || !c->staging_dirty) return LBMZ_OK;
  int rc = produce_state(c, AUX_INIT, c->dense[0]);
  if (rc) return rc;
  HIPCHK(c, hipStreamSynchronize(c->stream));
  dfree(c, c->dense[0]);
  c->dense[0] = nullptr;
  c->staging_dirty = false;
  return LBMZ_OK;
}

// Decompress every field of the current compressed state into dst [M][n][n]
// (field_only >= 0, 3-D: that field alone into dst [n][n][n]).
int decompress_all(lbmz_ctx* c, void* dst, int field_only = -1) {
  PatchArgs a = args_for(c, c->cur, c->cur, 0);
  a.mode = AUX_DECOMP;
  a.dense_out = dst;
  a.field_only = field_only;
  HIPCHK(c, launch_aux(c->key, a, c->npatch, c->stream));
  return LBMZ_OK;
}

// Dense staging holding the current state (compressed context).
int ensure_staging(lbmz_ctx* c, bool fill) {
  if (c->dense[0]) return LBMZ_OK;
  c->dense[0] = dalloc(c, dense_bytes(c));
  if (!c->dense[0]) return fail(c, LBMZ_ENOMEM, "staging allocation failed");
  if (fill && c->have_state) {
    int rc = decompress_all(c, c->dense[0]);
    if (rc) return rc;
  } else {
    HIPCHK(c, hipMemsetAsync(c->dense[0], 0, dense_bytes(c), c->stream));
  }
  return LBMZ_OK;
}

int copy_in(lbmz_ctx* c, void* dst, const void* src, size_t bytes, int on_device) {
  HIPCHK(c, hipMemcpyAsync(dst, src, bytes, on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice,
                           c->stream));
  if (!on_device) HIPCHK(c, hipStreamSynchronize(c->stream));
  return LBMZ_OK;
}

int validate_common(const lbmz_grid* g, const lbmz_scheme* sc, lbmz_ctx* c) {
  if (!g || !sc) return fail(c, LBMZ_EINVAL, "null argument");
  if (g->dim != 2 && g->dim != 3) return fail(c, LBMZ_EINVAL, "grids are 2-D or 3-D (dim=%d)", g->dim);
  if (!g->periodic) return fail(c, LBMZ_EINVAL, "only periodic grids are supported");
  if (g->dim == 3) {
    if (sc->kind != LBMZ_LBM_D3Q19_BGK) return fail(c, LBMZ_EINVAL, "3-D grids run the D3Q19 scheme only");
    if (g->n[0] <= 0 || g->n[0] != g->n[1] || g->n[0] != g->n[2] || g->n[0] > 2048)
      return fail(c, LBMZ_EINVAL, "3-D grid must be cubic with 0 < n <= 2048");
    if (sc->dtype != LBMZ_F32) return fail(c, LBMZ_EINVAL, "the D3Q19 scheme is float32");
  } else {
    if (sc->kind == LBMZ_LBM_D3Q19_BGK) return fail(c, LBMZ_EINVAL, "the D3Q19 scheme needs a 3-D grid");
    if (g->n[0] <= 0 || g->n[0] != g->n[1] || g->n[0] > (1 << 16))
      return fail(c, LBMZ_EINVAL, "grid must be square with 0 < n <= 65536");
  }
  if (sc->dtype != LBMZ_F32 && sc->dtype != LBMZ_F64) return fail(c, LBMZ_EINVAL, "bad dtype");
  if (sc->kind == LBMZ_FV_UPWIND) {
    const double vmax = std::max(std::fabs(sc->vel[0]), std::fabs(sc->vel[1]));
    if (!(vmax > 0.0) || !std::isfinite(vmax)) return fail(c, LBMZ_EINVAL, "FV velocity must be non-zero");
    if (!(sc->cfl > 0.0) || !std::isfinite(sc->cfl)) return fail(c, LBMZ_EINVAL, "cfl must be > 0");
  } else if (sc->kind == LBMZ_LBM_D2Q9_BGK || sc->kind == LBMZ_LBM_D3Q19_BGK) {
    if (!(sc->tau > 0.5) || !std::isfinite(sc->tau)) return fail(c, LBMZ_EINVAL, "tau must be > 1/2");
  } else if (sc->kind == LBMZ_EULER_RUSANOV) {
    if (!(sc->vel[0] > 0.0) || !std::isfinite(sc->vel[0]))
      return fail(c, LBMZ_EINVAL, "Euler: vel[0] (the bound of |u| + c) must be > 0");
    if (!(sc->cfl > 0.0) || !std::isfinite(sc->cfl)) return fail(c, LBMZ_EINVAL, "cfl must be > 0");
    if (!(sc->gamma > 1.0) || !std::isfinite(sc->gamma)) return fail(c, LBMZ_EINVAL, "gamma must be > 1");
  } else {
    return fail(c, LBMZ_EINVAL, "unknown scheme kind %d", (int)sc->kind);
  }
  c->n = (int)g->n[0];
  c->dim = g->dim;
  c->dtype = sc->dtype == LBMZ_F64 ? 1 : 0;
  c->esize = c->dtype ? 8 : 4;
  c->scheme = sc->kind == LBMZ_LBM_D2Q9_BGK ? S_LBM
              : sc->kind == LBMZ_EULER_RUSANOV ? S_EULER
              : sc->kind == LBMZ_LBM_D3Q19_BGK ? S_LBM3
                                               : S_FV;
  c->nfields = c->scheme == S_LBM ? 9 : (c->scheme == S_EULER ? 4 : (c->scheme == S_LBM3 ? 19 : 1));
  c->nslot = c->scheme == S_LBM ? 3 : c->nfields;
  PatchArgs& a = c->base;
  memset(&a, 0, sizeof a);
  a.field_only = -1;
  a.n = c->n;
  if (c->scheme == S_EULER) {
    a.dt_over_h = sc->cfl / sc->vel[0];
    a.gamma = sc->gamma;
  } else if (c->scheme == S_FV) {
    const double vmax = std::max(std::fabs(sc->vel[0]), std::fabs(sc->vel[1]));
    a.dt_over_h = sc->cfl / vmax;
    const double an[4] = {sc->vel[0], -sc->vel[0], sc->vel[1], -sc->vel[1]};
    for (int k = 0; k < 4; ++k) {
      a.cp[k] = std::max(an[k], 0.0);
      a.cm[k] = std::min(an[k], 0.0);
    }
  } else {
    a.omega = 1.0 / sc->tau;
  }
  HIPCHK(c, hipGetDevice(&c->device));
  return LBMZ_OK;
}

constexpr int GRAPH_STEPS = 6;   // a whole number of buffer swaps (2) and counter rotations (3)

void drop_graphs(lbmz_ctx* c) {
  for (int b = 0; b < 2; ++b) {
    if (c->gexec[b]) (void)hipGraphExecDestroy(c->gexec[b]);
    if (c->graph[b]) (void)hipGraphDestroy(c->graph[b]);
    c->gexec[b] = nullptr;
    c->graph[b] = nullptr;
    c->graph_mode[b] = -1;
  }
}

// The step kernel with per-patch controls runs when any of them is set.
bool uses_controls(const lbmz_ctx* c) {
  return c->dim == 2 && (c->eps_patch || c->lev_patch || c->features);
}

// Graph mode of the current launches: persistent or not, with controls or not.
int exec_mode(const lbmz_ctx* c) { return c->exec_persistent + 2 * (uses_controls(c) ? 1 : 0); }

int step_grid(lbmz_ctx* c) {
  if (c->dim == 3) return c->slots3;   // the 3-D step kernel is always persistent
  return c->exec_persistent ? c->persist_grid : c->npatch;
}

// Arguments of the six launches of a graph chunk starting at buffer parity `par`.
void chunk_args(lbmz_ctx* c, int par, unsigned e0) {
  for (int i = 0; i < GRAPH_STEPS; ++i) {
    const int in = par ^ (i & 1);
    c->gargs[i] = args_for(c, in, in ^ 1, e0 + (unsigned)i);
  }
}

hipKernelNodeParams node_params(lbmz_ctx* c, int i, void** slot) {
  hipKernelNodeParams p{};
  p.func = const_cast<void*>(step_kernel_entry(c->key, c->exec_persistent != 0, uses_controls(c)));
  p.gridDim = dim3((unsigned)step_grid(c));
  p.blockDim = dim3((unsigned)kernel_threads(c->key));
  p.sharedMemBytes = 0;
  slot[0] = &c->gargs[i];
  p.kernelParams = slot;
  p.extra = nullptr;
  return p;
}

// Launch GRAPH_STEPS steps from buffer parity `par` with epochs e0.. as one graph.
int launch_chunk(lbmz_ctx* c, int par, unsigned e0) {
  chunk_args(c, par, e0);
  void* slots[GRAPH_STEPS][1];
  if (!c->gexec[par] || c->graph_mode[par] != exec_mode(c)) {
    if (c->gexec[par]) (void)hipGraphExecDestroy(c->gexec[par]);
    if (c->graph[par]) (void)hipGraphDestroy(c->graph[par]);
    c->gexec[par] = nullptr;
    c->graph[par] = nullptr;
    HIPCHK(c, hipGraphCreate(&c->graph[par], 0));
    for (int i = 0; i < GRAPH_STEPS; ++i) {
      hipKernelNodeParams p = node_params(c, i, slots[i]);
      if (!p.func) return fail(c, LBMZ_EINVAL, "no step kernel for this configuration");
      hipGraphNode_t* dep = i ? &c->gnode[par][i - 1] : nullptr;
      HIPCHK(c, hipGraphAddKernelNode(&c->gnode[par][i], c->graph[par], dep, i ? 1 : 0, &p));
    }
    HIPCHK(c, hipGraphInstantiate(&c->gexec[par], c->graph[par], nullptr, nullptr, 0));
    c->graph_mode[par] = exec_mode(c);
  } else {
    for (int i = 0; i < GRAPH_STEPS; ++i) {
      hipKernelNodeParams p = node_params(c, i, slots[i]);
      HIPCHK(c, hipGraphExecKernelNodeSetParams(c->gexec[par], c->gnode[par][i], &p));
    }
  }
  HIPCHK(c, hipGraphLaunch(c->gexec[par], c->stream));
  return LBMZ_OK;
}

int launch_one(lbmz_ctx* c, int in, unsigned e) {
  PatchArgs a = args_for(c, in, in ^ 1, e);
  const bool ctl = uses_controls(c);
  if (c->exec_persistent) HIPCHK(c, launch_step_persistent(c->key, a, step_grid(c), c->stream, ctl));
  else HIPCHK(c, launch_step(c->key, a, step_grid(c), c->stream, ctl));
  return LBMZ_OK;
}

}  // namespace

extern "C" {

int lbmz_create(const lbmz_grid* grid, const lbmz_scheme* scheme, const lbmz_patch* patch, int levels,
                double eps, lbmz_ctx** out) {
  if (!out) return LBMZ_EINVAL;
  *out = nullptr;
  lbmz_ctx* c = new (std::nothrow) lbmz_ctx();
  if (!c) return LBMZ_ENOMEM;
  int rc = validate_common(grid, scheme, c);
  if (rc == LBMZ_OK && !patch) rc = fail(c, LBMZ_EINVAL, "null patch");
  if (rc == LBMZ_OK) {
    const int p = patch->p[0];
    if (c->dim == 3 && (patch->p[1] != p || patch->p[2] != p || !(p == 16 || p == 32)))
      rc = fail(c, LBMZ_EINVAL, "3-D patch must be cubic with p in {16, 32}");
    else if (c->dim == 3 && patch->wavelet != LBMZ_BL53)
      rc = fail(c, LBMZ_EINVAL, "3-D patches use the folded BL5/3 wavelet");
    else if (c->dim == 3 && patch->values != LBMZ_VALUES_F32)
      rc = fail(c, LBMZ_EINVAL, "3-D records store float32 values");
    else if (patch->p[1] != p || !(p == 8 || p == 16 || p == 32 || p == 64))
      rc = fail(c, LBMZ_EINVAL, "patch must be square with p in {8, 16, 32, 64}");
    else if (c->n % p != 0)
      rc = fail(c, LBMZ_EINVAL, "grid size %d is not a multiple of the patch size %d", c->n, p);
    else if (patch->wavelet != LBMZ_HAAR && patch->wavelet != LBMZ_BL53)
      rc = fail(c, LBMZ_EINVAL, "unknown wavelet");
    else if (patch->rule != LBMZ_THR_CAPPED && patch->rule != LBMZ_THR_CONSTANT && patch->rule != LBMZ_THR_ACCUM)
      rc = fail(c, LBMZ_EINVAL, "unknown threshold rule");
    else if (!(eps >= 0.0) || !std::isfinite(eps))
      rc = fail(c, LBMZ_EINVAL, "eps must be finite and >= 0");
    if (rc == LBMZ_OK) {
      int j = 0;
      while ((1 << j) < p) ++j;
      const int cap = patch->wavelet == LBMZ_BL53 ? j - 1 : j;
      if (levels < 0 || levels > cap)
        rc = fail(c, LBMZ_EINVAL, "levels=%d outside [0, %d] for this wavelet and patch size", levels, cap);
      c->p = p;
      c->npx = c->n / p;
      c->npatch = c->npx * c->npx * (c->dim == 3 ? c->npx : 1);
      c->wavelet = patch->wavelet == LBMZ_BL53 ? W_BL53 : W_HAAR;
      c->s = c->wavelet == W_BL53 ? p + 1 : p;
      c->levels = levels;
      c->rule = patch->rule == LBMZ_THR_CAPPED ? R_CAPPED : patch->rule == LBMZ_THR_ACCUM ? R_ACCUM : R_CONSTANT;
      c->eps = eps;
      if (patch->values != LBMZ_VALUES_F32 && patch->values != LBMZ_VALUES_F16 && patch->values != LBMZ_VALUES_E4M3 &&
          patch->values != LBMZ_VALUES_E4M3_BOUNDED)
        rc = fail(c, LBMZ_EINVAL, "unknown value format");
      else if (patch->values != LBMZ_VALUES_F32 && c->dtype != 0)
        rc = fail(c, LBMZ_EINVAL, "the narrow value formats need a float32 state");
      c->vf = patch->values == LBMZ_VALUES_F16        ? VF_F16
              : patch->values == LBMZ_VALUES_E4M3     ? VF_E4M3
              : patch->values == LBMZ_VALUES_E4M3_BOUNDED ? VF_E4M3B
                                                      : VF_F32;
      c->key = KernelKey{c->dtype, p, c->wavelet, c->scheme, c->vf};
    }
  }
  if (rc == LBMZ_OK) {
    const size_t lds = kernel_lds_bytes(c->key);
    int maxlds = 0;
    if (lds == 0) {
      rc = fail(c, LBMZ_EINVAL, "no kernel compiled for this dtype / patch size / wavelet / scheme");
    } else if (hipDeviceGetAttribute(&maxlds, hipDeviceAttributeMaxSharedMemoryPerBlock, c->device) != hipSuccess) {
      rc = fail(c, LBMZ_EDEVICE, "cannot query the LDS limit");
    } else if ((size_t)maxlds < lds) {
      rc = fail(c, LBMZ_EINVAL, "patch needs %zu bytes of LDS, device allows %d", lds, maxlds);
    }
  }
  if (rc == LBMZ_OK && c->dim == 3) {
    int ncu = 0, per_cu = 0;
    const void* fn = step_kernel_entry(c->key, true, false);
    if (hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, c->device) != hipSuccess || !fn ||
        hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, kernel_threads(c->key), 0) != hipSuccess)
      rc = fail(c, LBMZ_EDEVICE, "cannot size the 3-D step grid");
    c->slots3 = std::max(1, std::min(c->npatch, ncu * std::max(1, per_cu)));
    c->persist_grid = c->slots3;
  }
  if (rc == LBMZ_OK) {
    PatchArgs& a = c->base;
    a.npx = c->npx;
    a.npatch = c->npatch;
    a.npx_shift = -1;
    for (int k = 0; (1 << k) <= c->npx; ++k)
      if ((1 << k) == c->npx) a.npx_shift = k;
    a.levels = c->levels;
    a.rule = c->rule;
    a.eps = c->eps;
  }
  if (rc != LBMZ_OK) {
    // the message is lost with the context; callers get the code only
    delete c;
    return rc;
  }
  *out = c;
  return LBMZ_OK;
}

int lbmz_create_reference(const lbmz_grid* grid, const lbmz_scheme* scheme, lbmz_ctx** out) {
  if (!out) return LBMZ_EINVAL;
  *out = nullptr;
  lbmz_ctx* c = new (std::nothrow) lbmz_ctx();
  if (!c) return LBMZ_ENOMEM;
  c->reference = true;
  int rc = validate_common(grid, scheme, c);
  if (rc != LBMZ_OK) {
    delete c;
    return rc;
  }
  c->p = c->n;
  c->npx = 1;
  c->npatch = 1;
  c->s = c->n;
  c->have_state = true;
  *out = c;
  return LBMZ_OK;
}

int lbmz_set_allocator(lbmz_ctx* c, void* (*alloc)(size_t, void*), void (*free_)(void*, void*), void* user) {
  if (!c) return LBMZ_EINVAL;
  if (c->allocated) return fail(c, LBMZ_ESTATE, "allocator must be set before the first allocation");
  if ((alloc == nullptr) != (free_ == nullptr)) return fail(c, LBMZ_EINVAL, "alloc and free go together");
  c->ualloc = alloc;
  c->ufree = free_;
  c->uuser = user;
  return LBMZ_OK;
}

int lbmz_set_stream(lbmz_ctx* c, void* hip_stream) {
  if (!c) return LBMZ_EINVAL;
  c->stream = static_cast<hipStream_t>(hip_stream);
  return LBMZ_OK;
}

int lbmz_set_pool_capacity(lbmz_ctx* c, int64_t bytes) {
  if (!c) return LBMZ_EINVAL;
  if (c->reference) return LBMZ_OK;
  if (bytes < 16) return fail(c, LBMZ_EINVAL, "capacity must be >= 16 bytes");
  if (!c->allocated) {
    c->cap_bytes = align_up(bytes, 16);
    return LBMZ_OK;
  }
  if (c->have_state && bytes < (int64_t)c->used16 * 16)
    return fail(c, LBMZ_EINVAL, "capacity below the current store size");
  return regrow(c, bytes);
}

int lbmz_set_field(lbmz_ctx* c, int field, const void* src, size_t bytes, int src_on_device) {
  if (!c || !src) return LBMZ_EINVAL;
  if (field < 0 || field >= c->nfields) return fail(c, LBMZ_EINVAL, "field %d out of range", field);
  if (bytes != field_bytes(c)) return fail(c, LBMZ_EINVAL, "expected %zu bytes, got %zu", field_bytes(c), bytes);
  int rc = ensure_buffers(c);
  if (rc) return rc;
  if (c->reference) {
    rc = copy_in(c, static_cast<uint8_t*>(c->dense[c->cur]) + field * field_bytes(c), src, bytes, src_on_device);
    if (rc == LBMZ_OK) c->steps = 0;
    return rc;
  }
  rc = ensure_staging(c, true);
  if (rc) return rc;
  rc = copy_in(c, static_cast<uint8_t*>(c->dense[0]) + field * field_bytes(c), src, bytes, src_on_device);
  if (rc) return rc;
  c->staging_dirty = true;
  return LBMZ_OK;
}

int lbmz_set_macroscopic(lbmz_ctx* c, const void* rho, const void* ux, const void* uy, size_t bytes_each,
                         int on_device) {
  if (!c || !rho || !ux || !uy) return LBMZ_EINVAL;
  if (c->scheme != S_LBM) return fail(c, LBMZ_EINVAL, "macroscopic set-up is for the D2Q9 scheme (3-D: lbmz_set_macroscopic3)");
  if (bytes_each != field_bytes(c)) return fail(c, LBMZ_EINVAL, "expected %zu bytes per field", field_bytes(c));
  int rc = ensure_buffers(c);
  if (rc) return rc;
  void* tmp = dalloc(c, 3 * bytes_each);
  if (!tmp) return fail(c, LBMZ_ENOMEM, "temporary allocation failed");
  uint8_t* t8 = static_cast<uint8_t*>(tmp);
  rc = copy_in(c, t8, rho, bytes_each, on_device);
  if (!rc) rc = copy_in(c, t8 + bytes_each, ux, bytes_each, on_device);
  if (!rc) rc = copy_in(c, t8 + 2 * bytes_each, uy, bytes_each, on_device);
  void* dst = nullptr;
  if (!rc) {
    if (c->reference) {
      dst = c->dense[c->cur];
    } else {
      rc = ensure_staging(c, false);
      dst = c->dense[0];
    }
  }
  if (!rc) {
    hipError_t e = launch_equilibrium(c->dtype, t8, t8 + bytes_each, t8 + 2 * bytes_each, dst, c->n, c->stream);
    if (e != hipSuccess) rc = fail(c, LBMZ_EDEVICE, "equilibrium kernel: %s", hipGetErrorString(e));
  }
  if (!rc) {
    hipError_t e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) rc = fail(c, LBMZ_EDEVICE, "sync: %s", hipGetErrorString(e));
  }
  dfree(c, tmp);
  if (rc) return rc;
  if (c->reference) {
    c->steps = 0;
    return LBMZ_OK;
  }
  c->staging_dirty = true;
  return commit(c);
}

int lbmz_step(lbmz_ctx* c, int n) {
  if (!c) return LBMZ_EINVAL;
  if (n < 0) return fail(c, LBMZ_EINVAL, "negative step count");
  int rc = ensure_buffers(c);
  if (rc) return rc;
  rc = commit(c);
  if (rc) return rc;
  if (!c->reference && !c->have_state) {
    rc = ensure_staging(c, false);
    if (rc) return rc;
    c->staging_dirty = true;
    rc = commit(c);
    if (rc) return rc;
  }
  if (n == 0) {   // nothing to time: no event pair is recorded
    c->ms_last = 0.0;
    return LBMZ_OK;
  }
  HIPCHK(c, hipEventRecord(c->ev0, c->stream));
  if (c->reference) {
    for (int k = 0; k < n; ++k) {
      if (c->scheme == S_LBM3)
        HIPCHK(c, launch_reference_step3(c->dense[c->cur], c->dense[c->cur ^ 1], c->n, c->base.omega, c->stream));
      else
        HIPCHK(c, launch_reference_step(c->dtype, c->scheme, c->dense[c->cur], c->dense[c->cur ^ 1], c->n, c->base,
                                        c->stream));
      c->cur ^= 1;
    }
    HIPCHK(c, hipEventRecord(c->ev1, c->stream));
    HIPCHK(c, hipEventSynchronize(c->ev1));
    float ms = 0.f;
    HIPCHK(c, hipEventElapsedTime(&ms, c->ev0, c->ev1));
    c->ms_last = ms;
    c->steps += n;
    return LBMZ_OK;
  }
  int remaining = n;
  for (int attempt = 0; remaining > 0; ++attempt) {
    if (attempt > 64) return fail(c, LBMZ_EOVERFLOW, "pool kept overflowing");
    const unsigned e0 = c->epoch_next;
    const int cur0 = c->cur;
    for (int k = 0; k < remaining;) {
      if (c->exec_graph && remaining - k >= GRAPH_STEPS) {
        rc = launch_chunk(c, c->cur, c->epoch_next);
        if (rc) return rc;
        c->epoch_next += GRAPH_STEPS;
        k += GRAPH_STEPS;   // an even number of swaps: the parity is unchanged
      } else {
        rc = launch_one(c, c->cur, c->epoch_next++);
        if (rc) return rc;
        c->cur ^= 1;
        ++k;
      }
    }
    HIPCHK(c, hipEventRecord(c->ev1, c->stream));
    rc = read_ctrl(c);
    if (rc) return rc;
    const Ctrl h = *c->ctrl_host;
    if (h.abort == 0) {
      c->used16 = h.top16[(c->epoch_next - 1) % 3];
      c->steps += remaining;
      remaining = 0;
      break;
    }
    const int kbad = (int)(h.abort_epoch - e0);   // first failing step of this batch
    c->cur = cur0 ^ (kbad & 1);
    if (kbad > 0) c->used16 = h.top16[(h.abort_epoch - 1) % 3];
    c->steps += kbad;
    remaining -= kbad;
    if (h.abort & ABORT_NONFINITE) {
      reset_ctrl(c);
      c->features_valid = false;
      return fail(c, LBMZ_ENAN, "non-finite coefficient at step %lld; state kept at the previous step",
                  (long long)c->steps + 1);
    }
    const int64_t need = (int64_t)h.top16[h.abort_epoch % 3] * 16;
    rc = regrow(c, std::max<int64_t>(2 * c->cap_bytes, need + need / 4));
    if (rc) return rc;
    c->regrows++;
    rc = reset_ctrl(c);
    if (rc) return rc;
  }
  HIPCHK(c, hipEventSynchronize(c->ev1));
  float ms = 0.f;
  HIPCHK(c, hipEventElapsedTime(&ms, c->ev0, c->ev1));
  c->ms_last = ms;
  c->features_valid = c->features != nullptr && n > 0;
  return LBMZ_OK;
}

int lbmz_decompress_field(lbmz_ctx* c, int field, void* dst, size_t bytes, int dst_on_device) {
  if (!c || !dst) return LBMZ_EINVAL;
  if (field < 0 || field >= c->nfields) return fail(c, LBMZ_EINVAL, "field %d out of range", field);
  if (bytes != field_bytes(c)) return fail(c, LBMZ_EINVAL, "expected %zu bytes, got %zu", field_bytes(c), bytes);
  int rc = ensure_buffers(c);
  if (rc) return rc;
  const hipMemcpyKind kind = dst_on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost;
  if (c->reference) {
    HIPCHK(c, hipMemcpyAsync(dst, static_cast<uint8_t*>(c->dense[c->cur]) + field * field_bytes(c), bytes, kind,
                             c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    return LBMZ_OK;
  }
  rc = commit(c);
  if (rc) return rc;
  if (!c->have_state) {
    HIPCHK(c, dst_on_device ? hipMemsetAsync(dst, 0, bytes, c->stream) : hipSuccess);
    if (!dst_on_device) memset(dst, 0, bytes);
    HIPCHK(c, hipStreamSynchronize(c->stream));
    return LBMZ_OK;
  }
  // 3-D: the requested field alone (one n^3 buffer); 2-D: all fields (the
  // expansion reads every record of a patch at once)
  const bool one = c->dim == 3;
  void* tmp = dalloc(c, one ? field_bytes(c) : dense_bytes(c));
  if (!tmp) return fail(c, LBMZ_ENOMEM, "decompression scratch allocation failed");
  rc = decompress_all(c, tmp, one ? field : -1);
  if (!rc) {
    hipError_t e = hipMemcpyAsync(dst, static_cast<uint8_t*>(tmp) + (one ? 0 : field * field_bytes(c)), bytes, kind,
                                  c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) rc = fail(c, LBMZ_EDEVICE, "decompress copy: %s", hipGetErrorString(e));
  }
  dfree(c, tmp);
  return rc;
}

int lbmz_stats(lbmz_ctx* c, lbmz_stats_t* out) {
  if (!c || !out) return LBMZ_EINVAL;
  int rc = ensure_buffers(c);
  if (rc) return rc;
  rc = commit(c);
  if (rc) return rc;
  memset(out, 0, sizeof *out);
  out->steps = c->steps;
  out->dense_bytes = (int64_t)dense_bytes(c);
  out->nfields = c->nfields;
  out->npatch = c->npatch;
  out->regrows = c->regrows;
  out->ms_last_call = c->ms_last;
  if (c->reference) {
    const int nb = 256;
    HIPCHK(c, launch_dense_totals(c->dtype, c->dense[c->cur], c->nfields, cells(c), c->partials[0], nb, c->stream));
    std::vector<double> part((size_t)nb * c->nfields);
    HIPCHK(c, hipMemcpyAsync(part.data(), c->partials[0], part.size() * sizeof(double), hipMemcpyDeviceToHost,
                             c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    for (int f = 0; f < c->nfields && f < 16; ++f) {
      double s = 0.0;
      for (int b = 0; b < nb; ++b) s += part[(size_t)f * nb + b];
      out->totals[f] = s;
    }
    out->store_bytes = out->dense_bytes;
    out->capacity_bytes = out->dense_bytes;
    out->nnz_total = (int64_t)cells(c) * c->nfields;
    out->ratio = 1.0;
    return LBMZ_OK;
  }
  const size_t ne = (size_t)c->npatch * c->nfields;
  std::vector<uint32_t> tab(2 * ne);
  std::vector<double> part(ne);
  if (c->have_state) {
    HIPCHK(c, hipMemcpyAsync(tab.data(), c->table[c->cur], tab.size() * 4, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipMemcpyAsync(part.data(), c->partials[c->cur], part.size() * 8, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
  }
  int64_t rec = 0;
  for (size_t i = 0; i < ne; ++i) {
    const int64_t nnz = tab[2 * i + 1] & ~MASK_BIT;
    out->nnz_total += nnz;
    bool mask = false;
    rec += record_bytes(c, nnz, &mask);
    if (tab[2 * i + 1] & MASK_BIT) out->mask_records++;
    else out->list_records++;
  }
  // narrow records depend on their subband count too; the pool is packed
  // without gaps, so its used size is the sum of the record sizes
  if (c->vf != VF_F32) rec = c->have_state ? (int64_t)c->used16 * 16 : 0;
  for (int f = 0; f < c->nfields && f < 16; ++f) {
    double s = 0.0;
    for (int q = 0; q < c->npatch; ++q) s += part[(size_t)q * c->nfields + f];
    out->totals[f] = s;
  }
  out->store_bytes = rec + (int64_t)(ne * 8);
  out->capacity_bytes = c->cap_bytes;
  out->ratio = (double)out->dense_bytes / (double)out->store_bytes;
  return LBMZ_OK;
}

int lbmz_get_totals(lbmz_ctx* c, double* out, int count) {
  if (!c || !out) return LBMZ_EINVAL;
  if (count != c->nfields) return fail(c, LBMZ_EINVAL, "expected %d totals, got %d", c->nfields, count);
  int rc = ensure_buffers(c);
  if (rc) return rc;
  rc = commit(c);
  if (rc) return rc;
  if (c->reference) {
    const int nb = 256;
    HIPCHK(c, launch_dense_totals(c->dtype, c->dense[c->cur], c->nfields, cells(c), c->partials[0], nb, c->stream));
    std::vector<double> part((size_t)nb * c->nfields);
    HIPCHK(c, hipMemcpyAsync(part.data(), c->partials[0], part.size() * sizeof(double), hipMemcpyDeviceToHost,
                             c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    for (int f = 0; f < c->nfields; ++f) {
      double s = 0.0;
      for (int b = 0; b < nb; ++b) s += part[(size_t)f * nb + b];
      out[f] = s;
    }
    return LBMZ_OK;
  }
  const size_t ne = (size_t)c->npatch * c->nfields;
  std::vector<double> part(ne, 0.0);
  if (c->have_state) {
    HIPCHK(c, hipMemcpyAsync(part.data(), c->partials[c->cur], ne * 8, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
  }
  for (int f = 0; f < c->nfields; ++f) {
    double s = 0.0;
    for (int q = 0; q < c->npatch; ++q) s += part[(size_t)q * c->nfields + f];
    out[f] = s;
  }
  return LBMZ_OK;
}

int lbmz_set_macroscopic3(lbmz_ctx* c, const void* rho, const void* ux, const void* uy, const void* uz,
                          size_t bytes_each, int on_device) {
  if (!c || !rho || !ux || !uy || !uz) return LBMZ_EINVAL;
  if (c->scheme != S_LBM3) return fail(c, LBMZ_EINVAL, "lbmz_set_macroscopic3 is for the D3Q19 scheme");
  if (bytes_each != field_bytes(c)) return fail(c, LBMZ_EINVAL, "expected %zu bytes per field", field_bytes(c));
  int rc = ensure_buffers(c);
  if (rc) return rc;
  void* tmp = dalloc(c, 4 * bytes_each);
  if (!tmp) return fail(c, LBMZ_ENOMEM, "temporary allocation failed");
  uint8_t* t8 = static_cast<uint8_t*>(tmp);
  rc = copy_in(c, t8, rho, bytes_each, on_device);
  if (!rc) rc = copy_in(c, t8 + bytes_each, ux, bytes_each, on_device);
  if (!rc) rc = copy_in(c, t8 + 2 * bytes_each, uy, bytes_each, on_device);
  if (!rc) rc = copy_in(c, t8 + 3 * bytes_each, uz, bytes_each, on_device);
  void* dst = nullptr;
  if (!rc) {
    if (c->reference) {
      dst = c->dense[c->cur];
    } else {
      rc = ensure_staging(c, false);
      dst = c->dense[0];
    }
  }
  if (!rc) {
    hipError_t e = launch_equilibrium3(t8, t8 + bytes_each, t8 + 2 * bytes_each, t8 + 3 * bytes_each, dst, c->n,
                                       c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) rc = fail(c, LBMZ_EDEVICE, "equilibrium kernel: %s", hipGetErrorString(e));
  }
  dfree(c, tmp);
  if (rc) return rc;
  if (c->reference) {
    c->steps = 0;
    return LBMZ_OK;
  }
  c->staging_dirty = true;
  return commit(c);
}

int lbmz_store_size(lbmz_ctx* c, int64_t* pool_bytes, int64_t* table_entries) {
  if (!c || !pool_bytes || !table_entries) return LBMZ_EINVAL;
  if (c->reference) return fail(c, LBMZ_ESTATE, "a reference context has no compressed store");
  int rc = ensure_buffers(c);
  if (rc) return rc;
  rc = commit(c);
  if (rc) return rc;
  *pool_bytes = (int64_t)c->used16 * 16;
  *table_entries = (int64_t)c->npatch * c->nfields;
  return LBMZ_OK;
}

int lbmz_get_store(lbmz_ctx* c, uint32_t* table_host, void* pool_host, size_t pool_bytes) {
  if (!c || !table_host || (!pool_host && pool_bytes)) return LBMZ_EINVAL;
  int64_t pb = 0, te = 0;
  int rc = lbmz_store_size(c, &pb, &te);
  if (rc) return rc;
  if ((int64_t)pool_bytes != pb) return fail(c, LBMZ_EINVAL, "pool buffer is %zu bytes, store is %lld", pool_bytes,
                                             (long long)pb);
  HIPCHK(c, hipMemcpyAsync(table_host, c->table[c->cur], (size_t)te * 8, hipMemcpyDeviceToHost, c->stream));
  if (pb) HIPCHK(c, hipMemcpyAsync(pool_host, c->pool[c->cur], (size_t)pb, hipMemcpyDeviceToHost, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  return LBMZ_OK;
}

int lbmz_put_store(lbmz_ctx* c, const uint32_t* table_host, const void* pool_host, size_t pool_bytes) {
  if (!c || !table_host || (!pool_host && pool_bytes)) return LBMZ_EINVAL;
  if (c->reference) return fail(c, LBMZ_ESTATE, "a reference context has no compressed store");
  if (pool_bytes % 16) return fail(c, LBMZ_EINVAL, "pool size must be a multiple of 16");
  const size_t ne = (size_t)c->npatch * c->nfields;
  const uint8_t* pool = static_cast<const uint8_t*>(pool_host);
  const int64_t nc = ncoef(c), w = nwords(c);
  // narrow records: record indices of the sample positions (never in a mask or list)
  std::vector<uint64_t> sample_bits((size_t)w, 0ull);
  if (c->vf != VF_F32) {
    const int step = 1 << c->levels, p = c->p;
    for (int y = 0; y < c->s; y += step)
      for (int x = 0; x < c->s; x += step) {
        int64_t k;
        if (c->wavelet == W_HAAR || (x < p && y < p)) k = (int64_t)y * p + x;
        else if (x == p && y < p) k = (int64_t)p * p + y;
        else if (y == p && x < p) k = (int64_t)p * p + p + x;
        else k = (int64_t)p * p + 2 * p;
        sample_bits[(size_t)(k / 64)] |= 1ull << (k % 64);
      }
  }
  const int64_t nbands = (int64_t)(c->levels + 1) * (c->levels + 1);
  for (size_t i = 0; i < ne; ++i) {
    const uint64_t off = (uint64_t)table_host[2 * i] * 16;
    const int64_t nnz = table_host[2 * i + 1] & ~MASK_BIT;
    const bool tagged_mask = (table_host[2 * i + 1] & MASK_BIT) != 0;
    bool mask = false;
    if (nnz > nc) return fail(c, LBMZ_EINVAL, "record %zu: nnz %lld > %lld", i, (long long)nnz, (long long)nc);
    int64_t rb, vb;
    if (c->vf != VF_F32) {
      if (off + 8 > pool_bytes) return fail(c, LBMZ_EINVAL, "record %zu overruns the pool", i);
      uint64_t occ;
      memcpy(&occ, pool + off, 8);
      int64_t code_bytes = narrow_code_bytes(c);
      if (c->vf == VF_E4M3B) {   // bit 63: an E4M3 record, else binary16
        code_bytes = (occ >> 63) ? 1 : 2;
        occ &= ~(1ull << 63);
      }
      if ((occ & 1ull) || (nbands < 64 && (occ >> nbands) != 0))
        return fail(c, LBMZ_EINVAL, "record %zu: bad subband mask", i);
      const NarrowLayout l = narrow_layout(c, nnz, __builtin_popcountll(occ), code_bytes);
      mask = l.mask;
      rb = l.rb;
      vb = l.vb;
    } else {
      rb = record_bytes(c, nnz, &mask);
      vb = align_up(nnz * (int64_t)c->esize, 8);
    }
    if (mask != tagged_mask) return fail(c, LBMZ_EINVAL, "record %zu: wrong encoding tag", i);
    if (off + (uint64_t)rb > pool_bytes) return fail(c, LBMZ_EINVAL, "record %zu overruns the pool", i);
    if (mask) {
      int64_t cnt = 0;
      for (int64_t k = 0; k < w; ++k) {
        uint64_t word;
        memcpy(&word, pool + off + vb + 8 * k, 8);
        const int64_t valid = std::min<int64_t>(64, nc - 64 * k);
        if (valid < 64 && (word >> valid) != 0) return fail(c, LBMZ_EINVAL, "record %zu: bits past the tile", i);
        if (word & sample_bits[(size_t)k]) return fail(c, LBMZ_EINVAL, "record %zu: sample in the detail mask", i);
        cnt += __builtin_popcountll(word);
      }
      if (cnt != nnz) return fail(c, LBMZ_EINVAL, "record %zu: mask count %lld != nnz", i, (long long)cnt);
    } else {
      int64_t prev = -1;
      for (int64_t k = 0; k < nnz; ++k) {
        uint16_t t;
        memcpy(&t, pool + off + vb + 2 * k, 2);
        if ((int64_t)t <= prev || t >= nc || ((sample_bits[t / 64] >> (t % 64)) & 1ull))
          return fail(c, LBMZ_EINVAL, "record %zu: bad index list", i);
        prev = t;
      }
    }
  }
  int rc = ensure_buffers(c);
  if (rc) return rc;
  if ((int64_t)pool_bytes > c->cap_bytes) {
    c->used16 = 0;
    rc = regrow(c, (int64_t)pool_bytes);
    if (rc) return rc;
  }
  HIPCHK(c, hipMemcpyAsync(c->table[c->cur], table_host, ne * 8, hipMemcpyHostToDevice, c->stream));
  if (pool_bytes) HIPCHK(c, hipMemcpyAsync(c->pool[c->cur], pool_host, pool_bytes, hipMemcpyHostToDevice, c->stream));
  PatchArgs a = args_for(c, c->cur, c->cur, 0);
  a.mode = AUX_RESTORE;
  HIPCHK(c, launch_aux(c->key, a, c->npatch, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  if (c->dense[0]) {
    dfree(c, c->dense[0]);
    c->dense[0] = nullptr;
  }
  c->staging_dirty = false;
  c->used16 = pool_bytes / 16;
  c->have_state = true;
  c->steps = 0;
  return LBMZ_OK;
}

int lbmz_set_coefficients(lbmz_ctx* c, const void* coef, size_t bytes, int on_device) {
  if (!c || !coef) return LBMZ_EINVAL;
  if (c->reference) return fail(c, LBMZ_ESTATE, "a reference context has no compressed store");
  const size_t want = (size_t)c->npatch * c->nfields * ncoef(c) * c->esize;
  if (bytes != want) return fail(c, LBMZ_EINVAL, "expected %zu bytes of coefficients, got %zu", want, bytes);
  int rc = ensure_buffers(c);
  if (rc) return rc;
  const void* src = coef;
  void* tmp = nullptr;
  if (!on_device) {
    tmp = dalloc(c, bytes);
    if (!tmp) return fail(c, LBMZ_ENOMEM, "temporary allocation failed");
    rc = copy_in(c, tmp, coef, bytes, 0);
    src = tmp;
  }
  if (!rc) rc = produce_state(c, AUX_COEF, src);
  if (!rc) {
    hipError_t e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) rc = fail(c, LBMZ_EDEVICE, "sync: %s", hipGetErrorString(e));
  }
  dfree(c, tmp);
  if (!rc && c->dense[0]) {
    dfree(c, c->dense[0]);
    c->dense[0] = nullptr;
    c->staging_dirty = false;
  }
  return rc;
}

int lbmz_set_patch_eps(lbmz_ctx* c, const double* eps, size_t count, int on_device) {
  if (!c) return LBMZ_EINVAL;
  if (c->reference) return fail(c, LBMZ_ESTATE, "a reference context has no threshold");
  if (count == 0) {
    if (c->eps_patch) {
      HIPCHK(c, hipStreamSynchronize(c->stream));
      dfree(c, c->eps_patch);
      c->eps_patch = nullptr;
    }
    return LBMZ_OK;
  }
  if (!eps) return LBMZ_EINVAL;
  if (c->dim == 3) return fail(c, LBMZ_EINVAL, "per-patch thresholds are for 2-D grids");
  if (c->vf != VF_F32) return fail(c, LBMZ_EINVAL, "per-patch thresholds need float32 records");
  if (count != (size_t)c->npatch)
    return fail(c, LBMZ_EINVAL, "expected %d per-patch thresholds, got %zu", c->npatch, count);
  if (!on_device) {
    for (size_t q = 0; q < count; ++q)
      if (!(eps[q] >= 0.0) || !std::isfinite(eps[q]))
        return fail(c, LBMZ_EINVAL, "threshold of patch %zu must be finite and >= 0", q);
  }
  if (!c->eps_patch) {
    c->eps_patch = static_cast<double*>(dalloc(c, count * sizeof(double)));
    if (!c->eps_patch) return fail(c, LBMZ_ENOMEM, "per-patch threshold allocation failed");
  }
  return copy_in(c, c->eps_patch, eps, count * sizeof(double), on_device);
}

int lbmz_set_patch_levels(lbmz_ctx* c, const int* levels, size_t count) {
  if (!c) return LBMZ_EINVAL;
  if (c->reference) return fail(c, LBMZ_ESTATE, "a reference context has no threshold");
  if (count == 0) {
    if (c->lev_patch) {
      HIPCHK(c, hipStreamSynchronize(c->stream));
      dfree(c, c->lev_patch);
      c->lev_patch = nullptr;
    }
    return LBMZ_OK;
  }
  if (!levels) return LBMZ_EINVAL;
  if (c->dim == 3) return fail(c, LBMZ_EINVAL, "per-patch level counts are for 2-D grids");
  if (c->vf != VF_F32) return fail(c, LBMZ_EINVAL, "per-patch level counts need float32 records");
  if (count != (size_t)c->npatch)
    return fail(c, LBMZ_EINVAL, "expected %d per-patch level counts, got %zu", c->npatch, count);
  std::vector<int8_t> lv(count);
  for (size_t q = 0; q < count; ++q) {
    if (levels[q] < 0 || levels[q] > c->levels)
      return fail(c, LBMZ_EINVAL, "level count %d of patch %zu outside [0, %d]", levels[q], q, c->levels);
    lv[q] = (int8_t)levels[q];
  }
  if (!c->lev_patch) {
    c->lev_patch = static_cast<int8_t*>(dalloc(c, count));
    if (!c->lev_patch) return fail(c, LBMZ_ENOMEM, "per-patch level allocation failed");
  }
  return copy_in(c, c->lev_patch, lv.data(), count, 0);
}

int lbmz_enable_features(lbmz_ctx* c, int on) {
  if (!c) return LBMZ_EINVAL;
  if (c->reference) return fail(c, LBMZ_ESTATE, "a reference context has no coefficients");
  if (on) {
    if (c->p != 64) return fail(c, LBMZ_EINVAL, "patch features need 64 x 64 patches");
    if (c->dim != 2 || c->vf != VF_F32) return fail(c, LBMZ_EINVAL, "patch features need 2-D float32 records");
    if (!c->features) {
      c->features = static_cast<float*>(dalloc(c, (size_t)c->npatch * c->nfields * 4 * 64 * sizeof(float)));
      if (!c->features) return fail(c, LBMZ_ENOMEM, "feature buffer allocation failed");
    }
  } else if (c->features) {
    HIPCHK(c, hipStreamSynchronize(c->stream));
    dfree(c, c->features);
    c->features = nullptr;
  }
  c->features_valid = false;
  return LBMZ_OK;
}

int lbmz_get_features(lbmz_ctx* c, float* dst, size_t bytes, int dst_on_device) {
  if (!c || !dst) return LBMZ_EINVAL;
  if (!c->features) return fail(c, LBMZ_ESTATE, "features are not enabled");
  if (!c->features_valid) return fail(c, LBMZ_ESTATE, "no step has written the features yet");
  const size_t want = (size_t)c->npatch * c->nfields * 4 * 64 * sizeof(float);
  if (bytes != want) return fail(c, LBMZ_EINVAL, "expected %zu bytes of features, got %zu", want, bytes);
  HIPCHK(c, hipMemcpyAsync(dst, c->features, bytes, dst_on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost,
                           c->stream));
  if (!dst_on_device) HIPCHK(c, hipStreamSynchronize(c->stream));
  return LBMZ_OK;
}

int lbmz_set_execution(lbmz_ctx* c, int persistent, int graph) {
  if (!c) return LBMZ_EINVAL;
  if (c->reference) return LBMZ_OK;
  if ((persistent != 0 && persistent != 1) || (graph != 0 && graph != 1))
    return fail(c, LBMZ_EINVAL, "execution flags must be 0 or 1");
  if (persistent && c->persist_grid <= 0) {
    int ncu = 0, per_cu = 0;
    HIPCHK(c, hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, c->device));
    const void* fn = step_kernel_entry(c->key, true, false);
    if (!fn) return fail(c, LBMZ_EINVAL, "no persistent kernel for this configuration");
    HIPCHK(c, hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, kernel_threads(c->key), 0));
    c->persist_grid = std::max(1, std::min(c->npatch, ncu * std::max(1, per_cu)));
  }
  HIPCHK(c, hipStreamSynchronize(c->stream));
  c->exec_persistent = persistent;
  c->exec_graph = graph;
  return LBMZ_OK;
}

int lbmz_get_execution(lbmz_ctx* c, int* persistent, int* graph) {
  if (!c || !persistent || !graph) return LBMZ_EINVAL;
  *persistent = c->exec_persistent;
  *graph = c->exec_graph;
  return LBMZ_OK;
}

int lbmz_autotune(lbmz_ctx* c, int steps_per_variant, float* ms_out) {
  if (!c || steps_per_variant < 1) return LBMZ_EINVAL;
  if (c->reference) return LBMZ_OK;
  float best = 0.f;
  int bp = 0, bg = 0;
  for (int v = 0; v < 4; ++v) {
    const int pv = v >> 1, gv = v & 1;
    int rc = lbmz_set_execution(c, pv, gv);
    if (rc) return rc;
    rc = lbmz_step(c, steps_per_variant);   // warms the variant (graph instantiation)
    if (rc) return rc;
    rc = lbmz_step(c, steps_per_variant);
    if (rc) return rc;
    const float ms = c->ms_last / (float)steps_per_variant;
    if (ms_out) ms_out[v] = ms;
    if (v == 0 || ms < best) {
      best = ms;
      bp = pv;
      bg = gv;
    }
  }
  return lbmz_set_execution(c, bp, bg);
}

const char* lbmz_last_error(const lbmz_ctx* c) { return c ? c->err.c_str() : "null context"; }

void lbmz_destroy(lbmz_ctx* c) {
  if (!c) return;
  if (c->allocated) (void)hipStreamSynchronize(c->stream);
  drop_graphs(c);
  for (int b = 0; b < 2; ++b) {
    dfree(c, c->pool[b]);
    dfree(c, c->table[b]);
    dfree(c, c->halo[b]);
    dfree(c, c->partials[b]);
    dfree(c, c->dense[b]);
  }
  dfree(c, c->ctrl);
  dfree(c, c->scratch);
  dfree(c, c->eps_patch);
  dfree(c, c->lev_patch);
  dfree(c, c->features);
  if (c->ctrl_host) (void)hipHostFree(c->ctrl_host);
  if (c->ev0) (void)hipEventDestroy(c->ev0);
  if (c->ev1) (void)hipEventDestroy(c->ev1);
  delete c;
}

}  // extern "C"
