// Three-dimensional patch kernels for gfx950: D3Q19 BGK lattice Boltzmann on
// cubic patches of 2^J cells, folded BL5/3 tiles of (2^J + 1)^3 nodes
// (Section 3.1.1: shared bordering values, one ghost layer), tensor 3-D
// transform (the 1-D transform along x on every line, then y, then z; the
// inverse z, y, x), thresholds of Section 2.2 with one rank per dimension.
//
// A 33^3 tile of 19 float32 populations is 2.7 MB, far beyond the 160 KB of
// LDS of a CU, so one step of a patch runs field by field through LDS (one
// field tile, 143.7 KB at P = 32) with the populations staged in a per-
// workgroup slice of global scratch:
//   A  for every population i: expand its record into LDS (S1), inverse
//      transform z, y, x (S2), and write the pull-streamed population
//      f_i^in(n) = f_i(n - c_i) to scratch; values that come from outside
//      the tile are read from the neighbours' exported halo (S3);
//   B  BGK collision node by node in scratch (S4);
//   C  for every population: load it into LDS, forward transform x, y, z
//      (S5), hard threshold (S6), compaction into a record of the output pool
//      (S7), FP64 trapezoid total from the coarse samples (S9), inverse
//      transform of the thresholded tile and export of the planes and lines
//      the neighbours pull from (S8).
// The step kernel is persistent: one workgroup per scratch slice takes
// patches from an atomic work queue until none is left.
//
// Record of one (patch, field): the kept coefficients in ascending flat tile
// index t = x + S*y + S*S*z, then (8-byte aligned) the u16 indices t when
// 2*nnz < 8*W, W = ceil(S^3 / 64), else W u64 mask words with bit t%64 of
// word t/64 set for a kept coefficient; padded to 16 bytes.
//
// Halo of one patch (floats): six faces, face 2a + (sign > 0) holding, for
// the five populations whose velocity has that sign along axis a (in
// numbering order), the tile plane at coordinate P - 1 (positive sign) or 1
// (negative sign), indexed u + S*v over the other two axes in increasing
// order; then twelve edges, edge 4*pair + (c_a > 0) + 2*(c_b > 0) for the
// axis pairs (x,y), (x,z), (y,z), holding the one population with that
// velocity on the line at those two coordinates, indexed by the third axis.
#include "lbmz_patch_kernel.h"

namespace lbmz {

struct D3Q19L {
  static constexpr int C[19][3] = {{0, 0, 0},  {1, 0, 0},  {-1, 0, 0}, {0, 1, 0},   {0, -1, 0},
                                   {0, 0, 1},  {0, 0, -1}, {1, 1, 0},  {-1, -1, 0}, {1, -1, 0},
                                   {-1, 1, 0}, {1, 0, 1},  {-1, 0, -1}, {1, 0, -1}, {-1, 0, 1},
                                   {0, 1, 1},  {0, -1, -1}, {0, 1, -1}, {0, -1, 1}};
  // position of population i among the populations with the same velocity
  // component along axis a (its slot in a halo face)
  static constexpr int slot(int i, int a) {
    int k = 0;
    for (int j = 0; j < i; ++j) k += (C[j][a] == C[i][a]) ? 1 : 0;
    return k;
  }
};

template <int P_>
struct Cfg3 {
  static constexpr int P = P_;
  static constexpr int S = P + 1;
  static constexpr int S2 = S * S;
  static constexpr int S3 = S * S * S;
  static constexpr int M = 19;
  static constexpr int NT = 1024;
  static constexpr int NW = NT / 64;
  static constexpr int W = (S3 + 63) / 64;
  static constexpr int LMAX = ilog2c(P) - 1;
  static constexpr int FACE = 5 * S2;
  static constexpr int HALO = 6 * FACE + 12 * S;
  static constexpr int SF = (S3 + 3) & ~3;   // scratch floats per field (16-byte aligned slices)
  static_assert(W <= NT, "one scan entry per thread");
  static_assert(S3 < 65536, "u16 indices");
};

template <class C>
struct Smem3 {
  float tile[C::S3];
  uint32_t pre[C::W];   // per-chunk counts, then their exclusive prefix
  uint32_t wsum[C::NW];
  double red[C::NW];
  uint32_t misc[8];
};

// Exclusive prefix of a[0 .. n) in place (n <= NT); returns the total to all.
template <class C, class SM>
__device__ __forceinline__ uint32_t scan_counts(uint32_t* a, int n, SM& sm) {
  const int t = threadIdx.x;
  const int lane = lane_id();
  const int wave = wave_id();
  const uint32_t v = t < n ? a[t] : 0u;
  const int incl = wave_incl_scan((int)v);
  if (lane == 63) sm.wsum[wave] = (uint32_t)incl;
  __syncthreads();
  uint32_t off = 0, tot = 0;
  for (int w = 0; w < C::NW; ++w) {
    const uint32_t s = sm.wsum[w];
    off += (w < wave) ? s : 0u;
    tot += s;
  }
  if (t < n) a[t] = off + (uint32_t)incl - v;
  __syncthreads();
  return tot;
}

// Set bits of m below the calling lane.
__device__ __forceinline__ uint32_t mbcnt64(unsigned long long m) {
  return __builtin_amdgcn_mbcnt_hi((unsigned)(m >> 32), __builtin_amdgcn_mbcnt_lo((unsigned)m, 0u));
}

// ---------------------------------------------------------------------------
// Lines of the tile in registers: DIR 0 = x-lines, 1 = y-lines, 2 = z-lines.
// ---------------------------------------------------------------------------
// S6 on a z-line after its forward transform: the x and y ranks are those of
// the line, the z rank is that of the element (a compile-time index).  A
// detail (a detail in at least one dimension) with |c| < eps * 2^r is zeroed,
// r = max (capped), sum (accumulation) or 0 (constant) of the three ranks.
// Returns true when the line keeps a detail.
template <class C>
__device__ __forceinline__ bool threshold_zline(float* v, int x, int y, int L, float eps, int rule) {
  const int rx = dim_rank(x, L), ry = dim_rank(y, L);
  const bool dxy = rx >= 0 || ry >= 0;
  const int ax = rx < 0 ? 0 : rx, ay = ry < 0 ? 0 : ry;
  const int rmax = ax > ay ? ax : ay, rsum = ax + ay;
  const int lmask = (1 << L) - 1;
  bool kept = false;
#pragma unroll
  for (int k = 0; k < C::S; ++k) {
    const bool zs = (k & lmask) == 0;
    const int rz = zs ? 0 : L - 1 - __builtin_ctz((unsigned)(k == 0 ? 1 : k));
    const int r = rule == R_CAPPED ? (rmax > rz ? rmax : rz) : (rule == R_ACCUM ? rsum + rz : 0);
    if ((dxy || !zs) && fabsf(v[k]) < ldexpf(eps, r)) v[k] = 0.f;
    kept |= (dxy || !zs) && v[k] != 0.f;
  }
  return kept;
}

template <class C, int DIR, bool FWD, bool THR = false>
__device__ __forceinline__ void line_pass(float* tile, int L, float eps = 0.f, int rule = 0,
                                          uint32_t* samples_only = nullptr) {
  using LF = Lift<float, C::S, W_BL53, 1, C::LMAX>;
  for (int l = threadIdx.x; l < C::S2; l += C::NT) {
    int base, stride;
    if constexpr (DIR == 0) {
      base = l * C::S;
      stride = 1;
    } else if constexpr (DIR == 1) {
      const int z = l / C::S;
      base = (l - z * C::S) + z * C::S2;
      stride = C::S;
    } else {
      base = l;
      stride = C::S2;
    }
    float v[C::S];
#pragma unroll
    for (int k = 0; k < C::S; ++k) v[k] = tile[base + k * stride];
    if constexpr (FWD) LF::fwd(v, L);
    else LF::inv(v, L);
    if constexpr (THR) {
      static_assert(DIR == 2, "the threshold rides on the last (z) forward pass");
      const int y = l / C::S;
      if (threshold_zline<C>(v, l - y * C::S, y, L, eps, rule)) *samples_only = 0u;
    }
#pragma unroll
    for (int k = 0; k < C::S; ++k) tile[base + k * stride] = v[k];
  }
  __syncthreads();
}

// Forward transform x, y, z, and the hard threshold of Section 2.2 fused into
// the z pass.  *samples_only ends up 1 when no detail survives the threshold,
// i.e. when every kept coefficient is a coarse sample.
template <class C>
__device__ __forceinline__ void forward3_threshold(const PatchArgs& a, float* tile, uint32_t* samples_only) {
  if (threadIdx.x == 0) *samples_only = 1u;   // until a line keeps a detail (after two barriers)
  line_pass<C, 0, true>(tile, a.levels);
  line_pass<C, 1, true>(tile, a.levels);
  line_pass<C, 2, true, true>(tile, a.levels, (float)a.eps, a.rule, samples_only);
}

template <class C>
__device__ __forceinline__ void inverse3(float* tile, int L) {
  line_pass<C, 2, false>(tile, L);
  line_pass<C, 1, false>(tile, L);
  line_pass<C, 0, false>(tile, L);
}

// inverse3 of a tile whose coefficients are coarse samples only (nonzero at
// most on the lattice of nodes whose three indices are multiples of 2^LC).
// At each pass only the lines through that lattice along the axes already
// inverted are nonzero, their details are zero, and the predict steps alone
// invert them: the other lines stay zero and each update would subtract
// exact zeros, so the bits are those of inverse3.  LC is a compile-time
// level count, so that the lattice positions are constants.
template <class C, int LC>
__device__ void inverse3_samples_l(float* tile) {
  using LF = Lift<float, C::S, W_BL53, 1, C::LMAX>;
  constexpr int SMASK = (1 << LC) - 1;
  // z-lines (x, y) with x and y on the lattice
  for (int l = threadIdx.x; l < C::S2; l += C::NT) {
    const int y = l / C::S;
    const int x = l - y * C::S;
    if (((x | y) & SMASK) == 0) {
      float v[C::S];
#pragma unroll
      for (int k = 0; k < C::S; ++k) v[k] = (k & SMASK) == 0 ? tile[l + k * C::S2] : 0.f;
      LF::inv_samples(v, LC);
#pragma unroll
      for (int k = 0; k < C::S; ++k) tile[l + k * C::S2] = v[k];
    }
  }
  __syncthreads();
  // y-lines (x, z) with x on the lattice
  for (int l = threadIdx.x; l < C::S2; l += C::NT) {
    const int z = l / C::S;
    const int x = l - z * C::S;
    if ((x & SMASK) == 0) {
      const int base = x + z * C::S2;
      float v[C::S];
#pragma unroll
      for (int k = 0; k < C::S; ++k) v[k] = (k & SMASK) == 0 ? tile[base + k * C::S] : 0.f;
      LF::inv_samples(v, LC);
#pragma unroll
      for (int k = 0; k < C::S; ++k) tile[base + k * C::S] = v[k];
    }
  }
  __syncthreads();
  // x-lines, every one
  for (int l = threadIdx.x; l < C::S2; l += C::NT) {
    const int base = l * C::S;
    float v[C::S];
#pragma unroll
    for (int k = 0; k < C::S; ++k) v[k] = (k & SMASK) == 0 ? tile[base + k] : 0.f;
    LF::inv_samples(v, LC);
#pragma unroll
    for (int k = 0; k < C::S; ++k) tile[base + k] = v[k];
  }
  __syncthreads();
}

// The samples-only inverse for a run-time level count 2 <= L <= LMAX.
template <class C, int LC = 2>
__device__ __forceinline__ void inverse3_samples(float* tile, int L) {
  if constexpr (LC <= C::LMAX) {
    if (L == LC) inverse3_samples_l<C, LC>(tile);
    else inverse3_samples<C, LC + 1>(tile, L);
  }
}

// Flags of the step in Smem3::misc: the record just expanded holds coarse
// samples only; the thresholded tile being compacted keeps coarse samples only.
constexpr int MISC_SAMPLES_IN = 5, MISC_SAMPLES_OUT = 7;

// Optional per-phase clocks of the 3-D step (profiling builds compiled with
// -DLBMZ_PHASE_CLOCK; the product build has none): accumulated wall-clock
// ticks per workgroup and phase.
#ifdef LBMZ_PHASE_CLOCK
static __device__ unsigned long long lbmz_phase3[1024 * 16];
#define P3_START() unsigned long long p3_t = wall_clock64()
#define P3_MARK(k)                                                                  \
  do {                                                                              \
    if (threadIdx.x == 0 && blockIdx.x < 1024) {                                    \
      const unsigned long long t_ = wall_clock64();                                 \
      lbmz_phase3[blockIdx.x * 16 + (k)] += t_ - p3_t;                              \
      p3_t = t_;                                                                    \
    }                                                                               \
  } while (0)
#else
#define P3_START() \
  do {             \
  } while (0)
#define P3_MARK(k) \
  do {             \
  } while (0)
#endif

// ---------------------------------------------------------------------------
// S1: record (patch q, field f) of the input store -> LDS tile
// ---------------------------------------------------------------------------
template <class C, class SM>
__device__ void expand_field(const PatchArgs& a, int q, int f, SM& sm) {
  const int tid = threadIdx.x;
  const int lane = lane_id();
  const int wave = wave_id();
  const size_t e = 2 * ((size_t)q * C::M + f);
  const uint32_t off16 = a.table_in[e];
  const uint32_t w = a.table_in[e + 1];
  const uint32_t nnz = w & ~MASK_BIT;
  const uint8_t* rec = a.pool_in + 16ull * off16;
  const float* vals = reinterpret_cast<const float*>(rec);
  const uint32_t vb = (4u * nnz + 7u) & ~7u;
  if (w & MASK_BIT) {
    const unsigned long long* words = reinterpret_cast<const unsigned long long*>(rec + vb);
    if (tid == 0) sm.misc[MISC_SAMPLES_IN] = 0u;   // a dense record
    if (tid < C::W) sm.pre[tid] = (uint32_t)__popcll(words[tid]);
    __syncthreads();
    scan_counts<C>(sm.pre, C::W, sm);
    constexpr int U = 4;   // chunks per wave and iteration (independent loads in flight)
    for (int c0 = wave; c0 < C::W; c0 += U * C::NW) {
      unsigned long long word[U];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int c = c0 + u * C::NW;
        word[u] = c < C::W ? words[c] : 0ull;
      }
      float v[U];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int c = c0 + u * C::NW;
        const bool bit = ((word[u] >> lane) & 1ull) != 0ull;
        v[u] = bit ? vals[sm.pre[c] + mbcnt64(word[u])] : 0.f;
      }
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int t = 64 * (c0 + u * C::NW) + lane;
        if (t < C::S3) sm.tile[t] = v[u];
      }
    }
  } else {
    const uint16_t* idx = reinterpret_cast<const uint16_t*>(rec + vb);
    // the first NT entries are loaded before the zeroing, under which their
    // latency passes; they are scattered after the barrier
    int k0 = -1;
    float v0 = 0.f;
    if (tid < (int)nnz) {
      k0 = idx[tid];
      v0 = vals[tid];
    }
    if (tid == 0) sm.misc[MISC_SAMPLES_IN] = 1u;   // until a node off the sample lattice is scattered
    zero_span<float>(sm.tile, C::S3, tid, C::NT);
    __syncthreads();
    const int lm = (1 << a.levels) - 1;
    auto off_lattice = [lm](int t) {
      const int z = t / C::S2;
      const int r = t - z * C::S2;
      const int y = r / C::S;
      return ((r - y * C::S) | y | z) & lm;
    };
    int det = 0;
    if (k0 >= 0) {
      sm.tile[k0] = v0;
      det |= off_lattice(k0);
    }
    for (int k = tid + C::NT; k < (int)nnz; k += C::NT) {
      const int t = idx[k];
      sm.tile[t] = vals[k];
      det |= off_lattice(t);
    }
    if (__ballot(det != 0) != 0ull && lane == 0) sm.misc[MISC_SAMPLES_IN] = 0u;
  }
  __syncthreads();
}

// ---------------------------------------------------------------------------
// S7 (with THR also S6): compact the thresholded tile in LDS into a record
// appended to the output pool.  Returns false when the pool is full (flag
// raised).
// ---------------------------------------------------------------------------
// Room for a record of nnz values (bitmask or index list) in the output pool
// and its table entry; thread 0 reserves, every thread gets the base (16-byte
// units) in sm.misc[1], or false when the pool is full.
template <class C, class SM>
__device__ __forceinline__ bool reserve_record(const PatchArgs& a, int q, int f, uint32_t nnz, bool ismask,
                                               uint32_t rb16, SM& sm) {
  if (threadIdx.x == 0) {
    const unsigned long long base = atomicAdd(&a.ctrl->top16[a.epoch % 3u], (unsigned long long)rb16);
    const bool ok = base + rb16 <= a.cap16;
    if (!ok) {
      atomicOr(&a.ctrl->abort, ABORT_OVERFLOW);
      atomicMin(&a.ctrl->abort_epoch, a.epoch);
    } else {
      const size_t e = 2 * ((size_t)q * C::M + f);
      a.table_out[e] = (uint32_t)base;
      a.table_out[e + 1] = nnz | (ismask ? MASK_BIT : 0u);
    }
    sm.misc[0] = ok ? 1u : 0u;
    sm.misc[1] = (uint32_t)base;
  }
  __syncthreads();
  return sm.misc[0] != 0u;
}

// S7 for a tile that keeps coarse samples only (L >= 2): the kept nodes lie on
// the lattice of nodes whose three indices are multiples of 2^L, at most NT
// of them, so one pass over that lattice in ascending flat order gives the
// index-list record the general compaction below writes, byte for byte.
template <class C, class SM>
__device__ bool compact_samples(const PatchArgs& a, int q, int f, SM& sm) {
  constexpr int NLMAX = (C::S - 1) / 4 + 1;   // lattice nodes per dimension at L = 2
  static_assert(NLMAX * NLMAX * NLMAX <= C::NT, "one lattice node per thread");
  static_assert(2 * NLMAX * NLMAX * NLMAX < 8 * C::W, "a samples-only record is an index list");
  const int tid = threadIdx.x;
  const int lane = lane_id();
  const int wave = wave_id();
  const int L = a.levels;
  const int nl = ((C::S - 1) >> L) + 1;
  int t = 0;
  float v = 0.f;
  if (tid < nl * nl * nl) {
    const int k = tid / (nl * nl);
    const int r = tid - k * nl * nl;
    const int j = r / nl;
    const int i = r - j * nl;
    t = (i << L) + C::S * (j << L) + C::S2 * (k << L);
    v = sm.tile[t];
  }
  const unsigned long long bits = __ballot(v != 0.f);
  if (lane == 0) sm.wsum[wave] = (uint32_t)__popcll(bits);
  __syncthreads();
  uint32_t off = 0, nnz = 0;
  for (int w = 0; w < C::NW; ++w) {
    const uint32_t c = sm.wsum[w];
    off += (w < wave) ? c : 0u;
    nnz += c;
  }
  const uint32_t vb = (4u * nnz + 7u) & ~7u;
  const uint32_t mb = 2u * nnz;
  const uint32_t rb16 = (vb + mb + 15u) / 16u;
  if (!reserve_record<C>(a, q, f, nnz, false, rb16, sm)) return false;
  uint8_t* rec = a.pool_out + 16ull * sm.misc[1];
  float* vals = reinterpret_cast<float*>(rec);
  uint16_t* idx = reinterpret_cast<uint16_t*>(rec + vb);
  if (v != 0.f) {
    const uint32_t k = off + mbcnt64(bits);
    vals[k] = v;
    idx[k] = (uint16_t)t;
  }
  if (tid == 0 && (nnz & 1u)) vals[nnz] = 0.f;
  const uint32_t tail0 = (vb + mb) / 2u, tail1 = rb16 * 8u;
  uint16_t* h = reinterpret_cast<uint16_t*>(rec);
  if (tid < (int)(tail1 - tail0)) h[tail0 + tid] = 0;
  return true;
}

// SAMPLES: the step path, where forward3_threshold has left the samples-only
// flag in sm.misc[MISC_SAMPLES_OUT].
template <class C, bool THR, bool SAMPLES = false, class SM>
__device__ bool compact_field(const PatchArgs& a, int q, int f, SM& sm) {
  const int tid = threadIdx.x;
  const int lane = lane_id();
  const int wave = wave_id();
  const int L = a.levels;
  const float eps = (float)a.eps;
  if constexpr (SAMPLES) {
    if (L >= 2 && __builtin_amdgcn_readfirstlane((int)sm.misc[MISC_SAMPLES_OUT]) != 0)
      return compact_samples<C>(a, q, f, sm);
  }
  P3_START();
  // counts: one ballot per 64-node chunk; wave w owns the chunks
  // c = w + NW k, keeps bit k of `nonempty` for those with a kept
  // coefficient (a wave-uniform mask, held across the barriers) and the
  // count of chunk k in lane k, stored once per wave after the loop
  static_assert((C::W + C::NW - 1) / C::NW <= 64, "one bit per owned chunk");
  unsigned long long nonempty = 0ull;
  int mycnt = 0;   // lane k: kept count of the wave's chunk wave + NW k
  constexpr int U = 4;   // chunks per wave and iteration (independent LDS reads in flight)
  for (int c0 = wave; c0 < C::W; c0 += U * C::NW) {
    float v[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      // clamped address, so that the reads are unconditional and overlap
      const int t = 64 * (c0 + u * C::NW) + lane;
      const float r = sm.tile[t < C::S3 ? t : C::S3 - 1];
      v[u] = t < C::S3 ? r : 0.f;
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int c = c0 + u * C::NW;
      if constexpr (THR) {
        // S6 here (coefficients given directly): zero a dropped detail in the
        // tile, the inverse for the export needs it zero
        const int t = 64 * c + lane;
        if (t < C::S3) {
          const int z = t / C::S2;
          const int r = t - z * C::S2;
          const int y = r / C::S;
          const int x = r - y * C::S;
          const int rx = dim_rank(x, L), ry = dim_rank(y, L), rz = dim_rank(z, L);
          if (rx >= 0 || ry >= 0 || rz >= 0) {   // a detail (pure samples are never zeroed)
            const int ax = rx < 0 ? 0 : rx, ay = ry < 0 ? 0 : ry, az = rz < 0 ? 0 : rz;
            int rk = 0;
            if (a.rule == R_CAPPED) rk = max(ax, max(ay, az));
            else if (a.rule == R_ACCUM) rk = ax + ay + az;
            if (fabsf(v[u]) < ldexpf(eps, rk)) {
              v[u] = 0.f;
              sm.tile[t] = 0.f;
            }
          }
        }
      }
      const unsigned long long bits = __ballot(v[u] != 0.f);
      const int k = (c - wave) / C::NW;
      if (bits != 0ull) nonempty |= 1ull << k;
      mycnt = (lane == k) ? __popcll(bits) : mycnt;
    }
  }
  {
    const int c = wave + C::NW * lane;
    if (c < C::W) sm.pre[c] = (uint32_t)mycnt;
  }
  __syncthreads();
  P3_MARK(10);
  const uint32_t nnz = scan_counts<C>(sm.pre, C::W, sm);
  P3_MARK(11);
  const bool ismask = !(2u * nnz < 8u * (uint32_t)C::W);
  const uint32_t vb = (4u * nnz + 7u) & ~7u;
  const uint32_t mb = ismask ? 8u * (uint32_t)C::W : 2u * nnz;
  const uint32_t rb16 = (vb + mb + 15u) / 16u;
  const bool ok = reserve_record<C>(a, q, f, nnz, ismask, rb16, sm);
  P3_MARK(12);
  if (!ok) return false;
  uint8_t* rec = a.pool_out + 16ull * sm.misc[1];
  float* vals = reinterpret_cast<float*>(rec);
  uint16_t* idx = reinterpret_cast<uint16_t*>(rec + vb);
  unsigned long long* words = reinterpret_cast<unsigned long long*>(rec + vb);
  if (ismask) {
    // bitmask record: every chunk's word is written, empty or not
    for (int c0 = wave; c0 < C::W; c0 += U * C::NW) {
      float v[U];
      uint32_t pre[U];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int c = c0 + u * C::NW;
        const int t = 64 * c + lane;
        const float r = sm.tile[t < C::S3 ? t : C::S3 - 1];
        const uint32_t p = sm.pre[c < C::W ? c : C::W - 1];
        v[u] = t < C::S3 ? r : 0.f;
        pre[u] = c < C::W ? p : 0u;
      }
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int c = c0 + u * C::NW;
        const unsigned long long bits = __ballot(v[u] != 0.f);
        if (v[u] != 0.f) vals[pre[u] + mbcnt64(bits)] = v[u];
        if (lane == 0 && c < C::W) words[c] = bits;
      }
    }
  } else {
    // index list: only the wave's chunks with a kept coefficient
    {
      unsigned long long m = nonempty;
      while (m != 0ull) {
        const int c = wave + C::NW * __builtin_ctzll(m);
        m &= m - 1ull;
        const int t = 64 * c + lane;
        const float v = t < C::S3 ? sm.tile[t] : 0.f;
        const unsigned long long bits = __ballot(v != 0.f);
        if (v != 0.f) {
          const uint32_t k = sm.pre[c] + mbcnt64(bits);
          vals[k] = v;
          idx[k] = (uint16_t)t;
        }
      }
    }
  }
  // zero padding: after the values, and from the end of the indices or
  // words to the end of the record
  if (tid == 0 && (nnz & 1u)) vals[nnz] = 0.f;
  const uint32_t tail0 = (vb + mb) / 2u, tail1 = rb16 * 8u;
  uint16_t* h = reinterpret_cast<uint16_t*>(rec);
  if (tid < (int)(tail1 - tail0)) h[tail0 + tid] = 0;
  P3_MARK(13);
  return true;
}

// ---------------------------------------------------------------------------
// S9: FP64 trapezoid total of the reconstructed tile from the coefficient tile
// in LDS.  By the conservation identity of the lifting (equation
// "conservation", once per dimension), the trapezoid mass of the
// reconstruction is 8^L times the trapezoid mass of the coarse samples (the
// nodes whose three indices are multiples of 2^L), whatever the details.
// With CHECK a non-finite total raises the abort flag: the forward lifting
// carries every element of a line into the line's coarse samples, so a
// non-finite value anywhere makes a sample, and the total, non-finite.
// ---------------------------------------------------------------------------
template <class C, bool CHECK, class SM>
__device__ void total_field(const PatchArgs& a, int q, int f, SM& sm) {
  const int tid = threadIdx.x;
  const int L = a.levels;
  const int sc = ((C::S - 1) >> L) + 1;   // coarse samples per dimension
  double part = 0.0;
  for (int n = tid; n < sc * sc * sc; n += C::NT) {
    const int k = n / (sc * sc);
    const int r = n - k * sc * sc;
    const int j = r / sc;
    const int i = r - j * sc;
    const int nb = (i == 0 || i == sc - 1) + (j == 0 || j == sc - 1) + (k == 0 || k == sc - 1);
    part += ldexp((double)sm.tile[(i << L) + C::S * (j << L) + C::S2 * (k << L)], 3 * L - nb);
  }
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) part += __shfl_down(part, d, 64);
  if (lane_id() == 0) sm.red[wave_id()] = part;
  __syncthreads();
  if (tid == 0) {
    double s = 0.0;
    for (int w = 0; w < C::NW; ++w) s += sm.red[w];
    a.partials_out[(size_t)q * C::M + f] = s;
    if (CHECK && !(fabs(s) <= 0x1.fffffffffffffp+1023)) {
      atomicOr(&a.ctrl->abort, ABORT_NONFINITE);
      atomicMin(&a.ctrl->abort_epoch, a.epoch);
    }
  }
}

// ---------------------------------------------------------------------------
// S8: export of population f's planes and line for the neighbours
// ---------------------------------------------------------------------------
template <class C, class SM>
__device__ void export_field(const PatchArgs& a, int q, int f, SM& sm) {
  if (f == 0) return;
  const int tid = threadIdx.x;
  float* h = static_cast<float*>(a.halo_out) + (size_t)q * C::HALO;
  int cc[3];
#pragma unroll
  for (int d = 0; d < 3; ++d) cc[d] = 0;
  // population f's velocity (f is wave-uniform; a small constant table walk)
#pragma unroll
  for (int i = 1; i < C::M; ++i)
    if (i == f) {
      cc[0] = D3Q19L::C[i][0];
      cc[1] = D3Q19L::C[i][1];
      cc[2] = D3Q19L::C[i][2];
    }
  int slots[3] = {0, 0, 0};
#pragma unroll
  for (int i = 1; i < C::M; ++i)
    if (i == f) {
      slots[0] = D3Q19L::slot(i, 0);
      slots[1] = D3Q19L::slot(i, 1);
      slots[2] = D3Q19L::slot(i, 2);
    }
#pragma unroll
  for (int ax = 0; ax < 3; ++ax) {
    if (cc[ax] == 0) continue;
    const int k = cc[ax] > 0 ? C::P - 1 : 1;
    // strides of the plane's own axis and of its (u, v) axes in increasing order
    const int s_ax = ax == 0 ? 1 : (ax == 1 ? C::S : C::S2);
    const int s_u = ax == 0 ? C::S : 1;
    const int s_v = ax == 2 ? C::S : C::S2;
    float* dst = h + (size_t)(2 * ax + (cc[ax] > 0 ? 1 : 0)) * C::FACE + (size_t)slots[ax] * C::S2;
    for (int i = tid; i < C::S2; i += C::NT) {
      const int v = i / C::S;
      const int u = i - v * C::S;
      dst[i] = sm.tile[k * s_ax + u * s_u + v * s_v];
    }
  }
  const int nz = (cc[0] != 0) + (cc[1] != 0) + (cc[2] != 0);
  if (nz == 2 && tid < C::S) {
    // axis pair (x,y), (x,z) or (y,z) with non-zero components, and the third axis
    const int pr = cc[2] == 0 ? 0 : (cc[1] == 0 ? 1 : 2);
    const int ca = pr == 2 ? cc[1] : cc[0];
    const int cb = pr == 0 ? cc[1] : cc[2];
    const int sa = pr == 2 ? C::S : 1;
    const int sb = pr == 0 ? C::S : C::S2;
    const int sw = pr == 0 ? C::S2 : (pr == 1 ? C::S : 1);
    const int e = 4 * pr + (ca > 0 ? 1 : 0) + 2 * (cb > 0 ? 1 : 0);
    const int ka = ca > 0 ? C::P - 1 : 1;
    const int kb = cb > 0 ? C::P - 1 : 1;
    h[6 * (size_t)C::FACE + (size_t)e * C::S + tid] = sm.tile[ka * sa + kb * sb + tid * sw];
  }
}

// Patch coordinates of q and of its neighbour at offset (ox, oy, oz), periodic.
__device__ __forceinline__ int neighbour(int px, int py, int pz, int ox, int oy, int oz, int npx) {
  int x = px + ox, y = py + oy, z = pz + oz;
  x += x < 0 ? npx : (x >= npx ? -npx : 0);
  y += y < 0 ? npx : (y >= npx ? -npx : 0);
  z += z < 0 ? npx : (z >= npx ? -npx : 0);
  return x + npx * (y + npx * z);
}

// S3 + streaming: f^in_f(n) = f_f(n - c_f) into scratch.  Nodes whose source
// lies in the tile copy it from LDS; the others (the planes n_a = 0 or S - 1
// of the axes along which c_f points) read it from the neighbours' halo,
// one independent load per node.
// Ghost node i (< S^2) of population f on the receiving plane of axis ax
// (c_f[ax] != 0): its value from the neighbour's halo into val; returns its
// index in the patch, or -1 when the node is taken by the plane of another
// axis (an edge line).
template <class C>
__device__ __forceinline__ int ghost_at(const float* halo, int px, int py, int pz, int npx, const int* cf,
                                        const int* sl, int ax, int i, float& val) {
  // receiving plane n_ax = 0 (c > 0) or S - 1 (c < 0); (u, v) over the
  // other two axes b1 < b2
  const int b1 = ax == 0 ? 1 : 0;
  const int b2 = ax == 2 ? 1 : 2;
  const int c1 = b1 == 0 ? cf[0] : cf[1];
  const int c2 = b2 == 1 ? cf[1] : cf[2];
  const int na = cf[ax] > 0 ? 0 : C::S - 1;
  const int o = cf[ax] > 0 ? -1 : 1;   // neighbour offset along ax
  const int s_ax = ax == 0 ? 1 : (ax == 1 ? C::S : C::S2);
  const int s_1 = b1 == 0 ? 1 : C::S;
  const int s_2 = b2 == 1 ? C::S : C::S2;
  const int v = i / C::S;
  const int u = i - v * C::S;
  const int m1 = u - c1, m2 = v - c2;
  const int o1 = m1 < 0 ? -1 : (m1 >= C::S ? 1 : 0);
  const int o2 = m2 < 0 ? -1 : (m2 >= C::S ? 1 : 0);
  if (o1 == 0 && o2 == 0) {
    // a face of the neighbour along ax
    const int qn = neighbour(px, py, pz, ax == 0 ? o : 0, ax == 1 ? o : 0, ax == 2 ? o : 0, npx);
    val = halo[(size_t)qn * C::HALO + (size_t)(2 * ax + (cf[ax] > 0 ? 1 : 0)) * C::FACE +
               (size_t)(ax == 0 ? sl[0] : (ax == 1 ? sl[1] : sl[2])) * C::S2 + m1 + C::S * m2];
  } else {
    // off the tile along ax and one more axis b: an edge line, taken by
    // the plane of the smaller of the two axes
    const int b = o1 != 0 ? b1 : b2;
    if (b < ax) return -1;
    const int ob = o1 != 0 ? o1 : o2;
    const int oxx = (ax == 0 ? o : 0) + (b == 0 ? ob : 0);
    const int oyy = (ax == 1 ? o : 0) + (b == 1 ? ob : 0);
    const int ozz = (ax == 2 ? o : 0) + (b == 2 ? ob : 0);
    const int qn = neighbour(px, py, pz, oxx, oyy, ozz, npx);
    // pair (x,y), (x,z) or (y,z) and the coordinate along the third axis
    const int lo = ax < b ? ax : b, hi = ax < b ? b : ax;
    const int pr = (lo == 0 && hi == 1) ? 0 : (lo == 0 ? 1 : 2);
    const int ca = lo == 0 ? cf[0] : cf[1];
    const int cb = hi == 1 ? cf[1] : cf[2];
    const int w = o1 != 0 ? m2 : m1;   // the in-range coordinate
    const int e = 4 * pr + (ca > 0 ? 1 : 0) + 2 * (cb > 0 ? 1 : 0);
    val = halo[(size_t)qn * C::HALO + 6 * (size_t)C::FACE + (size_t)e * C::S + w];
  }
  return na * s_ax + u * s_1 + v * s_2;
}

template <class C, class SM>
__device__ void stream_field(const PatchArgs& a, int q, int f, float* scr, SM& sm) {
  int cf[3] = {0, 0, 0}, sl[3] = {0, 0, 0};
#pragma unroll
  for (int i = 1; i < C::M; ++i)
    if (i == f) {
      cf[0] = D3Q19L::C[i][0];
      cf[1] = D3Q19L::C[i][1];
      cf[2] = D3Q19L::C[i][2];
      sl[0] = D3Q19L::slot(i, 0);
      sl[1] = D3Q19L::slot(i, 1);
      sl[2] = D3Q19L::slot(i, 2);
    }
  const int shift = cf[0] + C::S * cf[1] + C::S2 * cf[2];
  float* dst = scr + (size_t)f * C::SF;
  // the ghost values are loaded before the in-tile pass, under which their
  // latency passes, and stored after it (the two passes write disjoint nodes)
  const int npx = a.npx;
  const int pz = q / (npx * npx), py = (q / npx) % npx, px = q % npx;
  const float* halo = static_cast<const float*>(a.halo_in);
  constexpr int GI = (C::S2 + C::NT - 1) / C::NT;
  float gv[3][GI];
  int gd[3][GI];
#pragma unroll
  for (int ax = 0; ax < 3; ++ax) {
#pragma unroll
    for (int j = 0; j < GI; ++j) {
      const int i = threadIdx.x + j * C::NT;
      gv[ax][j] = 0.f;
      gd[ax][j] = -1;
      if (cf[ax] != 0 && i < C::S2) gd[ax][j] = ghost_at<C>(halo, px, py, pz, npx, cf, sl, ax, i, gv[ax][j]);
    }
  }
  // Each thread keeps one x and steps through the x-rows (y, z) RPP at a time
  // (RPP * S of the threads take part), so that y and z advance by additions.
  constexpr int RPP = C::NT / C::S;
  constexpr int U = 4;   // rows per thread and iteration (independent LDS reads in flight)
  if (threadIdx.x < RPP * C::S) {
    const int x = threadIdx.x % C::S;
    const int r0 = threadIdx.x / C::S;
    const bool inx = (unsigned)(x - cf[0]) < (unsigned)C::S;
    int y = r0 % C::S, z = r0 / C::S;   // row r = y + S z, starting at r0
    for (int r = r0; r < C::S2; r += U * RPP) {
      float val[U];
      bool in[U];
      int t[U];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        t[u] = x + C::S * (y + C::S * z);
        in[u] = r + u * RPP < C::S2 && inx && (unsigned)(y - cf[1]) < (unsigned)C::S &&
                (unsigned)(z - cf[2]) < (unsigned)C::S;
        // clamped address: the read is unconditional, the store is not
        const int src = t[u] - shift;
        val[u] = sm.tile[src < 0 ? 0 : (src >= C::S3 ? C::S3 - 1 : src)];
        // advance by RPP rows: RPP / S planes and RPP % S rows, at most one more wrap
        y += RPP % C::S;
        z += RPP / C::S;
        if (y >= C::S) {
          y -= C::S;
          ++z;
        }
      }
#pragma unroll
      for (int u = 0; u < U; ++u)
        if (in[u]) dst[t[u]] = val[u];
    }
  }
#pragma unroll
  for (int ax = 0; ax < 3; ++ax) {
#pragma unroll
    for (int j = 0; j < GI; ++j)
      if (gd[ax][j] >= 0) dst[gd[ax][j]] = gv[ax][j];
  }
}

// S4: BGK collision of every node of the patch in scratch (in place).
template <class C>
__device__ __forceinline__ void collide_node(float* fi, float om) {
  float rho = 0.f, jx = 0.f, jy = 0.f, jz = 0.f;
#pragma unroll
  for (int i = 0; i < 19; ++i) {
    rho += fi[i];
    if (D3Q19L::C[i][0]) jx += D3Q19L::C[i][0] > 0 ? fi[i] : -fi[i];
    if (D3Q19L::C[i][1]) jy += D3Q19L::C[i][1] > 0 ? fi[i] : -fi[i];
    if (D3Q19L::C[i][2]) jz += D3Q19L::C[i][2] > 0 ? fi[i] : -fi[i];
  }
  const float ux = jx / rho, uy = jy / rho, uz = jz / rho;
  const float usq = ux * ux + uy * uy + uz * uz;
#pragma unroll
  for (int i = 0; i < 19; ++i) {
    const float w = i == 0 ? (1.f / 3.f) : (i < 7 ? (1.f / 18.f) : (1.f / 36.f));
    const float cu = (float)D3Q19L::C[i][0] * ux + (float)D3Q19L::C[i][1] * uy + (float)D3Q19L::C[i][2] * uz;
    const float feq = w * rho * (1.f + 3.f * cu + 4.5f * cu * cu - 1.5f * usq);
    fi[i] = fi[i] - om * (fi[i] - feq);
  }
}

// Buffer resource over the workgroup's scratch slice (19 fields of SF
// floats): loads and stores address it by a per-thread byte offset and a
// per-population offset held in a scalar register, so that the 19 streams of
// the collision need no per-population 64-bit address in vector registers.
// Accesses outside the slice read 0 and write nothing.
template <class C>
__device__ __forceinline__ __amdgpu_buffer_rsrc_t scratch_rsrc(float* scr) {
  return __builtin_amdgcn_make_buffer_rsrc(scr, 0, (int)(sizeof(float) * C::M * C::SF), BUF_WORD3);
}

typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

template <class C>
__device__ void collide(const PatchArgs& a, float* scr) {
  const float om = (float)a.omega;
  const __amdgpu_buffer_rsrc_t rs = scratch_rsrc<C>(scr);
  constexpr int FB = (int)sizeof(float) * C::SF;   // bytes per population
  // Four consecutive nodes per thread and iteration: 19 16-byte loads in
  // flight per lane, then the four collisions, then 19 16-byte stores.
  for (int i4 = threadIdx.x; i4 < C::SF / 4; i4 += C::NT) {
    u32x4 q[19];
#pragma unroll
    for (int k = 0; k < 19; ++k) q[k] = __builtin_amdgcn_raw_buffer_load_b128(rs, 16 * i4, k * FB, 0);
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      float f[19];
#pragma unroll
      for (int k = 0; k < 19; ++k) f[k] = __uint_as_float(q[k][e]);
      collide_node<C>(f, om);
#pragma unroll
      for (int k = 0; k < 19; ++k) q[k][e] = __float_as_uint(f[k]);
    }
#pragma unroll
    for (int k = 0; k < 19; ++k) __builtin_amdgcn_raw_buffer_store_b128(q[k], rs, 16 * i4, k * FB, 0);
  }
}

// A field of scratch into the LDS tile, 16-byte loads, three in flight per thread.
template <class C, class SM>
__device__ void load_field(const float* src, SM& sm) {
  constexpr int U = 3;
  const float4* s4 = reinterpret_cast<const float4*>(src);
  for (int i0 = threadIdx.x; i0 < C::SF / 4; i0 += U * C::NT) {
    float4 v[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int i4 = i0 + u * C::NT;
      v[u] = i4 < C::SF / 4 ? s4[i4] : make_float4(0.f, 0.f, 0.f, 0.f);
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int t = 4 * (i0 + u * C::NT);
      if (t + 0 < C::S3) sm.tile[t + 0] = v[u].x;
      if (t + 1 < C::S3) sm.tile[t + 1] = v[u].y;
      if (t + 2 < C::S3) sm.tile[t + 2] = v[u].z;
      if (t + 3 < C::S3) sm.tile[t + 3] = v[u].w;
    }
  }
  __syncthreads();
}

// C: from a transformed-or-not tile in LDS to the record, totals and export.
template <class C, bool THR, class SM>
__device__ void finish_field(const PatchArgs& a, int q, int f, SM& sm) {
  compact_field<C, THR>(a, q, f, sm);
  total_field<C, true>(a, q, f, sm);   // its barrier also ends the record stores' tile reads
  inverse3<C>(sm.tile, a.levels);
  export_field<C>(a, q, f, sm);
  __syncthreads();
}

template <class C, class SM>
__device__ void step_patch(const PatchArgs& a, int q, float* scr, SM& sm) {
  const int L = a.levels;
  P3_START();
  for (int f = 0; f < C::M; ++f) {
    expand_field<C>(a, q, f, sm);
    P3_MARK(0);
    if (L >= 2 && __builtin_amdgcn_readfirstlane((int)sm.misc[MISC_SAMPLES_IN]) != 0) inverse3_samples<C>(sm.tile, L);
    else inverse3<C>(sm.tile, L);
    P3_MARK(1);
    stream_field<C>(a, q, f, scr, sm);
    __syncthreads();
    P3_MARK(2);
  }
  collide<C>(a, scr);
  __syncthreads();
  P3_MARK(3);
  for (int f = 0; f < C::M; ++f) {
    load_field<C>(scr + (size_t)f * C::SF, sm);
    P3_MARK(4);
    forward3_threshold<C>(a, sm.tile, &sm.misc[MISC_SAMPLES_OUT]);
    P3_MARK(5);
    compact_field<C, false, true>(a, q, f, sm);
    P3_MARK(6);
    total_field<C, true>(a, q, f, sm);
    P3_MARK(7);
    if (L >= 2 && __builtin_amdgcn_readfirstlane((int)sm.misc[MISC_SAMPLES_OUT]) != 0) inverse3_samples<C>(sm.tile, L);
    else inverse3<C>(sm.tile, L);
    P3_MARK(8);
    export_field<C>(a, q, f, sm);
    __syncthreads();
    P3_MARK(9);
  }
}

// One step of every patch: persistent workgroups, each with its own scratch
// slice (blockIdx.x), take patches from the work queue of this epoch.
template <int P>
__global__ __launch_bounds__(1024) void d3q19_step_kernel(PatchArgs a) {
  using C = Cfg3<P>;
  __shared__ Smem3<C> sm;
  if (step_stops(a, blockIdx.x == 0, sm)) return;
  float* scr = a.scratch + (size_t)blockIdx.x * C::M * C::SF;
  for (;;) {
    if (threadIdx.x == 0) sm.misc[3] = atomicAdd(&a.ctrl->queue[a.epoch % 3u], 1u);
    __syncthreads();
    const int q = __builtin_amdgcn_readfirstlane((int)sm.misc[3]);   // uniform: scalar addressing
    __syncthreads();
    if (q >= a.npatch) break;
    step_patch<C>(patch_args_reread(), q, scr, sm);
  }
}

// Auxiliary modes, one workgroup per patch.
template <int P>
__global__ __launch_bounds__(1024) void d3q19_aux_kernel(PatchArgs a) {
  using C = Cfg3<P>;
  __shared__ Smem3<C> sm;
  const int q = blockIdx.x;
  const int n = a.n;
  const int npx = a.npx;
  const int pz = q / (npx * npx), py = (q / npx) % npx, px = q % npx;
  for (int f = 0; f < C::M; ++f) {
    if (a.mode == AUX_DECOMP && a.field_only >= 0 && f != a.field_only) continue;
    if (a.mode == AUX_INIT) {
      const float* src = static_cast<const float*>(a.dense_in) + (size_t)f * n * n * n;
      for (int t = threadIdx.x; t < C::S3; t += C::NT) {
        const int z = t / C::S2;
        const int r = t - z * C::S2;
        const int y = r / C::S;
        const int x = r - y * C::S;
        const int gx = (px * C::P + x) % n, gy = (py * C::P + y) % n, gz = (pz * C::P + z) % n;
        sm.tile[t] = src[((size_t)gz * n + gy) * n + gx];
      }
      __syncthreads();
      forward3_threshold<C>(a, sm.tile, &sm.misc[MISC_SAMPLES_OUT]);
      finish_field<C, false>(a, q, f, sm);
    } else if (a.mode == AUX_COEF) {
      const float* src = static_cast<const float*>(a.coef_in) + ((size_t)q * C::M + f) * C::S3;
      for (int t = threadIdx.x; t < C::S3; t += C::NT) sm.tile[t] = src[t];
      __syncthreads();
      finish_field<C, true>(a, q, f, sm);
    } else {
      expand_field<C>(a, q, f, sm);
      if (a.mode == AUX_RESTORE) total_field<C, false>(a, q, f, sm);
      inverse3<C>(sm.tile, a.levels);
      if (a.mode == AUX_RESTORE) {
        export_field<C>(a, q, f, sm);
      } else {
        float* dst = static_cast<float*>(a.dense_out) + (a.field_only >= 0 ? 0 : (size_t)f * n * n * n);
        for (int t = threadIdx.x; t < C::P * C::P * C::P; t += C::NT) {
          const int z = t / (C::P * C::P);
          const int r = t - z * C::P * C::P;
          const int y = r / C::P;
          const int x = r - y * C::P;
          dst[((size_t)(pz * C::P + z) * n + (py * C::P + y)) * n + (px * C::P + x)] =
              sm.tile[x + C::S * y + C::S2 * z];
        }
      }
      __syncthreads();
    }
  }
}

// Uncompressed D3Q19 BGK step on a periodic [19][n][n][n] grid.
__global__ void d3q19_ref_kernel(const float* __restrict__ in, float* __restrict__ out, int n, float om) {
  const size_t nn = (size_t)n * n * n;
  const size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= nn) return;
  const int x = (int)(t % n);
  const int y = (int)((t / n) % n);
  const int z = (int)(t / ((size_t)n * n));
  float fi[19];
#pragma unroll
  for (int i = 0; i < 19; ++i) {
    const int sx = (x - D3Q19L::C[i][0] + n) % n;
    const int sy = (y - D3Q19L::C[i][1] + n) % n;
    const int sz = (z - D3Q19L::C[i][2] + n) % n;
    fi[i] = in[(size_t)i * nn + ((size_t)sz * n + sy) * n + sx];
  }
  float rho = 0.f, jx = 0.f, jy = 0.f, jz = 0.f;
#pragma unroll
  for (int i = 0; i < 19; ++i) {
    rho += fi[i];
    if (D3Q19L::C[i][0]) jx += D3Q19L::C[i][0] > 0 ? fi[i] : -fi[i];
    if (D3Q19L::C[i][1]) jy += D3Q19L::C[i][1] > 0 ? fi[i] : -fi[i];
    if (D3Q19L::C[i][2]) jz += D3Q19L::C[i][2] > 0 ? fi[i] : -fi[i];
  }
  const float ux = jx / rho, uy = jy / rho, uz = jz / rho;
  const float usq = ux * ux + uy * uy + uz * uz;
#pragma unroll
  for (int i = 0; i < 19; ++i) {
    const float w = i == 0 ? (1.f / 3.f) : (i < 7 ? (1.f / 18.f) : (1.f / 36.f));
    const float cu = (float)D3Q19L::C[i][0] * ux + (float)D3Q19L::C[i][1] * uy + (float)D3Q19L::C[i][2] * uz;
    const float feq = w * rho * (1.f + 3.f * cu + 4.5f * cu * cu - 1.5f * usq);
    out[(size_t)i * nn + t] = fi[i] - om * (fi[i] - feq);
  }
}

// Equilibrium populations [19][n^3] from rho, ux, uy, uz [n^3].
__global__ void d3q19_equilibrium_kernel(const float* rho, const float* ux, const float* uy, const float* uz,
                                         float* f, size_t nn) {
  const size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= nn) return;
  const float r = rho[t], u = ux[t], v = uy[t], w3 = uz[t];
  const float usq = u * u + v * v + w3 * w3;
#pragma unroll
  for (int i = 0; i < 19; ++i) {
    const float w = i == 0 ? (1.f / 3.f) : (i < 7 ? (1.f / 18.f) : (1.f / 36.f));
    const float cu = (float)D3Q19L::C[i][0] * u + (float)D3Q19L::C[i][1] * v + (float)D3Q19L::C[i][2] * w3;
    f[(size_t)i * nn + t] = w * r * (1.f + 3.f * cu + 4.5f * cu * cu - 1.5f * usq);
  }
}

hipError_t launch_reference_step3(const void* in, void* out, int n, double omega, hipStream_t s) {
  const size_t nn = (size_t)n * n * n;
  hipLaunchKernelGGL(d3q19_ref_kernel, dim3((unsigned)((nn + 255) / 256)), dim3(256), 0, s,
                     static_cast<const float*>(in), static_cast<float*>(out), n, (float)omega);
  return hipGetLastError();
}

hipError_t launch_equilibrium3(const void* rho, const void* ux, const void* uy, const void* uz, void* f, int n,
                               hipStream_t s) {
  const size_t nn = (size_t)n * n * n;
  hipLaunchKernelGGL(d3q19_equilibrium_kernel, dim3((unsigned)((nn + 255) / 256)), dim3(256), 0, s,
                     static_cast<const float*>(rho), static_cast<const float*>(ux), static_cast<const float*>(uy),
                     static_cast<const float*>(uz), static_cast<float*>(f), nn);
  return hipGetLastError();
}

template <int P>
static void d3q19_case(int op, const PatchArgs* a, int grid, hipStream_t s, hipError_t* err, size_t* out) {
  using C = Cfg3<P>;
  switch (op) {
    case 0:   // step (plain launch and persistent launch are the same kernel)
    case 3:
      hipLaunchKernelGGL(d3q19_step_kernel<P>, dim3((unsigned)grid), dim3(C::NT), 0, s, *a);
      *err = hipGetLastError();
      break;
    case 1:
      hipLaunchKernelGGL(d3q19_aux_kernel<P>, dim3((unsigned)grid), dim3(C::NT), 0, s, *a);
      *err = hipGetLastError();
      break;
    case 2:
      *out = sizeof(Smem3<C>);
      break;
    case 4:
    case 5:
      *out = reinterpret_cast<size_t>(reinterpret_cast<const void*>(&d3q19_step_kernel<P>));
      break;
    case 6:
      *out = (size_t)C::NT;
      break;
    case 7:   // halo floats per patch
      *out = (size_t)C::HALO;
      break;
    case 8:   // scratch floats per workgroup
      *out = (size_t)C::M * C::SF;
      break;
    default:
      *err = hipErrorInvalidValue;
  }
}

#ifdef LBMZ_PHASE_CLOCK
extern "C" int lbmz_debug_phase3(void* host, size_t bytes) {
  if (bytes > sizeof(lbmz_phase3)) bytes = sizeof(lbmz_phase3);
  return hipMemcpyFromSymbol(host, HIP_SYMBOL(lbmz_phase3), bytes, 0, hipMemcpyDeviceToHost) == hipSuccess ? 0 : -3;
}
#endif

bool dispatch_f32_d3q19(LBMZ_DISPATCH_ARGS) {
  if (k.dtype != 0 || k.scheme != S_LBM3 || k.wavelet != W_BL53 || k.vf != VF_F32) return false;
  switch (k.p) {
    case 16: d3q19_case<16>(op, a, grid, s, err, out); return true;
    case 32: d3q19_case<32>(op, a, grid, s, err, out); return true;
    default: return false;
  }
}

}  // namespace lbmz
