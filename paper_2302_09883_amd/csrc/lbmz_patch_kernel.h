// Fused patch kernels for gfx950: one workgroup owns one patch for the whole
// step and keeps all of its fields in LDS.
//
// Lines of a tile are lifted one per thread in registers.  In every pass,
// wave f (< M) owns field f, lane l its line l (l < P); with the folded
// BL5/3 tiles (shared bordering line P) wave M owns line P of every field,
// lane f for field f.  LDS rows use an odd stride so that row-per-lane and
// column-per-lane accesses are both bank-conflict free.
//
// One step of one patch:
//   S3  ghost values of the neighbours' previous export are loaded first
//       (D2Q9: the tiles are zeroed while those loads are in flight);
//   S1  the patch's records are expanded straight into the column registers
//       (bitmask records) or scattered through LDS (index-list records),
//   S2  inverse transform: columns (y) then rows (x), coarse to fine; for
//       D2Q9 the row pass also applies the x part of pull streaming;
//   S4  stencil (D2Q9: y part of streaming by row offsets + BGK collision;
//       FV: upwind flux sum) of every tile node;
//   S5  forward transform: rows (x), then in one column pass: columns (y),
//   S6  hard threshold (Section 2.2),
//   S7  compaction straight from registers: per-lane counts, one ballot
//       per 64-bit mask word, one bump allocation per patch, coalesced
//       value stores,
//   S9  FP64 totals from the coarse samples,
//   S8  column inverse in the same registers, then (BL5/3) only the values
//       the neighbours read at the next step: the rows' values at nodes 1
//       and P - 1 by their lifting dependency chain, and the full inverse of
//       the two exported rows (Haar: the full row inverse).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

#include "lbmz_internal.h"

namespace lbmz {

constexpr int ilog2c(int v) { return v <= 1 ? 0 : 1 + ilog2c(v / 2); }

struct D2Q9 {
  static constexpr int CX[9] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
  static constexpr int CY[9] = {0, 0, 1, 0, -1, 1, 1, -1, -1};
  // populations entering through each ghost side: W (x = -1), E (x = S),
  // S (y = -1), N (y = S), in numbering order (the slot of a population)
  static constexpr int SIDE_POP[4][3] = {{1, 5, 8}, {3, 6, 7}, {2, 5, 6}, {4, 7, 8}};
};

// LDS layout of the fields of a tile.  D2Q9 populations that pull from row
// y - 1 (c_y = +1) carry one ghost row before row 0, those that pull from
// row y + 1 carry one after row S - 1; the ghost rows are filled by the halo
// gather so that streaming in y becomes a fixed row offset.
template <int SCH, int S, int RS>
struct TileLayout {
  static constexpr int M = (SCH == S_LBM) ? 9 : (SCH == S_EULER ? 4 : 1);
  static constexpr int lo(int f) { return (SCH == S_LBM && D2Q9::CY[f] == 1) ? 1 : 0; }
  static constexpr int hi(int f) { return (SCH == S_LBM && D2Q9::CY[f] == -1) ? 1 : 0; }
  static constexpr int start(int f) {
    int s = 0;
    for (int g = 0; g < f; ++g) s += (S + lo(g) + hi(g)) * RS;
    return s;
  }
  static constexpr int fb(int f) { return start(f) + lo(f) * RS; }   // row 0 of field f
  static constexpr int total() { return start(M); }
};

template <class T, int P_, int WAV, int SCH, bool PERS = false>
struct Cfg {
  static constexpr bool PERSISTENT = PERS;                  // code of the persistent kernel's loop
  static constexpr int P = P_;
  static constexpr bool RIM = (WAV == W_BL53);              // tiles carry the shared line P
  static constexpr int S = RIM ? P + 1 : P;                 // tile nodes per side
  static constexpr int RS = (S & 1) ? S : S + 1;            // LDS row stride (odd)
  static constexpr int M = (SCH == S_LBM) ? 9 : (SCH == S_EULER ? 4 : 1);   // fields
  static constexpr int NC = S * S;                          // coefficients per field
  static constexpr int W = (NC + 63) / 64;                  // mask words per record
  static constexpr int CW = P * P / 64;                     // mask words of the owned block
  static constexpr int RPW = 64 / P;                        // owned rows per mask word
  static constexpr int NSLOT = (SCH == S_LBM) ? 3 : M;      // fields crossing one side
  static constexpr int LO = RIM ? 1 : 0;                    // first line a neighbour needs
  static constexpr int HI = P - 1;                          // last line a neighbour needs
  static constexpr int NT = (SCH == S_LBM) ? 1024 : (SCH == S_EULER ? 512 : 256);   // threads per workgroup
  static constexpr int NWAVES = NT / 64;
  static constexpr int J = ilog2c(P);
  static constexpr int LMAX = RIM ? J - 1 : J;
  static constexpr int NPER = (NC + NT - 1) / NT;           // stencil nodes per thread
  static constexpr int NPASS = M + (RIM ? 1 : 0);          // waves with a line in the passes
  static constexpr int NHT = NT - 64 * NPASS;               // helper threads (no line)
  static constexpr int LPT = (4 * W + NHT - 1) / NHT;       // index-list entries per helper
  using Lay = TileLayout<SCH, S, RS>;
  static constexpr int TILE = Lay::total();
  static_assert(P >= 8 && P <= 64, "patch size");
  static_assert(W <= 128, "two mask words per lane");
  static_assert(NWAVES > NPASS, "one wave per field, one for the shared line, and helpers");
};

// Shared memory of the patch kernels.
// Scratch of the narrow value formats (per-subband maxima and scale
// exponents, record section offsets, mask-word prefix counts).
template <class C>
struct NarrowLds {
  static constexpr int NB = (C::LMAX + 1) * (C::LMAX + 1);   // subbands, index cy * (L + 1) + cx
  float smax[C::M][NB];                  // max |kept detail| per subband, owned lines
  float rmax[C::M][C::LMAX + 1];         // the same for the shared column (x class 0), by y class
  unsigned long long occ[C::M];          // subbands holding a kept detail
  signed char kexp[C::M][NB];            // scale 2^kexp of each subband
  uint32_t hb[C::M];                     // byte offset of the samples in the record
  uint32_t sb[C::M];                     // byte offset of the detail values
  uint16_t wpre[C::M][C::W + 1];         // bitmask records: set bits before each word
  uint32_t e4[C::M];                     // 1: the record's codes are E4M3, 0: binary16
};
struct NoLds {};

template <class C, class T, int VF = VF_F32>
struct Smem {
  T tile[C::TILE];
  T ghost[4 * C::NSLOT * C::S];          // D2Q9: W/E strips (x shift); FV: W/E/S/N strips
  unsigned long long rowbits[C::M];      // bits of the shared row y = P (x < P)
  unsigned long long colbits[C::M];      // bits of the shared column x = P (y < P)
  double tot[C::M];
  double totface[C::M];
  unsigned corner[C::M];
  unsigned core_nnz[C::M];
  uint32_t rel16[C::M];                  // record offset inside the patch's allocation
  uint32_t nnz[C::M];
  uint32_t ismask[C::M];
  uint32_t vb[C::M];
  uint32_t rb[C::M];
  uint32_t te[2 * C::M];                 // offset-table entries of the patch being expanded
  uint32_t samples_only;                 // 1: every record of the patch holds coarse samples only
  unsigned misc[5];                      // pool status, allocation base, stop flag, queue slots
  typename std::conditional<VF == VF_F32, NoLds, NarrowLds<C>>::type nq;
};

// ---------------------------------------------------------------------------
// Small device helpers
// ---------------------------------------------------------------------------

// Word 3 of the buffer descriptors built here (raw, unswizzled, stride 0):
// data format 32-bit (bits 15..18 = 4; a zero format makes every access
// return 0 and write nothing), all other fields 0.  With stride 0 an access
// is in range when its offset is below the descriptor's byte count; outside
// it a load returns 0 and a store writes nothing.
constexpr int BUF_WORD3 = 0x00020000;

__device__ __forceinline__ int lane_id() { return threadIdx.x & 63; }
__device__ __forceinline__ int wave_id() { return __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6)); }

// Work-item id as the patch code of configuration C sees it.  In the
// persistent kernel it is opaque to the optimiser: values derived from it
// are recomputed where they are used instead of being hoisted out of the
// patch loop and held in registers across it.
template <class C>
__device__ __forceinline__ unsigned tid_of() {
  unsigned t = threadIdx.x;
  if constexpr (C::PERSISTENT) asm volatile("" : "+v"(t));
  return t;
}
template <class C>
__device__ __forceinline__ int lane_of() {
  return (int)(tid_of<C>() & 63u);
}
template <class C>
__device__ __forceinline__ int wave_of() {
  return __builtin_amdgcn_readfirstlane((int)(tid_of<C>() >> 6));
}

__device__ __forceinline__ unsigned long long readlane64(unsigned long long v, int lane) {
  const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)v, lane);
  const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(v >> 32), lane);
  return ((unsigned long long)hi << 32) | lo;
}

__device__ __forceinline__ unsigned long long below(int b) {   // bits [0, b), 0 <= b <= 63
  return (1ull << b) - 1ull;
}

__device__ __forceinline__ int wave_incl_scan(int v) {
  const int lane = lane_id();
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    const int u = __shfl_up(v, d, 64);
    if (lane >= d) v += u;
  }
  return v;
}

template <class T> __device__ __forceinline__ T max_finite();
template <> __device__ __forceinline__ float max_finite<float>() { return 3.402823466e+38f; }
template <> __device__ __forceinline__ double max_finite<double>() { return 1.7976931348623157e+308; }

__device__ __forceinline__ float ldexp_t(float v, int e) { return ldexpf(v, e); }
__device__ __forceinline__ double ldexp_t(double v, int e) { return ldexp(v, e); }

// Zero n elements from p, threads `t` of `nt` cooperating: 16-byte stores
// on the aligned body, element stores on the unaligned head and tail.
template <class T>
__device__ __forceinline__ void zero_span(T* p, int n, int t, int nt) {
  constexpr int E = 16 / sizeof(T);
  const int head = (int)(((16u - ((uintptr_t)p & 15u)) & 15u) / sizeof(T));
  const int h = head < n ? head : n;
  const int nv = (n - h) / E;
  if (t < h) p[t] = T(0);
  uint4* body = reinterpret_cast<uint4*>(p + h);
  for (int i = t; i < nv; i += nt) body[i] = make_uint4(0u, 0u, 0u, 0u);
  const int tail0 = h + nv * E;
  if (tail0 + t < n) p[tail0 + t] = T(0);
}

// Row 0 of field f in the tile (f may differ between lanes).
template <class C>
__device__ __forceinline__ int field_base(int f) {
  int r = 0;
#pragma unroll
  for (int g = 0; g < C::M; ++g) r = (f == g) ? C::Lay::fb(g) : r;
  return r;
}

// Per-dimension rank of tile index i for an L-level transform: -1 for a sample
// (i a multiple of 2^L), else L - lev with lev = 1 + ctz(i) the detail level.
__device__ __forceinline__ int dim_rank(int i, int L) {
  if ((i & ((1 << L) - 1)) == 0) return -1;
  return L - 1 - __builtin_ctz((unsigned)i);
}

// Level class of tile index i: 1 + ctz(i) (the detail level it would have),
// capped at LMAX + 1, which also stands for index 0 (a sample at any L).
template <int LMAX>
__device__ __forceinline__ constexpr int level_class(int i) {
  if (i == 0) return LMAX + 1;
  int lev = 1;
  while ((i & 1) == 0 && lev <= LMAX) {
    i >>= 1;
    ++lev;
  }
  return lev;
}

// Threshold of Section 2.2 for a coefficient with ranks (rx, ry); 0 for a
// pure sample, which is never zeroed.  Exact power-of-two scaling of eps.
template <class T>
__device__ __forceinline__ T thr_of(int rx, int ry, T eps, int rule) {
  if (rx < 0 && ry < 0) return T(0);
  const int ax = rx < 0 ? 0 : rx;
  const int ay = ry < 0 ? 0 : ry;
  const int r = (rule == R_CAPPED) ? (ax > ay ? ax : ay) : (rule == R_ACCUM) ? ax + ay : 0;
  return ldexp_t(eps, r);
}

// Tile node (x, y) of record index k: the owned P x P block row by row, then
// (shared border) the column x = P, the row y = P and the corner.
template <class C>
__device__ __forceinline__ void record_node(int k, int& x, int& y) {
  constexpr int PP = C::P * C::P;
  if (k < PP) { y = k / C::P; x = k - y * C::P; }
  else if (k < PP + C::P) { x = C::P; y = k - PP; }
  else if (k < PP + 2 * C::P) { y = C::P; x = k - PP - C::P; }
  else { x = C::P; y = C::P; }
}

// Shared-border bits of a bitmask record, after the CW words of the owned
// block: one bit stream with the column x = P at bits [0, P), the row y = P
// at bits [P, 2P) and the corner at bit 2P, cut into up to three words.
template <class C>
__device__ __forceinline__ void rim_join(unsigned long long col, unsigned long long row, bool corner,
                                         unsigned long long& r0, unsigned long long& r1, unsigned long long& r2) {
  const unsigned long long c = corner ? 1ull : 0ull;
  if constexpr (C::P == 64) {
    r0 = col;
    r1 = row;
    r2 = c;
  } else if constexpr (C::P == 32) {
    r0 = col | (row << 32);
    r1 = c;
    r2 = 0ull;
  } else {
    r0 = col | (row << C::P) | (c << (2 * C::P));
    r1 = 0ull;
    r2 = 0ull;
  }
}

template <class C>
__device__ __forceinline__ void rim_split(unsigned long long r0, unsigned long long r1, unsigned long long r2,
                                          unsigned long long& col, unsigned long long& row, bool& corner) {
  if constexpr (C::P == 64) {
    col = r0;
    row = r1;
    corner = (r2 & 1ull) != 0ull;
  } else if constexpr (C::P == 32) {
    col = r0 & below(32);
    row = r0 >> 32;
    corner = (r1 & 1ull) != 0ull;
  } else {
    col = r0 & below(C::P);
    row = (r0 >> C::P) & below(C::P);
    corner = ((r0 >> (2 * C::P)) & 1ull) != 0ull;
  }
}

// ---------------------------------------------------------------------------
// Lifting levels on a register line v[0 .. S-1] (Section 2.1.2)
// ---------------------------------------------------------------------------

// Folded BL5/3, level LEV on the sub-lattice of stride 2^(LEV-1) of 2^J + 1
// nodes: predict d_k = u_{2k+1} - (u_{2k} + u_{2k+2}) / 2, then update the
// interior samples s_k = (u_{2k} + a_{k-1} d_{k-1}) + a_k d_k with a = 1/2 at
// both ends of the detail range and 1/4 inside; boundary samples stay.
template <class T, int S, int LEV>
__device__ __forceinline__ void bl53_fwd(T* v) {
  constexpr int st = 1 << (LEV - 1);
  constexpr int m = (S - 1) / (2 * st);
#pragma unroll
  for (int k = 0; k < m; ++k)
    v[(2 * k + 1) * st] = v[(2 * k + 1) * st] - (v[2 * k * st] + v[(2 * k + 2) * st]) * T(0.5);
#pragma unroll
  for (int k = 1; k < m; ++k) {
    const T am = (k - 1 == 0) ? T(0.5) : T(0.25);
    const T ap = (k == m - 1) ? T(0.5) : T(0.25);
    v[2 * k * st] = (v[2 * k * st] + am * v[(2 * k - 1) * st]) + ap * v[(2 * k + 1) * st];
  }
}

template <class T, int S, int LEV>
__device__ __forceinline__ void bl53_inv(T* v) {
  constexpr int st = 1 << (LEV - 1);
  constexpr int m = (S - 1) / (2 * st);
#pragma unroll
  for (int k = 1; k < m; ++k) {
    const T am = (k - 1 == 0) ? T(0.5) : T(0.25);
    const T ap = (k == m - 1) ? T(0.5) : T(0.25);
    v[2 * k * st] = (v[2 * k * st] - am * v[(2 * k - 1) * st]) - ap * v[(2 * k + 1) * st];
  }
#pragma unroll
  for (int k = 0; k < m; ++k)
    v[(2 * k + 1) * st] = v[(2 * k + 1) * st] + (v[2 * k * st] + v[(2 * k + 2) * st]) * T(0.5);
}

// The predict half of bl53_inv alone.  When every detail of the line is
// zero, each update of bl53_inv subtracts exact zeros and returns its sample
// unchanged, so the predicts alone give the same bits.
template <class T, int S, int LEV>
__device__ __forceinline__ void bl53_inv_predict(T* v) {
  constexpr int st = 1 << (LEV - 1);
  constexpr int m = (S - 1) / (2 * st);
#pragma unroll
  for (int k = 0; k < m; ++k)
    v[(2 * k + 1) * st] = v[(2 * k + 1) * st] + (v[2 * k * st] + v[(2 * k + 2) * st]) * T(0.5);
}

// Haar lifting on 2^J nodes: d = b - a, s = a + d / 2 (pairwise mean).
template <class T, int S, int LEV>
__device__ __forceinline__ void haar_fwd(T* v) {
  constexpr int st = 1 << (LEV - 1);
  constexpr int m = S / (2 * st);
#pragma unroll
  for (int k = 0; k < m; ++k) {
    const T a = v[2 * k * st];
    const T d = v[(2 * k + 1) * st] - a;
    v[(2 * k + 1) * st] = d;
    v[2 * k * st] = a + d * T(0.5);
  }
}

template <class T, int S, int LEV>
__device__ __forceinline__ void haar_inv(T* v) {
  constexpr int st = 1 << (LEV - 1);
  constexpr int m = S / (2 * st);
#pragma unroll
  for (int k = 0; k < m; ++k) {
    const T d = v[(2 * k + 1) * st];
    const T a = v[2 * k * st] - d * T(0.5);
    v[2 * k * st] = a;
    v[(2 * k + 1) * st] = a + d;
  }
}

template <class T, int S, int WAV, int LEV, int LMAX>
struct Lift {
  static __device__ __forceinline__ void fwd(T* v, int L) {
    if constexpr (LEV <= LMAX) {
      if (LEV <= L) {
        if constexpr (WAV == W_BL53) bl53_fwd<T, S, LEV>(v); else haar_fwd<T, S, LEV>(v);
        Lift<T, S, WAV, LEV + 1, LMAX>::fwd(v, L);
      }
    }
  }
  static __device__ __forceinline__ void inv(T* v, int L) {
    if constexpr (LEV <= LMAX) {
      if (LEV <= L) {
        Lift<T, S, WAV, LEV + 1, LMAX>::inv(v, L);
        if constexpr (WAV == W_BL53) bl53_inv<T, S, LEV>(v); else haar_inv<T, S, LEV>(v);
      }
    }
  }
  // BL5/3 inverse of a line whose details are all zero (its only nonzero
  // entries are coarse samples): the predicts alone, the same bits as inv.
  static __device__ __forceinline__ void inv_samples(T* v, int L) {
    static_assert(WAV == W_BL53, "BL5/3 only");
    if constexpr (LEV <= LMAX) {
      if (LEV <= L) {
        Lift<T, S, WAV, LEV + 1, LMAX>::inv_samples(v, L);
        bl53_inv_predict<T, S, LEV>(v);
      }
    }
  }
};

// Line of the calling thread in a pass: field f and line index r (a column x
// in column passes, a row y in row passes).
template <class C>
__device__ __forceinline__ bool pass_line(int& f, int& r) {
  const int wave = tid_of<C>() >> 6;
  const int lane = tid_of<C>() & 63;
  if (wave < C::M) {
    f = wave;
    r = lane;
    return lane < C::P;
  }
  if (C::RIM && wave == C::M) {
    f = lane < C::M ? lane : 0;
    r = C::P;
    return lane < C::M;
  }
  f = 0;
  r = 0;
  return false;
}

template <class C, class T>
__device__ __forceinline__ void load_col(T* v, const T* tile, int fb, int x) {
#pragma unroll
  for (int y = 0; y < C::S; ++y) v[y] = tile[fb + y * C::RS + x];
}
template <class C, class T>
__device__ __forceinline__ void store_col(const T* v, T* tile, int fb, int x) {
#pragma unroll
  for (int y = 0; y < C::S; ++y) tile[fb + y * C::RS + x] = v[y];
}
template <class C, class T>
__device__ __forceinline__ void load_row(T* v, const T* tile, int fb, int y) {
#pragma unroll
  for (int x = 0; x < C::S; ++x) v[x] = tile[fb + y * C::RS + x];
}
template <class C, class T>
__device__ __forceinline__ void store_row(const T* v, T* tile, int fb, int y) {
#pragma unroll
  for (int x = 0; x < C::S; ++x) tile[fb + y * C::RS + x] = v[x];
}

// Hard threshold of column x (register index = y).  The threshold of element
// y depends on y only through its level class, so it is computed once per
// class per column.
template <class C, class T>
__device__ __forceinline__ void threshold_column(T* v, int x, int L, T eps, int rule) {
  const int rx = dim_rank(x, L);
  T tl[C::LMAX + 2];
#pragma unroll
  for (int k = 1; k <= C::LMAX + 1; ++k) tl[k] = thr_of<T>(rx, (k > L) ? -1 : L - k, eps, rule);
#pragma unroll
  for (int y = 0; y < C::S; ++y) {
    const T thr = tl[level_class<C::LMAX>(y)];
    v[y] = (fabs(v[y]) < thr) ? T(0) : v[y];
  }
}

// Periodic index of a patch coordinate (v within one period of [0, n)).
__device__ __forceinline__ int wrap(int v, int n) { return v < 0 ? v + n : (v >= n ? v - n : v); }

// Patch coordinates of patch q (row-major): a mask and a shift when the number
// of patches per side is a power of two, so that the start of a patch does not
// wait on an integer division.
__device__ __forceinline__ void patch_xy(const PatchArgs& a, int q, int& px, int& py) {
  if (a.npx_shift >= 0) {
    px = q & (a.npx - 1);
    py = q >> a.npx_shift;
  } else {
    px = q % a.npx;
    py = q / a.npx;
  }
}

// Threshold constant of patch q: the per-patch value when one is set.
__device__ __forceinline__ double patch_eps(const PatchArgs& a, int q) {
  return a.eps_patch ? a.eps_patch[q] : a.eps;
}

// Threshold level count of patch q: the L_q finest detail levels may be
// zeroed, with ranks counted from the coarsest of them (Section 2.2 with L_q
// in place of L); coarser coefficients are kept like samples.
__device__ __forceinline__ int patch_thr_levels(const PatchArgs& a, int q) {
  return a.lev_patch ? (int)a.lev_patch[q] : a.levels;
}

// Threshold of patch q's column x for level class k of y (see threshold_column).
template <class C, class T>
__device__ __forceinline__ T class_threshold(int x, int k, T eps, int lq, int rule) {
  return thr_of<T>(dim_rank(x, lq), (k > lq) ? -1 : lq - k, eps, rule);
}

// Hard threshold of column x of patch q with per-patch controls.  The
// column's own thresholds come from the patch's constant and level count.
// With BL5/3 tiles a bordering line is stored by both tiles that share it
// (Section 3.1.1), so it takes, entry by entry, the smaller of the two tiles'
// thresholds: both keep the same coefficients of it and reconstruct the same
// shared values, on which the conservation of the totals rests.  The columns
// x = 0 and x = P are shared with the left and right neighbours, the entries
// y = 0 and y = P with the lower and upper ones (corners are samples).
template <class C, class T>
__device__ __forceinline__ void threshold_patch_column(const PatchArgs& a, int q, T* v, int x, int L) {
  if (!a.eps_patch && !a.lev_patch) {
    threshold_column<C, T>(v, x, L, T(a.eps), a.rule);
    return;
  }
  const int rule = a.rule;
  const T e0 = T(patch_eps(a, q));
  const int l0 = patch_thr_levels(a, q);
  T tl[C::LMAX + 2];
#pragma unroll
  for (int k = 1; k <= C::LMAX + 1; ++k) tl[k] = class_threshold<C, T>(x, k, e0, l0, rule);
  T row0 = tl[C::LMAX + 1], rowp = tl[C::LMAX + 1];   // y = 0 and y = P: sample rows
  if constexpr (C::RIM) {
    int px, py;
    patch_xy(a, q, px, py);
    if (x == 0 || x == C::P) {
      const int nb = wrap(px + (x == 0 ? -1 : 1), a.npx) + a.npx * py;
      const T e1 = T(patch_eps(a, nb));
      const int l1 = patch_thr_levels(a, nb);
#pragma unroll
      for (int k = 1; k <= C::LMAX + 1; ++k) tl[k] = fmin(tl[k], class_threshold<C, T>(x, k, e1, l1, rule));
      row0 = tl[C::LMAX + 1];
      rowp = tl[C::LMAX + 1];
    }
    const int dn = px + a.npx * wrap(py - 1, a.npx);
    const int upn = px + a.npx * wrap(py + 1, a.npx);
    row0 = fmin(row0, class_threshold<C, T>(x, C::LMAX + 1, T(patch_eps(a, dn)), patch_thr_levels(a, dn), rule));
    rowp = fmin(rowp, class_threshold<C, T>(x, C::LMAX + 1, T(patch_eps(a, upn)), patch_thr_levels(a, upn), rule));
  }
#pragma unroll
  for (int y = 0; y < C::S; ++y) {
    T thr = tl[level_class<C::LMAX>(y)];
    if (y == 0) thr = row0;
    if (C::RIM && y == C::S - 1) thr = rowp;
    v[y] = (fabs(v[y]) < thr) ? T(0) : v[y];
  }
}

// Network input of patch q, per patch 4 M channels of 8 x 8 (64 x 64
// patches): channel f the stored coefficients of field f at the owned
// positions of stride 8 (written from the column of lane x = 8 i), channel
// M + 3 f + l - 1 the energy (sum of squares, before the threshold) of field
// f's coefficients of level l = 1, 2, 3 in each 8 x 8 block of owned
// positions.  The level of coefficient (x, y) is the finer of its two
// per-dimension levels (a sample index counts as coarser than any level);
// every coefficient of a block but the one at its stride-8 corner has a level
// of at most 3, the levels the stride-8 view does not hold.
constexpr int FEAT_CH_PER_FIELD = 4;

// Energies of column x (its coefficients before the threshold in v), by 8 x 8
// block and level; called by whole field waves (lane = column x < 64).  The
// eight lanes of a block add their sums by a fixed butterfly.
template <class C, class T>
__device__ __forceinline__ void export_energies(const PatchArgs& a, int q, int f, int x, const T* v, int L) {
  if constexpr (C::P == 64) {
    const int lm = (1 << L) - 1;
    const int cx = (x & lm) == 0 ? 64 : 1 + __builtin_ctz((unsigned)x);
    float* dst = a.features + ((size_t)q * FEAT_CH_PER_FIELD * C::M + C::M + 3 * f) * 64;
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      float e[3] = {0.f, 0.f, 0.f};
#pragma unroll
      for (int yy = 0; yy < 8; ++yy) {
        const int y = 8 * j + yy;
        const int cy = (y & lm) == 0 ? 64 : 1 + __builtin_ctz((unsigned)(y == 0 ? 1 : y));
        const int l = cx < cy ? cx : cy;
        const float c = (float)v[y];
#pragma unroll
        for (int k = 0; k < 3; ++k) e[k] = fmaf(l == k + 1 ? c : 0.f, c, e[k]);
      }
#pragma unroll
      for (int d = 1; d < 8; d <<= 1) {
#pragma unroll
        for (int k = 0; k < 3; ++k) e[k] += __shfl_xor(e[k], d, 64);
      }
      if ((x & 7) == 0) {
#pragma unroll
        for (int k = 0; k < 3; ++k) dst[k * 64 + 8 * j + (x >> 3)] = e[k];
      }
    }
  }
}

// Network input of patch q: the stored coefficients of the owned positions
// of stride 8 (8 x 8 per field), from the column of lane x (x = 8 i).
template <class C, class T>
__device__ __forceinline__ void export_features(const PatchArgs& a, int q, int f, int x, const T* v) {
  if constexpr (C::P == 64) {
    if (a.features && (x & 7) == 0 && x < C::P) {
      float* dst = a.features + ((size_t)q * FEAT_CH_PER_FIELD * C::M + f) * 64 + (x >> 3);
#pragma unroll
      for (int i = 0; i < 8; ++i) dst[8 * i] = (float)v[8 * i];
    }
  }
}

// S9 partial of one column of coefficients: trapezoid weights of the coarse
// samples (1/2 on the tile ends for BL5/3), FP64, ascending y.  The level
// count is uniform, so the branch on it is scalar and only the samples are
// converted and added.  0 for a detail column.
template <class C, class T, int LL = 1>
__device__ __forceinline__ double samples_of_column(const T* v, int L) {
  if constexpr (LL > C::LMAX) {
    return 0.0;
  } else {
    if (L == LL) {
      double acc = 0.0;
#pragma unroll
      for (int y = 0; y < C::S; y += (1 << LL)) {
        const double w = (C::RIM && (y == 0 || y == C::S - 1)) ? 0.5 : 1.0;
        acc += w * (double)v[y];
      }
      return acc;
    }
    return samples_of_column<C, T, LL + 1>(v, L);
  }
}

template <class C, class T>
__device__ __forceinline__ double column_sample_sum(const T* v, int x, int L) {
  if ((x & ((1 << L) - 1)) != 0) return 0.0;
  const double wx = (C::RIM && (x == 0 || x == C::S - 1)) ? 0.5 : 1.0;
  return wx * samples_of_column<C, T>(v, L);
}

// Waves 0..M-1 reduce the column partials of their field into sm.tot[f]; the
// shared-column wave stores one partial per lane (field) in sm.totface.
template <class C, class T, class SM>
__device__ __forceinline__ void totals_partial(double part, SM& sm) {
  const int wave = tid_of<C>() >> 6;
  const int lane = lane_of<C>();
  if (wave < C::M) {
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) part += __shfl_xor(part, d, 64);
    if (lane == 0) sm.tot[wave] = part;
  } else if (C::RIM && wave == C::M && lane < C::M) {
    sm.totface[lane] = part;
  }
}

// Per-field totals of the patch: by the conservation identity of the lifting
// (equation "conservation", per dimension), the trapezoid mass of the
// reconstructed tile is 4^L times the coarse trapezoid mass of its samples,
// whatever the thresholded details are.
//
// With CHECK, a non-finite total raises the abort flag: the forward lifting
// carries every element into the coarse samples of its lines (each detail
// enters at least one interior sample update at every level), so a
// non-finite value anywhere in the transformed tile makes a sample, and
// hence its field's total, non-finite.
template <class C, class T, bool CHECK, class SM>
__device__ __forceinline__ void totals_finish(const PatchArgs& a, double* out, int L, SM& sm) {
  const int tid = tid_of<C>();
  if (tid < C::M) {
    const double s = (double)(1 << L) * (double)(1 << L);
    const double t = s * (sm.tot[tid] + (C::RIM ? sm.totface[tid] : 0.0));
    out[tid] = t;
    if (CHECK && !(fabs(t) <= 0x1.fffffffffffffp+1023)) {
      atomicOr(&a.ctrl->abort, ABORT_NONFINITE);
      atomicMin(&a.ctrl->abort_epoch, a.epoch);
    }
  }
}

// ---------------------------------------------------------------------------
// S3: ghost values
// ---------------------------------------------------------------------------
// halo[q][side][slot][S] holds the line of patch q that fills ghost side
// `side` of the neighbour on the opposite side: W <- line x = HI of the west
// neighbour, E <- line x = LO of the east one, S <- line y = HI of the south
// one, N <- line y = LO of the north one.  For D2Q9 only the three
// populations streaming into the neighbour are kept; for FV every field.


// D2Q9: W/E strips (rows 0..S-1) for the x shift of the row pass, and the
// S/N ghost rows of the tile, already shifted in x: row -1 of population i
// holds f_i(x - c_ix, -1), row S holds f_i(x - c_ix, S).
// Ghost value k (0 <= k < 4 * 3 * S): loaded into v; returns its LDS slot.
// D2Q9::SIDE_POP[side][slot] and D2Q9::CX[pop] for per-lane indices, as shifts
// of packed constants: an indexed constant array is read from memory, and the
// two lookups would delay the ghost load of every patch by two dependent loads.
constexpr unsigned long long side_pop_packed() {
  unsigned long long v = 0ull;
  for (int s = 0; s < 4; ++s)
    for (int k = 0; k < 3; ++k) v |= (unsigned long long)D2Q9::SIDE_POP[s][k] << (4 * (3 * s + k));
  return v;
}
constexpr unsigned int cx_packed() {
  unsigned int v = 0u;
  for (int i = 0; i < 9; ++i) v |= (unsigned int)(D2Q9::CX[i] + 1) << (2 * i);
  return v;
}
__device__ __forceinline__ int side_pop(int side, int slot) {
  return (int)((side_pop_packed() >> (4 * (3 * side + slot))) & 15ull);
}
__device__ __forceinline__ int d2q9_cx(int pop) { return (int)((cx_packed() >> (2 * pop)) & 3u) - 1; }

template <class C, class T>
__device__ __forceinline__ T* gather_lbm_at(const PatchArgs& a, int q, int k, T* tile, T* ghost, T& v) {
  const T* h = static_cast<const T*>(a.halo_in);
  int px, py;
  patch_xy(a, q, px, py);
  const int side = k / (3 * C::S);
  const int rem = k - side * (3 * C::S);
  const int slot = rem / C::S;
  const int j = rem - slot * C::S;
  if (side < 2) {
    const int nb = wrap(px + (side == 0 ? -1 : 1), a.npx) + a.npx * py;
    v = h[((size_t)(nb * 4 + side) * 3 + slot) * C::S + j];
    return ghost + k;
  }
  const int pop = side_pop(side, slot);
  const int xs = j - d2q9_cx(pop);
  const int ox = xs < 0 ? -1 : (xs >= C::S ? 1 : 0);
  const int xl = xs - C::P * ox;
  const int nb = wrap(px + ox, a.npx) + a.npx * wrap(py + (side == 2 ? -1 : 1), a.npx);
  const int row = side == 2 ? -1 : C::S;
  v = h[((size_t)(nb * 4 + side) * 3 + slot) * C::S + xl];
  return tile + field_base<C>(pop) + row * C::RS + j;
}

template <class C, class T>
__device__ __forceinline__ void gather_lbm(const PatchArgs& a, int q, T* tile, T* ghost) {
  for (int k = tid_of<C>(); k < 4 * 3 * C::S; k += C::NT) {
    T v;
    T* d = gather_lbm_at<C, T>(a, q, k, tile, ghost, v);
    *d = v;
  }
}

// FV: the four ghost strips (no corners: the flux stencil has five points).
template <class C, class T>
__device__ __forceinline__ void gather_fv(const PatchArgs& a, int q, T* ghost) {
  const T* h = static_cast<const T*>(a.halo_in);
  int px, py;
  patch_xy(a, q, px, py);
  for (int k = tid_of<C>(); k < 4 * C::NSLOT * C::S; k += C::NT) {
    const int side = k / (C::NSLOT * C::S);
    const int rem = k - side * (C::NSLOT * C::S);
    const int slot = rem / C::S;
    const int j = rem - slot * C::S;
    int nx = px, ny = py;
    if (side < 2) nx = wrap(px + (side == 0 ? -1 : 1), a.npx);
    else ny = wrap(py + (side == 2 ? -1 : 1), a.npx);
    const int nb = nx + a.npx * ny;
    ghost[k] = h[((size_t)(nb * 4 + side) * C::NSLOT + slot) * C::S + j];
  }
}

// Slot of D2Q9 population f among those entering through side `side`.
__device__ __forceinline__ int pop_slot(int side, int f) {
  return side_pop(side, 0) == f ? 0 : (side_pop(side, 1) == f ? 1 : 2);
}

__device__ __forceinline__ bool pop_enters(int side, int f) {
  return side_pop(side, 0) == f || side_pop(side, 1) == f || side_pop(side, 2) == f;
}

// ---------------------------------------------------------------------------
// Row passes
// ---------------------------------------------------------------------------

enum RowMode : int {
  ROW_FWD = 0,        // forward x levels
  ROW_INV = 1,        // inverse x levels
  ROW_INV_SHIFT = 2,  // inverse, then D2Q9 streaming in x (ghosts at the ends)
  ROW_INV_EXPORT = 3, // inverse, then export of the lines neighbours need
  ROW_INV_DENSE = 4   // inverse, then owned nodes to the dense output
};

// SAMPLES: an inverse pass at the full level count over a tile whose
// coefficients are coarse samples only (after its column inverse, every row
// is zero but at the sample columns, and its details are zero): only those
// entries are read, and the predicts alone invert the row.
template <class C, class T, int WAV, int SCH, int MODE, bool SAMPLES = false>
__device__ __forceinline__ void row_pass(const PatchArgs& a, int q, T* tile, const T* ghost) {
  using LF = Lift<T, C::S, WAV, 1, C::LMAX>;
  int f, y;
  if (pass_line<C>(f, y)) {
    const int fb = field_base<C>(f);
    T v[C::S];
    if constexpr (SAMPLES) {
      constexpr int SMASK = (1 << C::LMAX) - 1;   // the full level count (checked by the caller)
#pragma unroll
      for (int x = 0; x < C::S; ++x) v[x] = ((x & SMASK) == 0) ? tile[fb + y * C::RS + x] : T(0);
      LF::inv_samples(v, C::LMAX);
    } else {
      load_row<C>(v, tile, fb, y);
      if constexpr (MODE == ROW_FWD) LF::fwd(v, a.levels); else LF::inv(v, a.levels);
    }
    if constexpr (MODE == ROW_INV_SHIFT) {
      // Streaming in x through the store address: node x of the row goes to
      // x + c_x; the freed end takes the ghost value (c_x = +1: x = 0 from
      // the W strip; c_x = -1: x = S - 1 from the E strip).
      const int cx = pop_enters(0, f) ? 1 : (pop_enters(1, f) ? -1 : 0);
      T* row = tile + fb + y * C::RS + cx;
#pragma unroll
      for (int x = 0; x < C::S; ++x) {
        if ((x > 0 || cx >= 0) && (x < C::S - 1 || cx <= 0)) row[x] = v[x];
      }
      if (cx == 1) tile[fb + y * C::RS] = ghost[(0 * 3 + pop_slot(0, f)) * C::S + y];
      else if (cx == -1) tile[fb + y * C::RS + C::S - 1] = ghost[(1 * 3 + pop_slot(1, f)) * C::S + y];
    } else if constexpr (MODE == ROW_INV_EXPORT) {
      T* h = static_cast<T*>(a.halo_out);
      const size_t hq = (size_t)q * 4;
      if constexpr (SCH == S_LBM) {
        if (pop_enters(0, f)) h[((hq + 0) * 3 + pop_slot(0, f)) * C::S + y] = v[C::HI];
        if (pop_enters(1, f)) h[((hq + 1) * 3 + pop_slot(1, f)) * C::S + y] = v[C::LO];
        if (y == C::HI && pop_enters(2, f)) {
#pragma unroll
          for (int x = 0; x < C::S; ++x) h[((hq + 2) * 3 + pop_slot(2, f)) * C::S + x] = v[x];
        }
        if (y == C::LO && pop_enters(3, f)) {
#pragma unroll
          for (int x = 0; x < C::S; ++x) h[((hq + 3) * 3 + pop_slot(3, f)) * C::S + x] = v[x];
        }
      } else {
        h[((hq + 0) * C::NSLOT + f) * C::S + y] = v[C::HI];
        h[((hq + 1) * C::NSLOT + f) * C::S + y] = v[C::LO];
        if (y == C::HI) {
#pragma unroll
          for (int x = 0; x < C::S; ++x) h[((hq + 2) * C::NSLOT + f) * C::S + x] = v[x];
        }
        if (y == C::LO) {
#pragma unroll
          for (int x = 0; x < C::S; ++x) h[((hq + 3) * C::NSLOT + f) * C::S + x] = v[x];
        }
      }
    } else if constexpr (MODE == ROW_INV_DENSE) {
      if (y < C::P) {
        const int px = q % a.npx;
        const int py = q / a.npx;
        T* out = static_cast<T*>(a.dense_out) + ((size_t)f * a.n + (size_t)py * C::P + y) * a.n +
                 (size_t)px * C::P;
#pragma unroll
        for (int x = 0; x < C::P; ++x) out[x] = v[x];
      }
    } else {
      store_row<C>(v, tile, fb, y);
    }
  }
}

// ---------------------------------------------------------------------------
// S8, row half, folded BL5/3: only what the neighbours read
// ---------------------------------------------------------------------------
// The x strips need each row's value at nodes LO = 1 and HI = P - 1 only.
// The inverse of levels L..1 at node 1 depends on the coarse sample at 2^L,
// the boundary node 0 and the details at 2^(lev-1) and 3 * 2^(lev-1) of each
// level: per level one update of the sample at 2 * st (k = 1) and one
// predict of the detail at st (k = 0), in the operation order of the full
// inverse, so the value is the one the full inverse gives.  Node P - 1 is the
// mirror image (update of k = m - 1, predict of k = m - 1).
template <class C, class T, bool MIRROR>
__device__ __forceinline__ T bl53_inv_edge(const T* row, int L) {
  auto at = [row](int j) { return MIRROR ? row[C::S - 1 - j] : row[j]; };
  T y = at(1 << L);
#pragma unroll
  for (int lev = C::LMAX; lev >= 1; --lev) {
    if (lev > L) continue;
    const int st = 1 << (lev - 1);
    const int m = (C::S - 1) / (2 * st);
    const T a1 = (m == 2) ? T(0.5) : T(0.25);
    T e;
    if constexpr (!MIRROR) e = (y - T(0.5) * at(st)) - a1 * at(3 * st);
    else e = (y - a1 * at(3 * st)) - T(0.5) * at(st);
    if constexpr (!MIRROR) y = at(st) + (at(0) + e) * T(0.5);
    else y = at(st) + (e + at(0)) * T(0.5);
  }
  return y;
}

// Export of the lines the neighbours need (the tile holds the column-inverted
// coefficients): the line waves compute the x strips' two values of their
// rows; the helper waves invert the full rows LO and HI of the y strips.
template <class C, class T, int SCH>
__device__ __forceinline__ void export_rows_bl53(const PatchArgs& a, int q, const T* tile) {
  using LF = Lift<T, C::S, W_BL53, 1, C::LMAX>;
  static_assert(C::NHT >= 2 * C::M, "one helper thread per exported full row");
  T* h = static_cast<T*>(a.halo_out);
  const size_t hq = (size_t)q * 4;
  const int L = a.levels;
  int f, y;
  if (pass_line<C>(f, y)) {
    const T* row = tile + field_base<C>(f) + y * C::RS;
    if constexpr (SCH == S_LBM) {
      if (pop_enters(0, f)) h[((hq + 0) * 3 + pop_slot(0, f)) * C::S + y] = bl53_inv_edge<C, T, true>(row, L);
      if (pop_enters(1, f)) h[((hq + 1) * 3 + pop_slot(1, f)) * C::S + y] = bl53_inv_edge<C, T, false>(row, L);
    } else {
      h[((hq + 0) * C::NSLOT + f) * C::S + y] = bl53_inv_edge<C, T, true>(row, L);
      h[((hq + 1) * C::NSLOT + f) * C::S + y] = bl53_inv_edge<C, T, false>(row, L);
    }
  } else if ((int)(tid_of<C>() >> 6) >= C::NPASS) {
    // helper item: field g, row HI (even item) or LO (odd item)
    const int ht = (int)tid_of<C>() - 64 * C::NPASS;
    const int g = ht >> 1;
    if (g < C::M) {
      const bool hi = (ht & 1) == 0;
      const int side = hi ? 2 : 3;
      const bool need = SCH == S_LBM ? pop_enters(side, g) : true;
      if (need) {
        T v[C::S];
        load_row<C>(v, tile, field_base<C>(g), hi ? C::HI : C::LO);
        LF::inv(v, L);
        T* dst = SCH == S_LBM ? h + ((hq + side) * 3 + pop_slot(side, g)) * C::S
                              : h + ((hq + side) * C::NSLOT + g) * C::S;
#pragma unroll
        for (int x = 0; x < C::S; ++x) dst[x] = v[x];
      }
    }
  }
}

template <class C, class T, int WAV, int SCH>
__device__ __forceinline__ void export_rows(const PatchArgs& a, int q, T* tile, const T* ghost) {
  if constexpr (WAV == W_BL53) export_rows_bl53<C, T, SCH>(a, q, tile);
  else row_pass<C, T, WAV, SCH, ROW_INV_EXPORT>(a, q, tile, ghost);
}

// ---------------------------------------------------------------------------
// Stencils (S4)
// ---------------------------------------------------------------------------

// D2Q9 BGK collision of the streamed populations f (moments, equilibrium
// w_i rho (1 + 3 c.u + 4.5 (c.u)^2 - 1.5 u.u), relaxation by omega = 1/tau).
template <class T>
__device__ __forceinline__ void d2q9_collide(const T* f, T omega, T* out) {
  const T rho = ((f[0] + f[1]) + (f[2] + f[3])) + ((f[4] + f[5]) + (f[6] + f[7])) + f[8];
  const T jx = ((f[1] - f[3]) + (f[5] - f[6])) + (f[8] - f[7]);
  const T jy = ((f[2] - f[4]) + (f[5] + f[6])) - (f[7] + f[8]);
  const T inv = T(1) / rho;
  const T ux = jx * inv;
  const T uy = jy * inv;
  const T usq = T(1.5) * (ux * ux + uy * uy);
  const T wr[3] = {T(4.0 / 9.0) * rho, T(1.0 / 9.0) * rho, T(1.0 / 36.0) * rho};
  const T cuv[9] = {T(0), ux, uy, -ux, -uy, ux + uy, uy - ux, -(ux + uy), ux - uy};
#pragma unroll
  for (int i = 0; i < 9; ++i) {
    const T cu = cuv[i];
    const T w = wr[i == 0 ? 0 : (i < 5 ? 1 : 2)];
    const T feq = w * ((T(1) + T(3) * cu) + (T(4.5) * cu * cu - usq));
    out[i] = f[i] - omega * (f[i] - feq);
  }
}

// D2Q9: the x part of streaming was applied by the row pass, so population i
// of node (x, y) is read at row y - c_iy of its field (a ghost row at the
// tile edge): a fixed offset per population.
template <class C, class T>
__device__ __forceinline__ void stencil_lbm(const PatchArgs& a, T* tile) {
  const T omega = T(a.omega);
  T res[C::NPER][9];
#pragma unroll
  for (int k = 0; k < C::NPER; ++k) {
    const int t = tid_of<C>() + k * C::NT;
    if (t < C::NC) {
      const int y = t / C::S;
      const int base = y * C::RS + (t - y * C::S);
      T fin[9];
#pragma unroll
      for (int i = 0; i < 9; ++i) fin[i] = tile[C::Lay::fb(i) - D2Q9::CY[i] * C::RS + base];
      d2q9_collide<T>(fin, omega, res[k]);
    }
  }
  __syncthreads();
#pragma unroll
  for (int k = 0; k < C::NPER; ++k) {
    const int t = tid_of<C>() + k * C::NT;
    if (t < C::NC) {
      const int y = t / C::S;
      const int base = y * C::RS + (t - y * C::S);
#pragma unroll
      for (int i = 0; i < 9; ++i) tile[C::Lay::fb(i) + base] = res[k][i];
    }
  }
  __syncthreads();
}

// Finite-volume update of equation "vf_scheme" in the order of the transport
// listing: W' = W, then W' -= dt/h * (W max(a.N^k,0) + W_k min(a.N^k,0)) for
// N^0..3 = +x, -x, +y, -y.  Ghost strips: 0 = W, 1 = E, 2 = S, 3 = N.
template <class C, class T>
__device__ __forceinline__ void stencil_fv(const PatchArgs& a, T* tile, const T* ghost) {
  const T r = T(a.dt_over_h);
  const T cp0 = T(a.cp[0]), cp1 = T(a.cp[1]), cp2 = T(a.cp[2]), cp3 = T(a.cp[3]);
  const T cm0 = T(a.cm[0]), cm1 = T(a.cm[1]), cm2 = T(a.cm[2]), cm3 = T(a.cm[3]);
  T res[C::M][C::NPER];
#pragma unroll
  for (int f = 0; f < C::M; ++f) {
    const T* tf = tile + C::Lay::fb(f);
    const T* g = ghost + f * C::S;
#pragma unroll
    for (int k = 0; k < C::NPER; ++k) {
      const int t = tid_of<C>() + k * C::NT;
      if (t < C::NC) {
        const int y = t / C::S;
        const int x = t - y * C::S;
        const T w = tf[y * C::RS + x];
        const T we = (x + 1 < C::S) ? tf[y * C::RS + x + 1] : g[(1 * C::NSLOT) * C::S + y];
        const T ww = (x >= 1) ? tf[y * C::RS + x - 1] : g[(0 * C::NSLOT) * C::S + y];
        const T wn = (y + 1 < C::S) ? tf[(y + 1) * C::RS + x] : g[(3 * C::NSLOT) * C::S + x];
        const T wsd = (y >= 1) ? tf[(y - 1) * C::RS + x] : g[(2 * C::NSLOT) * C::S + x];
        T o = w;
        o = o - r * (w * cp0 + we * cm0);
        o = o - r * (w * cp1 + ww * cm1);
        o = o - r * (w * cp2 + wn * cm2);
        o = o - r * (w * cp3 + wsd * cm3);
        res[f][k] = o;
      }
    }
  }
  __syncthreads();
#pragma unroll
  for (int f = 0; f < C::M; ++f) {
#pragma unroll
    for (int k = 0; k < C::NPER; ++k) {
      const int t = tid_of<C>() + k * C::NT;
      if (t < C::NC) {
        const int y = t / C::S;
        tile[C::Lay::fb(f) + y * C::RS + (t - y * C::S)] = res[f][k];
      }
    }
  }
  __syncthreads();
}

// Compressible Euler with the Rusanov flux: W = (rho, rho u, rho v, E),
// F(W).N = (rho un, rho u un + p Nx, rho v un + p Ny, (E + p) un),
// Q(W_L, W_R, N) = (F(W_L).N + F(W_R).N) / 2 - lambda (W_R - W_L) / 2 with
// lambda = max(|un_L| + c_L, |un_R| + c_R), applied as in equation
// "vf_scheme" in the direction order +x, -x, +y, -y.
template <class T>
__device__ __forceinline__ void euler_prim(const T* w, T gamma, T& u, T& v, T& p, T& c) {
  const T inv = T(1) / w[0];
  u = w[1] * inv;
  v = w[2] * inv;
  p = (gamma - T(1)) * (w[3] - T(0.5) * w[0] * (u * u + v * v));
  c = sqrt(gamma * p * inv);
}

template <class T, int NX, int NY>
__device__ __forceinline__ void euler_face(const T* wl, T ul, T vl, T pl, T cl, const T* wr, T gamma, T r,
                                           T* o) {
  T ur, vr, pr, cr;
  euler_prim<T>(wr, gamma, ur, vr, pr, cr);
  const T unl = ul * T(NX) + vl * T(NY);
  const T unr = ur * T(NX) + vr * T(NY);
  const T lam = fmax(fabs(unl) + cl, fabs(unr) + cr);
  const T fl[4] = {wl[0] * unl, wl[1] * unl + pl * T(NX), wl[2] * unl + pl * T(NY), (wl[3] + pl) * unl};
  const T fr[4] = {wr[0] * unr, wr[1] * unr + pr * T(NX), wr[2] * unr + pr * T(NY), (wr[3] + pr) * unr};
#pragma unroll
  for (int k = 0; k < 4; ++k) o[k] = o[k] - r * (T(0.5) * (fl[k] + fr[k]) - T(0.5) * lam * (wr[k] - wl[k]));
}

// One Euler update of a node from its state and its four neighbours.
template <class T>
__device__ __forceinline__ void euler_node(const T* w, const T* we, const T* ww, const T* wn, const T* ws,
                                           T gamma, T r, T* o) {
  T u, v, p, c;
  euler_prim<T>(w, gamma, u, v, p, c);
#pragma unroll
  for (int k = 0; k < 4; ++k) o[k] = w[k];
  euler_face<T, 1, 0>(w, u, v, p, c, we, gamma, r, o);
  euler_face<T, -1, 0>(w, u, v, p, c, ww, gamma, r, o);
  euler_face<T, 0, 1>(w, u, v, p, c, wn, gamma, r, o);
  euler_face<T, 0, -1>(w, u, v, p, c, ws, gamma, r, o);
}

template <class C, class T>
__device__ __forceinline__ void stencil_euler(const PatchArgs& a, T* tile, const T* ghost) {
  static_assert(C::M == 4, "four conserved fields");
  const T r = T(a.dt_over_h);
  const T gamma = T(a.gamma);
  T res[4][C::NPER];
#pragma unroll
  for (int k = 0; k < C::NPER; ++k) {
    const int t = tid_of<C>() + k * C::NT;
    if (t < C::NC) {
      const int y = t / C::S;
      const int x = t - y * C::S;
      T w[4], we[4], ww[4], wn[4], ws[4];
#pragma unroll
      for (int f = 0; f < 4; ++f) {
        const T* tf = tile + C::Lay::fb(f);
        const T* g = ghost + f * C::S;
        w[f] = tf[y * C::RS + x];
        we[f] = (x + 1 < C::S) ? tf[y * C::RS + x + 1] : g[(1 * C::NSLOT) * C::S + y];
        ww[f] = (x >= 1) ? tf[y * C::RS + x - 1] : g[(0 * C::NSLOT) * C::S + y];
        wn[f] = (y + 1 < C::S) ? tf[(y + 1) * C::RS + x] : g[(3 * C::NSLOT) * C::S + x];
        ws[f] = (y >= 1) ? tf[(y - 1) * C::RS + x] : g[(2 * C::NSLOT) * C::S + x];
      }
      T o[4];
      euler_node<T>(w, we, ww, wn, ws, gamma, r, o);
#pragma unroll
      for (int f = 0; f < 4; ++f) res[f][k] = o[f];
    }
  }
  __syncthreads();
#pragma unroll
  for (int f = 0; f < 4; ++f) {
#pragma unroll
    for (int k = 0; k < C::NPER; ++k) {
      const int t = tid_of<C>() + k * C::NT;
      if (t < C::NC) {
        const int y = t / C::S;
        tile[C::Lay::fb(f) + y * C::RS + (t - y * C::S)] = res[f][k];
      }
    }
  }
  __syncthreads();
}

// ---------------------------------------------------------------------------
// Optional per-phase wall-clock marks of the step kernel (profiling builds
// compiled with -DLBMZ_PHASE_CLOCK; the product build has none).
// ---------------------------------------------------------------------------
#ifdef LBMZ_PHASE_CLOCK
static __device__ unsigned long long lbmz_phase_clock[4096 * 16];
#define LBMZ_MARK(k)                                                                                    \
  do {                                                                                                  \
    if (threadIdx.x == 0 && blockIdx.x < 4096) lbmz_phase_clock[blockIdx.x * 16 + (k)] = wall_clock64(); \
  } while (0)
#else
#define LBMZ_MARK(k) \
  do {               \
  } while (0)
#endif

// Offset-table entries of patch q into LDS (read by the expansion after the
// next barrier); issued early so that their latency overlaps other loads.
template <class C, class SM>
__device__ __forceinline__ void prefetch_table(const PatchArgs& a, int q, SM& sm) {
  if (tid_of<C>() < 2 * C::M) sm.te[tid_of<C>()] = a.table_in[2 * (size_t)q * C::M + tid_of<C>()];
}

// ---------------------------------------------------------------------------
// S1 (+ the column half of S2): records -> inverse-transformed columns in LDS
// ---------------------------------------------------------------------------
// Bitmask records are read straight into the column registers: the mask
// words and their prefix counts come from one load per lane, and the value of
// column x, row y sits at the prefix of its word plus the set bits below it.
// Index-list records (sparse) are scattered into a zeroed LDS tile first.
// With TOT, the S9 totals of the stored coefficients are taken on the way.

// Entries of the patch's index-list records held by the helper waves (the
// waves without a line in the passes) from the start of the patch until the
// scatter of the expansion.
template <class C, class T>
struct ListRegs {
  T lv[C::M][C::LPT];
  int li[C::M][C::LPT];
};

// Issue the loads of patch q's index-list entries (helper waves; the offset
// table is read from global memory so that the loads start before the barrier
// that precedes the expansion).
template <class C, class T>
__device__ __forceinline__ void prefetch_lists(const PatchArgs& a, int q, ListRegs<C, T>& lr) {
  const int wave = wave_of<C>();
  if (wave < C::NPASS) return;
  const int ht = tid_of<C>() - 64 * C::NPASS;
  const uint32_t* tq = a.table_in + 2 * (size_t)q * C::M;
  // all table entries first (one round trip), then every field's loads
  uint32_t tw[2 * C::M];
#pragma unroll
  for (int i = 0; i < 2 * C::M; ++i) tw[i] = (uint32_t)__builtin_amdgcn_readfirstlane((int)tq[i]);
#pragma unroll
  for (int f = 0; f < C::M; ++f) {
    const uint32_t w = tw[2 * f + 1];
    const uint32_t nnz = w & ~MASK_BIT;
#pragma unroll
    for (int u = 0; u < C::LPT; ++u) {
      lr.li[f][u] = -1;
      lr.lv[f][u] = T(0);
    }
    if (!(w & MASK_BIT)) {
      const uint8_t* rec = a.pool_in + 16ull * tw[2 * f];
      const uint16_t* idx = reinterpret_cast<const uint16_t*>(rec + ((nnz * (uint32_t)sizeof(T) + 7u) & ~7u));
#pragma unroll
      for (int u = 0; u < C::LPT; ++u) {
        const int k = ht + u * C::NHT;
        if (k < (int)nnz) {
          lr.li[f][u] = idx[k];
          lr.lv[f][u] = reinterpret_cast<const T*>(rec)[k];
        }
      }
    }
  }
}

// Mask words of a bitmask record, word k in lane k of w0 (k < 64) or lane
// k - 64 of w1.
template <class C, class T>
__device__ __forceinline__ void load_mask_words(const uint8_t* rec, uint32_t nnz, int lane, unsigned long long& w0,
                                                unsigned long long& w1) {
  const unsigned long long* words =
      reinterpret_cast<const unsigned long long*>(rec + ((nnz * (uint32_t)sizeof(T) + 7u) & ~7u));
  w0 = lane < C::W ? words[lane] : 0ull;
  w1 = (64 + lane) < C::W ? words[64 + lane] : 0ull;
}

// One value of a record through a buffer resource: byte offset voff (per
// lane) + soff (uniform).  Reads outside the record return 0.
template <class T>
__device__ __forceinline__ T record_value(__amdgpu_buffer_rsrc_t rs, uint32_t voff, uint32_t soff);
template <>
__device__ __forceinline__ float record_value<float>(__amdgpu_buffer_rsrc_t rs, uint32_t voff, uint32_t soff) {
  return __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(rs, (int)voff, (int)soff, 0));
}
template <>
__device__ __forceinline__ double record_value<double>(__amdgpu_buffer_rsrc_t rs, uint32_t voff, uint32_t soff) {
  return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(rs, (int)voff, (int)soff, 0));
}

// Column x = lane of a bitmask record (values at rec, nnz of them; mask
// words in w0 / w1): node (x, y) of an owned row sits in word y / RPW at bit
// x + P (y % RPW), the shared row y = P in the rim words (see rim_join); its
// value is the one after the kept nodes before that bit.  The word of a row
// is wave-uniform (scalar registers; the values before it by scalar adds),
// the lane's rank inside it is one mbcnt, and the value comes through a
// buffer load with that rank as its only per-lane offset.  A lane whose bit
// is clear loads from an offset outside the record and so receives 0.
template <class C, class T>
__device__ __forceinline__ void gather_owned(const uint8_t* rec, uint32_t nnz, unsigned long long w0,
                                             unsigned long long w1, T* v) {
  constexpr unsigned long long LANES = (C::P == 64) ? ~0ull : ((1ull << C::P) - 1ull);
  constexpr uint32_t B = sizeof(T);
  constexpr uint32_t OUTSIDE = 0x80000000u;   // beyond any record (at most 64 KB)
  const __amdgpu_buffer_rsrc_t rs =
      __builtin_amdgcn_make_buffer_rsrc(const_cast<uint8_t*>(rec), 0, (int)(nnz * B), BUF_WORD3);
  auto word = [&](int k) { return k < 64 ? readlane64(w0, k) : readlane64(w1, k - 64); };
  uint32_t pk = 0u;   // values before the current word
  unsigned long long wk = 0ull;
#pragma unroll
  for (int y = 0; y < C::P; ++y) {
    const int r = y % C::RPW;
    if (r == 0) {
      if (y > 0) pk += (uint32_t)__popcll(wk);
      wk = word(y / C::RPW);
    }
    const unsigned long long sh = (wk >> (C::P * r)) & LANES;
    const uint32_t base = pk + (r ? (uint32_t)__popcll(wk & ((1ull << (C::P * r)) - 1ull)) : 0u);
    const uint32_t k = __builtin_amdgcn_mbcnt_hi((uint32_t)(sh >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)sh, 0u));
    v[y] = record_value<T>(rs, __builtin_amdgcn_inverse_ballot_w64(sh) ? k * B : OUTSIDE, base * B);
  }
  if constexpr (C::RIM) {
    pk += (uint32_t)__popcll(wk);   // the owned block's values
    unsigned long long sh;
    uint32_t base;
    if constexpr (C::P == 64) {
      // word CW: the shared column; word CW + 1: the shared row
      base = pk + (uint32_t)__popcll(word(C::CW));
      sh = word(C::CW + 1);
    } else {
      const unsigned long long r0 = word(C::CW);
      base = pk + (uint32_t)__popcll(r0 & ((1ull << C::P) - 1ull));
      sh = (r0 >> C::P) & LANES;
    }
    const uint32_t k = __builtin_amdgcn_mbcnt_hi((uint32_t)(sh >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)sh, 0u));
    v[C::P] = record_value<T>(rs, __builtin_amdgcn_inverse_ballot_w64(sh) ? k * B : OUTSIDE, base * B);
  }
}

template <class C, class T, int WAV, bool TOT, bool PREZ, class SM>
__device__ __forceinline__ void expand_columns(const PatchArgs& a, int q, SM& sm, const ListRegs<C, T>& lr) {
  using LF = Lift<T, C::S, WAV, 1, C::LMAX>;
  const int tid = tid_of<C>();
  const int lane = lane_of<C>();
  const int wave = wave_of<C>();
  const int L = a.levels;
  // offset-table entries, loaded into LDS by prefetch_table before the last barrier
  // te: wave-uniform index (one scalar value), tel: index that varies over the lanes
  auto te = [&sm](int i) { return (uint32_t)__builtin_amdgcn_readfirstlane((int)sm.te[i]); };
  auto tel = [&sm](int i) { return sm.te[i]; };
  const uint8_t* pool = a.pool_in;

  // Index-list records: the helper waves (no line in the passes) hold their
  // entries (prefetch_lists) and zero their tiles, so that the line waves
  // carry no list state.  With PREZ the tiles are already zero: the D2Q9
  // step zeroes every field's owned rows at the start of the patch, under
  // the latency of its ghost loads.
  const bool helper = wave >= C::NPASS;
  const int ht = tid - 64 * C::NPASS;
  if (!PREZ && helper) {
#pragma unroll
    for (int f = 0; f < C::M; ++f)
      if (!(te(2 * f + 1) & MASK_BIT)) zero_span<T>(sm.tile + C::Lay::fb(f), C::S * C::RS, ht, C::NHT);
  }

  // Bitmask records, owned columns (waves 0..M-1).
  if (wave < C::M) {
    const int f = wave;
    const uint32_t w = te(2 * f + 1);
    if (w & MASK_BIT) {
      const uint32_t nnz = w & ~MASK_BIT;
      const uint8_t* rec = pool + 16ull * te(2 * f);
      unsigned long long w0, w1;
      load_mask_words<C, T>(rec, nnz, lane, w0, w1);
      T v[C::S];
      gather_owned<C, T>(rec, nnz, w0, w1, v);
      const int x = lane;
      double part = 0.0;
      if (x < C::P) {
        if constexpr (TOT) part = column_sample_sum<C, T>(v, x, L);
        LF::inv(v, L);
        store_col<C>(v, sm.tile, field_base<C>(f), x);
      }
      if constexpr (TOT) totals_partial<C, T>(part, sm);
    }
  }
  // Bitmask records, the shared column x = P (wave M, lane = field).
  if (C::RIM && wave == C::M && lane < C::M) {
    const int f = lane;
    const uint32_t w = tel(2 * f + 1);
    if (w & MASK_BIT) {
      const uint32_t nnz = w & ~MASK_BIT;
      const uint8_t* rec = pool + 16ull * tel(2 * f);
      const T* vals = reinterpret_cast<const T*>(rec);
      const unsigned long long* words =
          reinterpret_cast<const unsigned long long*>(rec + ((nnz * (uint32_t)sizeof(T) + 7u) & ~7u));
      // rim bit stream: column y < P at bit y, row x < P at bit P + x, corner at 2P
      const unsigned long long r0 = words[C::CW];
      const unsigned long long r1 = (C::W > C::CW + 1) ? words[C::CW + 1] : 0ull;
      const unsigned long long r2 = (C::W > C::CW + 2) ? words[C::CW + 2] : 0ull;
      const int core = (int)nnz - (__popcll(r0) + __popcll(r1) + __popcll(r2));
      unsigned long long col, rowb;
      bool corner;
      rim_split<C>(r0, r1, r2, col, rowb, corner);
      T v[C::S];
#pragma unroll
      for (int y = 0; y < C::P; ++y) {
        v[y] = T(0);
        if ((col >> y) & 1ull) v[y] = vals[core + __popcll(col & below(y))];
      }
      v[C::P] = corner ? vals[core + __popcll(col) + __popcll(rowb)] : T(0);
      if constexpr (TOT) sm.totface[f] = column_sample_sum<C, T>(v, C::P, L);
      LF::inv(v, L);
      store_col<C>(v, sm.tile, field_base<C>(f), C::P);
    }
  }
  // samples_only (set at the start of the patch) is cleared by a bitmask
  // record here and by a detail in the scatter below
  if (tid < C::M && (tel(2 * tid + 1) & MASK_BIT)) sm.samples_only = 0u;
  __syncthreads();
  LBMZ_MARK(12);

  // Index-list records: scatter, then their columns.
  if (helper) {
    int nodes = 0;   // OR of the scattered nodes' coordinates
#pragma unroll
    for (int f = 0; f < C::M; ++f) {
#pragma unroll
      for (int u = 0; u < C::LPT; ++u) {
        const int k = lr.li[f][u];
        if (k >= 0 && k < C::NC) {
          int x, y;
          record_node<C>(k, x, y);
          sm.tile[C::Lay::fb(f) + y * C::RS + x] = lr.lv[f][u];
          nodes |= x | y;
        }
      }
    }
    // a detail: a node off the lattice of the coarse samples
    if (__ballot((nodes & ((1 << L) - 1)) != 0) != 0ull && lane == 0) sm.samples_only = 0u;
  }
  __syncthreads();
  LBMZ_MARK(13);
  if constexpr (!TOT && WAV == W_BL53) {
    if (L == C::LMAX && __builtin_amdgcn_readfirstlane((int)sm.samples_only) != 0) {
      // Coarse samples only (at the full level count, so their positions are
      // known at compile time): the tile is zero but at the samples; only
      // the sample columns have anything to invert, and their details are zero.
      constexpr int SMASK = (1 << C::LMAX) - 1;
      int f, x;
      const bool line = pass_line<C>(f, x);
      if (line && (x & SMASK) == 0) {
        const T* col = sm.tile + field_base<C>(f) + x;
        T v[C::S];
#pragma unroll
        for (int y = 0; y < C::S; ++y) v[y] = ((y & SMASK) == 0) ? col[y * C::RS] : T(0);
        LF::inv_samples(v, C::LMAX);
        store_col<C>(v, sm.tile, field_base<C>(f), x);
      }
      __syncthreads();
      return;
    }
  }
  bool any_list = false;
#pragma unroll
  for (int g = 0; g < C::M; ++g) any_list |= !(te(2 * g + 1) & MASK_BIT);
  if (any_list) {
    int f, x;
    const bool line = pass_line<C>(f, x);
    const bool act = line && !(tel(2 * f + 1) & MASK_BIT);
    double part = 0.0;
    if (act) {
      T v[C::S];
      load_col<C>(v, sm.tile, field_base<C>(f), x);
      if constexpr (TOT) part = column_sample_sum<C, T>(v, x, L);
      LF::inv(v, L);
      store_col<C>(v, sm.tile, field_base<C>(f), x);
    }
    if constexpr (TOT) {
      if (wave < C::M) {
        if (!(te(2 * wave + 1) & MASK_BIT)) totals_partial<C, T>(part, sm);
      } else if (act) {
        sm.totface[f] = part;
      }
    }
    __syncthreads();
  }
}

// Lane `lane` (wave-uniform) of `old` replaced by the wave-uniform value u
// (v_writelane with the lane in M0: it reads at most one other scalar).
__device__ __forceinline__ uint32_t write_lane(uint32_t old, uint32_t u, int lane) {
  asm("s_mov_b32 m0, %2\n\ts_nop 0\n\tv_writelane_b32 %0, %1, m0" : "+v"(old) : "s"(u), "s"(lane) : "m0");
  return old;
}

// One value (or index-list entry) into a record through a buffer resource;
// a store at an offset outside the resource writes nothing.
template <class T>
__device__ __forceinline__ void record_store(T v, __amdgpu_buffer_rsrc_t rs, uint32_t voff, uint32_t soff);
template <>
__device__ __forceinline__ void record_store<float>(float v, __amdgpu_buffer_rsrc_t rs, uint32_t voff, uint32_t soff) {
  __builtin_amdgcn_raw_buffer_store_b32(__float_as_uint(v), rs, (int)voff, (int)soff, 0);
}
template <>
__device__ __forceinline__ void record_store<double>(double v, __amdgpu_buffer_rsrc_t rs, uint32_t voff,
                                                     uint32_t soff) {
  typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));
  __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2, v), rs, (int)voff, (int)soff, 0);
}

// Stores of the owned rows of a column-pass line (S7): the rank of a kept
// coefficient is the count of kept ones before it in record order; in a row,
// the kept lanes below it (one mbcnt of the row's ballot).  Lanes with
// nothing to store take an offset outside the record.  Bitmask records (MASK)
// collect the row ballots into mask words, word y / RPW in lane y / RPW of
// myw; index-list records store the node index of each value.  Returns the
// count of kept owned coefficients.
template <class C, class T, bool MASK>
__device__ __forceinline__ int store_owned_rows(const T* v, unsigned long long actm, uint8_t* rec,
                                                uint32_t nnz, uint32_t vb, unsigned long long& myw) {
  constexpr uint32_t B = sizeof(T);
  constexpr uint32_t OUTSIDE = 0x80000000u;   // beyond any record (at most 64 KB)
  const __amdgpu_buffer_rsrc_t rv = __builtin_amdgcn_make_buffer_rsrc(rec, 0, (int)(nnz * B), BUF_WORD3);
  const __amdgpu_buffer_rsrc_t ri =
      __builtin_amdgcn_make_buffer_rsrc(rec + vb, 0, MASK ? 0 : (int)(2u * nnz), BUF_WORD3);
  const int x = lane_of<C>();
  int run = 0;
  unsigned long long wd = 0ull;
  uint32_t wlo = 0u, whi = 0u;
#pragma unroll
  for (int y = 0; y < C::P; ++y) {
    const unsigned long long b = __ballot(v[y] != T(0)) & actm;   // lanes without a line hold zeros
    if (b != 0ull) {
      const uint32_t k = __builtin_amdgcn_mbcnt_hi((uint32_t)(b >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)b, 0u));
      const bool kept = __builtin_amdgcn_inverse_ballot_w64(b);
      record_store<T>(v[y], rv, kept ? k * B : OUTSIDE, (uint32_t)run * B);
      if constexpr (!MASK)
        __builtin_amdgcn_raw_buffer_store_b16((unsigned short)(x + C::P * y), ri, (int)(kept ? 2u * k : OUTSIDE),
                                              2 * run, 0);
      run += __popcll(b);
    }
    if constexpr (MASK) {
      // mask word y / RPW collects RPW rows; lane y / RPW keeps it
      wd |= b << (C::P * (y % C::RPW));
      if (y % C::RPW == C::RPW - 1) {
        wlo = write_lane(wlo, (uint32_t)wd, y / C::RPW);
        whi = write_lane(whi, (uint32_t)(wd >> 32), y / C::RPW);
        wd = 0ull;
      }
    }
  }
  myw = ((unsigned long long)whi << 32) | wlo;
  return run;
}

// ---------------------------------------------------------------------------
// S5 (column half) + S6 + S7 + S9 + S8 (column half), one column pass
// ---------------------------------------------------------------------------
// Returns false (uniformly) when the pool overflowed; the records are then
// not written and the host replays the step with a larger pool.

// CTL selects the variant with per-patch controls and the network input
// export; without it the threshold is the uniform one of the context.
template <class C, class T, int WAV, bool FWD, bool CTL, class SM>
__device__ __forceinline__ bool column_compact(const PatchArgs& a, int q, SM& sm) {
  using LF = Lift<T, C::S, WAV, 1, C::LMAX>;
  static_assert(sizeof(sm.ghost) >= sizeof(T) * C::M * C::S, "shared-column staging does not fit");
  const int tid = tid_of<C>();
  const int lane = lane_of<C>();
  const int wave = wave_of<C>();
  const int L = a.levels;
  int f, x;
  const bool act = pass_line<C>(f, x);
  T v[C::S];
#pragma unroll
  for (int y = 0; y < C::S; ++y) v[y] = T(0);
  T mag = T(0);
  double part = 0.0;
  if (act) {
    load_col<C>(v, sm.tile, field_base<C>(f), x);
    if constexpr (FWD) LF::fwd(v, L);
    if constexpr (CTL) {
      if (a.features && wave < C::M) export_energies<C, T>(a, q, f, x, v, L);
      threshold_patch_column<C, T>(a, q, v, x, L);
    } else {
      threshold_column<C, T>(v, x, L, T(a.eps), a.rule);
    }
    if constexpr (!FWD) {
      // Given coefficients: a scaled sum of magnitudes stays finite for any
      // finite column and turns into Inf / NaN with any non-finite element.
      // (After a forward transform the totals carry the same information.)
#pragma unroll
      for (int y = 0; y < C::S; ++y) mag = fma(fabs(v[y]), T(0x1p-64), mag);
    }
    part = column_sample_sum<C, T>(v, x, L);
  }
  if constexpr (!FWD) {
    if (__ballot(!(mag <= max_finite<T>())) != 0ull && lane == 0) {
      atomicOr(&a.ctrl->abort, ABORT_NONFINITE);
      atomicMin(&a.ctrl->abort_epoch, a.epoch);
    }
  }
  totals_partial<C, T>(part, sm);
  LBMZ_MARK(8);

  // Counts: the owned rows by per-lane counts summed over the wave (vector
  // compares only: a ballot per row costs more scalar work than it saves),
  // the shared row by one ballot restricted to the lanes that hold a line.
  // The shared-column wave parks its thresholded coefficients in the ghost
  // buffer (unused from here on), where wave 0 counts them and the field
  // waves store them.
  T* rimc = sm.ghost;   // [field][y]
  const unsigned long long actm = __ballot(act);
  if (wave < C::M) {
    // lanes without a line hold zeros
    int cnt = 0;
#pragma unroll
    for (int y = 0; y < C::P; ++y) cnt += (v[y] != T(0)) ? 1 : 0;
    const int run = __shfl(wave_incl_scan(cnt), 63, 64);
    unsigned long long rowb = 0ull;
    if constexpr (C::RIM) rowb = __ballot(v[C::P] != T(0)) & actm;
    if (lane == 0) {
      sm.core_nnz[wave] = (unsigned)run;
      sm.rowbits[wave] = rowb;
    }
  } else if (C::RIM && wave == C::M && act) {
#pragma unroll
    for (int y = 0; y < C::S; ++y) rimc[f * C::S + y] = v[y];
  }
  __syncthreads();
  LBMZ_MARK(9);

  // Record layouts (lane g of wave 0 for field g), offsets inside the patch
  // by a wave scan, and one allocation for the patch.
  if (wave == 0) {
    unsigned long long mycol = 0ull;
    uint32_t mycorner = 0u;
    if constexpr (C::RIM) {
      const int yy = lane < C::P ? lane : 0;
#pragma unroll
      for (int g = 0; g < C::M; ++g) {
        const unsigned long long cb = __ballot(lane < C::P && rimc[g * C::S + yy] != T(0));
        if (lane == g) mycol = cb;
      }
      if (lane < C::M) mycorner = rimc[lane * C::S + C::P] != T(0) ? 1u : 0u;
    }
    uint32_t rb16 = 0;
    if (lane < C::M) {
      uint32_t nnz = sm.core_nnz[lane];
      if constexpr (C::RIM) {
        nnz += (uint32_t)(__popcll(mycol) + __popcll(sm.rowbits[lane])) + mycorner;
        sm.colbits[lane] = mycol;
        sm.corner[lane] = mycorner;
      }
      const uint32_t ismask = (2u * nnz < 8u * C::W) ? 0u : 1u;
      const uint32_t vb = (nnz * (uint32_t)sizeof(T) + 7u) & ~7u;
      const uint32_t mb = ismask ? 8u * C::W : 2u * nnz;
      rb16 = (vb + mb + 15u) / 16u;
      sm.nnz[lane] = nnz;
      sm.ismask[lane] = ismask;
      sm.vb[lane] = vb;
      sm.rb[lane] = rb16 * 16u;
    }
    const int incl = wave_incl_scan((int)rb16);
    const int total = __shfl(incl, 63, 64);
    if (lane < C::M) sm.rel16[lane] = (uint32_t)(incl - (int)rb16);
    if (lane == 0) {
      const unsigned long long base = atomicAdd(&a.ctrl->top16[a.epoch % 3u], (unsigned long long)total);
      const bool ok = base + (unsigned long long)total <= a.cap16;
      if (!ok) {
        atomicOr(&a.ctrl->abort, ABORT_OVERFLOW);
        atomicMin(&a.ctrl->abort_epoch, a.epoch);
      }
      sm.misc[0] = ok ? 1u : 0u;
      sm.misc[1] = (unsigned)base;
    }
  }
  __syncthreads();
  LBMZ_MARK(10);
  if (!sm.misc[0]) return false;
  const uint32_t base16 = sm.misc[1];
  if (tid < C::M) {
    a.table_out[2 * (q * C::M + tid)] = base16 + sm.rel16[tid];
    a.table_out[2 * (q * C::M + tid) + 1] = sm.nnz[tid] | (sm.ismask[tid] ? MASK_BIT : 0u);
  }

  // Stores: the rank of a kept coefficient is the count of kept ones before
  // it in record order (owned rows, shared column, shared row, corner); in a
  // row, the kept lanes below it (mbcnt).
  if (wave < C::M) {
    // wave-uniform record geometry (scalar registers)
    auto uni = [](uint32_t u) { return (uint32_t)__builtin_amdgcn_readfirstlane((int)u); };
    uint8_t* rec = a.pool_out + 16ull * uni(base16 + sm.rel16[f]);
    T* vals = reinterpret_cast<T*>(rec);
    const bool ismask = uni(sm.ismask[f]) != 0u;
    const uint32_t nnz = uni(sm.nnz[f]);
    const uint32_t vb = uni(sm.vb[f]);
    uint16_t* idx = reinterpret_cast<uint16_t*>(rec + vb);
    unsigned long long myw = 0ull;
    const int run = ismask ? store_owned_rows<C, T, true>(v, actm, rec, nnz, vb, myw)
                           : store_owned_rows<C, T, false>(v, actm, rec, nnz, vb, myw);
    if constexpr (C::RIM) {
      const unsigned long long col = sm.colbits[f];
      const unsigned long long rowb = sm.rowbits[f];
      if (col != 0ull) {
        // shared column, lane = y
        const int yy = lane < C::P ? lane : 0;
        const T c = rimc[f * C::S + yy];
        if (lane < C::P && ((col >> yy) & 1ull)) {
          const int rank = run + (int)__builtin_amdgcn_mbcnt_hi((unsigned)(col >> 32),
                                                                __builtin_amdgcn_mbcnt_lo((unsigned)col, 0u));
          vals[rank] = c;
          if (!ismask) idx[rank] = (uint16_t)(C::P * C::P + lane);
        }
      }
      const int after_col = run + __popcll(col);
      if (act && v[C::P] != T(0)) {
        const int rank = after_col + __popcll(rowb & below(x));
        vals[rank] = v[C::P];
        if (!ismask) idx[rank] = (uint16_t)(C::P * C::P + C::P + x);
      }
      if (lane == 0 && sm.corner[f] != 0u) {
        const int rank = after_col + __popcll(rowb);
        vals[rank] = rimc[f * C::S + C::P];
        if (!ismask) idx[rank] = (uint16_t)(C::P * C::P + 2 * C::P);
      }
    }
    if (ismask && lane < C::CW) reinterpret_cast<unsigned long long*>(rec + vb)[lane] = myw;
  }
  if (tid < C::M) {
    const int g = tid;
    uint8_t* rec = a.pool_out + 16ull * (base16 + sm.rel16[g]);
    if constexpr (C::RIM) {
      if (sm.ismask[g]) {
        unsigned long long r[3];
        rim_join<C>(sm.colbits[g], sm.rowbits[g], sm.corner[g] != 0u, r[0], r[1], r[2]);
        unsigned long long* wds = reinterpret_cast<unsigned long long*>(rec + sm.vb[g]);
#pragma unroll
        for (int j = 0; j < C::W - C::CW; ++j) wds[C::CW + j] = r[j];
      }
    }
    const uint32_t vend = sm.nnz[g] * (uint32_t)sizeof(T);
    if (vend < sm.vb[g]) *reinterpret_cast<uint32_t*>(rec + vend) = 0u;
    const uint32_t mend = sm.vb[g] + (sm.ismask[g] ? 8u * C::W : 2u * sm.nnz[g]);
    for (uint32_t o = mend; o < sm.rb[g]; o += 2) *reinterpret_cast<uint16_t*>(rec + o) = 0;
  }
  totals_finish<C, T, FWD>(a, a.partials_out + (size_t)q * C::M, L, sm);
  LBMZ_MARK(11);
  if constexpr (CTL) {
    if (wave < C::M && act) export_features<C, T>(a, q, f, x, v);
  }

  // S8, column half: inverse of the thresholded column, back to LDS.
  if (act) {
    LF::inv(v, L);
    store_col<C>(v, sm.tile, field_base<C>(f), x);
  }
  __syncthreads();
  return true;
}

}  // namespace lbmz

#include "lbmz_patch_narrow.h"

namespace lbmz {

// ---------------------------------------------------------------------------
// Kernels
// ---------------------------------------------------------------------------

template <class C, class T, int WAV, bool TOT, int VF, bool PREZ = false, class SM>
__device__ __forceinline__ void expand_any(const PatchArgs& a, int q, SM& sm, const ListRegs<C, T>& lr) {
  if constexpr (VF == VF_F32) expand_columns<C, T, WAV, TOT, PREZ>(a, q, sm, lr);
  else expand_columns_q<C, T, WAV, TOT, VF>(a, q, sm);
}

template <class C, class T, int WAV, bool FWD, int VF, bool CTL, class SM>
__device__ __forceinline__ bool compact_any(const PatchArgs& a, int q, SM& sm) {
  if constexpr (VF == VF_F32) return column_compact<C, T, WAV, FWD, CTL>(a, q, sm);
  else return column_compact_q<C, T, WAV, FWD, VF>(a, q, sm);
}

// The loads that start a patch, issued before the barrier that precedes the
// expansion: the index-list entries (float32 records), the ghost values (S3)
// and the offset-table entries; for D2Q9 with float32 records, also the
// zeroing of the fields' owned rows, between the loads and their LDS stores.
template <class C, class T, int SCH, int VF, class SM>
__device__ __forceinline__ void begin_patch(const PatchArgs& a, int q, SM& sm, ListRegs<C, T>& lr) {
  if (tid_of<C>() == 0) sm.samples_only = 1u;   // until the expansion finds a bitmask record or a detail
  if constexpr (VF == VF_F32) prefetch_lists<C, T>(a, q, lr);
  if constexpr (SCH == S_LBM && VF == VF_F32) {
    // The ghost value and the table entry of each thread are loaded into
    // registers; while they are in flight every thread zeroes its share of
    // the fields' owned rows (index-list records scatter into zeroed tiles;
    // the ghost rows outside them are not touched); then the loaded values
    // go to LDS.
    static_assert(4 * 3 * C::S <= C::NT, "one ghost value per thread");
    const int tid = tid_of<C>();
    T gv = T(0);
    T* gd = nullptr;
    if (tid < 4 * 3 * C::S) gd = gather_lbm_at<C, T>(a, q, tid, sm.tile, sm.ghost, gv);
    uint32_t tv = 0u;
    if (tid < 2 * C::M) tv = a.table_in[2 * (size_t)q * C::M + tid];
#pragma unroll
    for (int f = 0; f < C::M; ++f) zero_span<T>(sm.tile + C::Lay::fb(f), C::S * C::RS, tid, C::NT);
    if (gd != nullptr) *gd = gv;
    if (tid < 2 * C::M) sm.te[tid] = tv;
  } else {
    prefetch_table<C>(a, q, sm);
    if constexpr (SCH == S_LBM) gather_lbm<C, T>(a, q, sm.tile, sm.ghost);
    else gather_fv<C, T>(a, q, sm.ghost);
  }
}

// One step (time n -> n + 1) of patch q, S1..S9, after begin_patch and a barrier.
template <class C, class T, int WAV, int SCH, int VF, bool CTL, class SM>
__device__ __forceinline__ void step_one_patch(const PatchArgs& a, int q, SM& sm, const ListRegs<C, T>& lr) {
  LBMZ_MARK(0);
  LBMZ_MARK(14);
  expand_any<C, T, WAV, false, VF, SCH == S_LBM && VF == VF_F32>(a, q, sm, lr);
  LBMZ_MARK(1);
  constexpr int INV = SCH == S_LBM ? ROW_INV_SHIFT : ROW_INV;
  if constexpr (VF == VF_F32 && WAV == W_BL53) {
    if (a.levels == C::LMAX && __builtin_amdgcn_readfirstlane((int)sm.samples_only) != 0)
      row_pass<C, T, WAV, SCH, INV, true>(a, q, sm.tile, sm.ghost);
    else
      row_pass<C, T, WAV, SCH, INV>(a, q, sm.tile, sm.ghost);
  } else {
    row_pass<C, T, WAV, SCH, INV>(a, q, sm.tile, sm.ghost);
  }
  __syncthreads();
  LBMZ_MARK(2);
  if constexpr (SCH == S_LBM) stencil_lbm<C, T>(a, sm.tile);
  else if constexpr (SCH == S_EULER) stencil_euler<C, T>(a, sm.tile, sm.ghost);
  else stencil_fv<C, T>(a, sm.tile, sm.ghost);
  LBMZ_MARK(3);
  row_pass<C, T, WAV, SCH, ROW_FWD>(a, q, sm.tile, sm.ghost);
  __syncthreads();
  LBMZ_MARK(4);
  if (compact_any<C, T, WAV, true, VF, CTL>(a, q, sm)) {
    LBMZ_MARK(5);
    export_rows<C, T, WAV, SCH>(a, q, sm.tile, sm.ghost);
    LBMZ_MARK(6);
  }
}

// Stop if an earlier launch of this batch failed (its input is the last good
// state); a failure inside this launch lets every patch finish so that the
// pool counter ends at the exact size the step needs.  The workgroup that
// resets the next launch's counters is chosen by the caller.
template <class SM>
__device__ __forceinline__ bool step_stops(const PatchArgs& a, bool reset_next, SM& sm) {
  if (threadIdx.x == 0) {
    const bool stop = a.ctrl->abort != 0u && a.ctrl->abort_epoch < a.epoch;
    sm.misc[2] = stop ? 1u : 0u;
    if (!stop && reset_next) {
      a.ctrl->top16[(a.epoch + 1u) % 3u] = 0ull;
      a.ctrl->queue[(a.epoch + 1u) % 3u] = 0u;
    }
  }
  __syncthreads();
  return sm.misc[2] != 0u;
}

// One step of patch blockIdx.x (one workgroup per patch).  CTL: per-patch
// controls or network input export in use (float32 records only).
template <class T, int P, int WAV, int SCH, int VF = VF_F32, bool CTL = false>
__global__ __launch_bounds__((Cfg<T, P, WAV, SCH>::NT)) void patch_step_kernel(PatchArgs a) {
  using C = Cfg<T, P, WAV, SCH>;
  __shared__ Smem<C, T, VF> sm;
  ListRegs<C, T> lr;
  begin_patch<C, T, SCH, VF>(a, blockIdx.x, sm, lr);
  if (step_stops(a, blockIdx.x == 0, sm)) return;
  step_one_patch<C, T, WAV, SCH, VF, CTL>(a, blockIdx.x, sm, lr);
}

// The kernel arguments as a reference into the kernel-argument segment that
// the compiler cannot hoist out of a loop: the persistent kernel re-reads
// them (scalar loads) for every patch instead of holding them in registers
// across the whole loop.
__device__ __forceinline__ const PatchArgs& patch_args_reread() {
  auto kp = __builtin_amdgcn_kernarg_segment_ptr();
  asm volatile("" : "+s"(kp));
  return *(const PatchArgs*)kp;
}

// One step of every patch by a fixed set of resident workgroups that take
// patches from a work queue (an atomic counter) until none is left.
template <class T, int P, int WAV, int SCH, int VF = VF_F32, bool CTL = false>
__global__ __launch_bounds__((Cfg<T, P, WAV, SCH>::NT)) void patch_step_persistent_kernel(PatchArgs a) {
  using C = Cfg<T, P, WAV, SCH, true>;
  __shared__ Smem<C, T, VF> sm;
  if (step_stops(a, blockIdx.x == 0, sm)) return;
  if (threadIdx.x == 0) sm.misc[3] = atomicAdd(&a.ctrl->queue[a.epoch % 3u], 1u);
  __syncthreads();
  for (unsigned it = 0;; ++it) {
    // patch indices alternate between two LDS slots: the next one is taken
    // while this patch's loads are in flight, by the last wave (no line in
    // the passes), into the slot that no wave reads during this patch
    const int q = __builtin_amdgcn_readfirstlane((int)sm.misc[3 + (it & 1u)]);   // uniform: scalar addressing
    if (q >= a.npatch) break;   // every wave reads the same q and leaves together
    const PatchArgs& ap = patch_args_reread();
    ListRegs<C, T> lr;
    begin_patch<C, T, SCH, VF>(ap, q, sm, lr);
    if (threadIdx.x == C::NT - 64) sm.misc[3 + ((it + 1u) & 1u)] = atomicAdd(&ap.ctrl->queue[ap.epoch % 3u], 1u);
    __syncthreads();
    step_one_patch<C, T, WAV, SCH, VF, CTL>(ap, q, sm, lr);
    __syncthreads();
  }
}

// Auxiliary modes (state set-up, store restore, decompression).
template <class T, int P, int WAV, int SCH, int VF = VF_F32>
__global__ __launch_bounds__((Cfg<T, P, WAV, SCH>::NT)) void patch_aux_kernel(PatchArgs a) {
  using C = Cfg<T, P, WAV, SCH>;
  __shared__ Smem<C, T, VF> sm;
  const int q = blockIdx.x;
  int px, py;
  patch_xy(a, q, px, py);
  if (a.mode == AUX_INIT || a.mode == AUX_COEF) {
    if (q == 0 && threadIdx.x == 0) a.ctrl->top16[(a.epoch + 1u) % 3u] = 0ull;
    for (int f = 0; f < C::M; ++f) {
      for (int t = threadIdx.x; t < C::NC; t += C::NT) {
        const int y = t / C::S;
        const int x = t - y * C::S;
        T v;
        if (a.mode == AUX_INIT) {
          const int gx = (px * P + x) % a.n;
          const int gy = (py * P + y) % a.n;
          v = static_cast<const T*>(a.dense_in)[((size_t)f * a.n + gy) * a.n + gx];
        } else {
          v = static_cast<const T*>(a.coef_in)[((size_t)q * C::M + f) * C::NC + t];
        }
        sm.tile[field_base<C>(f) + y * C::RS + x] = v;
      }
    }
    __syncthreads();
    bool ok;
    if (a.mode == AUX_INIT) {
      row_pass<C, T, WAV, SCH, ROW_FWD>(a, q, sm.tile, sm.ghost);
      __syncthreads();
      ok = compact_any<C, T, WAV, true, VF, true>(a, q, sm);
    } else {
      ok = compact_any<C, T, WAV, false, VF, true>(a, q, sm);
    }
    if (!ok) return;
    export_rows<C, T, WAV, SCH>(a, q, sm.tile, sm.ghost);
    return;
  }
  ListRegs<C, T> lr;
  if (threadIdx.x == 0) sm.samples_only = 1u;   // until the expansion finds a bitmask record or a detail
  if constexpr (VF == VF_F32) prefetch_lists<C, T>(a, q, lr);
  prefetch_table<C>(a, q, sm);
  __syncthreads();
  if (a.mode == AUX_RESTORE) {
    expand_any<C, T, WAV, true, VF>(a, q, sm, lr);
    totals_finish<C, T, false>(a, a.partials_out + (size_t)q * C::M, a.levels, sm);
    export_rows<C, T, WAV, SCH>(a, q, sm.tile, sm.ghost);
  } else {
    expand_any<C, T, WAV, false, VF>(a, q, sm, lr);
    row_pass<C, T, WAV, SCH, ROW_INV_DENSE>(a, q, sm.tile, sm.ghost);
  }
}

template <class T, int P, int WAV, int SCH, int VF = VF_F32>
constexpr size_t patch_lds_bytes() {
  return sizeof(Smem<Cfg<T, P, WAV, SCH>, T, VF>);
}

// Operations of one compiled kernel family (see the dispatch of the runtime):
// 0 step (one workgroup per patch), 1 auxiliary kernel, 2 LDS bytes,
// 3 persistent step on `grid` workgroups, 4 / 5 the step / persistent kernel's
// entry (for graph nodes), 6 threads per workgroup.  OP_CTL added to 0, 3, 4
// or 5 selects the step kernels with per-patch controls (float32 records).
template <class T, int P, int WAV, int SCH, int VF>
size_t dispatch_op(int op, const PatchArgs* a, int grid, hipStream_t s, hipError_t* err) {
  using C = Cfg<T, P, WAV, SCH>;
  if (op & OP_CTL) {
    if constexpr (VF == VF_F32) {
      switch (op & ~OP_CTL) {
        case 0:
          hipLaunchKernelGGL((patch_step_kernel<T, P, WAV, SCH, VF, true>), dim3(grid), dim3(C::NT), 0, s, *a);
          *err = hipGetLastError();
          return 0;
        case 3:
          hipLaunchKernelGGL((patch_step_persistent_kernel<T, P, WAV, SCH, VF, true>), dim3(grid), dim3(C::NT), 0,
                             s, *a);
          *err = hipGetLastError();
          return 0;
        case 4:
          return reinterpret_cast<size_t>(reinterpret_cast<const void*>(&patch_step_kernel<T, P, WAV, SCH, VF, true>));
        case 5:
          return reinterpret_cast<size_t>(
              reinterpret_cast<const void*>(&patch_step_persistent_kernel<T, P, WAV, SCH, VF, true>));
        default:
          break;
      }
    }
    *err = hipErrorInvalidValue;
    return 0;
  }
  switch (op) {
    case 0:
      hipLaunchKernelGGL((patch_step_kernel<T, P, WAV, SCH, VF>), dim3(grid), dim3(C::NT), 0, s, *a);
      *err = hipGetLastError();
      return 0;
    case 1:
      hipLaunchKernelGGL((patch_aux_kernel<T, P, WAV, SCH, VF>), dim3(grid), dim3(C::NT), 0, s, *a);
      *err = hipGetLastError();
      return 0;
    case 2:
      return patch_lds_bytes<T, P, WAV, SCH, VF>();
    case 3:
      hipLaunchKernelGGL((patch_step_persistent_kernel<T, P, WAV, SCH, VF>), dim3(grid), dim3(C::NT), 0, s, *a);
      *err = hipGetLastError();
      return 0;
    case 4:
      return reinterpret_cast<size_t>(reinterpret_cast<const void*>(&patch_step_kernel<T, P, WAV, SCH, VF>));
    case 5:
      return reinterpret_cast<size_t>(
          reinterpret_cast<const void*>(&patch_step_persistent_kernel<T, P, WAV, SCH, VF>));
    case 6:
      return (size_t)C::NT;
    default:
      *err = hipErrorInvalidValue;
      return 0;
  }
}

#define LBMZ_CASE_T(T_, P_, W_, S_, V_)                                      \
  if (k.p == P_ && k.wavelet == W_ && k.vf == V_) {                          \
    *out = dispatch_op<T_, P_, W_, S_, V_>(op, a, grid, s, err);             \
    return true;                                                             \
  }

}  // namespace lbmz
