// Fused patch kernels for gfx950: one workgroup owns one patch for the whole
// step and keeps all of its fields in LDS.
//
//   S3  ghost ring: strips the neighbours exported at the end of the previous
//       step (their lossy reconstructions), loaded first so that the loads
//       overlap the decompression;
//   S1  expand the patch's records (values + u16 index list or u64 bitmask)
//       into the LDS tile;
//   S2  inverse wavelet transform: columns (y), then rows (x), coarse to fine;
//   S4  stencil update of every tile node (FV upwind flux sum or D2Q9 pull
//       stream + BGK collision), in place through registers;
//   S5  forward transform: rows, then columns (the tensor 2-D decomposition of
//       Section 2.1), with S6, the hard threshold of Section 2.2, applied in
//       registers at the end of the column pass;
//   S7  compaction: wave64 ballot of the non-zero mask, per-field prefix sums
//       of the word counts, one bump allocation per patch in the output pool,
//       coalesced stores of values and indices or mask words;
//   S8  inverse transform of the thresholded tile (what neighbours and the
//       next step will see) and export of the boundary lines they need;
//   S9  FP64 per-field trapezoid sums of that reconstruction.
//
// Lifting runs one line per thread entirely in registers (the line is read
// from LDS once and written back once per pass); LDS rows use an odd stride so
// that both row-per-lane and column-per-lane access are bank-conflict free.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "lbmz_internal.h"

namespace lbmz {

constexpr int ilog2c(int v) { return v <= 1 ? 0 : 1 + ilog2c(v / 2); }

template <class T, int P, int WAV, int SCH>
struct Cfg {
  static constexpr int S = (WAV == W_BL53) ? P + 1 : P;     // tile nodes per side
  static constexpr int RS = (S & 1) ? S : S + 1;            // LDS row stride (odd)
  static constexpr int M = (SCH == S_LBM) ? 9 : 1;          // fields
  static constexpr int FS = S * RS;                         // LDS field stride
  static constexpr int NC = S * S;                          // coefficients per field
  static constexpr int W = (NC + 63) / 64;                  // mask words per field
  static constexpr int NSLOT = (SCH == S_LBM) ? 3 : M;      // fields crossing one side
  static constexpr int GL = S + 2;                          // ghost strip length, j = -1 .. S
  static constexpr int LO = (WAV == W_BL53) ? 1 : 0;        // first line a neighbour needs
  static constexpr int HI = P - 1;                          // last line a neighbour needs
  static constexpr int NT = (M * S >= 256) ? 1024 : 256;    // threads per workgroup
  static constexpr int NWAVES = NT / 64;
  static constexpr int J = ilog2c(P);
  static constexpr int LMAX = (WAV == W_BL53) ? J - 1 : J;
  static constexpr int NPER = (NC + NT - 1) / NT;           // stencil nodes per thread
  static constexpr int IPW = (M * W + NWAVES - 1) / NWAVES; // mask words per wave
  static constexpr int LPT = (4 * W + NT - 1) / NT;         // index-list entries per thread
  static_assert(W <= 128, "tile too large for the two-word-per-lane scans");
  static_assert(NC <= 65536, "u16 indices");
};

struct FieldInfo {
  uint32_t off16;   // record offset (16-byte units)
  uint32_t nnz;
  uint32_t ismask;
  uint32_t vb;      // bytes of values incl. padding to 8
  uint32_t rel16;   // record offset inside the patch's allocation
  uint32_t rb;      // record bytes
};

// ---------------------------------------------------------------------------
// Small device helpers
// ---------------------------------------------------------------------------

__device__ __forceinline__ int lane_id() { return threadIdx.x & 63; }

__device__ __forceinline__ unsigned mbcnt64(unsigned long long m) {
  return __builtin_amdgcn_mbcnt_hi((unsigned)(m >> 32), __builtin_amdgcn_mbcnt_lo((unsigned)m, 0u));
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

template <class C>
__device__ __forceinline__ int lds_index(int t) {
  if constexpr (C::RS == C::S) {
    return t;
  } else {
    const int y = t / C::S;
    return y * C::RS + (t - y * C::S);
  }
}

// Per-dimension rank of tile index i for an L-level transform: -1 for a sample
// (i a multiple of 2^L), else L - lev with lev = 1 + ctz(i) the detail level.
__device__ __forceinline__ int dim_rank(int i, int L) {
  if ((i & ((1 << L) - 1)) == 0) return -1;
  return L - 1 - __builtin_ctz((unsigned)i);
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
};

// One pass over all lines of all fields.  ROWS: lines along x (row-major in
// LDS); otherwise along y.  THR: apply the hard threshold after a forward
// column pass (the column index is then the x index of every element).
template <class C, class T, int WAV, bool ROWS, bool FWD, bool THR>
__device__ __forceinline__ void lift_pass(T* tile, int L, T eps, int rule) {
  using LF = Lift<T, C::S, WAV, 1, C::LMAX>;
  for (int line = threadIdx.x; line < C::M * C::S; line += C::NT) {
    const int f = line / C::S;
    const int r = line - f * C::S;
    T* base = tile + f * C::FS + (ROWS ? r * C::RS : r);
    constexpr int STR = ROWS ? 1 : C::RS;
    T v[C::S];
#pragma unroll
    for (int i = 0; i < C::S; ++i) v[i] = base[i * STR];
    if constexpr (FWD) LF::fwd(v, L); else LF::inv(v, L);
    if constexpr (THR) {
      const int rx = dim_rank(r, L);
#pragma unroll
      for (int i = 0; i < C::S; ++i) {
        const T thr = thr_of<T>(rx, dim_rank(i, L), eps, rule);
        v[i] = (fabs(v[i]) < thr) ? T(0) : v[i];
      }
    }
#pragma unroll
    for (int i = 0; i < C::S; ++i) base[i * STR] = v[i];
  }
}

template <class C, class T, int WAV>
__device__ __forceinline__ void inverse_transform(T* tile, int L) {
  lift_pass<C, T, WAV, false, false, false>(tile, L, T(0), 0);
  __syncthreads();
  lift_pass<C, T, WAV, true, false, false>(tile, L, T(0), 0);
  __syncthreads();
}

template <class C, class T, int WAV>
__device__ __forceinline__ void forward_transform_threshold(T* tile, int L, T eps, int rule) {
  lift_pass<C, T, WAV, true, true, false>(tile, L, eps, rule);
  __syncthreads();
  lift_pass<C, T, WAV, false, true, true>(tile, L, eps, rule);
  __syncthreads();
}

// Threshold of given coefficients (no transform), same decision as above.
template <class C, class T>
__device__ __forceinline__ void threshold_pass(T* tile, int L, T eps, int rule) {
  for (int f = 0; f < C::M; ++f) {
    for (int t = threadIdx.x; t < C::NC; t += C::NT) {
      const int y = t / C::S;
      const int x = t - y * C::S;
      const T thr = thr_of<T>(dim_rank(x, L), dim_rank(y, L), eps, rule);
      T& c = tile[f * C::FS + y * C::RS + x];
      c = (fabs(c) < thr) ? T(0) : c;
    }
  }
  __syncthreads();
}

// ---------------------------------------------------------------------------
// Halo strips
// ---------------------------------------------------------------------------
// Ghost sides: 0 = W (x = -1), 1 = E (x = S), 2 = S (y = -1), 3 = N (y = S).
// halo[q][side][slot][S] holds the line of patch q that fills the ghost strip
// `side` of the neighbour on the opposite side: side W <- line x = HI of the
// west neighbour, E <- line x = LO of the east one, S <- line y = HI of the
// south one, N <- line y = LO of the north one.  For D2Q9 only the three
// populations streaming into the neighbour are kept (slots in numbering
// order); for FV every field is kept.

struct D2Q9 {
  static constexpr int CX[9] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
  static constexpr int CY[9] = {0, 0, 1, 0, -1, 1, 1, -1, -1};
  // populations entering through each ghost side
  static constexpr int SIDE_POP[4][3] = {{1, 5, 8}, {3, 6, 7}, {2, 5, 6}, {4, 7, 8}};
};

template <int SCH>
__device__ __forceinline__ int side_field(int side, int slot) {
  if constexpr (SCH == S_LBM) {
    constexpr int tab[12] = {1, 5, 8, 3, 6, 7, 2, 5, 6, 4, 7, 8};
    return tab[side * 3 + slot];
  } else {
    (void)side;
    return slot;
  }
}

// Slot of population i in ghost side `side` (compile-time i in the stencil).
__host__ __device__ constexpr int pop_slot(int side, int i) {
  return D2Q9::SIDE_POP[side][0] == i ? 0 : D2Q9::SIDE_POP[side][1] == i ? 1
       : D2Q9::SIDE_POP[side][2] == i ? 2 : 0;
}

template <class C, class T, int SCH>
__device__ __forceinline__ void gather_ghosts(const PatchArgs& a, int q, T* ghost) {
  const T* h = static_cast<const T*>(a.halo_in);
  const int px = q % a.npx;
  const int py = q / a.npx;
  for (int k = threadIdx.x; k < 4 * C::NSLOT * C::GL; k += C::NT) {
    const int side = k / (C::NSLOT * C::GL);
    const int rem = k - side * (C::NSLOT * C::GL);
    const int slot = rem / C::GL;
    const int j = rem - slot * C::GL - 1;
    int nx = px, ny = py, src = j;
    if (side < 2) {
      nx = px + (side == 0 ? -1 : 1);
      if (j < 0) { ny = py - 1; src = C::HI; }
      else if (j >= C::S) { ny = py + 1; src = C::LO; }
    } else {
      ny = py + (side == 2 ? -1 : 1);
      if (j < 0 || j >= C::S) continue;   // corners come from the W / E strips
    }
    nx = (nx + a.npx) % a.npx;
    ny = (ny + a.npx) % a.npx;
    const int nb = nx + a.npx * ny;
    ghost[k] = h[((size_t)(nb * 4 + side) * C::NSLOT + slot) * C::S + src];
  }
}

template <class C, class T, int SCH>
__device__ __forceinline__ void export_halo(const PatchArgs& a, int q, const T* tile) {
  T* h = static_cast<T*>(a.halo_out);
  for (int k = threadIdx.x; k < 4 * C::NSLOT * C::S; k += C::NT) {
    const int side = k / (C::NSLOT * C::S);
    const int rem = k - side * (C::NSLOT * C::S);
    const int slot = rem / C::S;
    const int j = rem - slot * C::S;
    const int f = side_field<SCH>(side, slot);
    int x, y;
    if (side == 0) { x = C::HI; y = j; }
    else if (side == 1) { x = C::LO; y = j; }
    else if (side == 2) { x = j; y = C::HI; }
    else { x = j; y = C::LO; }
    h[((size_t)(q * 4 + side) * C::NSLOT + slot) * C::S + j] = tile[f * C::FS + y * C::RS + x];
  }
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

template <class C, class T>
__device__ __forceinline__ const T* pop_src(const T* tile, const T* ghost, int i, int sx, int sy,
                                            int ws, int es, int ss, int ns) {
  if ((unsigned)sx < (unsigned)C::S && (unsigned)sy < (unsigned)C::S)
    return tile + i * C::FS + sy * C::RS + sx;
  if (sx < 0) return ghost + (0 * C::NSLOT + ws) * C::GL + sy + 1;
  if (sx >= C::S) return ghost + (1 * C::NSLOT + es) * C::GL + sy + 1;
  if (sy < 0) return ghost + (2 * C::NSLOT + ss) * C::GL + sx + 1;
  return ghost + (3 * C::NSLOT + ns) * C::GL + sx + 1;
}

template <class C, class T>
__device__ __forceinline__ void stencil_lbm(const PatchArgs& a, T* tile, const T* ghost) {
  const T omega = T(a.omega);
  T res[C::NPER][9];
#pragma unroll
  for (int k = 0; k < C::NPER; ++k) {
    const int t = threadIdx.x + k * C::NT;
    if (t < C::NC) {
      const int y = t / C::S;
      const int x = t - y * C::S;
      T fin[9];
#pragma unroll
      for (int i = 0; i < 9; ++i)
        fin[i] = *pop_src<C, T>(tile, ghost, i, x - D2Q9::CX[i], y - D2Q9::CY[i],
                               pop_slot(0, i), pop_slot(1, i), pop_slot(2, i), pop_slot(3, i));
      d2q9_collide<T>(fin, omega, res[k]);
    }
  }
  __syncthreads();
#pragma unroll
  for (int k = 0; k < C::NPER; ++k) {
    const int t = threadIdx.x + k * C::NT;
    if (t < C::NC) {
      const int y = t / C::S;
      const int x = t - y * C::S;
#pragma unroll
      for (int i = 0; i < 9; ++i) tile[i * C::FS + y * C::RS + x] = res[k][i];
    }
  }
  __syncthreads();
}

// Finite-volume update of equation "vf_scheme" in the order of the transport
// listing: W' = W, then W' -= dt/h * (W max(a.N^k,0) + W_k min(a.N^k,0)) for
// N^0..3 = +x, -x, +y, -y.
template <class C, class T>
__device__ __forceinline__ void stencil_fv(const PatchArgs& a, T* tile, const T* ghost) {
  const T r = T(a.dt_over_h);
  const T cp0 = T(a.cp[0]), cp1 = T(a.cp[1]), cp2 = T(a.cp[2]), cp3 = T(a.cp[3]);
  const T cm0 = T(a.cm[0]), cm1 = T(a.cm[1]), cm2 = T(a.cm[2]), cm3 = T(a.cm[3]);
  T res[C::M][C::NPER];
#pragma unroll
  for (int f = 0; f < C::M; ++f) {
    const T* tf = tile + f * C::FS;
#pragma unroll
    for (int k = 0; k < C::NPER; ++k) {
      const int t = threadIdx.x + k * C::NT;
      if (t < C::NC) {
        const int y = t / C::S;
        const int x = t - y * C::S;
        const T w = tf[y * C::RS + x];
        const T we = (x + 1 < C::S) ? tf[y * C::RS + x + 1] : ghost[(1 * C::NSLOT + f) * C::GL + y + 1];
        const T ww = (x >= 1) ? tf[y * C::RS + x - 1] : ghost[(0 * C::NSLOT + f) * C::GL + y + 1];
        const T wn = (y + 1 < C::S) ? tf[(y + 1) * C::RS + x] : ghost[(3 * C::NSLOT + f) * C::GL + x + 1];
        const T wsd = (y >= 1) ? tf[(y - 1) * C::RS + x] : ghost[(2 * C::NSLOT + f) * C::GL + x + 1];
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
      const int t = threadIdx.x + k * C::NT;
      if (t < C::NC) {
        const int y = t / C::S;
        tile[f * C::FS + y * C::RS + (t - y * C::S)] = res[f][k];
      }
    }
  }
  __syncthreads();
}

// ---------------------------------------------------------------------------
// S1: expand records into the LDS tile
// ---------------------------------------------------------------------------
// Two rounds of global loads: the offset-table entries, then (in parallel)
// the mask words and the contiguous values.  Values of bitmask records are
// staged at the front of their field's tile, read back at their ranks into
// registers, and written to their positions after a barrier.

template <class C, class T>
__device__ __forceinline__ void expand(const uint8_t* pool, const uint32_t* table, int q, T* tile,
                                       FieldInfo* fi, uint16_t* wpre, unsigned long long* words) {
  const int tid = threadIdx.x;
  const int lane = lane_id();
  const int wave = tid >> 6;
  if (tid < C::M) {
    const uint32_t off16 = table[2 * (q * C::M + tid)];
    const uint32_t word = table[2 * (q * C::M + tid) + 1];
    const uint32_t nnz = word & ~MASK_BIT;
    fi[tid].off16 = off16;
    fi[tid].nnz = nnz;
    fi[tid].ismask = word >> 31;
    fi[tid].vb = (nnz * (uint32_t)sizeof(T) + 7u) & ~7u;
  }
  __syncthreads();

  // Round 2: words (+ prefix scan), staged values, index-list entries.
  for (int f = wave; f < C::M; f += C::NWAVES) {
    if (!fi[f].ismask) continue;
    const unsigned long long* wsrc =
        reinterpret_cast<const unsigned long long*>(pool + 16ull * fi[f].off16 + fi[f].vb);
    const unsigned long long w0 = lane < C::W ? wsrc[lane] : 0ull;
    const unsigned long long w1 = (64 + lane) < C::W ? wsrc[64 + lane] : 0ull;
    const int c0 = __popcll(w0);
    const int c1 = __popcll(w1);
    const int i0 = wave_incl_scan(c0);
    const int tot0 = __shfl(i0, 63, 64);
    const int i1 = wave_incl_scan(c1);
    if (lane < C::W) { wpre[f * C::W + lane] = (uint16_t)(i0 - c0); words[f * C::W + lane] = w0; }
    if (64 + lane < C::W) {
      wpre[f * C::W + 64 + lane] = (uint16_t)(tot0 + i1 - c1);
      words[f * C::W + 64 + lane] = w1;
    }
  }
  T lv[C::M][C::LPT];
  int li[C::M][C::LPT];
#pragma unroll
  for (int f = 0; f < C::M; ++f) {
    const uint8_t* rec = pool + 16ull * fi[f].off16;
    const T* vals = reinterpret_cast<const T*>(rec);
    const uint32_t nnz = fi[f].nnz;
    if (fi[f].ismask) {
      for (int k = tid; k < (int)nnz; k += C::NT) tile[f * C::FS + k] = vals[k];
#pragma unroll
      for (int u = 0; u < C::LPT; ++u) li[f][u] = -1;
    } else {
      const uint16_t* idx = reinterpret_cast<const uint16_t*>(rec + fi[f].vb);
#pragma unroll
      for (int u = 0; u < C::LPT; ++u) {
        const int k = tid + u * C::NT;
        li[f][u] = -1;
        if (k < (int)nnz) { li[f][u] = idx[k]; lv[f][u] = vals[k]; }
      }
    }
  }
  __syncthreads();

  // Round 3 (LDS only): staged values -> registers, then tile positions.
  T vv[C::IPW];
#pragma unroll
  for (int u = 0; u < C::IPW; ++u) {
    const int item = wave + u * C::NWAVES;
    vv[u] = T(0);
    if (item < C::M * C::W) {
      const int f = item / C::W;
      if (fi[f].ismask) {
        const unsigned long long w = words[item];
        if ((w >> lane) & 1ull) vv[u] = tile[f * C::FS + wpre[item] + mbcnt64(w)];
      }
    }
  }
  __syncthreads();
#pragma unroll
  for (int u = 0; u < C::IPW; ++u) {
    const int item = wave + u * C::NWAVES;
    if (item < C::M * C::W) {
      const int f = item / C::W;
      const int t = (item - f * C::W) * 64 + lane;
      if (fi[f].ismask && t < C::NC) tile[f * C::FS + lds_index<C>(t)] = vv[u];
    }
  }
#pragma unroll
  for (int f = 0; f < C::M; ++f) {
    if (!fi[f].ismask) {
      for (int t = tid; t < C::NC; t += C::NT) tile[f * C::FS + lds_index<C>(t)] = T(0);
    }
  }
  __syncthreads();
#pragma unroll
  for (int f = 0; f < C::M; ++f) {
#pragma unroll
    for (int u = 0; u < C::LPT; ++u) {
      const int t = li[f][u];
      if (t >= 0 && t < C::NC) tile[f * C::FS + lds_index<C>(t)] = lv[f][u];
    }
  }
  __syncthreads();
}

// ---------------------------------------------------------------------------
// S7: compaction into the output pool
// ---------------------------------------------------------------------------
// Returns false (uniformly) when the pool overflowed; the records are then not
// written and the host replays the step with a larger pool.

template <class C, class T>
__device__ __forceinline__ bool compact(const PatchArgs& a, int q, const T* tile, FieldInfo* fi,
                                        uint16_t* wcnt, unsigned* misc) {
  const int tid = threadIdx.x;
  const int lane = lane_id();
  const int wave = tid >> 6;
  bool bad = false;
  for (int item = wave; item < C::M * C::W; item += C::NWAVES) {
    const int f = item / C::W;
    const int t = (item - f * C::W) * 64 + lane;
    const T v = (t < C::NC) ? tile[f * C::FS + lds_index<C>(t)] : T(0);
    bad |= !(fabs(v) <= max_finite<T>());
    const unsigned long long b = __ballot(v != T(0));
    if (lane == 0) wcnt[item] = (uint16_t)__popcll(b);
  }
  if (__ballot(bad) != 0ull && lane == 0) {
    atomicOr(&a.ctrl->abort, ABORT_NONFINITE);
    atomicMin(&a.ctrl->abort_epoch, a.epoch);
  }
  __syncthreads();
  for (int f = wave; f < C::M; f += C::NWAVES) {
    const int c0 = lane < C::W ? (int)wcnt[f * C::W + lane] : 0;
    const int c1 = (64 + lane) < C::W ? (int)wcnt[f * C::W + 64 + lane] : 0;
    const int i0 = wave_incl_scan(c0);
    const int tot0 = __shfl(i0, 63, 64);
    const int i1 = wave_incl_scan(c1);
    const int tot1 = __shfl(i1, 63, 64);
    if (lane < C::W) wcnt[f * C::W + lane] = (uint16_t)(i0 - c0);
    if (64 + lane < C::W) wcnt[f * C::W + 64 + lane] = (uint16_t)(tot0 + i1 - c1);
    if (lane == 0) fi[f].nnz = (uint32_t)(tot0 + tot1);
  }
  __syncthreads();
  if (tid == 0) {
    uint32_t acc16 = 0;
    for (int f = 0; f < C::M; ++f) {
      const uint32_t nnz = fi[f].nnz;
      const uint32_t ismask = (2u * nnz < 8u * C::W) ? 0u : 1u;
      const uint32_t vb = (nnz * (uint32_t)sizeof(T) + 7u) & ~7u;
      const uint32_t mb = ismask ? 8u * C::W : 2u * nnz;
      const uint32_t rb16 = (vb + mb + 15u) / 16u;
      fi[f].ismask = ismask;
      fi[f].vb = vb;
      fi[f].rel16 = acc16;
      fi[f].rb = rb16 * 16u;
      acc16 += rb16;
    }
    const unsigned long long base =
        atomicAdd(&a.ctrl->top16[a.epoch % 3u], (unsigned long long)acc16);
    const bool ok = base + acc16 <= a.cap16;
    if (!ok) {
      atomicOr(&a.ctrl->abort, ABORT_OVERFLOW);
      atomicMin(&a.ctrl->abort_epoch, a.epoch);
    }
    misc[0] = ok ? 1u : 0u;
    misc[1] = (unsigned)base;
  }
  __syncthreads();
  if (!misc[0]) return false;
  const uint32_t base16 = misc[1];
  if (tid < C::M) {
    a.table_out[2 * (q * C::M + tid)] = base16 + fi[tid].rel16;
    a.table_out[2 * (q * C::M + tid) + 1] = fi[tid].nnz | (fi[tid].ismask ? MASK_BIT : 0u);
  }
  for (int item = wave; item < C::M * C::W; item += C::NWAVES) {
    const int f = item / C::W;
    const int wd = item - f * C::W;
    const int t = wd * 64 + lane;
    const T v = (t < C::NC) ? tile[f * C::FS + lds_index<C>(t)] : T(0);
    const bool keep = v != T(0);
    const unsigned long long b = __ballot(keep);
    uint8_t* rec = a.pool_out + 16ull * (base16 + fi[f].rel16);
    const uint32_t rank = wcnt[item] + mbcnt64(b);
    if (keep) reinterpret_cast<T*>(rec)[rank] = v;
    if (fi[f].ismask) {
      if (lane == 0) reinterpret_cast<unsigned long long*>(rec + fi[f].vb)[wd] = b;
    } else if (keep) {
      reinterpret_cast<uint16_t*>(rec + fi[f].vb)[rank] = (uint16_t)t;
    }
  }
  if (tid < C::M) {
    uint8_t* rec = a.pool_out + 16ull * (base16 + fi[tid].rel16);
    const uint32_t vend = fi[tid].nnz * (uint32_t)sizeof(T);
    if (vend < fi[tid].vb) *reinterpret_cast<uint32_t*>(rec + vend) = 0u;
    const uint32_t mend = fi[tid].vb + (fi[tid].ismask ? 8u * C::W : 2u * fi[tid].nnz);
    for (uint32_t o = mend; o < fi[tid].rb; o += 2) *reinterpret_cast<uint16_t*>(rec + o) = 0;
  }
  return true;
}

// ---------------------------------------------------------------------------
// S9: FP64 trapezoid sums per field (fixed reduction order)
// ---------------------------------------------------------------------------

template <class C, class T, int WAV>
__device__ __forceinline__ void field_totals(double* out, const T* tile, double* red) {
  const int tid = threadIdx.x;
  const int lane = lane_id();
  const int wave = tid >> 6;
  double acc[C::M];
#pragma unroll
  for (int f = 0; f < C::M; ++f) acc[f] = 0.0;
  for (int t = tid; t < C::NC; t += C::NT) {
    const int y = t / C::S;
    const int x = t - y * C::S;
    double w = 1.0;
    if constexpr (WAV == W_BL53) {
      if (x == 0 || x == C::S - 1) w *= 0.5;
      if (y == 0 || y == C::S - 1) w *= 0.5;
    }
#pragma unroll
    for (int f = 0; f < C::M; ++f) acc[f] += w * (double)tile[f * C::FS + y * C::RS + x];
  }
#pragma unroll
  for (int f = 0; f < C::M; ++f) {
    double v = acc[f];
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) v += __shfl_xor(v, d, 64);
    if (lane == 0) red[wave * C::M + f] = v;
  }
  __syncthreads();
  if (tid < C::M) {
    double s = 0.0;
    for (int w = 0; w < C::NWAVES; ++w) s += red[w * C::M + tid];
    out[tid] = s;
  }
}

// ---------------------------------------------------------------------------
// Kernels
// ---------------------------------------------------------------------------

// Optional per-phase wall-clock marks of the step kernel (profiling builds
// compiled with -DLBMZ_PHASE_CLOCK; the product build has none).
#ifdef LBMZ_PHASE_CLOCK
static __device__ unsigned long long lbmz_phase_clock[4096 * 16];
#define LBMZ_MARK(k)                                                                  \
  do {                                                                                \
    if (threadIdx.x == 0 && blockIdx.x < 4096) lbmz_phase_clock[blockIdx.x * 16 + (k)] = wall_clock64(); \
  } while (0)
#else
#define LBMZ_MARK(k) \
  do {               \
  } while (0)
#endif

#define LBMZ_PATCH_SHARED(C, T)                                   \
  __shared__ T s_tile[C::M * C::FS];                              \
  __shared__ T s_ghost[4 * C::NSLOT * C::GL];                     \
  __shared__ uint16_t s_w[C::M * C::W];                           \
  __shared__ unsigned long long s_words[C::M * C::W];             \
  __shared__ FieldInfo s_fi[C::M];                                \
  __shared__ double s_red[C::NWAVES * C::M];                      \
  __shared__ unsigned s_misc[4];

// One step (time n -> n + 1) of one patch: S3, S1, S2, S4, S5+S6, S7, S8, S9.
template <class T, int P, int WAV, int SCH>
__global__ __launch_bounds__((Cfg<T, P, WAV, SCH>::NT)) void patch_step_kernel(PatchArgs a) {
  using C = Cfg<T, P, WAV, SCH>;
  LBMZ_PATCH_SHARED(C, T)
  const int q = blockIdx.x;
  if (threadIdx.x == 0) {
    // Stop if an earlier launch of this batch failed (its input is the last
    // good state); a failure inside this launch lets every patch finish so
    // that the pool counter ends at the exact size the step needs.
    const bool stop = a.ctrl->abort != 0u && a.ctrl->abort_epoch < a.epoch;
    s_misc[2] = stop ? 1u : 0u;
    if (!stop && q == 0) a.ctrl->top16[(a.epoch + 1u) % 3u] = 0ull;
  }
  __syncthreads();
  if (s_misc[2] != 0u) return;
  LBMZ_MARK(0);
  gather_ghosts<C, T, SCH>(a, q, s_ghost);
  expand<C, T>(a.pool_in, a.table_in, q, s_tile, s_fi, s_w, s_words);
  LBMZ_MARK(1);
  inverse_transform<C, T, WAV>(s_tile, a.levels);
  LBMZ_MARK(2);
  if constexpr (SCH == S_LBM) stencil_lbm<C, T>(a, s_tile, s_ghost);
  else stencil_fv<C, T>(a, s_tile, s_ghost);
  LBMZ_MARK(3);
  forward_transform_threshold<C, T, WAV>(s_tile, a.levels, T(a.eps), a.rule);
  LBMZ_MARK(4);
  if (!compact<C, T>(a, q, s_tile, s_fi, s_w, s_misc)) return;
  __syncthreads();
  LBMZ_MARK(5);
  inverse_transform<C, T, WAV>(s_tile, a.levels);
  LBMZ_MARK(6);
  export_halo<C, T, SCH>(a, q, s_tile);
  field_totals<C, T, WAV>(a.partials_out + (size_t)q * C::M, s_tile, s_red);
  LBMZ_MARK(7);
}

// Auxiliary modes (state set-up, store restore, decompression).
template <class T, int P, int WAV, int SCH>
__global__ __launch_bounds__((Cfg<T, P, WAV, SCH>::NT)) void patch_aux_kernel(PatchArgs a) {
  using C = Cfg<T, P, WAV, SCH>;
  LBMZ_PATCH_SHARED(C, T)
  const int q = blockIdx.x;
  const int px = q % a.npx;
  const int py = q / a.npx;
  constexpr int pp = P;   // owned nodes per side
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
        s_tile[f * C::FS + y * C::RS + x] = v;
      }
    }
    __syncthreads();
    if (a.mode == AUX_INIT) forward_transform_threshold<C, T, WAV>(s_tile, a.levels, T(a.eps), a.rule);
    else threshold_pass<C, T>(s_tile, a.levels, T(a.eps), a.rule);
    if (!compact<C, T>(a, q, s_tile, s_fi, s_w, s_misc)) return;
    __syncthreads();
    inverse_transform<C, T, WAV>(s_tile, a.levels);
    export_halo<C, T, SCH>(a, q, s_tile);
    field_totals<C, T, WAV>(a.partials_out + (size_t)q * C::M, s_tile, s_red);
    return;
  }
  expand<C, T>(a.pool_in, a.table_in, q, s_tile, s_fi, s_w, s_words);
  inverse_transform<C, T, WAV>(s_tile, a.levels);
  if (a.mode == AUX_RESTORE) {
    export_halo<C, T, SCH>(a, q, s_tile);
    field_totals<C, T, WAV>(a.partials_out + (size_t)q * C::M, s_tile, s_red);
  } else {
    T* out = static_cast<T*>(a.dense_out);
    for (int f = 0; f < C::M; ++f) {
      for (int t = threadIdx.x; t < pp * pp; t += C::NT) {
        const int y = t / pp;
        const int x = t - y * pp;
        out[((size_t)f * a.n + (py * P + y)) * a.n + px * P + x] = s_tile[f * C::FS + y * C::RS + x];
      }
    }
  }
}

template <class T, int P, int WAV, int SCH>
hipError_t launch_patch_kernels(bool step, const PatchArgs& a, int npatch, hipStream_t s) {
  using C = Cfg<T, P, WAV, SCH>;
  if (step)
    hipLaunchKernelGGL((patch_step_kernel<T, P, WAV, SCH>), dim3(npatch), dim3(C::NT), 0, s, a);
  else
    hipLaunchKernelGGL((patch_aux_kernel<T, P, WAV, SCH>), dim3(npatch), dim3(C::NT), 0, s, a);
  return hipGetLastError();
}

template <class T, int P, int WAV, int SCH>
constexpr size_t patch_lds_bytes() {
  using C = Cfg<T, P, WAV, SCH>;
  return sizeof(T) * (C::M * C::FS + 4 * C::NSLOT * C::GL) + 2 * C::M * C::W + 8 * C::M * C::W +
         sizeof(FieldInfo) * C::M + 8 * C::NWAVES * C::M + 16;
}

}  // namespace lbmz
