// Reduced-precision records: float32 samples, binary16 or OCP E4M3 details
// with one power-of-two scale per subband (included by lbmz_patch_kernel.h).
//
// Layout of one (patch, field) record in a narrow format (little-endian):
//   u64 OCC (bit b: subband b = cy * (L + 1) + cx holds a kept detail; with
//   the bounded E4M3 format bit 63 marks a record of E4M3 codes, a record
//   without it holds binary16 codes),
//   one float32 scale 2^k per set bit of OCC (increasing b), pad to 8;
//   float32 samples of every sample position, slot (y >> L) * SC + (x >> L)
//   with SC samples per side, pad to 8;
//   the kept details' codes in record order, pad to 8;
//   u16 record indices of the kept details, or W u64 mask words, pad to 16.
// The offset-table count is the number of kept details.  The samples carry
// the tile's mass (equation "conservation": the trapezoid mass of a
// reconstructed tile is 4^L times the coarse trapezoid mass of its samples),
// so storing them exactly keeps the mass whatever the quantisation does.
#pragma once

namespace lbmz {

template <int VF>
struct VFmt;

// IEEE binary16, round to nearest even (the hardware conversion).
template <>
struct VFmt<VF_F16> {
  static constexpr int BYTES = 2;
  static constexpr float MAXV = 65504.0f;
  __device__ static uint32_t enc(float x) {
    const _Float16 h = (_Float16)x;
    return (uint32_t)__builtin_bit_cast(uint16_t, h);
  }
  __device__ static float dec(uint32_t c) { return (float)__builtin_bit_cast(_Float16, (uint16_t)c); }
};

// OCP E4M3 (FN): sign, 4 exponent bits with bias 7, 3 mantissa bits,
// subnormals at exponent 0, largest finite 448.  Encoded from the float32
// bits with round to nearest even; callers keep |x| <= 448.
template <>
struct VFmt<VF_E4M3> {
  static constexpr int BYTES = 1;
  static constexpr float MAXV = 448.0f;
  __device__ static uint32_t enc(float x) {
    const uint32_t bits = __float_as_uint(x);
    const uint32_t sign = (bits >> 24) & 0x80u;
    const float a = fabsf(x);
    uint32_t code;
    if (a < 0x1p-6f) {
      // zero and the subnormal range: multiples of 2^-9 (code 8 is 2^-6)
      code = (uint32_t)__float2int_rn(a * 512.0f);
    } else {
      const uint32_t ab = __float_as_uint(a);
      const uint32_t r = ab + 0x7FFFFu + ((ab >> 20) & 1u);   // keep 3 mantissa bits, ties to even
      code = (r >> 20) - (120u << 3);                           // exponent bias 127 -> 7
    }
    return sign | code;
  }
  __device__ static float dec(uint32_t c) {
    const uint32_t e = (c >> 3) & 15u;
    const uint32_t m = c & 7u;
    const float a = (e == 0u) ? (float)m * 0x1p-9f : __uint_as_float(((e + 120u) << 23) | (m << 20));
    return (c & 0x80u) ? -a : a;
  }
};

// Class of one index of a dimension: 0 for a sample, else its detail level (1 = finest).
__device__ __forceinline__ int idx_class(int i, int L) {
  return (i & ((1 << L) - 1)) == 0 ? 0 : __builtin_ctz((unsigned)i) + 1;
}

// Scale exponent of a subband: the smallest k with m <= MAXV 2^k, at least -126.
template <int VF>
__device__ __forceinline__ int scale_exp(float m) {
  const float mx = VFmt<VF>::MAXV;
  int k = ilogbf(m) - ilogbf(mx);
  if (m > ldexpf(mx, k)) ++k;
  if (m <= ldexpf(mx, k - 1)) --k;
  return k < -126 ? -126 : k;
}

// Codes of one record: e4 selects E4M3 (1 byte), else binary16 (2 bytes).
// For the fixed formats e4 is a compile-time constant (fixed_e4) and the
// selection folds away; the bounded format decides it per record.
template <int VF>
__device__ __forceinline__ constexpr bool fixed_e4() { return VF == VF_E4M3; }

__device__ __forceinline__ uint32_t q_enc(bool e4, float c, int k) {
  const float x = ldexpf(c, -k);
  return e4 ? VFmt<VF_E4M3>::enc(x) : VFmt<VF_F16>::enc(x);
}
__device__ __forceinline__ float q_dec(bool e4, uint32_t code, int k) {
  return ldexpf(e4 ? VFmt<VF_E4M3>::dec(code) : VFmt<VF_F16>::dec(code), k);
}
__device__ __forceinline__ void q_store(bool e4, uint8_t* base, int i, uint32_t code) {
  if (e4) base[i] = (uint8_t)code;
  else reinterpret_cast<uint16_t*>(base)[i] = (uint16_t)code;
}
__device__ __forceinline__ uint32_t q_load(bool e4, const uint8_t* base, int i) {
  return e4 ? (uint32_t)base[i] : (uint32_t)reinterpret_cast<const uint16_t*>(base)[i];
}

constexpr unsigned long long OCC_E4M3 = 1ull << 63;   // bounded format: an E4M3 record

// Bounded E4M3: a kept detail c of a subband with largest kept magnitude m
// and E4M3 scale 2^k reads back within max(2^-4 |c|, 2^(k-10)) (half a unit
// of the 3-bit mantissa in the normal range, half the subnormal spacing
// below it).  The record may use E4M3 when that bound at m is at most half
// of the subband's threshold thr (exact float32 arithmetic: powers of two).
__device__ __forceinline__ bool e4m3_bounded(float m, float thr) {
  const int k = scale_exp<VF_E4M3>(m);
  const float bound = fmaxf(ldexpf(m, -4), ldexpf(1.0f, k - 10));
  return bound <= 0.5f * thr;
}

__device__ __forceinline__ void zero_bytes(uint8_t* p, uint32_t from, uint32_t to) {
  for (uint32_t o = from; o < to; ++o) p[o] = 0;
}

// Position of the set bit of rank r (0-based) in w.
__device__ __forceinline__ int select_bit(unsigned long long w, int r) {
  int pos = 0;
#pragma unroll
  for (int width = 32; width >= 1; width >>= 1) {
    const unsigned long long low = (width == 64) ? ~0ull : ((1ull << width) - 1ull);
    const int c = __popcll(w & low);
    if (r >= c) {
      r -= c;
      w >>= width;
      pos += width;
    }
  }
  return pos;
}

// ---------------------------------------------------------------------------
// S5 (column half) + S6 + S7 + S9 + S8 (column half) for a narrow format
// ---------------------------------------------------------------------------
template <class C, class T, int WAV, bool FWD, int VF, class SM>
__device__ __forceinline__ bool column_compact_q(const PatchArgs& a, int q, SM& sm) {
  static_assert(sizeof(T) == 4, "narrow formats store float32 coefficients");
  static_assert(sizeof(sm.ghost) >= sizeof(T) * C::M * C::S, "shared-column staging does not fit");
  using LF = Lift<T, C::S, WAV, 1, C::LMAX>;
  const int tid = tid_of<C>();
  const int lane = lane_of<C>();
  const int wave = wave_of<C>();
  const int L = a.levels;
  const int L1 = L + 1;
  const int lmask = (1 << L) - 1;
  const int SC = ((C::S - 1) >> L) + 1;   // samples per side
  const int NS = SC * SC;
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
    threshold_column<C, T>(v, x, L, T(a.eps), a.rule);
    if constexpr (!FWD) {
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

  // Largest kept magnitude per y class of this line; index ctz(y) + 1 is a
  // compile-time constant, the classes above L are the sample rows.
  const int cx = idx_class(x, L);
  float mk[C::J + 2];
#pragma unroll
  for (int k = 0; k < C::J + 2; ++k) mk[k] = 0.0f;
#pragma unroll
  for (int y = 0; y < C::S; ++y) {
    const int k = (y == 0) ? C::J + 1 : __builtin_ctz((unsigned)y) + 1;
    mk[k] = fmaxf(mk[k], fabsf(v[y]));
  }
  float mc[C::LMAX + 1];
  mc[0] = 0.0f;
#pragma unroll
  for (int k = 1; k < C::J + 2; ++k)
    if (k > L) mc[0] = fmaxf(mc[0], mk[k]);
#pragma unroll
  for (int c = 1; c <= C::LMAX; ++c) mc[c] = (c <= L) ? mk[c] : 0.0f;
  if (!act) {
#pragma unroll
    for (int c = 0; c <= C::LMAX; ++c) mc[c] = 0.0f;
  }

  T* rimc = sm.ghost;   // [field][y]
  const unsigned long long actm = __ballot(act);
  const unsigned long long samp_lanes = __ballot(act && cx == 0);
  if (wave < C::M) {
    // segmented maximum over the lanes of one x class: the members of class
    // c > 0 share the bits below c, the sample columns the bits below L
    const int B = (cx == 0) ? L : cx;
#pragma unroll
    for (int c = 0; c <= C::LMAX; ++c) {
      float m = mc[c];
#pragma unroll
      for (int bit = 0; bit < 6; ++bit) {
        const float t = __shfl_xor(m, 1 << bit, 64);
        if (bit >= B) m = fmaxf(m, t);
      }
      mc[c] = m;
    }
    const bool rep = act && (cx == 0 ? x == 0 : x == (1 << (cx - 1)));
    if (rep) {
#pragma unroll
      for (int c = 0; c <= C::LMAX; ++c)
        if (c <= L) sm.nq.smax[f][c * L1 + cx] = mc[c];
    }
    // kept details (sample positions excluded): per-lane counts summed over
    // the wave; lanes without a line hold zeros
    const bool samp_lane = act && cx == 0;
    int cnt = 0;
#pragma unroll
    for (int y = 0; y < C::P; ++y) cnt += (v[y] != T(0) && !((y & lmask) == 0 && samp_lane)) ? 1 : 0;
    const int run = __shfl(wave_incl_scan(cnt), 63, 64);
    unsigned long long rowb = 0ull;
    if constexpr (C::RIM) rowb = __ballot(v[C::P] != T(0)) & actm & ~samp_lanes;
    if (lane == 0) {
      sm.core_nnz[wave] = (unsigned)run;
      sm.rowbits[wave] = rowb;
    }
  } else if (C::RIM && wave == C::M && act) {
#pragma unroll
    for (int c = 0; c <= C::LMAX; ++c)
      if (c <= L) sm.nq.rmax[f][c] = mc[c];
#pragma unroll
    for (int y = 0; y < C::S; ++y) rimc[f * C::S + y] = v[y];
  }
  if (tid < C::M) sm.nq.occ[tid] = 0ull;
  __syncthreads();

  // Scales, record layouts and one allocation for the patch (wave 0).
  if (wave == 0) {
    const int nb = L1 * L1;
    // largest kept magnitude of subband b of field g (0 for the samples)
    auto band_max = [&sm](int g, int b, int L1_) {
      const int cyy = b / L1_;
      const int cxx = b - cyy * L1_;
      float m = (b == 0) ? 0.0f : sm.nq.smax[g][b];
      if (C::RIM && cxx == 0 && b != 0) m = fmaxf(m, sm.nq.rmax[g][cyy]);
      return m;
    };
    // bounded format: bit g of f16need when field g's record needs binary16
    uint32_t f16need = 0u;
    if constexpr (VF == VF_E4M3B) {
      const float epsq = (float)a.eps;
      for (int i = lane; i < C::M * nb; i += 64) {
        const int g = i / nb;
        const int b = i - g * nb;
        const float m = band_max(g, b, L1);
        if (m > 0.0f) {
          const int cyy = b / L1;
          const int cxx = b - cyy * L1;
          const float thr = thr_of<float>(cxx == 0 ? -1 : L - cxx, cyy == 0 ? -1 : L - cyy, epsq, a.rule);
          if (!e4m3_bounded(m, thr)) f16need |= 1u << g;
        }
      }
#pragma unroll
      for (int d = 1; d < 64; d <<= 1) f16need |= (uint32_t)__shfl_xor((int)f16need, d, 64);
    }
    for (int i = lane; i < C::M * nb; i += 64) {
      const int g = i / nb;
      const int b = i - g * nb;
      const float m = band_max(g, b, L1);
      const bool e4 = VF == VF_E4M3B ? ((f16need >> g) & 1u) == 0u : fixed_e4<VF>();
      int k = 0;
      if (m > 0.0f) {
        k = e4 ? scale_exp<VF_E4M3>(m) : scale_exp<VF_F16>(m);
        atomicOr(&sm.nq.occ[g], 1ull << b);
      }
      sm.nq.kexp[g][b] = (signed char)k;
    }
    if (lane < C::M)
      sm.nq.e4[lane] = (VF == VF_E4M3B ? ((f16need >> lane) & 1u) == 0u : fixed_e4<VF>()) ? 1u : 0u;
    unsigned long long mycol = 0ull;
    if constexpr (C::RIM) {
      const int yy = lane < C::P ? lane : 0;
      const bool det_row = (lane & lmask) != 0;
#pragma unroll
      for (int g = 0; g < C::M; ++g) {
        const unsigned long long cb = __ballot(lane < C::P && det_row && rimc[g * C::S + yy] != T(0));
        if (lane == g) mycol = cb;
      }
    }
    uint32_t rb16 = 0;
    if (lane < C::M) {
      uint32_t ndet = sm.core_nnz[lane];
      if constexpr (C::RIM) {
        ndet += (uint32_t)(__popcll(mycol) + __popcll(sm.rowbits[lane]));
        sm.colbits[lane] = mycol;
        sm.corner[lane] = 0u;
      }
      const uint32_t nocc = (uint32_t)__popcll(sm.nq.occ[lane]);
      const uint32_t by = (VF == VF_E4M3B ? ((f16need >> lane) & 1u) == 0u : fixed_e4<VF>()) ? 1u : 2u;
      const uint32_t ismask = (2u * ndet < 8u * C::W) ? 0u : 1u;
      const uint32_t hb = (8u + 4u * nocc + 7u) & ~7u;
      const uint32_t sb = hb + ((4u * (uint32_t)NS + 7u) & ~7u);
      const uint32_t vb = sb + ((ndet * by + 7u) & ~7u);
      const uint32_t mb = ismask ? 8u * C::W : 2u * ndet;
      rb16 = (vb + mb + 15u) / 16u;
      sm.nnz[lane] = ndet;
      sm.ismask[lane] = ismask;
      sm.vb[lane] = vb;
      sm.rb[lane] = rb16 * 16u;
      sm.nq.hb[lane] = hb;
      sm.nq.sb[lane] = sb;
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
  if (!sm.misc[0]) return false;
  const uint32_t base16 = sm.misc[1];
  if (tid < C::M) {
    a.table_out[2 * (q * C::M + tid)] = base16 + sm.rel16[tid];
    a.table_out[2 * (q * C::M + tid) + 1] = sm.nnz[tid] | (sm.ismask[tid] ? MASK_BIT : 0u);
  }

  if (wave < C::M) {
    uint8_t* rec = a.pool_out + 16ull * (base16 + sm.rel16[f]);
    float* samp = reinterpret_cast<float*>(rec + sm.nq.hb[f]);
    uint8_t* qv = rec + sm.nq.sb[f];
    const bool e4 = VF == VF_E4M3B ? sm.nq.e4[f] != 0u : fixed_e4<VF>();
    const bool ismask = sm.ismask[f] != 0u;
    uint16_t* idx = reinterpret_cast<uint16_t*>(rec + sm.vb[f]);
    // samples of the owned lines and of the shared row, exact
    if (act && cx == 0) {
#pragma unroll
      for (int y = 0; y < C::S; ++y)
        if ((y & lmask) == 0) samp[(y >> L) * SC + (x >> L)] = v[y];
    }
    unsigned long long myw = 0ull;
    unsigned long long wd = 0ull;
    int run = 0;
#pragma unroll
    for (int y = 0; y < C::P; ++y) {
      unsigned long long b = __ballot(v[y] != T(0)) & actm;
      if ((y & lmask) == 0) b &= ~samp_lanes;
      if (b != 0ull) {
        if ((b >> lane) & 1ull) {
          const int rank = run + (int)__builtin_amdgcn_mbcnt_hi((unsigned)(b >> 32),
                                                                __builtin_amdgcn_mbcnt_lo((unsigned)b, 0u));
          const int k = sm.nq.kexp[f][idx_class(y, L) * L1 + cx];
          const uint32_t code = q_enc(e4, v[y], k);
          q_store(e4, qv, rank, code);
          v[y] = q_dec(e4, code, k);
          if (!ismask) idx[rank] = (uint16_t)(x + C::P * y);
        }
        run += __popcll(b);
      }
      if (ismask) {
        wd |= b << (C::P * (y % C::RPW));
        if (y % C::RPW == C::RPW - 1) {
          if (lane == y / C::RPW) myw = wd;
          wd = 0ull;
        }
      }
    }
    if constexpr (C::RIM) {
      const unsigned long long col = sm.colbits[f];
      const unsigned long long rowb = sm.rowbits[f];
      if (col != 0ull) {
        const int yy = lane < C::P ? lane : 0;
        const T c = rimc[f * C::S + yy];
        if (lane < C::P && ((col >> yy) & 1ull)) {
          const int rank = run + (int)__builtin_amdgcn_mbcnt_hi((unsigned)(col >> 32),
                                                                __builtin_amdgcn_mbcnt_lo((unsigned)col, 0u));
          const int k = sm.nq.kexp[f][idx_class(yy, L) * L1];
          q_store(e4, qv, rank, q_enc(e4, c, k));
          if (!ismask) idx[rank] = (uint16_t)(C::P * C::P + yy);
        }
      }
      if ((rowb >> lane) & 1ull) {
        const int rank = run + __popcll(col) + __popcll(rowb & below(x));
        const int k = sm.nq.kexp[f][cx];
        const uint32_t code = q_enc(e4, v[C::P], k);
        q_store(e4, qv, rank, code);
        v[C::P] = q_dec(e4, code, k);
        if (!ismask) idx[rank] = (uint16_t)(C::P * C::P + C::P + x);
      }
    }
    if (ismask && lane < C::CW) reinterpret_cast<unsigned long long*>(rec + sm.vb[f])[lane] = myw;
  } else if (C::RIM && wave == C::M && act) {
    // the shared column: samples to their slots; details read back as stored
    uint8_t* rec = a.pool_out + 16ull * (base16 + sm.rel16[f]);
    float* samp = reinterpret_cast<float*>(rec + sm.nq.hb[f]);
    const bool e4 = VF == VF_E4M3B ? sm.nq.e4[f] != 0u : fixed_e4<VF>();
#pragma unroll
    for (int y = 0; y < C::S; ++y) {
      if ((y & lmask) == 0) {
        samp[(y >> L) * SC + (C::P >> L)] = v[y];
      } else if (v[y] != T(0)) {
        const int k = sm.nq.kexp[f][idx_class(y, L) * L1];
        v[y] = q_dec(e4, q_enc(e4, v[y], k), k);
      }
    }
  }
  if (tid < C::M) {
    const int g = tid;
    uint8_t* rec = a.pool_out + 16ull * (base16 + sm.rel16[g]);
    const unsigned long long occ = sm.nq.occ[g];
    const bool e4g = sm.nq.e4[g] != 0u;
    *reinterpret_cast<unsigned long long*>(rec) = occ | ((VF == VF_E4M3B && e4g) ? OCC_E4M3 : 0ull);
    float* scl = reinterpret_cast<float*>(rec + 8);
    int i = 0;
    for (int b = 1; b < L1 * L1; ++b)
      if ((occ >> b) & 1ull) scl[i++] = ldexpf(1.0f, sm.nq.kexp[g][b]);
    zero_bytes(rec, 8u + 4u * (uint32_t)i, sm.nq.hb[g]);
    zero_bytes(rec, sm.nq.hb[g] + 4u * (uint32_t)NS, sm.nq.sb[g]);
    zero_bytes(rec, sm.nq.sb[g] + (e4g ? 1u : 2u) * sm.nnz[g], sm.vb[g]);
    if constexpr (C::RIM) {
      if (sm.ismask[g]) {
        unsigned long long r[3];
        rim_join<C>(sm.colbits[g], sm.rowbits[g], false, r[0], r[1], r[2]);
        unsigned long long* wds = reinterpret_cast<unsigned long long*>(rec + sm.vb[g]);
#pragma unroll
        for (int j = 0; j < C::W - C::CW; ++j) wds[C::CW + j] = r[j];
      }
    }
    const uint32_t mend = sm.vb[g] + (sm.ismask[g] ? 8u * C::W : 2u * sm.nnz[g]);
    zero_bytes(rec, mend, sm.rb[g]);
  }
  totals_finish<C, T, FWD>(a, a.partials_out + (size_t)q * C::M, L, sm);
  if (wave < C::M && act) export_features<C, T>(a, q, f, x, v);

  // S8, column half: inverse of the stored column, back to LDS.
  if (act) {
    LF::inv(v, L);
    store_col<C>(v, sm.tile, field_base<C>(f), x);
  }
  __syncthreads();
  return true;
}

// ---------------------------------------------------------------------------
// S1 (+ the column half of S2) for a narrow format: every record is scattered
// into a zeroed LDS tile (samples, then details with their subband scale),
// then every column is inverse-transformed from LDS.
// ---------------------------------------------------------------------------
template <class C, class T, int WAV, bool TOT, int VF, class SM>
__device__ __forceinline__ void expand_columns_q(const PatchArgs& a, int q, SM& sm) {
  using LF = Lift<T, C::S, WAV, 1, C::LMAX>;
  const int tid = tid_of<C>();
  const int lane = lane_of<C>();
  const int wave = wave_of<C>();
  const int L = a.levels;
  const int L1 = L + 1;
  const int SC = ((C::S - 1) >> L) + 1;
  const int NS = SC * SC;
  // te: wave-uniform index (one scalar value), tel: index that varies over the lanes
  auto te = [&sm](int i) { return (uint32_t)__builtin_amdgcn_readfirstlane((int)sm.te[i]); };
  auto tel = [&sm](int i) { return sm.te[i]; };
  const uint8_t* pool = a.pool_in;

#pragma unroll
  for (int f = 0; f < C::M; ++f) zero_span<T>(sm.tile + C::Lay::fb(f), C::S * C::RS, tid, C::NT);
  if (tid < C::M) {
    const int g = tid;
    const uint32_t ndet = tel(2 * g + 1) & ~MASK_BIT;
    const uint8_t* rec = pool + 16ull * tel(2 * g);
    const unsigned long long occ0 = *reinterpret_cast<const unsigned long long*>(rec);
    const bool e4 = VF == VF_E4M3B ? (occ0 & OCC_E4M3) != 0ull : fixed_e4<VF>();
    const unsigned long long occ = VF == VF_E4M3B ? occ0 & ~OCC_E4M3 : occ0;
    const uint32_t nocc = (uint32_t)__popcll(occ);
    const uint32_t hb = (8u + 4u * nocc + 7u) & ~7u;
    const uint32_t sb = hb + ((4u * (uint32_t)NS + 7u) & ~7u);
    sm.nq.hb[g] = hb;
    sm.nq.sb[g] = sb;
    sm.nq.e4[g] = e4 ? 1u : 0u;
    sm.vb[g] = sb + ((ndet * (e4 ? 1u : 2u) + 7u) & ~7u);
    const float* scl = reinterpret_cast<const float*>(rec + 8);
    int i = 0;
    for (int b = 1; b < L1 * L1; ++b)
      if ((occ >> b) & 1ull) sm.nq.kexp[g][b] = (signed char)ilogbf(scl[i++]);
  }
  if (wave < C::M) {
    const int g = wave;
    const uint32_t w = te(2 * g + 1);
    if (w & MASK_BIT) {
      const uint32_t ndet = w & ~MASK_BIT;
      const uint8_t* rec = pool + 16ull * te(2 * g);
      const unsigned long long occ0 = *reinterpret_cast<const unsigned long long*>(rec);
      const bool e4 = VF == VF_E4M3B ? (occ0 & OCC_E4M3) != 0ull : fixed_e4<VF>();
      const uint32_t nocc = (uint32_t)__popcll(VF == VF_E4M3B ? occ0 & ~OCC_E4M3 : occ0);
      const uint32_t vb = ((8u + 4u * nocc + 7u) & ~7u) + ((4u * (uint32_t)NS + 7u) & ~7u) +
                          ((ndet * (e4 ? 1u : 2u) + 7u) & ~7u);
      const unsigned long long* words = reinterpret_cast<const unsigned long long*>(rec + vb);
      const int c0 = lane < C::W ? __popcll(words[lane]) : 0;
      const int c1 = (64 + lane) < C::W ? __popcll(words[64 + lane]) : 0;
      const int i0 = wave_incl_scan(c0);
      const int tot0 = __shfl(i0, 63, 64);
      const int i1 = wave_incl_scan(c1);
      if (lane < C::W) sm.nq.wpre[g][lane] = (uint16_t)(i0 - c0);
      if (64 + lane < C::W) sm.nq.wpre[g][64 + lane] = (uint16_t)(tot0 + i1 - c1);
    }
  }
  __syncthreads();

  int pre[C::M + 1];
  pre[0] = 0;
#pragma unroll
  for (int g = 0; g < C::M; ++g) pre[g + 1] = pre[g] + NS + (int)(te(2 * g + 1) & ~MASK_BIT);
  for (int i = tid; i < pre[C::M]; i += C::NT) {
    int g = 0;
#pragma unroll
    for (int h = 1; h < C::M; ++h) g += (i >= pre[h]) ? 1 : 0;
    int j = i - pre[g];
    const uint32_t w = tel(2 * g + 1);
    const uint8_t* rec = pool + 16ull * tel(2 * g);
    int xx, yy;
    T val;
    if (j < NS) {
      yy = (j / SC) << L;
      xx = (j - (j / SC) * SC) << L;
      val = reinterpret_cast<const float*>(rec + sm.nq.hb[g])[j];
    } else {
      j -= NS;
      int k;
      if (w & MASK_BIT) {
        // the word holding the j-th set bit: last word whose prefix is <= j
        int lo = 0, hi = C::W - 1;
        while (lo < hi) {
          const int mid = (lo + hi + 1) >> 1;
          if ((int)sm.nq.wpre[g][mid] <= j) lo = mid; else hi = mid - 1;
        }
        const unsigned long long wd = reinterpret_cast<const unsigned long long*>(rec + sm.vb[g])[lo];
        k = 64 * lo + select_bit(wd, j - (int)sm.nq.wpre[g][lo]);
      } else {
        k = reinterpret_cast<const uint16_t*>(rec + sm.vb[g])[j];
      }
      record_node<C>(k, xx, yy);
      const int e = sm.nq.kexp[g][idx_class(yy, L) * L1 + idx_class(xx, L)];
      const bool e4 = VF == VF_E4M3B ? sm.nq.e4[g] != 0u : fixed_e4<VF>();
      val = q_dec(e4, q_load(e4, rec + sm.nq.sb[g], j), e);
    }
    sm.tile[C::Lay::fb(g) + yy * C::RS + xx] = val;
  }
  __syncthreads();

  int f, x;
  const bool line = pass_line<C>(f, x);
  double part = 0.0;
  if (line) {
    T v[C::S];
    load_col<C>(v, sm.tile, field_base<C>(f), x);
    if constexpr (TOT) part = column_sample_sum<C, T>(v, x, L);
    LF::inv(v, L);
    store_col<C>(v, sm.tile, field_base<C>(f), x);
  }
  if constexpr (TOT) {
    if (wave < C::M) totals_partial<C, T>(part, sm);
    else if (line) sm.totface[f] = part;
  }
  __syncthreads();
}

}  // namespace lbmz
