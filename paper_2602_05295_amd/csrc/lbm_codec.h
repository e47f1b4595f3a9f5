// lbm_codec.h -- the stored integer formats behind one interface: words per
// cell, decode to the pre-collision cell, encode of new moments, and the
// codes of the rest state.  FMT_Q16 is Sec. 5.3's paired 16-bit layout with
// its packed-conversion encoder; the FMT_P formats are the b_rho_u / b_S
// allocations (Packed in lbm_device.h).  FMT_F32 stores floats and has its
// own paths in the kernels.
#pragma once

#include "lbm_device.h"
#include "lbm_internal.h"

namespace lbm {

template <int FMT>
struct Codec {
  static_assert(fmt_packed(FMT), "FMT_F32 has no codes");
  using PK = Packed<fmt_b1(FMT), fmt_b2(FMT)>;
  static constexpr int W = PK::W;
  static constexpr float DR = PK::DR, DU = PK::DU;
  static __device__ inline CellIn decode(const uint32_t* w) { return cell_from_packed<PK>(w); }
  // the ten codes as floats (exact), in the stored order
  static __device__ inline void code_floats(const uint32_t* w, float q[10]) {
    uint32_t k[10];
    packed_codes<PK>(w, k);
#pragma unroll
    for (int i = 0; i < 10; ++i) q[i] = float(k[i]);
  }
  static __device__ inline void encode(float dr, const float j[3], const float P[6], uint32_t cell, uint32_t key,
                                       bool dith, uint32_t* w) {
    encode_packed<PK>(dr, j, P, cell, key, dith, w);
  }
  // codes at 0 or at their maximum (the health scan's saturation test)
  static __device__ inline uint32_t saturated(const uint32_t* w) {
    uint32_t q[10];
    packed_codes<PK>(w, q);
    uint32_t n = 0;
#pragma unroll
    for (int k = 0; k < 10; ++k) n += (q[k] == 0u || q[k] == PK::qmax(k)) ? 1u : 0u;
    return n;
  }
};

template <>
struct Codec<FMT_Q16> {
  static constexpr int W = 5;
  static constexpr float DR = Q_RHO_D, DU = Q_U_D;
  static __device__ inline CellIn decode(const uint32_t* w) { return cell_from_words(w); }
  static __device__ inline void code_floats(const uint32_t* w, float q[10]) {
#pragma unroll
    for (int i = 0; i < 5; ++i) {
      q[2 * i] = float(lo16(w[i]));
      q[2 * i + 1] = float(hi16(w[i]));
    }
  }
  static __device__ inline void encode(float dr, const float j[3], const float P[6], uint32_t cell, uint32_t key,
                                       bool dith, uint32_t* w) {
    encode_cell(dr, j, P, cell, key, dith, w);
  }
  static __device__ inline uint32_t saturated(const uint32_t* w) {
    uint32_t n = 0;
#pragma unroll
    for (int k = 0; k < 5; ++k) {
      n += (lo16(w[k]) == 0u || lo16(w[k]) == 0xFFFFu) ? 1u : 0u;
      n += (hi16(w[k]) == 0u || hi16(w[k]) == 0xFFFFu) ? 1u : 0u;
    }
    return n;
  }
};

// App. A without force, applied to a cell's codes.  With N = lo + q dN the
// post-collision stress (1 - 1/tau) dev(N) is om1 dN q + om1 lo off the
// diagonal and om1 dN (q - (q_xx + q_yy + q_zz)/3) on it, where lo cancels:
// N itself is never formed (nq_s = om1 dN, nq_d = nq_s / 3, nq_c = om1 lo).
// Gives the moments of collide_neq applied to Codec<FMT>::decode(w).
template <int FMT>
__device__ inline void collide_codes(const uint32_t* w, float nq_s, float nq_d, float nq_c, float& dr, float& rho,
                                     float u[3], float j[3], float Nn[6]) {
  float q[10];
  Codec<FMT>::code_floats(w, q);
  dr = fmaf(q[0], Codec<FMT>::DR, Q_DRHO_LO);
  rho = dr + 1.0f;
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    u[a] = fmaf(q[1 + a], Codec<FMT>::DU, Q_U_LO);
    j[a] = rho * u[a];
  }
  const float m = (q[4] + q[5] + q[6]) * nq_d;  // the sum of three codes is exact
  Nn[0] = fmaf(q[4], nq_s, -m);
  Nn[1] = fmaf(q[5], nq_s, -m);
  Nn[2] = fmaf(q[6], nq_s, -m);
  Nn[3] = fmaf(q[7], nq_s, nq_c);
  Nn[4] = fmaf(q[8], nq_s, nq_c);
  Nn[5] = fmaf(q[9], nq_s, nq_c);
}

// Post-collision coefficients of a cell's codes (App. A without force).
template <int FMT>
__device__ inline void post_collision_codes(const uint32_t* w, float nq_s, float nq_d, float nq_c, float A[NA]) {
  float dr, rho, u[3], j[3], Nn[6];
  collide_codes<FMT>(w, nq_s, nq_d, nq_c, dr, rho, u, j, Nn);
  hermite_coeffs(dr, j, u, Nn, A);
}

// Codes of the rest state (rho = 1, u = 0, N = 0), rounded without dither.
template <int FMT>
__device__ inline void rest_codes(uint32_t* w) {
  if constexpr (FMT == FMT_Q16) {
    const uint32_t qr = quantize(1.0f - Q_RHO_LO, Q_RHO_S, 0.0f);
    const uint32_t qu = quantize(0.0f - Q_U_LO, Q_U_S, 0.0f);
    const uint32_t qn = quantize(0.0f - Q_N_LO, Q_N_S, 0.0f);
    w[0] = qr | (qu << 16);
    w[1] = qu | (qu << 16);
    w[2] = qn | (qn << 16);
    w[3] = qn | (qn << 16);
    w[4] = qn | (qn << 16);
  } else {
    // the same expressions as the undithered encode of full moments
    using PK = typename Codec<FMT>::PK;
    uint32_t q[10];
    q[0] = quantize_b(1.0f - Q_RHO_LO, PK::SR, 0.0f, PK::qmax(0));
#pragma unroll
    for (int a = 0; a < 3; ++a) q[1 + a] = quantize_b(0.0f - Q_U_LO, PK::SU, 0.0f, PK::qmax(1));
#pragma unroll
    for (int p = 0; p < 6; ++p) q[4 + p] = quantize_b(0.0f - Q_N_LO, PK::SN, 0.0f, PK::qmax(4));
    pack_codes<PK>(q, w);
  }
}

// The dither key of a step: the host's, or in a captured step sequence the
// one of the device-side step counter plus the step's place in the sequence.
__device__ inline uint32_t step_key(const StepParams& a) {
  return a.step_ctr ? dither_key(*a.step_ctr + a.step_off, a.seed, a.dither_mode) : a.key;
}

// Calls f.template operator()<FMT>() for the integer format fmt (runtime
// dispatch over the instantiated formats); returns false for FMT_F32 or an
// unknown value.
template <class Fn>
inline bool dispatch_codes(int fmt, Fn&& f) {
  switch (fmt) {
    case FMT_Q16: f.template operator()<FMT_Q16>(); return true;
    case FMT_P16_15: f.template operator()<FMT_P16_15>(); return true;
    case FMT_P15_14: f.template operator()<FMT_P15_14>(); return true;
    case FMT_P14_13: f.template operator()<FMT_P14_13>(); return true;
    case FMT_P13_12: f.template operator()<FMT_P13_12>(); return true;
    case FMT_P12_11: f.template operator()<FMT_P12_11>(); return true;
    default: return false;
  }
}

}  // namespace lbm
