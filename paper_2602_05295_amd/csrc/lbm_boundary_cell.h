// lbm_boundary_cell.h -- the boundary pass of one listed cell (device code
// shared by the single-domain and the batched boundary kernels).
//
// A listed fluid cell is recomputed from scratch: each of its 27 incoming
// distributions is the pull-streamed f+ of its source, except on links whose
// source is solid (halfway bounce-back: f_i(x) = f+_opp(i)(x)), links entering
// through the inflow face (the moment boundary of Sec. 3.2 with p on the face:
// rho^p = rho^x, u^p = u_in and the post-collision non-equilibrium stress of
// x) and links entering through the outflow face (zero gradient:
// f+_i(nx-1, y - c_y, z - c_z)).  The new moments are encoded once and
// overwrite what the fluid pass wrote, so each cell has one writer, no atomics
// and a single rounding.  Solid cells next to fluid are reset to rest.
#pragma once

#include "lbm_device.h"
#include "lbm_internal.h"

namespace lbm {

// P_n(c) = w1(c) h_n(c) / s_n for c in {-1, 0, 1}, in the index scaling of
// hermite_coeffs and with the same float constants as the 1D passes.
__device__ inline void basis1(int c, float P[3]) {
  if (c == 0) {
    P[0] = C0;
    P[1] = 0.0f;
    P[2] = -2.0f;
  } else {
    P[0] = C6;
    P[1] = c > 0 ? 0.5f : -0.5f;
    P[2] = 1.0f;
  }
}

// f+_i - w_i = sum A_nml P_n(cx) P_m(cy) P_l(cz) (rest part removed with rho - 1).
__device__ inline float eval_dir(const float A[NA], int cx, int cy, int cz) {
  float px[3], py[3], pz[3];
  basis1(cx, px);
  basis1(cy, py);
  basis1(cz, pz);
  float s = A[A000] * px[0] * py[0] * pz[0];
  s = fmaf(A[A100] * px[1], py[0] * pz[0], s);
  s = fmaf(A[A010] * px[0], py[1] * pz[0], s);
  s = fmaf(A[A001] * px[0], py[0] * pz[1], s);
  s = fmaf(A[A200] * px[2], py[0] * pz[0], s);
  s = fmaf(A[A020] * px[0], py[2] * pz[0], s);
  s = fmaf(A[A002] * px[0], py[0] * pz[2], s);
  s = fmaf(A[A110] * px[1], py[1] * pz[0], s);
  s = fmaf(A[A101] * px[1], py[0] * pz[1], s);
  s = fmaf(A[A011] * px[0], py[1] * pz[1], s);
  s = fmaf(A[A210] * px[2], py[1] * pz[0], s);
  s = fmaf(A[A120] * px[1], py[2] * pz[0], s);
  s = fmaf(A[A201] * px[2], py[0] * pz[1], s);
  s = fmaf(A[A102] * px[1], py[0] * pz[2], s);
  s = fmaf(A[A021] * px[0], py[2] * pz[1], s);
  s = fmaf(A[A012] * px[0], py[1] * pz[2], s);
  s = fmaf(A[A111] * px[1], py[1] * pz[1], s);
  return s;
}

template <int FMT>
__device__ inline CellIn load_cell_b(const StepParams& a, uint32_t cell) {
  const uint32_t off = cell * 4u;
  if constexpr (FMT == FMT_F32) {
    float m[10];
#pragma unroll
    for (int k = 0; k < 10; ++k) m[k] = *reinterpret_cast<const float*>(static_cast<const char*>(a.in[k]) + off);
    return cell_from_moments(m);
  } else {
    uint32_t w[5];
#pragma unroll
    for (int k = 0; k < 5; ++k) w[k] = *reinterpret_cast<const uint32_t*>(static_cast<const char*>(a.in[k]) + off);
    return cell_from_words(w);
  }
}

template <int FMT>
__device__ inline void post_coeffs(const StepParams& a, uint32_t cell, float A[NA]) {
  const CellIn c = load_cell_b<FMT>(a, cell);
  float Nn[6];
  collide_neq(c.N, a.om1, Nn);
  hermite_coeffs(c.dr, c.j, c.u, Nn, A);
}

template <int FMT>
__device__ inline void store_cell_b(const StepParams& a, uint32_t cell, float dr, const float j[3], const float P[6]) {
  const uint32_t off = cell * 4u;
  if constexpr (FMT == FMT_F32) {
    const float v[10] = {dr, j[0], j[1], j[2], P[0], P[1], P[2], P[3], P[4], P[5]};
#pragma unroll
    for (int k = 0; k < 10; ++k) *reinterpret_cast<float*>(static_cast<char*>(a.out[k]) + off) = v[k];
  } else {
    uint32_t w[5];
    encode_cell(dr, j, P, cell, a.key, a.dither != 0, w);
#pragma unroll
    for (int k = 0; k < 5; ++k) *reinterpret_cast<uint32_t*>(static_cast<char*>(a.out[k]) + off) = w[k];
  }
}

// Code words of the rest state (rho = 1, u = 0, N = 0), rounded without dither.
__device__ inline void rest_words(uint32_t w[5]) {
  const uint32_t qr = quantize(1.0f - Q_RHO_LO, Q_RHO_S, 0.5f);
  const uint32_t qu = quantize(0.0f - Q_U_LO, Q_U_S, 0.5f);
  const uint32_t qn = quantize(0.0f - Q_N_LO, Q_N_S, 0.5f);
  w[0] = qr | (qu << 16);
  w[1] = qu | (qu << 16);
  w[2] = qn | (qn << 16);
  w[3] = qn | (qn << 16);
  w[4] = qn | (qn << 16);
}

// Recomputes one listed cell (cell index within the planes of `a`, flags b)
// and writes its new moments to a.out.
template <int FMT>
__device__ inline void boundary_entry(const StepParams& a, uint32_t cell, uint32_t b) {
  if (b & BIT_SOLID) {
    const float j[3] = {0, 0, 0}, P[6] = {0, 0, 0, 0, 0, 0};
    if constexpr (FMT == FMT_F32) {
      store_cell_b<FMT>(a, cell, 0.0f, j, P);
    } else {
      uint32_t w[5];
      rest_words(w);
#pragma unroll
      for (int k = 0; k < 5; ++k) *reinterpret_cast<uint32_t*>(static_cast<char*>(a.out[k]) + cell * 4u) = w[k];
    }
    return;
  }
  const int nx = a.g.nx, ny = a.g.ny, nz = a.g.nz;
  const int x = int(cell % uint32_t(nx));
  const int y = int((cell / uint32_t(nx)) % uint32_t(ny));
  const int z = int(cell / (uint32_t(nx) * uint32_t(ny)));

  // own post-collision coefficients (bounce-back and inflow links use them)
  const CellIn c0 = load_cell_b<FMT>(a, cell);
  float Nn0[6];
  collide_neq(c0.N, a.om1, Nn0);
  float Aown[NA];
  hermite_coeffs(c0.dr, c0.j, c0.u, Nn0, Aown);
  float Ain[NA];
  if (b & BIT_INFLOW) {
    const float jin[3] = {c0.rho * a.u_in[0], c0.rho * a.u_in[1], c0.rho * a.u_in[2]};
    hermite_coeffs(c0.dr, jin, a.u_in, Nn0, Ain);
  }

  float m[10];
#pragma unroll
  for (int k = 0; k < 10; ++k) m[k] = 0.0f;
  for (int i = 0; i < 27; ++i) {
    const int cx = i % 3 - 1, cy = (i / 3) % 3 - 1, cz = i / 9 - 1;
    float f;
    if ((b & BIT_INFLOW) && cx == 1) {
      f = eval_dir(Ain, cx, cy, cz);
    } else if ((b & BIT_OUTFLOW) && cx == -1) {
      const uint32_t s = uint32_t(nx - 1) + uint32_t(nx) * (uint32_t(wrapi(y - cy, ny)) + uint32_t(ny) * uint32_t(wrapi(z - cz, nz)));
      float As[NA];
      post_coeffs<FMT>(a, s, As);
      f = eval_dir(As, cx, cy, cz);
    } else if ((b >> i) & 1u) {
      f = eval_dir(Aown, -cx, -cy, -cz);
    } else {
      const uint32_t s = uint32_t(wrapi(x - cx, nx)) +
                         uint32_t(nx) * (uint32_t(wrapi(y - cy, ny)) + uint32_t(ny) * uint32_t(wrapi(z - cz, nz)));
      float As[NA];
      post_coeffs<FMT>(a, s, As);
      f = eval_dir(As, cx, cy, cz);
    }
    const float fx = float(cx), fy = float(cy), fz = float(cz);
    m[0] += f;
    m[1] = fmaf(fx, f, m[1]);
    m[2] = fmaf(fy, f, m[2]);
    m[3] = fmaf(fz, f, m[3]);
    m[4] = fmaf(fx * fx - R3, f, m[4]);
    m[5] = fmaf(fy * fy - R3, f, m[5]);
    m[6] = fmaf(fz * fz - R3, f, m[6]);
    m[7] = fmaf(fx * fy, f, m[7]);
    m[8] = fmaf(fx * fz, f, m[8]);
    m[9] = fmaf(fy * fz, f, m[9]);
  }
  const float j[3] = {m[1], m[2], m[3]};
  const float P[6] = {m[4], m[5], m[6], m[7], m[8], m[9]};
  store_cell_b<FMT>(a, cell, m[0], j, P);
}

}  // namespace lbm
