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

// f+_c - w_c = sum A_nml P_n(cx) P_m(cy) P_l(cz) (the rest part removed with
// rho - 1), contracted one axis at a time (z, then y, then x): 17 + 5 + 3
// multiply-adds once the basis values are known.
__device__ inline float eval_link(const float A[NA], int cx, int cy, int cz) {
  float px[3], py[3], pz[3];
  basis1(cx, px);
  basis1(cy, py);
  basis1(cz, pz);
  const float b00 = fmaf(A[A002], pz[2], fmaf(A[A001], pz[1], A[A000] * pz[0]));
  const float b10 = fmaf(A[A102], pz[2], fmaf(A[A101], pz[1], A[A100] * pz[0]));
  const float b01 = fmaf(A[A012], pz[2], fmaf(A[A011], pz[1], A[A010] * pz[0]));
  const float b20 = fmaf(A[A201], pz[1], A[A200] * pz[0]);
  const float b02 = fmaf(A[A021], pz[1], A[A020] * pz[0]);
  const float b11 = fmaf(A[A111], pz[1], A[A110] * pz[0]);
  const float b21 = A[A210] * pz[0];
  const float b12 = A[A120] * pz[0];
  const float c0 = fmaf(b02, py[2], fmaf(b01, py[1], b00 * py[0]));
  const float c1 = fmaf(b12, py[2], fmaf(b11, py[1], b10 * py[0]));
  const float c2 = fmaf(b21, py[1], b20 * py[0]);
  return fmaf(c2, px[2], fmaf(c1, px[1], c0 * px[0]));
}

// v + d wrapped into [0, n) for |d| <= 1.
__device__ inline int wrap_step(int v, int d, int n) {
  const int w = v + d;
  return w < 0 ? w + n : (w >= n ? w - n : w);
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

// The distribution that listed fluid cell `cell` (coordinates x, y, z; flags
// b) receives on link i = (cx + 1) + 3 (cy + 1) + 9 (cz + 1) under the
// boundary rules: one source cell, its post-collision coefficients (with the
// inflow velocity on inflow links), evaluated in the link's direction (the
// opposite one on bounce-back links).
template <int FMT>
__device__ inline float boundary_link(const StepParams& a, uint32_t cell, uint32_t b, int x, int y, int z, int i) {
  const int nx = a.g.nx, ny = a.g.ny, nz = a.g.nz;
  const int cx = i % 3 - 1, cy = (i / 3) % 3 - 1, cz = i / 9 - 1;
  uint32_t q = cell;
  bool flip = false, inflow = false;
  if ((b & BIT_INFLOW) && cx == 1) {
    inflow = true;
  } else if ((b & BIT_OUTFLOW) && cx == -1) {
    q = uint32_t(nx - 1) + uint32_t(nx) * (uint32_t(wrap_step(y, -cy, ny)) + uint32_t(ny) * uint32_t(wrap_step(z, -cz, nz)));
  } else if ((b >> i) & 1u) {
    flip = true;
  } else {
    q = uint32_t(wrap_step(x, -cx, nx)) +
        uint32_t(nx) * (uint32_t(wrap_step(y, -cy, ny)) + uint32_t(ny) * uint32_t(wrap_step(z, -cz, nz)));
  }
  const CellIn c = load_cell_b<FMT>(a, q);
  float Nn[6];
  collide_neq(c.N, a.om1, Nn);
  float A[NA];
  if (inflow) {
    const float jin[3] = {c.rho * a.u_in[0], c.rho * a.u_in[1], c.rho * a.u_in[2]};
    hermite_coeffs(c.dr, jin, a.u_in, Nn, A);
  } else {
    hermite_coeffs(c.dr, c.j, c.u, Nn, A);
  }
  return flip ? eval_link(A, -cx, -cy, -cz) : eval_link(A, cx, cy, cz);
}

// Sum over the 32 lanes of a half-wavefront, complete in its last lane (31 or
// 63): an inclusive scan inside each row of 16 lanes (DPP row shifts 1, 2, 4,
// 8, reading 0 past the row start), then the total of row 0 (2) added into
// row 1 (3) with a row broadcast of lane 15.
__device__ inline float half_wave_sum(float v) {
  v += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x111, 0xF, 0xF, true));  // row_shr:1
  v += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x112, 0xF, 0xF, true));  // row_shr:2
  v += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x114, 0xF, 0xF, true));  // row_shr:4
  v += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x118, 0xF, 0xF, true));  // row_shr:8
  v += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x142, 0xA, 0xF, false));  // row_bcast:15
  return v;
}

// One listed fluid cell per 32-lane group, link i on lane i (lanes 27..31
// add nothing): each lane takes its link's distribution and its share of the
// ten moments, the group sums them, and its last lane writes the cell once.
// All lanes of a group must be active (the caller keeps groups whole) and a
// group must be one half of a wavefront.
// yz: the cell's y | z << 16 (stored with the list, so no division is needed).
template <int FMT>
__device__ inline void boundary_group(const StepParams& a, uint32_t cell, uint32_t b, uint32_t yz, int i) {
  const int nx = a.g.nx, ny = a.g.ny;
  const int y = int(yz & 0xFFFFu), z = int(yz >> 16);
  const int x = int(cell - uint32_t(nx) * (uint32_t(y) + uint32_t(ny) * uint32_t(z)));
  float m[10];
#pragma unroll
  for (int k = 0; k < 10; ++k) m[k] = 0.0f;
  if (i < 27) {
    const float f = boundary_link<FMT>(a, cell, b, x, y, z, i);
    const float fx = float(i % 3 - 1), fy = float((i / 3) % 3 - 1), fz = float(i / 9 - 1);
    m[0] = f;
    m[1] = fx * f;
    m[2] = fy * f;
    m[3] = fz * f;
    m[4] = (fx * fx - R3) * f;
    m[5] = (fy * fy - R3) * f;
    m[6] = (fz * fz - R3) * f;
    m[7] = fx * fy * f;
    m[8] = fx * fz * f;
    m[9] = fy * fz * f;
  }
#pragma unroll
  for (int k = 0; k < 10; ++k) m[k] = half_wave_sum(m[k]);
  if (i == 31) {
    const float j[3] = {m[1], m[2], m[3]};
    const float P[6] = {m[4], m[5], m[6], m[7], m[8], m[9]};
    store_cell_b<FMT>(a, cell, m[0], j, P);
  }
}

// A listed solid cell: reset to rest.
template <int FMT>
__device__ inline void boundary_solid(const StepParams& a, uint32_t cell) {
  if constexpr (FMT == FMT_F32) {
    const float j[3] = {0, 0, 0}, P[6] = {0, 0, 0, 0, 0, 0};
    store_cell_b<FMT>(a, cell, 0.0f, j, P);
  } else {
    uint32_t w[5];
    rest_words(w);
#pragma unroll
    for (int k = 0; k < 5; ++k) *reinterpret_cast<uint32_t*>(static_cast<char*>(a.out[k]) + cell * 4u) = w[k];
  }
}

}  // namespace lbm
