// lbm_device.h -- device building blocks of the HOME-LBM step on gfx950.
//
// Formulation.  The step of Sec. 4.2 (Alg. 2) collides in moment space
// (App. A), reconstructs f+ with the third-order Hermite expansion of
// Eq. (three_order_f), pull-streams and projects back (Eq. rho_u_stress).
// With D3Q27's tensor-product weights w_i = w1(cx) w1(cy) w1(cz), the
// reconstruction is a separable sum
//     f+(c) = sum_{n,m,l} A_nml P_n(cx) P_m(cy) P_l(cz),
//     P_n(c) = w1(c) h_n(c),  h_0 = 1, h_1 = c, h_2 = c^2 - 1/3,
// over 17 coefficients A_nml (the Hermite coefficients a0, a1, a2, a3 times
// 1/(n! cs^2n) factors 1, 3, 9/2 per axis), and the projection is the same
// tensor product with g_a = h_a.  Pull-streaming then projecting commutes
// with the other axes, so the whole step factorises into three 1D passes,
// one per axis, each a D1Q3 "reconstruct -> shift by one cell -> project" of
// 3-channel groups.  No 27-value distribution set is ever formed.
//
// Precision.  Everything is FP32.  The rest state is taken out analytically:
// the density channel carries rho - 1, so a uniform rest state is an exact
// fixed point and the cancellation in the second moment (1/3 - 1/3) never
// happens.  FP32 storage keeps rho - 1 too: stored as rho, the density would
// be quantised at ulp(1) = 1.2e-7, and the second moment, which sees the
// density's discrete Laplacian, would inherit errors near 1e-5 of its size.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace lbm {

// ------------------------------------------------------------ 16-bit codec ---
// Sec. 5.3: rho in [0.8, 1.5], u in [-0.4, 0.4], rho S^neq = P - rho u u in
// [-0.1, 0.1]; q = floor((m - min)/(max - min) (2^16 - 1) + 1/2 + xi).
constexpr float Q_RHO_LO = 0.8f, Q_RHO_HI = 1.5f;
constexpr float Q_U_LO = -0.4f, Q_U_HI = 0.4f;
constexpr float Q_N_LO = -0.1f, Q_N_HI = 0.1f;
constexpr float QMAXF = 65535.0f;
// scales (2^16 - 1)/(max - min) and steps (max - min)/(2^16 - 1), rounded once
constexpr float Q_RHO_S = float(65535.0 / (1.5 - 0.8));
constexpr float Q_U_S = float(65535.0 / 0.8);
constexpr float Q_N_S = float(65535.0 / 0.2);
constexpr float Q_RHO_D = float((1.5 - 0.8) / 65535.0);
constexpr float Q_U_D = float(0.8 / 65535.0);
constexpr float Q_N_D = float(0.2 / 65535.0);
// rho - 1 at code 0, i.e. the decode offset of the density channel
constexpr float Q_DRHO_LO = float(0.8 - 1.0);

// pcg_hash (Jarzynski & Olano, "Hash Functions for GPU Rendering", JCGT 2020):
// one LCG step, then the RXS-M-XS output permutation.
__host__ __device__ inline uint32_t pcg_hash(uint32_t v) {
  const uint32_t state = v * 747796405u + 2891336453u;
  const uint32_t word = ((state >> ((state >> 28u) + 4u)) ^ state) * 277803737u;
  return (word >> 22u) ^ word;
}

// Key of step t (mode 2: one key for all steps).
__host__ __device__ inline uint32_t dither_key(uint32_t t, uint32_t seed, int mode) {
  return pcg_hash(seed ^ pcg_hash(mode == 2 ? 0u : t));
}

// The two hash words of one cell; component k uses the 6-bit field
// (h[k / 5] >> (6 (k % 5))) & 63, and 1/2 + xi = (v + 1/2)/64.
__device__ inline void dither_words(uint32_t idx, uint32_t key, uint32_t& h1, uint32_t& h2) {
  h1 = pcg_hash(idx ^ key);
  h2 = pcg_hash(h1 ^ 0x9E3779B9u);
}

// 1/2 + xi for component k (or 1/2 without dither).
template <int K>
__device__ inline float half_plus_xi(uint32_t h1, uint32_t h2, bool dith) {
  if (!dith) return 0.5f;
  const uint32_t src = (K < 5) ? h1 : h2;
  const uint32_t v = (src >> (6 * (K % 5))) & 63u;
  return fmaf(float(v), 1.0f / 64.0f, 1.0f / 128.0f);
}

// floor((m - lo) * s + (1/2 + xi)), saturated to [0, 65535].
__device__ inline uint32_t quantize(float d_from_lo, float s, float hpx) {
  float v = fmaf(d_from_lo, s, hpx);
  v = fminf(fmaxf(v, 0.0f), QMAXF);
  return uint32_t(v);
}

__device__ inline uint32_t lo16(uint32_t w) { return w & 0xFFFFu; }
__device__ inline uint32_t hi16(uint32_t w) { return w >> 16; }

// ------------------------------------------------------------- cell state ---
// Decoded pre-collision cell: dr = rho - 1, rho, j = rho u, u, non-equilibrium
// stress N = P - rho u u.
struct CellIn {
  float dr, rho, j[3], u[3], N[6];  // N order xx, yy, zz, xy, xz, yz
};

// FP32 state (rho - 1, j, P) -> cell (u = j / rho, N = P - j u).
__device__ inline CellIn cell_from_moments(const float m[10]) {
  CellIn c;
  c.dr = m[0];
  c.rho = 1.0f + m[0];
  c.j[0] = m[1];
  c.j[1] = m[2];
  c.j[2] = m[3];
  const float inv = 1.0f / c.rho;
  c.u[0] = m[1] * inv;
  c.u[1] = m[2] * inv;
  c.u[2] = m[3] * inv;
  c.N[0] = fmaf(-m[1], c.u[0], m[4]);
  c.N[1] = fmaf(-m[2], c.u[1], m[5]);
  c.N[2] = fmaf(-m[3], c.u[2], m[6]);
  c.N[3] = fmaf(-m[1], c.u[1], m[7]);
  c.N[4] = fmaf(-m[1], c.u[2], m[8]);
  c.N[5] = fmaf(-m[2], c.u[2], m[9]);
  return c;
}

// Q16 words -> cell.
__device__ inline CellIn cell_from_words(const uint32_t w[5]) {
  CellIn c;
  c.dr = fmaf(float(lo16(w[0])), Q_RHO_D, Q_DRHO_LO);
  c.rho = c.dr + 1.0f;
  c.u[0] = fmaf(float(hi16(w[0])), Q_U_D, Q_U_LO);
  c.u[1] = fmaf(float(lo16(w[1])), Q_U_D, Q_U_LO);
  c.u[2] = fmaf(float(hi16(w[1])), Q_U_D, Q_U_LO);
  c.N[0] = fmaf(float(lo16(w[2])), Q_N_D, Q_N_LO);
  c.N[1] = fmaf(float(hi16(w[2])), Q_N_D, Q_N_LO);
  c.N[2] = fmaf(float(lo16(w[3])), Q_N_D, Q_N_LO);
  c.N[3] = fmaf(float(hi16(w[3])), Q_N_D, Q_N_LO);
  c.N[4] = fmaf(float(lo16(w[4])), Q_N_D, Q_N_LO);
  c.N[5] = fmaf(float(hi16(w[4])), Q_N_D, Q_N_LO);
  c.j[0] = c.rho * c.u[0];
  c.j[1] = c.rho * c.u[1];
  c.j[2] = c.rho * c.u[2];
  return c;
}

// App. A, force-free, in non-equilibrium form: rho and u are kept and
// rho (S+ - u u) = (1 - 1/tau) dev(N).
__device__ inline void collide_neq(const float N[6], float om1, float Nn[6]) {
  const float t = (N[0] + N[1] + N[2]) * (1.0f / 3.0f);
  Nn[0] = om1 * (N[0] - t);
  Nn[1] = om1 * (N[1] - t);
  Nn[2] = om1 * (N[2] - t);
  Nn[3] = om1 * N[3];
  Nn[4] = om1 * N[4];
  Nn[5] = om1 * N[5];
}

// Channel order of the 17 coefficients A_nml (n along x, m along y, l along z).
enum {
  A000, A100, A010, A001, A200, A020, A002, A110, A101, A011,
  A210, A120, A201, A102, A021, A012, A111, NA
};

// Coefficients of h(rho, u, S) with rho S = rho u u + Nn (post-collision neq
// Nn) in the separable basis, each axis index scaled by s_0 = 1, s_1 = 1/3,
// s_2 = 1/9 relative to the Hermite normalisation 1, 3, 9/2 (so per index
// 1, 1, 1/2 times the raw Hermite coefficient):
//   A000 = rho - 1, A100 = jx, A200 = a2_xx / 2, A110 = a2_xy,
//   A210 = a3_xxy / 2, A111 = a3_xyz,
// with a2 = rho u u + Nn and a3 = rho T, rho T_aab = u_b a2_aa + 2 Nn_ab u_a,
// rho T_xyz = u_z a2_xy + Nn_xz u_y + Nn_yz u_x (the third-order term of
// Eq. three_order_f with T built from S = u u + Nn / rho).  The scaling makes
// every constant of the 1D passes below either exact or chosen so that the
// conservation and orthogonality identities hold exactly in float.
__device__ inline void hermite_coeffs(float dr, const float j[3], const float u[3], const float Nn[6], float A[NA]) {
  const float jx = j[0], jy = j[1], jz = j[2];
  const float hxx = 0.5f * fmaf(jx, u[0], Nn[0]);
  const float hyy = 0.5f * fmaf(jy, u[1], Nn[1]);
  const float hzz = 0.5f * fmaf(jz, u[2], Nn[2]);
  const float xy = fmaf(jx, u[1], Nn[3]);
  const float xz = fmaf(jx, u[2], Nn[4]);
  const float yz = fmaf(jy, u[2], Nn[5]);
  A[A000] = dr;
  A[A100] = jx;
  A[A010] = jy;
  A[A001] = jz;
  A[A200] = hxx;
  A[A020] = hyy;
  A[A002] = hzz;
  A[A110] = xy;
  A[A101] = xz;
  A[A011] = yz;
  A[A210] = fmaf(u[1], hxx, Nn[3] * u[0]);  // xxy
  A[A120] = fmaf(u[0], hyy, Nn[3] * u[1]);  // yyx
  A[A201] = fmaf(u[2], hxx, Nn[4] * u[0]);  // xxz
  A[A102] = fmaf(u[0], hzz, Nn[4] * u[2]);  // zzx
  A[A021] = fmaf(u[2], hyy, Nn[5] * u[1]);  // yyz
  A[A012] = fmaf(u[1], hzz, Nn[5] * u[2]);  // zzy
  A[A111] = fmaf(u[2], xy, fmaf(Nn[4], u[1], Nn[5] * u[0]));
}

// ------------------------------------------------- 1D reconstruct / project ---
// Along one axis, a group of up to three channels (i0, i1, i2) at a cell gives
// the distributions leaving it in directions 0, +1, -1 (D1Q3 weights 2/3, 1/6):
//   f0  = 2/3 i0 - 2 i2
//   f+- = 1/6 i0 +- 1/2 i1 + i2
// (with the index scaling above).  After the shift (F+ from the cell at -1,
// F- from the cell at +1) the projections are the moments 1, c, c^2 - 1/3:
//   o0 = F0 + F+ + F-,  o1 = F+ - F-,  o2 = 2/3 (F+ + F-) - 1/3 F0.
// In float, C6 = fl(1/6), C0 = 1 - 2 C6, R3 = fl(1/3) = 2 C6, P3 = 1 - R3 are
// exact relations, so C0 + 2 C6 = 1 (mass and momentum keep their value),
// P3 (2 C6) - R3 C0 = 0 (a uniform density makes no stress) and
// 2 (P3 + R3) = 2 (the second-moment channel keeps its value) hold exactly.
constexpr float C6 = 1.0f / 6.0f;
constexpr float C0 = 1.0f - 2.0f * C6;
constexpr float R3 = 1.0f / 3.0f;
constexpr float P3 = 1.0f - R3;

__device__ inline void recon3(float i0, float i1, float i2, float& f0, float& fp, float& fm) {
  f0 = fmaf(C0, i0, -2.0f * i2);
  const float q = fmaf(C6, i0, i2);
  fp = fmaf(0.5f, i1, q);
  fm = fmaf(-0.5f, i1, q);
}
__device__ inline void recon2(float i0, float i1, float& f0, float& fp, float& fm) {
  f0 = C0 * i0;
  const float q = C6 * i0;
  fp = fmaf(0.5f, i1, q);
  fm = fmaf(-0.5f, i1, q);
}
__device__ inline void recon1(float i0, float& f0, float& fp, float& fm) {
  f0 = C0 * i0;
  fp = C6 * i0;
  fm = fp;
}
__device__ inline void proj3(float F0, float Fp, float Fm, float& o0, float& o1, float& o2) {
  const float s = Fp + Fm;
  o0 = F0 + s;
  o1 = Fp - Fm;
  o2 = fmaf(P3, s, -R3 * F0);
}
__device__ inline void proj2(float F0, float Fp, float Fm, float& o0, float& o1) {
  o0 = F0 + (Fp + Fm);
  o1 = Fp - Fm;
}
__device__ inline float proj1(float F0, float Fp, float Fm) { return F0 + (Fp + Fm); }

// ------------------------------------------------------------ int helpers ---
__device__ inline int wrapi(int v, int n) {
  int r = v % n;
  return r < 0 ? r + n : r;
}

}  // namespace lbm
