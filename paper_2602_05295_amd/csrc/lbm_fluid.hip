// lbm_fluid.hip -- the fused fluid pass (Sec. 4.2, Alg. 2) for gfx950.
//
// One workgroup owns an x-y tile of (FTX-2) x (FTY-2) output cells plus a
// one-cell halo ring, and marches through a chunk of z planes.  Per plane each
// thread loads its cell's moments once (coalesced along x), collides in moment
// space (App. A) and forms the 17 Hermite coefficients; then
//   x pass: reconstruct the x-directional distributions of 8 groups, exchange
//           the +x / -x movers with the x neighbours through LDS, project;
//   y pass: the same on 9 groups with the y neighbours;
//   z pass: the same on 6 groups, with the z neighbours held in registers
//           from the previous planes of the march (no exchange at all).
// Only the ten new moments are written, so a cell's state crosses HBM once in
// and once out per step.  Every axis is treated as periodic here; faces and
// walls are overwritten afterwards by the boundary pass.
#include "lbm_device.h"
#include "lbm_internal.h"

namespace lbm {

constexpr int FTX = 32;  // threads along x (30 outputs)
constexpr int FTY = 16;  // threads along y (14 outputs)

template <int FMT>
__device__ inline CellIn load_cell(const StepParams& a, uint32_t off) {
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

// Writes the new moments of one cell: dr = rho - 1, j, P (xx yy zz xy xz yz).
template <int FMT>
__device__ inline void store_cell(const StepParams& a, uint32_t cell, float dr, const float j[3], const float P[6]) {
  const uint32_t off = cell * 4u;
  if constexpr (FMT == FMT_F32) {
    const float v[10] = {dr, j[0], j[1], j[2], P[0], P[1], P[2], P[3], P[4], P[5]};
#pragma unroll
    for (int k = 0; k < 10; ++k) *reinterpret_cast<float*>(static_cast<char*>(a.out[k]) + off) = v[k];
  } else {
    const float rho = 1.0f + dr;
    const float inv = 1.0f / rho;
    const float u[3] = {j[0] * inv, j[1] * inv, j[2] * inv};
    const float N[6] = {fmaf(-j[0], u[0], P[0]), fmaf(-j[1], u[1], P[1]), fmaf(-j[2], u[2], P[2]),
                        fmaf(-j[0], u[1], P[3]), fmaf(-j[0], u[2], P[4]), fmaf(-j[1], u[2], P[5])};
    uint32_t h1 = 0, h2 = 0;
    const bool dith = a.dither != 0;
    if (dith) dither_words(cell, a.key, h1, h2);
    const uint32_t q0 = quantize(dr - Q_DRHO_LO, Q_RHO_S, half_plus_xi<0>(h1, h2, dith));
    const uint32_t q1 = quantize(u[0] - Q_U_LO, Q_U_S, half_plus_xi<1>(h1, h2, dith));
    const uint32_t q2 = quantize(u[1] - Q_U_LO, Q_U_S, half_plus_xi<2>(h1, h2, dith));
    const uint32_t q3 = quantize(u[2] - Q_U_LO, Q_U_S, half_plus_xi<3>(h1, h2, dith));
    const uint32_t q4 = quantize(N[0] - Q_N_LO, Q_N_S, half_plus_xi<4>(h1, h2, dith));
    const uint32_t q5 = quantize(N[1] - Q_N_LO, Q_N_S, half_plus_xi<5>(h1, h2, dith));
    const uint32_t q6 = quantize(N[2] - Q_N_LO, Q_N_S, half_plus_xi<6>(h1, h2, dith));
    const uint32_t q7 = quantize(N[3] - Q_N_LO, Q_N_S, half_plus_xi<7>(h1, h2, dith));
    const uint32_t q8 = quantize(N[4] - Q_N_LO, Q_N_S, half_plus_xi<8>(h1, h2, dith));
    const uint32_t q9 = quantize(N[5] - Q_N_LO, Q_N_S, half_plus_xi<9>(h1, h2, dith));
    *reinterpret_cast<uint32_t*>(static_cast<char*>(a.out[0]) + off) = q0 | (q1 << 16);
    *reinterpret_cast<uint32_t*>(static_cast<char*>(a.out[1]) + off) = q2 | (q3 << 16);
    *reinterpret_cast<uint32_t*>(static_cast<char*>(a.out[2]) + off) = q4 | (q5 << 16);
    *reinterpret_cast<uint32_t*>(static_cast<char*>(a.out[3]) + off) = q6 | (q7 << 16);
    *reinterpret_cast<uint32_t*>(static_cast<char*>(a.out[4]) + off) = q8 | (q9 << 16);
  }
}

template <int FMT>
__global__ void __launch_bounds__(FTX* FTY) fluid_kernel(StepParams a) {
  __shared__ float lx[16][FTY][FTX];  // x movers: (+, -) of 8 groups
  __shared__ float ly[18][FTY][FTX];  // y movers: (+, -) of 9 groups

  const int nx = a.g.nx, ny = a.g.ny, nz = a.g.nz;
  const int tx = threadIdx.x, ty = threadIdx.y;
  const int gx = int(blockIdx.x) * (FTX - 2) - 1 + tx;
  const int gy = int(blockIdx.y) * (FTY - 2) - 1 + ty;
  const int xw = wrapi(gx, nx), yw = wrapi(gy, ny);
  const bool own = tx >= 1 && tx <= FTX - 2 && ty >= 1 && ty <= FTY - 2 && gx < nx && gy < ny;
  const int txm = tx > 0 ? tx - 1 : 0, txp = tx < FTX - 1 ? tx + 1 : FTX - 1;
  const int tym = ty > 0 ? ty - 1 : 0, typ = ty < FTY - 1 ? ty + 1 : FTY - 1;
  const int z0 = int(blockIdx.z) * a.zchunk;
  const int z1 = min(z0 + a.zchunk, nz);
  const uint32_t plane = uint32_t(nx) * uint32_t(ny);
  const uint32_t row = uint32_t(xw) + uint32_t(nx) * uint32_t(yw);

  // z window: f+ of the plane two back, f+ and f0 of the previous plane
  float wp2[6], wp1[6], w0[6];
#pragma unroll
  for (int g = 0; g < 6; ++g) wp2[g] = wp1[g] = w0[g] = 0.0f;

  for (int p = z0 - 1; p <= z1; ++p) {
    const int zw = wrapi(p, nz);
    const uint32_t cell = row + plane * uint32_t(zw);
    const CellIn c = load_cell<FMT>(a, cell * 4u);
    float Nn[6];
    collide_neq(c.N, a.om1, Nn);
    float A[NA];
    hermite_coeffs(c.dr, c.j, c.u, Nn, A);

    // ---- x pass: groups (m, l) with inputs n = 0, 1, 2 along x
    float f0[8], fp[8], fm[8];
    recon3(A[A000], A[A100], A[A200], f0[0], fp[0], fm[0]);  // (0,0)
    recon3(A[A010], A[A110], A[A210], f0[1], fp[1], fm[1]);  // (1,0)
    recon3(A[A001], A[A101], A[A201], f0[2], fp[2], fm[2]);  // (0,1)
    recon2(A[A020], A[A120], f0[3], fp[3], fm[3]);           // (2,0)
    recon2(A[A002], A[A102], f0[4], fp[4], fm[4]);           // (0,2)
    recon2(A[A011], A[A111], f0[5], fp[5], fm[5]);           // (1,1)
    recon1(A[A021], f0[6], fp[6], fm[6]);                    // (2,1)
    recon1(A[A012], f0[7], fp[7], fm[7]);                    // (1,2)
#pragma unroll
    for (int g = 0; g < 8; ++g) {
      lx[2 * g][ty][tx] = fp[g];
      lx[2 * g + 1][ty][tx] = fm[g];
    }
    __syncthreads();
    float X[8][3];  // X[g][a] = channel (a, m, l)
#pragma unroll
    for (int g = 0; g < 8; ++g) proj3(f0[g], lx[2 * g][ty][txm], lx[2 * g + 1][ty][txp], X[g][0], X[g][1], X[g][2]);

    // ---- y pass: groups (a, l) with inputs m = 0, 1, 2 along y
    float y0[9], yp[9], ym[9];
#pragma unroll
    for (int a3 = 0; a3 < 3; ++a3) {
      recon3(X[0][a3], X[1][a3], X[3][a3], y0[3 * a3 + 0], yp[3 * a3 + 0], ym[3 * a3 + 0]);  // l = 0
      recon3(X[2][a3], X[5][a3], X[6][a3], y0[3 * a3 + 1], yp[3 * a3 + 1], ym[3 * a3 + 1]);  // l = 1
      recon2(X[4][a3], X[7][a3], y0[3 * a3 + 2], yp[3 * a3 + 2], ym[3 * a3 + 2]);            // l = 2
    }
#pragma unroll
    for (int h = 0; h < 9; ++h) {
      ly[2 * h][ty][tx] = yp[h];
      ly[2 * h + 1][ty][tx] = ym[h];
    }
    __syncthreads();
    float Y00[3], Y01[3], Y02[3], Y10[3], Y11[3], Y20[3];  // Yab[l] = channel (a, b, l)
#pragma unroll
    for (int l = 0; l < 3; ++l) {
      proj3(y0[l], ly[2 * l][tym][tx], ly[2 * l + 1][typ][tx], Y00[l], Y01[l], Y02[l]);
      proj2(y0[3 + l], ly[2 * (3 + l)][tym][tx], ly[2 * (3 + l) + 1][typ][tx], Y10[l], Y11[l]);
      Y20[l] = proj1(y0[6 + l], ly[2 * (6 + l)][tym][tx], ly[2 * (6 + l) + 1][typ][tx]);
    }

    // ---- z pass: groups (a, b) = (0,0) (1,0) (0,1) (2,0) (1,1) (0,2), inputs l = 0, 1, 2
    float zf0[6], zfp[6], zfm[6];
    recon3(Y00[0], Y00[1], Y00[2], zf0[0], zfp[0], zfm[0]);
    recon3(Y10[0], Y10[1], Y10[2], zf0[1], zfp[1], zfm[1]);
    recon3(Y01[0], Y01[1], Y01[2], zf0[2], zfp[2], zfm[2]);
    recon3(Y20[0], Y20[1], Y20[2], zf0[3], zfp[3], zfm[3]);
    recon3(Y11[0], Y11[1], Y11[2], zf0[4], zfp[4], zfm[4]);
    recon3(Y02[0], Y02[1], Y02[2], zf0[5], zfp[5], zfm[5]);

    if (p > z0) {  // plane q = p - 1 is complete
      float dr, j[3], P[6];
      proj3(w0[0], wp2[0], zfm[0], dr, j[2], P[2]);  // (0,0,c): rho-1, jz, Pzz
      proj2(w0[1], wp2[1], zfm[1], j[0], P[4]);      // (1,0,c): jx, Pxz
      proj2(w0[2], wp2[2], zfm[2], j[1], P[5]);      // (0,1,c): jy, Pyz
      P[0] = proj1(w0[3], wp2[3], zfm[3]);           // Pxx
      P[3] = proj1(w0[4], wp2[4], zfm[4]);           // Pxy
      P[1] = proj1(w0[5], wp2[5], zfm[5]);           // Pyy
      if (own) store_cell<FMT>(a, row + plane * uint32_t(p - 1), dr, j, P);
    }
#pragma unroll
    for (int g = 0; g < 6; ++g) {
      wp2[g] = wp1[g];
      wp1[g] = zfp[g];
      w0[g] = zf0[g];
    }
  }
}

void fluid_tiling(const Geometry& g, dim3* grid, dim3* block, int* zchunk) {
  const int ntx = (g.nx + FTX - 3) / (FTX - 2);
  const int nty = (g.ny + FTY - 3) / (FTY - 2);
  const int tiles = ntx * nty;
  int chunks = (2048 + tiles - 1) / tiles;
  const int maxchunks = (g.nz + 7) / 8;
  if (chunks > maxchunks) chunks = maxchunks;
  if (chunks < 1) chunks = 1;
  int zc = (g.nz + chunks - 1) / chunks;
  chunks = (g.nz + zc - 1) / zc;
  *grid = dim3(ntx, nty, chunks);
  *block = dim3(FTX, FTY, 1);
  *zchunk = zc;
}

hipError_t launch_fluid(int fmt, const StepParams& p, hipStream_t s) {
  dim3 grid, block;
  int zc;
  fluid_tiling(p.g, &grid, &block, &zc);
  StepParams q = p;
  q.zchunk = zc;
  if (fmt == FMT_F32)
    hipLaunchKernelGGL(fluid_kernel<FMT_F32>, grid, block, 0, s, q);
  else
    hipLaunchKernelGGL(fluid_kernel<FMT_Q16>, grid, block, 0, s, q);
  return hipGetLastError();
}

}  // namespace lbm
