// lbm_adjoint.hip -- adjoint of one FP32 step: lam(t) = J(m(t))^T lam(t+1).
//
// The step is m(t+1) = S(A(m(t))) with A the per-cell map (decode, App. A
// collision, Hermite coefficients) and S the linear pull-stream + projection,
// which factorises into three commuting 1D passes.  Its adjoint is
// lam(t) = A'(m)^T S^T lam(t+1): the transposed 1D passes (adjoint of the
// projection, the shift reversed, adjoint of the reconstruction) followed by
// the per-cell transpose of A' (lbm_device.h, coeffs_T).  The boundary pass
// overwrote the listed solid cells with rest, so the fluid adjoint reads lam(t+1) as zero
// there; the boundary pass's corrections of changed links are then added by
// two small kernels (adjoint_bounce_kernel, adjoint_face_kernel).
//
// The fluid adjoint uses the forward pass's tiling and work split (64-wide
// tiles of 8 or 13 rows, phase-aligned z segments): y pass first (the halo
// rows only load and take the first transposed projection), x pass with the
// halo-column wavefront, z pass in a register window.
#include "lbm_device.h"
#include "lbm_internal.h"

namespace lbm {

namespace {

constexpr int RW = 64;

template <int TYR>
struct AdjLds {
  float ly[9][TYR + 2][RW];   // y movers of 6 groups (9 values: 3 groups carry one value)
  float lyc[9][2][16];
  float lx[15][TYR][RW + 2];  // x movers of 9 groups (15 values)
};

__device__ inline int wrap1(int v, int n) { return v < 0 ? v + n : (v >= n ? v - n : v); }

__device__ inline void load10(const float* const p[10], uint32_t cell, float v[10]) {
#pragma unroll
  for (int k = 0; k < 10; ++k) v[k] = p[k][cell];
}

}  // namespace

template <int TYR>
__global__ void __launch_bounds__((TYR + 3) * RW) adjoint_fluid_kernel(AdjParams a, int ntx, int nty, int nseg,
                                                                       int nwg) {
  constexpr int NRW = TYR + 2;
  __shared__ AdjLds<TYR> L;
  const int nx = a.g.nx, ny = a.g.ny, nz = a.g.nz;
  const int wave = int(threadIdx.x) >> 6, lane = int(threadIdx.x) & 63;
  const bool colw = wave == NRW;
  int r, dx, side = 0;
  bool active = true;
  if (!colw) {
    r = wave;
    dx = lane;
  } else {
    side = lane >> 5;
    r = lane & 31;
    active = r < NRW;
    if (!active) r = NRW - 1;
    dx = side ? RW : -1;
  }
  const bool inner = r >= 1 && r <= TYR;
  const bool compute = !colw && inner;

  const int ntiles = ntx * nty;
  const int items = ntiles * nseg;
  const uint32_t plane = uint32_t(nx) * uint32_t(ny);

  // the same phase-aligned, XCD-grouped (tile, z segment) items as the forward pass
  for (int q = xcd_logical_block(int(blockIdx.x), nwg); q < items; q += nwg) {
    const int t = q % ntiles, sg = q / ntiles;
    const int za = int(int64_t(nz) * sg / nseg);
    const int zb = int(int64_t(nz) * (sg + 1) / nseg);
    const int x0 = (t % ntx) * RW, y0 = (t / ntx) * TYR;
    const int gx = x0 + dx, gy = y0 - 1 + r;
    const int xw = wrapi(gx, nx), yw = wrapi(gy, ny);
    const uint32_t row = uint32_t(xw) + uint32_t(nx) * uint32_t(yw);
    const bool own = compute && gx < nx && gy < ny;

    float w0[8], wm1[8], wm2[8];  // z window: G0 of the previous plane, G- of the previous two
#pragma unroll
    for (int g = 0; g < 8; ++g) w0[g] = wm1[g] = wm2[g] = 0.0f;
    // the next plane's adjoint input and flag in flight while this one is computed
    float gn[10];
    uint8_t fn;
    {
      const uint32_t c0 = row + plane * uint32_t(wrap1(za - 1, nz));
      load10(a.lam_in, c0, gn);
      fn = a.flags[c0];
    }
    uint8_t fprev = 0;  // flag of plane p - 1
    for (int p = za - 1; p <= zb; ++p) {
      float g[10];
#pragma unroll
      for (int k = 0; k < 10; ++k) g[k] = gn[k];
      const uint8_t fl = fn;
      if (p + 1 <= zb) {
        const uint32_t c1 = row + plane * uint32_t(wrap1(p + 1, nz));
        load10(a.lam_in, c1, gn);
        fn = a.flags[c1];
      }
      if (fl == 2) {  // a solid cell's new moments are overwritten with rest: no dependence
#pragma unroll
        for (int k = 0; k < 10; ++k) g[k] = 0.0f;
      }
      // forward state of plane p - 1, completed at the end of this iteration
      float mq[10];
      if (compute && p > za) load10(a.m, row + plane * uint32_t(p - 1), mq);

      // ---- transposed y pass: groups (a, c) with outputs b; movers to the y neighbours
      // g order: rho(000) jx(100) jy(010) jz(001) Pxx(200) Pyy(020) Pzz(002) Pxy(110) Pxz(101) Pyz(011)
      float G0[6], Gp[6], Gm[6];
      projT3(g[0], g[2], g[5], G0[0], Gp[0], Gm[0]);  // (0,0): b = 0, 1, 2
      projT2(g[1], g[7], G0[1], Gp[1], Gm[1]);        // (1,0): b = 0, 1
      projT1(g[4], G0[2], Gp[2], Gm[2]);              // (2,0)
      projT2(g[3], g[9], G0[3], Gp[3], Gm[3]);        // (0,1)
      projT1(g[8], G0[4], Gp[4], Gm[4]);              // (1,1)
      projT1(g[6], G0[5], Gp[5], Gm[5]);              // (0,2)
      {
        const float mv[9] = {Gp[0], Gm[0], Gp[1], Gm[1], Gp[3], Gm[3], G0[2], G0[4], G0[5]};
        if (!colw) {
#pragma unroll
          for (int k = 0; k < 9; ++k) L.ly[k][r][lane] = mv[k];
        } else if (active) {
#pragma unroll
          for (int k = 0; k < 9; ++k) L.lyc[k][side][r] = mv[k];
        }
      }
      __syncthreads();

      float Y[6][3];  // Y[group (a, c)][m]
      float H0[9];    // G0 of the x groups (m, c), kept across the barrier
      if (inner) {
        float up[9], dn[9];  // values of the cells at y + 1 (up) and y - 1 (dn)
        if (!colw) {
#pragma unroll
          for (int k = 0; k < 9; ++k) {
            up[k] = L.ly[k][r + 1][lane];
            dn[k] = L.ly[k][r - 1][lane];
          }
        } else {
#pragma unroll
          for (int k = 0; k < 9; ++k) {
            up[k] = L.lyc[k][side][r + 1];
            dn[k] = L.lyc[k][side][r - 1];
          }
        }
        // g_f+(y) = G+(y + 1), g_f-(y) = G-(y - 1)
        reconT3(G0[0], up[0], dn[1], Y[0][0], Y[0][1], Y[0][2]);
        reconT3(G0[1], up[2], dn[3], Y[1][0], Y[1][1], Y[1][2]);
        reconT3(G0[2], up[6], dn[6], Y[2][0], Y[2][1], Y[2][2]);
        reconT3(G0[3], up[4], dn[5], Y[3][0], Y[3][1], Y[3][2]);
        reconT3(G0[4], up[7], dn[7], Y[4][0], Y[4][1], Y[4][2]);
        reconT3(G0[5], up[8], dn[8], Y[5][0], Y[5][1], Y[5][2]);
        // ---- transposed x pass: groups (m, c) with outputs a; 15 mover values
        // per cell: for each m, (G+, G-) of c = 0, (G+, G-) of c = 1, G of c = 2
        float mv[15];
#pragma unroll
        for (int m = 0; m < 3; ++m) {
          float hp, hm;
          projT3(Y[0][m], Y[1][m], Y[2][m], H0[3 * m + 0], hp, hm);  // c = 0: a = 0, 1, 2
          mv[5 * m + 0] = hp;
          mv[5 * m + 1] = hm;
          projT2(Y[3][m], Y[4][m], H0[3 * m + 1], hp, hm);  // c = 1: a = 0, 1
          mv[5 * m + 2] = hp;
          mv[5 * m + 3] = hm;
          H0[3 * m + 2] = Y[5][m];  // c = 2: a = 0 (G0 = G+ = G-)
          mv[5 * m + 4] = Y[5][m];
        }
        if (!colw) {
#pragma unroll
          for (int k = 0; k < 15; ++k) L.lx[k][r - 1][lane + 1] = mv[k];
        } else if (active) {
          const int col = side ? RW + 1 : 0;
#pragma unroll
          for (int k = 0; k < 15; ++k) L.lx[k][r - 1][col] = mv[k];
        }
      }
      __syncthreads();

      if (compute) {
        // neighbours at x + 1 (right) and x - 1 (left): g_f+(x) = G+(x + 1), g_f-(x) = G-(x - 1)
        float rt[15], lt[15];
#pragma unroll
        for (int k = 0; k < 15; ++k) {
          rt[k] = L.lx[k][r - 1][lane + 2];
          lt[k] = L.lx[k][r - 1][lane];
        }
        float xn[3][3][3];  // xn[m][c][n]
#pragma unroll
        for (int m = 0; m < 3; ++m) {
          const int o = 5 * m;
          if (m < 2) {
            reconT3(H0[3 * m + 0], rt[o + 0], lt[o + 1], xn[m][0][0], xn[m][0][1], xn[m][0][2]);
            reconT3(H0[3 * m + 1], rt[o + 2], lt[o + 3], xn[m][1][0], xn[m][1][1], xn[m][1][2]);
            reconT3(H0[3 * m + 2], rt[o + 4], lt[o + 4], xn[m][2][0], xn[m][2][1], xn[m][2][2]);
          } else {
            reconT2(H0[3 * m + 0], rt[o + 0], lt[o + 1], xn[m][0][0], xn[m][0][1]);
            reconT2(H0[3 * m + 1], rt[o + 2], lt[o + 3], xn[m][1][0], xn[m][1][1]);
            reconT2(H0[3 * m + 2], rt[o + 4], lt[o + 4], xn[m][2][0], xn[m][2][1]);
            xn[m][0][2] = xn[m][1][2] = xn[m][2][2] = 0.0f;
          }
        }
        float X[8][3];  // X[(n, m) group][c]
        // z groups (n, m): (0,0) (1,0) (0,1) (2,0) (0,2) (1,1) (2,1) (1,2)
        const int gn[8] = {0, 1, 0, 2, 0, 1, 2, 1};
        const int gm[8] = {0, 0, 1, 0, 2, 1, 1, 2};
#pragma unroll
        for (int q = 0; q < 8; ++q) {
          X[q][0] = xn[gm[q]][0][gn[q]];
          X[q][1] = xn[gm[q]][1][gn[q]];
          X[q][2] = xn[gm[q]][2][gn[q]];
        }
        // ---- transposed z pass
        float Z0[8], Zp[8], Zm[8];
#pragma unroll
        for (int q = 0; q < 8; ++q) projT3(X[q][0], X[q][1], X[q][2], Z0[q], Zp[q], Zm[q]);
        if (p > za) {  // plane p - 1: g_f0 = G0(p - 1), g_f+ = G+(p), g_f- = G-(p - 2)
          float gA[NA];
          reconT3(w0[0], Zp[0], wm2[0], gA[A000], gA[A001], gA[A002]);
          reconT3(w0[1], Zp[1], wm2[1], gA[A100], gA[A101], gA[A102]);
          reconT3(w0[2], Zp[2], wm2[2], gA[A010], gA[A011], gA[A012]);
          reconT2(w0[3], Zp[3], wm2[3], gA[A200], gA[A201]);
          reconT2(w0[4], Zp[4], wm2[4], gA[A020], gA[A021]);
          reconT2(w0[5], Zp[5], wm2[5], gA[A110], gA[A111]);
          gA[A210] = reconT1(w0[6], Zp[6], wm2[6]);
          gA[A120] = reconT1(w0[7], Zp[7], wm2[7]);
          if (own) {
            const uint32_t qc = row + plane * uint32_t(p - 1);
            float out[10];
#pragma unroll
            for (int k = 0; k < 10; ++k) out[k] = 0.0f;
            if (fprev != 2) {
              const CellLin cl = cell_lin(mq, a.om1, nullptr);
              coeffs_T(cl, a.om1, gA, true, out);
            }
#pragma unroll
            for (int k = 0; k < 10; ++k) a.lam_out[k][qc] = out[k];
          }
        }
#pragma unroll
        for (int q = 0; q < 8; ++q) {
          wm2[q] = wm1[q];
          wm1[q] = Zm[q];
          w0[q] = Z0[q];
        }
      }
      fprev = fl;
    }
  }
}

// --------------------------------------------------------- boundary adjoint ---

// basis values P_n(c) in the index scaling of hermite_coeffs (as in eval_link)
__device__ inline void basis1_adj(int c, float P[3]) {
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

// gA += gf * d f_(cx,cy,cz) / d A
__device__ inline void add_basis(float gf, int cx, int cy, int cz, float gA[NA]) {
  float px[3], py[3], pz[3];
  basis1_adj(cx, px);
  basis1_adj(cy, py);
  basis1_adj(cz, pz);
  gA[A000] += gf * px[0] * py[0] * pz[0];
  gA[A100] += gf * px[1] * py[0] * pz[0];
  gA[A010] += gf * px[0] * py[1] * pz[0];
  gA[A001] += gf * px[0] * py[0] * pz[1];
  gA[A200] += gf * px[2] * py[0] * pz[0];
  gA[A020] += gf * px[0] * py[2] * pz[0];
  gA[A002] += gf * px[0] * py[0] * pz[2];
  gA[A110] += gf * px[1] * py[1] * pz[0];
  gA[A101] += gf * px[1] * py[0] * pz[1];
  gA[A011] += gf * px[0] * py[1] * pz[1];
  gA[A210] += gf * px[2] * py[1] * pz[0];
  gA[A120] += gf * px[1] * py[2] * pz[0];
  gA[A201] += gf * px[2] * py[0] * pz[1];
  gA[A102] += gf * px[1] * py[0] * pz[2];
  gA[A021] += gf * px[0] * py[2] * pz[1];
  gA[A012] += gf * px[0] * py[1] * pz[2];
  gA[A111] += gf * px[1] * py[1] * pz[1];
}

// gf = d(new moments of a cell)/d f_i . g for link c = (cx, cy, cz)
__device__ inline float link_dot(const float g[10], int cx, int cy, int cz) {
  const float fx = float(cx), fy = float(cy), fz = float(cz);
  float gf = g[0] + fx * g[1] + fy * g[2] + fz * g[3];
  gf = fmaf(fx * fx - R3, g[4], gf);
  gf = fmaf(fy * fy - R3, g[5], gf);
  gf = fmaf(fz * fz - R3, g[6], gf);
  gf = fmaf(fx * fy, g[7], gf);
  gf = fmaf(fx * fz, g[8], gf);
  gf = fmaf(fy * fz, g[9], gf);
  return gf;
}

// The adjoint writes the step as a fully periodic pull plus, at each listed
// fluid cell, (new - pulled) distribution on every changed link (the same
// function as the forward passes, whatever share of the faces the forward
// fluid pass takes on itself).  The fluid adjoint carries the periodic pull
// (the solid sources' share being discarded at those cells).  What remains:
//   - bounce-back link i of x: + f+_opp(i)(x), through x's own coefficients;
//     the pulled rest state is a constant;
//   - inflow link of x (cx = 1): + f+_i with x's inflow coefficients, - f+_i of
//     the periodic image (nx-1, y-cy, z-cz);
//   - outflow link of x (cx = -1): + f+_i of the face cell (nx-1, y-cy, z-cz),
//     - f+_i of the periodic image (0, y-cy, z-cz).
// The first is added by adjoint_bounce_kernel (one lane per listed fluid
// cell, its own data only); the face terms by adjoint_face_kernel, a gather
// over the two x-face planes.  Both add to what the fluid adjoint wrote (one
// writer per cell in each kernel, no atomics).
__global__ void __launch_bounds__(256) adjoint_bounce_kernel(AdjParams a, const uint32_t* __restrict__ cells,
                                                             const uint32_t* __restrict__ bits, int count) {
  const int e = int(blockIdx.x) * blockDim.x + threadIdx.x;
  if (e >= count) return;
  // The lane's loads go out in two round trips: its entry, then everything
  // at its cell (the adjoint input, the state and the output it adds to,
  // read up front because the compiler cannot tell that the output planes
  // do not alias the others; written back once at the end).  An entry with
  // no bounce-back link (a face cell) adds zero: it is not skipped, so that
  // no branch waits for the entry's bits before the cell's loads are issued.
  const uint32_t b0 = bits[e], x = cells[e];
  float g[10], m[10], acc[10];
  load10(a.lam_in, x, g);
  load10(a.m, x, m);
#pragma unroll
  for (int k = 0; k < 10; ++k) acc[k] = a.lam_out[k][x];
  uint32_t bb = b0 & 0x7FFFFFFu & ~(1u << 13);
  float gA[NA];
#pragma unroll
  for (int k = 0; k < NA; ++k) gA[k] = 0.0f;
  while (bb) {
    const int i = __ffs(bb) - 1;
    bb &= bb - 1u;
    const int cx = i % 3 - 1, cy = (i / 3) % 3 - 1, cz = i / 9 - 1;
    add_basis(link_dot(g, cx, cy, cz), -cx, -cy, -cz, gA);
  }
  float out[10];
#pragma unroll
  for (int k = 0; k < 10; ++k) out[k] = 0.0f;
  const CellLin cl = cell_lin(m, a.om1, nullptr);
  coeffs_T(cl, a.om1, gA, true, out);
#pragma unroll
  for (int k = 0; k < 10; ++k) a.lam_out[k][x] = acc[k] + out[k];
}

// One thread per cell of the two x-face planes (inflow on: x = 0 inflow,
// x = nx - 1 outflow).  s at x = nx - 1 is the periodic image of the inflow
// cells (0, y+cy, z+cz) (-) and the zero-gradient source of the outflow cells
// (nx-1, y+cy, z+cz) (+); s at x = 0 is the periodic image of the outflow
// cells (nx-1, y+cy, z+cz) (-) and takes its own inflow links (+, through its
// inflow coefficients).  Every face cell is listed (faces hold no solids).
__global__ void __launch_bounds__(256) adjoint_face_kernel(AdjParams a) {
  const int nx = a.g.nx, ny = a.g.ny, nz = a.g.nz;
  const int t = int(blockIdx.x) * blockDim.x + threadIdx.x;
  if (t >= 2 * ny * nz) return;
  const bool out_face = t >= ny * nz;
  const int yz = out_face ? t - ny * nz : t;
  const int y = yz % ny, z = yz / ny;
  const int x = out_face ? nx - 1 : 0;
  const uint32_t s = uint32_t(x) + uint32_t(nx) * (uint32_t(y) + uint32_t(ny) * uint32_t(z));
  // the output this lane adds to, read before any other work (see
  // adjoint_bounce_kernel) and written back once
  float acc[10];
#pragma unroll
  for (int k = 0; k < 10; ++k) acc[k] = a.lam_out[k][s];
  float gA[NA], gin[NA];
#pragma unroll
  for (int k = 0; k < NA; ++k) gA[k] = gin[k] = 0.0f;
  for (int cz = -1; cz <= 1; ++cz) {
    for (int cy = -1; cy <= 1; ++cy) {
      const uint32_t yzn = uint32_t(nx) * (uint32_t(wrapi(y + cy, ny)) + uint32_t(ny) * uint32_t(wrapi(z + cz, nz)));
      float g[10];
      if (out_face) {
        load10(a.lam_in, yzn, g);  // inflow cell (0, y+cy, z+cz): s is its image on link (1, cy, cz)
        add_basis(-link_dot(g, 1, cy, cz), 1, cy, cz, gA);
        load10(a.lam_in, uint32_t(nx - 1) + yzn, g);  // outflow cell reading s on link (-1, cy, cz)
        add_basis(link_dot(g, -1, cy, cz), -1, cy, cz, gA);
      } else {
        load10(a.lam_in, uint32_t(nx - 1) + yzn, g);  // outflow cell: s is its image on link (-1, cy, cz)
        add_basis(-link_dot(g, -1, cy, cz), -1, cy, cz, gA);
      }
    }
  }
  float m[10];
  load10(a.m, s, m);
  float out[10];
#pragma unroll
  for (int k = 0; k < 10; ++k) out[k] = 0.0f;
  {
    const CellLin cl = cell_lin(m, a.om1, nullptr);
    coeffs_T(cl, a.om1, gA, true, out);
  }
  if (!out_face) {  // own inflow links
    float g[10];
    load10(a.lam_in, s, g);
    for (int cz = -1; cz <= 1; ++cz)
      for (int cy = -1; cy <= 1; ++cy) add_basis(link_dot(g, 1, cy, cz), 1, cy, cz, gin);
    const CellLin cl = cell_lin(m, a.om1, a.u_in);
    coeffs_T(cl, a.om1, gin, false, out);
  }
#pragma unroll
  for (int k = 0; k < 10; ++k) a.lam_out[k][s] = acc[k] + out[k];
}

// flags: 1 = listed fluid cell, 2 = solid cell, 0 = other fluid cell
__global__ void adjoint_flags_kernel(const uint8_t* __restrict__ mask, uint32_t N, const uint32_t* __restrict__ cells,
                                     const uint32_t* __restrict__ bits, int count, uint8_t* __restrict__ flags) {
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < N) flags[i] = (mask && mask[i]) ? 2 : 0;
  (void)cells;
  (void)bits;
  (void)count;
}

__global__ void adjoint_flags_list_kernel(const uint32_t* __restrict__ cells, const uint32_t* __restrict__ bits,
                                          int count, uint8_t* __restrict__ flags) {
  const int e = int(blockIdx.x * blockDim.x + threadIdx.x);
  if (e >= count) return;
  if (!(bits[e] & BIT_SOLID)) flags[cells[e]] = 1;
}

// Adjoint of the equilibrium initialisation m = (rho, rho u, rho u u):
// grad_rho = lam_rho + u . lam_j + u u : lam_P, grad_u = rho (lam_j + 2 sym(lam_P) u).
__global__ void equilibrium_vjp_kernel(const float* __restrict__ rho, const float* __restrict__ u,
                                       const float* __restrict__ lam, const uint8_t* __restrict__ mask, uint32_t N,
                                       float* __restrict__ grho, float* __restrict__ gu) {
  const uint32_t c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= N) return;
  float gr = 0.0f, g0 = 0.0f, g1 = 0.0f, g2 = 0.0f;
  if (!(mask && mask[c])) {
    const float r = rho[c];
    const float ux = u[c], uy = u[size_t(N) + c], uz = u[2 * size_t(N) + c];
    float l[10];
#pragma unroll
    for (int k = 0; k < 10; ++k) l[k] = lam[size_t(k) * N + c];
    gr = l[0] + ux * l[1] + uy * l[2] + uz * l[3] + ux * ux * l[4] + uy * uy * l[5] + uz * uz * l[6] +
         ux * uy * l[7] + ux * uz * l[8] + uy * uz * l[9];
    g0 = r * (l[1] + 2.0f * ux * l[4] + uy * l[7] + uz * l[8]);
    g1 = r * (l[2] + 2.0f * uy * l[5] + ux * l[7] + uz * l[9]);
    g2 = r * (l[3] + 2.0f * uz * l[6] + ux * l[8] + uy * l[9]);
  }
  if (grho) grho[c] = gr;
  gu[c] = g0;
  gu[size_t(N) + c] = g1;
  gu[2 * size_t(N) + c] = g2;
}

namespace {
int cus() {
  int dev = 0, n = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 256;
  if (hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || n <= 0) return 256;
  return n;
}
}  // namespace

hipError_t launch_adjoint(const AdjParams& p, int rows, const uint32_t* cells, const uint32_t* bits, int nfluid,
                          hipStream_t s) {
  // the forward pass's split at one of the two compiled tile heights (8 unless
  // 13 is asked for: the 13-row tile needs more registers than fit)
  const FluidPlan c = fluid_plan(p.g, rows == 13 ? 13 : 8, cus(), /*allow_tail=*/false);
  if (c.rows == 8)
    hipLaunchKernelGGL(adjoint_fluid_kernel<8>, dim3(uint32_t(c.nwg)), dim3(11 * RW), 0, s, p, c.ntx, c.nty, c.nseg,
                       c.nwg);
  else
    hipLaunchKernelGGL(adjoint_fluid_kernel<13>, dim3(uint32_t(c.nwg)), dim3(16 * RW), 0, s, p, c.ntx, c.nty, c.nseg,
                       c.nwg);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  if (nfluid > 0) {
    hipLaunchKernelGGL(adjoint_bounce_kernel, dim3((nfluid + 255) / 256), dim3(256), 0, s, p, cells, bits, nfluid);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  if (p.g.inflow) {
    const int n = 2 * p.g.ny * p.g.nz;
    hipLaunchKernelGGL(adjoint_face_kernel, dim3((n + 255) / 256), dim3(256), 0, s, p);
    e = hipGetLastError();
  }
  return e;
}

hipError_t launch_adjoint_flags(const uint8_t* mask, int64_t N, const uint32_t* cells, const uint32_t* bits,
                                int count, uint8_t* flags, hipStream_t s) {
  hipLaunchKernelGGL(adjoint_flags_kernel, dim3(uint32_t((N + 255) / 256)), dim3(256), 0, s, mask, uint32_t(N), cells,
                     bits, count, flags);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess || count <= 0) return e;
  hipLaunchKernelGGL(adjoint_flags_list_kernel, dim3((count + 255) / 256), dim3(256), 0, s, cells, bits, count, flags);
  return hipGetLastError();
}

hipError_t launch_equilibrium_vjp(const float* rho, const float* u, const float* lam, const uint8_t* mask, int64_t N,
                                  float* grho, float* gu, hipStream_t s) {
  hipLaunchKernelGGL(equilibrium_vjp_kernel, dim3(uint32_t((N + 255) / 256)), dim3(256), 0, s, rho, u, lam, mask,
                     uint32_t(N), grho, gu);
  return hipGetLastError();
}

}  // namespace lbm
