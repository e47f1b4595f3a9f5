// lbm_boundary_cell.h -- the boundary pass of one listed cell (device code
// shared by the single-domain and the batched boundary kernels).
//
// The rules are those of a listed fluid cell recomputed from scratch: each of
// its 27 incoming distributions is the pull-streamed f+ of its source, except
// on links whose source is solid (halfway bounce-back: f_i(x) = f+_opp(i)(x)),
// links entering through the inflow face (the moment boundary of Sec. 3.2
// with p on the face: rho^p = rho^x, u^p = u_in and the post-collision
// non-equilibrium stress of x) and links entering through the outflow face
// (zero gradient: f+_i(nx-1, y - c_y, z - c_z)).  Since the fluid pass already
// pulled every other link, the pass starts from the fluid pass's unrounded
// moments and replaces only the changed links.  The new moments are encoded
// once and overwrite what the fluid pass wrote, so each cell has one writer,
// no atomics and a single rounding.  Solid cells next to fluid are reset to
// rest.
#pragma once

#include "lbm_codec.h"

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
    uint32_t w[Codec<FMT>::W];
#pragma unroll
    for (int k = 0; k < Codec<FMT>::W; ++k)
      w[k] = *reinterpret_cast<const uint32_t*>(static_cast<const char*>(a.in[k]) + off);
    return Codec<FMT>::decode(w);
  }
}

template <int FMT>
__device__ inline void store_cell_b(const StepParams& a, uint32_t cell, float dr, const float j[3], const float P[6]) {
  const uint32_t off = cell * 4u;
  if constexpr (FMT == FMT_F32) {
    const float v[10] = {dr, j[0], j[1], j[2], P[0], P[1], P[2], P[3], P[4], P[5]};
#pragma unroll
    for (int k = 0; k < 10; ++k) *reinterpret_cast<float*>(static_cast<char*>(a.out[k]) + off) = v[k];
  } else {
    uint32_t w[Codec<FMT>::W];
    Codec<FMT>::encode(dr, j, P, cell, a.key, a.dither != 0, w);
#pragma unroll
    for (int k = 0; k < Codec<FMT>::W; ++k) *reinterpret_cast<uint32_t*>(static_cast<char*>(a.out[k]) + off) = w[k];
  }
}

// Post-collision moments of a cell: rho - 1, rho, j+, u+ and the
// non-equilibrium stress rho (S+ - u+ u+) (App. A, with the body force if any).
struct PostCell {
  float dr, rho, j[3], u[3], Nn[6];
};

template <int FMT>
__device__ inline PostCell post_cell(const StepParams& a, uint32_t q) {
  PostCell s;
  if constexpr (FMT != FMT_F32) {
    if (!a.force) {  // the arithmetic of the fluid pass
      uint32_t w[Codec<FMT>::W];
#pragma unroll
      for (int k = 0; k < Codec<FMT>::W; ++k)
        w[k] = *reinterpret_cast<const uint32_t*>(static_cast<const char*>(a.in[k]) + q * 4u);
      collide_codes<FMT>(w, a.nq_s, a.nq_d, a.nq_c, s.dr, s.rho, s.u, s.j, s.Nn);
      return s;
    }
  }
  const CellIn c = load_cell_b<FMT>(a, q);
  s.dr = c.dr;
  s.rho = c.rho;
  if (a.force) {
    collide_force(c, a.hF, a.om1, s.j, s.u, s.Nn);
  } else {
    collide_neq(c.N, a.om1, s.Nn);
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      s.j[k] = c.j[k];
      s.u[k] = c.u[k];
    }
  }
  return s;
}

// Coefficients of the moments (rho^p = rho^x, u^p, S^p = u^p u^p + (S^x -
// u^x u^x)) that Sec. 3.2 reconstructs at a boundary point p next to x: the
// inflow face (u^p = u_in) and the moment wall (u^p of the solid).
__device__ inline void boundary_point_coeffs(const PostCell& x, const float up[3], float A[NA]) {
  const float jp[3] = {x.rho * up[0], x.rho * up[1], x.rho * up[2]};
  hermite_coeffs(x.dr, jp, up, x.Nn, A);
}

// Velocity of object id at the midpoint p = x - c/2 of the link from cell
// (x, y, z) along -c: V + W x (p - C), positions taken from the fluid cell
// without wrapping.
__device__ inline void wall_velocity(const float* obj, int x, int y, int z, int cx, int cy, int cz, float u[3],
                                     float r[3]) {
  r[0] = float(x) - 0.5f * float(cx) - obj[0];
  r[1] = float(y) - 0.5f * float(cy) - obj[1];
  r[2] = float(z) - 0.5f * float(cz) - obj[2];
  const float* V = obj + 3;
  const float* W = obj + 6;
  u[0] = V[0] + (W[1] * r[2] - W[2] * r[1]);
  u[1] = V[1] + (W[2] * r[0] - W[0] * r[2]);
  u[2] = V[2] + (W[0] * r[1] - W[1] * r[0]);
}

// dm += (moments of link c) * df
__device__ inline void add_link(float m[10], int cx, int cy, int cz, float df) {
  const float fx = float(cx), fy = float(cy), fz = float(cz);
  m[0] += df;
  m[1] = fmaf(fx, df, m[1]);
  m[2] = fmaf(fy, df, m[2]);
  m[3] = fmaf(fz, df, m[3]);
  m[4] = fmaf(fx * fx - R3, df, m[4]);
  m[5] = fmaf(fy * fy - R3, df, m[5]);
  m[6] = fmaf(fz * fz - R3, df, m[6]);
  m[7] = fmaf(fx * fy, df, m[7]);
  m[8] = fmaf(fx * fz, df, m[8]);
  m[9] = fmaf(fy * fz, df, m[9]);
}

// Post-collision coefficients of the rest state as stored: FP32 rest is
// exactly zero; the 16-bit rest codes decode to a fixed state near rest.
// Every solid cell a fluid cell reads is listed, and listed solid cells hold
// these codes at the start of every step (the boundary pass writes them, and
// every way of setting the state keeps them), so the distribution the fluid
// pass pulled from a solid neighbour is a constant of its direction.
// With a body force the fluid pass collides the solid cells' rest state
// with the force as well, and so does this.
template <int FMT>
__device__ inline void rest_coeffs(const StepParams& a, float A[NA]) {
  CellIn c;
  if constexpr (FMT == FMT_F32) {
    if (!a.force) {
#pragma unroll
      for (int k = 0; k < NA; ++k) A[k] = 0.0f;
      return;
    }
    const float m[10] = {0.0f, 0.0f, 0.0f, 0.0f, 0.0f, 0.0f, 0.0f, 0.0f, 0.0f, 0.0f};
    c = cell_from_moments(m);
  } else {
    uint32_t w[Codec<FMT>::W];
    rest_codes<FMT>(w);
    if (!a.force) {  // the arithmetic of the fluid pass
      post_collision_codes<FMT>(w, a.nq_s, a.nq_d, a.nq_c, A);
      return;
    }
    c = Codec<FMT>::decode(w);
  }
  if (a.force)
    post_collision<true>(c, a.om1, a.hF, A);
  else
    post_collision<false>(c, a.om1, a.hF, A);
}

// Listed fluid cell `cell` (list entry / side slot e, flags b, yz = y | z << 16).
// The fluid pass pulled every link periodically and left its unrounded
// moments in the side buffer; only the links the boundary rules change are
// corrected here (new minus pulled distribution of each such link), and the
// cell is written once:
//   - bounce-back link i (source solid): new f+_opp(i)(x); pulled: f+_i of
//     the stored rest state (rest_coeffs), no load;
//   - inflow link (cx = 1 on the inflow face): new f+_i with the inflow
//     coefficients of x; the fluid pass pulled nothing there (zero), so no
//     source is read;
//   - outflow link (cx = -1 on the outflow face): the fluid pass pulled it
//     from a copy of the plane x = nx - 1, which is the zero-gradient value,
//     so nothing changes (a cell with no other flag is not visited at all).
// Bounce-back links are walked per lane (a bit scan).
//   - with wall rule 1 a solid link's new f+ is instead reconstructed at the
//     link midpoint from (rho^x, u^p of the object, S^p) (Sec. 3.2);
//   - TRACK: each solid link adds the momentum -(f_i(x) + f+_opp(i)(x)) c_i
//     it delivers to its object, and the torque of that about the object's
//     center, to acc (256 x 6, the workgroup's sums in LDS).
// The distribution f+_i the fluid pass pulled from a listed solid neighbour,
// for every direction i (eval_link of rest_coeffs), into rest[27].
template <int FMT>
__device__ inline void rest_links(const StepParams& a, int i, float* rest) {
  float Arest[NA];
  rest_coeffs<FMT>(a, Arest);
  rest[i] = eval_link(Arest, i % 3 - 1, (i / 3) % 3 - 1, i / 9 - 1);
}

// TABLE: rest holds the 27 values of rest_links (one launch's constants, in
// LDS); else they are evaluated here (the batch, whose cells differ in tau).
template <int FMT, bool TRACK, bool TABLE = false>
__device__ inline void boundary_fix(const StepParams& a, uint32_t e, uint32_t cell, uint32_t b, uint32_t yz,
                                    float* acc, const float* rest = nullptr) {
  const int nx = a.g.nx, ny = a.g.ny, nz = a.g.nz;
  const int y = int(yz & 0xFFFFu), z = int(yz >> 16);
  float m[10];
  side_load(a.lc.side, e, m);
  const PostCell own = post_cell<FMT>(a, cell);
  float Aown[NA];
  hermite_coeffs(own.dr, own.j, own.u, own.Nn, Aown);
  uint32_t bb = b & 0x7FFFFFFu & ~(1u << 13);
  if (bb) {
    float Arest[TABLE ? 1 : NA];
    if constexpr (!TABLE) rest_coeffs<FMT>(a, Arest);
    const int x = int(cell - uint32_t(nx) * (uint32_t(y) + uint32_t(ny) * uint32_t(z)));
    while (bb) {
      const int i = __ffs(bb) - 1;
      bb &= bb - 1u;
      const int cx = i % 3 - 1, cy = (i / 3) % 3 - 1, cz = i / 9 - 1;
      const float fout = eval_link(Aown, -cx, -cy, -cz);  // f+_opp(i)(x) - w_i
      float fnew = fout;                                   // bounce-back
      int id = 0;
      float r[3] = {0.0f, 0.0f, 0.0f};
      if (a.wall_rule != 0 || TRACK) {
        const uint32_t s = uint32_t(wrap_step(x, -cx, nx)) +
                           uint32_t(nx) * (uint32_t(wrap_step(y, -cy, ny)) + uint32_t(ny) * uint32_t(wrap_step(z, -cz, nz)));
        id = a.mask[s];
        float up[3];
        wall_velocity(a.objects + 9 * id, x, y, z, cx, cy, cz, up, r);
        if (a.wall_rule != 0) {
          float Ap[NA];
          boundary_point_coeffs(own, up, Ap);
          fnew = eval_link(Ap, cx, cy, cz);
        }
      }
      float pulled;
      if constexpr (TABLE)
        pulled = rest[i];
      else
        pulled = eval_link(Arest, cx, cy, cz);
      add_link(m, cx, cy, cz, fnew - pulled);
      if constexpr (TRACK) {
        float px[3], py[3], pz[3];
        basis1(cx, px);
        basis1(cy, py);
        basis1(cz, pz);
        const float g = -((fnew + fout) + 2.0f * (px[0] * py[0] * pz[0]));  // -(f_i + f+_opp(i)), w_i = w1 w1 w1
        const float dp[3] = {g * float(cx), g * float(cy), g * float(cz)};
        float* o = acc + 6 * id;
        atomicAdd(o + 0, dp[0]);
        atomicAdd(o + 1, dp[1]);
        atomicAdd(o + 2, dp[2]);
        atomicAdd(o + 3, r[1] * dp[2] - r[2] * dp[1]);
        atomicAdd(o + 4, r[2] * dp[0] - r[0] * dp[2]);
        atomicAdd(o + 5, r[0] * dp[1] - r[1] * dp[0]);
      }
    }
  }
  if (b & BIT_INFLOW) {
    float Ain[NA];
    boundary_point_coeffs(own, a.u_in, Ain);  // rho^p = rho^x, u^p = u_in, the stress of x
#pragma unroll
    for (int cz = -1; cz <= 1; ++cz)
#pragma unroll
      for (int cy = -1; cy <= 1; ++cy) add_link(m, 1, cy, cz, eval_link(Ain, 1, cy, cz));
  }
  const float j[3] = {m[1], m[2], m[3]};
  const float P[6] = {m[4], m[5], m[6], m[7], m[8], m[9]};
  store_cell_b<FMT>(a, cell, m[0], j, P);
}

// A listed solid cell: reset to rest.
template <int FMT>
__device__ inline void boundary_solid(const StepParams& a, uint32_t cell) {
  if constexpr (FMT == FMT_F32) {
    const float j[3] = {0, 0, 0}, P[6] = {0, 0, 0, 0, 0, 0};
    store_cell_b<FMT>(a, cell, 0.0f, j, P);
  } else {
    uint32_t w[Codec<FMT>::W];
    rest_codes<FMT>(w);
#pragma unroll
    for (int k = 0; k < Codec<FMT>::W; ++k) *reinterpret_cast<uint32_t*>(static_cast<char*>(a.out[k]) + cell * 4u) = w[k];
  }
}

}  // namespace lbm
