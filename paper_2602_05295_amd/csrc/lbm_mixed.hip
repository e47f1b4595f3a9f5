// lbm_mixed.hip -- the solid correction and requantize passes of the paper's
// mixed-precision pipeline (Sec. 5.3, "atomic accumulation with mixed
// precision"), kept beside the library's own scheme so the two can be
// compared on the same scene.
//
// The 16-bit buffer holds post-collision moments.  A step is
//   1. the stream pass (fluid_kernel<FMT_Q16, R, false, true>): every cell's
//      post-collision moments are reconstructed, pull-streamed periodically
//      and projected into ten FP32 post-stream planes;
//   2. the link corrections (here): one thread per changed link adds
//      (new - pulled distribution) times the link's moment vector to its
//      cell's FP32 moments with atomicAdd, so several links of one cell may
//      land in any order;
//   3. requantize (here): every cell's FP32 moments are collided (App. A)
//      and encoded, with the dither, into the 16-bit buffer; then the solid
//      cells next to fluid are put back to rest.
// The FP32 planes are written and read once per step beside the codes: 120 B
// per cell and step against the 40 B of the fluid pass that keeps only the
// listed cells' unrounded moments.
#include "lbm_boundary_cell.h"

namespace lbm {

namespace {

// Decoded post-collision cell (the codes of the mixed pipeline need no
// collision): the fields of PostCell.
__device__ inline PostCell post_from_codes(const StepParams& a, uint32_t q) {
  const CellIn c = load_cell_b<FMT_Q16>(a, q);
  PostCell s;
  s.dr = c.dr;
  s.rho = c.rho;
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    s.j[k] = c.j[k];
    s.u[k] = c.u[k];
  }
#pragma unroll
  for (int k = 0; k < 6; ++k) s.Nn[k] = c.N[k];
  return s;
}

__device__ inline void coeffs_of(const PostCell& s, float A[NA]) { hermite_coeffs(s.dr, s.j, s.u, s.Nn, A); }

__global__ void __launch_bounds__(256) mixed_links_kernel(StepParams a, const uint32_t* __restrict__ links, int nlinks,
                                                          const uint32_t* __restrict__ cells,
                                                          const uint32_t* __restrict__ yz,
                                                          const uint32_t* __restrict__ bits) {
  const int k = int(blockIdx.x) * 256 + int(threadIdx.x);
  if (k >= nlinks) return;
  const uint32_t e = links[k] >> 5, i = links[k] & 31u;
  const uint32_t cell = cells[e], b = bits[e], yzv = yz[e];
  const int nx = a.g.nx, ny = a.g.ny, nz = a.g.nz;
  const int y = int(yzv & 0xFFFFu), z = int(yzv >> 16);
  const int x = int(cell - uint32_t(nx) * (uint32_t(y) + uint32_t(ny) * uint32_t(z)));
  const int cx = int(i % 3) - 1, cy = int((i / 3) % 3) - 1, cz = int(i / 9) - 1;
  const PostCell own = post_from_codes(a, cell);
  float fnew, fpulled;
  if ((b >> i) & 1u && i != 13u && !(b & (BIT_INFLOW | BIT_OUTFLOW))) {
    // a solid source: the stream pass pulled its rest codes
    uint32_t w[5];
    rest_codes<FMT_Q16>(w);
    const CellIn r = cell_from_words(w);
    float Ar[NA];
    hermite_coeffs(r.dr, r.j, r.u, r.N, Ar);
    fpulled = eval_link(Ar, cx, cy, cz);
    float A[NA];
    if (a.wall_rule == 0) {
      coeffs_of(own, A);
      fnew = eval_link(A, -cx, -cy, -cz);
    } else {
      const uint32_t s = uint32_t(wrap_step(x, -cx, nx)) +
                         uint32_t(nx) * (uint32_t(wrap_step(y, -cy, ny)) + uint32_t(ny) * uint32_t(wrap_step(z, -cz, nz)));
      float up[3], r3[3];
      wall_velocity(a.objects + 9 * a.mask[s], x, y, z, cx, cy, cz, up, r3);
      boundary_point_coeffs(own, up, A);
      fnew = eval_link(A, cx, cy, cz);
    }
  } else {
    // a face link: inflow (x = 0, cx = 1) or zero-gradient outflow (x = nx - 1, cx = -1)
    const uint32_t yzo =
        uint32_t(nx) * (uint32_t(wrap_step(y, -cy, ny)) + uint32_t(ny) * uint32_t(wrap_step(z, -cz, nz)));
    const bool in = cx > 0;
    float A[NA];
    coeffs_of(post_from_codes(a, (in ? uint32_t(nx - 1) : 0u) + yzo), A);  // the periodic image the pass pulled
    fpulled = eval_link(A, cx, cy, cz);
    if (in)
      boundary_point_coeffs(own, a.u_in, A);
    else
      coeffs_of(post_from_codes(a, uint32_t(nx - 1) + yzo), A);
    fnew = eval_link(A, cx, cy, cz);
  }
  const float df = fnew - fpulled;
  const float fx = float(cx), fy = float(cy), fz = float(cz);
  const float dm[10] = {df, fx * df, fy * df, fz * df, (fx * fx - R3) * df, (fy * fy - R3) * df,
                        (fz * fz - R3) * df, fx * fy * df, fx * fz * df, fy * fz * df};
#pragma unroll
  for (int q = 0; q < 10; ++q)
    if (dm[q] != 0.0f) atomicAdd(static_cast<float*>(a.out[q]) + cell, dm[q]);
}

// ------------------------------------------ per-triangle solid correction ---
// Sec. 4.2, Alg. 3: one thread per triangle visits the lattice nodes of the
// triangle's bounding box (widened by one cell: a link reaches one cell from
// its node on every axis), skips those that are not listed fluid cells (the
// paper's voxel skip), and tests each of a node's links to a solid source
// against the triangle.  A link can meet several triangles (a shared edge, a
// second surface behind the first); the correction belongs to the nearest
// hit (ties to the lowest triangle index), found by a first sweep that keeps,
// per link, the smallest key (t, triangle) with atomicMin.  The second sweep,
// run every step, recomputes its hits and corrects the links it wins:
// Delta f_i = f_i(p) - f_i(x - c_i), f_i(p) the moment wall of Sec. 3.2 at
// p = x - t c_i with the velocity of the triangle's object there, projected
// to Delta m and added to x's FP32 post-stream moments with atomicAdd.

// Parameter t in [0, 1] where the segment from the origin to d meets the
// triangle (v0, v1, v2) (coordinates relative to the segment's start), or -1.
// Moller-Trumbore, restricted to the segment; points within `tol` of an edge
// in barycentric terms count as hits on both sides, so no link slips between
// two triangles (the nearest-hit key then picks one).
__device__ inline float segment_triangle_f(const float d[3], const float v0[3], const float v1[3], const float v2[3]) {
  const float tol = 1e-5f;
  const float e1[3] = {v1[0] - v0[0], v1[1] - v0[1], v1[2] - v0[2]};
  const float e2[3] = {v2[0] - v0[0], v2[1] - v0[1], v2[2] - v0[2]};
  const float p[3] = {d[1] * e2[2] - d[2] * e2[1], d[2] * e2[0] - d[0] * e2[2], d[0] * e2[1] - d[1] * e2[0]};
  const float det = e1[0] * p[0] + e1[1] * p[1] + e1[2] * p[2];
  if (fabsf(det) < 1e-20f) return -1.0f;
  const float inv = 1.0f / det;
  const float sv[3] = {-v0[0], -v0[1], -v0[2]};
  const float u = (sv[0] * p[0] + sv[1] * p[1] + sv[2] * p[2]) * inv;
  if (u < -tol || u > 1.0f + tol) return -1.0f;
  const float q[3] = {sv[1] * e1[2] - sv[2] * e1[1], sv[2] * e1[0] - sv[0] * e1[2], sv[0] * e1[1] - sv[1] * e1[0]};
  const float v = (d[0] * q[0] + d[1] * q[1] + d[2] * q[2]) * inv;
  if (v < -tol || u + v > 1.0f + tol) return -1.0f;
  const float t = (e2[0] * q[0] + e2[1] * q[1] + e2[2] * q[2]) * inv;
  if (t < -tol || t > 1.0f + tol) return -1.0f;
  return fminf(fmaxf(t, 0.0f), 1.0f);
}

// Visits the links triangle k meets: calls f(slot, cell, x, y, z, i, t) for
// each listed fluid node x of the widened box and each of its links to a
// solid source that the triangle meets at parameter t.
template <class F>
__device__ inline void for_triangle_links(const StepParams& a, const TriangleSet& T, int k, F&& f) {
  const float* tv = T.tris + 9 * size_t(k);
  float v[9];
#pragma unroll
  for (int q = 0; q < 9; ++q) v[q] = tv[q];
  const int nx = a.g.nx, ny = a.g.ny, nz = a.g.nz;
  int lo[3], hi[3];
  const int n[3] = {nx, ny, nz};
#pragma unroll
  for (int ax = 0; ax < 3; ++ax) {
    // clamped to the grid in float first, so far-away vertices convert safely
    const float mn = fminf(v[ax], fminf(v[3 + ax], v[6 + ax]));
    const float mx = fmaxf(v[ax], fmaxf(v[3 + ax], v[6 + ax]));
    lo[ax] = int(fminf(fmaxf(floorf(mn) - 1.0f, 0.0f), float(n[ax])));
    hi[ax] = int(fmaxf(fminf(ceilf(mx) + 1.0f, float(n[ax] - 1)), -1.0f));
  }
  for (int z = lo[2]; z <= hi[2]; ++z)
    for (int y = lo[1]; y <= hi[1]; ++y)
      for (int x = lo[0]; x <= hi[0]; ++x) {
        const uint32_t cell = uint32_t(x) + uint32_t(nx) * (uint32_t(y) + uint32_t(ny) * uint32_t(z));
        const int slot = listed_slot_in(T.lpack[cell >> 6], cell);
        if (slot < 0) continue;
        const uint32_t b = T.bits[slot];
        if (b & (BIT_INFLOW | BIT_OUTFLOW)) continue;  // face cells keep the face rules (no solid links there)
        uint32_t bb = b & 0x7FFFFFFu & ~(1u << 13);
        if (!bb) continue;
        const float fx = float(x), fy = float(y), fz = float(z);
        const float v0[3] = {v[0] - fx, v[1] - fy, v[2] - fz};
        const float v1[3] = {v[3] - fx, v[4] - fy, v[5] - fz};
        const float v2[3] = {v[6] - fx, v[7] - fy, v[8] - fz};
        while (bb) {
          const int i = __ffs(bb) - 1;
          bb &= bb - 1u;
          const float d[3] = {-float(i % 3 - 1), -float((i / 3) % 3 - 1), -float(i / 9 - 1)};
          const float t = segment_triangle_f(d, v0, v1, v2);
          if (t >= 0.0f) f(uint32_t(slot), cell, x, y, z, i, t);
        }
      }
}

__device__ inline unsigned long long hit_key(float t, int k) {
  return (static_cast<unsigned long long>(__float_as_uint(t)) << 32) | uint32_t(k);
}

__global__ void __launch_bounds__(256) triangle_winner_kernel(StepParams a, TriangleSet T,
                                                              unsigned long long* __restrict__ winner) {
  const int k = int(blockIdx.x) * 256 + int(threadIdx.x);
  if (k >= T.n) return;
  for_triangle_links(a, T, k, [&](uint32_t slot, uint32_t, int, int, int, int i, float t) {
    atomicMin(winner + size_t(slot) * 27 + i, hit_key(t, k));
  });
}

__global__ void __launch_bounds__(256) triangle_correction_kernel(StepParams a, TriangleSet T,
                                                                  const unsigned long long* __restrict__ winner) {
  const int k = int(blockIdx.x) * 256 + int(threadIdx.x);
  if (k >= T.n) return;
  const float* obj = a.objects + 9 * int(T.obj[k]);
  float rest[NA];
  {
    uint32_t w[5];
    rest_codes<FMT_Q16>(w);
    const CellIn r = cell_from_words(w);
    hermite_coeffs(r.dr, r.j, r.u, r.N, rest);
  }
  // corrections of one node at a time: links of a node are visited together
  uint32_t cur = 0xFFFFFFFFu;
  float dm[10];
  auto flush = [&]() {
    if (cur == 0xFFFFFFFFu) return;
#pragma unroll
    for (int q = 0; q < 10; ++q)
      if (dm[q] != 0.0f) atomicAdd(static_cast<float*>(a.out[q]) + cur, dm[q]);
  };
  for_triangle_links(a, T, k, [&](uint32_t slot, uint32_t cell, int x, int y, int z, int i, float t) {
    if (winner[size_t(slot) * 27 + i] != hit_key(t, k)) return;
    if (cell != cur) {
      flush();
      cur = cell;
#pragma unroll
      for (int q = 0; q < 10; ++q) dm[q] = 0.0f;
    }
    const int cx = i % 3 - 1, cy = (i / 3) % 3 - 1, cz = i / 9 - 1;
    const float p[3] = {float(x) - t * float(cx), float(y) - t * float(cy), float(z) - t * float(cz)};
    const float r3[3] = {p[0] - obj[0], p[1] - obj[1], p[2] - obj[2]};
    const float up[3] = {obj[3] + (obj[7] * r3[2] - obj[8] * r3[1]), obj[4] + (obj[8] * r3[0] - obj[6] * r3[2]),
                         obj[5] + (obj[6] * r3[1] - obj[7] * r3[0])};
    float A[NA];
    boundary_point_coeffs(post_from_codes(a, cell), up, A);
    const float df = eval_link(A, cx, cy, cz) - eval_link(rest, cx, cy, cz);
    add_link(dm, cx, cy, cz, df);
  });
  flush();
}

__global__ void fill_u64_kernel(unsigned long long* p, size_t n, unsigned long long v) {
  const size_t k = size_t(blockIdx.x) * 256 + threadIdx.x;
  if (k < n) p[k] = v;
}

// FP32 post-stream moments (rho - 1, j, P) -> collide -> codes of the
// post-collision moments (rho, u, N+), with the dither of p.key.
__global__ void __launch_bounds__(256) requantize_kernel(StepParams a, uint32_t N) {
  const uint32_t c = blockIdx.x * 256u + threadIdx.x;
  if (c >= N) return;
  float m[10];
#pragma unroll
  for (int k = 0; k < 10; ++k) m[k] = static_cast<const float*>(a.in[k])[c];
  const CellIn s = cell_from_moments(m);
  float Nn[6];
  collide_neq(s.N, a.om1, Nn);
  const float P[6] = {fmaf(s.j[0], s.u[0], Nn[0]), fmaf(s.j[1], s.u[1], Nn[1]), fmaf(s.j[2], s.u[2], Nn[2]),
                      fmaf(s.j[0], s.u[1], Nn[3]), fmaf(s.j[0], s.u[2], Nn[4]), fmaf(s.j[1], s.u[2], Nn[5])};
  uint32_t w[5];
  encode_cell(s.dr, s.j, P, c, a.key, a.dither != 0, w);
#pragma unroll
  for (int k = 0; k < 5; ++k) static_cast<uint32_t*>(a.out[k])[c] = w[k];
}

}  // namespace

hipError_t launch_mixed_links(const StepParams& p, const uint32_t* links, int nlinks, const uint32_t* cells,
                              const uint32_t* yz, const uint32_t* bits, hipStream_t s) {
  if (nlinks <= 0) return hipSuccess;
  hipLaunchKernelGGL(mixed_links_kernel, dim3(uint32_t((nlinks + 255) / 256)), dim3(256), 0, s, p, links, nlinks,
                     cells, yz, bits);
  return hipGetLastError();
}

hipError_t launch_triangle_winners(const StepParams& p, const TriangleSet& T, unsigned long long* winner,
                                   int64_t nslots, hipStream_t s) {
  const size_t n = size_t(nslots) * 27;
  if (n > 0) {
    hipLaunchKernelGGL(fill_u64_kernel, dim3(uint32_t((n + 255) / 256)), dim3(256), 0, s, winner, n, ~0ull);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  if (T.n <= 0 || nslots <= 0 || !T.lpack || !T.bits || !winner) return hipSuccess;
  hipLaunchKernelGGL(triangle_winner_kernel, dim3(uint32_t((T.n + 255) / 256)), dim3(256), 0, s, p, T, winner);
  return hipGetLastError();
}

hipError_t launch_triangle_correction(const StepParams& p, const TriangleSet& T, const unsigned long long* winner,
                                      hipStream_t s) {
  if (T.n <= 0 || !T.lpack || !T.bits || !winner) return hipSuccess;  // no listed cells: nothing to correct
  hipLaunchKernelGGL(triangle_correction_kernel, dim3(uint32_t((T.n + 255) / 256)), dim3(256), 0, s, p, T, winner);
  return hipGetLastError();
}

hipError_t launch_requantize(const StepParams& p, int64_t N, hipStream_t s) {
  hipLaunchKernelGGL(requantize_kernel, dim3(uint32_t((N + 255) / 256)), dim3(256), 0, s, p, uint32_t(N));
  return hipGetLastError();
}

}  // namespace lbm
