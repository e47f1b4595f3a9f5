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

hipError_t launch_requantize(const StepParams& p, int64_t N, hipStream_t s) {
  hipLaunchKernelGGL(requantize_kernel, dim3(uint32_t((N + 255) / 256)), dim3(256), 0, s, p, uint32_t(N));
  return hipGetLastError();
}

}  // namespace lbm
