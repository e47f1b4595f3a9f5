// lbm_boundary.hip -- the boundary pass over the compacted cell list, and the
// list's construction.
//
// The fluid pass treats every cell alike (Sec. 4.2) and keeps, for each listed
// fluid cell, its unrounded result; this pass then visits only the listed
// cells (lbm_boundary_cell.h holds the per-cell update).
#include "lbm_boundary_cell.h"

namespace lbm {

// Listed fluid cells: one lane each; entry e is slot e of the side buffer.
// The pulled rest distributions, the same for every cell of the launch, are
// evaluated once per workgroup into LDS.
template <int FMT>
__global__ void __launch_bounds__(256) boundary_fluid_kernel(StepParams ap, const uint32_t* __restrict__ cells,
                                                             const uint32_t* __restrict__ bits,
                                                             const uint32_t* __restrict__ yz,
                                                             const uint32_t* __restrict__ order, int count) {
  StepParams a = ap;
  a.key = step_key(ap);
  __shared__ float rest[27];
  if (threadIdx.x < 27) rest_links<FMT>(a, int(threadIdx.x), rest);
  __syncthreads();
  const int t = int(blockIdx.x) * 256 + int(threadIdx.x);
  if (t >= count) return;
  const uint32_t e = order ? order[t] : uint32_t(t);
  boundary_fix<FMT, false, true>(a, e, cells[e], bits[e], yz[e], nullptr, rest);
}

// The same with the force and torque on each object summed (Sec. 3.2, last
// step): per workgroup in LDS, then one double add per nonzero sum into
// a.forces.
template <int FMT>
__global__ void __launch_bounds__(256) boundary_fluid_forces_kernel(StepParams ap, const uint32_t* __restrict__ cells,
                                                                    const uint32_t* __restrict__ bits,
                                                                    const uint32_t* __restrict__ yz,
                                                                    const uint32_t* __restrict__ order, int count) {
  StepParams a = ap;
  a.key = step_key(ap);
  __shared__ float acc[256 * 6];
  __shared__ float rest[27];
  for (int k = int(threadIdx.x); k < 256 * 6; k += 256) acc[k] = 0.0f;
  if (threadIdx.x < 27) rest_links<FMT>(a, int(threadIdx.x), rest);
  __syncthreads();
  const int t = int(blockIdx.x) * 256 + int(threadIdx.x);
  if (t < count) {
    const uint32_t e = order ? order[t] : uint32_t(t);
    boundary_fix<FMT, true, true>(a, e, cells[e], bits[e], yz[e], acc, rest);
  }
  __syncthreads();
  for (int k = int(threadIdx.x); k < 256 * 6; k += 256)
    if (acc[k] != 0.0f) atomicAdd(a.forces + k, double(acc[k]));
}

// Listed solid cells: one lane each.
template <int FMT>
__global__ void __launch_bounds__(256) boundary_solid_kernel(StepParams ap, const uint32_t* __restrict__ cells,
                                                             int count) {
  const int e = int(blockIdx.x) * 256 + int(threadIdx.x);
  if (e >= count) return;
  boundary_solid<FMT>(ap, cells[e]);
}

// Both lists in one launch: the fluid fixes' workgroups first, then the
// solid resets', which fill the gaps as the fixes drain.  No cell is in both
// lists, and a fluid fix reads only the old state (p.in), never a cell a
// reset writes.
template <int FMT>
__global__ void __launch_bounds__(256) boundary_kernel(StepParams ap, const uint32_t* __restrict__ cells,
                                                       const uint32_t* __restrict__ bits,
                                                       const uint32_t* __restrict__ yz,
                                                       const uint32_t* __restrict__ order, int nfluid,
                                                       const uint32_t* __restrict__ solid_cells, int nsolid) {
  const int bf = (nfluid + 255) / 256;
  const int b = int(blockIdx.x);
  const bool fluid = b < bf;
  const int k = fluid ? b : b - bf;
  if (!fluid) {  // the whole workgroup
    const int e = k * 256 + int(threadIdx.x);
    if (e < nsolid) boundary_solid<FMT>(ap, solid_cells[e]);
    return;
  }
  StepParams a = ap;
  a.key = step_key(ap);
  __shared__ float rest[27];
  if (threadIdx.x < 27) rest_links<FMT>(a, int(threadIdx.x), rest);
  __syncthreads();
  const int t = k * 256 + int(threadIdx.x);
  if (t >= nfluid) return;
  const uint32_t e = order ? order[t] : uint32_t(t);
  boundary_fix<FMT, false, true>(a, e, cells[e], bits[e], yz[e], nullptr, rest);
}

namespace {
template <int FMT>
hipError_t launch_boundary_fmt(const StepParams& p, const uint32_t* cells, const uint32_t* bits, const uint32_t* yz,
                               const uint32_t* order, int nfluid, const uint32_t* solid_cells, int nsolid,
                               hipStream_t s) {
  if (nfluid > 0 && nsolid > 0 && !p.forces) {
    const dim3 grid(uint32_t((nfluid + 255) / 256 + (nsolid + 255) / 256));
    hipLaunchKernelGGL(boundary_kernel<FMT>, grid, dim3(256), 0, s, p, cells, bits, yz, order, nfluid, solid_cells,
                       nsolid);
    return hipGetLastError();
  }
  if (nfluid > 0) {
    const dim3 grid(uint32_t((nfluid + 255) / 256));
    if (p.forces)
      hipLaunchKernelGGL(boundary_fluid_forces_kernel<FMT>, grid, dim3(256), 0, s, p, cells, bits, yz, order, nfluid);
    else
      hipLaunchKernelGGL(boundary_fluid_kernel<FMT>, grid, dim3(256), 0, s, p, cells, bits, yz, order, nfluid);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  if (nsolid > 0) {
    const dim3 grid(uint32_t((nsolid + 255) / 256));
    hipLaunchKernelGGL(boundary_solid_kernel<FMT>, grid, dim3(256), 0, s, p, solid_cells, nsolid);
    return hipGetLastError();
  }
  return hipSuccess;
}
}  // namespace

hipError_t launch_boundary(int fmt, const StepParams& p, const uint32_t* cells, const uint32_t* bits,
                           const uint32_t* yz, const uint32_t* order, int nfluid, const uint32_t* solid_cells,
                           int nsolid, hipStream_t s) {
  if (fmt == FMT_F32)
    return launch_boundary_fmt<FMT_F32>(p, cells, bits, yz, order, nfluid, solid_cells, nsolid, s);
  hipError_t e = hipErrorInvalidValue;
  dispatch_codes(fmt, [&]<int F>() {
    e = launch_boundary_fmt<F>(p, cells, bits, yz, order, nfluid, solid_cells, nsolid, s);
  });
  return e;
}

// ------------------------------------------------------------ compaction ---
// Word w of the solid bitmap holds cells 32 w .. 32 w + 31 (bit k: cell
// 32 w + k), built from one ballot per wavefront: lanes 0 and 32 write the
// two words their wavefront covers.  Bits past the last cell are zero.
__global__ void __launch_bounds__(256) solid_bits_kernel(const uint8_t* __restrict__ mask, uint32_t N,
                                                         uint32_t* __restrict__ out) {
  const uint32_t i = blockIdx.x * 256u + threadIdx.x;
  const unsigned long long b = __ballot(i < N && mask[i] != 0);
  const uint32_t lane = threadIdx.x & 63u;
  if ((lane & 31u) == 0u && i < N) out[i >> 5] = uint32_t(b >> lane);
}

hipError_t launch_solid_bits(const uint8_t* mask, uint32_t N, uint32_t* out, hipStream_t s) {
  if (N == 0) return hipSuccess;
  hipLaunchKernelGGL(solid_bits_kernel, dim3((N + 255u) / 256u), dim3(256), 0, s, mask, N, out);
  return hipGetLastError();
}

// Classifies every cell of a domain.  Listed fluid cells are kept in raster
// order (their slot comes from the global bitmap and its prefix counts, so
// the fluid pass can find a cell's slot without searching); listed solid
// cells are appended with one atomic per wavefront (their order does not
// matter).
__global__ void __launch_bounds__(256) classify_kernel(const uint8_t* __restrict__ mask, Geometry g, uint32_t goff,
                                                       uint32_t* counters, unsigned long long* lmask,
                                                       const uint32_t* __restrict__ lbase, uint32_t* cells_f,
                                                       uint32_t* bits_f, uint32_t* yz_f, uint32_t* cells_s,
                                                       uint32_t* bits_s, uint32_t cap_s) {
  const uint32_t N = uint32_t(g.nx) * uint32_t(g.ny) * uint32_t(g.nz);
  const uint32_t cell = blockIdx.x * blockDim.x + threadIdx.x;
  bool listed = false;
  uint32_t b = 0, yz = 0;
  bool solid = false;
  if (cell < N) {
    const int x = int(cell % uint32_t(g.nx));
    const int y = int((cell / uint32_t(g.nx)) % uint32_t(g.ny));
    const int z = int(cell / (uint32_t(g.nx) * uint32_t(g.ny)));
    yz = uint32_t(y) | (uint32_t(z) << 16);
    solid = mask != nullptr && mask[cell] != 0;
    if (solid) {
      // shell: any neighbour (26) inside the domain is fluid
      for (int i = 0; i < 27 && !listed; ++i) {
        if (i == 13) continue;
        const int cx = i % 3 - 1, cy = (i / 3) % 3 - 1, cz = i / 9 - 1;
        int sx = x - cx;
        if (g.inflow) {
          if (sx < 0 || sx >= g.nx) continue;
        } else {
          sx = wrapi(sx, g.nx);
        }
        const uint32_t s = uint32_t(sx) + uint32_t(g.nx) * (uint32_t(wrapi(y - cy, g.ny)) + uint32_t(g.ny) * uint32_t(wrapi(z - cz, g.nz)));
        if (mask[s] == 0) listed = true;
      }
      if (listed) b = BIT_SOLID;
    } else {
      if (g.inflow && x == 0) b |= BIT_INFLOW;
      if (g.inflow && x == g.nx - 1) b |= BIT_OUTFLOW;
      if (mask != nullptr) {
        for (int i = 0; i < 27; ++i) {
          if (i == 13) continue;
          const int cx = i % 3 - 1, cy = (i / 3) % 3 - 1, cz = i / 9 - 1;
          if ((b & BIT_INFLOW) && cx == 1) continue;
          if ((b & BIT_OUTFLOW) && cx == -1) continue;
          int sx = x - cx;
          if (!g.inflow) sx = wrapi(sx, g.nx);
          const uint32_t s = uint32_t(sx) + uint32_t(g.nx) * (uint32_t(wrapi(y - cy, g.ny)) + uint32_t(g.ny) * uint32_t(wrapi(z - cz, g.nz)));
          if (mask[s]) b |= 1u << i;
        }
      }
      listed = b != 0;
    }
  }
  const bool lfluid = listed && !solid;
  const unsigned long long fvote = __ballot(lfluid);
  const unsigned long long svote = __ballot(listed && solid);
  if ((fvote | svote) == 0ull) return;
  const int lane = __lane_id();
  const uint32_t gcell = goff + cell;
  if (lbase == nullptr) {
    // count pass: counts, and the fluid cells into the global bitmap (a
    // domain need not start on a 64-cell boundary, hence the atomic OR)
    const int leader = __ffsll(static_cast<long long>(fvote | svote)) - 1;
    if (lane == leader) {
      atomicAdd(&counters[0], uint32_t(__popcll(fvote)));
      atomicAdd(&counters[1], uint32_t(__popcll(svote)));
    }
    if (lfluid) atomicOr(&lmask[gcell >> 6], 1ull << (gcell & 63u));
    return;
  }
  // fill pass
  const unsigned long long below = lane == 0 ? 0ull : ((~0ull) >> (64 - lane));
  const int sleader = svote ? __ffsll(static_cast<long long>(svote)) - 1 : -1;
  uint32_t sbase = 0;
  if (lane == sleader) sbase = atomicAdd(&counters[3], uint32_t(__popcll(svote)));
  if (sleader >= 0) sbase = __shfl(sbase, sleader);
  if (listed && solid) {
    const uint32_t k = sbase + uint32_t(__popcll(svote & below));
    if (k < cap_s) {
      cells_s[k] = cell;
      bits_s[k] = b;
    }
  }
  if (lfluid) {
    const unsigned long long w = lmask[gcell >> 6];
    const uint32_t bit = gcell & 63u;
    const unsigned long long wb = bit == 0 ? 0ull : (w & ((~0ull) >> (64u - bit)));
    const uint32_t k = lbase[gcell >> 6] + uint32_t(__popcll(wb));
    cells_f[k] = cell;
    bits_f[k] = b;
    yz_f[k] = yz;
  }
}

hipError_t launch_classify(const uint8_t* mask, const Geometry& g, uint32_t goff, uint32_t* counters,
                           unsigned long long* lmask, const uint32_t* lbase, uint32_t* cells_f, uint32_t* bits_f,
                           uint32_t* yz_f, uint32_t* cells_s, uint32_t* bits_s, uint32_t cap_s, hipStream_t s) {
  const uint64_t N = uint64_t(g.nx) * g.ny * g.nz;
  const dim3 block(256), grid(uint32_t((N + 255) / 256));
  hipLaunchKernelGGL(classify_kernel, grid, block, 0, s, mask, g, goff, counters, lmask, lbase, cells_f, bits_f, yz_f,
                     cells_s, bits_s, cap_s);
  return hipGetLastError();
}

}  // namespace lbm
