// lbm_boundary.hip -- the boundary pass over the compacted cell list, and the
// list's construction.
//
// The fluid pass treats every cell alike (Sec. 4.2); this pass then visits
// only the listed cells (lbm_boundary_cell.h holds the per-cell update).
#include "lbm_boundary_cell.h"

namespace lbm {

// Listed fluid cells: 32 lanes each (8 cells per 256-thread block).
template <int FMT>
__global__ void __launch_bounds__(256) boundary_fluid_kernel(StepParams a, const uint32_t* __restrict__ cells,
                                                             const uint32_t* __restrict__ bits,
                                                             const uint32_t* __restrict__ yz, int count) {
  const int t = int(blockIdx.x) * 256 + int(threadIdx.x);
  const int e = t >> 5;
  if (e >= count) return;  // whole 32-lane groups leave together
  boundary_group<FMT>(a, cells[e], bits[e], yz[e], t & 31);
}

// Listed solid cells: one lane each.
template <int FMT>
__global__ void __launch_bounds__(256) boundary_solid_kernel(StepParams a, const uint32_t* __restrict__ cells,
                                                             int count) {
  const int e = int(blockIdx.x) * 256 + int(threadIdx.x);
  if (e >= count) return;
  boundary_solid<FMT>(a, cells[e]);
}

hipError_t launch_boundary(int fmt, const StepParams& p, const uint32_t* cells, const uint32_t* bits,
                           const uint32_t* yz, int nfluid, int nsolid, hipStream_t s) {
  if (nfluid > 0) {
    const dim3 grid(uint32_t((int64_t(nfluid) * 32 + 255) / 256));
    if (fmt == FMT_F32)
      hipLaunchKernelGGL(boundary_fluid_kernel<FMT_F32>, grid, dim3(256), 0, s, p, cells, bits, yz, nfluid);
    else
      hipLaunchKernelGGL(boundary_fluid_kernel<FMT_Q16>, grid, dim3(256), 0, s, p, cells, bits, yz, nfluid);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  if (nsolid > 0) {
    const dim3 grid(uint32_t((nsolid + 255) / 256));
    if (fmt == FMT_F32)
      hipLaunchKernelGGL(boundary_solid_kernel<FMT_F32>, grid, dim3(256), 0, s, p, cells + nfluid, nsolid);
    else
      hipLaunchKernelGGL(boundary_solid_kernel<FMT_Q16>, grid, dim3(256), 0, s, p, cells + nfluid, nsolid);
    return hipGetLastError();
  }
  return hipSuccess;
}

// ------------------------------------------------------------ compaction ---
// Classifies every cell; the listed ones are appended with one atomic per
// wavefront and kind (ballot + popcount): fluid entries to cells_f / bits_f,
// solid ones to cells_s / bits_s.  counters[0] counts fluid entries,
// counters[1] solid ones, counters[2] and [3] are the two fill cursors.  Order
// within each part is irrelevant: entries are independent.
__global__ void __launch_bounds__(256) classify_kernel(const uint8_t* __restrict__ mask, Geometry g,
                                                       uint32_t* counters, uint32_t* cells_f, uint32_t* bits_f,
                                                       uint32_t* yz_f, uint32_t cap_f, uint32_t* cells_s,
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
  // wavefront compaction
  const unsigned long long fvote = __ballot(listed && !solid);
  const unsigned long long svote = __ballot(listed && solid);
  if ((fvote | svote) == 0ull) return;
  const int lane = __lane_id();
  const int leader = __ffsll(static_cast<long long>(fvote | svote)) - 1;
  uint32_t fbase = 0, sbase = 0;
  if (lane == leader) {
    atomicAdd(&counters[0], uint32_t(__popcll(fvote)));
    atomicAdd(&counters[1], uint32_t(__popcll(svote)));
    if (cells_f != nullptr) {
      fbase = atomicAdd(&counters[2], uint32_t(__popcll(fvote)));
      sbase = atomicAdd(&counters[3], uint32_t(__popcll(svote)));
    }
  }
  if (cells_f == nullptr) return;
  fbase = __shfl(fbase, leader);
  sbase = __shfl(sbase, leader);
  if (listed) {
    const unsigned long long below = lane == 0 ? 0ull : ((~0ull) >> (64 - lane));
    if (solid) {
      const uint32_t k = sbase + uint32_t(__popcll(svote & below));
      if (k < cap_s) {
        cells_s[k] = cell;
        bits_s[k] = b;
      }
    } else {
      const uint32_t k = fbase + uint32_t(__popcll(fvote & below));
      if (k < cap_f) {
        cells_f[k] = cell;
        bits_f[k] = b;
        yz_f[k] = yz;
      }
    }
  }
}

hipError_t launch_classify(const uint8_t* mask, const Geometry& g, uint32_t* counters, uint32_t* cells_f,
                           uint32_t* bits_f, uint32_t* yz_f, uint32_t cap_f, uint32_t* cells_s, uint32_t* bits_s,
                           uint32_t cap_s, hipStream_t s) {
  const uint64_t N = uint64_t(g.nx) * g.ny * g.nz;
  const dim3 block(256), grid(uint32_t((N + 255) / 256));
  hipLaunchKernelGGL(classify_kernel, grid, block, 0, s, mask, g, counters, cells_f, bits_f, yz_f, cap_f, cells_s,
                     bits_s, cap_s);
  return hipGetLastError();
}

}  // namespace lbm
