// lbm_boundary.hip -- the boundary pass over the compacted cell list, and the
// list's construction.
//
// The fluid pass treats every cell alike (Sec. 4.2); this pass then visits
// only the listed cells (lbm_boundary_cell.h holds the per-cell update).
#include "lbm_boundary_cell.h"

namespace lbm {

template <int FMT>
__global__ void __launch_bounds__(256) boundary_kernel(StepParams a, const uint32_t* __restrict__ cells,
                                                       const uint32_t* __restrict__ bits, int count) {
  const int e = int(blockIdx.x) * blockDim.x + threadIdx.x;
  if (e >= count) return;
  boundary_entry<FMT>(a, cells[e], bits[e]);
}

hipError_t launch_boundary(int fmt, const StepParams& p, const uint32_t* cells, const uint32_t* bits, int count,
                           hipStream_t s) {
  if (count <= 0) return hipSuccess;
  const dim3 block(256), grid((count + 255) / 256);
  if (fmt == FMT_F32)
    hipLaunchKernelGGL(boundary_kernel<FMT_F32>, grid, block, 0, s, p, cells, bits, count);
  else
    hipLaunchKernelGGL(boundary_kernel<FMT_Q16>, grid, block, 0, s, p, cells, bits, count);
  return hipGetLastError();
}

// ------------------------------------------------------------ compaction ---
// Classifies every cell; the listed ones are appended with one atomic per
// wavefront (ballot + popcount).  counters[0] counts fluid entries, counters[1]
// solid ones, counters[2] is the fill cursor.  Order within the list is
// irrelevant: entries are independent.
__global__ void __launch_bounds__(256) classify_kernel(const uint8_t* __restrict__ mask, Geometry g,
                                                       uint32_t* counters, uint32_t* cells, uint32_t* bits,
                                                       uint32_t capacity) {
  const uint32_t N = uint32_t(g.nx) * uint32_t(g.ny) * uint32_t(g.nz);
  const uint32_t cell = blockIdx.x * blockDim.x + threadIdx.x;
  bool listed = false;
  uint32_t b = 0;
  bool solid = false;
  if (cell < N) {
    const int x = int(cell % uint32_t(g.nx));
    const int y = int((cell / uint32_t(g.nx)) % uint32_t(g.ny));
    const int z = int(cell / (uint32_t(g.nx) * uint32_t(g.ny)));
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
  const unsigned long long vote = __ballot(listed);
  if (vote == 0ull) return;
  const int lane = __lane_id();
  const int leader = __ffsll(static_cast<long long>(vote)) - 1;
  const unsigned long long solid_vote = __ballot(listed && solid);
  uint32_t base = 0;
  if (lane == leader) {
    atomicAdd(&counters[0], uint32_t(__popcll(vote & ~solid_vote)));
    atomicAdd(&counters[1], uint32_t(__popcll(solid_vote)));
    if (cells != nullptr) base = atomicAdd(&counters[2], uint32_t(__popcll(vote)));
  }
  if (cells == nullptr) return;
  base = __shfl(base, leader);
  if (listed) {
    const unsigned long long below = lane == 0 ? 0ull : (vote & ((~0ull) >> (64 - lane)));
    const uint32_t k = base + uint32_t(__popcll(below));
    if (k < capacity) {
      cells[k] = cell;
      bits[k] = b;
    }
  }
}

hipError_t launch_classify(const uint8_t* mask, const Geometry& g, uint32_t* counters, uint32_t* cells,
                           uint32_t* bits, uint32_t capacity, hipStream_t s) {
  const uint64_t N = uint64_t(g.nx) * g.ny * g.nz;
  const dim3 block(256), grid(uint32_t((N + 255) / 256));
  hipLaunchKernelGGL(classify_kernel, grid, block, 0, s, mask, g, counters, cells, bits, capacity);
  return hipGetLastError();
}

}  // namespace lbm
