// lbm_batch.h -- device-side tables and launchers of the batched step (many
// independent periodic domains advanced by the same launches).
#pragma once

#include "lbm_internal.h"

namespace lbm {

// One domain of the batch.  Its cells occupy [off, off + nx*ny*nz) of every
// state plane (planes are shared by all domains, x fastest within a domain).
// The fluid pass cuts the domain into strips of full x rows: a strip loads
// `rows` rows (ty output rows plus one halo row on each side) or, when `span`
// is set, all ny rows, which then wrap inside the strip and need no halo.
struct BatchDomain {
  uint32_t off;
  int nx, ny, nz;
  int rows;
  int ty;
  int span;
  float om1;  // 1 - 1/tau of this domain
  float nq_s, nq_d, nq_c;  // its code-space collision constants (16-bit codes)
};

// A run of planes [za, zb) of one strip: the unit of work of the fluid pass.
struct BatchSeg {
  uint16_t dom, strip, za, zb;
};

struct BatchStepParams {
  const void* in[10];         // concatenated state planes read (FP32: 10, Q16: 5)
  void* out[10];              // concatenated state planes written
  const BatchDomain* doms;
  const BatchSeg* segs;
  const uint32_t* wg_first;   // segments of logical workgroup w: [wg_first[w], wg_first[w + 1])
  const uint32_t* step;       // device step counter: step k of a launch sequence uses *step + k
  uint32_t step_offset;
  uint32_t seed;
  int dither_mode;            // 0 off, 1 per step, 2 static (Q16 only)
  int stream_out;             // non-temporal stores of the new state (stream_out_state)
  int nwg;
  ListedCells lc;             // listed fluid cells by global cell index (lc.side == nullptr: none)
};

// Threads per fluid workgroup the strip kernel is compiled for.
extern const int kBatchBlocks[3];

// LDS bytes of one fluid workgroup of `block` threads.
size_t batch_fluid_lds(int block);

hipError_t launch_batch_fluid(int fmt, int block, const BatchStepParams& p, hipStream_t s);
// Boundary pass: nfluid fluid entries, then nsolid solid entries (at + nfluid).
hipError_t launch_batch_boundary(int fmt, const BatchStepParams& p, const uint32_t* cells, const uint32_t* bits,
                                 const uint32_t* yz, const uint16_t* dom, int nfluid, int nsolid, hipStream_t s);
hipError_t launch_step_advance(uint32_t* step, uint32_t n, hipStream_t s);
// Blocks of the strip kernel that fit on one CU (0 on error).
int batch_fluid_occupancy(int fmt, int block);

}  // namespace lbm
