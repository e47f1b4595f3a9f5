// lbm_internal.h -- host-side declarations shared by the runtime and the kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace lbm {

// FMT_P<b1>_<b2>: the b_rho_u / b_S allocations of the double-layer vortex
// study (codes of rho and u with b1 bits, of the non-equilibrium stress with
// b2 bits), packed low bit first into ceil((4 b1 + 6 b2)/32) words per cell.
enum Format { FMT_F32 = 0, FMT_Q16 = 1, FMT_P16_15 = 2, FMT_P15_14 = 3, FMT_P14_13 = 4, FMT_P13_12 = 5, FMT_P12_11 = 6 };
constexpr int kNumFormats = 7;

// Bits of the rho / u codes and of the stress codes, and words per cell.
constexpr int fmt_b1(int f) { return f == FMT_Q16 ? 16 : f == FMT_P16_15 ? 16 : f == FMT_P15_14 ? 15 : f == FMT_P14_13 ? 14 : f == FMT_P13_12 ? 13 : f == FMT_P12_11 ? 12 : 0; }
constexpr int fmt_b2(int f) { return f == FMT_Q16 ? 16 : f == FMT_P16_15 ? 15 : f == FMT_P15_14 ? 14 : f == FMT_P14_13 ? 13 : f == FMT_P13_12 ? 12 : f == FMT_P12_11 ? 11 : 0; }
constexpr int fmt_words(int f) { return f == FMT_F32 ? 10 : (4 * fmt_b1(f) + 6 * fmt_b2(f) + 31) / 32; }
constexpr bool fmt_packed(int f) { return f >= FMT_P16_15 && f < kNumFormats; }

// Boundary-list entry flags (bits 0..26 mark links i whose source x - c_i is solid).
constexpr uint32_t BIT_INFLOW = 1u << 27;   // cell on the inflow face x = 0
constexpr uint32_t BIT_OUTFLOW = 1u << 28;  // cell on the outflow face x = nx-1
constexpr uint32_t BIT_SOLID = 1u << 29;    // solid cell next to fluid: reset to rest

struct Geometry {
  int nx, ny, nz;
  int inflow;
};

// Listed fluid cells, in raster order: for each 64-cell word c >> 6,
// lpack holds {bits 0..31, bits 32..63, prefix count, 0}; bit (c & 63) marks
// cell c, and its slot (position in the list) is the prefix count plus the
// marked cells before it in that word.  One 16-byte load gives both.
struct ListedCells {
  const uint4* lpack;
  float* side;      // nside records of 12 floats (48 B): the fluid pass's unrounded moments of each listed cell
  uint32_t nside;
  // One bit per cell, set where the cell is solid: bit (c & 31) of word
  // c >> 5.  Given to the fluid pass of open-face domains, which then writes
  // the solid cells' rest state itself (null: the boundary pass does).
  const uint32_t* solid;
};

// Side-buffer record of one listed cell: (rho - 1, j, P) and two pad floats,
// written and read as three 16-byte words.
__device__ inline void side_store(float* side, uint32_t slot, float dr, const float j[3], const float P[6]) {
  float4* r = reinterpret_cast<float4*>(side) + size_t(slot) * 3;
  r[0] = make_float4(dr, j[0], j[1], j[2]);
  r[1] = make_float4(P[0], P[1], P[2], P[3]);
  r[2] = make_float4(P[4], P[5], 0.0f, 0.0f);
}

__device__ inline void side_load(const float* side, uint32_t slot, float m[10]) {
  const float4* r = reinterpret_cast<const float4*>(side) + size_t(slot) * 3;
  const float4 a = r[0], b = r[1], c = r[2];
  m[0] = a.x;
  m[1] = a.y;
  m[2] = a.z;
  m[3] = a.w;
  m[4] = b.x;
  m[5] = b.y;
  m[6] = b.z;
  m[7] = b.w;
  m[8] = c.x;
  m[9] = c.y;
}

// Whether the fluid pass writes the new state with non-temporal stores: when
// the state read and the state written do not both fit in the 256 MiB
// Infinity Cache of the MI355X.  Then keeping the written lines out of the
// caches leaves L2 to the halo rows and columns that neighbouring tiles read
// (measured 1.5% on the 16-bit and 3% on the FP32 256^3 pass); a smaller
// state stays cache-resident between steps, and writing past the cache made
// the 128^3 FP32 pass 24% slower.
inline int stream_out_state(size_t state_bytes_one_buffer) {
  return 2 * state_bytes_one_buffer > (size_t(256) << 20) ? 1 : 0;
}

// The constants of the code-space collision (post_collision_codes) for the
// relaxation om1 = 1 - 1/tau and b2-bit stress codes: nq_s = om1 dN,
// nq_d = nq_s / 3, nq_c = om1 lo_N, with the decode step dN and the range's
// lower end lo_N = -0.1 (Sec. 5.3) as the kernels round them to float.
inline void code_collision_consts(double om1, int b2, float& nq_s, float& nq_d, float& nq_c) {
  const double dn = double(float(0.2 / double((1u << b2) - 1u)));
  nq_s = float(om1 * dn);
  nq_d = float(om1 * dn / 3.0);
  nq_c = float(om1 * double(-0.1f));
}

struct StepParams {
  const void* in[10];  // state planes read (FP32: 10 float planes, Q16: 5 word planes)
  void* out[10];       // state planes written
  Geometry g;
  float om1;           // 1 - 1/tau
  // App. A taken from the stress codes q of an integer format (no force):
  // om1 dev(N) is nq_s q + nq_c off the diagonal and nq_s q - nq_d (q_xx +
  // q_yy + q_zz) on it, with nq_s = om1 dN, nq_d = nq_s / 3, nq_c = om1 lo_N
  float nq_s, nq_d, nq_c;
  uint32_t key;        // dither key of this step (when step_ctr is null)
  int dither;          // 0: round to nearest; else add the dither of `key`
  // In a captured step sequence the key comes from a device-side step
  // counter instead: dither_key(*step_ctr + step_off, seed, dither_mode), so
  // the sequence can be replayed at any later step.
  const uint32_t* step_ctr;
  uint32_t step_off;
  uint32_t seed;
  int dither_mode;
  int stream_out;      // the fluid pass writes the new state with non-temporal stores (stream_out_state)
  float u_in[3];
  float hF[3];         // half the body force, F / 2 (App. A); zero without force
  int force;           // hF != 0
  int wall_rule;       // 0: halfway bounce-back; 1: the moment wall of Sec. 3.2
  const uint8_t* mask;   // solid mask, value = object id (read by the wall rules)
  const float* objects;  // 256 x 9 per object id: center C, velocity V, angular velocity W
  double* forces;        // 256 x 6 sums of force and torque per object id, or nullptr
  ListedCells lc;      // lc.side == nullptr: no listed cells
};

// The packed words of the 64-cell blocks w0 and w0 + 1 (lpack holds one
// padding entry at the end), for a wavefront whose stored cells are
// consecutive and start in block w0: those cells lie in these two blocks.
// The block index is taken from the first active lane, so the two loads are
// scalar ones (no vector memory traffic).
struct ListedPair {
  uint4 a, b;
  uint32_t w0;
};

__device__ inline ListedPair listed_pair(const ListedCells& lc, uint32_t first_cell) {
  const uint32_t w0 = __builtin_amdgcn_readfirstlane(first_cell >> 6);
  return ListedPair{lc.lpack[w0], lc.lpack[w0 + 1], w0};
}

__device__ inline const uint4& listed_word(const ListedPair& pr, uint32_t c) { return (c >> 6) == pr.w0 ? pr.a : pr.b; }

// Slot of cell c given its packed word w, or -1 if c is not listed.
__device__ inline int listed_slot_in(const uint4& w, uint32_t c) {
  const uint32_t bit = c & 63u;
  const unsigned long long m = (static_cast<unsigned long long>(w.y) << 32) | w.x;
  if (((m >> bit) & 1ull) == 0ull) return -1;
  const unsigned long long below = bit == 0 ? 0ull : (m & ((~0ull) >> (64u - bit)));
  return int(w.z + uint32_t(__popcll(below)));
}

// Adjoint of one FP32 step: lam_out = J(m)^T lam_in.
struct AdjParams {
  const float* lam_in[10];  // adjoint of the new moments (10 planes, moment order)
  const float* m[10];       // forward FP32 state (rho - 1, j, P) the step was taken from
  float* lam_out[10];       // adjoint of the old moments
  const uint8_t* flags;     // 1: listed fluid cell, 2: solid cell, 0: other
  Geometry g;
  float om1;
  float u_in[3];
};
// Fluid adjoint (tile height `rows`: 8, 13, or 0 to choose), then the
// boundary pass's changed links: bounce-back over the nfluid listed fluid
// entries (cells / bits), face links over the two x-face planes.
hipError_t launch_adjoint(const AdjParams& p, int rows, const uint32_t* cells, const uint32_t* bits, int nfluid,
                          hipStream_t s);
hipError_t launch_adjoint_flags(const uint8_t* mask, int64_t N, const uint32_t* cells, const uint32_t* bits,
                                int count, uint8_t* flags, hipStream_t s);
hipError_t launch_equilibrium_vjp(const float* rho, const float* u, const float* lam, const uint8_t* mask, int64_t N,
                                  float* grho, float* gu, hipStream_t s);

// Fused fluid pass over every cell (all axes treated periodic).  rows: tile
// height (one of kFluidTileRows) or 0 to let fluid_plan choose.
// The regular items (tile, z segment) cover z in [0, nz - tail) in nseg equal
// segments; when they leave CUs idle, the top `tail` planes of every tile go
// to ntail more workgroups, each taking a contiguous run of tiles.
struct FluidPlan {
  int rows;   // output rows per tile
  int ntx, nty;
  int nseg;   // z segments per tile below the tail
  int nwg;    // workgroups launched (ntail of them on the tail)
  int tail;   // planes in the tail (0: none)
  int ntail;  // workgroups on the tail
};
extern const int kFluidTileRows[4];
FluidPlan fluid_plan(const Geometry& g, int rows, int cus, bool allow_tail = true);
hipError_t launch_fluid(int fmt, const StepParams& p, int rows, hipStream_t s);

// The paper's mixed-precision pipeline (Sec. 5.3, atomic accumulation), on
// 16-bit codes of post-collision moments:
//   stream pass: p.in = the codes, p.out = ten FP32 post-stream planes;
//   link corrections: one thread per changed link (links[k] = 32 e + i, e a
//     listed fluid entry, i its direction), atomicAdd of (new - pulled) times
//     the link's moments into p.out (p.in still the codes);
//   requantize: p.in = the FP32 planes, p.out = the codes: collide (App. A)
//     and encode every cell with the dither of p.key.
hipError_t launch_stream_mixed(const StepParams& p, int rows, hipStream_t s);
hipError_t launch_mixed_links(const StepParams& p, const uint32_t* links, int nlinks, const uint32_t* cells,
                              const uint32_t* yz, const uint32_t* bits, hipStream_t s);
hipError_t launch_requantize(const StepParams& p, int64_t N, hipStream_t s);
// Obstacle meshes of the per-triangle solid correction (Alg. 3): n triangles,
// 9 floats each (three vertices), and the object id of each.
struct TriangleSet {
  const float* tris;
  const uint8_t* obj;
  int n;
  const uint4* lpack;     // the boundary list's packed bitmap (ListedCells::lpack)
  const uint32_t* bits;   // flags of the listed fluid entries, in slot order
};
// Nearest-hit keys: winner[27 slot + i] = min over triangles meeting link i of
// listed fluid entry `slot` of (t bits << 32 | triangle); the list's
// nslots entries, filled first with ~0.
hipError_t launch_triangle_winners(const StepParams& p, const TriangleSet& T, unsigned long long* winner,
                                   int64_t nslots, hipStream_t s);
// One step's corrections (p.in = the post-collision codes, p.out = the FP32
// post-stream planes): each triangle corrects the links it wins.
hipError_t launch_triangle_correction(const StepParams& p, const TriangleSet& T, const unsigned long long* winner,
                                      hipStream_t s);

// Boundary pass: the nfluid listed fluid cells (list order = slot order,
// with their y | z << 16 in yz) take the fluid pass's moments from p.lc.side
// and the corrections of their boundary links; the nsolid listed solid cells
// (solid_cells) are reset to rest.  Without force tracking both lists share
// one launch; the two sets of cells are disjoint.
// order (may be null): the order in which the fluid entries are visited.
hipError_t launch_boundary(int fmt, const StepParams& p, const uint32_t* cells, const uint32_t* bits,
                           const uint32_t* yz, const uint32_t* order, int nfluid, const uint32_t* solid_cells,
                           int nsolid, hipStream_t s);

// Boundary list of one domain whose cells start at global index goff.
// Count pass (lbase == nullptr): counters[0] / [1] receive the fluid / solid
// counts and the fluid cells are OR-ed into lmask (indexed by global cell).
// Fill pass: fluid entries go to their slots (cells_f / bits_f / yz_f are the
// whole list), solid entries to cells_s / bits_s via the cursor counters[3].
hipError_t launch_classify(const uint8_t* mask, const Geometry& g, uint32_t goff, uint32_t* counters,
                           unsigned long long* lmask, const uint32_t* lbase, uint32_t* cells_f, uint32_t* bits_f,
                           uint32_t* yz_f, uint32_t* cells_s, uint32_t* bits_s, uint32_t cap_s, hipStream_t s);
// The solid bitmap of ListedCells::solid for the N cells of mask: (N + 31) / 32 words.
hipError_t launch_solid_bits(const uint8_t* mask, uint32_t N, uint32_t* out, hipStream_t s);

// Codec / initialisation / read-back.
hipError_t launch_set_moments(int fmt, const float* m, void* const out[10], const uint8_t* mask, int64_t N,
                              hipStream_t s);
hipError_t launch_set_equilibrium(int fmt, const float* rho, const float* u, void* const out[10],
                                  const uint8_t* mask, int64_t N, hipStream_t s);
hipError_t launch_get_moments(int fmt, const void* const in[10], float* m, const uint8_t* mask, int64_t N,
                              hipStream_t s);
hipError_t launch_set_rest(int fmt, void* const out[10], int64_t N, hipStream_t s);
hipError_t launch_health(int fmt, const void* const in[10], int64_t N, unsigned long long* bad, hipStream_t s);
hipError_t launch_debug_dither(int n, const uint32_t* idx, uint32_t key, uint32_t* out, hipStream_t s);
// *ctr = v (one thread), ordered on stream s: the step counter of captured sequences.
hipError_t launch_set_counter(uint32_t* ctr, uint32_t v, hipStream_t s);

}  // namespace lbm
