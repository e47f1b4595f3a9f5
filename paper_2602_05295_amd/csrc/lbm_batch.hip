// lbm_batch.hip -- the batched step: many small periodic domains of uneven
// sizes advanced by one persistent fluid launch and one boundary launch.
//
// The fluid pass is the same factorised step as lbm_fluid.hip (the same three
// 1D "reconstruct -> shift -> project" passes in the same order, so a domain
// advanced here matches the single-domain pass up to the compiler's choice of
// fused multiply-adds), laid out for
// domains whose rows are short (24..96 cells in the intended workloads):
//   - a workgroup of NT threads holds a strip of whole x rows of one domain,
//     thread t at row t / nx, column t % nx, so a strip is one contiguous
//     range of every state plane (coalesced loads and stores, no x halo: the
//     x neighbours of the first and last column wrap inside the strip);
//   - a strip that holds every row of the domain (nx * ny <= NT) also wraps
//     in y and loads no halo; otherwise it loads one halo row above and below;
//   - the strip marches through z with the z movers in registers, as in the
//     single-domain pass.
// The host cuts every domain into strips and z runs and deals them to the
// workgroups in balanced, contiguous lists (domain-major), so the workgroups
// of one XCD (consecutive after xcd_logical_block) work on neighbouring strips.
// The dither key of a step comes from a device-side step counter, so a
// captured sequence of launches can be replayed at any later step.
#include "lbm_batch.h"
#include "lbm_boundary_cell.h"
#include "lbm_device.h"

namespace lbm {

const int kBatchBlocks[3] = {256, 512, 1024};

size_t batch_fluid_lds(int block) { return size_t(16 + 18) * size_t(block) * sizeof(float); }

namespace {

template <int FMT>
struct BRaw;
template <>
struct BRaw<FMT_F32> {
  float v[10];
};
template <>
struct BRaw<FMT_Q16> {
  uint32_t v[5];
};

template <int FMT>
__device__ inline BRaw<FMT> bload(const BatchStepParams& a, uint32_t byte_off) {
  BRaw<FMT> r;
  if constexpr (FMT == FMT_F32) {
#pragma unroll
    for (int k = 0; k < 10; ++k) r.v[k] = *reinterpret_cast<const float*>(static_cast<const char*>(a.in[k]) + byte_off);
  } else {
#pragma unroll
    for (int k = 0; k < 5; ++k)
      r.v[k] = *reinterpret_cast<const uint32_t*>(static_cast<const char*>(a.in[k]) + byte_off);
  }
  return r;
}

template <int FMT>
__device__ inline CellIn bdecode(const BRaw<FMT>& r) {
  if constexpr (FMT == FMT_F32)
    return cell_from_moments(r.v);
  else
    return cell_from_words(r.v);
}

// cell: index within the domain (dither input); byte_off: address in the planes.
// STREAM: non-temporal stores, for a state larger than the caches, as in the
// single-domain fluid pass.
template <class T, bool STREAM>
__device__ inline void bstore_word(void* plane, uint32_t byte_off, T v) {
  T* q = reinterpret_cast<T*>(static_cast<char*>(plane) + byte_off);
  if constexpr (STREAM)
    __builtin_nontemporal_store(v, q);
  else
    *q = v;
}

// rest: a solid cell, stored as the rest state whatever was computed.
template <int FMT, bool STREAM>
__device__ inline void bstore(const BatchStepParams& a, uint32_t byte_off, uint32_t cell, uint32_t key, bool dith,
                              float dr, const float j[3], const float P[6], bool rest) {
  if constexpr (FMT == FMT_F32) {
    const float v[10] = {dr, j[0], j[1], j[2], P[0], P[1], P[2], P[3], P[4], P[5]};
#pragma unroll
    for (int k = 0; k < 10; ++k) bstore_word<float, STREAM>(a.out[k], byte_off, rest ? 0.0f : v[k]);
  } else {
    uint32_t w[5], r[5];
    encode_cell(dr, j, P, cell, key, dith, w);
    rest_codes<FMT_Q16>(r);
#pragma unroll
    for (int k = 0; k < 5; ++k) bstore_word<uint32_t, STREAM>(a.out[k], byte_off, rest ? r[k] : w[k]);
  }
}

__device__ inline int wrap1b(int v, int n) { return v < 0 ? v + n : (v >= n ? v - n : v); }

// The point where a plane's state must have arrived: an empty asm that reads
// its registers and that no memory operation may cross.  The plane loop below
// stores a plane's moments at the start of the next iteration, after this
// point and before that iteration's loads, so the wait covers those loads
// alone (a store issued after them would have to complete as well, since one
// counter retires loads and stores in issue order).
template <int FMT>
__device__ inline void bstate_arrived(const BRaw<FMT>& r) {
  constexpr int K = FMT == FMT_F32 ? 10 : 5;
#pragma unroll
  for (int k = 0; k < K; ++k) asm volatile("" : : "v"(r.v[k]) : "memory");
}

template <int FMT, int NT, bool STREAM = false>
__global__ void __launch_bounds__(NT) strip_kernel(BatchStepParams a) {
  __shared__ float ly[16][NT];  // y movers (+, -) of 8 groups
  __shared__ float lx[18][NT];  // x movers (+, -) of 9 groups

  const int tid = int(threadIdx.x);
  const int w = xcd_logical_block(int(blockIdx.x), a.nwg);
  const int mode = FMT == FMT_Q16 ? a.dither_mode : 0;
  const uint32_t key = dither_key(*a.step + a.step_offset, a.seed, mode);
  const bool dith = mode != 0;
  const uint32_t s_end = a.wg_first[w + 1];

  for (uint32_t si = a.wg_first[w]; si < s_end; ++si) {
    const BatchSeg sg = a.segs[si];
    const BatchDomain D = a.doms[sg.dom];
    const int nx = D.nx, ny = D.ny, nz = D.nz, R = D.rows;
    const int r = tid / nx, dx = tid - r * nx;
    const bool active = r < R;
    const bool inner = active && (D.span != 0 || (r >= 1 && r <= R - 2));
    const int gy = D.span ? r : int(sg.strip) * D.ty - 1 + r;
    const bool own = inner && gy < ny;
    const int yw = active ? wrapi(gy, ny) : 0;
    const int up = (D.span && r == 0) ? tid + (R - 1) * nx : tid - nx;      // row r - 1
    const int dn = (D.span && r == R - 1) ? tid - (R - 1) * nx : tid + nx;  // row r + 1
    const int xl = dx == 0 ? tid + nx - 1 : tid - 1;
    const int xr = dx == nx - 1 ? tid - nx + 1 : tid + 1;
    const uint32_t plane = uint32_t(nx) * uint32_t(ny);
    const uint32_t rowc = uint32_t(dx) + uint32_t(nx) * uint32_t(yw);
    const float om1 = D.om1;
    const int za = sg.za, zb = sg.zb;

    // z window: fp of planes p - 2 / p - 1 and f0 of plane p - 1, in paired
    // buffers whose roles swap between the two planes of a trip (no register
    // copies from one plane to the next), as in the single-domain fluid pass
    float wA[6], wB[6], zA[6], zB[6];
#pragma unroll
    for (int g = 0; g < 6; ++g) wA[g] = wB[g] = zA[g] = zB[g] = 0.0f;

    BRaw<FMT> bufA{}, bufB{};
    if (active) bufA = bload<FMT>(a, (D.off + rowc + plane * uint32_t(wrap1b(za - 1, nz))) * 4u);
    const bool keep = own && a.lc.side != nullptr;  // listed cells to look for
    ListedPair lwA{}, lwB{};                        // packed bitmap words of the cells stored next
    // this lane's word of the solid bitmap for the cell stored next, loaded
    // a plane ahead: a solid cell is stored as the rest state
    const bool solids = own && a.lc.solid != nullptr;
    uint32_t swA = 0u, swB = 0u;
    // new moments of the plane finished by the previous step
    float sdr = 0.0f, sj[3] = {0.0f, 0.0f, 0.0f}, sP[6] = {0.0f, 0.0f, 0.0f, 0.0f, 0.0f, 0.0f};
    auto store_plane = [&](int ps, const ListedPair& lws, uint32_t sws) {
      if (own) {
        const uint32_t cell = rowc + plane * uint32_t(ps);
        bstore<FMT, STREAM>(a, (D.off + cell) * 4u, cell, key, dith, sdr, sj, sP,
                            solids && ((sws >> ((D.off + cell) & 31u)) & 1u) != 0u);
        const int slot = keep ? listed_slot_in(listed_word(lws, D.off + cell), D.off + cell) : -1;
        if (slot >= 0) side_store(a.lc.side, uint32_t(slot), sdr, sj, sP);  // a listed cell's unrounded moments
      }
    };
    // One plane p: cur holds its state, nxt receives plane p + 1's; wp2 holds
    // the fp of plane p - 2 and receives this plane's; w0 holds the f0 of plane
    // p - 1, w0out receives this plane's; lw_cur and sw_cur belong to the cell
    // of plane p - 2 (stored now), lw_nxt and sw_nxt receive those of plane
    // p - 1.
    auto plane_step = [&](int p, const BRaw<FMT>& cur, BRaw<FMT>& nxt, float (&wp2)[6], const float (&w0)[6],
                          float (&w0out)[6], const ListedPair& lw_cur, ListedPair& lw_nxt, uint32_t sw_cur,
                          uint32_t& sw_nxt) {
      bstate_arrived<FMT>(cur);
      if (p - 2 >= za) store_plane(p - 2, lw_cur, sw_cur);
      if (keep && p - 1 >= za && p - 1 < zb) lw_nxt = listed_pair(a.lc, D.off + rowc + plane * uint32_t(p - 1));
      if (solids && p - 1 >= za && p - 1 < zb) sw_nxt = a.lc.solid[(D.off + rowc + plane * uint32_t(p - 1)) >> 5];
      if (active && p + 1 <= zb) nxt = bload<FMT>(a, (D.off + rowc + plane * uint32_t(wrap1b(p + 1, nz))) * 4u);

      float f0[8];
      if (active) {
        float A[NA];
        if constexpr (FMT == FMT_F32) {
          const CellIn c = bdecode<FMT>(cur);
          float Nn[6];
          collide_neq(c.N, om1, Nn);
          hermite_coeffs(c.dr, c.j, c.u, Nn, A);
        } else {
          post_collision_codes<FMT_Q16>(cur.v, D.nq_s, D.nq_d, D.nq_c, A);
        }
        // ---- y pass: groups (n, l) with inputs m = 0, 1, 2 along y
        float fp[8], fm[8];
        recon3(A[A000], A[A010], A[A020], f0[0], fp[0], fm[0]);  // (0,0)
        recon3(A[A100], A[A110], A[A120], f0[1], fp[1], fm[1]);  // (1,0)
        recon3(A[A001], A[A011], A[A021], f0[2], fp[2], fm[2]);  // (0,1)
        recon2(A[A200], A[A210], f0[3], fp[3], fm[3]);           // (2,0)
        recon2(A[A002], A[A012], f0[4], fp[4], fm[4]);           // (0,2)
        recon2(A[A101], A[A111], f0[5], fp[5], fm[5]);           // (1,1)
        recon1(A[A201], f0[6], fp[6], fm[6]);                    // (2,1)
        recon1(A[A102], f0[7], fp[7], fm[7]);                    // (1,2)
#pragma unroll
        for (int g = 0; g < 8; ++g) {
          ly[2 * g][tid] = fp[g];
          ly[2 * g + 1][tid] = fm[g];
        }
      }
      __syncthreads();

      float x0v[9];
      if (inner) {
        float Y[8][3];  // Y[g][b] = channel (n, b, l) of y-group g = (n, l)
#pragma unroll
        for (int g = 0; g < 8; ++g) proj3(f0[g], ly[2 * g][up], ly[2 * g + 1][dn], Y[g][0], Y[g][1], Y[g][2]);
        // ---- x pass: groups (b, l) with inputs n = 0, 1, 2 along x
        float xp[9], xm[9];
#pragma unroll
        for (int bb = 0; bb < 3; ++bb) {
          recon3(Y[0][bb], Y[1][bb], Y[3][bb], x0v[3 * bb + 0], xp[3 * bb + 0], xm[3 * bb + 0]);  // l = 0
          recon3(Y[2][bb], Y[5][bb], Y[6][bb], x0v[3 * bb + 1], xp[3 * bb + 1], xm[3 * bb + 1]);  // l = 1
          recon2(Y[4][bb], Y[7][bb], x0v[3 * bb + 2], xp[3 * bb + 2], xm[3 * bb + 2]);            // l = 2
        }
#pragma unroll
        for (int h = 0; h < 9; ++h) {
          lx[2 * h][tid] = xp[h];
          lx[2 * h + 1][tid] = xm[h];
        }
      }
      __syncthreads();

      if (inner) {
        float X00[3], X10[3], X20[3], X01[3], X11[3], X02[3];  // Xab[l] = channel (a, b, l)
#pragma unroll
        for (int l = 0; l < 3; ++l) {
          proj3(x0v[l], lx[2 * l][xl], lx[2 * l + 1][xr], X00[l], X10[l], X20[l]);
          proj2(x0v[3 + l], lx[2 * (3 + l)][xl], lx[2 * (3 + l) + 1][xr], X01[l], X11[l]);
          X02[l] = proj1(x0v[6 + l], lx[2 * (6 + l)][xl], lx[2 * (6 + l) + 1][xr]);
        }
        // ---- z pass: groups (a, b) = (0,0) (1,0) (0,1) (2,0) (1,1) (0,2), inputs l = 0, 1, 2
        float zf0[6], zfp[6], zfm[6];
        recon3(X00[0], X00[1], X00[2], zf0[0], zfp[0], zfm[0]);
        recon3(X10[0], X10[1], X10[2], zf0[1], zfp[1], zfm[1]);
        recon3(X01[0], X01[1], X01[2], zf0[2], zfp[2], zfm[2]);
        recon3(X20[0], X20[1], X20[2], zf0[3], zfp[3], zfm[3]);
        recon3(X11[0], X11[1], X11[2], zf0[4], zfp[4], zfm[4]);
        recon3(X02[0], X02[1], X02[2], zf0[5], zfp[5], zfm[5]);
        if (p > za) {  // plane p - 1 is complete; stored in the next step
          proj3(w0[0], wp2[0], zfm[0], sdr, sj[2], sP[2]);  // (0,0,c): rho-1, jz, Pzz
          proj2(w0[1], wp2[1], zfm[1], sj[0], sP[4]);       // (1,0,c): jx, Pxz
          proj2(w0[2], wp2[2], zfm[2], sj[1], sP[5]);       // (0,1,c): jy, Pyz
          sP[0] = proj1(w0[3], wp2[3], zfm[3]);             // Pxx
          sP[3] = proj1(w0[4], wp2[4], zfm[4]);             // Pxy
          sP[1] = proj1(w0[5], wp2[5], zfm[5]);             // Pyy
        }
#pragma unroll
        for (int g = 0; g < 6; ++g) {
          wp2[g] = zfp[g];  // fp(p - 2) is used up: this slot now holds fp(p)
          w0out[g] = zf0[g];
        }
      }
    };

    // at the start of a trip: state in bufA, fp(p - 2) in wA, fp(p - 1) in wB, f0(p - 1) in zA
    for (int p = za - 1; p <= zb; p += 2) {
      plane_step(p, bufA, bufB, wA, zA, zB, lwA, lwB, swA, swB);
      if (p + 1 <= zb) plane_step(p + 1, bufB, bufA, wB, zB, zA, lwB, lwA, swB, swA);
    }
    // the last step (plane zb) loaded the words of plane zb - 1 into lwB and
    // swB when it ran first in its trip, else into lwA and swA
    if (zb - 1 >= za) {
      if (((zb - za) & 1) != 0)
        store_plane(zb - 1, lwB, swB);
      else
        store_plane(zb - 1, lwA, swA);
    }
  }
}

// The domain's planes are the batch planes offset by the domain's first cell.
template <int FMT>
__device__ inline StepParams domain_params(const BatchStepParams& a, const BatchDomain& D) {
  StepParams p{};
  constexpr int NP = FMT == FMT_F32 ? 10 : 5;
#pragma unroll
  for (int k = 0; k < NP; ++k) {
    p.in[k] = static_cast<const char*>(a.in[k]) + size_t(D.off) * 4u;
    p.out[k] = static_cast<char*>(a.out[k]) + size_t(D.off) * 4u;
  }
  p.g = Geometry{D.nx, D.ny, D.nz, 0};
  p.om1 = D.om1;
  p.nq_s = D.nq_s;
  p.nq_d = D.nq_d;
  p.nq_c = D.nq_c;
  const int mode = FMT == FMT_Q16 ? a.dither_mode : 0;
  p.key = dither_key(*a.step + a.step_offset, a.seed, mode);
  p.dither = mode != 0;
  p.lc = a.lc;
  return p;
}

// Listed fluid cells: one lane each; entry e is slot e of the side buffer
// (the list runs in global cell order, so a domain's entries are contiguous).
template <int FMT>
__global__ void __launch_bounds__(256) batch_boundary_fluid_kernel(BatchStepParams a, const uint32_t* __restrict__ cells,
                                                                   const uint32_t* __restrict__ bits,
                                                                   const uint32_t* __restrict__ yz,
                                                                   const uint16_t* __restrict__ dom, int count) {
  const int e = int(blockIdx.x) * 256 + int(threadIdx.x);
  if (e >= count) return;
  const StepParams p = domain_params<FMT>(a, a.doms[dom[e]]);
  boundary_fix<FMT, false>(p, uint32_t(e), cells[e], bits[e], yz[e], nullptr);
}

template <int FMT>
__global__ void __launch_bounds__(256) batch_boundary_solid_kernel(BatchStepParams a, const uint32_t* __restrict__ cells,
                                                                   const uint16_t* __restrict__ dom, int count) {
  const int e = int(blockIdx.x) * 256 + int(threadIdx.x);
  if (e >= count) return;
  const StepParams p = domain_params<FMT>(a, a.doms[dom[e]]);
  boundary_solid<FMT>(p, cells[e]);
}

__global__ void step_advance_kernel(uint32_t* step, uint32_t n) {
  if (threadIdx.x == 0) step[0] += n;
}

template <int FMT, bool STREAM>
hipError_t launch_nt(int block, const BatchStepParams& p, hipStream_t s) {
  const dim3 grid(uint32_t(p.nwg));
  switch (block) {
    case 256:
      hipLaunchKernelGGL((strip_kernel<FMT, 256, STREAM>), grid, dim3(256), 0, s, p);
      break;
    case 512:
      hipLaunchKernelGGL((strip_kernel<FMT, 512, STREAM>), grid, dim3(512), 0, s, p);
      break;
    case 1024:
      hipLaunchKernelGGL((strip_kernel<FMT, 1024, STREAM>), grid, dim3(1024), 0, s, p);
      break;
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <int FMT, int NT>
int occupancy_of() {
  int n = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, reinterpret_cast<const void*>(strip_kernel<FMT, NT>), NT, 0) !=
      hipSuccess)
    return 0;
  return n;
}

}  // namespace

hipError_t launch_batch_fluid(int fmt, int block, const BatchStepParams& p, hipStream_t s) {
  if (p.nwg <= 0) return hipSuccess;
  if (fmt == FMT_F32) return p.stream_out ? launch_nt<FMT_F32, true>(block, p, s) : launch_nt<FMT_F32, false>(block, p, s);
  return p.stream_out ? launch_nt<FMT_Q16, true>(block, p, s) : launch_nt<FMT_Q16, false>(block, p, s);
}

hipError_t launch_batch_boundary(int fmt, const BatchStepParams& p, const uint32_t* cells, const uint32_t* bits,
                                 const uint32_t* yz, const uint16_t* dom, int nfluid, int nsolid, hipStream_t s) {
  if (nfluid > 0) {
    const dim3 grid(uint32_t((nfluid + 255) / 256));
    if (fmt == FMT_F32)
      hipLaunchKernelGGL(batch_boundary_fluid_kernel<FMT_F32>, grid, dim3(256), 0, s, p, cells, bits, yz, dom, nfluid);
    else
      hipLaunchKernelGGL(batch_boundary_fluid_kernel<FMT_Q16>, grid, dim3(256), 0, s, p, cells, bits, yz, dom, nfluid);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  if (nsolid > 0) {
    const dim3 grid(uint32_t((nsolid + 255) / 256));
    if (fmt == FMT_F32)
      hipLaunchKernelGGL(batch_boundary_solid_kernel<FMT_F32>, grid, dim3(256), 0, s, p, cells + nfluid, dom + nfluid,
                         nsolid);
    else
      hipLaunchKernelGGL(batch_boundary_solid_kernel<FMT_Q16>, grid, dim3(256), 0, s, p, cells + nfluid, dom + nfluid,
                         nsolid);
    return hipGetLastError();
  }
  return hipSuccess;
}

hipError_t launch_step_advance(uint32_t* step, uint32_t n, hipStream_t s) {
  hipLaunchKernelGGL(step_advance_kernel, dim3(1), dim3(64), 0, s, step, n);
  return hipGetLastError();
}

int batch_fluid_occupancy(int fmt, int block) {
  if (fmt == FMT_F32) {
    if (block == 256) return occupancy_of<FMT_F32, 256>();
    if (block == 512) return occupancy_of<FMT_F32, 512>();
    if (block == 1024) return occupancy_of<FMT_F32, 1024>();
  } else {
    if (block == 256) return occupancy_of<FMT_Q16, 256>();
    if (block == 512) return occupancy_of<FMT_Q16, 512>();
    if (block == 1024) return occupancy_of<FMT_Q16, 1024>();
  }
  return 0;
}

}  // namespace lbm
