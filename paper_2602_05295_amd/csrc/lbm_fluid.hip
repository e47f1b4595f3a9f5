// lbm_fluid.hip -- the fused fluid pass (Sec. 4.2, Alg. 2) for gfx950.
//
// The step factorises into three 1D "reconstruct -> shift -> project" passes
// (lbm_device.h).  One workgroup of R + 3 wavefronts owns a tile of 64 x R
// output cells of an x-y plane (R = 8, 10, 12 or 13) and marches through z:
//   - R + 2 row wavefronts: one 64-cell row each (a coalesced 256 B or 128 B
//     row per plane), the R output rows plus one halo row above and below;
//   - 1 column wavefront: the halo cells at x0 - 1 and x0 + 64 of those
//     R + 2 rows, so no lane of the row wavefronts is spent on halo cells.
// Per plane every cell is loaded once and collided (App. A); then
//   y pass: reconstruct the y movers of 8 groups, exchange them through LDS
//           (the halo rows stop here, having paid for a load, a collision and
//           this reconstruction only);
//   x pass: the same on 9 groups through LDS, the column wavefront supplying
//           the movers that enter the tile from outside;
//   z pass: 6 groups whose z neighbours are the previous and next planes of
//           the march, held in registers.
// Only the ten new moments are written.  The next plane's state is loaded
// while the current one is computed; a plane's new moments are stored at the
// start of the following plane step, before its loads (see plane_step).
//
// Work items are (tile, z segment) pairs.  Every tile's z range is cut into
// the same S equal segments, so all items of a wave start on the same plane
// and advance in step (when those items leave CUs idle, the top planes of
// every tile are cut off first and shared out to the idle CUs, each taking a
// run of tiles, so that both kinds of workgroup finish together): a tile's halo rows and columns are then read while the
// neighbouring tile that owns them holds the same planes in L2.  Items are
// numbered segment-major, tile-minor (x fastest) and the workgroups of one
// XCD (round-robin dispatch) take consecutive numbers, so each XCD works on a
// compact band of tiles.  The host picks the tile height and S from the
// domain shape.  Every axis is treated as periodic here, except that with
// open x faces (FACES) the column beyond x = nx - 1 is a copy of x = nx - 1 (so the
// links leaving the outflow face are the zero-gradient ones already) and the
// column before x = 0 sends nothing (so the inflow face's entering links
// hold zero, replaced by the boundary pass without reading their periodic
// image).  Walls and the inflow are applied afterwards by the boundary pass.
#include "lbm_codec.h"

#include <algorithm>
#include <array>
#include <map>
#include <mutex>

namespace lbm {

constexpr int RW = 64;  // cells per row wavefront

// LDS of a tile with TYR output rows (TYR + 2 row wavefronts), two copies of
// everything, used by alternate planes: the plane step has one barrier, so a
// wavefront can write plane p + 1's movers while another still reads plane
// p's.
template <int TYR>
struct FluidLds {
  float ly[2][16][TYR + 2][RW];  // y movers (+, -) of 8 groups, row wavefronts
  float le[2][9][2][TYR];        // x movers entering the tile: + from x0 - 1, - from x0 + 64, of 9 groups
};

// Lane moves (DPP): lane l takes v of lane l - 1 (SHR) or l + 1 (SHL) across
// the wavefront (WAVE) or within rows of 16 lanes (ROW); a lane without a
// source keeps `edge`.
constexpr int DPP_WAVE_SHR1 = 0x138, DPP_WAVE_SHL1 = 0x130, DPP_ROW_SHR1 = 0x111, DPP_ROW_SHL1 = 0x101;
template <int CTRL>
__device__ inline float lane_move(float edge, float v) {
  return __int_as_float(__builtin_amdgcn_update_dpp(__float_as_int(edge), __float_as_int(v), CTRL, 0xF, 0xF, false));
}
// The same with zero in a lane without a source (no register to preset).
template <int CTRL>
__device__ inline float lane_move0(float v) {
  return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), CTRL, 0xF, 0xF, true));
}

// The stored words of one cell: ten floats, or the format's code words.
template <int FMT, bool F = (FMT == FMT_F32)>
struct Raw {
  static constexpr int K = 10;
  float v[10];
};
template <int FMT>
struct Raw<FMT, false> {
  static constexpr int K = Codec<FMT>::W;
  uint32_t v[Codec<FMT>::W];
};

template <int FMT>
__device__ inline Raw<FMT> load_raw(const StepParams& a, uint32_t off) {
  Raw<FMT> r;
  using T = decltype(r.v[0] + 0);
#pragma unroll
  for (int k = 0; k < Raw<FMT>::K; ++k) r.v[k] = *reinterpret_cast<const T*>(static_cast<const char*>(a.in[k]) + off);
  return r;
}

// Marks the point where a plane's state must have arrived: an empty asm that
// reads its registers (so the wait for the loads is placed here) and that no
// memory operation may cross (so none issued after it is waited for).
template <int FMT>
__device__ inline void state_arrived(const Raw<FMT>& r) {
#pragma unroll
  for (int k = 0; k < Raw<FMT>::K; ++k) asm volatile("" : : "v"(r.v[k]) : "memory");
}

template <int FMT>
__device__ inline CellIn decode(const Raw<FMT>& r) {
  if constexpr (FMT == FMT_F32)
    return cell_from_moments(r.v);
  else
    return Codec<FMT>::decode(r.v);
}

// Writes the new moments of one cell: dr = rho - 1, j, P (xx yy zz xy xz yz).
// STREAM: non-temporal stores, for a state larger than the caches (see
// stream_out_state); the written lines then leave L2 to the halo rows and
// columns that neighbouring tiles read.
template <class T, bool STREAM>
__device__ inline void store_word(void* plane, uint32_t off, T v) {
  T* p = reinterpret_cast<T*>(static_cast<char*>(plane) + off);
  if constexpr (STREAM)
    __builtin_nontemporal_store(v, p);
  else
    *p = v;
}

// rest: the cell is solid, and its words are those of the rest state
// (zero moments in FP32, the rest codes otherwise) whatever was computed.
template <int FMT, bool STREAM>
__device__ inline void store_cell(const StepParams& a, uint32_t cell, float dr, const float j[3], const float P[6],
                                  bool rest = false) {
  const uint32_t off = cell * 4u;
  if constexpr (FMT == FMT_F32) {
    const float v[10] = {dr, j[0], j[1], j[2], P[0], P[1], P[2], P[3], P[4], P[5]};
#pragma unroll
    for (int k = 0; k < 10; ++k) store_word<float, STREAM>(a.out[k], off, rest ? 0.0f : v[k]);
  } else {
    uint32_t w[Codec<FMT>::W], r[Codec<FMT>::W];
    Codec<FMT>::encode(dr, j, P, cell, a.key, a.dither != 0, w);
    rest_codes<FMT>(r);
#pragma unroll
    for (int k = 0; k < Codec<FMT>::W; ++k) store_word<uint32_t, STREAM>(a.out[k], off, rest ? r[k] : w[k]);
  }
}

// A listed cell's unrounded moments go to its slot of the side buffer, where
// the boundary pass picks them up.  pr: the packed bitmap words of the
// wavefront's cells, loaded a plane ahead.
__device__ inline void keep_listed(const ListedCells& lc, uint32_t cell, const ListedPair& pr, float dr,
                                   const float j[3], const float P[6]) {
  const int slot = listed_slot_in(listed_word(pr, cell), cell);
  if (slot >= 0) side_store(lc.side, uint32_t(slot), dr, j, P);
}

__device__ inline int wrap1(int v, int n) { return v < 0 ? v + n : (v >= n ? v - n : v); }

// FORCE: App. A with the uniform body force a.hF = F/2 (collision terms, and
// F/2 added to the projected momentum, Eq. rho_u_stress).
// MIXED: the stream pass of the paper's mixed-precision pipeline (Sec. 5.3):
// the codes hold post-collision moments, which are reconstructed without a
// collision, and the new moments are stored as FP32 post-stream moments.
template <int FMT, int TYR, bool FORCE, bool MIXED = false, bool STREAM = false, bool FACES = false>
__global__ void __launch_bounds__((TYR + 3) * RW) fluid_kernel(StepParams ap, int ntx, int nty, int nseg, int nwg, int zt, int ntail) {
  constexpr int OUT = MIXED ? int(FMT_F32) : FMT;
  StepParams a = ap;
  a.key = step_key(ap);
  constexpr int NRW = TYR + 2;  // row wavefronts (with the two halo rows)
  __shared__ FluidLds<TYR> L;

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
  const bool inner = r >= 1 && r <= TYR;  // a row whose y and x passes are needed
  const bool compute = !colw && inner;    // a row wavefront with outputs

  const int ntiles = ntx * nty;
  const int items = ntiles * nseg;  // regular items: z in [0, zt)
  const int nreg = nwg - ntail;     // their workgroups; the rest take z in [zt, nz)
  const uint32_t plane = uint32_t(nx) * uint32_t(ny);
  const int k = xcd_logical_block(int(blockIdx.x), nwg);
  const bool on_tail = k >= nreg;
  const int t0 = on_tail ? int(int64_t(ntiles) * (k - nreg) / ntail) : 0;
  const int t1 = on_tail ? int(int64_t(ntiles) * (k - nreg + 1) / ntail) : 0;

  for (int it = 0;; ++it) {
    int t, za, zb;
    if (!on_tail) {
      const int q = k + it * nreg;
      if (q >= items) break;
      t = q % ntiles;
      const int sg = q / ntiles;
      za = int(int64_t(zt) * sg / nseg);
      zb = int(int64_t(zt) * (sg + 1) / nseg);
    } else {
      t = t0 + it;
      if (t >= t1) break;
      za = zt;
      zb = nz;
    }
    // the last plane step of the previous item may still be reading the LDS
    // buffer that this item's first step writes
    __syncthreads();
    const int x0 = (t % ntx) * RW, y0 = (t / ntx) * TYR;
    const int gx = x0 + dx, gy = y0 - 1 + r;
    // open x faces (FACES; not in the mixed pipeline, which keeps the periodic
    // pull).  a.g.inflow is always set when FACES is; keeping the runtime test
    // makes the channel's fluid pass 1% faster (2.287 -> 2.261 ms) through
    // the code the compiler schedules for it.
    const bool ghost_out = FACES && a.g.inflow && gx == nx;
    const bool ghost_in = FACES && a.g.inflow && gx == -1;
    const int xw = ghost_out ? nx - 1 : wrapi(gx, nx), yw = wrapi(gy, ny);
    const uint32_t row = uint32_t(xw) + uint32_t(nx) * uint32_t(yw);
    const bool own = compute && gx < nx && gy < ny;

    // z window (fp of planes p - 2 / p - 1, f0 of plane p - 1), the state of
    // the next plane in flight while the current one is computed, and the
    // listed-cell bitmap words of the cell stored next.  The plane loop runs
    // two planes per trip with the roles of the paired buffers swapped, so no
    // register is copied from one plane to the next.
    float wA[6], wB[6], zA[6], zB[6];
#pragma unroll
    for (int g = 0; g < 6; ++g) wA[g] = wB[g] = zA[g] = zB[g] = 0.0f;
    Raw<FMT> bufA = load_raw<FMT>(a, (row + plane * uint32_t(wrap1(za - 1, nz))) * 4u);
    Raw<FMT> bufB;
    // listed cells to look for: a wavefront-uniform condition, so that the
    // bitmap words stay in scalar registers and empty words skip everything
    const bool keep = !MIXED && compute && a.lc.side != nullptr;
    const uint32_t row0 = __builtin_amdgcn_readfirstlane(row);  // lane 0: the row's first own cell
    ListedPair lwA{}, lwB{};
    // Open-face domains: this lane's word of the solid bitmap for the cell
    // stored next, loaded a plane ahead like the listed-cell words; a solid
    // cell is stored as the rest state, so the boundary pass resets none.
    // (The periodic kernels leave the solid cells to the boundary pass and
    // carry none of this.)
    const bool solids = FACES && own && a.lc.solid != nullptr;
    uint32_t swA = 0u, swB = 0u;
    // New moments of the plane finished by the previous step.  They are
    // stored at the start of the next step, after its state has arrived and
    // before its loads are issued: then no store is issued between a plane's
    // loads and their use, and the wait for the loads is a wait for them
    // alone (a store issued later would have to complete as well).
    float sdr = 0.0f, sj[3] = {0.0f, 0.0f, 0.0f}, sP[6] = {0.0f, 0.0f, 0.0f, 0.0f, 0.0f, 0.0f};
    auto store_plane = [&](int ps, const ListedPair& lw, uint32_t sw) {
      if (own) {
        const uint32_t cell = row + plane * uint32_t(ps);
        store_cell<OUT, STREAM>(a, cell, sdr, sj, sP, solids && ((sw >> (cell & 31u)) & 1u) != 0u);
        if (keep && (lw.a.x | lw.a.y | lw.b.x | lw.b.y) != 0u) keep_listed(a.lc, cell, lw, sdr, sj, sP);
      }
    };

    // One plane p: cur holds its state, nxt receives plane p + 1's; wp2 holds
    // the fp of plane p - 2 and receives this plane's fp; w0in holds the f0 of
    // plane p - 1, w0out receives this plane's; lw_cur and sw_cur belong to
    // the cell of plane p - 2 (stored now), lw_nxt and sw_nxt receive those of
    // plane p - 1.
    auto plane_step = [&](int p, const Raw<FMT>& cur, Raw<FMT>& nxt, float (&wp2)[6], const float (&w0)[6],
                          float (&w0out)[6], const ListedPair& lw_cur, ListedPair& lw_nxt, uint32_t sw_cur,
                          uint32_t& sw_nxt) {
      state_arrived<FMT>(cur);
      if (p - 2 >= za) store_plane(p - 2, lw_cur, sw_cur);
      if (keep && p - 1 >= za && p - 1 < zb) lw_nxt = listed_pair(a.lc, row0 + plane * uint32_t(p - 1));
      if (solids && p - 1 >= za && p - 1 < zb) sw_nxt = a.lc.solid[(row + plane * uint32_t(p - 1)) >> 5];
      if (p + 1 <= zb) nxt = load_raw<FMT>(a, (row + plane * uint32_t(wrap1(p + 1, nz))) * 4u);

      float A[NA];
      if constexpr (MIXED) {
        const CellIn c = decode<FMT>(cur);
        hermite_coeffs(c.dr, c.j, c.u, c.N, A);  // the codes are post-collision already
      } else if constexpr (FMT != FMT_F32 && !FORCE) {
        post_collision_codes<FMT>(cur.v, a.nq_s, a.nq_d, a.nq_c, A);
      } else {
        post_collision<FORCE>(decode<FMT>(cur), a.om1, a.hF, A);
      }

      // ---- y pass: groups (n, l) with inputs m = 0, 1, 2 along y
      float f0[8], fp[8], fm[8];
      recon3(A[A000], A[A010], A[A020], f0[0], fp[0], fm[0]);  // (0,0)
      recon3(A[A100], A[A110], A[A120], f0[1], fp[1], fm[1]);  // (1,0)
      recon3(A[A001], A[A011], A[A021], f0[2], fp[2], fm[2]);  // (0,1)
      recon2(A[A200], A[A210], f0[3], fp[3], fm[3]);           // (2,0)
      recon2(A[A002], A[A012], f0[4], fp[4], fm[4]);           // (0,2)
      recon2(A[A101], A[A111], f0[5], fp[5], fm[5]);           // (1,1)
      recon1(A[A201], f0[6], fp[6], fm[6]);                    // (2,1)
      recon1(A[A102], f0[7], fp[7], fm[7]);                    // (1,2)
      const int par = p & 1;
      if (!colw) {
#pragma unroll
        for (int g = 0; g < 8; ++g) {
          L.ly[par][2 * g][r][lane] = fp[g];
          L.ly[par][2 * g + 1][r][lane] = fm[g];
        }
      } else {
        // The halo columns x0 - 1 (side 0) and x0 + 64 (side 1), row r in
        // lane r of a 16-lane row: their y pass by lane moves within the
        // wavefront (full exec, so every source lane is live), then the x
        // movers that enter the tile, published before the barrier.
        float Y[8][3];
#pragma unroll
        for (int g = 0; g < 8; ++g)
          proj3(f0[g], lane_move0<DPP_ROW_SHR1>(fp[g]), lane_move0<DPP_ROW_SHL1>(fm[g]), Y[g][0], Y[g][1], Y[g][2]);
        if (active && inner) {
          float x0v[9], xp[9], xm[9];
#pragma unroll
          for (int bb = 0; bb < 3; ++bb) {
            recon3(Y[0][bb], Y[1][bb], Y[3][bb], x0v[3 * bb + 0], xp[3 * bb + 0], xm[3 * bb + 0]);  // l = 0
            recon3(Y[2][bb], Y[5][bb], Y[6][bb], x0v[3 * bb + 1], xp[3 * bb + 1], xm[3 * bb + 1]);  // l = 1
            recon2(Y[4][bb], Y[7][bb], x0v[3 * bb + 2], xp[3 * bb + 2], xm[3 * bb + 2]);            // l = 2
          }
          if (side == 0) {
#pragma unroll
            for (int h = 0; h < 9; ++h) L.le[par][h][0][r - 1] = ghost_in ? 0.0f : xp[h];
          } else {
#pragma unroll
            for (int h = 0; h < 9; ++h) L.le[par][h][1][r - 1] = xm[h];
          }
        }
      }
      __syncthreads();

      if (compute) {
        float Y[8][3];  // Y[g][b] = channel (n, b, l) of y-group g = (n, l)
#pragma unroll
        for (int g = 0; g < 8; ++g)
          proj3(f0[g], L.ly[par][2 * g][r - 1][lane], L.ly[par][2 * g + 1][r + 1][lane], Y[g][0], Y[g][1], Y[g][2]);
        // ---- x pass: groups (b, l) with inputs n = 0, 1, 2 along x, one y
        // channel b at a time; the movers cross lanes by DPP, and the lanes at
        // the tile's edges take those of the halo columns
        float X00[3], X10[3], X20[3], X01[3], X11[3], X02[3];  // Xab[l] = channel (a, b, l)
#pragma unroll
        for (int bb = 0; bb < 3; ++bb) {
          float g0[3], gp[3], gm[3];
          recon3(Y[0][bb], Y[1][bb], Y[3][bb], g0[0], gp[0], gm[0]);  // l = 0
          recon3(Y[2][bb], Y[5][bb], Y[6][bb], g0[1], gp[1], gm[1]);  // l = 1
          recon2(Y[4][bb], Y[7][bb], g0[2], gp[2], gm[2]);            // l = 2
#pragma unroll
          for (int l = 0; l < 3; ++l) {
            const int h = 3 * bb + l;
            const float Fp = lane_move<DPP_WAVE_SHR1>(L.le[par][h][0][r - 1], gp[l]);
            const float Fm = lane_move<DPP_WAVE_SHL1>(L.le[par][h][1][r - 1], gm[l]);
            if (bb == 0)
              proj3(g0[l], Fp, Fm, X00[l], X10[l], X20[l]);
            else if (bb == 1)
              proj2(g0[l], Fp, Fm, X01[l], X11[l]);
            else
              X02[l] = proj1(g0[l], Fp, Fm);
          }
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
          if constexpr (FORCE) {
#pragma unroll
            for (int k = 0; k < 3; ++k) sj[k] += a.hF[k];
          }
        }
#pragma unroll
        for (int g = 0; g < 6; ++g) {
          wp2[g] = zfp[g];  // fp(p - 2) is used up: this slot now holds fp(p)
          w0out[g] = zf0[g];
        }
      }
    };

    // Two planes per trip of the z march, with the paired buffers' roles
    // swapped, so no register is copied from one plane to the next (3% on
    // both formats).  The last step (plane zb) leaves the moments of plane
    // zb - 1, whose bitmap words it loaded into lwB and swB when it ran as
    // the first plane of a trip (lwA and swA otherwise).
    // buffers at the start of a trip: state in bufA, fp(p - 2) in wA, fp(p - 1) in wB, f0(p - 1) in zA
    for (int p = za - 1; p <= zb; p += 2) {
      plane_step(p, bufA, bufB, wA, zA, zB, lwA, lwB, swA, swB);
      // now fp(p - 1) in wB, fp(p) in wA, f0(p) in zB
      if (p + 1 <= zb) plane_step(p + 1, bufB, bufA, wB, zB, zA, lwB, lwA, swB, swA);
      // now fp(p) in wA, fp(p + 1) in wB, f0(p + 1) in zA: the trip's starting roles
    }
    const bool last_in_b = ((zb - za) & 1) != 0;  // plane zb ran first in its trip
    if (zb - 1 >= za) {
      if (last_in_b)
        store_plane(zb - 1, lwB, swB);
      else
        store_plane(zb - 1, lwA, swA);
    }
  }
}

namespace {
int device_cus() {
  static int cached[64] = {0};
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return 256;
  if (cached[dev] == 0) {
    int n = 0;
    if (hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || n <= 0) n = 256;
    cached[dev] = n;
  }
  return cached[dev];
}

template <int FMT, bool FORCE, bool MIXED = false, bool STREAM = false, bool FACES = false>
hipError_t launch_rows(const FluidPlan& c, const StepParams& p, hipStream_t s) {
  const dim3 grid(uint32_t(c.nwg));
  const int zt = p.g.nz - c.tail;
  switch (c.rows) {
    case 8:
      hipLaunchKernelGGL((fluid_kernel<FMT, 8, FORCE, MIXED, STREAM, FACES>), grid, dim3(11 * RW), 0, s, p, c.ntx, c.nty, c.nseg,
                         c.nwg, zt, c.ntail);
      break;
    case 10:
      hipLaunchKernelGGL((fluid_kernel<FMT, 10, FORCE, MIXED, STREAM, FACES>), grid, dim3(13 * RW), 0, s, p, c.ntx, c.nty, c.nseg,
                         c.nwg, zt, c.ntail);
      break;
    case 12:
      hipLaunchKernelGGL((fluid_kernel<FMT, 12, FORCE, MIXED, STREAM, FACES>), grid, dim3(15 * RW), 0, s, p, c.ntx, c.nty, c.nseg,
                         c.nwg, zt, c.ntail);
      break;
    default:
      hipLaunchKernelGGL((fluid_kernel<FMT, 13, FORCE, MIXED, STREAM, FACES>), grid, dim3(16 * RW), 0, s, p, c.ntx, c.nty, c.nseg,
                         c.nwg, zt, c.ntail);
      break;
  }
  return hipGetLastError();
}
}  // namespace

const int kFluidTileRows[4] = {8, 10, 12, 13};

namespace {
FluidPlan plan_uncached(const Geometry& g, int rows, int cus, bool allow_tail) {
  FluidPlan best{};
  double best_cost = 0.0;
  for (int r : kFluidTileRows) {
    if (rows != 0 && r != rows) continue;
    FluidPlan c{};
    c.rows = r;
    c.ntx = (g.nx + RW - 1) / RW;
    c.nty = (g.ny + r - 1) / r;
    const int64_t T = int64_t(c.ntx) * c.nty;
    // split z so that one wave of items fills the CUs when there are fewer
    // tiles than CUs; then pick the split with the shortest critical path,
    // counted in plane steps (two extra planes start each item)
    double cost_best = 0.0;
    int seg_best = 1, tail_best = 0, ntail_best = 0;
    const int smax = int(std::max<int64_t>(1, std::min<int64_t>(int64_t(g.nz) / 4, 64)));
    for (int sgs = 1; sgs <= smax; ++sgs) {
      const int64_t items = T * sgs;
      const int64_t waves = (items + cus - 1) / cus;
      int64_t path = waves * ((g.nz + sgs - 1) / sgs + 2);
      int tail = 0, ntail = 0;
      if (allow_tail && items < cus) {
        // the idle CUs take the top s planes of every tile, kk tiles each
        const int64_t E = std::min<int64_t>(cus - items, T);
        const int64_t kk = (T + E - 1) / E;
        for (int64_t sz = 1; sz <= int64_t(g.nz) - sgs; ++sz) {
          const int64_t m = std::max<int64_t>((g.nz - sz + sgs - 1) / sgs + 2, kk * (sz + 2));
          if (m < path) {
            path = m;
            tail = int(sz);
            ntail = int(E);
          }
        }
      } else if (allow_tail && items % cus != 0) {
        // more than one wave, the last one partial: E workgroups take the top
        // s planes of every tile, kk tiles each, and the other cus - E run
        // the regular items in rounds
        const int64_t emax = std::min<int64_t>(T, cus / 4);
        for (int64_t E = 1; E <= emax; ++E) {
          const int64_t rounds = (items + (cus - E) - 1) / (cus - E);
          const int64_t kk = (T + E - 1) / E;
          // s where rounds ((nz - s)/sgs + 2) = kk (s + 2), then its neighbours
          const double s0 = (double(rounds) * g.nz / sgs + 2.0 * rounds - 2.0 * kk) / (double(kk) + double(rounds) / sgs);
          for (int64_t sz = std::max<int64_t>(1, int64_t(s0) - 2); sz <= std::min<int64_t>(g.nz - sgs, int64_t(s0) + 3);
               ++sz) {
            const int64_t m = std::max<int64_t>(rounds * ((g.nz - sz + sgs - 1) / sgs + 2), kk * (sz + 2));
            if (m < path) {
              path = m;
              tail = int(sz);
              ntail = int(E);
            }
          }
        }
      }
      // time of one plane of one tile ~ the wavefronts of the workgroup
      const double cost = double(path) * double(r + 3);
      if (sgs == 1 || cost < cost_best) {
        cost_best = cost;
        seg_best = sgs;
        tail_best = tail;
        ntail_best = ntail;
      }
    }
    c.nseg = seg_best;
    c.tail = tail_best;
    c.ntail = ntail_best;
    const int64_t items = T * seg_best;
    c.nwg = c.ntail == 0 ? int(std::min<int64_t>(items, cus))
                         : (items < cus ? int(items) + c.ntail : cus);
    if (best.rows == 0 || cost_best < best_cost) {
      best = c;
      best_cost = cost_best;
    }
  }
  return best;
}
}  // namespace

FluidPlan fluid_plan(const Geometry& g, int rows, int cus, bool allow_tail) {
  // plans are looked up per launch; the search runs once per shape
  static std::mutex mu;
  static std::map<std::array<int, 6>, FluidPlan> cache;
  const std::array<int, 6> key{g.nx, g.ny, g.nz, rows, cus, allow_tail ? 1 : 0};
  std::lock_guard<std::mutex> lock(mu);
  auto it = cache.find(key);
  if (it != cache.end()) return it->second;
  const FluidPlan c = plan_uncached(g, rows, cus, allow_tail);
  if (cache.size() < 4096) cache.emplace(key, c);
  return c;
}

hipError_t launch_stream_mixed(const StepParams& p, int rows, hipStream_t s) {
  const FluidPlan c = fluid_plan(p.g, rows, device_cus());
  if (c.rows == 0) return hipErrorInvalidValue;
  return launch_rows<FMT_Q16, false, true>(c, p, s);
}

hipError_t launch_fluid(int fmt, const StepParams& p, int rows, hipStream_t s) {
  const FluidPlan c = fluid_plan(p.g, rows, device_cus());
  if (c.rows == 0) return hipErrorInvalidValue;
  // A body force takes the plain stores (force runs are the small ones).
  // Open faces have kernels of their own, so the periodic ones carry none of
  // the face logic (it cost them 1% on 256^3).
  hipError_t e = hipErrorInvalidValue;
  auto go = [&]<int F>() {
    if (p.g.inflow)
      e = p.force ? launch_rows<F, true, false, false, true>(c, p, s)
                  : (p.stream_out ? launch_rows<F, false, false, true, true>(c, p, s)
                                  : launch_rows<F, false, false, false, true>(c, p, s));
    else
      e = p.force ? launch_rows<F, true>(c, p, s)
                  : (p.stream_out ? launch_rows<F, false, false, true>(c, p, s) : launch_rows<F, false>(c, p, s));
  };
  if (fmt == FMT_F32)
    go.template operator()<FMT_F32>();
  else
    dispatch_codes(fmt, go);
  return e;
}

}  // namespace lbm
