// lbm_api.hip -- the C ABI declared in include/homelbm.h: context, buffers,
// boundary list, step loop.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <iterator>
#include <cstdio>
#include <map>
#include <mutex>
#include <utility>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "../../include/homelbm.h"
#include "lbm_device.h"
#include "lbm_internal.h"

using namespace lbm;

struct lbm_ctx {
  int nx = 0, ny = 0, nz = 0;
  int64_t N = 0;
  double tau = 0.0;
  int fmt = 0;
  lbm_options opt{};
  hipStream_t stream = nullptr;
  void* buf[2] = {nullptr, nullptr};  // ping-pong state buffers
  int cur = 0;
  uint8_t* d_mask = nullptr;          // copy of the solid mask (nullptr: no solids)
  uint32_t* d_cells = nullptr;        // boundary list
  uint32_t* d_bits = nullptr;
  uint32_t* d_yz = nullptr;           // y | z << 16 of the fluid entries
  unsigned long long* d_lmask = nullptr;  // listed fluid cells: bitmap, prefix counts, side buffer
  uint32_t* d_lbase = nullptr;
  uint4* d_lpack = nullptr;               // the two packed per word for the fluid and boundary passes
  uint32_t* d_order = nullptr;            // boundary pass order of the fluid entries: face cells first
  float* d_side = nullptr;
  uint32_t* d_solid = nullptr;            // solid bitmap (ListedCells::solid), built with the list
  int64_t n_fluid_b = 0, n_solid_b = 0;
  int64_t n_fluid_run = 0;                // fluid entries the boundary pass visits (d_order's length, if any)
  uint32_t* d_counters = nullptr;     // 3 list counters
  unsigned long long* d_bad = nullptr;
  uint8_t* d_flags = nullptr;         // adjoint cell flags (built on first use)
  float h_objects[256 * 9] = {};      // per object id: center, velocity, angular velocity
  float* d_objects = nullptr;         // device copy of h_objects
  double* d_forces = nullptr;         // 256 x 6 force and torque sums (track_forces)
  // the paper's mixed-precision pipeline (pipeline 1): buf[cur] holds the codes
  // of post-collision moments, d_ps the FP32 post-stream moments
  float* d_ps = nullptr;
  uint32_t* d_links = nullptr;        // changed links, 32 e + i
  int64_t n_links = 0;
  bool links_built = false;
  // obstacle meshes of wall rule 2 (per-triangle solid correction)
  float* d_tris = nullptr;
  uint8_t* d_tri_obj = nullptr;
  int64_t n_tris = 0;
  // tile height of the fluid pass picked by timing (options.tile_rows = 0); 0 until then
  int tuned_rows = 0;
  unsigned long long* d_winner = nullptr;  // nearest-hit key per listed fluid entry and link
  bool winners_built = false;
  bool flags_valid = false;
  bool list_built = false;
  int list_inflow = -1;
  uint64_t t = 0;
  // captured step sequences (graph_steps > 0): the dither key of each step
  // comes from the device-side counter d_step, set before every replay
  uint32_t* d_step = nullptr;
  hipStream_t cap = nullptr;                              // capture stream
  std::map<std::pair<int, int>, hipGraphExec_t> graphs;  // (steps, first buffer) -> sequence
  std::string err;
};

namespace {

thread_local std::string g_err;

int fail(lbm_ctx* c, int code, const std::string& msg) {
  if (c)
    c->err = msg;
  else
    g_err = msg;
  return code;
}

int hip_fail(lbm_ctx* c, hipError_t e, const char* what) {
  const int code = (e == hipErrorOutOfMemory) ? LBM_ERR_OUT_OF_MEMORY : LBM_ERR_DEVICE;
  return fail(c, code, std::string(what) + ": " + hipGetErrorString(e));
}

size_t plane_bytes(const lbm_ctx* c) { return size_t(c->N) * 4; }
int n_planes(const lbm_ctx* c) { return fmt_words(c->fmt); }
size_t state_bytes(const lbm_ctx* c) { return plane_bytes(c) * n_planes(c); }

void planes_of(const lbm_ctx* c, void* base, void* out[10]) {
  for (int k = 0; k < 10; ++k) out[k] = (k < n_planes(c)) ? static_cast<char*>(base) + size_t(k) * plane_bytes(c) : nullptr;
}

Geometry geom(const lbm_ctx* c) { return Geometry{c->nx, c->ny, c->nz, c->opt.inflow}; }

void drop_graphs(lbm_ctx* c) {
  for (auto& kv : c->graphs) (void)hipGraphExecDestroy(kv.second);
  c->graphs.clear();
}

void free_list(lbm_ctx* c) {
  drop_graphs(c);  // they hold the list's pointers
  if (c->d_cells) (void)hipFree(c->d_cells);
  if (c->d_bits) (void)hipFree(c->d_bits);
  if (c->d_yz) (void)hipFree(c->d_yz);
  if (c->d_lmask) (void)hipFree(c->d_lmask);
  if (c->d_lbase) (void)hipFree(c->d_lbase);
  if (c->d_lpack) (void)hipFree(c->d_lpack);
  if (c->d_order) (void)hipFree(c->d_order);
  if (c->d_side) (void)hipFree(c->d_side);
  if (c->d_solid) (void)hipFree(c->d_solid);
  c->d_cells = c->d_bits = c->d_yz = c->d_lbase = nullptr;
  c->d_solid = nullptr;
  c->d_lmask = nullptr;
  c->d_lpack = nullptr;
  c->d_order = nullptr;
  c->d_side = nullptr;
  c->n_fluid_b = c->n_solid_b = c->n_fluid_run = 0;
  c->list_built = false;
  c->flags_valid = false;
  c->links_built = false;
  c->winners_built = false;
  if (c->d_winner) (void)hipFree(c->d_winner);
  c->d_winner = nullptr;
}

// Builds the boundary list on the device: count pass (counts and the bitmap
// of listed fluid cells), prefix counts of the bitmap on the host, exact
// allocation, fill pass.
int build_list(lbm_ctx* c) {
  free_list(c);
  const Geometry g = geom(c);
  if (!c->d_mask && !g.inflow) {
    c->list_built = true;
    c->list_inflow = g.inflow;
    return LBM_OK;
  }
  const size_t nchunks = size_t((c->N + 63) / 64);
  hipError_t e = hipMalloc(&c->d_lmask, nchunks * 8);
  if (e == hipSuccess) e = hipMalloc(&c->d_lbase, nchunks * 4);
  if (e == hipSuccess) e = hipMemsetAsync(c->d_lmask, 0, nchunks * 8, c->stream);
  if (e == hipSuccess) e = hipMemsetAsync(c->d_counters, 0, 4 * sizeof(uint32_t), c->stream);
  if (e != hipSuccess) return hip_fail(c, e, "boundary list setup");
  e = launch_classify(c->d_mask, g, 0, c->d_counters, c->d_lmask, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr,
                      0, c->stream);
  if (e != hipSuccess) return hip_fail(c, e, "classify (count)");
  uint32_t cnt[4] = {0, 0, 0, 0};
  std::vector<unsigned long long> hmask(nchunks);
  e = hipMemcpyAsync(cnt, c->d_counters, sizeof(cnt), hipMemcpyDeviceToHost, c->stream);
  if (e == hipSuccess) e = hipMemcpyAsync(hmask.data(), c->d_lmask, nchunks * 8, hipMemcpyDeviceToHost, c->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
  if (e != hipSuccess) return hip_fail(c, e, "reading list counts");
  std::vector<uint32_t> hbase(nchunks);
  uint32_t run = 0;
  for (size_t k = 0; k < nchunks; ++k) {
    hbase[k] = run;
    run += uint32_t(__builtin_popcountll(hmask[k]));
  }
  if (run != cnt[0]) return fail(c, LBM_ERR_DEVICE, "boundary list: bitmap and count disagree");
  std::vector<uint4> hpack(nchunks + 1, make_uint4(0u, 0u, 0u, 0u));  // one padding entry
  for (size_t k = 0; k < nchunks; ++k)
    hpack[k] = make_uint4(uint32_t(hmask[k]), uint32_t(hmask[k] >> 32), hbase[k], 0u);
  e = hipMemcpy(c->d_lbase, hbase.data(), nchunks * 4, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMalloc(&c->d_lpack, (nchunks + 1) * sizeof(uint4));
  if (e == hipSuccess) e = hipMemcpy(c->d_lpack, hpack.data(), (nchunks + 1) * sizeof(uint4), hipMemcpyHostToDevice);
  if (e != hipSuccess) return hip_fail(c, e, "uploading list offsets");
  const int64_t total = int64_t(cnt[0]) + cnt[1];
  int64_t run_fluid = cnt[0];
  if (total > 0) {
    e = hipMalloc(&c->d_cells, size_t(total) * 4);
    if (e == hipSuccess) e = hipMalloc(&c->d_bits, size_t(total) * 4);
    if (e == hipSuccess) e = hipMalloc(&c->d_yz, size_t(std::max<uint32_t>(cnt[0], 1)) * 4);
    if (e == hipSuccess) e = hipMalloc(&c->d_side, size_t(std::max<uint32_t>(cnt[0], 1)) * 48);
    if (e != hipSuccess) return hip_fail(c, e, "hipMalloc(boundary list)");
    // fluid entries in raster order, solid entries after them
    e = hipMemsetAsync(c->d_counters, 0, 4 * sizeof(uint32_t), c->stream);
    if (e == hipSuccess)
      e = launch_classify(c->d_mask, g, 0, c->d_counters, c->d_lmask, c->d_lbase, c->d_cells, c->d_bits, c->d_yz,
                          c->d_cells + cnt[0], c->d_bits + cnt[0], cnt[1], c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) return hip_fail(c, e, "classify (fill)");
    if (g.inflow && cnt[0] > 0) {
      // The boundary pass visits the inflow face first (nine links each, in
      // wavefronts of their own), then the other cells with changed links.
      // An outflow face cell with no other flag is skipped: the fluid pass
      // already wrote its final state.  (The list keeps it for the mixed
      // pipeline and the adjoint.)
      std::vector<uint32_t> hbits(cnt[0]), order;
      order.reserve(cnt[0]);
      e = hipMemcpy(hbits.data(), c->d_bits, size_t(cnt[0]) * 4, hipMemcpyDeviceToHost);
      if (e != hipSuccess) return hip_fail(c, e, "reading list flags");
      for (uint32_t k = 0; k < cnt[0]; ++k)
        if (hbits[k] & BIT_INFLOW) order.push_back(k);
      for (uint32_t k = 0; k < cnt[0]; ++k)
        if (!(hbits[k] & BIT_INFLOW) && (hbits[k] & ~BIT_OUTFLOW) != 0u) order.push_back(k);
      if (!order.empty()) {
        e = hipMalloc(&c->d_order, order.size() * 4);
        if (e == hipSuccess) e = hipMemcpy(c->d_order, order.data(), order.size() * 4, hipMemcpyHostToDevice);
        if (e != hipSuccess) return hip_fail(c, e, "uploading the boundary order");
      }
      run_fluid = int64_t(order.size());
    }
  }
  if (c->d_mask) {
    e = hipMalloc(&c->d_solid, size_t((c->N + 31) / 32) * 4);
    if (e == hipSuccess) e = launch_solid_bits(c->d_mask, uint32_t(c->N), c->d_solid, c->stream);
    if (e != hipSuccess) return hip_fail(c, e, "solid bitmap");
  }
  c->n_fluid_b = cnt[0];
  c->n_fluid_run = run_fluid;
  c->n_solid_b = cnt[1];
  c->list_built = true;
  c->list_inflow = g.inflow;
  c->links_built = false;
  return LBM_OK;
}

int check_faces(lbm_ctx* c, const lbm_options& o) {
  if (!o.inflow) return LBM_OK;
  if (c->nx < 6) return fail(c, LBM_ERR_INVALID_ARG, "inflow needs nx >= 6");
  for (int a = 0; a < 3; ++a)
    if (!std::isfinite(o.u_in[a]) || std::fabs(o.u_in[a]) > 0.4f)
      return fail(c, LBM_ERR_INVALID_ARG, "u_in must be finite with |u_in| <= 0.4");
  return LBM_OK;
}

StepParams step_params(const lbm_ctx* c, const void* in, void* out) {
  StepParams p{};
  void* pin[10];
  planes_of(c, const_cast<void*>(in), pin);
  void* pout[10];
  planes_of(c, out, pout);
  for (int k = 0; k < 10; ++k) {
    p.in[k] = pin[k];
    p.out[k] = pout[k];
  }
  p.g = geom(c);
  p.om1 = float(1.0 - 1.0 / c->tau);
  if (c->fmt != FMT_F32) code_collision_consts(1.0 - 1.0 / c->tau, fmt_b2(c->fmt), p.nq_s, p.nq_d, p.nq_c);
  const int mode = c->fmt != FMT_F32 ? c->opt.dither_mode : 0;
  p.dither = mode != 0;
  p.key = dither_key(uint32_t(c->t), c->opt.seed, mode);
  p.stream_out = stream_out_state(state_bytes(c));
  for (int a = 0; a < 3; ++a) p.u_in[a] = c->opt.u_in[a];
  for (int a = 0; a < 3; ++a) p.hF[a] = 0.5f * c->opt.force[a];
  p.force = (c->opt.force[0] != 0.0f || c->opt.force[1] != 0.0f || c->opt.force[2] != 0.0f) ? 1 : 0;
  p.wall_rule = c->opt.wall_rule;
  p.mask = c->d_mask;
  p.objects = c->d_objects;
  p.forces = c->opt.track_forces ? c->d_forces : nullptr;
  if (c->n_fluid_b > 0) p.lc = ListedCells{c->d_lpack, c->d_side, uint32_t(c->n_fluid_b)};
  p.lc.solid = c->d_solid;
  return p;
}

// The kernels of one step on stream s: fluid pass then boundary pass.
// The fluid pass's tile height: the caller's, else the timed choice, else
// the planner's (before the timing has run).
int fluid_rows(const lbm_ctx* c) { return c->opt.tile_rows != 0 ? c->opt.tile_rows : c->tuned_rows; }

int launch_pass(lbm_ctx* c, const StepParams& p, hipStream_t s, hipEvent_t ev[4]) {
  hipError_t e = hipSuccess;
  if (ev) e = hipEventRecord(ev[0], s);
  if (e == hipSuccess) e = launch_fluid(c->fmt, p, fluid_rows(c), s);
  if (e == hipSuccess && ev) e = hipEventRecord(ev[1], s);
  if (e != hipSuccess) return hip_fail(c, e, "fluid pass");
  // the fluid pass of an open-face domain wrote the solid cells' rest state
  const int64_t nsolid = (p.g.inflow && p.lc.solid) ? 0 : c->n_solid_b;
  const int64_t n = c->n_fluid_b + nsolid;
  if (n > 0) {
    if (ev) e = hipEventRecord(ev[2], s);
    if (e == hipSuccess)
      e = launch_boundary(c->fmt, p, c->d_cells, c->d_bits, c->d_yz, c->d_order, int(c->n_fluid_run),
                          c->d_cells + c->n_fluid_b, int(nsolid), s);
    if (e == hipSuccess && ev) e = hipEventRecord(ev[3], s);
    if (e != hipSuccess) return hip_fail(c, e, "boundary pass");
  }
  return LBM_OK;
}

// With tile_rows = 0: times the fluid pass once for every tile height, from
// the current state into the other buffer (the state is unchanged), and keeps
// the fastest.  The heights take turns, three rounds after two warm-up
// launches, and each keeps its best time: a new context's first launches run
// slow, and no height should take them all.  Every tile height gives the
// same result, so the choice changes the speed only.
int tune_rows(lbm_ctx* c) {
  if (c->opt.tile_rows != 0 || c->tuned_rows != 0 || c->opt.pipeline == 1) return LBM_OK;
  const StepParams p = step_params(c, c->buf[c->cur], c->buf[1 - c->cur]);
  constexpr int NR = int(sizeof(kFluidTileRows) / sizeof(kFluidTileRows[0]));
  float best[NR];
  for (float& b : best) b = 3.0e38f;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  hipError_t e = hipEventCreate(&e0);
  if (e == hipSuccess) e = hipEventCreate(&e1);
  for (int k = 0; k < 2 && e == hipSuccess; ++k) e = launch_fluid(c->fmt, p, kFluidTileRows[k % NR], c->stream);
  for (int rep = 0; rep < 3 && e == hipSuccess; ++rep)
    for (int i = 0; i < NR && e == hipSuccess; ++i) {
      e = hipEventRecord(e0, c->stream);
      if (e == hipSuccess) e = launch_fluid(c->fmt, p, kFluidTileRows[i], c->stream);
      if (e == hipSuccess) e = hipEventRecord(e1, c->stream);
      if (e == hipSuccess) e = hipEventSynchronize(e1);
      float ms = 0.0f;
      if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
      if (e == hipSuccess) best[i] = std::min(best[i], ms);
    }
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  if (e != hipSuccess) return hip_fail(c, e, "timing the tile heights");
  int k = 0;
  for (int i = 1; i < NR; ++i)
    if (best[i] < best[k]) k = i;
  c->tuned_rows = kFluidTileRows[k];
  drop_graphs(c);  // none should hold another height, but captures made before the timing would
  return LBM_OK;
}

// One step from in to out: fluid pass then boundary pass.
int enqueue_pass(lbm_ctx* c, const void* in, void* out, hipEvent_t ev[4]) {
  const int r = launch_pass(c, step_params(c, in, out), c->stream, ev);
  if (r != LBM_OK) return r;
  c->t += 1;
  return LBM_OK;
}

// One step of the context's own state, buffers swapped.
int enqueue_step(lbm_ctx* c, hipEvent_t ev[4]) {
  const int r = enqueue_pass(c, c->buf[c->cur], c->buf[1 - c->cur], ev);
  if (r == LBM_OK) c->cur = 1 - c->cur;
  return r;
}

// The captured sequence of k steps starting from buffer `first`: step j reads
// buf[(first + j) & 1], writes the other, and takes its dither key from the
// device counter plus j.
int graph_for(lbm_ctx* c, int k, int first, hipGraphExec_t* out) {
  const auto key = std::make_pair(k, first);
  auto it = c->graphs.find(key);
  if (it != c->graphs.end()) {
    *out = it->second;
    return LBM_OK;
  }
  if (c->graphs.size() >= 8) drop_graphs(c);
  hipError_t e = hipSuccess;
  if (!c->cap) e = hipStreamCreateWithFlags(&c->cap, hipStreamNonBlocking);
  if (e != hipSuccess) return hip_fail(c, e, "hipStreamCreate (capture)");
  e = hipStreamBeginCapture(c->cap, hipStreamCaptureModeThreadLocal);
  if (e != hipSuccess) return hip_fail(c, e, "hipStreamBeginCapture");
  int r = LBM_OK;
  for (int j = 0; j < k && r == LBM_OK; ++j) {
    StepParams p = step_params(c, c->buf[(first + j) & 1], c->buf[(first + j + 1) & 1]);
    p.step_ctr = c->d_step;
    p.step_off = uint32_t(j);
    p.seed = c->opt.seed;
    p.dither_mode = c->fmt != FMT_F32 ? c->opt.dither_mode : 0;
    r = launch_pass(c, p, c->cap, nullptr);
  }
  hipGraph_t g = nullptr;
  const hipError_t e2 = hipStreamEndCapture(c->cap, &g);
  if (r != LBM_OK) {
    if (g) (void)hipGraphDestroy(g);
    return r;
  }
  if (e2 != hipSuccess) return hip_fail(c, e2, "hipStreamEndCapture");
  hipGraphExec_t x = nullptr;
  e = hipGraphInstantiate(&x, g, nullptr, nullptr, 0);
  (void)hipGraphDestroy(g);
  if (e != hipSuccess) return hip_fail(c, e, "hipGraphInstantiate");
  e = hipGraphUpload(x, c->stream);  // ahead of the first launch
  if (e != hipSuccess) {
    (void)hipGraphExecDestroy(x);
    return hip_fail(c, e, "hipGraphUpload");
  }
  c->graphs[key] = x;
  *out = x;
  return LBM_OK;
}

// ---- the mixed pipeline
void ps_planes(const lbm_ctx* c, void* pl[10]) {
  for (int k = 0; k < 10; ++k) pl[k] = c->d_ps + size_t(k) * size_t(c->N);
}

int build_links(lbm_ctx* c) {
  std::vector<uint32_t> hb(size_t(c->n_fluid_b));
  hipError_t e = hipSuccess;
  if (c->n_fluid_b > 0) e = hipMemcpy(hb.data(), c->d_bits, hb.size() * 4, hipMemcpyDeviceToHost);
  if (e != hipSuccess) return hip_fail(c, e, "reading the boundary list");
  std::vector<uint32_t> links;
  for (size_t k = 0; k < hb.size(); ++k) {
    const uint32_t b = hb[k];
    if (b & (BIT_INFLOW | BIT_OUTFLOW)) {
      const int cx = (b & BIT_INFLOW) ? 1 : -1;
      for (int cz = -1; cz <= 1; ++cz)
        for (int cy = -1; cy <= 1; ++cy) links.push_back(uint32_t(k) * 32u + uint32_t((cx + 1) + 3 * (cy + 1) + 9 * (cz + 1)));
    } else if (c->opt.wall_rule != 2) {  // wall rule 2: the triangles correct the solid links
      for (uint32_t i = 0; i < 27; ++i)
        if (i != 13 && ((b >> i) & 1u)) links.push_back(uint32_t(k) * 32u + i);
    }
  }
  if (c->d_links) (void)hipFree(c->d_links);
  c->d_links = nullptr;
  c->n_links = int64_t(links.size());
  if (!links.empty()) {
    e = hipMalloc(&c->d_links, links.size() * 4);
    if (e == hipSuccess) e = hipMemcpy(c->d_links, links.data(), links.size() * 4, hipMemcpyHostToDevice);
    if (e != hipSuccess) return hip_fail(c, e, "uploading the link list");
  }
  c->links_built = true;
  return LBM_OK;
}

// Codes of collide(d_ps) into buf[cur], then the listed solid cells to rest.
int mixed_requantize(lbm_ctx* c, bool dither, hipEvent_t ev0, hipEvent_t ev1) {
  StepParams p = step_params(c, c->buf[c->cur], c->buf[c->cur]);
  void* pl[10];
  ps_planes(c, pl);
  for (int k = 0; k < 10; ++k) p.in[k] = pl[k];
  if (!dither) p.dither = 0;
  hipError_t e = hipSuccess;
  if (ev0) e = hipEventRecord(ev0, c->stream);
  if (e == hipSuccess) e = launch_requantize(p, c->N, c->stream);
  if (e == hipSuccess && c->n_solid_b > 0)
    e = launch_boundary(c->fmt, p, nullptr, nullptr, nullptr, nullptr, 0, c->d_cells + c->n_fluid_b, int(c->n_solid_b),
                        c->stream);
  if (e == hipSuccess && ev1) e = hipEventRecord(ev1, c->stream);
  if (e != hipSuccess) return hip_fail(c, e, "requantize");
  return LBM_OK;
}

// Nearest-hit keys of wall rule 2's links (static geometry: built once per
// boundary list and triangle set).
int build_winners(lbm_ctx* c) {
  if (!c->d_tris || c->n_tris <= 0) return fail(c, LBM_ERR_INVALID_ARG, "wall_rule 2 needs lbm_set_triangles");
  hipError_t e = hipSuccess;
  if (!c->d_winner && c->n_fluid_b > 0) e = hipMalloc(&c->d_winner, size_t(c->n_fluid_b) * 27 * 8);
  if (e != hipSuccess) return hip_fail(c, e, "hipMalloc(triangle winners)");
  if (c->n_fluid_b > 0) {
    const StepParams p = step_params(c, c->buf[c->cur], c->buf[c->cur]);
    const TriangleSet T{c->d_tris, c->d_tri_obj, int(c->n_tris), c->d_lpack, c->d_bits};
    e = launch_triangle_winners(p, T, c->d_winner, c->n_fluid_b, c->stream);
    if (e != hipSuccess) return hip_fail(c, e, "triangle winners");
  }
  c->winners_built = true;
  return LBM_OK;
}

// One step of the mixed pipeline: stream pass, link corrections, requantize.
int enqueue_mixed_step(lbm_ctx* c, hipEvent_t ev[6]) {
  if (!c->links_built) {
    const int r = build_links(c);
    if (r != LBM_OK) return r;
  }
  if (c->opt.wall_rule == 2 && !c->winners_built) {
    const int r = build_winners(c);
    if (r != LBM_OK) return r;
  }
  StepParams p = step_params(c, c->buf[c->cur], c->buf[c->cur]);
  void* pl[10];
  ps_planes(c, pl);
  for (int k = 0; k < 10; ++k) p.out[k] = pl[k];
  p.lc = ListedCells{};
  hipError_t e = hipSuccess;
  if (ev) e = hipEventRecord(ev[0], c->stream);
  if (e == hipSuccess) e = launch_stream_mixed(p, c->opt.tile_rows, c->stream);
  if (e == hipSuccess && ev) e = hipEventRecord(ev[1], c->stream);
  if (e == hipSuccess && ev) e = hipEventRecord(ev[2], c->stream);
  if (e == hipSuccess)
    e = launch_mixed_links(p, c->d_links, int(c->n_links), c->d_cells, c->d_yz, c->d_bits, c->stream);
  if (e == hipSuccess && c->opt.wall_rule == 2) {
    // the stream pass keeps no side records (p.lc is empty); the triangles
    // find listed cells through the list's own bitmap
    const TriangleSet T{c->d_tris, c->d_tri_obj, int(c->n_tris), c->d_lpack, c->d_bits};
    e = launch_triangle_correction(p, T, c->d_winner, c->stream);
  }
  if (e == hipSuccess && ev) e = hipEventRecord(ev[3], c->stream);
  if (e != hipSuccess) return hip_fail(c, e, "mixed stream pass");
  const int r = mixed_requantize(c, true, ev ? ev[4] : nullptr, ev ? ev[5] : nullptr);
  if (r != LBM_OK) return r;
  c->t += 1;
  return LBM_OK;
}

// Moves the state between the two pipelines (same moments, other storage).
int switch_pipeline(lbm_ctx* c, int to) {
  hipError_t e = hipSuccess;
  if (!c->d_ps) {
    e = hipMalloc(&c->d_ps, size_t(c->N) * 40);
    if (e != hipSuccess) return hip_fail(c, e, "allocating the FP32 post-stream buffer");
  }
  void* pl[10];
  ps_planes(c, pl);
  const void* cpl[10];
  for (int k = 0; k < 10; ++k) cpl[k] = pl[k];
  void* qpl[10];
  planes_of(c, c->buf[c->cur], qpl);
  const void* cqpl[10];
  for (int k = 0; k < 10; ++k) cqpl[k] = qpl[k];
  if (to == 1) {
    // codes of pre-collision moments -> full moments in d_ps -> FP32 state layout (in place) -> requantize
    e = launch_get_moments(c->fmt, cqpl, c->d_ps, c->d_mask, c->N, c->stream);
    if (e == hipSuccess) e = launch_set_moments(FMT_F32, c->d_ps, pl, c->d_mask, c->N, c->stream);
    if (e != hipSuccess) return hip_fail(c, e, "entering the mixed pipeline");
    return mixed_requantize(c, false, nullptr, nullptr);
  }
  // FP32 post-stream moments -> full moments (in place) -> codes of pre-collision moments
  e = launch_get_moments(FMT_F32, cpl, c->d_ps, c->d_mask, c->N, c->stream);
  if (e == hipSuccess) e = launch_set_moments(c->fmt, c->d_ps, qpl, c->d_mask, c->N, c->stream);
  if (e != hipSuccess) return hip_fail(c, e, "leaving the mixed pipeline");
  return LBM_OK;
}

int scan_health(lbm_ctx* c, uint64_t* bad) {
  hipError_t e = hipMemsetAsync(c->d_bad, 0, sizeof(unsigned long long), c->stream);
  void* pl[10];
  planes_of(c, c->buf[c->cur], pl);
  const void* cpl[10];
  for (int k = 0; k < 10; ++k) cpl[k] = pl[k];
  if (e == hipSuccess) e = launch_health(c->fmt, cpl, c->N, c->d_bad, c->stream);
  unsigned long long h = 0;
  if (e == hipSuccess) e = hipMemcpyAsync(&h, c->d_bad, sizeof(h), hipMemcpyDeviceToHost, c->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
  if (e != hipSuccess) return hip_fail(c, e, "health scan");
  *bad = h;
  return LBM_OK;
}

}  // namespace

extern "C" {

int lbm_default_options(lbm_options* o) {
  if (!o) return LBM_ERR_INVALID_ARG;
  std::memset(o, 0, sizeof(*o));
  o->dither_mode = LBM_DITHER_PER_STEP;
  o->seed = 0;
  o->inflow = 0;
  o->check_health = 1;
  o->graph_steps = 256;
  return LBM_OK;
}

const char* lbm_last_error(const lbm_ctx* c) { return c ? c->err.c_str() : g_err.c_str(); }

namespace {
int scratch_device_ptr(lbm_ctx* c, uint8_t** out);
}

int lbm_create(const int dims[3], double tau, const uint8_t* mask, int fmt, lbm_ctx** out) {
  if (!out) return fail(nullptr, LBM_ERR_INVALID_ARG, "out is NULL");
  *out = nullptr;
  if (!dims) return fail(nullptr, LBM_ERR_INVALID_ARG, "dims is NULL");
  for (int a = 0; a < 3; ++a)
    if (dims[a] < 1 || dims[a] > 65535)
      return fail(nullptr, LBM_ERR_INVALID_ARG, "every dimension must be in [1, 65535]");
  const int64_t N = int64_t(dims[0]) * dims[1] * dims[2];
  if (N > (int64_t(1) << 30)) return fail(nullptr, LBM_ERR_INVALID_ARG, "nx*ny*nz must be <= 2^30");
  if (!(tau > 0.5) || !std::isfinite(tau)) return fail(nullptr, LBM_ERR_INVALID_ARG, "tau must be > 1/2");
  if (fmt < LBM_MOMENTS_FP32 || fmt > LBM_MOMENTS_P12_11)
    return fail(nullptr, LBM_ERR_INVALID_ARG, "unknown moment format");
  bool any_solid = false;
  if (mask)
    for (int64_t k = 0; k < N && !any_solid; ++k) any_solid = mask[k] != 0;
  lbm_ctx* c = new (std::nothrow) lbm_ctx();
  if (!c) return fail(nullptr, LBM_ERR_OUT_OF_MEMORY, "host allocation failed");
  c->nx = dims[0];
  c->ny = dims[1];
  c->nz = dims[2];
  c->N = N;
  c->tau = tau;
  c->fmt = fmt;
  lbm_default_options(&c->opt);
  hipError_t e = hipSuccess;
  for (int b = 0; b < 2 && e == hipSuccess; ++b) e = hipMalloc(&c->buf[b], state_bytes(c));
  if (e == hipSuccess) e = hipMalloc(&c->d_counters, 4 * sizeof(uint32_t));
  if (e == hipSuccess) e = hipMalloc(&c->d_step, sizeof(uint32_t));
  if (e == hipSuccess) e = hipMalloc(&c->d_bad, sizeof(unsigned long long));
  if (e == hipSuccess) e = hipMalloc(&c->d_objects, sizeof(c->h_objects));
  if (e == hipSuccess) e = hipMemcpy(c->d_objects, c->h_objects, sizeof(c->h_objects), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMalloc(&c->d_forces, 256 * 6 * sizeof(double));
  if (e == hipSuccess) e = hipMemset(c->d_forces, 0, 256 * 6 * sizeof(double));
  if (e == hipSuccess && any_solid) {
    e = hipMalloc(&c->d_mask, size_t(N));
    if (e == hipSuccess) e = hipMemcpy(c->d_mask, mask, size_t(N), hipMemcpyHostToDevice);
  }
  if (e != hipSuccess) {
    hip_fail(nullptr, e, "lbm_create allocation");
    const int code = (e == hipErrorOutOfMemory) ? LBM_ERR_OUT_OF_MEMORY : LBM_ERR_DEVICE;
    lbm_destroy(c);
    return code;
  }
  // rest state
  void* pl[10];
  planes_of(c, c->buf[0], pl);
  e = launch_set_rest(fmt, pl, c->N, c->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
  if (e != hipSuccess) {
    hip_fail(nullptr, e, "lbm_create initial state");
    lbm_destroy(c);
    return LBM_ERR_DEVICE;
  }
  const int r = build_list(c);
  if (r != LBM_OK) {
    g_err = c->err;
    lbm_destroy(c);
    return r;
  }
  // set-up of the allocation-free adjoint: the device address of its scratch
  // array on this device, taken here, before any caller starts a capture
  uint8_t* ignored = nullptr;
  (void)scratch_device_ptr(c, &ignored);  // a failure is reported by lbm_adjoint_step_noalloc itself
  c->err.clear();
  *out = c;
  return LBM_OK;
}

int lbm_destroy(lbm_ctx* c) {
  if (!c) return LBM_OK;
  (void)hipStreamSynchronize(c->stream);
  for (int b = 0; b < 2; ++b)
    if (c->buf[b]) (void)hipFree(c->buf[b]);
  if (c->d_mask) (void)hipFree(c->d_mask);
  free_list(c);
  if (c->d_counters) (void)hipFree(c->d_counters);
  if (c->d_step) (void)hipFree(c->d_step);
  if (c->cap) (void)hipStreamDestroy(c->cap);
  if (c->d_bad) (void)hipFree(c->d_bad);
  if (c->d_flags) (void)hipFree(c->d_flags);
  if (c->d_objects) (void)hipFree(c->d_objects);
  if (c->d_forces) (void)hipFree(c->d_forces);
  if (c->d_ps) (void)hipFree(c->d_ps);
  if (c->d_tris) (void)hipFree(c->d_tris);
  if (c->d_tri_obj) (void)hipFree(c->d_tri_obj);
  if (c->d_winner) (void)hipFree(c->d_winner);
  if (c->d_links) (void)hipFree(c->d_links);
  delete c;
  return LBM_OK;
}

int lbm_set_stream(lbm_ctx* c, void* s) {
  if (!c) return fail(nullptr, LBM_ERR_INVALID_ARG, "ctx is NULL");
  c->stream = static_cast<hipStream_t>(s);
  return LBM_OK;
}

int lbm_set_options(lbm_ctx* c, const lbm_options* o) {
  if (!c || !o) return fail(c, LBM_ERR_INVALID_ARG, "NULL argument");
  if (o->dither_mode < 0 || o->dither_mode > 2) return fail(c, LBM_ERR_INVALID_ARG, "unknown dither mode");
  if (o->tile_rows != 0 && std::find(std::begin(kFluidTileRows), std::end(kFluidTileRows), o->tile_rows) ==
                               std::end(kFluidTileRows))
    return fail(c, LBM_ERR_INVALID_ARG, "tile_rows must be 0, 8, 10, 12 or 13");
  for (int a = 0; a < 3; ++a)
    if (!std::isfinite(o->force[a]) || std::fabs(o->force[a]) > 0.01f)
      return fail(c, LBM_ERR_INVALID_ARG, "force must be finite with |F_a| <= 0.01");
  if (o->wall_rule < 0 || o->wall_rule > 2) return fail(c, LBM_ERR_INVALID_ARG, "wall_rule must be 0, 1 or 2");
  if (o->wall_rule == 2 && o->pipeline != 1)
    return fail(c, LBM_ERR_UNSUPPORTED, "wall_rule 2 (per-triangle solid correction) runs in the mixed pipeline");
  if (o->pipeline != 0 && o->pipeline != 1) return fail(c, LBM_ERR_INVALID_ARG, "pipeline must be 0 or 1");
  if (o->pipeline == 1 && (c->fmt != FMT_Q16 || o->force[0] != 0.0f || o->force[1] != 0.0f ||
                           o->force[2] != 0.0f || o->track_forces != 0))
    return fail(c, LBM_ERR_UNSUPPORTED, "the mixed pipeline runs 16-bit contexts without body force or force tracking");
  if (o->track_forces != 0 && o->track_forces != 1) return fail(c, LBM_ERR_INVALID_ARG, "track_forces must be 0 or 1");
  if (o->graph_steps < 0 || o->graph_steps > 4096)
    return fail(c, LBM_ERR_INVALID_ARG, "graph_steps must be in [0, 4096]");
  int r = check_faces(c, *o);
  if (r != LBM_OK) return r;
  if (o->inflow && c->d_mask) {
    // no solid cell within two cells of the x faces
    const int64_t plane = int64_t(c->nx);
    std::vector<uint8_t> h(size_t(c->N));
    hipError_t e = hipMemcpy(h.data(), c->d_mask, size_t(c->N), hipMemcpyDeviceToHost);
    if (e != hipSuccess) return hip_fail(c, e, "reading mask");
    for (int64_t k = 0; k < c->N; ++k) {
      const int x = int(k % plane);
      if (h[size_t(k)] && (x < 3 || x > c->nx - 4))
        return fail(c, LBM_ERR_INVALID_ARG, "solid cells within two cells of an open x face");
    }
  }
  const int old_inflow = c->opt.inflow, old_pipeline = c->opt.pipeline;
  drop_graphs(c);  // captured steps hold the old options
  // another kernel variant may prefer another tile height
  const bool forced = c->opt.force[0] != 0.0f || c->opt.force[1] != 0.0f || c->opt.force[2] != 0.0f;
  const bool forced_new = o->force[0] != 0.0f || o->force[1] != 0.0f || o->force[2] != 0.0f;
  if (old_inflow != o->inflow || forced != forced_new || o->tile_rows != c->opt.tile_rows) c->tuned_rows = 0;
  if (o->wall_rule != c->opt.wall_rule) c->links_built = false;  // wall rule 2 keeps only the face links
  c->opt = *o;
  c->opt.pipeline = old_pipeline;
  if (!c->list_built || old_inflow != o->inflow) {
    r = build_list(c);
    if (r != LBM_OK) return r;
  }
  if (o->pipeline != old_pipeline) {
    r = switch_pipeline(c, o->pipeline);
    if (r != LBM_OK) return r;
    c->opt.pipeline = o->pipeline;
  }
  return LBM_OK;
}

int lbm_get_options(const lbm_ctx* c, lbm_options* o) {
  if (!c || !o) return LBM_ERR_INVALID_ARG;
  *o = c->opt;
  return LBM_OK;
}

static int stage_in(lbm_ctx* c, const void* src, size_t bytes, int on_device, void** dev, bool* owned) {
  *owned = false;
  if (on_device) {
    *dev = const_cast<void*>(src);
    return LBM_OK;
  }
  hipError_t e = hipMalloc(dev, bytes);
  if (e == hipSuccess) e = hipMemcpyAsync(*dev, src, bytes, hipMemcpyHostToDevice, c->stream);
  if (e != hipSuccess) return hip_fail(c, e, "staging host input");
  *owned = true;
  return LBM_OK;
}

int lbm_set_moments(lbm_ctx* c, const float* m, int on_device) {
  if (!c || !m) return fail(c, LBM_ERR_INVALID_ARG, "NULL argument");
  void* dm;
  bool owned;
  int r = stage_in(c, m, size_t(c->N) * 40, on_device, &dm, &owned);
  if (r != LBM_OK) return r;
  void* pl[10];
  planes_of(c, c->buf[c->cur], pl);
  const bool mixed = c->opt.pipeline == 1;
  if (mixed) ps_planes(c, pl);
  hipError_t e = launch_set_moments(mixed ? int(FMT_F32) : c->fmt, static_cast<const float*>(dm), pl, c->d_mask, c->N,
                                    c->stream);
  if (e == hipSuccess && mixed && mixed_requantize(c, false, nullptr, nullptr) != LBM_OK) e = hipErrorUnknown;
  if (e == hipSuccess && owned) e = hipStreamSynchronize(c->stream);
  if (owned) (void)hipFree(dm);
  if (e != hipSuccess) return hip_fail(c, e, "set_moments");
  return LBM_OK;
}

int lbm_set_equilibrium(lbm_ctx* c, const float* rho, const float* u, int on_device) {
  if (!c || !rho || !u) return fail(c, LBM_ERR_INVALID_ARG, "NULL argument");
  void *dr, *du;
  bool o1, o2;
  int r = stage_in(c, rho, size_t(c->N) * 4, on_device, &dr, &o1);
  if (r != LBM_OK) return r;
  r = stage_in(c, u, size_t(c->N) * 12, on_device, &du, &o2);
  if (r != LBM_OK) {
    if (o1) (void)hipFree(dr);
    return r;
  }
  void* pl[10];
  planes_of(c, c->buf[c->cur], pl);
  const bool mixed = c->opt.pipeline == 1;
  if (mixed) ps_planes(c, pl);
  hipError_t e = launch_set_equilibrium(mixed ? int(FMT_F32) : c->fmt, static_cast<const float*>(dr),
                                        static_cast<const float*>(du), pl, c->d_mask, c->N, c->stream);
  if (e == hipSuccess && mixed && mixed_requantize(c, false, nullptr, nullptr) != LBM_OK) e = hipErrorUnknown;
  if (e == hipSuccess && (o1 || o2)) e = hipStreamSynchronize(c->stream);
  if (o1) (void)hipFree(dr);
  if (o2) (void)hipFree(du);
  if (e != hipSuccess) return hip_fail(c, e, "set_equilibrium");
  return LBM_OK;
}

int lbm_step(lbm_ctx* c, int n) {
  if (!c) return fail(nullptr, LBM_ERR_INVALID_ARG, "ctx is NULL");
  if (n < 0) return fail(c, LBM_ERR_INVALID_ARG, "n must be >= 0");
  if (!c->list_built) {
    const int r = build_list(c);
    if (r != LBM_OK) return r;
  }
  if (n > 0) {
    const int r = tune_rows(c);
    if (r != LBM_OK) return r;
  }
  const bool graphs = c->opt.graph_steps > 0 && c->opt.pipeline != 1;
  int left = n;
  while (left > 0) {
    if (graphs && left >= 2) {
      // a replay of up to graph_steps captured steps, keys from the counter set here
      const int k = std::min(left, c->opt.graph_steps);
      hipGraphExec_t x = nullptr;
      int r = graph_for(c, k, c->cur, &x);
      if (r != LBM_OK) return r;
      hipError_t e = launch_set_counter(c->d_step, uint32_t(c->t), c->stream);
      if (e == hipSuccess) e = hipGraphLaunch(x, c->stream);
      if (e != hipSuccess) return hip_fail(c, e, "hipGraphLaunch");
      c->cur = (c->cur + k) & 1;
      c->t += uint64_t(k);
      left -= k;
      continue;
    }
    const int r = c->opt.pipeline == 1 ? enqueue_mixed_step(c, nullptr) : enqueue_step(c, nullptr);
    if (r != LBM_OK) return r;
    --left;
  }
  if (c->opt.check_health && n > 0) {
    uint64_t bad = 0;
    const int r = scan_health(c, &bad);
    if (r != LBM_OK) return r;
    if (bad) return fail(c, LBM_ERR_UNSTABLE, "state holds " + std::to_string(bad) + " non-finite or saturated values");
  }
  return LBM_OK;
}

int lbm_set_object(lbm_ctx* c, int id, const float center[3], const float velocity[3], const float omega[3]) {
  if (!c) return fail(nullptr, LBM_ERR_INVALID_ARG, "ctx is NULL");
  if (id < 1 || id > 255) return fail(c, LBM_ERR_INVALID_ARG, "object ids are 1..255");
  if (!center || !velocity || !omega) return fail(c, LBM_ERR_INVALID_ARG, "NULL argument");
  for (int a = 0; a < 3; ++a)
    if (!std::isfinite(center[a]) || !std::isfinite(velocity[a]) || !std::isfinite(omega[a]))
      return fail(c, LBM_ERR_INVALID_ARG, "object motion must be finite");
  float* o = c->h_objects + 9 * id;
  for (int a = 0; a < 3; ++a) {
    o[a] = center[a];
    o[3 + a] = velocity[a];
    o[6 + a] = omega[a];
  }
  // ordered after earlier steps on the context stream
  const hipError_t e = hipMemcpyAsync(c->d_objects + 9 * id, o, 9 * sizeof(float), hipMemcpyHostToDevice, c->stream);
  if (e == hipSuccess) {
    const hipError_t e2 = hipStreamSynchronize(c->stream);
    if (e2 != hipSuccess) return hip_fail(c, e2, "set_object");
  } else {
    return hip_fail(c, e, "set_object");
  }
  return LBM_OK;
}

int lbm_prepare(lbm_ctx* c, int n) {
  if (!c) return fail(nullptr, LBM_ERR_INVALID_ARG, "ctx is NULL");
  if (n < 0) return fail(c, LBM_ERR_INVALID_ARG, "n must be >= 0");
  if (!c->list_built) {
    const int r = build_list(c);
    if (r != LBM_OK) return r;
  }
  {
    const int r = tune_rows(c);
    if (r != LBM_OK) return r;
  }
  const int G = c->opt.graph_steps;
  if (G <= 0 || c->opt.pipeline == 1) return LBM_OK;
  // lbm_step(n) replays sequences of min(n, G) steps and, past G, one of the
  // remainder (a single step is launched directly), from either buffer
  const int sizes[2] = {std::min(n, G), n > G ? n % G : 0};
  for (const int k : sizes) {
    if (k < 2) continue;
    for (int first = 0; first < 2; ++first) {
      hipGraphExec_t x = nullptr;
      const int r = graph_for(c, k, first, &x);
      if (r != LBM_OK) return r;
    }
  }
  return LBM_OK;
}

int lbm_set_triangles(lbm_ctx* c, int64_t ntris, const float* tris, const uint8_t* obj) {
  if (!c) return fail(nullptr, LBM_ERR_INVALID_ARG, "ctx is NULL");
  if (ntris < 0 || ntris > (int64_t(1) << 31) - 1 || (ntris > 0 && (!tris || !obj)))
    return fail(c, LBM_ERR_INVALID_ARG, "bad triangle list");
  for (int64_t k = 0; k < 9 * ntris; ++k)
    if (!std::isfinite(tris[k])) return fail(c, LBM_ERR_INVALID_ARG, "triangle vertices must be finite");
  hipError_t e = hipStreamSynchronize(c->stream);
  if (c->d_tris) (void)hipFree(c->d_tris);
  if (c->d_tri_obj) (void)hipFree(c->d_tri_obj);
  c->d_tris = nullptr;
  c->d_tri_obj = nullptr;
  c->n_tris = 0;
  c->winners_built = false;
  if (e == hipSuccess && ntris > 0) {
    e = hipMalloc(&c->d_tris, size_t(ntris) * 9 * sizeof(float));
    if (e == hipSuccess) e = hipMalloc(&c->d_tri_obj, size_t(ntris));
    if (e == hipSuccess) e = hipMemcpy(c->d_tris, tris, size_t(ntris) * 9 * sizeof(float), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(c->d_tri_obj, obj, size_t(ntris), hipMemcpyHostToDevice);
  }
  if (e != hipSuccess) return hip_fail(c, e, "set_triangles");
  c->n_tris = ntris;
  return LBM_OK;
}

int lbm_get_object_forces(lbm_ctx* c, double* out, int reset) {
  if (!c || !out) return fail(c, LBM_ERR_INVALID_ARG, "NULL argument");
  hipError_t e = hipMemcpyAsync(out, c->d_forces, 256 * 6 * sizeof(double), hipMemcpyDeviceToHost, c->stream);
  if (e == hipSuccess && reset) e = hipMemsetAsync(c->d_forces, 0, 256 * 6 * sizeof(double), c->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
  if (e != hipSuccess) return hip_fail(c, e, "get_object_forces");
  return LBM_OK;
}

int lbm_step_into(lbm_ctx* c, const void* in, void* out) {
  if (!c) return fail(nullptr, LBM_ERR_INVALID_ARG, "ctx is NULL");
  if (!in || !out) return fail(c, LBM_ERR_INVALID_ARG, "NULL state buffer");
  if (c->opt.pipeline == 1) return fail(c, LBM_ERR_UNSUPPORTED, "the mixed pipeline has no lbm_step_into");
  const uintptr_t a = reinterpret_cast<uintptr_t>(in), b = reinterpret_cast<uintptr_t>(out);
  const uintptr_t n = state_bytes(c);
  if (a < b + n && b < a + n) return fail(c, LBM_ERR_INVALID_ARG, "in and out overlap");
  if (!c->list_built) {
    const int r = build_list(c);
    if (r != LBM_OK) return r;
  }
  {
    const int r = tune_rows(c);
    if (r != LBM_OK) return r;
  }
  return enqueue_pass(c, in, out, nullptr);
}

int lbm_get_moments(lbm_ctx* c, float* m, int on_device) {
  if (!c || !m) return fail(c, LBM_ERR_INVALID_ARG, "NULL argument");
  float* dm = m;
  hipError_t e = hipSuccess;
  if (!on_device) e = hipMalloc(&dm, size_t(c->N) * 40);
  if (e != hipSuccess) return hip_fail(c, e, "hipMalloc(get_moments staging)");
  void* pl[10];
  planes_of(c, c->buf[c->cur], pl);
  const bool mixed = c->opt.pipeline == 1;
  if (mixed) ps_planes(c, pl);
  const void* cpl[10];
  for (int k = 0; k < 10; ++k) cpl[k] = pl[k];
  e = launch_get_moments(mixed ? int(FMT_F32) : c->fmt, cpl, dm, c->d_mask, c->N, c->stream);
  if (e == hipSuccess && !on_device) e = hipMemcpyAsync(m, dm, size_t(c->N) * 40, hipMemcpyDeviceToHost, c->stream);
  if (e == hipSuccess && !on_device) e = hipStreamSynchronize(c->stream);
  if (!on_device) (void)hipFree(dm);
  if (e != hipSuccess) return hip_fail(c, e, "get_moments");
  return LBM_OK;
}

size_t lbm_raw_bytes(const lbm_ctx* c) { return c ? state_bytes(c) : 0; }

int lbm_get_raw(lbm_ctx* c, void* out, size_t bytes, int on_device) {
  if (!c || !out) return fail(c, LBM_ERR_INVALID_ARG, "NULL argument");
  if (bytes != state_bytes(c)) return fail(c, LBM_ERR_INVALID_ARG, "bytes must equal lbm_raw_bytes()");
  hipError_t e = hipMemcpyAsync(out, c->buf[c->cur], bytes, on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost,
                                c->stream);
  if (e == hipSuccess && !on_device) e = hipStreamSynchronize(c->stream);
  if (e != hipSuccess) return hip_fail(c, e, "get_raw");
  return LBM_OK;
}

int lbm_set_raw(lbm_ctx* c, const void* in, size_t bytes, int on_device) {
  if (!c || !in) return fail(c, LBM_ERR_INVALID_ARG, "NULL argument");
  if (c->opt.pipeline == 1) return fail(c, LBM_ERR_UNSUPPORTED, "the mixed pipeline has no raw states");
  if (bytes != state_bytes(c)) return fail(c, LBM_ERR_INVALID_ARG, "bytes must equal lbm_raw_bytes()");
  hipError_t e = hipMemcpyAsync(c->buf[c->cur], in, bytes, on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice,
                                c->stream);
  if (e == hipSuccess && !c->list_built) {
    const int r = build_list(c);
    if (r != LBM_OK) return r;
  }
  if (e == hipSuccess && c->n_solid_b > 0) {
    // solid cells next to fluid hold the rest state at every step
    StepParams p = step_params(c, c->buf[c->cur], c->buf[c->cur]);
    e = launch_boundary(c->fmt, p, nullptr, nullptr, nullptr, nullptr, 0, c->d_cells + c->n_fluid_b, int(c->n_solid_b),
                        c->stream);
  }
  if (e == hipSuccess && !on_device) e = hipStreamSynchronize(c->stream);
  if (e != hipSuccess) return hip_fail(c, e, "set_raw");
  return LBM_OK;
}

int lbm_get_step_count(const lbm_ctx* c, uint64_t* t) {
  if (!c || !t) return LBM_ERR_INVALID_ARG;
  *t = c->t;
  return LBM_OK;
}

int lbm_set_step_count(lbm_ctx* c, uint64_t t) {
  if (!c) return LBM_ERR_INVALID_ARG;
  c->t = t;
  return LBM_OK;
}

int lbm_memory_bytes(const lbm_ctx* c, size_t* sb, size_t* tb) {
  if (!c) return LBM_ERR_INVALID_ARG;
  const size_t s = 2 * state_bytes(c);
  if (sb) *sb = s;
  if (tb)
    *tb = s + (c->d_ps ? size_t(c->N) * 40 : 0) + size_t(c->n_links) * 4 + (c->d_mask ? size_t(c->N) : 0) + size_t(c->n_fluid_b + c->n_solid_b) * 8 + size_t(c->n_fluid_b) * 52 +
          (c->d_lmask ? size_t((c->N + 63) / 64) * 28 : 0) + (c->d_solid ? size_t((c->N + 31) / 32) * 4 : 0) + 4 * 4 + 8;
  return LBM_OK;
}

int lbm_boundary_counts(const lbm_ctx* c, int64_t* fl, int64_t* so) {
  if (!c) return LBM_ERR_INVALID_ARG;
  if (fl) *fl = c->n_fluid_b;
  if (so) *so = c->n_solid_b;
  return LBM_OK;
}

int lbm_tile_rows(const lbm_ctx* c, int* rows) {
  if (!c || !rows) return fail(const_cast<lbm_ctx*>(c), LBM_ERR_INVALID_ARG, "NULL argument");
  *rows = fluid_rows(c);
  return LBM_OK;
}

int lbm_check(lbm_ctx* c, uint64_t* bad) {
  if (!c || !bad) return fail(c, LBM_ERR_INVALID_ARG, "NULL argument");
  const int r = scan_health(c, bad);
  if (r != LBM_OK) return r;
  return *bad ? LBM_ERR_UNSTABLE : LBM_OK;
}

int lbm_synchronize(lbm_ctx* c) {
  if (!c) return LBM_ERR_INVALID_ARG;
  const hipError_t e = hipStreamSynchronize(c->stream);
  return e == hipSuccess ? LBM_OK : hip_fail(c, e, "hipStreamSynchronize");
}

int lbm_profile_stages(lbm_ctx* c, int n, double ms[3]) {
  if (!c || n < 0 || !ms) return fail(c, LBM_ERR_INVALID_ARG, "bad argument");
  if (!c->list_built) {
    const int r = build_list(c);
    if (r != LBM_OK) return r;
  }
  const bool mixed = c->opt.pipeline == 1;
  if (n > 0) {
    const int r = tune_rows(c);
    if (r != LBM_OK) return r;
  }
  const bool has_b = mixed || (c->n_fluid_b + c->n_solid_b) > 0;
  std::vector<hipEvent_t> ev(size_t(6) * n);
  hipError_t e = hipSuccess;
  for (size_t k = 0; k < ev.size() && e == hipSuccess; ++k) e = hipEventCreate(&ev[k]);
  if (e != hipSuccess) return hip_fail(c, e, "hipEventCreate");
  int r = LBM_OK;
  for (int s = 0; s < n && r == LBM_OK; ++s)
    r = mixed ? enqueue_mixed_step(c, &ev[size_t(6) * s]) : enqueue_step(c, &ev[size_t(6) * s]);
  if (r == LBM_OK) e = hipStreamSynchronize(c->stream);
  double t[3] = {0, 0, 0};
  for (int s = 0; s < n && r == LBM_OK && e == hipSuccess; ++s) {
    for (int st = 0; st < (mixed ? 3 : (has_b ? 2 : 1)) && e == hipSuccess; ++st) {
      float m = 0;
      e = hipEventElapsedTime(&m, ev[size_t(6) * s + 2 * st], ev[size_t(6) * s + 2 * st + 1]);
      t[st] += m;
    }
  }
  for (auto& x : ev) (void)hipEventDestroy(x);
  if (r != LBM_OK) return r;
  if (e != hipSuccess) return hip_fail(c, e, "profiling events");
  for (int st = 0; st < 3; ++st) ms[st] = t[st];
  return LBM_OK;
}

int lbm_profile_steps(lbm_ctx* c, int n, double* fluid_ms, double* boundary_ms, int* nf, int* nb) {
  double ms[3] = {0, 0, 0};
  const int r = lbm_profile_stages(c, n, ms);
  if (r != LBM_OK) return r;
  const bool has_b = c->opt.pipeline == 1 || (c->n_fluid_b + c->n_solid_b) > 0;
  if (fluid_ms) *fluid_ms = ms[0];
  if (boundary_ms) *boundary_ms = ms[1] + ms[2];
  if (nf) *nf = n;
  if (nb) *nb = has_b ? n : 0;
  return LBM_OK;
}

namespace {
int adjoint_args_ok(lbm_ctx* c, const float* m_t, const float* lam_next, float* lam_prev) {
  if (!c || !m_t || !lam_next || !lam_prev) return fail(c, LBM_ERR_INVALID_ARG, "NULL argument");
  if (c->fmt != FMT_F32) return fail(c, LBM_ERR_UNSUPPORTED, "the adjoint step needs FP32 moments");
  if (c->opt.force[0] != 0.0f || c->opt.force[1] != 0.0f || c->opt.force[2] != 0.0f)
    return fail(c, LBM_ERR_UNSUPPORTED, "the adjoint step has no body-force terms");
  if (c->opt.wall_rule != 0) return fail(c, LBM_ERR_UNSUPPORTED, "the adjoint step follows bounce-back walls only");
  if (static_cast<const void*>(lam_prev) == static_cast<const void*>(lam_next) ||
      static_cast<const void*>(lam_prev) == static_cast<const void*>(m_t))
    return fail(c, LBM_ERR_INVALID_ARG, "lam_prev must not alias lam_next or m_t");
  return LBM_OK;
}

// The adjoint passes over the cell flags `flags` (1 listed fluid, 2 solid, 0 other).
int adjoint_launch(lbm_ctx* c, const uint8_t* flags, const float* m_t, const float* lam_next, float* lam_prev) {
  AdjParams p{};
  const size_t P = size_t(c->N);
  for (int k = 0; k < 10; ++k) {
    p.lam_in[k] = lam_next + k * P;
    p.m[k] = m_t + k * P;
    p.lam_out[k] = lam_prev + k * P;
  }
  p.flags = flags;
  p.g = geom(c);
  p.om1 = float(1.0 - 1.0 / c->tau);
  for (int a = 0; a < 3; ++a) p.u_in[a] = c->opt.u_in[a];
  const hipError_t e = launch_adjoint(p, c->opt.tile_rows, c->d_cells, c->d_bits, int(c->n_fluid_b), c->stream);
  if (e != hipSuccess) return hip_fail(c, e, "adjoint step");
  return LBM_OK;
}
}  // namespace

int lbm_adjoint_step(lbm_ctx* c, const float* m_t, const float* lam_next, float* lam_prev) {
  int r = adjoint_args_ok(c, m_t, lam_next, lam_prev);
  if (r != LBM_OK) return r;
  if (!c->list_built) {
    r = build_list(c);
    if (r != LBM_OK) return r;
  }
  hipError_t e = hipSuccess;
  const int count = int(c->n_fluid_b + c->n_solid_b);
  if (!c->flags_valid) {
    // cell flags: 1 listed fluid, 2 solid
    if (!c->d_flags) e = hipMalloc(&c->d_flags, size_t(c->N));
    if (e == hipSuccess) e = launch_adjoint_flags(c->d_mask, c->N, c->d_cells, c->d_bits, count, c->d_flags, c->stream);
    if (e != hipSuccess) return hip_fail(c, e, "adjoint flags");
    c->flags_valid = true;
  }
  return adjoint_launch(c, c->d_flags, m_t, lam_next, lam_prev);
}

// ------------------------------------------------ allocation-free adjoint ---
// lbm_adjoint_step_noalloc keeps the cell flags (one byte per cell) in this
// fixed device array instead of the context's lazily allocated buffer.  Each
// device holds its own copy until the process ends.  Host code never passes
// the array's name to a kernel: it uses the device address taken once per
// device with hipGetSymbolAddress (scratch_device_ptr).
constexpr size_t kAdjointScratchBytes = size_t(32) << 20;  // cells of one context at most
static __device__ __align__(256) uint8_t scratch[kAdjointScratchBytes];

namespace {
std::mutex g_scratch_mu;
void* g_scratch_dev[64] = {};  // per device: the address of `scratch`

// The current device's address of `scratch`, looked up on the first call on
// that device (lbm_create primes it).
int scratch_device_ptr(lbm_ctx* c, uint8_t** out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return hip_fail(c, e, "hipGetDevice");
  if (dev < 0 || dev >= 64) return fail(c, LBM_ERR_UNSUPPORTED, "device index above 63");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_dev[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) return hip_fail(c, e != hipSuccess ? e : hipErrorInvalidSymbol, "hipGetSymbolAddress(scratch)");
    g_scratch_dev[dev] = p;
  }
  *out = static_cast<uint8_t*>(g_scratch_dev[dev]);
  return LBM_OK;
}
}  // namespace

int lbm_adjoint_step_noalloc(lbm_ctx* c, const float* m_t, const float* lam_next, float* lam_prev) {
  int r = adjoint_args_ok(c, m_t, lam_next, lam_prev);
  if (r != LBM_OK) return r;
  if (!c->list_built)
    return fail(c, LBM_ERR_INVALID_ARG,
                "the boundary list is not built (it is rebuilt by the first lbm_step, lbm_step_into or "
                "lbm_adjoint_step after the inflow setting changes)");
  if (size_t(c->N) > kAdjointScratchBytes)
    return fail(c, LBM_ERR_INVALID_ARG,
                "lbm_adjoint_step_noalloc takes at most " + std::to_string(kAdjointScratchBytes) +
                    " cells (nx*ny*nz = " + std::to_string(c->N) + "); use lbm_adjoint_step");
  uint8_t* flags = nullptr;
  r = scratch_device_ptr(c, &flags);
  if (r != LBM_OK) return r;
  // every one of the N flags is written, so nothing of an earlier call survives
  const hipError_t e =
      launch_adjoint_flags(c->d_mask, c->N, c->d_cells, c->d_bits, int(c->n_fluid_b + c->n_solid_b), flags, c->stream);
  if (e != hipSuccess) return hip_fail(c, e, "adjoint flags");
  return adjoint_launch(c, flags, m_t, lam_next, lam_prev);
}

int lbm_equilibrium_vjp(lbm_ctx* c, const float* rho, const float* u, const float* lam, float* grad_rho,
                        float* grad_u) {
  if (!c || !rho || !u || !lam || !grad_u) return fail(c, LBM_ERR_INVALID_ARG, "NULL argument");
  const hipError_t e = launch_equilibrium_vjp(rho, u, lam, c->d_mask, c->N, grad_rho, grad_u, c->stream);
  if (e != hipSuccess) return hip_fail(c, e, "equilibrium vjp");
  return LBM_OK;
}

int lbm_fluid_plan(const int dims[3], int tile_rows, int cus, int out[7]) {
  if (!dims || !out || cus < 1) return fail(nullptr, LBM_ERR_INVALID_ARG, "bad argument");
  for (int a = 0; a < 3; ++a)
    if (dims[a] < 1) return fail(nullptr, LBM_ERR_INVALID_ARG, "every dimension must be >= 1");
  if (tile_rows != 0 &&
      std::find(std::begin(kFluidTileRows), std::end(kFluidTileRows), tile_rows) == std::end(kFluidTileRows))
    return fail(nullptr, LBM_ERR_INVALID_ARG, "tile_rows must be 0, 8, 10, 12 or 13");
  const FluidPlan p = fluid_plan(Geometry{dims[0], dims[1], dims[2], 0}, tile_rows, cus);
  out[0] = p.rows;
  out[1] = p.ntx;
  out[2] = p.nty;
  out[3] = p.nseg;
  out[4] = p.nwg;
  out[5] = p.tail;
  out[6] = p.ntail;
  return LBM_OK;
}

int lbm_debug_dither(int n, const uint32_t* idx, uint32_t t, uint32_t seed, int mode, uint32_t* h_out) {
  if (n < 0 || (n > 0 && (!idx || !h_out))) return fail(nullptr, LBM_ERR_INVALID_ARG, "bad argument");
  if (n == 0) return LBM_OK;
  uint32_t *d_idx = nullptr, *d_out = nullptr;
  hipError_t e = hipMalloc(&d_idx, size_t(n) * 4);
  if (e == hipSuccess) e = hipMalloc(&d_out, size_t(n) * 8);
  if (e == hipSuccess) e = hipMemcpy(d_idx, idx, size_t(n) * 4, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = launch_debug_dither(n, d_idx, dither_key(t, seed, mode), d_out, nullptr);
  if (e == hipSuccess) e = hipMemcpy(h_out, d_out, size_t(n) * 8, hipMemcpyDeviceToHost);
  if (d_idx) (void)hipFree(d_idx);
  if (d_out) (void)hipFree(d_out);
  if (e != hipSuccess) return hip_fail(nullptr, e, "debug_dither");
  return LBM_OK;
}

}  // extern "C"
