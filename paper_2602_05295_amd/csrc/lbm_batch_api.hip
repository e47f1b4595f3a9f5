// lbm_batch_api.hip -- the batched C ABI declared in include/homelbm.h:
// domain table, work split, boundary lists, step-sequence capture in a HIP
// graph, and the tile-shape autotuner with its JSON cache.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <map>
#include <new>
#include <sstream>
#include <string>
#include <utility>
#include <vector>

#include "../../include/homelbm.h"
#include "lbm_batch.h"
#include "lbm_device.h"
#include "lbm_internal.h"

using namespace lbm;

namespace {

// ------------------------------------------------------------ work split ---

struct HostPlan {
  std::vector<BatchDomain> doms;
  std::vector<BatchSeg> segs;
  std::vector<uint32_t> wg_first;  // nwg + 1
  double max_cost = 0, mean_cost = 0;
};

// Strip shape of an nx x ny plane in a workgroup of `block` threads.
bool strip_shape(int nx, int ny, int block, int* rows, int* ty, int* span, int* nstrips) {
  if (int64_t(nx) * ny <= block) {
    *span = 1;
    *rows = ny;
    *ty = ny;
    *nstrips = 1;
    return true;
  }
  const int rmax = block / nx;
  if (rmax < 3) return false;
  const int tymax = rmax - 2;
  *nstrips = (ny + tymax - 1) / tymax;
  *ty = (ny + *nstrips - 1) / *nstrips;
  *rows = *ty + 2;
  *span = 0;
  return true;
}

struct Column {
  int dom, strip, nz;
  double c;  // cost of one plane: the wavefronts that hold rows of the strip
};

// Deals the columns' planes to workgroups in order, no workgroup above `cap`
// (a z run of k planes costs (k + 2) c: two extra planes start it).  Returns
// the number of workgroups used; fills segs / first when given.
int deal(const std::vector<Column>& cols, double cap, std::vector<BatchSeg>* segs, std::vector<uint32_t>* first,
         std::vector<double>* loads) {
  int w = 0;
  double load = 0.0;
  if (first) first->assign(1, 0);
  if (loads) loads->clear();
  for (const Column& col : cols) {
    int z = 0;
    while (z < col.nz) {
      int k = int(std::floor((cap - load) / col.c)) - 2;
      if (k < 1) {
        if (load > 0.0) {
          if (first) first->push_back(uint32_t(segs ? segs->size() : 0));
          if (loads) loads->push_back(load);
          ++w;
          load = 0.0;
          continue;
        }
        k = 1;
      }
      const int take = std::min(k, col.nz - z);
      if (segs) segs->push_back(BatchSeg{uint16_t(col.dom), uint16_t(col.strip), uint16_t(z), uint16_t(z + take)});
      load += (take + 2) * col.c;
      z += take;
    }
  }
  if (load > 0.0) {
    if (first) first->push_back(uint32_t(segs ? segs->size() : 0));
    if (loads) loads->push_back(load);
    ++w;
  }
  return w;
}

// Returns an empty message on success.
std::string make_plan(const std::vector<int>& dims, const std::vector<double>& taus, const std::vector<uint32_t>& offs,
                      int block, int nwg, HostPlan* out) {
  const int count = int(taus.size());
  out->doms.resize(size_t(count));
  std::vector<Column> cols;
  double total = 0.0;
  for (int d = 0; d < count; ++d) {
    const int nx = dims[3 * d], ny = dims[3 * d + 1], nz = dims[3 * d + 2];
    int rows, ty, span, nstrips;
    if (!strip_shape(nx, ny, block, &rows, &ty, &span, &nstrips))
      return "domain " + std::to_string(d) + ": nx = " + std::to_string(nx) + " is too wide for " +
             std::to_string(block) + "-thread workgroups (at most " + std::to_string(block / 3) + ")";
    BatchDomain& bd = out->doms[size_t(d)];
    bd = BatchDomain{offs[size_t(d)], nx, ny, nz, rows, ty, span, float(1.0 - 1.0 / taus[size_t(d)]), 0.0f, 0.0f, 0.0f};
    code_collision_consts(1.0 - 1.0 / taus[size_t(d)], 16, bd.nq_s, bd.nq_d, bd.nq_c);
    const double c = std::ceil(double(rows) * nx / 64.0);
    for (int s = 0; s < nstrips; ++s) {
      cols.push_back(Column{d, s, nz, c});
      total += c * (nz + 2);
    }
  }
  // smallest cap that needs at most nwg workgroups
  double lo = total / nwg, hi = total + 1.0;
  for (const Column& col : cols) hi = std::max(hi, 3.0 * col.c);
  for (int it = 0; it < 60; ++it) {
    const double mid = 0.5 * (lo + hi);
    if (deal(cols, mid, nullptr, nullptr, nullptr) <= nwg)
      hi = mid;
    else
      lo = mid;
  }
  std::vector<double> loads;
  out->segs.clear();
  const int used = deal(cols, hi, &out->segs, &out->wg_first, &loads);
  if (used > nwg) return "work split failed";
  while (int(out->wg_first.size()) < nwg + 1) out->wg_first.push_back(uint32_t(out->segs.size()));
  out->max_cost = loads.empty() ? 0.0 : *std::max_element(loads.begin(), loads.end());
  double sum = 0.0;
  for (double v : loads) sum += v;
  out->mean_cost = sum / nwg;
  return std::string();
}

int device_cus() {
  int dev = 0, n = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 256;
  if (hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || n <= 0) return 256;
  return n;
}

std::string device_arch() {
  int dev = 0;
  hipDeviceProp_t prop;
  if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess) return "unknown";
  std::string a = prop.gcnArchName;
  const size_t colon = a.find(':');
  return colon == std::string::npos ? a : a.substr(0, colon);
}

thread_local std::string g_berr;

}  // namespace

struct lbm_batch {
  int count = 0;
  int fmt = 0;
  std::vector<int> dims;        // 3 per domain
  std::vector<double> taus;
  std::vector<uint32_t> offs;   // first cell of each domain
  std::vector<uint8_t> has_mask;
  int64_t N = 0;                // total cells
  lbm_options opt{};
  hipStream_t stream = nullptr;
  hipStream_t cap = nullptr;    // capture stream (created on first capture)
  void* buf[2] = {nullptr, nullptr};
  int cur = 0;
  uint8_t* d_mask = nullptr;    // concatenated masks (nullptr: no solids anywhere)
  uint32_t* d_cells = nullptr;  // boundary list: domain-local cell, flags, domain
  uint32_t* d_bits = nullptr;
  uint32_t* d_yz = nullptr;     // y | z << 16 of the fluid entries
  uint16_t* d_dom = nullptr;
  unsigned long long* d_lmask = nullptr;  // listed fluid cells: bitmap, prefix counts, side buffer
  uint32_t* d_lbase = nullptr;
  uint4* d_lpack = nullptr;               // the two packed per word for the fluid and boundary passes
  uint32_t* d_solid = nullptr;            // solid bitmap (ListedCells::solid): the fluid pass stores solid cells at rest
  float* d_side = nullptr;
  int64_t n_fluid_b = 0, n_solid_b = 0;
  uint32_t* d_counters = nullptr;
  unsigned long long* d_bad = nullptr;
  uint32_t* d_step = nullptr;   // device step counter (dither keys)
  BatchDomain* d_doms = nullptr;
  BatchSeg* d_segs = nullptr;
  uint32_t* d_wg_first = nullptr;
  lbm_batch_tuning tuning{};
  int nwg = 0;
  HostPlan plan;
  std::map<std::pair<int, int>, hipGraphExec_t> graphs;  // (steps, parity) -> replayable sequence
  std::vector<int64_t> solid_first, solid_count;           // each domain's listed solid entries
  uint64_t t = 0;
  std::string err;
};

namespace {

int bfail(lbm_batch* b, int code, const std::string& msg) {
  if (b)
    b->err = msg;
  else
    g_berr = msg;
  return code;
}

int bhip(lbm_batch* b, hipError_t e, const char* what) {
  const int code = (e == hipErrorOutOfMemory) ? LBM_ERR_OUT_OF_MEMORY : LBM_ERR_DEVICE;
  return bfail(b, code, std::string(what) + ": " + hipGetErrorString(e));
}

int nplanes(const lbm_batch* b) { return b->fmt == FMT_F32 ? 10 : 5; }
size_t plane_bytes(const lbm_batch* b) { return size_t(b->N) * 4; }
int64_t cells_of(const lbm_batch* b, int d) {
  return int64_t(b->dims[3 * d]) * b->dims[3 * d + 1] * b->dims[3 * d + 2];
}

// The planes of the whole batch (d < 0) or of domain d.
void planes(const lbm_batch* b, const void* base, int d, void* out[10]) {
  const size_t off = d < 0 ? 0 : size_t(b->offs[size_t(d)]) * 4;
  for (int k = 0; k < 10; ++k)
    out[k] = k < nplanes(b) ? static_cast<char*>(const_cast<void*>(base)) + size_t(k) * plane_bytes(b) + off : nullptr;
}

void drop_graphs(lbm_batch* b) {
  for (auto& kv : b->graphs) (void)hipGraphExecDestroy(kv.second);
  b->graphs.clear();
}

BatchStepParams params(const lbm_batch* b, int src, uint32_t k) {
  BatchStepParams p{};
  void* pin[10];
  void* pout[10];
  planes(b, b->buf[src], -1, pin);
  planes(b, b->buf[1 - src], -1, pout);
  for (int q = 0; q < 10; ++q) {
    p.in[q] = pin[q];
    p.out[q] = pout[q];
  }
  p.doms = b->d_doms;
  p.segs = b->d_segs;
  p.wg_first = b->d_wg_first;
  p.step = b->d_step;
  p.step_offset = k;
  p.seed = b->opt.seed;
  p.dither_mode = b->fmt == FMT_Q16 ? b->opt.dither_mode : 0;
  p.stream_out = stream_out_state(plane_bytes(b) * size_t(nplanes(b)));
  p.nwg = b->nwg;
  if (b->n_fluid_b > 0) p.lc = ListedCells{b->d_lpack, b->d_side, uint32_t(b->n_fluid_b)};
  p.lc.solid = b->d_solid;
  return p;
}

// Uploads the work split for `block`-thread workgroups, `wgpc` per CU.
int apply_tuning(lbm_batch* b, int block, int wgpc) {
  HostPlan hp;
  const int nwg = device_cus() * wgpc;
  const std::string msg = make_plan(b->dims, b->taus, b->offs, block, nwg, &hp);
  if (!msg.empty()) return bfail(b, LBM_ERR_UNSUPPORTED, msg);
  hipError_t e = hipStreamSynchronize(b->stream);
  if (b->d_segs) (void)hipFree(b->d_segs);
  if (b->d_wg_first) (void)hipFree(b->d_wg_first);
  b->d_segs = nullptr;
  b->d_wg_first = nullptr;
  if (e == hipSuccess) e = hipMalloc(&b->d_segs, std::max<size_t>(1, hp.segs.size()) * sizeof(BatchSeg));
  if (e == hipSuccess) e = hipMalloc(&b->d_wg_first, hp.wg_first.size() * sizeof(uint32_t));
  if (e == hipSuccess && !hp.segs.empty())
    e = hipMemcpy(b->d_segs, hp.segs.data(), hp.segs.size() * sizeof(BatchSeg), hipMemcpyHostToDevice);
  if (e == hipSuccess)
    e = hipMemcpy(b->d_wg_first, hp.wg_first.data(), hp.wg_first.size() * sizeof(uint32_t), hipMemcpyHostToDevice);
  if (e == hipSuccess)
    e = hipMemcpy(b->d_doms, hp.doms.data(), hp.doms.size() * sizeof(BatchDomain), hipMemcpyHostToDevice);
  if (e != hipSuccess) return bhip(b, e, "uploading the work split");
  drop_graphs(b);
  b->plan = std::move(hp);
  b->nwg = nwg;
  b->tuning.block = block;
  b->tuning.wg_per_cu = wgpc;
  b->tuning.workgroups = nwg;
  b->tuning.segments = int(b->plan.segs.size());
  b->tuning.balance = b->plan.max_cost > 0 ? b->plan.mean_cost / b->plan.max_cost : 1.0;
  return LBM_OK;
}

// Launches n steps (fluid + boundary each, then the counter advance) on s,
// starting from buffer `src`.  ev (optional): 4 events per step.
int enqueue_steps(lbm_batch* b, int n, int src, hipStream_t s, hipEvent_t* ev) {
  // the fluid pass stores the solid cells at rest when it has their bitmap
  const int64_t nsolid = b->d_solid ? 0 : b->n_solid_b;
  const int64_t nb = b->n_fluid_b + nsolid;
  hipError_t e = hipSuccess;
  for (int k = 0; k < n && e == hipSuccess; ++k) {
    const BatchStepParams p = params(b, (src + k) & 1, uint32_t(k));
    if (ev) e = hipEventRecord(ev[4 * k], s);
    if (e == hipSuccess) e = launch_batch_fluid(b->fmt, b->tuning.block, p, s);
    if (e == hipSuccess && ev) e = hipEventRecord(ev[4 * k + 1], s);
    if (e == hipSuccess && ev) e = hipEventRecord(ev[4 * k + 2], s);
    if (e == hipSuccess && nb > 0)
      e = launch_batch_boundary(b->fmt, p, b->d_cells, b->d_bits, b->d_yz, b->d_dom, int(b->n_fluid_b),
                                int(nsolid), s);
    if (e == hipSuccess && ev) e = hipEventRecord(ev[4 * k + 3], s);
  }
  if (e == hipSuccess && n > 0) e = launch_step_advance(b->d_step, uint32_t(n), s);
  if (e != hipSuccess) return bhip(b, e, "batched step launch");
  return LBM_OK;
}

int graph_for(lbm_batch* b, int n, hipGraphExec_t* out) {
  const auto key = std::make_pair(n, b->cur);
  auto it = b->graphs.find(key);
  if (it != b->graphs.end()) {
    *out = it->second;
    return LBM_OK;
  }
  if (b->graphs.size() >= 8) drop_graphs(b);
  hipError_t e = hipSuccess;
  if (!b->cap) e = hipStreamCreateWithFlags(&b->cap, hipStreamNonBlocking);
  if (e != hipSuccess) return bhip(b, e, "hipStreamCreate (capture)");
  e = hipStreamBeginCapture(b->cap, hipStreamCaptureModeThreadLocal);
  if (e != hipSuccess) return bhip(b, e, "hipStreamBeginCapture");
  const int r = enqueue_steps(b, n, b->cur, b->cap, nullptr);
  hipGraph_t g = nullptr;
  const hipError_t e2 = hipStreamEndCapture(b->cap, &g);
  if (r != LBM_OK) {
    if (g) (void)hipGraphDestroy(g);
    return r;
  }
  if (e2 != hipSuccess) return bhip(b, e2, "hipStreamEndCapture");
  hipGraphExec_t x = nullptr;
  e = hipGraphInstantiate(&x, g, nullptr, nullptr, 0);
  (void)hipGraphDestroy(g);
  if (e != hipSuccess) return bhip(b, e, "hipGraphInstantiate");
  b->graphs[key] = x;
  *out = x;
  return LBM_OK;
}

// Boundary lists of all domains: per-domain count passes (counts and the
// global bitmap of listed fluid cells), prefix counts on the host, one list
// (fluid entries in global cell order, then solid entries) and the side
// buffer the fluid pass fills for the listed fluid cells.
int build_lists(lbm_batch* b) {
  std::vector<uint32_t> nf(size_t(b->count), 0), ns(size_t(b->count), 0);
  bool any = false;
  for (int d = 0; d < b->count; ++d) any = any || b->has_mask[size_t(d)];
  b->n_fluid_b = 0;
  b->n_solid_b = 0;
  if (!any) return LBM_OK;
  const size_t nchunks = size_t((b->N + 63) / 64);
  hipError_t e = hipMalloc(&b->d_lmask, nchunks * 8);
  if (e == hipSuccess) e = hipMalloc(&b->d_lbase, nchunks * 4);
  if (e == hipSuccess) e = hipMemsetAsync(b->d_lmask, 0, nchunks * 8, b->stream);
  for (int d = 0; d < b->count && e == hipSuccess; ++d) {
    if (!b->has_mask[size_t(d)]) continue;
    const Geometry g{b->dims[3 * d], b->dims[3 * d + 1], b->dims[3 * d + 2], 0};
    uint32_t cnt[4] = {0, 0, 0, 0};
    e = hipMemsetAsync(b->d_counters, 0, 4 * sizeof(uint32_t), b->stream);
    if (e == hipSuccess)
      e = launch_classify(b->d_mask + b->offs[size_t(d)], g, b->offs[size_t(d)], b->d_counters, b->d_lmask, nullptr,
                          nullptr, nullptr, nullptr, nullptr, nullptr, 0, b->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(cnt, b->d_counters, sizeof(cnt), hipMemcpyDeviceToHost, b->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(b->stream);
    nf[size_t(d)] = cnt[0];
    ns[size_t(d)] = cnt[1];
  }
  if (e != hipSuccess) return bhip(b, e, "boundary list (count)");
  int64_t nf_all = 0, total = 0;
  for (int d = 0; d < b->count; ++d) {
    nf_all += nf[size_t(d)];
    total += int64_t(nf[size_t(d)]) + ns[size_t(d)];
  }
  if (total > int64_t(INT32_MAX)) return bfail(b, LBM_ERR_UNSUPPORTED, "boundary list too long");
  if (total == 0) return LBM_OK;
  std::vector<unsigned long long> hmask(nchunks);
  e = hipMemcpy(hmask.data(), b->d_lmask, nchunks * 8, hipMemcpyDeviceToHost);
  if (e != hipSuccess) return bhip(b, e, "reading the list bitmap");
  std::vector<uint32_t> hbase(nchunks);
  uint32_t run = 0;
  for (size_t k = 0; k < nchunks; ++k) {
    hbase[k] = run;
    run += uint32_t(__builtin_popcountll(hmask[k]));
  }
  if (int64_t(run) != nf_all) return bfail(b, LBM_ERR_DEVICE, "boundary list: bitmap and counts disagree");
  std::vector<uint4> hpack(nchunks + 1, make_uint4(0u, 0u, 0u, 0u));  // one padding entry
  for (size_t k = 0; k < nchunks; ++k)
    hpack[k] = make_uint4(uint32_t(hmask[k]), uint32_t(hmask[k] >> 32), hbase[k], 0u);
  e = hipMemcpy(b->d_lbase, hbase.data(), nchunks * 4, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMalloc(&b->d_lpack, (nchunks + 1) * sizeof(uint4));
  if (e == hipSuccess) e = hipMemcpy(b->d_lpack, hpack.data(), (nchunks + 1) * sizeof(uint4), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMalloc(&b->d_cells, size_t(total) * 4);
  if (e == hipSuccess) e = hipMalloc(&b->d_bits, size_t(total) * 4);
  if (e == hipSuccess) e = hipMalloc(&b->d_yz, size_t(std::max<int64_t>(nf_all, 1)) * 4);
  if (e == hipSuccess) e = hipMalloc(&b->d_side, size_t(std::max<int64_t>(nf_all, 1)) * 48);
  if (e == hipSuccess) e = hipMalloc(&b->d_dom, size_t(total) * 2);
  if (e != hipSuccess) return bhip(b, e, "hipMalloc(boundary list)");
  // fluid entries in global cell order (so each domain's are contiguous), then solid entries
  std::vector<uint16_t> hdom(static_cast<size_t>(total));
  int64_t fbase = 0, sbase = nf_all;
  for (int d = 0; d < b->count && e == hipSuccess; ++d) {
    if (nf[size_t(d)] + ns[size_t(d)] == 0) continue;
    const Geometry g{b->dims[3 * d], b->dims[3 * d + 1], b->dims[3 * d + 2], 0};
    e = hipMemsetAsync(b->d_counters, 0, 4 * sizeof(uint32_t), b->stream);
    if (e == hipSuccess)
      e = launch_classify(b->d_mask + b->offs[size_t(d)], g, b->offs[size_t(d)], b->d_counters, b->d_lmask, b->d_lbase,
                          b->d_cells, b->d_bits, b->d_yz, b->d_cells + sbase, b->d_bits + sbase, ns[size_t(d)],
                          b->stream);
    std::fill(hdom.begin() + fbase, hdom.begin() + fbase + nf[size_t(d)], uint16_t(d));
    std::fill(hdom.begin() + sbase, hdom.begin() + sbase + ns[size_t(d)], uint16_t(d));
    fbase += nf[size_t(d)];
    sbase += ns[size_t(d)];
  }
  if (e == hipSuccess) e = hipMemcpyAsync(b->d_dom, hdom.data(), hdom.size() * 2, hipMemcpyHostToDevice, b->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(b->stream);
  if (e != hipSuccess) return bhip(b, e, "boundary list (fill)");
  b->solid_first.assign(size_t(b->count), 0);
  b->solid_count.assign(size_t(b->count), 0);
  int64_t sb = nf_all;
  for (int d = 0; d < b->count; ++d) {
    b->solid_first[size_t(d)] = sb;
    b->solid_count[size_t(d)] = ns[size_t(d)];
    sb += ns[size_t(d)];
  }
  b->n_fluid_b = nf_all;
  b->n_solid_b = total - nf_all;
  e = hipMalloc(&b->d_solid, size_t((b->N + 31) / 32) * 4);
  if (e == hipSuccess) e = launch_solid_bits(b->d_mask, uint32_t(b->N), b->d_solid, b->stream);
  if (e != hipSuccess) return bhip(b, e, "solid bitmap");
  return LBM_OK;
}

int check_domain(lbm_batch* b, int d) {
  if (!b) return bfail(nullptr, LBM_ERR_INVALID_ARG, "batch is NULL");
  if (d < 0 || d >= b->count) return bfail(b, LBM_ERR_INVALID_ARG, "domain index out of range");
  return LBM_OK;
}

int stage(lbm_batch* b, const void* src, size_t bytes, int on_device, void** dev, bool* owned) {
  *owned = false;
  if (on_device) {
    *dev = const_cast<void*>(src);
    return LBM_OK;
  }
  hipError_t e = hipMalloc(dev, bytes);
  if (e == hipSuccess) e = hipMemcpyAsync(*dev, src, bytes, hipMemcpyHostToDevice, b->stream);
  if (e != hipSuccess) return bhip(b, e, "staging host input");
  *owned = true;
  return LBM_OK;
}

// ------------------------------------------------------- autotune cache ---

std::string tune_key(const lbm_batch* b) {
  // FNV-1a over the format and the domain shapes
  uint64_t h = 1469598103934665603ull;
  auto mix = [&h](uint64_t v) {
    for (int i = 0; i < 8; ++i) {
      h ^= (v >> (8 * i)) & 0xFFu;
      h *= 1099511628211ull;
    }
  };
  mix(uint64_t(b->fmt));
  mix(uint64_t(b->count));
  for (int v : b->dims) mix(uint64_t(v));
  char hex[17];
  std::snprintf(hex, sizeof(hex), "%016llx", static_cast<unsigned long long>(h));
  return device_arch() + "/" + std::to_string(device_cus()) + "cu/" + (b->fmt == FMT_F32 ? "fp32" : "q16") + "/" + hex;
}

// Cache file: a JSON object, one entry per line:
//   "<key>": {"block": B, "wg_per_cu": W, "fluid_ms": T},
bool cache_lookup(const char* path, const std::string& key, int* block, int* wgpc, double* ms) {
  std::ifstream in(path);
  if (!in) return false;
  std::string line;
  const std::string pat = "\"" + key + "\":";
  while (std::getline(in, line)) {
    const size_t at = line.find(pat);
    if (at == std::string::npos) continue;
    const char* s = line.c_str() + at + pat.size();
    int bl = 0, w = 0;
    double t = 0;
    if (std::sscanf(s, " {\"block\": %d, \"wg_per_cu\": %d, \"fluid_ms\": %lf", &bl, &w, &t) >= 2) {
      *block = bl;
      *wgpc = w;
      *ms = t;
      return true;
    }
  }
  return false;
}

bool cache_store(const char* path, const std::string& key, int block, int wgpc, double ms) {
  std::vector<std::string> entries;
  {
    std::ifstream in(path);
    std::string line;
    while (in && std::getline(in, line)) {
      const size_t q = line.find('"');
      if (q == std::string::npos || line.find("\": {") == std::string::npos) continue;
      if (line.find("\"" + key + "\":") != std::string::npos) continue;
      while (!line.empty() && (line.back() == ',' || line.back() == ' ')) line.pop_back();
      entries.push_back(line.substr(q));
    }
  }
  char buf[256];
  std::snprintf(buf, sizeof(buf), "\"%s\": {\"block\": %d, \"wg_per_cu\": %d, \"fluid_ms\": %.6f}", key.c_str(), block,
                wgpc, ms);
  entries.push_back(buf);
  const std::string tmp = std::string(path) + ".tmp" + std::to_string(reinterpret_cast<uintptr_t>(&entries));
  {
    std::ofstream out(tmp);
    if (!out) return false;
    out << "{\n";
    for (size_t i = 0; i < entries.size(); ++i) out << "  " << entries[i] << (i + 1 < entries.size() ? ",\n" : "\n");
    out << "}\n";
    if (!out) return false;
  }
  return std::rename(tmp.c_str(), path) == 0;
}

// Mean fluid-pass time of the current split (reads the state, writes the
// other buffer; no state change).
int time_fluid(lbm_batch* b, int reps, double* ms) {
  hipEvent_t e0, e1;
  hipError_t e = hipEventCreate(&e0);
  if (e == hipSuccess) e = hipEventCreate(&e1);
  if (e != hipSuccess) return bhip(b, e, "hipEventCreate");
  const BatchStepParams p = params(b, b->cur, 0);
  for (int k = 0; k < 2 && e == hipSuccess; ++k) e = launch_batch_fluid(b->fmt, b->tuning.block, p, b->stream);
  if (e == hipSuccess) e = hipEventRecord(e0, b->stream);
  for (int k = 0; k < reps && e == hipSuccess; ++k) e = launch_batch_fluid(b->fmt, b->tuning.block, p, b->stream);
  if (e == hipSuccess) e = hipEventRecord(e1, b->stream);
  if (e == hipSuccess) e = hipEventSynchronize(e1);
  float t = 0;
  if (e == hipSuccess) e = hipEventElapsedTime(&t, e0, e1);
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (e != hipSuccess) return bhip(b, e, "timing the fluid pass");
  *ms = double(t) / reps;
  return LBM_OK;
}

}  // namespace

extern "C" {

const char* lbm_batch_last_error(const lbm_batch* b) { return b ? b->err.c_str() : g_berr.c_str(); }

int lbm_batch_create(int count, const int* dims, const double* taus, const uint8_t* const* masks, int fmt,
                     lbm_batch** out) {
  if (!out) return bfail(nullptr, LBM_ERR_INVALID_ARG, "out is NULL");
  *out = nullptr;
  if (count < 1 || count > 65535) return bfail(nullptr, LBM_ERR_INVALID_ARG, "count must be in 1..65535");
  if (!dims || !taus) return bfail(nullptr, LBM_ERR_INVALID_ARG, "dims or taus is NULL");
  if (fmt >= LBM_MOMENTS_P16_15 && fmt <= LBM_MOMENTS_P12_11)
    return bfail(nullptr, LBM_ERR_UNSUPPORTED, "batches store FP32 or 16-bit moments");
  if (fmt != LBM_MOMENTS_FP32 && fmt != LBM_MOMENTS_Q16)
    return bfail(nullptr, LBM_ERR_INVALID_ARG, "unknown moment format");
  int64_t total = 0;
  for (int d = 0; d < count; ++d) {
    for (int a = 0; a < 3; ++a)
      if (dims[3 * d + a] < 1 || dims[3 * d + a] > 65535)
        return bfail(nullptr, LBM_ERR_INVALID_ARG, "domain " + std::to_string(d) + ": dimensions must be in 1..65535");
    if (dims[3 * d] > 1024 / 3 && int64_t(dims[3 * d]) * dims[3 * d + 1] > 1024)
      return bfail(nullptr, LBM_ERR_INVALID_ARG,
                   "domain " + std::to_string(d) + ": nx must be <= 341 (or nx*ny <= 1024) in a batch");
    if (!(taus[d] > 0.5) || !std::isfinite(taus[d]))
      return bfail(nullptr, LBM_ERR_INVALID_ARG, "domain " + std::to_string(d) + ": tau must be > 1/2");
    total += int64_t(dims[3 * d]) * dims[3 * d + 1] * dims[3 * d + 2];
    if (total > (int64_t(1) << 30)) return bfail(nullptr, LBM_ERR_INVALID_ARG, "total cells must be <= 2^30");
  }
  lbm_batch* b = new (std::nothrow) lbm_batch();
  if (!b) return bfail(nullptr, LBM_ERR_OUT_OF_MEMORY, "host allocation failed");
  b->count = count;
  b->fmt = fmt;
  b->dims.assign(dims, dims + 3 * count);
  b->taus.assign(taus, taus + count);
  b->N = total;
  b->offs.resize(size_t(count));
  b->has_mask.assign(size_t(count), 0);
  int64_t off = 0;
  bool any = false;
  for (int d = 0; d < count; ++d) {
    b->offs[size_t(d)] = uint32_t(off);
    const int64_t n = cells_of(b, d);
    if (masks && masks[d]) {
      for (int64_t k = 0; k < n; ++k) {
        if (masks[d][k] > 1) {
          delete b;
          return bfail(nullptr, LBM_ERR_INVALID_ARG, "domain " + std::to_string(d) + ": mask values must be 0 or 1");
        }
        if (masks[d][k]) b->has_mask[size_t(d)] = 1;
      }
    }
    any = any || b->has_mask[size_t(d)];
    off += n;
  }
  lbm_default_options(&b->opt);
  hipError_t e = hipSuccess;
  for (int k = 0; k < 2 && e == hipSuccess; ++k) e = hipMalloc(&b->buf[k], plane_bytes(b) * size_t(nplanes(b)));
  if (e == hipSuccess) e = hipMalloc(&b->d_counters, 4 * sizeof(uint32_t));
  if (e == hipSuccess) e = hipMalloc(&b->d_bad, sizeof(unsigned long long));
  if (e == hipSuccess) e = hipMalloc(&b->d_step, sizeof(uint32_t));
  if (e == hipSuccess) e = hipMemset(b->d_step, 0, sizeof(uint32_t));
  if (e == hipSuccess) e = hipMalloc(&b->d_doms, size_t(count) * sizeof(BatchDomain));
  if (e == hipSuccess && any) {
    e = hipMalloc(&b->d_mask, size_t(total));
    for (int d = 0; d < count && e == hipSuccess; ++d) {
      const size_t n = size_t(cells_of(b, d));
      if (b->has_mask[size_t(d)])
        e = hipMemcpy(b->d_mask + b->offs[size_t(d)], masks[d], n, hipMemcpyHostToDevice);
      else
        e = hipMemset(b->d_mask + b->offs[size_t(d)], 0, n);
    }
  }
  if (e != hipSuccess) {
    const int code = bhip(nullptr, e, "lbm_batch_create allocation");
    lbm_batch_destroy(b);
    return code;
  }
  void* pl[10];
  planes(b, b->buf[0], -1, pl);
  e = launch_set_rest(fmt, pl, b->N, b->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(b->stream);
  if (e != hipSuccess) {
    const int code = bhip(nullptr, e, "lbm_batch_create initial state");
    lbm_batch_destroy(b);
    return code;
  }
  int r = build_lists(b);
  // default split: the largest workgroup that every domain fits, one per CU
  if (r == LBM_OK) r = apply_tuning(b, 1024, 1);
  if (r != LBM_OK) {
    g_berr = b->err;
    lbm_batch_destroy(b);
    return r;
  }
  *out = b;
  return LBM_OK;
}

int lbm_batch_destroy(lbm_batch* b) {
  if (!b) return LBM_OK;
  (void)hipStreamSynchronize(b->stream);
  drop_graphs(b);
  if (b->cap) (void)hipStreamDestroy(b->cap);
  for (int k = 0; k < 2; ++k)
    if (b->buf[k]) (void)hipFree(b->buf[k]);
  void* ptrs[] = {b->d_mask,  b->d_cells, b->d_bits, b->d_yz,       b->d_dom,  b->d_lmask, b->d_lbase, b->d_lpack,
                  b->d_side,  b->d_solid, b->d_counters, b->d_bad, b->d_step, b->d_doms, b->d_segs, b->d_wg_first};
  for (void* p : ptrs)
    if (p) (void)hipFree(p);
  delete b;
  return LBM_OK;
}

int lbm_batch_set_stream(lbm_batch* b, void* s) {
  if (!b) return bfail(nullptr, LBM_ERR_INVALID_ARG, "batch is NULL");
  b->stream = static_cast<hipStream_t>(s);
  return LBM_OK;
}

int lbm_batch_set_options(lbm_batch* b, const lbm_options* o) {
  if (!b || !o) return bfail(b, LBM_ERR_INVALID_ARG, "NULL argument");
  if (o->dither_mode < 0 || o->dither_mode > 2) return bfail(b, LBM_ERR_INVALID_ARG, "unknown dither mode");
  if (o->inflow) return bfail(b, LBM_ERR_UNSUPPORTED, "batched domains are periodic (inflow must be 0)");
  if (o->force[0] != 0.0f || o->force[1] != 0.0f || o->force[2] != 0.0f)
    return bfail(b, LBM_ERR_UNSUPPORTED, "batched domains have no body force (force must be 0)");
  if (o->wall_rule != 0 || o->track_forces != 0)
    return bfail(b, LBM_ERR_UNSUPPORTED, "batched domains use bounce-back walls without force tracking");
  if (o->tile_rows != 0) return bfail(b, LBM_ERR_INVALID_ARG, "tile_rows must be 0 in a batch (see lbm_batch_set_tuning)");
  b->opt = *o;
  drop_graphs(b);
  return LBM_OK;
}

int lbm_batch_get_options(const lbm_batch* b, lbm_options* o) {
  if (!b || !o) return LBM_ERR_INVALID_ARG;
  *o = b->opt;
  return LBM_OK;
}

int lbm_batch_info(const lbm_batch* b, int d, int dims[3], int64_t* offset, int64_t* cells) {
  if (!b || d < 0 || d >= b->count) return LBM_ERR_INVALID_ARG;
  if (dims)
    for (int a = 0; a < 3; ++a) dims[a] = b->dims[3 * d + a];
  if (offset) *offset = b->offs[size_t(d)];
  if (cells) *cells = cells_of(b, d);
  return LBM_OK;
}

int lbm_batch_total_cells(const lbm_batch* b, int64_t* cells) {
  if (!b || !cells) return LBM_ERR_INVALID_ARG;
  *cells = b->N;
  return LBM_OK;
}

int lbm_batch_set_moments(lbm_batch* b, int d, const float* m, int on_device) {
  int r = check_domain(b, d);
  if (r != LBM_OK) return r;
  if (!m) return bfail(b, LBM_ERR_INVALID_ARG, "NULL argument");
  const int64_t n = cells_of(b, d);
  void* dm;
  bool owned;
  r = stage(b, m, size_t(n) * 40, on_device, &dm, &owned);
  if (r != LBM_OK) return r;
  void* pl[10];
  planes(b, b->buf[b->cur], d, pl);
  hipError_t e = launch_set_moments(b->fmt, static_cast<const float*>(dm), pl,
                                    b->has_mask[size_t(d)] ? b->d_mask + b->offs[size_t(d)] : nullptr, n, b->stream);
  if (e == hipSuccess && owned) e = hipStreamSynchronize(b->stream);
  if (owned) (void)hipFree(dm);
  if (e != hipSuccess) return bhip(b, e, "set_moments");
  return LBM_OK;
}

int lbm_batch_set_equilibrium(lbm_batch* b, int d, const float* rho, const float* u, int on_device) {
  int r = check_domain(b, d);
  if (r != LBM_OK) return r;
  if (!rho || !u) return bfail(b, LBM_ERR_INVALID_ARG, "NULL argument");
  const int64_t n = cells_of(b, d);
  void *dr, *du;
  bool o1, o2;
  r = stage(b, rho, size_t(n) * 4, on_device, &dr, &o1);
  if (r != LBM_OK) return r;
  r = stage(b, u, size_t(n) * 12, on_device, &du, &o2);
  if (r != LBM_OK) {
    if (o1) (void)hipFree(dr);
    return r;
  }
  void* pl[10];
  planes(b, b->buf[b->cur], d, pl);
  hipError_t e = launch_set_equilibrium(b->fmt, static_cast<const float*>(dr), static_cast<const float*>(du), pl,
                                        b->has_mask[size_t(d)] ? b->d_mask + b->offs[size_t(d)] : nullptr, n,
                                        b->stream);
  if (e == hipSuccess && (o1 || o2)) e = hipStreamSynchronize(b->stream);
  if (o1) (void)hipFree(dr);
  if (o2) (void)hipFree(du);
  if (e != hipSuccess) return bhip(b, e, "set_equilibrium");
  return LBM_OK;
}

int lbm_batch_get_moments(lbm_batch* b, int d, float* m, int on_device) {
  int r = check_domain(b, d);
  if (r != LBM_OK) return r;
  if (!m) return bfail(b, LBM_ERR_INVALID_ARG, "NULL argument");
  const int64_t n = cells_of(b, d);
  float* dm = m;
  hipError_t e = hipSuccess;
  if (!on_device) e = hipMalloc(&dm, size_t(n) * 40);
  if (e != hipSuccess) return bhip(b, e, "hipMalloc(get_moments staging)");
  void* pl[10];
  planes(b, b->buf[b->cur], d, pl);
  const void* cpl[10];
  for (int k = 0; k < 10; ++k) cpl[k] = pl[k];
  e = launch_get_moments(b->fmt, cpl, dm, b->has_mask[size_t(d)] ? b->d_mask + b->offs[size_t(d)] : nullptr, n,
                         b->stream);
  if (e == hipSuccess && !on_device) e = hipMemcpyAsync(m, dm, size_t(n) * 40, hipMemcpyDeviceToHost, b->stream);
  if (e == hipSuccess && !on_device) e = hipStreamSynchronize(b->stream);
  if (!on_device) (void)hipFree(dm);
  if (e != hipSuccess) return bhip(b, e, "get_moments");
  return LBM_OK;
}

size_t lbm_batch_raw_bytes(const lbm_batch* b, int d) {
  if (!b || d < 0 || d >= b->count) return 0;
  return size_t(cells_of(b, d)) * 4 * size_t(nplanes(b));
}

static int raw_copy(lbm_batch* b, int d, void* host_or_dev, size_t bytes, int on_device, bool to_state) {
  int r = check_domain(b, d);
  if (r != LBM_OK) return r;
  if (!host_or_dev) return bfail(b, LBM_ERR_INVALID_ARG, "NULL argument");
  if (bytes != lbm_batch_raw_bytes(b, d)) return bfail(b, LBM_ERR_INVALID_ARG, "bytes must equal lbm_batch_raw_bytes()");
  const size_t pb = size_t(cells_of(b, d)) * 4;
  void* pl[10];
  planes(b, b->buf[b->cur], d, pl);
  hipError_t e = hipSuccess;
  for (int k = 0; k < nplanes(b) && e == hipSuccess; ++k) {
    char* user = static_cast<char*>(host_or_dev) + size_t(k) * pb;
    if (to_state)
      e = hipMemcpyAsync(pl[k], user, pb, on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice, b->stream);
    else
      e = hipMemcpyAsync(user, pl[k], pb, on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost, b->stream);
  }
  if (e == hipSuccess && !on_device) e = hipStreamSynchronize(b->stream);
  if (e != hipSuccess) return bhip(b, e, to_state ? "set_raw" : "get_raw");
  return LBM_OK;
}

int lbm_batch_get_raw(lbm_batch* b, int d, void* out, size_t bytes, int on_device) {
  return raw_copy(b, d, out, bytes, on_device, false);
}

int lbm_batch_set_raw(lbm_batch* b, int d, const void* in, size_t bytes, int on_device) {
  const int r = raw_copy(b, d, const_cast<void*>(in), bytes, on_device, true);
  if (r != LBM_OK) return r;
  if (size_t(d) < b->solid_count.size() && b->solid_count[size_t(d)] > 0) {
    // solid cells next to fluid hold the rest state at every step
    BatchStepParams p = params(b, b->cur, 0);
    for (int k = 0; k < 10; ++k) p.out[k] = const_cast<void*>(p.in[k]);
    const int64_t f = b->solid_first[size_t(d)];
    const hipError_t e = launch_batch_boundary(b->fmt, p, b->d_cells + f, nullptr, nullptr, b->d_dom + f, 0,
                                               int(b->solid_count[size_t(d)]), b->stream);
    if (e != hipSuccess) return bhip(b, e, "set_raw (solid cells)");
  }
  return LBM_OK;
}

int lbm_batch_step(lbm_batch* b, int n) {
  if (!b) return bfail(nullptr, LBM_ERR_INVALID_ARG, "batch is NULL");
  if (n < 0) return bfail(b, LBM_ERR_INVALID_ARG, "n must be >= 0");
  const int chunk = 256;  // steps per captured sequence
  int left = n;
  while (left > 0) {
    const int k = std::min(left, chunk);
    hipGraphExec_t x;
    int r = graph_for(b, k, &x);
    if (r != LBM_OK) return r;
    const hipError_t e = hipGraphLaunch(x, b->stream);
    if (e != hipSuccess) return bhip(b, e, "hipGraphLaunch");
    b->cur = (b->cur + k) & 1;
    b->t += uint64_t(k);
    left -= k;
  }
  if (b->opt.check_health && n > 0) {
    uint64_t bad = 0;
    const int r = lbm_batch_check(b, &bad);
    if (r != LBM_OK) return r;
  }
  return LBM_OK;
}

int lbm_batch_step_eager(lbm_batch* b, int n) {
  if (!b) return bfail(nullptr, LBM_ERR_INVALID_ARG, "batch is NULL");
  if (n < 0) return bfail(b, LBM_ERR_INVALID_ARG, "n must be >= 0");
  const int r = enqueue_steps(b, n, b->cur, b->stream, nullptr);
  if (r != LBM_OK) return r;
  b->cur = (b->cur + n) & 1;
  b->t += uint64_t(n);
  return LBM_OK;
}

int lbm_batch_profile_steps(lbm_batch* b, int n, double* fluid_ms, double* boundary_ms) {
  if (!b || n < 0) return bfail(b, LBM_ERR_INVALID_ARG, "bad argument");
  std::vector<hipEvent_t> ev(size_t(4) * n);
  hipError_t e = hipSuccess;
  for (size_t k = 0; k < ev.size() && e == hipSuccess; ++k) e = hipEventCreate(&ev[k]);
  if (e != hipSuccess) return bhip(b, e, "hipEventCreate");
  int r = enqueue_steps(b, n, b->cur, b->stream, ev.data());
  if (r == LBM_OK) e = hipStreamSynchronize(b->stream);
  double tf = 0, tb = 0;
  for (int s = 0; s < n && r == LBM_OK && e == hipSuccess; ++s) {
    float ms = 0;
    e = hipEventElapsedTime(&ms, ev[size_t(4) * s], ev[size_t(4) * s + 1]);
    tf += ms;
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, ev[size_t(4) * s + 2], ev[size_t(4) * s + 3]);
    tb += ms;
  }
  for (auto& x : ev) (void)hipEventDestroy(x);
  if (r != LBM_OK) return r;
  if (e != hipSuccess) return bhip(b, e, "profiling events");
  b->cur = (b->cur + n) & 1;
  b->t += uint64_t(n);
  if (fluid_ms) *fluid_ms = tf;
  if (boundary_ms) *boundary_ms = tb;
  return LBM_OK;
}

int lbm_batch_get_step_count(const lbm_batch* b, uint64_t* t) {
  if (!b || !t) return LBM_ERR_INVALID_ARG;
  *t = b->t;
  return LBM_OK;
}

int lbm_batch_set_step_count(lbm_batch* b, uint64_t t) {
  if (!b) return LBM_ERR_INVALID_ARG;
  const uint32_t v = uint32_t(t);
  hipError_t e = hipMemcpyAsync(b->d_step, &v, sizeof(v), hipMemcpyHostToDevice, b->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(b->stream);
  if (e != hipSuccess) return bhip(b, e, "set_step_count");
  b->t = t;
  return LBM_OK;
}

int lbm_batch_boundary_counts(const lbm_batch* b, int64_t* fl, int64_t* so) {
  if (!b) return LBM_ERR_INVALID_ARG;
  if (fl) *fl = b->n_fluid_b;
  if (so) *so = b->n_solid_b;
  return LBM_OK;
}

int lbm_batch_memory_bytes(const lbm_batch* b, size_t* state_bytes, size_t* total_bytes) {
  if (!b) return LBM_ERR_INVALID_ARG;
  const size_t s = 2 * plane_bytes(b) * size_t(nplanes(b));
  if (state_bytes) *state_bytes = s;
  if (total_bytes)
    *total_bytes = s + (b->d_mask ? size_t(b->N) : 0) + size_t(b->n_fluid_b + b->n_solid_b) * 10 +
                   size_t(b->n_fluid_b) * 52 + (b->d_lmask ? size_t((b->N + 63) / 64) * 28 : 0) +
                   (b->d_solid ? size_t((b->N + 31) / 32) * 4 : 0) +
                   b->plan.segs.size() * sizeof(BatchSeg) + b->plan.wg_first.size() * 4 +
                   size_t(b->count) * sizeof(BatchDomain) + 32;
  return LBM_OK;
}

int lbm_batch_check(lbm_batch* b, uint64_t* bad) {
  if (!b || !bad) return bfail(b, LBM_ERR_INVALID_ARG, "NULL argument");
  void* pl[10];
  planes(b, b->buf[b->cur], -1, pl);
  const void* cpl[10];
  for (int k = 0; k < 10; ++k) cpl[k] = pl[k];
  hipError_t e = hipMemsetAsync(b->d_bad, 0, sizeof(unsigned long long), b->stream);
  if (e == hipSuccess) e = launch_health(b->fmt, cpl, b->N, b->d_bad, b->stream);
  unsigned long long h = 0;
  if (e == hipSuccess) e = hipMemcpyAsync(&h, b->d_bad, sizeof(h), hipMemcpyDeviceToHost, b->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(b->stream);
  if (e != hipSuccess) return bhip(b, e, "health scan");
  *bad = h;
  if (h) return bfail(b, LBM_ERR_UNSTABLE, "state holds " + std::to_string(h) + " non-finite or saturated values");
  return LBM_OK;
}

int lbm_batch_synchronize(lbm_batch* b) {
  if (!b) return LBM_ERR_INVALID_ARG;
  const hipError_t e = hipStreamSynchronize(b->stream);
  return e == hipSuccess ? LBM_OK : bhip(b, e, "hipStreamSynchronize");
}

int lbm_batch_get_tuning(const lbm_batch* b, lbm_batch_tuning* t) {
  if (!b || !t) return LBM_ERR_INVALID_ARG;
  *t = b->tuning;
  return LBM_OK;
}

int lbm_batch_set_tuning(lbm_batch* b, int block, int wg_per_cu) {
  if (!b) return bfail(nullptr, LBM_ERR_INVALID_ARG, "batch is NULL");
  if (std::find(std::begin(kBatchBlocks), std::end(kBatchBlocks), block) == std::end(kBatchBlocks))
    return bfail(b, LBM_ERR_INVALID_ARG, "block must be 256, 512 or 1024");
  const int occ = batch_fluid_occupancy(b->fmt, block);
  if (wg_per_cu < 1 || wg_per_cu > std::max(1, occ))
    return bfail(b, LBM_ERR_INVALID_ARG, "wg_per_cu must be in 1.." + std::to_string(std::max(1, occ)));
  const int r = apply_tuning(b, block, wg_per_cu);
  if (r == LBM_OK) b->tuning.from_cache = 0;
  return r;
}

int lbm_batch_tune(lbm_batch* b, const char* cache_path, lbm_batch_tuning* result) {
  if (!b) return bfail(nullptr, LBM_ERR_INVALID_ARG, "batch is NULL");
  const char* path = cache_path ? cache_path : std::getenv("LBM_AUTOTUNE_CACHE");
  if (path && !*path) path = nullptr;
  const std::string key = tune_key(b);
  int bl = 0, w = 0;
  double ms = 0;
  if (path && cache_lookup(path, key, &bl, &w, &ms) &&
      std::find(std::begin(kBatchBlocks), std::end(kBatchBlocks), bl) != std::end(kBatchBlocks) && w >= 1 &&
      w <= std::max(1, batch_fluid_occupancy(b->fmt, bl))) {
    const int r = apply_tuning(b, bl, w);
    if (r != LBM_OK) return r;
    b->tuning.fluid_ms = ms;
    b->tuning.from_cache = 1;
    if (result) *result = b->tuning;
    return LBM_OK;
  }
  double best = 0;
  int best_bl = 0, best_w = 0;
  for (int block : kBatchBlocks) {
    const int occ = batch_fluid_occupancy(b->fmt, block);
    for (int wgpc = 1; wgpc <= occ && wgpc <= 4; wgpc *= 2) {
      if (apply_tuning(b, block, wgpc) != LBM_OK) continue;  // a domain too wide for this block
      double t = 0;
      const int r = time_fluid(b, 5, &t);
      if (r != LBM_OK) return r;
      if (best_bl == 0 || t < best) {
        best = t;
        best_bl = block;
        best_w = wgpc;
      }
    }
  }
  if (best_bl == 0) return bfail(b, LBM_ERR_UNSUPPORTED, "no workgroup shape fits every domain");
  const int r = apply_tuning(b, best_bl, best_w);
  if (r != LBM_OK) return r;
  b->tuning.fluid_ms = best;
  b->tuning.from_cache = 0;
  if (path) cache_store(path, key, best_bl, best_w, best);
  if (result) *result = b->tuning;
  return LBM_OK;
}

int lbm_batch_plan(int count, const int* dims, int block, int nwg, int* n_segments, uint16_t* segments,
                   uint32_t* wg_first, int* strips, double* balance) {
  if (count < 1 || !dims || nwg < 1 || !n_segments) return bfail(nullptr, LBM_ERR_INVALID_ARG, "bad argument");
  if (std::find(std::begin(kBatchBlocks), std::end(kBatchBlocks), block) == std::end(kBatchBlocks))
    return bfail(nullptr, LBM_ERR_INVALID_ARG, "block must be 256, 512 or 1024");
  std::vector<int> dv(dims, dims + 3 * count);
  for (int v : dv)
    if (v < 1 || v > 65535) return bfail(nullptr, LBM_ERR_INVALID_ARG, "dimensions must be in 1..65535");
  std::vector<double> taus(size_t(count), 0.6);
  std::vector<uint32_t> offs(size_t(count), 0);
  HostPlan hp;
  const std::string msg = make_plan(dv, taus, offs, block, nwg, &hp);
  if (!msg.empty()) return bfail(nullptr, LBM_ERR_UNSUPPORTED, msg);
  const int ns = int(hp.segs.size());
  if (segments && *n_segments < ns) {
    *n_segments = ns;
    return bfail(nullptr, LBM_ERR_INVALID_ARG, "segments array too small");
  }
  *n_segments = ns;
  if (segments)
    for (int i = 0; i < ns; ++i) {
      segments[4 * i] = hp.segs[size_t(i)].dom;
      segments[4 * i + 1] = hp.segs[size_t(i)].strip;
      segments[4 * i + 2] = hp.segs[size_t(i)].za;
      segments[4 * i + 3] = hp.segs[size_t(i)].zb;
    }
  if (wg_first)
    for (int i = 0; i <= nwg; ++i) wg_first[i] = hp.wg_first[size_t(i)];
  if (strips)
    for (int d = 0; d < count; ++d) {
      const BatchDomain& D = hp.doms[size_t(d)];
      strips[3 * d] = D.rows;
      strips[3 * d + 1] = D.ty;
      strips[3 * d + 2] = D.span;
    }
  if (balance) *balance = hp.max_cost > 0 ? hp.mean_cost / hp.max_cost : 1.0;
  return LBM_OK;
}

}  // extern "C"
