// lbm_aux.hip -- state set-up, read-back, health scan and the dither probe.
#include "lbm_codec.h"

namespace lbm {

namespace {

__device__ inline uint32_t grid_index() { return blockIdx.x * blockDim.x + threadIdx.x; }

// Encode full moments (rho, j, P) without dither (Sec. 5.3 codec).
template <int FMT>
__device__ inline void encode_plain(const float m[10], uint32_t* w) {
  const float rho = m[0];
  const float inv = 1.0f / rho;
  const float u[3] = {m[1] * inv, m[2] * inv, m[3] * inv};
  const float N[6] = {fmaf(-m[1], u[0], m[4]), fmaf(-m[2], u[1], m[5]), fmaf(-m[3], u[2], m[6]),
                      fmaf(-m[1], u[1], m[7]), fmaf(-m[1], u[2], m[8]), fmaf(-m[2], u[2], m[9])};
  uint32_t q[10];
  if constexpr (FMT == FMT_Q16) {
    q[0] = quantize(rho - Q_RHO_LO, Q_RHO_S, 0.0f);
#pragma unroll
    for (int a = 0; a < 3; ++a) q[1 + a] = quantize(u[a] - Q_U_LO, Q_U_S, 0.0f);
#pragma unroll
    for (int p = 0; p < 6; ++p) q[4 + p] = quantize(N[p] - Q_N_LO, Q_N_S, 0.0f);
#pragma unroll
    for (int k = 0; k < 5; ++k) w[k] = q[2 * k] | (q[2 * k + 1] << 16);
  } else {
    using PK = typename Codec<FMT>::PK;
    q[0] = quantize_b(rho - Q_RHO_LO, PK::SR, 0.0f, PK::qmax(0));
#pragma unroll
    for (int a = 0; a < 3; ++a) q[1 + a] = quantize_b(u[a] - Q_U_LO, PK::SU, 0.0f, PK::qmax(1));
#pragma unroll
    for (int p = 0; p < 6; ++p) q[4 + p] = quantize_b(N[p] - Q_N_LO, PK::SN, 0.0f, PK::qmax(4));
    pack_codes<PK>(q, w);
  }
}

// Writes full moments (rho, j, P); the FP32 state keeps rho - 1 in plane 0.
template <int FMT>
__device__ inline void write_state(void* const out[10], uint32_t c, const float m[10]) {
  if constexpr (FMT == FMT_F32) {
    static_cast<float*>(out[0])[c] = m[0] - 1.0f;
#pragma unroll
    for (int k = 1; k < 10; ++k) static_cast<float*>(out[k])[c] = m[k];
  } else {
    uint32_t w[Codec<FMT>::W];
    encode_plain<FMT>(m, w);
#pragma unroll
    for (int k = 0; k < Codec<FMT>::W; ++k) static_cast<uint32_t*>(out[k])[c] = w[k];
  }
}

struct Planes10 {
  void* p[10];
};
struct CPlanes10 {
  const void* p[10];
};

template <int FMT>
__global__ void set_moments_kernel(const float* __restrict__ m, Planes10 out, const uint8_t* __restrict__ mask,
                                   uint32_t N) {
  const uint32_t c = grid_index();
  if (c >= N) return;
  float v[10] = {1, 0, 0, 0, 0, 0, 0, 0, 0, 0};
  if (!(mask && mask[c])) {
#pragma unroll
    for (int k = 0; k < 10; ++k) v[k] = m[size_t(k) * N + c];
  }
  write_state<FMT>(out.p, c, v);
}

template <int FMT>
__global__ void set_equilibrium_kernel(const float* __restrict__ rho, const float* __restrict__ u, Planes10 out,
                                       const uint8_t* __restrict__ mask, uint32_t N) {
  const uint32_t c = grid_index();
  if (c >= N) return;
  float v[10] = {1, 0, 0, 0, 0, 0, 0, 0, 0, 0};
  if (!(mask && mask[c])) {
    const float r = rho[c];
    const float ux = u[c], uy = u[size_t(N) + c], uz = u[2 * size_t(N) + c];
    v[0] = r;
    v[1] = r * ux;
    v[2] = r * uy;
    v[3] = r * uz;
    v[4] = v[1] * ux;
    v[5] = v[2] * uy;
    v[6] = v[3] * uz;
    v[7] = v[1] * uy;
    v[8] = v[1] * uz;
    v[9] = v[2] * uz;
  }
  write_state<FMT>(out.p, c, v);
}

template <int FMT>
__global__ void get_moments_kernel(CPlanes10 in, float* __restrict__ m, const uint8_t* __restrict__ mask, uint32_t N) {
  const uint32_t c = grid_index();
  if (c >= N) return;
  float v[10] = {1, 0, 0, 0, 0, 0, 0, 0, 0, 0};
  if (!(mask && mask[c])) {
    if constexpr (FMT == FMT_F32) {
#pragma unroll
      for (int k = 0; k < 10; ++k) v[k] = static_cast<const float*>(in.p[k])[c];
      v[0] += 1.0f;
    } else {
      uint32_t w[Codec<FMT>::W];
#pragma unroll
      for (int k = 0; k < Codec<FMT>::W; ++k) w[k] = static_cast<const uint32_t*>(in.p[k])[c];
      const CellIn q = Codec<FMT>::decode(w);
      v[0] = q.rho;
      v[1] = q.rho * q.u[0];
      v[2] = q.rho * q.u[1];
      v[3] = q.rho * q.u[2];
      v[4] = fmaf(v[1], q.u[0], q.N[0]);
      v[5] = fmaf(v[2], q.u[1], q.N[1]);
      v[6] = fmaf(v[3], q.u[2], q.N[2]);
      v[7] = fmaf(v[1], q.u[1], q.N[3]);
      v[8] = fmaf(v[1], q.u[2], q.N[4]);
      v[9] = fmaf(v[2], q.u[2], q.N[5]);
    }
  }
#pragma unroll
  for (int k = 0; k < 10; ++k) m[size_t(k) * N + c] = v[k];
}

template <int FMT>
__global__ void health_kernel(CPlanes10 in, uint32_t N, unsigned long long* bad) {
  const uint32_t c = grid_index();
  uint32_t n = 0;
  if (c < N) {
    if constexpr (FMT == FMT_F32) {
#pragma unroll
      for (int k = 0; k < 10; ++k) n += isfinite(static_cast<const float*>(in.p[k])[c]) ? 0u : 1u;
    } else {
      uint32_t w[Codec<FMT>::W];
#pragma unroll
      for (int k = 0; k < Codec<FMT>::W; ++k) w[k] = static_cast<const uint32_t*>(in.p[k])[c];
      n = Codec<FMT>::saturated(w);
    }
  }
  // one atomic per wavefront with offenders
  const unsigned long long vote = __ballot(n != 0);
  if (vote == 0ull) return;
  uint32_t tot = n;
  for (int off = 32; off > 0; off >>= 1) tot += __shfl_xor(tot, off);
  if (__lane_id() == __ffsll(static_cast<long long>(vote)) - 1) atomicAdd(bad, static_cast<unsigned long long>(tot));
}

template <int FMT>
__global__ void set_rest_kernel(Planes10 out, uint32_t N) {
  const uint32_t c = grid_index();
  if (c >= N) return;
  const float v[10] = {1, 0, 0, 0, 0, 0, 0, 0, 0, 0};
  write_state<FMT>(out.p, c, v);
}

// Runs f.template operator()<FMT>() for any stored format.
template <class Fn>
hipError_t for_format(int fmt, Fn&& f) {
  if (fmt == FMT_F32) {
    f.template operator()<FMT_F32>();
  } else if (!dispatch_codes(fmt, f)) {
    return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

__global__ void debug_dither_kernel(int n, const uint32_t* __restrict__ idx, uint32_t key, uint32_t* __restrict__ out) {
  const int k = int(grid_index());
  if (k >= n) return;
  uint32_t h1, h2;
  dither_words(idx[k], key, h1, h2);
  out[2 * k] = h1;
  out[2 * k + 1] = h2;
}

dim3 grid_for(int64_t N) { return dim3(uint32_t((N + 255) / 256)); }

__global__ void set_counter_kernel(uint32_t* ctr, uint32_t v) {
  if (threadIdx.x == 0) *ctr = v;
}

}  // namespace

hipError_t launch_set_counter(uint32_t* ctr, uint32_t v, hipStream_t s) {
  hipLaunchKernelGGL(set_counter_kernel, dim3(1), dim3(64), 0, s, ctr, v);
  return hipGetLastError();
}

hipError_t launch_set_moments(int fmt, const float* m, void* const out[10], const uint8_t* mask, int64_t N,
                              hipStream_t s) {
  Planes10 o;
  for (int k = 0; k < 10; ++k) o.p[k] = out[k];
  return for_format(fmt, [&]<int F>() {
    hipLaunchKernelGGL(set_moments_kernel<F>, grid_for(N), dim3(256), 0, s, m, o, mask, uint32_t(N));
  });
}

hipError_t launch_set_equilibrium(int fmt, const float* rho, const float* u, void* const out[10],
                                  const uint8_t* mask, int64_t N, hipStream_t s) {
  Planes10 o;
  for (int k = 0; k < 10; ++k) o.p[k] = out[k];
  return for_format(fmt, [&]<int F>() {
    hipLaunchKernelGGL(set_equilibrium_kernel<F>, grid_for(N), dim3(256), 0, s, rho, u, o, mask, uint32_t(N));
  });
}

hipError_t launch_get_moments(int fmt, const void* const in[10], float* m, const uint8_t* mask, int64_t N,
                              hipStream_t s) {
  CPlanes10 i;
  for (int k = 0; k < 10; ++k) i.p[k] = in[k];
  return for_format(fmt, [&]<int F>() {
    hipLaunchKernelGGL(get_moments_kernel<F>, grid_for(N), dim3(256), 0, s, i, m, mask, uint32_t(N));
  });
}

hipError_t launch_health(int fmt, const void* const in[10], int64_t N, unsigned long long* bad, hipStream_t s) {
  CPlanes10 i;
  for (int k = 0; k < 10; ++k) i.p[k] = in[k];
  return for_format(fmt, [&]<int F>() {
    hipLaunchKernelGGL(health_kernel<F>, grid_for(N), dim3(256), 0, s, i, uint32_t(N), bad);
  });
}

hipError_t launch_set_rest(int fmt, void* const out[10], int64_t N, hipStream_t s) {
  Planes10 o;
  for (int k = 0; k < 10; ++k) o.p[k] = out[k];
  return for_format(fmt, [&]<int F>() {
    hipLaunchKernelGGL(set_rest_kernel<F>, grid_for(N), dim3(256), 0, s, o, uint32_t(N));
  });
}

hipError_t launch_debug_dither(int n, const uint32_t* idx, uint32_t key, uint32_t* out, hipStream_t s) {
  hipLaunchKernelGGL(debug_dither_kernel, grid_for(n), dim3(256), 0, s, n, idx, key, out);
  return hipGetLastError();
}

}  // namespace lbm
