// DMRS least-squares channel estimation (channel estimation is one of the PHY blocks the
// paper's Sec. III-B names as suited to data-level parallelism; LS is the standard
// estimator).  One thread per output value; the value is
//   h(o, j, r, p) = (1/T) sum_t rx(sym0[o] + t, k, r) conj(pilot(o, t, j, p)),
//   k = (p mod C) + C j,
// and for the full-resolution output the linear interpolation between the port's two
// nearest pilots.  Output order [..][rx][layer] puts consecutive threads on consecutive
// layers of one antenna, so the writes are contiguous.
#include "geom.h"

namespace ranphy {
namespace {

template <int T>
__device__ __forceinline__ float2 ls_at(const Geom& g, const float2* __restrict__ rx,
                                        const float2* __restrict__ pil, int64_t slot, int o,
                                        int j, int r, int p) {
  const int k = (p & (g.comb - 1)) + g.comb * j;
  float2 acc = make_float2(0.f, 0.f);
#pragma unroll
  for (int t = 0; t < T; ++t) {
    const int s = g.sym0[o] + t;
    const float2 y = rx[((slot * g.n_symb + s) * g.n_sc + k) * g.n_rx + r];
    const float2 q = pil[(((slot * g.n_occ + o) * T + t) * g.n_pilot + j) * g.n_layers + p];
    const float2 m = cmulc(q, y);  // y * conj(q)
    acc.x += m.x;
    acc.y += m.y;
  }
  const float inv = 1.f / (float)T;
  return make_float2(acc.x * inv, acc.y * inv);
}

template <int T>
__global__ void __launch_bounds__(256) chest_pilot_kernel(Geom g, const float2* __restrict__ rx,
                                                          const float2* __restrict__ pil,
                                                          float2* __restrict__ h) {
  const int64_t total = (int64_t)g.n_slots * g.n_occ * g.n_pilot * g.n_rx * g.n_layers;
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= total) return;
  const int p = (int)(e % g.n_layers);
  int64_t q = e / g.n_layers;
  const int r = (int)(q % g.n_rx);
  q /= g.n_rx;
  const int j = (int)(q % g.n_pilot);
  q /= g.n_pilot;
  const int o = (int)(q % g.n_occ);
  const int64_t slot = q / g.n_occ;
  const int k = (p & (g.comb - 1)) + g.comb * j;
  h[e] = (k < g.n_sc) ? ls_at<T>(g, rx, pil, slot, o, j, r, p) : make_float2(0.f, 0.f);
}

template <int T>
__global__ void __launch_bounds__(256) chest_full_kernel(Geom g, const float2* __restrict__ rx,
                                                         const float2* __restrict__ pil,
                                                         float2* __restrict__ h) {
  const int64_t total = (int64_t)g.n_slots * g.n_occ * g.n_sc * g.n_rx * g.n_layers;
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= total) return;
  const int p = (int)(e % g.n_layers);
  int64_t q = e / g.n_layers;
  const int r = (int)(q % g.n_rx);
  q /= g.n_rx;
  const int k = (int)(q % g.n_sc);
  q /= g.n_sc;
  const int o = (int)(q % g.n_occ);
  const int64_t slot = q / g.n_occ;
  int j0, j1;
  float a;
  freq_rule(g, p, k, j0, j1, a);
  const float2 v0 = ls_at<T>(g, rx, pil, slot, o, j0, r, p);
  const float2 v1 = ls_at<T>(g, rx, pil, slot, o, j1, r, p);
  h[e] = make_float2(v0.x + a * (v1.x - v0.x), v0.y + a * (v1.y - v0.y));
}

}  // namespace

hipError_t launch_chest_ls(const Geom& g, const float2* rx, const float2* pilots, float2* h,
                           int h_res, hipStream_t s) {
  const int64_t per = (int64_t)g.n_occ * g.n_rx * g.n_layers * (h_res == 0 ? g.n_pilot : g.n_sc);
  const int64_t total = per * g.n_slots;
  if (total == 0) return hipSuccess;
  const dim3 block(256), grid((unsigned)((total + 255) / 256));
  if (h_res == 0) {
    if (g.td == 1) hipLaunchKernelGGL(chest_pilot_kernel<1>, grid, block, 0, s, g, rx, pilots, h);
    else hipLaunchKernelGGL(chest_pilot_kernel<2>, grid, block, 0, s, g, rx, pilots, h);
  } else {
    if (g.td == 1) hipLaunchKernelGGL(chest_full_kernel<1>, grid, block, 0, s, g, rx, pilots, h);
    else hipLaunchKernelGGL(chest_full_kernel<2>, grid, block, 0, s, g, rx, pilots, h);
  }
  return hipGetLastError();
}

}  // namespace ranphy
