// DMRS least-squares channel estimation (channel estimation is one of the PHY blocks the
// paper's Sec. III-B names as suited to data-level parallelism; LS is the standard
// estimator).  The value of each output is
//   h(o, j, r, p) = (1/T) sum_t rx(sym0[o] + t, k, r) conj(pilot(o, t, j, p)),
//   k = (p mod C) + C j,
// and for the full-resolution output the linear interpolation between the port's two
// nearest pilots.  Output order [..][rx][layer] puts consecutive threads on consecutive
// layers of one antenna, so the writes are contiguous.  Comb C <= 8, Nr <= 64, Nl <= 16.
#include "geom.h"
#include "rx_load.h"

namespace ranphy {
namespace {

template <int T, int RXF>
__device__ __forceinline__ float2 ls_at(const Geom& g, const float2* __restrict__ rx,
                                        const float2* __restrict__ pil, int64_t slot, int o,
                                        int j, int r, int p) {
  const int k = (p & (g.comb - 1)) + g.comb * j;
  float2 y[T], q[T];
#pragma unroll
  for (int t = 0; t < T; ++t) {
    const int s = g.sym0[o] + t;
    y[t] = rx_at<RXF>(rx, (slot * g.n_symb + s) * g.n_sc + k, g.n_rx, r);
    q[t] = pil[(((slot * g.n_occ + o) * T + t) * g.n_pilot + j) * g.n_layers + p];
  }
  return ls_pilot<T>(q, y);
}

// Pilot resolution: one block per (slot, occasion, pilot index j).  The C subcarriers
// C j .. C j + C - 1 hold pilot j of every comb offset; their samples on the T DMRS symbols
// (C x Nr contiguous values per symbol) are read with consecutive threads on consecutive
// values into LDS, rows padded by one value so that threads of different comb offsets read
// different banks, and the Nr x Nl output row h[j][rx][layer] is written contiguously.
template <int T, int RXF>
__global__ void __launch_bounds__(256) chest_pilot_kernel(Geom g, const float2* __restrict__ rx,
                                                          const float2* __restrict__ pil,
                                                          float2* __restrict__ h) {
  __shared__ float2 ys[T * 8 * (kMaxRx + 1)];
  __shared__ float2 ps[T * kMaxLayers];
  const int C = g.comb, NR = g.n_rx, NL = g.n_layers;
  const int j = blockIdx.x % g.n_pilot;
  const int so = blockIdx.x / g.n_pilot;  // slot * n_occ + occasion
  const int o = so % g.n_occ;
  const int64_t slot = so / g.n_occ;
  const int n_in = T * C * NR;
  for (int f = threadIdx.x; f < n_in; f += 256) {
    const int t = f / (C * NR);
    const int rem = f - t * (C * NR);
    const int c = rem / NR;
    const int r = rem - c * NR;
    const int k = C * j + c;
    float2 v = make_float2(0.f, 0.f);
    if (k < g.n_sc) v = rx_at<RXF>(rx, (slot * g.n_symb + g.sym0[o] + t) * g.n_sc + k, NR, r);
    ys[(t * C + c) * (NR + 1) + r] = v;
  }
  if (threadIdx.x < T * NL) {
    const int t = threadIdx.x / NL, p = threadIdx.x - t * NL;
    ps[threadIdx.x] = pil[(((int64_t)so * T + t) * g.n_pilot + j) * NL + p];
  }
  __syncthreads();
  float2* __restrict__ dst = h + ((int64_t)so * g.n_pilot + j) * NR * NL;
  for (int e = threadIdx.x; e < NR * NL; e += 256) {
    const int r = e / NL;
    const int p = e - r * NL;
    const int c = p & (C - 1);
    float2 v = make_float2(0.f, 0.f);
    if (C * j + c < g.n_sc) {
      float2 q[T], y[T];
#pragma unroll
      for (int t = 0; t < T; ++t) {
        q[t] = ps[t * NL + p];
        y[t] = ys[(t * C + c) * (NR + 1) + r];
      }
      v = ls_pilot<T>(q, y);
    }
    dst[e] = v;
  }
}

// chest_pilot_kernel for power-of-two Nr >= 2 and Nl >= 2 on 16-byte aligned complex64
// buffers (the usual arrays): the same values, with shifts in place of the index divisions
// (the kernel is short, so its index arithmetic is a visible share of its time), each
// thread loading two antennas and storing two layers per 16-byte access.
template <int T>
__global__ void __launch_bounds__(256) chest_pilot2_kernel(Geom g, const float2* __restrict__ rx,
                                                           const float2* __restrict__ pil,
                                                           float2* __restrict__ h, int lnr,
                                                           int lnl) {
  __shared__ float2 ys[T * 8 * (kMaxRx + 1)];
  __shared__ float2 ps[T * kMaxLayers];
  const int C = g.comb, lc = g.comb_log2, NR = 1 << lnr, NL = 1 << lnl;
  const int j = blockIdx.x % g.n_pilot;
  const int so = blockIdx.x / g.n_pilot;  // slot * n_occ + occasion
  const int o = so % g.n_occ;
  const int64_t slot = so / g.n_occ;
  const int n_in = (T * C * NR) >> 1;  // antenna pairs
  for (int f = threadIdx.x; f < n_in; f += 256) {
    const int t = f >> (lc + lnr - 1);
    const int c = (f >> (lnr - 1)) & (C - 1);
    const int r = (f & ((NR >> 1) - 1)) << 1;
    const int k = C * j + c;
    float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
    if (k < g.n_sc)
      v = *reinterpret_cast<const float4*>(
          rx + ((slot * g.n_symb + g.sym0[o] + t) * g.n_sc + k) * NR + r);
    float2* y = ys + (t * C + c) * (NR + 1) + r;
    y[0] = make_float2(v.x, v.y);
    y[1] = make_float2(v.z, v.w);
  }
  if (threadIdx.x < T * NL) {
    const int t = threadIdx.x >> lnl, p = threadIdx.x & (NL - 1);
    ps[threadIdx.x] = pil[(((int64_t)so * T + t) * g.n_pilot + j) * NL + p];
  }
  __syncthreads();
  float4* __restrict__ dst = reinterpret_cast<float4*>(h + ((int64_t)so * g.n_pilot + j) * NR * NL);
  for (int e = threadIdx.x; e < (NR * NL) >> 1; e += 256) {  // layer pairs
    const int r = e >> (lnl - 1);
    const int p = (e & ((NL >> 1) - 1)) << 1;
    float2 v[2];
#pragma unroll
    for (int w = 0; w < 2; ++w) {
      const int c = (p + w) & (C - 1);
      v[w] = make_float2(0.f, 0.f);
      if (C * j + c < g.n_sc) {
        float2 q[T], y[T];
#pragma unroll
        for (int t = 0; t < T; ++t) {
          q[t] = ps[t * NL + p + w];
          y[t] = ys[(t * C + c) * (NR + 1) + r];
        }
        v[w] = ls_pilot<T>(q, y);
      }
    }
    dst[e] = make_float4(v[0].x, v[0].y, v[1].x, v[1].y);
  }
}

// Pilot resolution for small arrays: one block per (slot, occasion, run of up to jb
// consecutive pilot indices), so that every block has work for its 256 threads.  Pilots
// j0 .. j0 + jb - 1 of every comb offset sit on the C jb contiguous subcarriers
// C j0 .. C (j0 + jb) - 1, so the run's samples on each of the T DMRS symbols are C jb Nr
// contiguous values: read with consecutive threads on consecutive values into LDS,
// rows padded by one value so that threads of different comb offsets read different banks.
// The run's output rows h[j][rx][layer] (jb Nr Nl contiguous values) are written
// contiguously.  jb = 1 takes chest_pilot_kernel, which needs fewer index divisions.
constexpr int kRunPadded = 520;  // C jb (Nr + 1) <= 520 values per DMRS symbol
constexpr int kRunPilots = 512;  // T jb Nl <= 512 pilot values

template <int T, int RXF>
__global__ void __launch_bounds__(256) chest_run_kernel(Geom g, const float2* __restrict__ rx,
                                                          const float2* __restrict__ pil,
                                                          float2* __restrict__ h, int jb) {
  __shared__ float2 ys[T * kRunPadded];
  __shared__ float2 ps[kRunPilots];
  const int C = g.comb, NR = g.n_rx, NL = g.n_layers;
  const int nrun = (g.n_pilot + jb - 1) / jb;
  const int run = blockIdx.x % nrun;
  const int so = blockIdx.x / nrun;  // slot * n_occ + occasion
  const int o = so % g.n_occ;
  const int64_t slot = so / g.n_occ;
  const int j0 = run * jb;
  const int nj = min(jb, g.n_pilot - j0);
  const int pitch = NR + 1;
  const int rowv = C * nj * NR;  // the run's values per DMRS symbol
  for (int f = threadIdx.x; f < T * rowv; f += 256) {
    const int t = f / rowv;
    const int rem = f - t * rowv;
    const int kk = rem / NR;  // subcarrier offset in the run
    const int r = rem - kk * NR;
    const int k = C * j0 + kk;
    float2 v = make_float2(0.f, 0.f);
    if (k < g.n_sc) v = rx_at<RXF>(rx, (slot * g.n_symb + g.sym0[o] + t) * g.n_sc + k, NR, r);
    ys[(t * C * jb + kk) * pitch + r] = v;
  }
  for (int f = threadIdx.x; f < T * nj * NL; f += 256) {
    const int t = f / (nj * NL);
    const int rem = f - t * (nj * NL);
    const int jj = rem / NL;
    const int p = rem - jj * NL;
    ps[(t * jb + jj) * NL + p] = pil[(((int64_t)so * T + t) * g.n_pilot + j0 + jj) * NL + p];
  }
  __syncthreads();
  float2* __restrict__ dst = h + ((int64_t)so * g.n_pilot + j0) * NR * NL;
  for (int e = threadIdx.x; e < nj * NR * NL; e += 256) {
    const int jj = e / (NR * NL);
    const int rem = e - jj * (NR * NL);
    const int r = rem / NL;
    const int p = rem - r * NL;
    const int c = p & (C - 1);
    const int kk = C * jj + c;
    float2 v = make_float2(0.f, 0.f);
    if (C * j0 + kk < g.n_sc) {
      float2 q[T], y[T];
#pragma unroll
      for (int t = 0; t < T; ++t) {
        q[t] = ps[(t * jb + jj) * NL + p];
        y[t] = ys[(t * C * jb + kk) * pitch + r];
      }
      v = ls_pilot<T>(q, y);
    }
    dst[e] = v;
  }
}

template <int T, int RXF>
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
  const float2 v0 = ls_at<T, RXF>(g, rx, pil, slot, o, j0, r, p);
  const float2 v1 = ls_at<T, RXF>(g, rx, pil, slot, o, j1, r, p);
  h[e] = make_float2(v0.x + a * (v1.x - v0.x), v0.y + a * (v1.y - v0.y));
}

template <int RXF>
hipError_t launch_chest_rxf(const Geom& g, const float2* rx, const float2* pilots, float2* h,
                            int h_res, hipStream_t s) {
  const int64_t per = (int64_t)g.n_occ * g.n_rx * g.n_layers * (h_res == 0 ? g.n_pilot : g.n_sc);
  const int64_t total = per * g.n_slots;
  if (total == 0) return hipSuccess;
  const dim3 block(256), grid((unsigned)((total + 255) / 256));
  if (h_res == 0) {
    int jb = min(kRunPadded / (g.comb * (g.n_rx + 1)), kRunPilots / (g.td * g.n_layers));
    jb = max(1, min(64, jb));
    const int nrun = (g.n_pilot + jb - 1) / jb;
    const dim3 pgrid((unsigned)((int64_t)g.n_slots * g.n_occ * nrun));
    const bool pow2 = g.n_rx >= 2 && g.n_layers >= 2 && (g.n_rx & (g.n_rx - 1)) == 0 &&
                      (g.n_layers & (g.n_layers - 1)) == 0;
    const bool al16 = ((reinterpret_cast<uintptr_t>(rx) | reinterpret_cast<uintptr_t>(h)) & 15) == 0;
    if (jb == 1 && RXF == 0 && pow2 && al16) {
      const int lnr = __builtin_ctz(g.n_rx), lnl = __builtin_ctz(g.n_layers);
      if (g.td == 1)
        hipLaunchKernelGGL((chest_pilot2_kernel<1>), pgrid, block, 0, s, g, rx, pilots, h, lnr, lnl);
      else
        hipLaunchKernelGGL((chest_pilot2_kernel<2>), pgrid, block, 0, s, g, rx, pilots, h, lnr, lnl);
    } else if (jb == 1) {
      if (g.td == 1)
        hipLaunchKernelGGL((chest_pilot_kernel<1, RXF>), pgrid, block, 0, s, g, rx, pilots, h);
      else
        hipLaunchKernelGGL((chest_pilot_kernel<2, RXF>), pgrid, block, 0, s, g, rx, pilots, h);
    } else if (g.td == 1) {
      hipLaunchKernelGGL((chest_run_kernel<1, RXF>), pgrid, block, 0, s, g, rx, pilots, h, jb);
    } else {
      hipLaunchKernelGGL((chest_run_kernel<2, RXF>), pgrid, block, 0, s, g, rx, pilots, h, jb);
    }
  } else {
    if (g.td == 1)
      hipLaunchKernelGGL((chest_full_kernel<1, RXF>), grid, block, 0, s, g, rx, pilots, h);
    else
      hipLaunchKernelGGL((chest_full_kernel<2, RXF>), grid, block, 0, s, g, rx, pilots, h);
  }
  return hipGetLastError();
}

}  // namespace

// rx: the complex64 grid, or (bfp) its block floating point words.
hipError_t launch_chest_ls(const Geom& g, const float2* rx, bool bfp, const float2* pilots,
                           float2* h, int h_res, hipStream_t s) {
  return bfp ? launch_chest_rxf<1>(g, rx, pilots, h, h_res, s)
             : launch_chest_rxf<0>(g, rx, pilots, h, h_res, s);
}

}  // namespace ranphy
