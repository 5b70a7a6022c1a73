// Linear MMSE detection, one thread per data resource element (the general path: any
// layer count, any number of DMRS occasions, pilot- or full-resolution channel input).
//
// Per resource element (Sec. IV / Fig. 4 of the paper: LMMSE detection through a
// triangular factorisation and forward/backward substitution; the layer-domain covariance
// is Hermitian positive definite, so the factorisation is Cholesky):
//   1. H(k, s): frequency interpolation of the estimate at occasions o0, o1, then linear
//      interpolation in time with the data symbol's weight;
//   2. streamed over receive antennas: G += h_r^H h_r (lower triangle), z += h_r^H y_r;
//   3. G += s2 I;  G = L L^H;  x_hat = L^-H L^-1 z;
//   4. d_l = (G^-1)_ll = || L^-1 e_l ||^2;  mu = 1 - s2 d;  x = x_hat / mu;
//      nv = s2 d / mu  (= (1 - mu) / mu without the cancellation of 1 - mu).
// A pivot that is not positive relative to its diagonal entry marks the element as failed:
// NaN symbols and +inf variance for every layer.
#include <float.h>

#include "geom.h"

namespace ranphy {
namespace {

constexpr float kPivotRel = 16.f * FLT_EPSILON;

template <int HRES>
__device__ __forceinline__ float2 hval(const Geom& g, const float2* __restrict__ h, int64_t slot,
                                       int o, int k, int r, int p, int j0, int j1, float a) {
  if (HRES == 0) {
    const int64_t base = (slot * g.n_occ + o) * g.n_pilot;
    const float2 v0 = h[((base + j0) * g.n_rx + r) * g.n_layers + p];
    const float2 v1 = h[((base + j1) * g.n_rx + r) * g.n_layers + p];
    return make_float2(v0.x + a * (v1.x - v0.x), v0.y + a * (v1.y - v0.y));
  } else {
    return h[(((slot * g.n_occ + o) * g.n_sc + k) * g.n_rx + r) * g.n_layers + p];
  }
}

__host__ __device__ constexpr int tri(int i, int j) { return i * (i + 1) / 2 + j; }

template <int NL, int HRES>
__global__ void __launch_bounds__(256) mmse_re_kernel(Geom g, const float2* __restrict__ rx,
                                                      const float2* __restrict__ h,
                                                      const float* __restrict__ nvar,
                                                      float2* __restrict__ x,
                                                      float* __restrict__ nv) {
  const int64_t total = (int64_t)g.n_slots * g.n_dsym * g.n_sc;
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= total) return;
  const int k = (int)(e % g.n_sc);
  const int64_t q = e / g.n_sc;
  const int di = (int)(q % g.n_dsym);
  const int64_t slot = q / g.n_dsym;
  const int s = g.dsym[di];
  const int o0 = g.t_o0[di], o1 = g.t_o1[di];
  const float w = g.t_w[di];

  int j0[NL], j1[NL];
  float a[NL];
#pragma unroll
  for (int p = 0; p < NL; ++p) {
    if (HRES == 0) {
      freq_rule(g, p, k, j0[p], j1[p], a[p]);
    } else {
      j0[p] = j1[p] = 0;
      a[p] = 0.f;
    }
  }

  constexpr int NP = NL * (NL + 1) / 2;
  float2 G[NP];
  float2 z[NL];
#pragma unroll
  for (int i = 0; i < NP; ++i) G[i] = make_float2(0.f, 0.f);
#pragma unroll
  for (int i = 0; i < NL; ++i) z[i] = make_float2(0.f, 0.f);

  const float2* __restrict__ yrow = rx + ((slot * g.n_symb + s) * g.n_sc + k) * g.n_rx;
  for (int r = 0; r < g.n_rx; ++r) {
    float2 hr[NL];
#pragma unroll
    for (int p = 0; p < NL; ++p) {
      float2 v = hval<HRES>(g, h, slot, o0, k, r, p, j0[p], j1[p], a[p]);
      if (o1 != o0) {
        const float2 v1 = hval<HRES>(g, h, slot, o1, k, r, p, j0[p], j1[p], a[p]);
        v = make_float2(v.x + w * (v1.x - v.x), v.y + w * (v1.y - v.y));
      }
      hr[p] = v;
    }
    const float2 y = yrow[r];
#pragma unroll
    for (int i = 0; i < NL; ++i) {
      const float2 m = cmulc(hr[i], y);
      z[i].x += m.x;
      z[i].y += m.y;
#pragma unroll
      for (int j = 0; j <= i; ++j) {
        const float2 gg = cmulc(hr[i], hr[j]);
        G[tri(i, j)].x += gg.x;
        G[tri(i, j)].y += gg.y;
      }
    }
  }

  const float s2 = nvar[slot];
  float gd[NL];
#pragma unroll
  for (int i = 0; i < NL; ++i) {
    G[tri(i, i)].x += s2;
    gd[i] = G[tri(i, i)].x;
  }

  // Cholesky G = L L^H in place (lower triangle), reciprocal diagonal kept aside.
  bool ok = true;
  float linv[NL];
#pragma unroll
  for (int j = 0; j < NL; ++j) {
    float dj = G[tri(j, j)].x;
#pragma unroll
    for (int kk = 0; kk < j; ++kk) dj -= G[tri(j, kk)].x * G[tri(j, kk)].x + G[tri(j, kk)].y * G[tri(j, kk)].y;
    ok = ok && (dj > kPivotRel * gd[j]);
    const float ljj = sqrtf(fmaxf(dj, FLT_MIN));
    const float inv = 1.f / ljj;
    G[tri(j, j)] = make_float2(ljj, 0.f);
    linv[j] = inv;
#pragma unroll
    for (int i = j + 1; i < NL; ++i) {
      float2 acc = G[tri(i, j)];
#pragma unroll
      for (int kk = 0; kk < j; ++kk) {
        // acc -= L[i][kk] conj(L[j][kk])
        const float2 m = cmulc(G[tri(j, kk)], G[tri(i, kk)]);
        acc.x -= m.x;
        acc.y -= m.y;
      }
      G[tri(i, j)] = make_float2(acc.x * inv, acc.y * inv);
    }
  }

  // Forward substitution L w = z.
  float2 wv[NL];
#pragma unroll
  for (int i = 0; i < NL; ++i) {
    float2 acc = z[i];
#pragma unroll
    for (int kk = 0; kk < i; ++kk) {
      const float2 m = cmul(G[tri(i, kk)], wv[kk]);
      acc.x -= m.x;
      acc.y -= m.y;
    }
    wv[i] = make_float2(acc.x * linv[i], acc.y * linv[i]);
  }
  // Backward substitution L^H x = w.
  float2 xh[NL];
#pragma unroll
  for (int i = NL - 1; i >= 0; --i) {
    float2 acc = wv[i];
#pragma unroll
    for (int kk = i + 1; kk < NL; ++kk) {
      const float2 m = cmulc(G[tri(kk, i)], xh[kk]);
      acc.x -= m.x;
      acc.y -= m.y;
    }
    xh[i] = make_float2(acc.x * linv[i], acc.y * linv[i]);
  }

  // d_l = || L^-1 e_l ||^2 by forward substitution from index l.
  float dl[NL];
#pragma unroll
  for (int l = 0; l < NL; ++l) {
    float2 u[NL];
    u[l] = make_float2(linv[l], 0.f);
    float acc2 = linv[l] * linv[l];
#pragma unroll
    for (int i = l + 1; i < NL; ++i) {
      float2 acc = make_float2(0.f, 0.f);
#pragma unroll
      for (int kk = l; kk < i; ++kk) {
        const float2 m = cmul(G[tri(i, kk)], u[kk]);
        acc.x -= m.x;
        acc.y -= m.y;
      }
      u[i] = make_float2(acc.x * linv[i], acc.y * linv[i]);
      acc2 += u[i].x * u[i].x + u[i].y * u[i].y;
    }
    dl[l] = acc2;
  }

  float2* __restrict__ xo = x + e * NL;
  float* __restrict__ nvo = nv + e * NL;
#pragma unroll
  for (int l = 0; l < NL; ++l) {
    const float sd = s2 * dl[l];
    const float mu = 1.f - sd;
    const float im = 1.f / mu;
    if (ok) {
      xo[l] = make_float2(xh[l].x * im, xh[l].y * im);
      nvo[l] = sd * im;
    } else {
      xo[l] = make_float2(__builtin_nanf(""), __builtin_nanf(""));
      nvo[l] = __builtin_inff();
    }
  }
}

template <int NL>
hipError_t launch_nl(const Geom& g, const float2* rx, const float2* h, int h_res,
                     const float* nvar, float2* x, float* nv, hipStream_t s) {
  const int64_t total = (int64_t)g.n_slots * g.n_dsym * g.n_sc;
  const dim3 block(256), grid((unsigned)((total + 255) / 256));
  if (h_res == 0)
    hipLaunchKernelGGL((mmse_re_kernel<NL, 0>), grid, block, 0, s, g, rx, h, nvar, x, nv);
  else
    hipLaunchKernelGGL((mmse_re_kernel<NL, 1>), grid, block, 0, s, g, rx, h, nvar, x, nv);
  return hipGetLastError();
}

}  // namespace

hipError_t launch_mmse_re(const Geom& g, const float2* rx, const float2* h, int h_res,
                          const float* nvar, float2* x, float* nv, hipStream_t s) {
  switch (g.n_layers) {
    case 1: return launch_nl<1>(g, rx, h, h_res, nvar, x, nv, s);
    case 2: return launch_nl<2>(g, rx, h, h_res, nvar, x, nv, s);
    case 3: return launch_nl<3>(g, rx, h, h_res, nvar, x, nv, s);
    case 4: return launch_nl<4>(g, rx, h, h_res, nvar, x, nv, s);
    case 5: return launch_nl<5>(g, rx, h, h_res, nvar, x, nv, s);
    case 6: return launch_nl<6>(g, rx, h, h_res, nvar, x, nv, s);
    case 7: return launch_nl<7>(g, rx, h, h_res, nvar, x, nv, s);
    case 8: return launch_nl<8>(g, rx, h, h_res, nvar, x, nv, s);
    case 9: return launch_nl<9>(g, rx, h, h_res, nvar, x, nv, s);
    case 10: return launch_nl<10>(g, rx, h, h_res, nvar, x, nv, s);
    case 11: return launch_nl<11>(g, rx, h, h_res, nvar, x, nv, s);
    case 12: return launch_nl<12>(g, rx, h, h_res, nvar, x, nv, s);
    case 13: return launch_nl<13>(g, rx, h, h_res, nvar, x, nv, s);
    case 14: return launch_nl<14>(g, rx, h, h_res, nvar, x, nv, s);
    case 15: return launch_nl<15>(g, rx, h, h_res, nvar, x, nv, s);
    case 16: return launch_nl<16>(g, rx, h, h_res, nvar, x, nv, s);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace ranphy
