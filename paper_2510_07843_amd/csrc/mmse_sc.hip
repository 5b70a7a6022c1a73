// Linear MMSE detection for small MIMO shapes with one DMRS occasion: Nr in {1, 2, 4, 8},
// Nl <= 8, Nr Nl <= 64 (the paper's square 2x2 / 4x4 / 8x8 evaluation shapes, Sec. IV).
//
// With one occasion the channel estimate is held over the slot (no time interpolation), so
// the Gram G = H^H H + s2 I, its factorisation, d_l = (G^-1)_ll and the MMSE filter
// W = G^-1 H^H are the same for every data symbol of a subcarrier.  One thread per
// (slot, subcarrier) computes them once and then applies W to each data symbol:
//   1. H(k) at the subcarrier (frequency interpolation between the port's pilots, or the
//      full-resolution estimate), Nr x Nl in registers;
//   2. G = H^H H + s2 I (lower triangle), Cholesky G = L L^H (Sec. IV / Fig. 4: LMMSE through
//      a triangular factorisation and forward/backward substitution; G is Hermitian positive
//      definite), d_l = || L^-1 e_l ||^2;
//   3. column r of W = L^-H L^-1 conj(H[r][:]), written over row r of H;
//   4. per data symbol: x_hat = W y, mu = 1 - s2 d, x = x_hat / mu, nv = s2 d / mu.
// A pivot that is not positive relative to its diagonal entry marks the subcarrier as failed:
// NaN symbols and +inf variance for every layer of every data symbol, as in the per-RE path.
// Versus one thread per resource element this does the Gram and the factorisation once per
// subcarrier instead of once per data symbol (Nr Nl^2 + Nl^3/3 complex multiply-accumulates
// against Nd (Nr Nl^2 / 2 + Nl^3 / 3)), and each thread streams its subcarrier's samples.
#include <float.h>

#include "geom.h"

namespace ranphy {
namespace {

constexpr float kPivotRel = 16.f * FLT_EPSILON;

__host__ __device__ constexpr int tri(int i, int j) { return i * (i + 1) / 2 + j; }

template <int NR, int NL, int HRES>
__global__ void __launch_bounds__(256) mmse_sc_kernel(Geom g, const float2* __restrict__ rx,
                                                      const float2* __restrict__ h,
                                                      const float* __restrict__ nvar,
                                                      float2* __restrict__ x,
                                                      float* __restrict__ nv) {
  const int64_t total = (int64_t)g.n_slots * g.n_sc;
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= total) return;
  const int k = (int)(e % g.n_sc);
  const int64_t slot = e / g.n_sc;

  // 1. channel at subcarrier k: Hm[r][p]
  float2 Hm[NR][NL];
  if (HRES == 0) {
#pragma unroll
    for (int p = 0; p < NL; ++p) {
      int j0, j1;
      float a;
      freq_rule(g, p, k, j0, j1, a);
      const float2* __restrict__ r0 = h + ((slot * g.n_pilot + j0) * NR) * NL + p;
      const float2* __restrict__ r1 = h + ((slot * g.n_pilot + j1) * NR) * NL + p;
#pragma unroll
      for (int r = 0; r < NR; ++r) {
        const float2 v0 = r0[r * NL];
        const float2 v1 = r1[r * NL];
        Hm[r][p] = make_float2(v0.x + a * (v1.x - v0.x), v0.y + a * (v1.y - v0.y));
      }
    }
  } else {
    const float2* __restrict__ row = h + ((slot * g.n_sc + k) * NR) * NL;
#pragma unroll
    for (int r = 0; r < NR; ++r)
#pragma unroll
      for (int p = 0; p < NL; ++p) Hm[r][p] = row[r * NL + p];
  }

  // 2. Gram (lower triangle), Cholesky in place, reciprocal diagonal aside, d_l
  constexpr int NP = NL * (NL + 1) / 2;
  float2 G[NP];
#pragma unroll
  for (int i = 0; i < NP; ++i) G[i] = make_float2(0.f, 0.f);
#pragma unroll
  for (int r = 0; r < NR; ++r)
#pragma unroll
    for (int i = 0; i < NL; ++i)
#pragma unroll
      for (int j = 0; j <= i; ++j) {
        const float2 m = cmulc(Hm[r][i], Hm[r][j]);  // conj(H[r][i]) H[r][j]
        G[tri(i, j)].x += m.x;
        G[tri(i, j)].y += m.y;
      }
  const float s2 = nvar[slot];
  float gd[NL];
#pragma unroll
  for (int i = 0; i < NL; ++i) {
    G[tri(i, i)].x += s2;
    gd[i] = G[tri(i, i)].x;
  }
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
        const float2 m = cmulc(G[tri(j, kk)], G[tri(i, kk)]);  // L[i][kk] conj(L[j][kk])
        acc.x -= m.x;
        acc.y -= m.y;
      }
      G[tri(i, j)] = make_float2(acc.x * inv, acc.y * inv);
    }
  }
  float im[NL], vo[NL];  // 1 / mu and the post-equalisation variance per layer
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
    const float sd = s2 * acc2;
    im[l] = 1.f / (1.f - sd);
    vo[l] = ok ? sd * im[l] : __builtin_inff();
  }

  // 3. W[:, r] = L^-H L^-1 conj(H[r][:]), over row r of Hm
#pragma unroll
  for (int r = 0; r < NR; ++r) {
    float2 w[NL];
#pragma unroll
    for (int i = 0; i < NL; ++i) {  // forward: L w = conj(H[r][:])
      float2 acc = make_float2(Hm[r][i].x, -Hm[r][i].y);
#pragma unroll
      for (int kk = 0; kk < i; ++kk) {
        const float2 m = cmul(G[tri(i, kk)], w[kk]);
        acc.x -= m.x;
        acc.y -= m.y;
      }
      w[i] = make_float2(acc.x * linv[i], acc.y * linv[i]);
    }
#pragma unroll
    for (int i = NL - 1; i >= 0; --i) {  // backward: L^H v = w
      float2 acc = w[i];
#pragma unroll
      for (int kk = i + 1; kk < NL; ++kk) {
        const float2 m = cmulc(G[tri(kk, i)], Hm[r][kk]);
        acc.x -= m.x;
        acc.y -= m.y;
      }
      Hm[r][i] = make_float2(acc.x * linv[i], acc.y * linv[i]);
    }
  }

  // 4. every data symbol of the subcarrier
  const int nd = g.n_dsym;
  for (int di = 0; di < nd; ++di) {
    const int s = g.dsym[di];
    const float2* __restrict__ yrow = rx + ((slot * g.n_symb + s) * g.n_sc + k) * NR;
    float2 y[NR];
#pragma unroll
    for (int r = 0; r < NR; ++r) y[r] = yrow[r];
    const int64_t o = ((slot * nd + di) * g.n_sc + k) * NL;
#pragma unroll
    for (int l = 0; l < NL; ++l) {
      float2 acc = make_float2(0.f, 0.f);
#pragma unroll
      for (int r = 0; r < NR; ++r) {
        const float2 m = cmul(Hm[r][l], y[r]);
        acc.x += m.x;
        acc.y += m.y;
      }
      x[o + l] = ok ? make_float2(acc.x * im[l], acc.y * im[l])
                    : make_float2(__builtin_nanf(""), __builtin_nanf(""));
      nv[o + l] = vo[l];
    }
  }
}

template <int NR, int NL>
hipError_t launch_rl(const Geom& g, const float2* rx, const float2* h, int h_res,
                     const float* nvar, float2* x, float* nv, hipStream_t s) {
  const int64_t total = (int64_t)g.n_slots * g.n_sc;
  const dim3 block(256), grid((unsigned)((total + 255) / 256));
  if (h_res == 0)
    hipLaunchKernelGGL((mmse_sc_kernel<NR, NL, 0>), grid, block, 0, s, g, rx, h, nvar, x, nv);
  else
    hipLaunchKernelGGL((mmse_sc_kernel<NR, NL, 1>), grid, block, 0, s, g, rx, h, nvar, x, nv);
  return hipGetLastError();
}

template <int NR>
hipError_t launch_r(const Geom& g, const float2* rx, const float2* h, int h_res,
                    const float* nvar, float2* x, float* nv, hipStream_t s) {
  switch (g.n_layers) {
    case 1: return launch_rl<NR, 1>(g, rx, h, h_res, nvar, x, nv, s);
    case 2: if constexpr (NR * 2 <= 64) return launch_rl<NR, 2>(g, rx, h, h_res, nvar, x, nv, s); break;
    case 3: if constexpr (NR * 3 <= 64) return launch_rl<NR, 3>(g, rx, h, h_res, nvar, x, nv, s); break;
    case 4: if constexpr (NR * 4 <= 64) return launch_rl<NR, 4>(g, rx, h, h_res, nvar, x, nv, s); break;
    case 5: if constexpr (NR * 5 <= 64) return launch_rl<NR, 5>(g, rx, h, h_res, nvar, x, nv, s); break;
    case 6: if constexpr (NR * 6 <= 64) return launch_rl<NR, 6>(g, rx, h, h_res, nvar, x, nv, s); break;
    case 7: if constexpr (NR * 7 <= 64) return launch_rl<NR, 7>(g, rx, h, h_res, nvar, x, nv, s); break;
    case 8: if constexpr (NR * 8 <= 64) return launch_rl<NR, 8>(g, rx, h, h_res, nvar, x, nv, s); break;
    default: break;
  }
  return hipErrorInvalidValue;
}

}  // namespace

bool mmse_sc_eligible(const Geom& g) {
  const int nr = g.n_rx, nl = g.n_layers;
  return g.n_occ == 1 && (nr == 1 || nr == 2 || nr == 4 || nr == 8) && nl <= 8 && nr * nl <= 64;
}

hipError_t launch_mmse_sc(const Geom& g, const float2* rx, const float2* h, int h_res,
                          const float* nvar, float2* x, float* nv, hipStream_t s) {
  switch (g.n_rx) {
    case 1: return launch_r<1>(g, rx, h, h_res, nvar, x, nv, s);
    case 2: return launch_r<2>(g, rx, h, h_res, nvar, x, nv, s);
    case 4: return launch_r<4>(g, rx, h, h_res, nvar, x, nv, s);
    case 8: return launch_r<8>(g, rx, h, h_res, nvar, x, nv, s);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace ranphy
