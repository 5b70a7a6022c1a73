// LMMSE detection on the matrix cores: one wavefront per subcarrier, for slots whose
// channel estimate is constant over the slot (one DMRS occasion), 5..16 layers and 16, 32,
// 48 or 64 receive antennas.
//
// Per subcarrier k (everything below is per wave; the 4 waves of a block take 4
// consecutive subcarriers):
//   1. H (Nr x Nl) by frequency interpolation of the pilot-resolution estimate (or read at
//      full resolution), held in registers in the MFMA operand layout;
//   2. Y (Nr x Nd): the received samples of all Nd <= 16 data symbols of subcarrier k;
//   3. on MFMA (v_mfma_f32_16x16x4f32, FP32 in, FP32 accumulate), contracting over the
//      receive antennas:  Re G = Hr^T Hr + Hi^T Hi,  P = Hr^T Hi (Im G = P - P^T),
//      Z = H^H Y  (all Nd data symbols as the 16 columns of one tile);
//   4. G + s2 I inverted in place by Gauss-Jordan elimination without pivoting (valid for a
//      Hermitian positive definite matrix: every pivot is a Schur-complement diagonal,
//      >= s2 > 0), in the MFMA accumulator layout, with ds_swizzle / ds_bpermute
//      broadcasts of the pivot column and row;
//   5. X_hat = G^-1 Z on MFMA: G^-1 is Hermitian, so the accumulator layout of G^-1 is,
//      after conjugation, exactly the A-operand layout, and Z's accumulator layout is the
//      B-operand layout -- no data movement between 4 and 5;
//   6. d = diag(G^-1), mu = 1 - s2 d, x = X_hat / mu, nv = s2 d / mu.
//
// The paper's detector (Sec. IV, Fig. 4) reduces the LMMSE inversion to LU elimination and
// forward/backward substitution; Gauss-Jordan elimination performs the same eliminations
// and both substitutions in one sweep over the matrix, which suits a 64-lane wave holding a
// 16 x 16 matrix as 4 values per lane.
//
// MFMA operand layouts (16x16x4, single block), lane l = 16 q + c:
//   A[i][kk] <- lane (i + 16 kk);  B[kk][j] <- lane (j + 16 kk);  D[i][j] -> lane (j + 16 (i/4)),
//   register i % 4.  The K index of step s is mapped to receive antenna 16 q + s, so that
//   each lane's 16 samples of one symbol are contiguous in memory.
#include <float.h>

#include "geom.h"

namespace ranphy {
namespace {

typedef float floatx4 __attribute__((ext_vector_type(4)));

constexpr float kPivotRel = 16.f * FLT_EPSILON;

__device__ __forceinline__ floatx4 mfma(float a, float b, floatx4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

// Value of lane (16 * (lane / 16) + src) within each row of 16 lanes.
template <int SRC>
__device__ __forceinline__ float row_bcast(float v) {
  constexpr int pattern = 0x10 | (SRC << 5);  // bit mode: and 0x10, or SRC
  return __int_as_float(__builtin_amdgcn_ds_swizzle(__float_as_int(v), pattern));
}

__device__ __forceinline__ float lane_read(float v, int src_lane) {
  return __int_as_float(__builtin_amdgcn_ds_bpermute(src_lane << 2, __float_as_int(v)));
}

__device__ __forceinline__ float uniform_read(float v, int lane) {
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), lane));
}

// One Gauss-Jordan step on pivot K.  Lane (q, c) holds A[4q+v][c] in (ar[v], ai[v]).
template <int K>
__device__ __forceinline__ void gj_step(float (&ar)[4], float (&ai)[4], int q, int c, int nl,
                                        float tiny, bool& ok) {
  constexpr int KV = K & 3;
  constexpr int KL = 16 * (K >> 2) + K;
  const float p = uniform_read(ar[KV], KL);
  ok = ok && (K >= nl || p > tiny);  // padded layers carry an identity block
  const float pinv = 1.f / p;
  // Row K at this lane's column c (held by lane (K/4, c), register K%4), scaled.
  const float rr = lane_read(ar[KV], 16 * (K >> 2) + c) * pinv;
  const float ri = lane_read(ai[KV], 16 * (K >> 2) + c) * pinv;
  const bool col_k = (c == K);
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    const float cr = row_bcast<K>(ar[v]);  // A[4q+v][K]
    const float ci = row_bcast<K>(ai[v]);
    const bool row_k = (4 * q + v == K);
    // Generic entry: A - A[i][K] A[K][j] / p.
    float nr = ar[v] - (cr * rr - ci * ri);
    float ni = ai[v] - (cr * ri + ci * rr);
    if (col_k) {
      nr = -cr * pinv;
      ni = -ci * pinv;
    }
    if (row_k) {
      nr = col_k ? pinv : rr;
      ni = col_k ? 0.f : ri;
    }
    ar[v] = nr;
    ai[v] = ni;
  }
}

template <int K>
__device__ __forceinline__ void gj_all(float (&ar)[4], float (&ai)[4], int q, int c, int nl,
                                       float tiny, bool& ok) {
  if constexpr (K < 16) {
    gj_step<K>(ar, ai, q, c, nl, tiny, ok);
    gj_all<K + 1>(ar, ai, q, c, nl, tiny, ok);
  }
}

template <int HRES>
__global__ void __launch_bounds__(256) mmse_mfma_kernel(Geom g, const float2* __restrict__ rx,
                                                        const float2* __restrict__ h,
                                                        const float* __restrict__ nvar,
                                                        float2* __restrict__ x,
                                                        float* __restrict__ nv) {
  __shared__ float lds_t[4][16 * 17];
  const int wave = threadIdx.x >> 6;
  const int lane = threadIdx.x & 63;
  const int q = lane >> 4;  // K group / accumulator row group
  const int c = lane & 15;  // layer (A/B operands), column (accumulators)
  const int NR = g.n_rx, NL = g.n_layers, ND = g.n_dsym;

  const int64_t total = (int64_t)g.n_slots * g.n_sc;
  int64_t sid = (int64_t)blockIdx.x * 4 + wave;
  const bool live = sid < total;
  if (!live) sid = total - 1;  // dead waves mirror the last subcarrier and store nothing
  const int64_t slot = sid / g.n_sc;
  const int k = (int)(sid % g.n_sc);

  // ---- 1. channel in registers: lane (q, p = c), step s: antenna 16 q + s ----------------
  float hr[16], hi[16];
  {
    const int p = c;
    const bool pv = p < NL;
    const float2* __restrict__ b0;
    const float2* __restrict__ b1;
    float a = 0.f;
    if (HRES == 0) {
      int j0 = 0, j1 = 0;
      if (pv) freq_rule(g, p, k, j0, j1, a);
      const int64_t base = slot * g.n_pilot;  // one occasion
      b0 = h + (base + j0) * NR * NL;
      b1 = h + (base + j1) * NR * NL;
    } else {
      b0 = h + (slot * g.n_sc + k) * NR * NL;
      b1 = b0;
    }
#pragma unroll
    for (int s = 0; s < 16; ++s) {
      const int r = 16 * q + s;
      float vr = 0.f, vi = 0.f;
      if (pv && r < NR) {
        const float2 v0 = b0[r * NL + p];
        if (HRES == 0) {
          const float2 v1 = b1[r * NL + p];
          vr = v0.x + a * (v1.x - v0.x);
          vi = v0.y + a * (v1.y - v0.y);
        } else {
          vr = v0.x;
          vi = v0.y;
        }
      }
      hr[s] = vr;
      hi[s] = vi;
    }
  }

  // ---- 2. received samples: lane (q, d = c), antennas 16 q .. 16 q + 15 (128 B) ----------
  float yr[16], yi[16];
  {
    const int d = c;
    // One occasion: data symbols are those before and after its T DMRS symbols.
    const int s = (d < g.sym0[0]) ? d : d + g.td;
    if (d < ND && 16 * q < NR) {
      const float4* __restrict__ src = reinterpret_cast<const float4*>(
          rx + ((slot * g.n_symb + s) * g.n_sc + k) * NR + 16 * q);
#pragma unroll
      for (int i = 0; i < 8; ++i) {
        const float4 v = src[i];
        yr[2 * i] = v.x;
        yi[2 * i] = v.y;
        yr[2 * i + 1] = v.z;
        yi[2 * i + 1] = v.w;
      }
    } else {
#pragma unroll
      for (int i = 0; i < 16; ++i) yr[i] = yi[i] = 0.f;
    }
  }

  // ---- 3. Gram and matched filter on the matrix cores -------------------------------------
  floatx4 acc_g = {0.f, 0.f, 0.f, 0.f}, acc_p = acc_g, acc_zr = acc_g, acc_za = acc_g,
          acc_zb = acc_g;
#pragma unroll
  for (int s = 0; s < 16; ++s) {
    acc_g = mfma(hr[s], hr[s], acc_g);
    acc_g = mfma(hi[s], hi[s], acc_g);
    acc_p = mfma(hr[s], hi[s], acc_p);
    acc_zr = mfma(hr[s], yr[s], acc_zr);
    acc_zr = mfma(hi[s], yi[s], acc_zr);
    acc_za = mfma(hr[s], yi[s], acc_za);
    acc_zb = mfma(hi[s], yr[s], acc_zb);
  }

  // ---- 4. G = Re + j (P - P^T) + s2 I, padded layers -> identity; invert in place ---------
  float* __restrict__ tp = lds_t[wave];
#pragma unroll
  for (int v = 0; v < 4; ++v) tp[(4 * q + v) * 17 + c] = acc_p[v];
  __syncthreads();
  const float s2 = nvar[slot];
  float ar[4], ai[4];
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    const int i = 4 * q + v;
    const bool in = (i < NL) && (c < NL);
    ar[v] = in ? acc_g[v] + ((i == c) ? s2 : 0.f) : ((i == c) ? 1.f : 0.f);
    ai[v] = in ? acc_p[v] - tp[c * 17 + i] : 0.f;
  }
  // Pivot threshold relative to the largest diagonal entry.
  float dmax = 0.f;
#pragma unroll
  for (int v = 0; v < 4; ++v) dmax = fmaxf(dmax, (4 * q + v == c) ? ar[v] : 0.f);
  dmax = fmaxf(dmax, __shfl_xor(dmax, 1));
  dmax = fmaxf(dmax, __shfl_xor(dmax, 2));
  dmax = fmaxf(dmax, __shfl_xor(dmax, 4));
  dmax = fmaxf(dmax, __shfl_xor(dmax, 8));
  dmax = fmaxf(dmax, __shfl_xor(dmax, 16));
  dmax = fmaxf(dmax, __shfl_xor(dmax, 32));
  const float tiny = kPivotRel * uniform_read(dmax, 0);
  bool ok = true;
  gj_all<0>(ar, ai, q, c, NL, tiny, ok);

  // ---- 5. X_hat = G^-1 Z on the matrix cores ---------------------------------------------
  // A[i = c][m = 4q + s] = G^-1[c][4q+s] = conj(G^-1[4q+s][c]) = (ar[s], -ai[s]);
  // B[m = 4q + s][d = c] = Z[4q+s][c].
  floatx4 acc_xr = {0.f, 0.f, 0.f, 0.f}, acc_xi = acc_xr;
#pragma unroll
  for (int s = 0; s < 4; ++s) {
    const float zr = acc_zr[s];
    const float zi = acc_za[s] - acc_zb[s];
    acc_xr = mfma(ar[s], zr, acc_xr);
    acc_xr = mfma(ai[s], zi, acc_xr);
    acc_xi = mfma(ar[s], zi, acc_xi);
    acc_xi = mfma(-ai[s], zr, acc_xi);
  }

  // ---- 6. unbias and store: lane (q, d = c) holds layers 4q .. 4q+3 of data symbol d ------
  float dl[4];
#pragma unroll
  for (int v = 0; v < 4; ++v) dl[v] = lane_read(ar[v], 16 * q + 4 * q + v);  // G^-1[4q+v][4q+v]
  const int d = c;
  if (live && d < ND) {
    const int64_t o = ((slot * ND + d) * g.n_sc + k) * NL;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int l = 4 * q + v;
      if (l < NL) {
        const float sd = s2 * dl[v];
        const float im = 1.f / (1.f - sd);
        if (ok) {
          x[o + l] = make_float2(acc_xr[v] * im, acc_xi[v] * im);
          nv[o + l] = sd * im;
        } else {
          x[o + l] = make_float2(__builtin_nanf(""), __builtin_nanf(""));
          nv[o + l] = __builtin_inff();
        }
      }
    }
  }
}

}  // namespace

bool mmse_mfma_eligible(const Geom& g, const void* rx) {
  // 16-byte aligned received grid: each lane reads its antennas with 16-byte loads.
  return ((uintptr_t)rx & 15u) == 0 && g.n_occ == 1 && g.n_layers >= 5 && g.n_layers <= 16 && g.n_rx % 16 == 0 &&
         g.n_rx <= 64 && g.n_dsym <= 16;
}

hipError_t launch_mmse_mfma(const Geom& g, const float2* rx, const float2* h, int h_res,
                            const float* nvar, float2* x, float* nv, hipStream_t s) {
  const int64_t waves = (int64_t)g.n_slots * g.n_sc;
  const dim3 block(256), grid((unsigned)((waves + 3) / 4));
  if (h_res == 0)
    hipLaunchKernelGGL(mmse_mfma_kernel<0>, grid, block, 0, s, g, rx, h, nvar, x, nv);
  else
    hipLaunchKernelGGL(mmse_mfma_kernel<1>, grid, block, 0, s, g, rx, h, nvar, x, nv);
  return hipGetLastError();
}

}  // namespace ranphy
