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
constexpr int kXcds = 8;

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
//   pivot row:     A[K][j]  <- A[K][j] / p
//   pivot column:  A[i][K]  <- -A[i][K] / p
//   pivot:         A[K][K]  <- 1 / p
//   elsewhere:     A[i][j]  <- A[i][j] - A[i][K] A[K][j] / p
template <int K>
__device__ __forceinline__ void gj_step(float (&ar)[4], float (&ai)[4], int q, int c, int nl,
                                        float tiny, bool& ok) {
  constexpr int KV = K & 3;
  constexpr int KQ = K >> 2;
  const float p = uniform_read(ar[KV], 16 * KQ + K);
  ok = ok && (K >= nl || p > tiny);  // padded layers carry an identity block
  const float pinv = __builtin_amdgcn_rcpf(p);
  // Row K at this lane's column c (held by lane (K/4, c), register K%4), scaled.
  const int src = 16 * KQ + c;
  const float rr = lane_read(ar[KV], src) * pinv;
  const float ri = lane_read(ai[KV], src) * pinv;
  const bool col_k = (c == K);
  const bool q_k = (q == KQ);
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    const float cr = row_bcast<K>(ar[v]);  // A[4q+v][K]
    const float ci = row_bcast<K>(ai[v]);
    float nr = fmaf(-cr, rr, fmaf(ci, ri, ar[v]));
    float ni = fmaf(-cr, ri, fmaf(-ci, rr, ai[v]));
    if (col_k) {
      nr = -cr * pinv;
      ni = -ci * pinv;
    }
    if (v == KV && q_k) {  // pivot row (4q + v == K only for v == K % 4)
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

template <int HRES, int NL>
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
  const int NR = g.n_rx, ND = g.n_dsym;

  // Blocks are dispatched round-robin over the 8 XCDs; give each XCD a contiguous run of
  // subcarriers so that its L2 reads every pilot of the run once.
  const int64_t total = (int64_t)g.n_slots * g.n_sc;
  const int64_t per_xcd = gridDim.x / kXcds;
  const int64_t blk = (int64_t)(blockIdx.x % kXcds) * per_xcd + blockIdx.x / kXcds;
  int64_t sid = blk * 4 + wave;
  const bool live = sid < total;
  if (!live) sid = total - 1;  // dead waves mirror the last subcarrier and store nothing
  const int64_t slot = sid / g.n_sc;
  const int k = (int)(sid % g.n_sc);
  const bool qv = 16 * q < NR;  // this lane group's antennas exist

  // ---- 1. channel in registers: lane (q, p = c), step s: antenna 16 q + s ----------------
  float hr[16], hi[16];
  if (c < NL && qv) {
    const int p = c;
    if (HRES == 0) {
      int j0, j1;
      float a;
      freq_rule(g, p, k, j0, j1, a);
      const float2* __restrict__ b0 = h + ((slot * g.n_pilot + j0) * NR + 16 * q) * NL + p;
      const float2* __restrict__ b1 = h + ((slot * g.n_pilot + j1) * NR + 16 * q) * NL + p;
#pragma unroll
      for (int s = 0; s < 16; ++s) {
        const float2 v0 = b0[s * NL];
        const float2 v1 = b1[s * NL];
        hr[s] = v0.x + a * (v1.x - v0.x);
        hi[s] = v0.y + a * (v1.y - v0.y);
      }
    } else {
      const float2* __restrict__ b0 = h + ((slot * g.n_sc + k) * NR + 16 * q) * NL + p;
#pragma unroll
      for (int s = 0; s < 16; ++s) {
        const float2 v0 = b0[s * NL];
        hr[s] = v0.x;
        hi[s] = v0.y;
      }
    }
  } else {
#pragma unroll
    for (int s = 0; s < 16; ++s) hr[s] = hi[s] = 0.f;
  }

  // ---- 2. received samples: lane (q, d = c), antennas 16 q .. 16 q + 15 (128 B) ----------
  float yr[16], yi[16];
  {
    const int d = c;
    // One occasion: data symbols are those before and after its T DMRS symbols.
    const int s = (d < g.sym0[0]) ? d : d + g.td;
    if (d < ND && qv) {
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
  // Z = H^H Y with three real products (conj(a) b, a = hr + j hi, b = yr + j yi):
  //   m1 = hr yr,  m2 = hi yi,  m3 = (hr - hi)(yr + yi);  Re = m1 + m2,  Im = m3 - m1 + m2.
  floatx4 acc_g = {0.f, 0.f, 0.f, 0.f}, acc_p = acc_g, acc_m1 = acc_g, acc_m2 = acc_g,
          acc_m3 = acc_g;
#pragma unroll
  for (int s = 0; s < 16; ++s) {
    acc_g = mfma(hr[s], hr[s], acc_g);
    acc_g = mfma(hi[s], hi[s], acc_g);
    acc_p = mfma(hr[s], hi[s], acc_p);
    acc_m1 = mfma(hr[s], yr[s], acc_m1);
    acc_m2 = mfma(hi[s], yi[s], acc_m2);
    acc_m3 = mfma(hr[s] - hi[s], yr[s] + yi[s], acc_m3);
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
  // Three real products again: Re = ar zr + ai zi,  Im = (ar - ai)(zr + zi) - ar zr + ai zi.
  floatx4 acc_n1 = {0.f, 0.f, 0.f, 0.f}, acc_n2 = acc_n1, acc_n3 = acc_n1;
#pragma unroll
  for (int s = 0; s < 4; ++s) {
    const float zr = acc_m1[s] + acc_m2[s];
    const float zi = acc_m3[s] - acc_m1[s] + acc_m2[s];
    acc_n1 = mfma(ar[s], zr, acc_n1);
    acc_n2 = mfma(ai[s], zi, acc_n2);
    acc_n3 = mfma(ar[s] - ai[s], zr + zi, acc_n3);
  }
  floatx4 acc_xr, acc_xi;
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    acc_xr[v] = acc_n1[v] + acc_n2[v];
    acc_xi[v] = acc_n3[v] - acc_n1[v] + acc_n2[v];
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
        const float im = __builtin_amdgcn_rcpf(1.f - sd);
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

template <int HRES, int NL>
void launch_one(const Geom& g, dim3 grid, const float2* rx, const float2* h, const float* nvar,
                float2* x, float* nv, hipStream_t s) {
  hipLaunchKernelGGL((mmse_mfma_kernel<HRES, NL>), grid, dim3(256), 0, s, g, rx, h, nvar, x, nv);
}

template <int HRES>
void launch_nl(const Geom& g, dim3 grid, const float2* rx, const float2* h, const float* nvar,
               float2* x, float* nv, hipStream_t s) {
  switch (g.n_layers) {
    case 5: launch_one<HRES, 5>(g, grid, rx, h, nvar, x, nv, s); break;
    case 6: launch_one<HRES, 6>(g, grid, rx, h, nvar, x, nv, s); break;
    case 7: launch_one<HRES, 7>(g, grid, rx, h, nvar, x, nv, s); break;
    case 8: launch_one<HRES, 8>(g, grid, rx, h, nvar, x, nv, s); break;
    case 9: launch_one<HRES, 9>(g, grid, rx, h, nvar, x, nv, s); break;
    case 10: launch_one<HRES, 10>(g, grid, rx, h, nvar, x, nv, s); break;
    case 11: launch_one<HRES, 11>(g, grid, rx, h, nvar, x, nv, s); break;
    case 12: launch_one<HRES, 12>(g, grid, rx, h, nvar, x, nv, s); break;
    case 13: launch_one<HRES, 13>(g, grid, rx, h, nvar, x, nv, s); break;
    case 14: launch_one<HRES, 14>(g, grid, rx, h, nvar, x, nv, s); break;
    case 15: launch_one<HRES, 15>(g, grid, rx, h, nvar, x, nv, s); break;
    default: launch_one<HRES, 16>(g, grid, rx, h, nvar, x, nv, s); break;
  }
}

}  // namespace

bool mmse_mfma_eligible(const Geom& g, const void* rx) {
  // 16-byte aligned received grid: each lane reads its antennas with 16-byte loads.
  return ((uintptr_t)rx & 15u) == 0 && g.n_occ == 1 && g.n_layers >= 5 && g.n_layers <= 16 &&
         g.n_rx % 16 == 0 && g.n_rx <= 64 && g.n_dsym <= 16;
}

hipError_t launch_mmse_mfma(const Geom& g, const float2* rx, const float2* h, int h_res,
                            const float* nvar, float2* x, float* nv, hipStream_t s) {
  const int64_t waves = (int64_t)g.n_slots * g.n_sc;
  const int64_t blocks = (waves + 3) / 4;
  const dim3 grid((unsigned)((blocks + kXcds - 1) / kXcds * kXcds));
  if (h_res == 0) launch_nl<0>(g, grid, rx, h, nvar, x, nv, s);
  else launch_nl<1>(g, grid, rx, h, nvar, x, nv, s);
  return hipGetLastError();
}

}  // namespace ranphy
