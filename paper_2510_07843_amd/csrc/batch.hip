// Many UEs of uneven allocations in one persistent launch: LS estimation, interpolation,
// LMMSE detection and max-log demapping for every UE of a batch.  The paper names divergence
// and scheduling overhead as the weak points of SIMT processing for PHY work (Sec. V); here
// the launch does not depend on the batch's composition and the work is dealt out in
// homogeneous pieces.
//
// A plan (built on the host, resident in device memory) holds one record per UE (its
// geometry and buffers) and a list of work items, each a tile of consecutive subcarriers of
// one UE, sorted so that items of one class (layers, modulation, antennas) are adjacent and
// the heaviest come first.  Every block of the persistent grid takes the next item from an
// atomic counter until the list is exhausted, so the grid is as large as the chip holds and
// no more; a one-thread kernel clears the counter before each run (both capture into a HIP
// graph).  An item is processed by one block without depending on any other:
//   1. the LS estimate (Sec. III-B: channel estimation) of every pilot the tile's
//      subcarriers interpolate from, per occasion, into LDS;
//   2. with one DMRS occasion (the channel held over the slot): each subcarrier's Gram
//      G = H^H H + s2 I, one (subcarrier, entry) per thread, then its Cholesky factor
//      (Sec. IV, Fig. 4), reciprocal diagonal and d = diag(G^-1), one subcarrier per
//      thread, staged in LDS; per resource element (all data symbols) the matched filter
//      streamed over the receive antennas, forward / backward substitution with the staged
//      factor, unbiasing, and the max-log LLRs written to the UE's output;
//   2'. with several occasions (a time-varying estimate): per resource element the
//      interpolation in frequency and time, Gram and matched filter, factorisation,
//      substitution, unbiasing and LLRs.
// Layers 1..8 (a template parameter: one branch per item, uniform over the block),
// antennas 1..64, every modulation and DMRS configuration of the library.
#include <float.h>

#include "batch.h"
#include "llr_math.h"

namespace ranphy {

namespace {

constexpr float kPivotRel = 16.f * FLT_EPSILON;

__host__ __device__ constexpr int tri(int i, int j) { return i * (i + 1) / 2 + j; }

// LLRs of one layer of one RE (compile-time Qm: the values stay in registers).
template <int QM>
__device__ __forceinline__ void demap_store(float* __restrict__ dst, float2 xo, float vo) {
  float out[QM];
  llr_one<QM>(xo, vo, out);
#pragma unroll
  for (int b = 0; b < QM; b += 2)
    *reinterpret_cast<float2*>(dst + b) = make_float2(out[b], out[b + 1]);
}

template <int NL>
__device__ void detect_tile(const BatchUe& u, const Geom& g, int k0, int nk, int jlo, int nj,
                            const float2* __restrict__ lds) {
  const int NR = g.n_rx, ND = g.n_dsym;
  const float s2 = *u.nv;
  for (int e = threadIdx.x; e < nk * ND; e += blockDim.x) {
    const int d = e / nk;
    const int k = k0 + (e - d * nk);
    const int s = g.dsym[d];
    const int o0 = g.t_o0[d], o1 = g.t_o1[d];
    const float w = g.t_w[d];
    int r0[NL], r1[NL];
    float a[NL];
#pragma unroll
    for (int p = 0; p < NL; ++p) {
      int j0, j1;
      freq_rule(g, p, k, j0, j1, a[p]);
      r0[p] = j0 - jlo;
      r1[p] = j1 - jlo;
    }
    constexpr int NP = NL * (NL + 1) / 2;
    float2 G[NP], z[NL];
#pragma unroll
    for (int i = 0; i < NP; ++i) G[i] = make_float2(0.f, 0.f);
#pragma unroll
    for (int i = 0; i < NL; ++i) z[i] = make_float2(0.f, 0.f);
    const float2* __restrict__ yrow = u.rx + ((int64_t)s * g.n_sc + k) * NR;
    for (int r = 0; r < NR; ++r) {
      float2 hr[NL];
#pragma unroll
      for (int p = 0; p < NL; ++p) {
        const float2* b = lds + r * NL + p;
        const float2 v0 = b[(o0 * nj + r0[p]) * NR * NL], v1 = b[(o0 * nj + r1[p]) * NR * NL];
        float2 v = make_float2(v0.x + a[p] * (v1.x - v0.x), v0.y + a[p] * (v1.y - v0.y));
        if (o1 != o0) {
          const float2 u0 = b[(o1 * nj + r0[p]) * NR * NL], u1 = b[(o1 * nj + r1[p]) * NR * NL];
          const float2 vv = make_float2(u0.x + a[p] * (u1.x - u0.x), u0.y + a[p] * (u1.y - u0.y));
          v = make_float2(v.x + w * (vv.x - v.x), v.y + w * (vv.y - v.y));
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
    float gd[NL];
#pragma unroll
    for (int i = 0; i < NL; ++i) {
      G[tri(i, i)].x += s2;
      gd[i] = G[tri(i, i)].x;
    }
    bool ok = true;
    float linv[NL];
#pragma unroll
    for (int j = 0; j < NL; ++j) {  // Cholesky G = L L^H in place
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
          const float2 m = cmulc(G[tri(j, kk)], G[tri(i, kk)]);
          acc.x -= m.x;
          acc.y -= m.y;
        }
        G[tri(i, j)] = make_float2(acc.x * inv, acc.y * inv);
      }
    }
    float2 wv[NL], xh[NL];
#pragma unroll
    for (int i = 0; i < NL; ++i) {  // L w = z
      float2 acc = z[i];
#pragma unroll
      for (int kk = 0; kk < i; ++kk) {
        const float2 m = cmul(G[tri(i, kk)], wv[kk]);
        acc.x -= m.x;
        acc.y -= m.y;
      }
      wv[i] = make_float2(acc.x * linv[i], acc.y * linv[i]);
    }
#pragma unroll
    for (int i = NL - 1; i >= 0; --i) {  // L^H x = w
      float2 acc = wv[i];
#pragma unroll
      for (int kk = i + 1; kk < NL; ++kk) {
        const float2 m = cmulc(G[tri(kk, i)], xh[kk]);
        acc.x -= m.x;
        acc.y -= m.y;
      }
      xh[i] = make_float2(acc.x * linv[i], acc.y * linv[i]);
    }
    float* __restrict__ dst = u.llr + (((int64_t)d * g.n_sc + k) * NL) * g.qm;
#pragma unroll
    for (int l = 0; l < NL; ++l) {  // d_l = || L^-1 e_l ||^2, unbias, demap
      float2 uu[NL];
      uu[l] = make_float2(linv[l], 0.f);
      float acc2 = linv[l] * linv[l];
#pragma unroll
      for (int i = l + 1; i < NL; ++i) {
        float2 acc = make_float2(0.f, 0.f);
#pragma unroll
        for (int kk = l; kk < i; ++kk) {
          const float2 m = cmul(G[tri(i, kk)], uu[kk]);
          acc.x -= m.x;
          acc.y -= m.y;
        }
        uu[i] = make_float2(acc.x * linv[i], acc.y * linv[i]);
        acc2 += uu[i].x * uu[i].x + uu[i].y * uu[i].y;
      }
      const float sd = s2 * acc2;
      const float im = 1.f / (1.f - sd);
      const float2 xo = ok ? make_float2(xh[l].x * im, xh[l].y * im)
                           : make_float2(__builtin_nanf(""), __builtin_nanf(""));
      const float vo = ok ? sd * im : __builtin_inff();
      switch (g.qm) {  // uniform over the item
        case 2: demap_store<2>(dst + l * 2, xo, vo); break;
        case 4: demap_store<4>(dst + l * 4, xo, vo); break;
        case 6: demap_store<6>(dst + l * 6, xo, vo); break;
        default: demap_store<8>(dst + l * 8, xo, vo); break;
      }
    }
  }
}

// Channel value of port p at antenna r for the subcarrier whose interpolation rows and
// weight are (r0, r1, a), one occasion: rows[j][r][p].
__device__ __forceinline__ float2 row_interp(const float2* __restrict__ rows, int NR, int NL,
                                             int r0, int r1, float a, int r, int p) {
  const float2 v0 = rows[(r0 * NR + r) * NL + p], v1 = rows[(r1 * NR + r) * NL + p];
  return make_float2(v0.x + a * (v1.x - v0.x), v0.y + a * (v1.y - v0.y));
}

// One occasion: Gram, Cholesky factor, reciprocal diagonal and d = diag(G^-1) of each of the
// tile's subcarriers into LDS.  fac[kk][tri(i, j)] holds L, aux[kk][0..NL) 1 / L_ii,
// aux[kk][NL..2NL) d, aux[kk][2NL] 1 where the factorisation succeeded, else 0.
template <int NL>
__device__ void factor_tile(const BatchUe& u, const Geom& g, int k0, int nk, int jlo,
                            const float2* __restrict__ rows, float2* __restrict__ fac,
                            float* __restrict__ aux) {
  constexpr int NP = NL * (NL + 1) / 2;
  const int NR = g.n_rx;
  for (int f = threadIdx.x; f < nk * NP; f += blockDim.x) {
    const int kk = f / NP;
    const int e = f - kk * NP;
    int i = 0;
    while ((i + 1) * (i + 2) / 2 <= e) ++i;
    const int j = e - i * (i + 1) / 2;
    const int k = k0 + kk;
    int ri0, ri1, rj0, rj1;
    float ai, aj;
    freq_rule(g, i, k, ri0, ri1, ai);
    freq_rule(g, j, k, rj0, rj1, aj);
    ri0 -= jlo; ri1 -= jlo; rj0 -= jlo; rj1 -= jlo;
    float2 acc = make_float2(0.f, 0.f);
    for (int r = 0; r < NR; ++r) {  // the order of the per-RE path's sums
      const float2 hi = row_interp(rows, NR, NL, ri0, ri1, ai, r, i);
      const float2 hj = row_interp(rows, NR, NL, rj0, rj1, aj, r, j);
      const float2 gg = cmulc(hi, hj);
      acc.x += gg.x;
      acc.y += gg.y;
    }
    fac[kk * kBatchFactNP + e] = acc;
  }
  __syncthreads();
  const float s2 = *u.nv;
  for (int kk = threadIdx.x; kk < nk; kk += blockDim.x) {
    float2 G[NP];
#pragma unroll
    for (int e = 0; e < NP; ++e) G[e] = fac[kk * kBatchFactNP + e];
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
      for (int kq = 0; kq < j; ++kq) dj -= G[tri(j, kq)].x * G[tri(j, kq)].x + G[tri(j, kq)].y * G[tri(j, kq)].y;
      ok = ok && (dj > kPivotRel * gd[j]);
      const float ljj = sqrtf(fmaxf(dj, FLT_MIN));
      const float inv = 1.f / ljj;
      G[tri(j, j)] = make_float2(ljj, 0.f);
      linv[j] = inv;
#pragma unroll
      for (int i = j + 1; i < NL; ++i) {
        float2 acc = G[tri(i, j)];
#pragma unroll
        for (int kq = 0; kq < j; ++kq) {
          const float2 m = cmulc(G[tri(j, kq)], G[tri(i, kq)]);
          acc.x -= m.x;
          acc.y -= m.y;
        }
        G[tri(i, j)] = make_float2(acc.x * inv, acc.y * inv);
      }
    }
    float* ax = aux + kk * (2 * kBatchMaxLayers + 1);
#pragma unroll
    for (int l = 0; l < NL; ++l) {  // d_l = || L^-1 e_l ||^2
      float2 uu[NL];
      uu[l] = make_float2(linv[l], 0.f);
      float acc2 = linv[l] * linv[l];
#pragma unroll
      for (int i = l + 1; i < NL; ++i) {
        float2 acc = make_float2(0.f, 0.f);
#pragma unroll
        for (int kq = l; kq < i; ++kq) {
          const float2 m = cmul(G[tri(i, kq)], uu[kq]);
          acc.x -= m.x;
          acc.y -= m.y;
        }
        uu[i] = make_float2(acc.x * linv[i], acc.y * linv[i]);
        acc2 += uu[i].x * uu[i].x + uu[i].y * uu[i].y;
      }
      ax[l] = linv[l];
      ax[NL + l] = acc2;
    }
    ax[2 * NL] = ok ? 1.f : 0.f;
#pragma unroll
    for (int e = 0; e < NP; ++e) fac[kk * kBatchFactNP + e] = G[e];
  }
  __syncthreads();
}

// One occasion, per resource element with the staged factor: matched filter, substitutions,
// unbiasing, LLRs.
template <int NL>
__device__ void detect_tile_fact(const BatchUe& u, const Geom& g, int k0, int nk, int jlo,
                                 const float2* __restrict__ rows,
                                 const float2* __restrict__ fac, const float* __restrict__ aux) {
  constexpr int NP = NL * (NL + 1) / 2;
  const int NR = g.n_rx, ND = g.n_dsym;
  const float s2 = *u.nv;
  for (int e = threadIdx.x; e < nk * ND; e += blockDim.x) {
    const int d = e / nk;
    const int kk = e - d * nk;
    const int k = k0 + kk;
    int r0[NL], r1[NL];
    float a[NL];
#pragma unroll
    for (int p = 0; p < NL; ++p) {
      int j0, j1;
      freq_rule(g, p, k, j0, j1, a[p]);
      r0[p] = j0 - jlo;
      r1[p] = j1 - jlo;
    }
    float2 z[NL];
#pragma unroll
    for (int i = 0; i < NL; ++i) z[i] = make_float2(0.f, 0.f);
    const float2* __restrict__ yrow = u.rx + ((int64_t)g.dsym[d] * g.n_sc + k) * NR;
    for (int r = 0; r < NR; ++r) {
      const float2 y = yrow[r];
#pragma unroll
      for (int i = 0; i < NL; ++i) {
        const float2 m = cmulc(row_interp(rows, NR, NL, r0[i], r1[i], a[i], r, i), y);
        z[i].x += m.x;
        z[i].y += m.y;
      }
    }
    const float2* L = fac + kk * kBatchFactNP;
    const float* ax = aux + kk * (2 * kBatchMaxLayers + 1);
    const bool ok = ax[2 * NL] != 0.f;
    float2 wv[NL], xh[NL];
#pragma unroll
    for (int i = 0; i < NL; ++i) {  // L w = z
      float2 acc = z[i];
#pragma unroll
      for (int kq = 0; kq < i; ++kq) {
        const float2 m = cmul(L[tri(i, kq)], wv[kq]);
        acc.x -= m.x;
        acc.y -= m.y;
      }
      wv[i] = make_float2(acc.x * ax[i], acc.y * ax[i]);
    }
#pragma unroll
    for (int i = NL - 1; i >= 0; --i) {  // L^H x = w
      float2 acc = wv[i];
#pragma unroll
      for (int kq = i + 1; kq < NL; ++kq) {
        const float2 m = cmulc(L[tri(kq, i)], xh[kq]);
        acc.x -= m.x;
        acc.y -= m.y;
      }
      xh[i] = make_float2(acc.x * ax[i], acc.y * ax[i]);
    }
    float* __restrict__ dst = u.llr + (((int64_t)d * g.n_sc + k) * NL) * g.qm;
#pragma unroll
    for (int l = 0; l < NL; ++l) {
      const float sd = s2 * ax[NL + l];
      const float im = 1.f / (1.f - sd);
      const float2 xo = ok ? make_float2(xh[l].x * im, xh[l].y * im)
                           : make_float2(__builtin_nanf(""), __builtin_nanf(""));
      const float vo = ok ? sd * im : __builtin_inff();
      switch (g.qm) {
        case 2: demap_store<2>(dst + l * 2, xo, vo); break;
        case 4: demap_store<4>(dst + l * 4, xo, vo); break;
        case 6: demap_store<6>(dst + l * 6, xo, vo); break;
        default: demap_store<8>(dst + l * 8, xo, vo); break;
      }
    }
  }
}

template <int NL>
__device__ void process_tile(const BatchUe& u, const Geom& g, int k0, int nk, int jlo, int nj,
                             const float2* rows, float2* fac, float* aux) {
  if (g.n_occ == 1) {
    factor_tile<NL>(u, g, k0, nk, jlo, rows, fac, aux);
    detect_tile_fact<NL>(u, g, k0, nk, jlo, rows, fac, aux);
  } else {
    detect_tile<NL>(u, g, k0, nk, jlo, nj, rows);
  }
}

// The LS estimate (Sec. III-B) of every pilot the tile k0 .. k0 + nk - 1 interpolates from,
// every occasion, into rows[o][j - jlo][r][p]; returns jlo and the pilot count nj.  Ends with
// a barrier.
__device__ __forceinline__ void stage_pilots(const BatchUe& u, const Geom& g, int k0, int nk,
                             float2* __restrict__ rows, int& jlo, int& nj) {
  const int C = g.comb, T = g.td, NR = g.n_rx, NL = g.n_layers, J = g.n_pilot;
  // pilot range of the tile: a port's pilot indices do not decrease with the subcarrier
  int lo = J, hi = 0;
  for (int p = 0; p < NL; ++p) {
    int j0, j1;
    float a;
    freq_rule(g, p, k0, j0, j1, a);
    lo = min(lo, j0);
    freq_rule(g, p, k0 + nk - 1, j0, j1, a);
    hi = max(hi, j1);
  }
  jlo = lo;
  nj = hi - lo + 1;
  const int n_ls = g.n_occ * nj * NR * NL;
  const float inv_t = 1.f / (float)T;
  for (int f = threadIdx.x; f < n_ls; f += blockDim.x) {
    const int p = f % NL;
    const int r = (f / NL) % NR;
    const int jj = (f / (NL * NR)) % nj;
    const int o = f / (NL * NR * nj);
    const int j = jlo + jj;
    const int k = C * j + (p & (C - 1));
    float2 acc = make_float2(0.f, 0.f);
    if (k < g.n_sc) {
      for (int t = 0; t < T; ++t) {
        const float2 y = u.rx[((int64_t)(g.sym0[o] + t) * g.n_sc + k) * NR + r];
        const float2 q = u.pil[(((int64_t)o * T + t) * J + j) * NL + p];
        const float2 m = cmulc(q, y);  // y conj(q)
        acc.x += m.x;
        acc.y += m.y;
      }
    }
    rows[f] = make_float2(acc.x * inv_t, acc.y * inv_t);
  }
  __syncthreads();
}

__device__ __forceinline__ void process_any(const BatchUe& u, const Geom& g, int k0, int nk, int jlo, int nj,
                            const float2* rows, float2* fac, float* aux) {
  switch (g.n_layers) {  // uniform over the block
    case 1: process_tile<1>(u, g, k0, nk, jlo, nj, rows, fac, aux); break;
    case 2: process_tile<2>(u, g, k0, nk, jlo, nj, rows, fac, aux); break;
    case 3: process_tile<3>(u, g, k0, nk, jlo, nj, rows, fac, aux); break;
    case 4: process_tile<4>(u, g, k0, nk, jlo, nj, rows, fac, aux); break;
    case 5: process_tile<5>(u, g, k0, nk, jlo, nj, rows, fac, aux); break;
    case 6: process_tile<6>(u, g, k0, nk, jlo, nj, rows, fac, aux); break;
    case 7: process_tile<7>(u, g, k0, nk, jlo, nj, rows, fac, aux); break;
    default: process_tile<8>(u, g, k0, nk, jlo, nj, rows, fac, aux); break;
  }
}

__global__ void batch_reset_kernel(BatchHdr* __restrict__ hdr) {
  if (threadIdx.x == 0 && blockIdx.x == 0) hdr->head = 0u;
}

__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(3, 8))) batch_kernel(
    char* __restrict__ plan) {
  __shared__ float2 lds[kBatchLds];
  __shared__ float2 fac[kBatchFactSc * kBatchFactNP];
  __shared__ float aux[kBatchFactSc * (2 * kBatchMaxLayers + 1)];
  __shared__ int s_item;
  BatchHdr* hdr = reinterpret_cast<BatchHdr*>(plan);
  const BatchUe* ues = reinterpret_cast<const BatchUe*>(plan + kBatchUeOff);
  const int n_items = hdr->n_items;
  const BatchItem* items = reinterpret_cast<const BatchItem*>(plan + hdr->items_off);
  for (;;) {
    if (threadIdx.x == 0) s_item = (int)atomicAdd(&hdr->head, 1u);
    __syncthreads();
    const int it = s_item;
    __syncthreads();  // every thread has read s_item before it is overwritten
    if (it >= n_items) break;  // uniform over the block: every wave leaves the loop here
    const BatchItem item = items[it];
    const BatchUe& u = ues[item.ue];
    const Geom& g = u.g;  // read in place (a private copy indexed at run time would spill)
    int jlo, nj;
    stage_pilots(u, g, item.k0, item.nk, lds, jlo, nj);
    process_any(u, g, item.k0, item.nk, jlo, nj, lds, fac, aux);
    __syncthreads();  // LDS is reused by the next item
  }
}

// The whole chain for a batch of slots of one shape (up to 8 layers) in one launch: block
// (slot, tile of nk subcarriers) stages the tile's pilot estimates and detects and demaps its
// resource elements, as a work item of the multi-UE launch does.
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(3, 8)))
receive_kernel(Geom g, const float2* __restrict__ rx, const float2* __restrict__ pil,
               const float* __restrict__ nvar, float* __restrict__ llr, int nk) {
  __shared__ float2 lds[kBatchLds];
  __shared__ float2 fac[kBatchFactSc * kBatchFactNP];
  __shared__ float aux[kBatchFactSc * (2 * kBatchMaxLayers + 1)];
  const int ntiles = (g.n_sc + nk - 1) / nk;
  const int slot = blockIdx.x / ntiles;
  const int k0 = (blockIdx.x - slot * ntiles) * nk;
  BatchUe u;
  u.g = g;
  u.rx = rx + (int64_t)slot * g.n_symb * g.n_sc * g.n_rx;
  u.pil = pil + (int64_t)slot * g.n_occ * g.td * g.n_pilot * g.n_layers;
  u.nv = nvar + slot;
  u.llr = llr + (int64_t)slot * g.n_dsym * g.n_sc * g.n_layers * g.qm;
  const int n = min(nk, g.n_sc - k0);
  int jlo, nj;
  stage_pilots(u, g, k0, n, lds, jlo, nj);
  process_any(u, g, k0, n, jlo, nj, lds, fac, aux);
}

}  // namespace

// Tile width of the one-launch chain: about tile_re resource elements, at most kBatchFactSc
// subcarriers, and pilot rows that fit the block's LDS for every tile.
int receive_tile(const Geom& g, int tile_re) {
  int nk = tile_re / g.n_dsym;
  nk = nk < 1 ? 1 : (nk > kBatchFactSc ? kBatchFactSc : nk);
  const int per = g.n_rx * g.n_layers;
  for (;;) {
    int worst = 0;
    for (int k0 = 0; k0 < g.n_sc; k0 += nk) {
      const int n = g.n_sc - k0 < nk ? g.n_sc - k0 : nk;
      const int r = batch_tile_rows(g, k0, n);
      worst = r > worst ? r : worst;
    }
    if (worst * per <= kBatchLds || nk == 1) return worst * per <= kBatchLds ? nk : 0;
    nk = (nk + 1) / 2;
  }
}

hipError_t launch_receive(const Geom& g, const float2* rx, const float2* pil, const float* nvar,
                          float* llr, int nk, hipStream_t s) {
  const int64_t ntiles = (g.n_sc + nk - 1) / nk;
  hipLaunchKernelGGL(receive_kernel, dim3((unsigned)(g.n_slots * ntiles)), dim3(256), 0, s, g,
                     rx, pil, nvar, llr, nk);
  return hipGetLastError();
}

// Pilot rows a tile of nk subcarriers starting at k0 needs (exact, by the interpolation rule).
int batch_tile_rows(const Geom& g, int k0, int nk) {
  int jlo = g.n_pilot, jhi = 0;
  for (int p = 0; p < g.n_layers; ++p) {
    const int c = p & (g.comb - 1);
    const int jp = (g.n_sc - c + g.comb - 1) / g.comb;
    const int last = c + g.comb * (jp - 1);
    auto rule = [&](int k, int& j0, int& j1) {
      if (k <= c) j0 = j1 = 0;
      else if (k >= last) j0 = j1 = jp - 1;
      else { j0 = (k - c) / g.comb; j1 = j0 + 1; }
    };
    int j0, j1;
    rule(k0, j0, j1);
    jlo = j0 < jlo ? j0 : jlo;
    rule(k0 + nk - 1, j0, j1);
    jhi = j1 > jhi ? j1 : jhi;
  }
  return g.n_occ * (jhi - jlo + 1);
}

hipError_t launch_batch(void* plan, int blocks, hipStream_t s) {
  hipLaunchKernelGGL(batch_reset_kernel, dim3(1), dim3(64), 0, s, reinterpret_cast<BatchHdr*>(plan));
  hipLaunchKernelGGL(batch_kernel, dim3(blocks), dim3(256), 0, s, static_cast<char*>(plan));
  return hipGetLastError();
}

}  // namespace ranphy
