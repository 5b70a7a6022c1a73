// Tiles of the whole receive chain -- LS estimation, interpolation, LMMSE detection and
// max-log demapping -- each processed by one block without depending on any other, and the
// two launches built from them:
//   * receive_kernel (ranphy_receive): one launch over the slots of one shape, block = (slot,
//     tile of consecutive subcarriers), in three compiled forms by layer count and DMRS
//     occasions (the LDS and registers each needs set how many blocks share a CU);
//   * batch_kernel (ranphy_batch_*): many UEs of uneven allocations in one persistent
//     launch.  The paper names divergence and scheduling overhead as the weak points of SIMT
//     processing (Sec. V); here the launch does not depend on the batch's composition and the
//     work is dealt out in homogeneous pieces.  A plan (built on the host, resident in device
//     memory) holds one record per UE (its geometry and buffers) and a list of work items,
//     each a tile of one UE, sorted so that items of one class (layers, modulation, antennas)
//     are adjacent and the heaviest come first.  Every block of the persistent grid takes the
//     next item from an atomic counter until the list is exhausted; a one-thread kernel
//     clears the counter before each run (both capture into a HIP graph).
// A tile is processed as
//   1. the LS estimate (Sec. III-B: channel estimation) of every pilot the tile's
//      subcarriers interpolate from, per occasion, into LDS, with the per-symbol tables;
//   2. one DMRS occasion (the channel held over the slot): each subcarrier's Gram
//      G = H^H H + s2 I, one (subcarrier, entry) per thread, then its Cholesky factor
//      (Sec. IV, Fig. 4), reciprocal diagonal and d = diag(G^-1), one subcarrier per thread,
//      staged in LDS; per resource element the matched filter streamed over the receive
//      antennas, forward / backward substitution with the staged factor, unbiasing, and the
//      max-log LLRs written to the output;
//   2'. two occasions, up to 4 layers: per subcarrier the channel pair (H0, H1 - H0) and the
//      three Gram pieces whose blend is the Gram at any time weight; per resource element the
//      blended Gram, its factorisation, the matched filter from the staged pairs,
//      substitution, unbiasing and LLRs;
//   2''. otherwise: per resource element the interpolation in frequency and time, Gram and
//      matched filter, factorisation, substitution, unbiasing and LLRs.
// Layers 1..8 (a template parameter: one branch per tile, uniform over the block), antennas
// 1..64, every modulation and DMRS configuration of the library.
#include <float.h>

#include "batch.h"
#include "rx_load.h"
#include "llr_math.h"

namespace ranphy {

namespace {

constexpr float kPivotRel = 16.f * FLT_EPSILON;

__host__ __device__ constexpr int tri(int i, int j) { return i * (i + 1) / 2 + j; }

// The per-data-symbol tables of a UE's geometry (symbol index and time-interpolation rule),
// staged in LDS with the pilots: the resource elements of a wave span several data symbols,
// and reading these lane-varying entries from the geometry in device memory would put a
// dependent memory round trip before every element's received-signal loads.
struct SymTab {
  int dsym[16];
  int o0[16];
  int o1[16];
  float w[16];
};

// n / d for 0 <= n < 2^22 by a float reciprocal and one correction step: an integer division
// by a run-time divisor costs tens of instructions, and the tile loops take one per element.
// The float quotient is exact or one below (n is exact as a float, the reciprocal within half
// an ulp), so a single remainder test fixes it.
struct FastDiv {
  int d;
  float inv;
  __device__ explicit FastDiv(int dd) : d(dd), inv(1.f / (float)dd) {}
  __device__ __forceinline__ int operator()(int n) const {
    int q = (int)((float)n * inv);
    if (n - q * d >= d) ++q;
    return q;
  }
};

// acc += conj(a) b and acc -= a b, acc -= conj(a) b: two fused multiply-adds per component
__device__ __forceinline__ void cmac_c(float2& acc, float2 a, float2 b) {
  acc.x = fmaf(a.x, b.x, acc.x);
  acc.x = fmaf(a.y, b.y, acc.x);
  acc.y = fmaf(a.x, b.y, acc.y);
  acc.y = fmaf(-a.y, b.x, acc.y);
}
__device__ __forceinline__ void cmsb(float2& acc, float2 a, float2 b) {
  acc.x = fmaf(-a.x, b.x, acc.x);
  acc.x = fmaf(a.y, b.y, acc.x);
  acc.y = fmaf(-a.x, b.y, acc.y);
  acc.y = fmaf(-a.y, b.x, acc.y);
}
__device__ __forceinline__ void cmsb_c(float2& acc, float2 a, float2 b) {
  acc.x = fmaf(-a.x, b.x, acc.x);
  acc.x = fmaf(-a.y, b.y, acc.x);
  acc.y = fmaf(-a.x, b.y, acc.y);
  acc.y = fmaf(a.y, b.x, acc.y);
}

// One exchange stage of the in-group chunk transpose (group_transpose), for the member-index
// bit S that lane bit LB carries (LB = 2 or 3: the partner lies 4 or 8 lanes away in the same
// DPP row, and the DPP bank mask picks the lanes that take the moved value, so the stage is
// one DPP move per value).  Members with the bit clear take the partner's chunk a into slot
// a | S; members with it set take the partner's chunk a | S into slot a.
template <int P, int S, int LB>
__device__ __forceinline__ void xpose_stage_bank(int (&c)[P][4]) {
  constexpr int up = 0x100 | (1 << LB), down = 0x110 | (1 << LB);  // row_shl / row_shr
  constexpr int lo_banks = LB == 2 ? 0x5 : 0x3, hi_banks = LB == 2 ? 0xA : 0xC;
#pragma unroll
  for (int a = 0; a < P; ++a) {
    if (a & S) continue;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int hi = __builtin_amdgcn_update_dpp(c[a | S][q], c[a][q], up, 0xF, lo_banks, false);
      const int lo = __builtin_amdgcn_update_dpp(c[a][q], c[a | S][q], down, 0xF, hi_banks, false);
      c[a | S][q] = hi;
      c[a][q] = lo;
    }
  }
}

// The same stage for member bit S carried by lane bit 0 (partner: the neighbouring lane of
// the quad), where lanes are told apart by a select.
template <int P, int S>
__device__ __forceinline__ void xpose_stage_quad(int (&c)[P][4], bool odd) {
#pragma unroll
  for (int a = 0; a < P; ++a) {
    if (a & S) continue;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int from_a = __builtin_amdgcn_mov_dpp(c[a][q], 0xB1, 0xF, 0xF, false);      // lane ^ 1
      const int from_as = __builtin_amdgcn_mov_dpp(c[a | S][q], 0xB1, 0xF, 0xF, false);
      const int hi = odd ? c[a | S][q] : from_a;
      const int lo = odd ? from_as : c[a][q];
      c[a | S][q] = hi;
      c[a][q] = lo;
    }
  }
}

// Groups of P = 2, 4 or 8 lanes exchanging 16-byte chunks (store_records, load_lines16).  A
// lane's member index within its group takes bit 0 from lane bit 2, bit 1 from lane bit 3
// and bit 2 from lane bit 0 (group_member); group_lane(lane, i) is the lane of member i of
// lane's group.
template <int P>
__device__ __forceinline__ int group_member(int lane) {
  return ((lane >> 2) & 1) | (P >= 4 ? ((lane >> 3) & 1) << 1 : 0) |
         (P == 8 ? (lane & 1) << 2 : 0);
}
template <int P>
__device__ __forceinline__ int group_lane(int lane, int i) {
  return (lane & ~(P == 8 ? 0xD : (P == 4 ? 0xC : 0x4))) | ((i & 1) << 2) |
         (((i >> 1) & 1) << 3) | ((i >> 2) & 1);
}
// Transpose within each group: afterwards member m's slot i holds what member i's slot m held.
template <int P>
__device__ __forceinline__ void group_transpose(int (&c)[P][4], int lane) {
  xpose_stage_bank<P, 1, 2>(c);
  if constexpr (P >= 4) xpose_stage_bank<P, 2, 3>(c);
  if constexpr (P == 8) xpose_stage_quad<P, 4>(c, lane & 1);
}

// Writes the LLR records of the resource elements the lanes of a wave hold (R floats per
// lane, R a multiple of 4, 8..32) so that every store instruction writes whole records:
// stored lane by lane, one 16-byte piece of a record per instruction, each instruction would
// touch a different cache line per lane, and the address and data path handles a line at a
// time.  A record is split into P >= R / 4 chunks of 16 bytes, the chunks are transposed
// within the lane groups (member m then holds chunk m of every member's record), and store i
// writes member i's record, one chunk per lane.  off is the record's offset in floats from
// base, negative where the lane holds no element.  Every lane of the wave must call this
// (the exchanges read the other lanes).
template <int R>
__device__ __forceinline__ void store_records(float* __restrict__ base, int off,
                                              const float (&out)[R]) {
  constexpr int NC = R / 4;
  constexpr int P = NC <= 2 ? 2 : (NC <= 4 ? 4 : 8);
  const int lane = (int)(threadIdx.x & 63);
  const int me = group_member<P>(lane);
  int c[P][4];
#pragma unroll
  for (int i = 0; i < P; ++i)
#pragma unroll
    for (int q = 0; q < 4; ++q) c[i][q] = i < NC ? __float_as_int(out[4 * i + q]) : 0;
  group_transpose<P>(c, lane);
  int oi[P];
#pragma unroll
  for (int i = 0; i < P; ++i) oi[i] = __builtin_amdgcn_ds_bpermute(group_lane<P>(lane, i) << 2, off);
  // 16-byte pieces where the buffer allows (the branch is uniform; the two store loops are
  // kept apart so that each compiles to its own access width)
  if ((reinterpret_cast<uintptr_t>(base) & 15) == 0) {
    float4* __restrict__ b4 = reinterpret_cast<float4*>(base);
#pragma unroll
    for (int i = 0; i < P; ++i)
      if (oi[i] >= 0 && me < NC)
        b4[(oi[i] >> 2) + me] = make_float4(__int_as_float(c[i][0]), __int_as_float(c[i][1]),
                                            __int_as_float(c[i][2]), __int_as_float(c[i][3]));
  } else {
    float2* __restrict__ b2 = reinterpret_cast<float2*>(base);
#pragma unroll
    for (int i = 0; i < P; ++i)
      if (oi[i] >= 0 && me < NC) {
        b2[(oi[i] >> 1) + 2 * me] = make_float2(__int_as_float(c[i][0]), __int_as_float(c[i][1]));
        b2[(oi[i] >> 1) + 2 * me + 1] =
            make_float2(__int_as_float(c[i][2]), __int_as_float(c[i][3]));
      }
  }
}

// The mirror of store_records for loads: each lane's 16 consecutive complex values from
// base + off (its resource element's samples of 16 antennas, one 128-byte line) into y, read
// so that load i fetches member i's whole line, one chunk per lane, and transposed back
// within the groups of 8.  Every lane of the wave must call this with an in-range off.
__device__ __forceinline__ void load_lines16(const float2* __restrict__ base, int off,
                                             float2 (&y)[16]) {
  const int lane = (int)(threadIdx.x & 63);
  const int me = group_member<8>(lane);
  int oi[8];
#pragma unroll
  for (int i = 0; i < 8; ++i) oi[i] = __builtin_amdgcn_ds_bpermute(group_lane<8>(lane, i) << 2, off);
  int c[8][4];
  if ((reinterpret_cast<uintptr_t>(base) & 15) == 0) {  // 16-byte pieces (uniform branch)
    const float4* __restrict__ b4 = reinterpret_cast<const float4*>(base);
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      const float4 v = b4[(oi[i] >> 1) + me];
      c[i][0] = __float_as_int(v.x);
      c[i][1] = __float_as_int(v.y);
      c[i][2] = __float_as_int(v.z);
      c[i][3] = __float_as_int(v.w);
    }
  } else {
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      const float2 a = base[oi[i] + 2 * me], b = base[oi[i] + 2 * me + 1];
      c[i][0] = __float_as_int(a.x);
      c[i][1] = __float_as_int(a.y);
      c[i][2] = __float_as_int(b.x);
      c[i][3] = __float_as_int(b.y);
    }
  }
  group_transpose<8>(c, lane);
#pragma unroll
  for (int i = 0; i < 8; ++i) {
    y[2 * i] = make_float2(__int_as_float(c[i][0]), __int_as_float(c[i][1]));
    y[2 * i + 1] = make_float2(__int_as_float(c[i][2]), __int_as_float(c[i][3]));
  }
}

// f(r, y_r) for the antennas r = 0 .. NR - 1 of one resource element (re: its index in the
// slot's grid), the samples read by lane groups in whole 16-antenna lines where the grid is
// complex64 and NR a multiple of 16 (each lane reading its own 16-byte pieces of 64
// different lines would fetch a line's halves at different times, and L2 refetches some),
// else lane by lane (LINES false: always, where the kernel form has no registers to spare).
// Every lane of the wave must call this.
template <int RXF, bool LINES, class F>
__device__ __forceinline__ void for_rx(const BatchUe& u, int64_t re, int NR, F&& f) {
  if (LINES && RXF == 0 && (NR & 15) == 0) {
    for (int r0 = 0; r0 < NR; r0 += 16) {
      float2 y[16];
      load_lines16(u.rx, (int)(re * NR) + r0, y);
#pragma unroll
      for (int c = 0; c < 16; ++c) f(r0 + c, y[c]);
    }
  } else {
#pragma unroll 8
    for (int r = 0; r < NR; ++r) f(r, rx_at<RXF>(u.rx, re, NR, r));
  }
}

// Layers L0 .. NL - 1 of one element's LLRs into its record llr[off ..], NS layers at a time
// (a slice of NS * QM floats held in registers at once): by store_records where a slice is a
// whole number of 16-byte chunks (8..32 floats), else lane by lane; off < 0: the lane holds
// no element (it still takes part in the exchanges).
template <int NL, int QM, int NS, int L0, int MAXR>
__device__ __forceinline__ void emit_slices(float* __restrict__ llr, int off,
                                            const float2 (&xo)[NL], const float (&vo)[NL]) {
  if constexpr (L0 < NL) {
    constexpr int N = NS < NL - L0 ? NS : NL - L0;
    constexpr int R = N * QM;
    float out[R];
#pragma unroll
    for (int l = 0; l < N; ++l) llr_one<QM>(xo[L0 + l], vo[L0 + l], out + l * QM);
    const int o = off >= 0 ? off + L0 * QM : -1;
    if constexpr (R % 4 == 0 && R >= 8 && R <= 32 && R <= MAXR) {
      store_records<R>(llr, o, out);
    } else if (o >= 0) {
#pragma unroll
      for (int b = 0; b < R; b += 2)
        *reinterpret_cast<float2*>(llr + o + b) = make_float2(out[b], out[b + 1]);
    }
    emit_slices<NL, QM, NS, L0 + N, MAXR>(llr, off, xo, vo);
  }
}

// The element's LLRs for the launch's modulation (uniform over the launch), in slices of at
// most MAXR floats (the register room of the kernel form; 64QAM slices hold an even number
// of layers, so that they stay whole 16-byte chunks; MAXR below 8: lane by lane).  off: the element's record in floats
// from llr (one slot's or UE's LLRs stay below 2^31), negative for none.
template <int NL, int MAXR>
__device__ __forceinline__ void emit_element(const Geom& g, float* __restrict__ llr, int off,
                                             const float2 (&xo)[NL], const float (&vo)[NL]) {
  constexpr int NS2 = MAXR / 2 < 1 ? 1 : MAXR / 2, NS4 = MAXR / 4 < 1 ? 1 : MAXR / 4;
  constexpr int NS8 = MAXR / 8 < 1 ? 1 : MAXR / 8;
  constexpr int NS6 = MAXR / 12 * 2 < 1 ? 1 : MAXR / 12 * 2;
  switch (g.qm) {
    case 2: emit_slices<NL, 2, NS2, 0, MAXR>(llr, off, xo, vo); break;
    case 4: emit_slices<NL, 4, NS4, 0, MAXR>(llr, off, xo, vo); break;
    case 6: emit_slices<NL, 6, NS6, 0, MAXR>(llr, off, xo, vo); break;
    default: emit_slices<NL, 8, NS8, 0, MAXR>(llr, off, xo, vo); break;
  }
}

// Resource element (data symbol d, subcarrier k) from its Gram G = H^H H (lower triangle) and
// matched filter z = H^H y: G + s2 I = L L^H (Cholesky, Sec. IV, Fig. 4), forward and backward
// substitution, d_l = || L^-1 e_l ||^2, unbiasing, max-log LLRs into llr[d][k][layer][qm].
template <int NL, int MAXR>
__device__ __forceinline__ void solve_emit(const Geom& g, float* __restrict__ llr, int d, int k,
                                           bool valid, float2 (&G)[NL * (NL + 1) / 2],
                                           float2 (&z)[NL], float s2) {
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
    for (int kk = 0; kk < j; ++kk) {
      dj = fmaf(-G[tri(j, kk)].x, G[tri(j, kk)].x, dj);
      dj = fmaf(-G[tri(j, kk)].y, G[tri(j, kk)].y, dj);
    }
    ok = ok && (dj > kPivotRel * gd[j]);
    const float dc = fmaxf(dj, FLT_MIN);
    const float inv = __builtin_amdgcn_rsqf(dc);  // 1 / L_jj (hardware, about 1 ulp)
    G[tri(j, j)] = make_float2(dc * inv, 0.f);
    linv[j] = inv;
#pragma unroll
    for (int i = j + 1; i < NL; ++i) {
      float2 acc = G[tri(i, j)];
#pragma unroll
      for (int kk = 0; kk < j; ++kk) {
        cmsb_c(acc, G[tri(j, kk)], G[tri(i, kk)]);
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
      cmsb(acc, G[tri(i, kk)], wv[kk]);
    }
    wv[i] = make_float2(acc.x * linv[i], acc.y * linv[i]);
  }
#pragma unroll
  for (int i = NL - 1; i >= 0; --i) {  // L^H x = w
    float2 acc = wv[i];
#pragma unroll
    for (int kk = i + 1; kk < NL; ++kk) {
      cmsb_c(acc, G[tri(kk, i)], xh[kk]);
    }
    xh[i] = make_float2(acc.x * linv[i], acc.y * linv[i]);
  }
  float2 xo[NL];
  float vo[NL];
#pragma unroll
  for (int l = 0; l < NL; ++l) {  // d_l = || L^-1 e_l ||^2, unbias
    float2 uu[NL];
    uu[l] = make_float2(linv[l], 0.f);
    float acc2 = linv[l] * linv[l];
#pragma unroll
    for (int i = l + 1; i < NL; ++i) {
      float2 acc = make_float2(0.f, 0.f);
#pragma unroll
      for (int kk = l; kk < i; ++kk) {
        cmsb(acc, G[tri(i, kk)], uu[kk]);
      }
      uu[i] = make_float2(acc.x * linv[i], acc.y * linv[i]);
      acc2 += uu[i].x * uu[i].x + uu[i].y * uu[i].y;
    }
    const float sd = s2 * acc2;
    const float im = __builtin_amdgcn_rcpf(1.f - sd);
    xo[l] = ok ? make_float2(xh[l].x * im, xh[l].y * im)
               : make_float2(__builtin_nanf(""), __builtin_nanf(""));
    vo[l] = ok ? sd * im : __builtin_inff();
  }
  emit_element<NL, MAXR>(g, llr, valid ? (d * g.n_sc + k) * NL * g.qm : -1, xo, vo);
}

template <int NL, int RXF, int MAXR>
__device__ __forceinline__ void detect_tile(const BatchUe& u, const Geom& g, int k0, int nk,
                                            int jlo, int nj,
                            const float2* __restrict__ lds, const SymTab& tab) {
  const int NR = g.n_rx, ND = g.n_dsym, RS = batch_row_stride(NR, NL);
  const float s2 = *u.nv;
  const FastDiv by_nk(nk);
  const int total = nk * ND, lane = (int)(threadIdx.x & 63);
  // wave-uniform trips: every lane takes part in the record stores of solve_emit
  for (int e0 = (int)threadIdx.x - lane; e0 < total; e0 += blockDim.x) {
    const bool valid = e0 + lane < total;
    const int e = valid ? e0 + lane : total - 1;
    const int d = by_nk(e);
    const int k = k0 + (e - d * nk);
    const int s = tab.dsym[d];
    const int o0 = tab.o0[d], o1 = tab.o1[d];
    const float w = tab.w[d];
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
    const int64_t re = (int64_t)s * g.n_sc + k;
    for (int r = 0; r < NR; ++r) {
      const float2 y = rx_at<RXF>(u.rx, re, NR, r);
      float2 hr[NL];
#pragma unroll
      for (int p = 0; p < NL; ++p) {
        const float2* b = lds + r * NL + p;
        const float2 v0 = b[(o0 * nj + r0[p]) * RS], v1 = b[(o0 * nj + r1[p]) * RS];
        float2 v = make_float2(v0.x + a[p] * (v1.x - v0.x), v0.y + a[p] * (v1.y - v0.y));
        if (o1 != o0) {
          const float2 u0 = b[(o1 * nj + r0[p]) * RS], u1 = b[(o1 * nj + r1[p]) * RS];
          const float2 vv = make_float2(u0.x + a[p] * (u1.x - u0.x), u0.y + a[p] * (u1.y - u0.y));
          v = make_float2(v.x + w * (vv.x - v.x), v.y + w * (vv.y - v.y));
        }
        hr[p] = v;
      }
#pragma unroll
      for (int i = 0; i < NL; ++i) {
        cmac_c(z[i], hr[i], y);
#pragma unroll
        for (int j = 0; j <= i; ++j) cmac_c(G[tri(i, j)], hr[i], hr[j]);
      }
    }
    solve_emit<NL, MAXR>(g, u.llr, d, k, valid, G, z, s2);
  }
}

// Two DMRS occasions, up to 4 layers.  The channel at a data symbol is H0 + t (H1 - H0) with
// t from the time rule (0 or 1 before the first or after the last occasion), so its Gram is
// (1-t)^2 A + t(1-t) S + t^2 C with A = H0^H H0, C = H1^H H1 and S = H0^H H1 + H1^H H0, the
// same quantity with the antenna sums taken once per subcarrier instead of per resource
// element.  The tile stages, per subcarrier, H0 and D = H1 - H0 (interpolated in frequency
// once; float4 (H0, D) per antenna and layer in pair[]) and A, S, C (in gram[]); each
// resource element then blends its Gram, forms z = (H0 + t D)^H y from the staged pairs and
// finishes as the other paths do.
template <int NL, int RXF, int MAXR, bool LINES>
__device__ __forceinline__ void detect_tile_pair(const BatchUe& u, const Geom& g, int k0, int nk,
                                                 int jlo, int nj,
                                 const float2* __restrict__ rows, float4* __restrict__ pair,
                                 float2* __restrict__ gram, const SymTab& tab) {
  constexpr int NP = NL * (NL + 1) / 2;
  const int NR = g.n_rx, ND = g.n_dsym, RS = batch_row_stride(NR, NL);
  const int PS = batch_pair_stride(NR, NL), GS = batch_gram_stride(NL);
  // channel pairs: items (subcarrier, layer, group of 8 antennas), so that a layer's
  // interpolation rule is found once per 8 antennas
  const int nch = (NR + 7) >> 3;
  const FastDiv by_nch(nch);
  for (int f = threadIdx.x; f < nk * NL * nch; f += blockDim.x) {
    const int kp = by_nch(f);
    const int c = f - kp * nch;
    const int kk = kp / NL;
    const int p = kp - kk * NL;
    int j0, j1;
    float a;
    freq_rule(g, p, k0 + kk, j0, j1, a);
    const float2* b0 = rows + (j0 - jlo) * RS + p;
    const float2* b1 = rows + (j1 - jlo) * RS + p;
    const float2* c0 = rows + (nj + j0 - jlo) * RS + p;
    const float2* c1 = rows + (nj + j1 - jlo) * RS + p;
    float4* dst = pair + kk * PS + p;
#pragma unroll
    for (int rr = 0; rr < 8; ++rr) {
      const int r = 8 * c + rr;
      if (r < NR) {
        const float2 v0 = b0[r * NL], v1 = b1[r * NL], u0 = c0[r * NL], u1 = c1[r * NL];
        const float2 h0 = make_float2(v0.x + a * (v1.x - v0.x), v0.y + a * (v1.y - v0.y));
        const float2 h1 = make_float2(u0.x + a * (u1.x - u0.x), u0.y + a * (u1.y - u0.y));
        dst[r * NL] = make_float4(h0.x, h0.y, h1.x - h0.x, h1.y - h0.y);
      }
    }
  }
  __syncthreads();
  // Gram pieces: items (subcarrier, entry), the strictly lower entries first and then the
  // diagonal ones, so that most waves hold one kind; a diagonal entry is real (its imaginary
  // part is not used) and S_ii = 2 Re(h0_i^H h1_i), a third of the off-diagonal work
  constexpr int NOFF = NP - NL, NOFF1 = NOFF > 0 ? NOFF : 1;
  const int n_off = nk * NOFF;
  for (int f = threadIdx.x; f < n_off + nk * NL; f += blockDim.x) {
    const bool off = f < n_off;
    const int kk = off ? f / NOFF1 : (f - n_off) / NL;
    const float4* q = pair + kk * PS;
    float2* gg = gram + kk * GS;
    if (off) {
      const int m = f - kk * NOFF;
      int i = 1;
#pragma unroll
      for (int cc = 2; cc < NL; ++cc) i += m >= cc * (cc - 1) / 2;
      const int j = m - i * (i - 1) / 2;
      float2 A = make_float2(0.f, 0.f), S = A, C = A;
      for (int r = 0; r < NR; ++r) {
        const float4 qi = q[r * NL + i], qj = q[r * NL + j];
        const float2 h0i = make_float2(qi.x, qi.y), h0j = make_float2(qj.x, qj.y);
        const float2 h1i = make_float2(qi.x + qi.z, qi.y + qi.w);
        const float2 h1j = make_float2(qj.x + qj.z, qj.y + qj.w);
        cmac_c(A, h0i, h0j);
        cmac_c(C, h1i, h1j);
        cmac_c(S, h0i, h1j);
        cmac_c(S, h1i, h0j);
      }
      const int e = tri(i, j);
      gg[e] = A;
      gg[NP + e] = S;
      gg[2 * NP + e] = C;
    } else {
      const int i = f - n_off - kk * NL;
      float a = 0.f, sr = 0.f, cr = 0.f;
      for (int r = 0; r < NR; ++r) {
        const float4 qi = q[r * NL + i];
        const float h1x = qi.x + qi.z, h1y = qi.y + qi.w;
        a = fmaf(qi.y, qi.y, fmaf(qi.x, qi.x, a));
        cr = fmaf(h1y, h1y, fmaf(h1x, h1x, cr));
        sr = fmaf(qi.y, h1y, fmaf(qi.x, h1x, sr));
      }
      const int e = tri(i, i);
      gg[e] = make_float2(a, 0.f);
      gg[NP + e] = make_float2(2.f * sr, 0.f);
      gg[2 * NP + e] = make_float2(cr, 0.f);
    }
  }
  __syncthreads();
  const float s2 = *u.nv;
  const FastDiv by_nk(nk);
  const int total = nk * ND, lane = (int)(threadIdx.x & 63);
  // resource elements, wave-uniform trips: every lane takes part in the record stores
  for (int e0 = (int)threadIdx.x - lane; e0 < total; e0 += blockDim.x) {
    const bool valid = e0 + lane < total;
    const int e = valid ? e0 + lane : total - 1;
    const int d = by_nk(e);
    const int kk = e - d * nk;
    const int k = k0 + kk;
    const int o0 = tab.o0[d], o1 = tab.o1[d];
    const float t = o0 == o1 ? (float)o0 : tab.w[d];
    const float w0 = (1.f - t) * (1.f - t), w1 = t * (1.f - t), w2 = t * t;
    float2 G[NP], z[NL];
#pragma unroll
    for (int i = 0; i < NL; ++i) z[i] = make_float2(0.f, 0.f);
    const int64_t re = (int64_t)tab.dsym[d] * g.n_sc + k;
    const float4* q = pair + kk * PS;
    for_rx<RXF, LINES>(u, re, NR, [&](int r, float2 y) {
#pragma unroll
      for (int p = 0; p < NL; ++p) {
        const float4 v = q[r * NL + p];
        const float2 h = make_float2(v.x + t * v.z, v.y + t * v.w);
        cmac_c(z[p], h, y);
      }
    });
    const float2* gg = gram + kk * GS;  // blended after the matched filter: fewer live values
#pragma unroll
    for (int i = 0; i < NP; ++i) {
      const float2 A = gg[i], S = gg[NP + i], C = gg[2 * NP + i];
      G[i] = make_float2(w0 * A.x + w1 * S.x + w2 * C.x, w0 * A.y + w1 * S.y + w2 * C.y);
    }
    solve_emit<NL, MAXR>(g, u.llr, d, k, valid, G, z, s2);
  }
}

// Channel value of port p at antenna r for the subcarrier whose interpolation rows and
// weight are (r0, r1, a), one occasion: rows[j][r][p], RS complex values per row.
__device__ __forceinline__ float2 row_interp(const float2* __restrict__ rows, int RS, int NL,
                                             int r0, int r1, float a, int r, int p) {
  const float2 v0 = rows[r0 * RS + r * NL + p], v1 = rows[r1 * RS + r * NL + p];
  return make_float2(v0.x + a * (v1.x - v0.x), v0.y + a * (v1.y - v0.y));
}

// One occasion: Gram, Cholesky factor, reciprocal diagonal and d = diag(G^-1) of each of the
// tile's subcarriers into LDS.  fac[kk][tri(i, j)] holds L, aux[kk][0..NL) 1 / L_ii,
// aux[kk][NL..2NL) d, aux[kk][2NL] 1 where the factorisation succeeded, else 0.
template <int NL, class CAP>
__device__ __forceinline__ void factor_tile(const BatchUe& u, const Geom& g, int k0, int nk,
                                            int jlo,
                            const float2* __restrict__ rows, float2* __restrict__ fac,
                            float* __restrict__ aux) {
  constexpr int NP = NL * (NL + 1) / 2;
  const int NR = g.n_rx, RS = batch_row_stride(NR, NL);
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
      const float2 hi = row_interp(rows, RS, NL, ri0, ri1, ai, r, i);
      const float2 hj = row_interp(rows, RS, NL, rj0, rj1, aj, r, j);
      cmac_c(acc, hi, hj);
    }
    fac[kk * CAP::fnp + e] = acc;
  }
  __syncthreads();
  const float s2 = *u.nv;
  for (int kk = threadIdx.x; kk < nk; kk += blockDim.x) {
    float2 G[NP];
#pragma unroll
    for (int e = 0; e < NP; ++e) G[e] = fac[kk * CAP::fnp + e];
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
      for (int kq = 0; kq < j; ++kq)
        dj -= G[tri(j, kq)].x * G[tri(j, kq)].x + G[tri(j, kq)].y * G[tri(j, kq)].y;
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
          cmsb_c(acc, G[tri(j, kq)], G[tri(i, kq)]);
        }
        G[tri(i, j)] = make_float2(acc.x * inv, acc.y * inv);
      }
    }
    float* ax = aux + kk * CAP::aux;
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
          cmsb(acc, G[tri(i, kq)], uu[kq]);
        }
        uu[i] = make_float2(acc.x * linv[i], acc.y * linv[i]);
        acc2 += uu[i].x * uu[i].x + uu[i].y * uu[i].y;
      }
      ax[l] = linv[l];
      ax[NL + l] = acc2;
    }
    ax[2 * NL] = ok ? 1.f : 0.f;
#pragma unroll
    for (int e = 0; e < NP; ++e) fac[kk * CAP::fnp + e] = G[e];
  }
  __syncthreads();
}

// One occasion, per resource element with the staged factor: matched filter, substitutions,
// unbiasing, LLRs.
template <int NL, class CAP, int RXF>
__device__ __forceinline__ void detect_tile_fact(const BatchUe& u, const Geom& g, int k0, int nk,
                                                 int jlo,
                                 const float2* __restrict__ rows,
                                 const float2* __restrict__ fac, const float* __restrict__ aux,
                                 const SymTab& tab) {
  constexpr int NP = NL * (NL + 1) / 2;
  const int NR = g.n_rx, ND = g.n_dsym, RS = batch_row_stride(NR, NL);
  const float s2 = *u.nv;
  const FastDiv by_nk(nk);
  const int total = nk * ND, lane = (int)(threadIdx.x & 63);
  // wave-uniform trips: every lane takes part in the record stores
  for (int e0 = (int)threadIdx.x - lane; e0 < total; e0 += blockDim.x) {
    const bool valid = e0 + lane < total;
    const int e = valid ? e0 + lane : total - 1;
    const int d = by_nk(e);
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
    const int64_t re = (int64_t)tab.dsym[d] * g.n_sc + k;
    for_rx<RXF, CAP::line_loads>(u, re, NR, [&](int r, float2 y) {
#pragma unroll
      for (int i = 0; i < NL; ++i)
        cmac_c(z[i], row_interp(rows, RS, NL, r0[i], r1[i], a[i], r, i), y);
    });
    const float2* L = fac + kk * CAP::fnp;
    const float* ax = aux + kk * CAP::aux;
    const bool ok = ax[2 * NL] != 0.f;
    float2 wv[NL], xh[NL];
#pragma unroll
    for (int i = 0; i < NL; ++i) {  // L w = z
      float2 acc = z[i];
#pragma unroll
      for (int kq = 0; kq < i; ++kq) {
        cmsb(acc, L[tri(i, kq)], wv[kq]);
      }
      wv[i] = make_float2(acc.x * ax[i], acc.y * ax[i]);
    }
#pragma unroll
    for (int i = NL - 1; i >= 0; --i) {  // L^H x = w
      float2 acc = wv[i];
#pragma unroll
      for (int kq = i + 1; kq < NL; ++kq) {
        cmsb_c(acc, L[tri(kq, i)], xh[kq]);
      }
      xh[i] = make_float2(acc.x * ax[i], acc.y * ax[i]);
    }
    float2 xo[NL];
    float vo[NL];
#pragma unroll
    for (int l = 0; l < NL; ++l) {
      const float sd = s2 * ax[NL + l];
      const float im = 1.f / (1.f - sd);
      xo[l] = ok ? make_float2(xh[l].x * im, xh[l].y * im)
                 : make_float2(__builtin_nanf(""), __builtin_nanf(""));
      vo[l] = ok ? sd * im : __builtin_inff();
    }
    emit_element<NL, CAP::store_floats>(g, u.llr, valid ? (d * g.n_sc + k) * NL * g.qm : -1, xo,
                                        vo);
  }
}

// The LS estimates of the tile's pilot rows, every occasion: each thread's estimates are
// taken kStageBatch at a time with every load issued before the first is used (one memory
// round trip per batch instead of one per estimate); indices are clamped into range and the
// surplus discarded, so the loads need no branches.  T (the time cover length) is a template
// parameter so that its loop unrolls.
template <int T, int kStageBatch, int RXF>
__device__ __forceinline__ void stage_rows(const BatchUe& u, const Geom& g, int jlo, int nj,
                                           float2* __restrict__ rows) {
  const int C = g.comb, NR = g.n_rx, NL = g.n_layers, J = g.n_pilot, NSC = g.n_sc;
  const int per_occ = nj * NR * NL, total = g.n_occ * per_occ, RS = batch_row_stride(NR, NL);
  const int s00 = g.sym0[0], s01 = g.sym0[1], s02 = g.sym0[2], s03 = g.sym0[3];
  const FastDiv by_nl(NL), by_nr(NR), by_occ(per_occ);
  constexpr float inv_t = 1.f / (float)T;
  for (int f0 = threadIdx.x; f0 < total; f0 += kStageBatch * blockDim.x) {
    float2 yv[kStageBatch][T], qv[kStageBatch][T];
    int dst[kStageBatch];
    bool in_band[kStageBatch];
#pragma unroll
    for (int b = 0; b < kStageBatch; ++b) {
      const int f = min(f0 + b * (int)blockDim.x, total - 1);
      const int o = by_occ(f);
      const int fo = f - o * per_occ;
      const int fl = by_nl(fo);
      const int p = fo - fl * NL;
      const int jj = by_nr(fl);
      const int r = fl - jj * NR;
      const int j = jlo + jj;
      const int k = C * j + (p & (C - 1));
      const int s0 = o == 0 ? s00 : (o == 1 ? s01 : (o == 2 ? s02 : s03));
      const int kc = min(k, NSC - 1);
      in_band[b] = k < NSC;
      dst[b] = (o * nj + jj) * RS + r * NL + p;
#pragma unroll
      for (int t = 0; t < T; ++t) {
        yv[b][t] = rx_at<RXF>(u.rx, (int64_t)(s0 + t) * NSC + kc, NR, r);
        qv[b][t] = u.pil[(((int64_t)o * T + t) * J + j) * NL + p];
      }
    }
#pragma unroll
    for (int b = 0; b < kStageBatch; ++b) {
      if (f0 + b * (int)blockDim.x < total) {
        float2 acc = make_float2(0.f, 0.f);
#pragma unroll
        for (int t = 0; t < T; ++t) cmac_c(acc, qv[b][t], yv[b][t]);  // y conj(q)
        if (!in_band[b]) acc = make_float2(0.f, 0.f);
        rows[dst[b]] = make_float2(acc.x * inv_t, acc.y * inv_t);
      }
    }
  }
}

// The LS estimate (Sec. III-B) of every pilot the tile k0 .. k0 + nk - 1 interpolates from,
// every occasion, into rows[o][j - jlo][r][p] (rows of batch_row_stride values), and the
// symbol tables into tab; returns jlo and the pilot count nj.  Ends with a barrier.
template <int SB, int RXF>
__device__ __forceinline__ void stage_pilots(const BatchUe& u, const Geom& g, int k0, int nk,
                                             float2* __restrict__ rows, SymTab& tab, int& jlo,
                                             int& nj) {
  const int T = g.td, NL = g.n_layers, J = g.n_pilot;
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
  if (T == 1)
    stage_rows<1, SB, RXF>(u, g, jlo, nj, rows);
  else
    stage_rows<2, SB, RXF>(u, g, jlo, nj, rows);
  if (threadIdx.x < g.n_dsym) {
    const int d = threadIdx.x;
    tab.dsym[d] = g.dsym[d];
    tab.o0[d] = g.t_o0[d];
    tab.o1[d] = g.t_o1[d];
    tab.w[d] = g.t_w[d];
  }
  __syncthreads();
}

// One occasion, filter form: per (subcarrier, antenna) item the column W[:, r] of
// W = diag(1/mu) G^-1 H^H, i.e. the two substitutions with the staged factor applied to
// conj(H[r][:]) and each layer scaled by 1/mu_l = 1 / (1 - s2 d_l), into wf[kk][r][l]; then
// per resource element x~ = W y, the variance s2 d_l / mu_l from the staged d, and the LLRs.
// Same quantities as detect_tile_fact, with the substitutions taken once per subcarrier and
// antenna instead of once per resource element.
template <int NL, class CAP, int RXF>
__device__ __forceinline__ void detect_tile_w(const BatchUe& u, const Geom& g, int k0, int nk,
                                              int jlo, const float2* __restrict__ rows,
                                              const float2* __restrict__ fac,
                                              const float* __restrict__ aux,
                                              float2* __restrict__ wf, const SymTab& tab) {
  const int NR = g.n_rx, ND = g.n_dsym, RS = batch_row_stride(NR, NL);
  const int WS = batch_w_stride(NR, NL);
  const float s2 = *u.nv;
  const FastDiv by_nr(NR);
  for (int f = threadIdx.x; f < nk * NR; f += blockDim.x) {  // (subcarrier, antenna)
    const int kk = by_nr(f);
    const int r = f - kk * NR;
    const int k = k0 + kk;
    const float2* L = fac + kk * CAP::fnp;
    const float* ax = aux + kk * CAP::aux;
    float2 wv[NL], xh[NL];
#pragma unroll
    for (int i = 0; i < NL; ++i) {  // L w = conj(h_r)
      int j0, j1;
      float a;
      freq_rule(g, i, k, j0, j1, a);
      const float2 h = row_interp(rows, RS, NL, j0 - jlo, j1 - jlo, a, r, i);
      float2 acc = make_float2(h.x, -h.y);
#pragma unroll
      for (int kq = 0; kq < i; ++kq) cmsb(acc, L[tri(i, kq)], wv[kq]);
      wv[i] = make_float2(acc.x * ax[i], acc.y * ax[i]);
    }
#pragma unroll
    for (int i = NL - 1; i >= 0; --i) {  // L^H x = w
      float2 acc = wv[i];
#pragma unroll
      for (int kq = i + 1; kq < NL; ++kq) cmsb_c(acc, L[tri(kq, i)], xh[kq]);
      xh[i] = make_float2(acc.x * ax[i], acc.y * ax[i]);
    }
    float2* w = wf + kk * WS + r * NL;
#pragma unroll
    for (int l = 0; l < NL; ++l) {
      const float im = __builtin_amdgcn_rcpf(1.f - s2 * ax[NL + l]);
      w[l] = make_float2(xh[l].x * im, xh[l].y * im);
    }
  }
  __syncthreads();
  const FastDiv by_nk(nk);
  const int total = nk * ND, lane = (int)(threadIdx.x & 63);
  // wave-uniform trips: every lane takes part in the record stores
  for (int e0 = (int)threadIdx.x - lane; e0 < total; e0 += blockDim.x) {
    const bool valid = e0 + lane < total;
    const int e = valid ? e0 + lane : total - 1;
    const int d = by_nk(e);
    const int kk = e - d * nk;
    const int k = k0 + kk;
    const float* ax = aux + kk * CAP::aux;
    const bool ok = ax[2 * NL] != 0.f;
    float2 x[NL];
#pragma unroll
    for (int i = 0; i < NL; ++i) x[i] = make_float2(0.f, 0.f);
    const int64_t re = (int64_t)tab.dsym[d] * g.n_sc + k;
    const float2* w = wf + kk * WS;
    for_rx<RXF, CAP::line_loads>(u, re, NR, [&](int r, float2 y) {
#pragma unroll
      for (int l = 0; l < NL; ++l) {  // x_l += W[l][r] y_r
        const float2 c = w[r * NL + l];
        x[l].x = fmaf(c.x, y.x, x[l].x);
        x[l].x = fmaf(-c.y, y.y, x[l].x);
        x[l].y = fmaf(c.x, y.y, x[l].y);
        x[l].y = fmaf(c.y, y.x, x[l].y);
      }
    });
    float2 xo[NL];
    float vo[NL];
#pragma unroll
    for (int l = 0; l < NL; ++l) {
      const float sd = s2 * ax[NL + l];
      vo[l] = ok ? sd * __builtin_amdgcn_rcpf(1.f - sd) : __builtin_inff();
      xo[l] = ok ? x[l] : make_float2(__builtin_nanf(""), __builtin_nanf(""));
    }
    emit_element<NL, CAP::store_floats>(g, u.llr, valid ? (d * g.n_sc + k) * NL * g.qm : -1, xo,
                                        vo);
  }
}

// One tile of nk subcarriers starting at k0: pilots staged, then the path for the DMRS layout.
template <int NL, class CAP, int RXF>
__device__ __forceinline__ void process_tile(const BatchUe& u, const Geom& g, int k0, int nk,
                                             float2* rows, float2* fac, float* aux,
                                             SymTab& tab) {
  int jlo, nj;
  stage_pilots<CAP::stage_batch, RXF>(u, g, k0, nk, rows, tab, jlo, nj);
  if constexpr (CAP::multi_occ) {  // launched for several occasions only
    if constexpr (NL <= 4) {
      float4* pair = reinterpret_cast<float4*>(
          rows + batch_pair_base(g.n_occ * nj, batch_row_stride(g.n_rx, NL)));
      if (batch_pair_path(g, CAP::rows, CAP::fac)) {
        detect_tile_pair<NL, RXF, CAP::store_floats, CAP::line_loads>(u, g, k0, nk, jlo, nj, rows, pair, fac, tab);
        return;
      }
    }
    detect_tile<NL, RXF, CAP::store_floats>(u, g, k0, nk, jlo, nj, rows, tab);
    return;
  }
  if (CAP::one_occ || g.n_occ == 1) {  // a one-occasion form is launched for those only
    factor_tile<NL, CAP>(u, g, k0, nk, jlo, rows, fac, aux);
    const int rs = batch_row_stride(g.n_rx, NL);
    if (batch_w_path(g, CAP::rows))  // the host's tile widths fit for such shapes
      detect_tile_w<NL, CAP, RXF>(u, g, k0, nk, jlo, rows, fac, aux,
                                  rows + batch_pair_base(g.n_occ * nj, rs), tab);
    else
      detect_tile_fact<NL, CAP, RXF>(u, g, k0, nk, jlo, rows, fac, aux, tab);
    return;
  }
  if constexpr (NL <= 4) {
    if (batch_pair_path(g, CAP::rows, CAP::fac)) {  // the host's tile widths fit
      float4* pair = reinterpret_cast<float4*>(
          rows + batch_pair_base(g.n_occ * nj, batch_row_stride(g.n_rx, NL)));
      detect_tile_pair<NL, RXF, CAP::store_floats, CAP::line_loads>(u, g, k0, nk, jlo, nj, rows, pair, fac, tab);
      return;
    }
  }
  detect_tile<NL, RXF, CAP::store_floats>(u, g, k0, nk, jlo, nj, rows, tab);
}

template <int MAXNL, int BLOCKS, int RXF>
__device__ __forceinline__ void process_any(const BatchUe& u, const Geom& g, int k0, int nk,
                                            float2* rows, float2* fac, float* aux, SymTab& tab) {
  using CAP = TileCap<MAXNL, BLOCKS>;
  switch (g.n_layers) {  // uniform over the block
    case 1: process_tile<1, CAP, RXF>(u, g, k0, nk, rows, fac, aux, tab); break;
    case 2: process_tile<2, CAP, RXF>(u, g, k0, nk, rows, fac, aux, tab); break;
    case 3: process_tile<3, CAP, RXF>(u, g, k0, nk, rows, fac, aux, tab); break;
    default:
      if constexpr (MAXNL == 4) {
        process_tile<4, CAP, RXF>(u, g, k0, nk, rows, fac, aux, tab);
      } else {
        switch (g.n_layers) {
          case 4: process_tile<4, CAP, RXF>(u, g, k0, nk, rows, fac, aux, tab); break;
          case 5: process_tile<5, CAP, RXF>(u, g, k0, nk, rows, fac, aux, tab); break;
          case 6: process_tile<6, CAP, RXF>(u, g, k0, nk, rows, fac, aux, tab); break;
          case 7: process_tile<7, CAP, RXF>(u, g, k0, nk, rows, fac, aux, tab); break;
          default: process_tile<8, CAP, RXF>(u, g, k0, nk, rows, fac, aux, tab); break;
        }
      }
      break;
  }
}

__global__ void batch_reset_kernel(BatchHdr* __restrict__ hdr) {
  if (threadIdx.x == 0 && blockIdx.x == 0) hdr->head = 0u;
}

__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(3, 8))) batch_kernel(
    char* __restrict__ plan) {
  using CAP = TileCap<8, 3>;
  __shared__ __align__(16) float2 lds[CAP::rows];
  __shared__ float2 fac[CAP::fac];
  __shared__ float aux[CAP::fsc * CAP::aux];
  __shared__ SymTab tab;
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
    process_any<8, 3, 0>(u, g, item.k0, item.nk, lds, fac, aux, tab);
    __syncthreads();  // LDS is reused by the next item
  }
}

// The whole chain for a batch of slots of one shape (up to MAXNL layers) in one launch: block
// (slot, tile of nk subcarriers) stages the tile's pilot estimates and detects and demaps its
// resource elements, as a work item of the multi-UE launch does.  BLOCKS blocks fit a CU
// (LDS and registers).
// RXF = 1: rx holds the grid's block floating point words (rx_load.h), decoded where loaded.
template <int MAXNL, int BLOCKS, int RXF>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(BLOCKS, 8)))
receive_kernel(Geom g, const float2* __restrict__ rx, const float2* __restrict__ pil,
               const float* __restrict__ nvar, float* __restrict__ llr, int nk) {
  using CAP = TileCap<MAXNL, BLOCKS>;
  __shared__ __align__(16) float2 lds[CAP::rows];
  __shared__ float2 fac[CAP::fac];
  __shared__ float aux[CAP::fsc * CAP::aux];
  __shared__ SymTab tab;
  const int ntiles = (g.n_sc + nk - 1) / nk;
  const int slot = blockIdx.x / ntiles;
  const int k0 = (blockIdx.x - slot * ntiles) * nk;
  BatchUe u;
  u.g = g;
  const int64_t slot_re = (int64_t)slot * g.n_symb * g.n_sc;
  if constexpr (RXF == 0) {
    u.rx = rx + slot_re * g.n_rx;
  } else {  // words per resource element: blocks of 16 antennas (or all, below 16)
    const int B = g.n_rx >= 16 ? 16 : g.n_rx;
    const int64_t w_re = (int64_t)(g.n_rx / B) * (1 + (18 * B + 31) / 32);
    u.rx = reinterpret_cast<const float2*>(reinterpret_cast<const unsigned*>(rx) + slot_re * w_re);
  }
  u.pil = pil + (int64_t)slot * g.n_occ * g.td * g.n_pilot * g.n_layers;
  u.nv = nvar + slot;
  u.llr = llr + (int64_t)slot * g.n_dsym * g.n_sc * g.n_layers * g.qm;
  const int n = min(nk, g.n_sc - k0);
  process_any<MAXNL, BLOCKS, RXF>(u, g, k0, n, lds, fac, aux, tab);
}

}  // namespace

namespace {
struct CapRT {
  int rows, fac, fsc;
};
// The kernel form for a shape: up to 4 layers 5 blocks per CU (one occasion) or 4 (several:
// the channel pairs need the room), else the 8-layer form at 3.
int receive_form(const Geom& g) { return g.n_layers > 4 ? 0 : (g.n_occ == 1 ? 2 : 1); }
template <class CAP>
CapRT cap_rt() {
  return {CAP::rows, CAP::fac, CAP::fsc};
}
CapRT receive_cap(const Geom& g) {
  switch (receive_form(g)) {
    case 2: return cap_rt<TileCap<4, 5>>();
    case 1: return cap_rt<TileCap<4, 4>>();
    default: return cap_rt<TileCap<8, 3>>();
  }
}
}  // namespace

// Tile width of the one-launch chain: about tile_re resource elements, at most fsc
// subcarriers, and the widest below that whose staged data (channel pairs, filters or pilot
// rows, by the shape's path) fit the block's LDS at every tile; 0 if none does.
int receive_tile(const Geom& g, int tile_re) {
  const CapRT cap = receive_cap(g);
  int want = tile_re / g.n_dsym;
  want = want < 1 ? 1 : (want > cap.fsc ? cap.fsc : want);
  const int per = batch_row_stride(g.n_rx, g.n_layers);
  const bool pair = g.n_occ == 2 && batch_pair_path(g, cap.rows, cap.fac);
  const bool wpath = g.n_occ == 1 && batch_w_path(g, cap.rows);
  for (int nk = want; nk >= 1; --nk) {
    bool ok = true;
    for (int k0 = 0; k0 < g.n_sc && ok; k0 += nk) {
      const int n = g.n_sc - k0 < nk ? g.n_sc - k0 : nk;
      const int rows = batch_tile_rows(g, k0, n);
      ok = pair ? batch_pair_fits(g, rows, n, cap.rows, cap.fac)
                : (wpath ? batch_w_fits(g, rows, n, cap.rows) : rows * per <= cap.rows);
    }
    if (ok) return nk;
  }
  return 0;
}

template <int RXF>
void launch_receive_rxf(const Geom& g, dim3 grid, const float2* rx, const float2* pil,
                        const float* nvar, float* llr, int nk, hipStream_t s) {
  switch (receive_form(g)) {
    case 2:
      hipLaunchKernelGGL((receive_kernel<4, 5, RXF>), grid, dim3(256), 0, s, g, rx, pil, nvar, llr,
                         nk);
      break;
    case 1:
      hipLaunchKernelGGL((receive_kernel<4, 4, RXF>), grid, dim3(256), 0, s, g, rx, pil, nvar, llr,
                         nk);
      break;
    default:
      hipLaunchKernelGGL((receive_kernel<8, 3, RXF>), grid, dim3(256), 0, s, g, rx, pil, nvar, llr,
                         nk);
      break;
  }
}

hipError_t launch_receive(const Geom& g, const float2* rx, bool bfp, const float2* pil,
                          const float* nvar, float* llr, int nk, hipStream_t s) {
  const int64_t ntiles = (g.n_sc + nk - 1) / nk;
  const dim3 grid((unsigned)(g.n_slots * ntiles));
  if (bfp)
    launch_receive_rxf<1>(g, grid, rx, pil, nvar, llr, nk, s);
  else
    launch_receive_rxf<0>(g, grid, rx, pil, nvar, llr, nk, s);
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
  hipLaunchKernelGGL(batch_reset_kernel, dim3(1), dim3(64), 0, s,
                     reinterpret_cast<BatchHdr*>(plan));
  hipLaunchKernelGGL(batch_kernel, dim3(blocks), dim3(256), 0, s, static_cast<char*>(plan));
  return hipGetLastError();
}

}  // namespace ranphy
