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
// The received grid may also arrive in block floating point form (RXF = 1): 16-antenna
// blocks of 10 words, a shared exponent e then the 9-bit two's complement mantissas m of the
// block's 32 reals (I and Q interleaved) as a little-endian bit stream, each value m 2^e.
// A lane's 16 antennas of one symbol are exactly one block, read as five 8-byte loads and
// decoded in registers just before the matched filter; the decoded values equal those of
// the separate decompression kernel bit for bit, so the results do too.
//
// With LSF = 1 (pilot resolution, the one-launch chain) the block estimates its pilot rows
// itself from the received DMRS samples and the pilots, with the same arithmetic as the LS
// kernels (ls_pilot), so the whole chain gives the bits of ranphy_chest_ls -> this detector.
//
// MFMA operand layouts (16x16x4, single block), lane l = 16 q + c:
//   A[i][kk] <- lane (i + 16 kk);  B[kk][j] <- lane (j + 16 kk);  D[i][j] -> lane (j + 16 (i/4)),
//   register i % 4.  The K index of step s is mapped to receive antenna 16 q + s, so that
//   each lane's 16 samples of one symbol are contiguous in memory.
#include <float.h>

#include <type_traits>

#include "geom.h"
#include "llr_math.h"
#include "rx_load.h"

namespace ranphy {
namespace {

typedef float floatx4 __attribute__((ext_vector_type(4)));
typedef _Float16 half8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

// Precision of the Gram and matched-filter products (inputs; accumulation is always FP32).
// The refined modes add one iterative-refinement step to the 16-bit products.
enum { kPrecF32 = 0, kPrecF16 = 1, kPrecBF16 = 2, kPrecF16R = 3, kPrecBF16R = 4 };

template <int PREC>
struct Lowp {
  static constexpr bool half = PREC == kPrecF16 || PREC == kPrecF16R;
  static constexpr bool refine = PREC == kPrecF16R || PREC == kPrecBF16R;
  using V = typename std::conditional<half, half8, bf16x8>::type;
  using E = typename std::conditional<half, _Float16, __bf16>::type;
};

constexpr int kXcds = 8;
// Condition estimate above which a subcarrier's system is solved again in FP64: the ratio
// of the largest to the smallest elimination pivot, (max L_ii / min L_ii)^2 of the Gram's
// Cholesky factor L.
constexpr float kCondMax = 1e6f;

// A pivot at or below this multiple of its original diagonal entry means the matrix is not
// numerically positive definite in that precision.
template <typename T>
struct PivotRel;
template <> struct PivotRel<float> { static constexpr float v = 16.f * FLT_EPSILON; };
template <> struct PivotRel<double> { static constexpr double v = 16.0 * DBL_EPSILON; };

__device__ __forceinline__ floatx4 mfma(float a, float b, floatx4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ floatx4 mfma(half8 a, half8 b, floatx4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_f16(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ floatx4 mfma(bf16x8 a, bf16x8 b, floatx4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}

// Eight FP32 values rounded to the MFMA input type (round to nearest even).
template <typename V, typename E>
__device__ __forceinline__ V pack8(const float* v, float sign) {
  V r;
#pragma unroll
  for (int e = 0; e < 8; ++e) r[e] = (E)(sign * v[e]);
  return r;
}

// Channel operands in a 16-bit input type for v_mfma_f32_16x16x32_{f16,bf16}: step t covers
// antennas 16 q + 8 t .. 16 q + 8 t + 7 of lane group q (both operands of every product use
// the same element order, so the K ordering inside an instruction does not matter).
template <typename V>
struct LowpH {
  V r[2], i[2];  // H real, imaginary
};

template <typename V, typename E>
__device__ __forceinline__ LowpH<V> pack_h(const float (&hr)[16], const float (&hi)[16]) {
  LowpH<V> o;
#pragma unroll
  for (int t = 0; t < 2; ++t) {
    o.r[t] = pack8<V, E>(hr + 8 * t, 1.f);
    o.i[t] = pack8<V, E>(hi + 8 * t, 1.f);
  }
  return o;
}

// The remainders of the same operands: x - (float)round16(x), rounded to the 16-bit type, so
// that x = hi + lo to 22 (FP16) or 16 (BF16) significant bits.
template <typename V, typename E>
__device__ __forceinline__ V pack8_lo(const float* v) {
  V r;
#pragma unroll
  for (int e = 0; e < 8; ++e) r[e] = (E)(v[e] - (float)(E)v[e]);
  return r;
}

template <typename V, typename E>
__device__ __forceinline__ LowpH<V> pack_h_lo(const float (&hr)[16], const float (&hi)[16]) {
  LowpH<V> o;
#pragma unroll
  for (int t = 0; t < 2; ++t) {
    o.r[t] = pack8_lo<V, E>(hr + 8 * t);
    o.i[t] = pack8_lo<V, E>(hi + 8 * t);
  }
  return o;
}

// A^H B of two channel operands (16 x 16 complex): the real part into re, the imaginary part
// as the difference im_p - im_n of two FP32 sums (the 16-bit operands are not negated).
template <typename V>
__device__ __forceinline__ void herm_cross(const LowpH<V>& a, const LowpH<V>& b, floatx4& re,
                                           floatx4& im_p, floatx4& im_n) {
#pragma unroll
  for (int t = 0; t < 2; ++t) {
    re = mfma(a.r[t], b.r[t], re);
    re = mfma(a.i[t], b.i[t], re);
    im_p = mfma(a.r[t], b.i[t], im_p);
    im_n = mfma(a.i[t], b.r[t], im_n);
  }
}

// K step t of Z += A^H Y for a channel operand A and received samples packed as (br, bi),
// with four products (no cancellation on top of the input rounding); Im Z = zi_p - zi_n.
template <typename V>
__device__ __forceinline__ void mf_step(const LowpH<V>& a, int t, const V& br, const V& bi,
                                        floatx4& zr, floatx4& zi_p, floatx4& zi_n) {
  zr = mfma(a.r[t], br, zr);
  zr = mfma(a.i[t], bi, zr);
  zi_p = mfma(a.r[t], bi, zi_p);
  zi_n = mfma(a.i[t], br, zi_n);
}

// Largest magnitude over the wave of the 32 values a lane holds: a per-lane maximum, then
// within each row of 16 lanes (DPP row_shr 1, 2, 4, 8; lanes without a source keep their
// value) and across rows (row_bcast 15 into rows 1 and 3, row_bcast 31 into rows 2 and 3),
// which leaves the wave's maximum in lane 63.  NaN is ignored (fmax).
template <int CTRL, int ROW_MASK>
__device__ __forceinline__ float dpp_max(float v) {
  return fmaxf(v, __int_as_float(__builtin_amdgcn_update_dpp(
                      __float_as_int(v), __float_as_int(v), CTRL, ROW_MASK, 0xF, false)));
}
__device__ __forceinline__ float wave_absmax(const float (&a)[16], const float (&b)[16]) {
  float m = 0.f;
#pragma unroll
  for (int s = 0; s < 16; ++s) m = fmaxf(m, fmaxf(fabsf(a[s]), fabsf(b[s])));
  m = dpp_max<0x111, 0xF>(m);
  m = dpp_max<0x112, 0xF>(m);
  m = dpp_max<0x114, 0xF>(m);
  m = dpp_max<0x118, 0xF>(m);
  m = dpp_max<0x142, 0xA>(m);
  m = dpp_max<0x143, 0xC>(m);
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(m), 63));
}

// FP16 operands are scaled by a power of two 2^e before rounding, e chosen from the wave's
// largest magnitude m so that m * 2^e lies in [2^13, 2^14).  Without refinement the scale is
// only applied when m lies outside [2^-2, 2^14) (e = 0 there: every operand then rounds to a
// normal FP16 value or is negligible against m); the refined modes always apply it, so that
// the remainders (2^-11 of their values) stay normal too.  A power of two commutes with every
// rounding while values stay normal, so scaled products, scaled back exactly, equal the
// unscaled ones wherever those are in range.  m = 0, infinite or NaN: e = 0.
template <bool ALWAYS>
__device__ __forceinline__ int f16_scale_exp(float m) {
  if (!(m > 0.f) || m > FLT_MAX) return 0;
  const int e = __builtin_amdgcn_frexp_expf(m) - 1;  // m in [2^e, 2^(e+1))
  return (!ALWAYS && e >= -2 && e < 14) ? 0 : 13 - e;
}

template <typename V>
__device__ __forceinline__ void gram_lowp(const LowpH<V>& a, floatx4& acc_g, floatx4& acc_p) {
#pragma unroll
  for (int t = 0; t < 2; ++t) {
    acc_g = mfma(a.r[t], a.r[t], acc_g);
    acc_g = mfma(a.i[t], a.i[t], acc_g);
    acc_p = mfma(a.r[t], a.i[t], acc_p);
  }
}

// Value of lane SRC of each row of 16 lanes (DPP row_newbcast; a VALU move, no LDS trip).
template <int SRC>
__device__ __forceinline__ float row_bcast(float v) {
  // Every lane reads a valid source lane, so bound_ctrl changes nothing; it lets the move be
  // emitted without first materialising an "old" value.
  return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), 0x150 + SRC, 0xF, 0xF, true));
}

// Value held by row group G (lanes 16 G .. 16 G + 15) at the same position in the row, for
// every row group: permlane16_swap(x, x) yields rows (x0,x0,x2,x2) and (x1,x1,x3,x3);
// permlane32_swap(e, e) of e = (a,a,b,b) yields (a,a,a,a) and (b,b,b,b).
template <int G>
__device__ __forceinline__ float group_bcast(float v) {
  const int x = __float_as_int(v);
  const auto p = __builtin_amdgcn_permlane16_swap(x, x, false, false);
  const int e = (G & 1) ? p[1] : p[0];
  const auto r = __builtin_amdgcn_permlane32_swap(e, e, false, false);
  return __int_as_float((G & 2) ? r[1] : r[0]);
}

__device__ __forceinline__ float lane_read(float v, int src_lane) {
  return __int_as_float(__builtin_amdgcn_ds_bpermute(src_lane << 2, __float_as_int(v)));
}

__device__ __forceinline__ float uniform_read(float v, int lane) {
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), lane));
}

// The same moves for FP64 values, one 32-bit half at a time.
__device__ __forceinline__ int lo32(double v) { return (int)(unsigned)__double_as_longlong(v); }
__device__ __forceinline__ int hi32(double v) { return (int)(__double_as_longlong(v) >> 32); }
__device__ __forceinline__ double join64(int lo, int hi) {
  return __longlong_as_double((long long)(((unsigned long long)(unsigned)hi << 32) | (unsigned)lo));
}
template <int SRC>
__device__ __forceinline__ double row_bcast(double v) {
  return join64(__builtin_amdgcn_mov_dpp(lo32(v), 0x150 + SRC, 0xF, 0xF, true),
                __builtin_amdgcn_mov_dpp(hi32(v), 0x150 + SRC, 0xF, 0xF, true));
}
__device__ __forceinline__ double lane_read(double v, int src_lane) {
  return join64(__builtin_amdgcn_ds_bpermute(src_lane << 2, lo32(v)),
                __builtin_amdgcn_ds_bpermute(src_lane << 2, hi32(v)));
}
__device__ __forceinline__ double uniform_read(double v, int lane) {
  return join64(__builtin_amdgcn_readlane(lo32(v), lane), __builtin_amdgcn_readlane(hi32(v), lane));
}

__device__ __forceinline__ float recip(float p) { return __builtin_amdgcn_rcpf(p); }
__device__ __forceinline__ double recip(double p) { return 1.0 / p; }

// ---- block floating point received grid (16-antenna blocks) --------------------------------
constexpr int kBfpWords = 10;  // exponent + 288 bits of mantissas
// Value f (0..31: I, Q of antenna f / 2) of a block held in w[0..9], w[0] the exponent.
template <int F>
__device__ __forceinline__ float bfp_value(const unsigned (&w)[kBfpWords]) {
  constexpr int bit = 9 * F, word = 1 + (bit >> 5), sh = bit & 31;
  unsigned m = w[word] >> sh;
  if constexpr (sh > 23) m |= w[word + 1] << (32 - sh);
  return ldexpf((float)((int)(m << 23) >> 23), (int)w[0]);
}
template <int F>
__device__ __forceinline__ void bfp_decode(const unsigned (&w)[kBfpWords], float (&yr)[16],
                                           float (&yi)[16]) {
  if constexpr (F < 16) {
    yr[F] = bfp_value<2 * F>(w);
    yi[F] = bfp_value<2 * F + 1>(w);
    bfp_decode<F + 1>(w, yr, yi);
  }
}
// Sample of antenna r (of NR, a multiple of 16) at resource element re of a BFP grid.
__device__ __forceinline__ float2 bfp_sample(const unsigned* __restrict__ words, int64_t re,
                                             int NR, int r) {
  const unsigned* b = words + (re * (NR >> 4) + (r >> 4)) * kBfpWords;
  const int i = r & 15, bit = 18 * i, word = 1 + (bit >> 5), sh = bit & 31;
  const unsigned long long f =
      (((unsigned long long)b[word + (sh > 14 ? 1 : 0)] << 32) | b[word]) >> sh;
  const int e = (int)b[0];
  return make_float2(ldexpf((float)((int)((unsigned)f << 23) >> 23), e),
                     ldexpf((float)((int)((unsigned)(f >> 9) << 23) >> 23), e));
}

// OUT = P^H Q for 16 x 16 complex P, Q held as lane (q, c) <- row 4q + s of column c in
// register s (P^H Q = P Q for a Hermitian P): the accumulator layout of P, conjugated, is
// the A-operand layout of P^H (A[c][4q+s] = conj(P[4q+s][c])) and the accumulator layout of
// Q is the B-operand layout.  Three real products:
//   Re = pr qr + pi qi,  Im = (pr - pi)(qr + qi) - pr qr + pi qi.
__device__ __forceinline__ void herm_mul(const float (&pr)[4], const float (&pi)[4],
                                         const floatx4& qr, const floatx4& qi, floatx4& outr,
                                         floatx4& outi) {
  floatx4 n1 = {0.f, 0.f, 0.f, 0.f}, n2 = n1, n3 = n1;
#pragma unroll
  for (int s = 0; s < 4; ++s) {
    n1 = mfma(pr[s], qr[s], n1);
    n2 = mfma(pi[s], qi[s], n2);
    n3 = mfma(pr[s] - pi[s], qr[s] + qi[s], n3);
  }
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    outr[v] = n1[v] + n2[v];
    outi[v] = n3[v] - n1[v] + n2[v];
  }
}

// dst += (src0 of lane K of the lane's row of 16) * src1; K is asm operand 10.
#define DPP_FMAC(dst, src0, src1) \
  "v_fmac_f32_dpp " dst ", " src0 ", " src1 " row_newbcast:%10 row_mask:0xf bank_mask:0xf bound_ctrl:1\n\t"

// One Gauss-Jordan step on pivot K, with the pivot-column scaling deferred.  Lane (q, c)
// holds R[4q+v][c] in (ar[v], ai[v]); the matrix of the textbook in-place elimination is
// A[i][j] = R[i][j] s_j, where s_j = 1 until column j has been the pivot column and
// s_j = -1/p_j afterwards.  One step on the stored values:
//   pivot row:     R[K][j]  <- R[K][j] / p      (j != K),   R[K][K] <- -1
//   pivot column:  unchanged (its scale becomes s_K = -1/p)
//   elsewhere:     R[i][j]  <- R[i][j] - R[i][K] R[K][j] / p
// Every other update is linear in each column, so a uniform column scale commutes with it.
// Each lane keeps s_c of its own column c in `scale`.  The pivots of the real layers are
// also tracked: pmin / pmax hold the bit patterns of the smallest and largest.
//
// The pivot tests run on the scalar unit, on bit patterns: the pivot p must exceed its
// threshold th (16 FLT_EPSILON times the original diagonal entry, rounded as an FP32
// product; th >= 0) and be finite.  For th >= 0 and p not NaN, p > th exactly when the
// patterns read as signed integers compare so (positive floats order as their patterns,
// negative ones read as negative integers); NaN and +inf have patterns at or above
// 0x7f800000 and fail (an infinite pivot only comes from an overflowed Gram).
template <int K>
__device__ __forceinline__ void gj_step(float (&ar)[4], float (&ai)[4], float& scale, int q,
                                        int c, int nl, const int (&thb)[16], bool& ok,
                                        unsigned& pmin, unsigned& pmax) {
  constexpr int KV = K & 3;
  constexpr int KQ = K >> 2;
  const unsigned pb = (unsigned)__builtin_amdgcn_readlane(__float_as_int(ar[KV]), 16 * KQ + K);
  const float p = __uint_as_float(pb);
  // A pivot that is not positive relative to its original diagonal entry means the matrix
  // is not numerically positive definite; padded layers carry an identity block.
  if (K < nl) {
    ok = ok && (int)pb > thb[K] && pb < 0x7f800000u;
    // scalar min / max (the compiler would fold pairs of them into vector min3 / max3)
    asm("s_min_u32 %0, %1, %2" : "=s"(pmin) : "s"(pmin), "s"(pb) : "scc");
    asm("s_max_u32 %0, %1, %2" : "=s"(pmax) : "s"(pmax), "s"(pb) : "scc");
  }
  const float pinv = __builtin_amdgcn_rcpf(p);
  // Row K at this lane's column c (row group K/4, register K%4), scaled; zero in the pivot
  // column so that the rank-1 update leaves that column untouched.
  const bool col_k = (c == K);
  const float rw = lane_read(ar[KV], 16 * KQ + c);  // ds_bpermute: no VALU work
  const float iw = lane_read(ai[KV], 16 * KQ + c);
  const float rr = col_k ? 0.f : rw * pinv;
  const float ri = col_k ? 0.f : iw * pinv;
  scale = col_k ? -pinv : scale;
  // Rank-1 update of every element, with the broadcast of the pivot column folded into the
  // multiply-adds (DPP row_newbcast on the first source of v_fmac_f32):
  //   R[i][j] += bcast(ai) ri - bcast(ar) rr      (real part)
  //   I[i][j] += -bcast(ai) rr - bcast(ar) ri     (imaginary part)
  // with bcast(.) the value of lane K of the lane's row of 16, i.e. R[4q+v][K].  Lane K holds
  // rr = ri = 0, so the broadcast sources never change during the update and each read sees
  // the step's starting values; the two products of each part are added in the order
  // fma(-cr, rr, fma(ci, ri, ar)) and fma(-cr, ri, fma(-ci, rr, ai)).  A VALU write followed
  // by a DPP read of the same register needs two wait states: the block starts with them
  // (values written just before it) and inside it every DPP source was written at least four
  // instructions earlier.
  asm volatile(
      "s_nop 1\n\t"
      DPP_FMAC("%0", "%4", "%8") DPP_FMAC("%1", "%5", "%8")
      DPP_FMAC("%2", "%6", "%8") DPP_FMAC("%3", "%7", "%8")
      DPP_FMAC("%4", "%4", "-%9") DPP_FMAC("%5", "%5", "-%9")
      DPP_FMAC("%6", "%6", "-%9") DPP_FMAC("%7", "%7", "-%9")
      DPP_FMAC("%0", "%0", "-%9") DPP_FMAC("%1", "%1", "-%9")
      DPP_FMAC("%2", "%2", "-%9") DPP_FMAC("%3", "%3", "-%9")
      DPP_FMAC("%4", "%0", "-%8") DPP_FMAC("%5", "%1", "-%8")
      DPP_FMAC("%6", "%2", "-%8") DPP_FMAC("%7", "%3", "-%8")
      : "+v"(ar[0]), "+v"(ar[1]), "+v"(ar[2]), "+v"(ar[3]), "+v"(ai[0]), "+v"(ai[1]),
        "+v"(ai[2]), "+v"(ai[3])
      : "v"(ri), "v"(rr), "n"(K));
  if (q == KQ) {  // pivot row (4q + v == K only for v == K % 4)
    ar[KV] = col_k ? -1.f : rr;
    ai[KV] = ri;
  }
}

template <int K>
__device__ __forceinline__ void gj_all(float (&ar)[4], float (&ai)[4], float& scale, int q,
                                       int c, int nl, const int (&thb)[16], bool& ok,
                                       unsigned& pmin, unsigned& pmax) {
  if constexpr (K < 16) {
    gj_step<K>(ar, ai, scale, q, c, nl, thb, ok, pmin, pmax);
    gj_all<K + 1>(ar, ai, scale, q, c, nl, thb, ok, pmin, pmax);
  }
}

// Bit patterns of the pivot thresholds 16 FLT_EPSILON G[K][K] (G[K][K] is register K % 4 of
// lane 16 (K / 4) + K), read onto the scalar unit.
template <int K>
__device__ __forceinline__ void read_thresholds(const float (&th)[4], int (&thb)[16]) {
  if constexpr (K < 16) {
    thb[K] = __builtin_amdgcn_readlane(__float_as_int(th[K & 3]), 16 * (K >> 2) + K);
    read_thresholds<K + 1>(th, thb);
  }
}

__device__ __forceinline__ double pick4(const double (&a)[4], int i) {
  return i == 0 ? a[0] : i == 1 ? a[1] : i == 2 ? a[2] : a[3];
}

// The same Gauss-Jordan inversion in FP64, with the pivot index a runtime (wave-uniform)
// loop variable and every cross-lane move a ds_bpermute or readlane.  Only the NL real
// pivots are eliminated; the padded identity block is its own inverse.  Leaves G^-1[4q+v][c]
// in (ar[v], ai[v]).
template <int NL>
__device__ __forceinline__ void gj_f64(double (&ar)[4], double (&ai)[4], int q, int c,
                                       bool& ok) {
  // Original diagonal entry of this lane's column: G[c][c] is register c % 4 of lane (c/4, c).
  const double dg = lane_read(pick4(ar, c & 3), 16 * (c >> 2) + c);
  double scale = 1.0;
#pragma unroll 1
  for (int K = 0; K < NL; ++K) {
    const int KV = K & 3, KQ = K >> 2;
    const double p = uniform_read(pick4(ar, KV), 16 * KQ + K);
    ok = ok && p > PivotRel<double>::v * uniform_read(dg, K);
    const double pinv = 1.0 / p;
    const bool col_k = (c == K);
    const double rw = lane_read(pick4(ar, KV), 16 * KQ + c);
    const double iw = lane_read(pick4(ai, KV), 16 * KQ + c);
    const double rr = col_k ? 0.0 : rw * pinv;
    const double ri = col_k ? 0.0 : iw * pinv;
    scale = col_k ? -pinv : scale;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const double cr = lane_read(ar[v], 16 * q + K);  // R[4q+v][K]
      const double ci = lane_read(ai[v], 16 * q + K);
      double nr = fma(-cr, rr, fma(ci, ri, ar[v]));
      double ni = fma(-cr, ri, fma(-ci, rr, ai[v]));
      if (v == KV && q == KQ) {
        nr = col_k ? -1.0 : rr;
        ni = ri;
      }
      ar[v] = nr;
      ai[v] = ni;
    }
  }
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    ar[v] *= scale;
    ai[v] *= scale;
  }
}

// The FP64 route for one subcarrier (a wave): Gram, Gauss-Jordan inverse, matched filter,
// solve and unbiasing in FP64 from the same FP32 channel rows and received samples, giving
// the outputs of layers 4q .. 4q+3 of data symbol d = c in the lane's xo / vo.  The channel
// is interpolated in FP64 as (1 - a) v0 + a v1 between the port's two staged pilot rows
// (a, a multiple of 1/C, is exact in FP32).  Rolled loops and cross-lane reads keep it
// within the FP32 path's registers: it runs only for the rare subcarriers whose FP32
// condition estimate exceeds kCondMax (or whose FP32 elimination failed).
template <int HRES, int NL, int RXF>
__device__ __forceinline__ void solve_f64(const Geom& g, const float2* rows, int jlo, int k0,
                                          int k, int slot, const float2* __restrict__ rx,
                                          float s2f, int q, int c, float (&xo)[8],
                                          float (&vo)[4]) {
  const int NR = g.n_rx, ND = g.n_dsym;
  const double s2 = s2f;
  // Layers this lane needs: 4q .. 4q+3 (v = 0..3: rows of G and Z) and c (v = 4: column of
  // G); padded layers read layer NL-1 and are replaced below.  Row pointers at antenna 0.
  const float2* b0[5];
  const float2* b1[5];
  float wa[5];
#pragma unroll
  for (int v = 0; v < 5; ++v) {
    int l = v < 4 ? 4 * q + v : c;
    l = l < NL ? l : NL - 1;
    int r0 = k - k0, r1 = r0;
    float af = 0.f;
    if (HRES == 0) {
      int j0, j1;
      freq_rule(g, l, k, j0, j1, af);
      r0 = j0 - jlo;
      r1 = j1 - jlo;
    }
    b0[v] = rows + r0 * NR * NL + l;
    b1[v] = rows + r1 * NR * NL + l;
    wa[v] = af;
  }
  auto chan = [&](int v, int r, double& re, double& im) {
    const float2 v0 = b0[v][r * NL];
    const float2 v1 = b1[v][r * NL];
    const double w = wa[v];
    re = (1.0 - w) * (double)v0.x + w * (double)v1.x;
    im = (1.0 - w) * (double)v0.y + w * (double)v1.y;
  };
  // Gram column c, rows 4q .. 4q+3: G[i][c] = sum_r conj(H[r][i]) H[r][c] + s2 delta.
  double ar[4] = {0, 0, 0, 0}, ai[4] = {0, 0, 0, 0};
#pragma unroll 1
  for (int r = 0; r < NR; ++r) {
    double cr, ci;
    chan(4, r, cr, ci);
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      double hr, hi;
      chan(v, r, hr, hi);
      ar[v] = fma(hr, cr, fma(hi, ci, ar[v]));
      ai[v] = fma(hr, ci, fma(-hi, cr, ai[v]));
    }
  }
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    const int i = 4 * q + v;
    const bool in = (i < NL) && (c < NL);
    ar[v] = in ? ar[v] + ((i == c) ? s2 : 0.0) : ((i == c) ? 1.0 : 0.0);
    ai[v] = in ? ai[v] : 0.0;
  }
  bool ok = true;
  gj_f64<NL>(ar, ai, q, c, ok);
  // Matched filter for data symbol d = c (clamped), layers 4q .. 4q+3.  The lane index is
  // passed through an empty asm so that the sample address is recomputed here rather than
  // shared with (and kept alive from) the FP32 route's loads of the same row.
  int cl = c;
  asm volatile("" : "+v"(cl));
  const int d = cl < ND ? cl : ND - 1;
  const int sym = (d < g.sym0[0]) ? d : d + g.td;  // one occasion: skip its T DMRS symbols
  const int64_t re = (int64_t)(slot * g.n_symb + sym) * g.n_sc + k;
  const float2* __restrict__ y = rx + re * NR;
  double zr[4] = {0, 0, 0, 0}, zi[4] = {0, 0, 0, 0};
#pragma unroll 1
  for (int r = 0; r < NR; ++r) {
    const float2 yy =
        RXF == 0 ? y[r] : bfp_sample(reinterpret_cast<const unsigned*>(rx), re, NR, r);
    const double yr = yy.x, yi = yy.y;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      double hr, hi;
      chan(v, r, hr, hi);
      zr[v] = fma(hr, yr, fma(hi, yi, zr[v]));
      zi[v] = fma(hr, yi, fma(-hi, yr, zi[v]));
    }
  }
  // X[4q+v][d] = sum_m G^-1[4q+v][m] Z[m][d]: G^-1[4q+v][m] is register v of lane (q, m),
  // Z[m][d] register m % 4 of lane (m / 4, d).
  double xr[4] = {0, 0, 0, 0}, xi[4] = {0, 0, 0, 0};
#pragma unroll 1
  for (int m = 0; m < NL; ++m) {
    const int mv = m & 3;
    const double zmr = mv == 0 ? zr[0] : mv == 1 ? zr[1] : mv == 2 ? zr[2] : zr[3];
    const double zmi = mv == 0 ? zi[0] : mv == 1 ? zi[1] : mv == 2 ? zi[2] : zi[3];
    const double br = lane_read(zmr, 16 * (m >> 2) + c);
    const double bi = lane_read(zmi, 16 * (m >> 2) + c);
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const double gr = lane_read(ar[v], 16 * q + m);
      const double gi = lane_read(ai[v], 16 * q + m);
      xr[v] = fma(gr, br, fma(-gi, bi, xr[v]));
      xi[v] = fma(gr, bi, fma(gi, br, xi[v]));
    }
  }
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    const double dl = lane_read(ar[v], 16 * q + 4 * q + v);  // G^-1[4q+v][4q+v]
    const double sd = s2 * dl;
    const double mu = 1.0 - sd;
    xo[2 * v] = ok ? (float)(xr[v] / mu) : __builtin_nanf("");
    xo[2 * v + 1] = ok ? (float)(xi[v] / mu) : __builtin_nanf("");
    vo[v] = ok ? (float)(sd / mu) : __builtin_inff();
  }
}

// Max-log LLRs of the 4 layers 4q .. 4q+3 a lane holds, written to their 4 Qm contiguous
// floats (16-byte stores when all 4 layers exist; llr 16-byte aligned).
template <int QM, int NL>
__device__ __forceinline__ void store_llr(float* __restrict__ dst, const float (&out)[4 * QM],
                                          int q) {
  if (NL % 4 == 0) {
    float4* __restrict__ d4 = reinterpret_cast<float4*>(dst);
#pragma unroll
    for (int i = 0; i < QM; ++i)
      d4[i] = make_float4(out[4 * i], out[4 * i + 1], out[4 * i + 2], out[4 * i + 3]);
  } else {
#pragma unroll
    for (int v = 0; v < 4; ++v)
      if (4 * q + v < NL) {
#pragma unroll
        for (int b = 0; b < QM; ++b) dst[v * QM + b] = out[v * QM + b];
      }
  }
}

// The fused demapping epilogue.  Lane (q, d) computes the LLRs of layers 4q .. 4q+3 of data
// symbol d; the Nl Qm LLRs of one RE are contiguous in the output, and the wave's ND REs are
// n_sc Nl Qm floats apart.  Written straight from the lanes, each store instruction touches
// 64 scattered 16-byte pieces.  With kStaged the wave instead stages its ND x Nl Qm block in
// LDS (its quarter of the channel-row buffer, free once every wave of the block is past the
// channel reads) and writes it back with consecutive lanes on consecutive 16-byte (8-byte
// when Nl Qm is not a multiple of 4) pieces of each RE's run; blocks whose ND x Nl Qm block
// does not fit their quarter store straight from the lanes.  Staging pays off where the
// detector itself is short (16-bit Gram and matched filter); with the FP32 products the
// extra LDS round trip and barrier cost more than the scattered stores (measured).  Called
// by every lane of the block (the barrier), with block-uniform qm, ND and live.
template <int QM, int NL, int kStage, bool kStaged>
__device__ __forceinline__ void emit_llr(float* __restrict__ llr, float* stage, int64_t seg0,
                                         int64_t dstride, int64_t o, const float (&xo)[8],
                                         const float (&vo)[4], int q, int d, int ND, bool mine,
                                         bool live) {
  float out[4 * QM];
#pragma unroll
  for (int v = 0; v < 4; ++v) llr_one<QM>(make_float2(xo[2 * v], xo[2 * v + 1]), vo[v], out + v * QM);
  constexpr int kRe = NL * QM;  // floats per RE
  if (!kStaged || ND * kRe > kStage) {
    if (mine) store_llr<QM, NL>(llr + (o + 4 * q) * QM, out, q);
    return;
  }
  __syncthreads();  // every wave of the block is done with the channel rows
  if (mine) {
    float* dst = stage + d * kRe + 4 * q * QM;
    if (kRe % 4 == 0) {
#pragma unroll
      for (int i = 0; i < QM; ++i)
        if (NL % 4 == 0 || 4 * i < (NL - 4 * q) * QM)
          reinterpret_cast<float4*>(dst)[i] =
              make_float4(out[4 * i], out[4 * i + 1], out[4 * i + 2], out[4 * i + 3]);
    } else {
#pragma unroll
      for (int i = 0; i < 2 * QM; ++i)
        if (2 * i < (NL - 4 * q) * QM)
          reinterpret_cast<float2*>(dst)[i] = make_float2(out[2 * i], out[2 * i + 1]);
    }
  }
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  if (!live) return;
  // Lane L takes pieces L, L + 64, ..: piece f is piece f mod kCh of RE f / kCh.
  using Piece = typename std::conditional<kRe % 4 == 0, float4, float2>::type;
  constexpr int kW = sizeof(Piece) / sizeof(float);
  constexpr int kCh = kRe / kW;  // pieces per RE
  const int n = ND * kCh;
  for (int f = d + 16 * q; f < n; f += 64) {
    const int dd = f / kCh, m = f - dd * kCh;
    reinterpret_cast<Piece*>(llr + (seg0 + dd * dstride) * QM)[m] =
        reinterpret_cast<const Piece*>(stage)[f];
  }
}

template <int HRES, int NL, int PREC, int RXF, int LSF>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(Lowp<PREC>::refine ? 3 : 5, 8))) mmse_mfma_kernel(Geom g, const float2* __restrict__ rx,
                                                        const float2* __restrict__ h,
                                                        const float2* __restrict__ pil,
                                                        const float* __restrict__ nvar,
                                                        float2* __restrict__ x,
                                                        float* __restrict__ nv,
                                                        float* __restrict__ llr) {
  __shared__ __attribute__((aligned(16))) float lds_t[4][16 * 17];
  // Channel rows staged per block: full resolution needs the 4 subcarriers' rows; at pilot
  // resolution 9..16 layers imply comb 8 (Nl <= C T), whose 4 subcarriers span at most 3
  // pilot rows, and 5..8 layers at most 4 (comb 4).
  constexpr int kRows = (HRES == 1 || NL <= 8) ? 4 : 3;
  __shared__ __attribute__((aligned(16))) float2 lds_h[kRows * kMaxRx * NL];
  const int wave = threadIdx.x >> 6;
  const int lane = threadIdx.x & 63;
  const int q = lane >> 4;  // K group / accumulator row group
  const int c = lane & 15;  // layer (A/B operands), column (accumulators)
  const int NR = g.n_rx, ND = g.n_dsym;

  // Blocks are dispatched round-robin over the 8 XCDs; give each XCD a contiguous run of
  // subcarriers so that its L2 reads every pilot of the run once.  All per-wave indices are
  // wave-uniform (kept in scalar registers).
  const int total = g.n_slots * g.n_sc;
  const int per_xcd = gridDim.x / kXcds;
  int blk = (int)(blockIdx.x % kXcds) * per_xcd + (int)(blockIdx.x / kXcds);
  const bool live = blk * 4 < total;  // total is a multiple of 4 (12 subcarriers per PRB)
  if (!live) blk = total / 4 - 1;     // dead blocks mirror the last block and store nothing
  const int sid = __builtin_amdgcn_readfirstlane(blk * 4 + wave);
  const int slot = __builtin_amdgcn_readfirstlane(sid / g.n_sc);
  const int k = __builtin_amdgcn_readfirstlane(sid - slot * g.n_sc);
  const int nq = NR >> 4;       // lane groups that carry antennas
  const bool qv = q < nq;
  const int qc = qv ? q : nq - 1;  // clamped: every address below is in bounds

  // ---- 1. the block's channel rows, staged once in LDS -------------------------------------
  // The 4 waves take subcarriers k0 .. k0+3 of one slot (n_sc is a multiple of 4).  With a
  // pilot-resolution estimate they need pilot rows jlo .. jhi only (at most 4 for comb 2,
  // 3 for comb 8); with a full-resolution one, rows k0 .. k0+3.  A row [rx][layer] is
  // contiguous, so the copy is one contiguous run read with 16-byte loads.
  const int k0 = k - wave;
  int jlo, nrow;
  if (HRES == 0) {
    const int C = g.comb, L = g.comb_log2;
    jlo = (k0 + 1 - C) < 0 ? 0 : ((k0 + 1 - C) >> L);
    const int jhi = min(g.n_pilot - 1, ((k0 + 3) >> L) + 1);
    nrow = jhi - jlo + 1;
  } else {
    jlo = k0;
    nrow = 4;
  }
  if constexpr (LSF == 0) {
    const int row_f4 = (NR * NL) >> 1;
    const int64_t row0 = (int64_t)slot * (HRES == 0 ? g.n_pilot : g.n_sc) + jlo;
    const float4* __restrict__ src = reinterpret_cast<const float4*>(h + row0 * NR * NL);
    float4* __restrict__ dst = reinterpret_cast<float4*>(lds_h);
    const int n4 = nrow * row_f4;
    for (int f = threadIdx.x; f < n4; f += 256) dst[f] = src[f];
  } else {
    // Rows jlo .. jlo + nrow - 1 estimated here.  The block's pilots go to LDS first (into
    // lds_t, free until the Gram transpose); thread (group gg, antenna r) then issues all of
    // its received-sample loads (the T DMRS samples of subcarrier C j + c, at most kItems
    // groups) before it forms, for every port on that comb offset, the estimate ranphy_chest_ls
    // would write (zero past the band edge).  More than 8 layers imply comb 8 and T = 2, so a
    // thread has at most nrow C NR / 256 <= 2 kRows groups.
    const int C = g.comb, T = g.td;
    const int npq = nrow * T * NL;
    float2* __restrict__ pst = reinterpret_cast<float2*>(&lds_t[0][0]);
    for (int e = threadIdx.x; e < npq; e += 256) {
      const int row = e / (T * NL), rem = e - row * (T * NL);
      const int t = rem / NL, p = rem - t * NL;
      pst[e] = pil[(((int64_t)slot * T + t) * g.n_pilot + jlo + row) * NL + p];
    }
    constexpr int kItems = 2 * kRows;
    // gs whole groups of NR threads (NR <= 64); with 48 antennas the last 16 threads idle
    const int r = threadIdx.x % NR, gs = 256 / NR, g0 = threadIdx.x / NR;
    const int64_t sym_re = ((int64_t)slot * g.n_symb + g.sym0[0]) * g.n_sc;
    // Only rows some subcarrier of the block interpolates from are formed: for comb offset c
    // (shared by its ports), pilots j0 at k0 .. j1 at k0 + 3 (the rule is monotone in k); the
    // rows left out are read by no wave of the block, the FP64 route included.
    auto needed = [&](int gg) {
      const int cc = gg & (C - 1), j = jlo + (gg >> g.comb_log2);
      int ja, jb, jc, jd;
      float a;
      freq_rule(g, cc, k0, ja, jb, a);
      freq_rule(g, cc, k0 + 3, jc, jd, a);
      return j >= ja && j <= jd;
    };
    float2 ys[kItems][2];
#pragma unroll
    for (int it = 0; it < kItems; ++it) {
      const int gg = g0 + it * gs;
      ys[it][0] = ys[it][1] = make_float2(0.f, 0.f);
      if (g0 < gs && gg < nrow * C && needed(gg)) {
        const int kc = min(C * (jlo + (gg >> g.comb_log2)) + (gg & (C - 1)), g.n_sc - 1);
        ys[it][0] = rx_at<RXF>(rx, sym_re + kc, NR, r);
        if (T == 2) ys[it][1] = rx_at<RXF>(rx, sym_re + g.n_sc + kc, NR, r);
      }
    }
    __syncthreads();  // the pilots are staged
#pragma unroll
    for (int it = 0; it < kItems; ++it) {
      const int gg = g0 + it * gs;
      if (g0 < gs && gg < nrow * C && needed(gg)) {
        const int row = gg >> g.comb_log2, cc = gg & (C - 1);
        const bool in = C * (jlo + row) + cc < g.n_sc;
        for (int p = cc; p < NL; p += C) {
          float2 v = make_float2(0.f, 0.f);
          if (in) {
            const float2* pq = pst + row * T * NL + p;
            if (T == 1) {
              const float2 q1[1] = {pq[0]}, y1[1] = {ys[it][0]};
              v = ls_pilot<1>(q1, y1);
            } else {
              const float2 q2[2] = {pq[0], pq[NL]}, y2[2] = {ys[it][0], ys[it][1]};
              v = ls_pilot<2>(q2, y2);
            }
          }
          lds_h[(row * NR + r) * NL + p] = v;
        }
      }
    }
  }
  __syncthreads();

  // ---- 2. received samples: issued now, consumed only after the inversion ---------------
  // Lane (q, d = c): antennas 16 q .. 16 q + 15 of data symbol d (128 B).  Symbols past ND
  // read symbol ND-1; their Z columns are never stored.  The Gram and the inversion need
  // only the channel, so this load's latency is hidden behind them.  (Issued after the
  // block's channel copy, which every wave of the block waits for.)
  float4 yv[8];
  unsigned yw[kBfpWords];  // RXF = 1: the lane's block, decoded before the matched filter
  {
    const int d = c < ND ? c : ND - 1;
    const int s = (d < g.sym0[0]) ? d : d + g.td;  // one occasion: skip its T DMRS symbols
    const int64_t re = (int64_t)(slot * g.n_symb + s) * g.n_sc + k;
    if constexpr (RXF == 0) {
      const float4* __restrict__ src = reinterpret_cast<const float4*>(rx + re * NR + 16 * qc);
#pragma unroll
      for (int i = 0; i < 8; ++i) yv[i] = src[i];
    } else {
      const uint2* __restrict__ src = reinterpret_cast<const uint2*>(
          reinterpret_cast<const unsigned*>(rx) + (re * (NR >> 4) + qc) * kBfpWords);
#pragma unroll
      for (int i = 0; i < kBfpWords / 2; ++i) {
        const uint2 v = src[i];
        yw[2 * i] = v.x;
        yw[2 * i + 1] = v.y;
      }
    }
  }
  const float s2 = nvar[slot];


  // Channel, lane (q, p = c), step s: antenna 16 q + s.  Layers past NL read layer NL-1; the
  // Gram rows and columns they produce are replaced by an identity block below.
  float hr[16], hi[16];
  {
    const int pc = c < NL ? c : NL - 1;
    float a = 0.f;
    int r0 = k - k0, r1 = r0;
    if (HRES == 0) {
      int j0, j1;
      freq_rule(g, pc, k, j0, j1, a);
      r0 = j0 - jlo;
      r1 = j1 - jlo;
    }
    const float2* __restrict__ b0 = lds_h + (r0 * NR + 16 * qc) * NL + pc;
    const float2* __restrict__ b1 = lds_h + (r1 * NR + 16 * qc) * NL + pc;
#pragma unroll
    for (int s = 0; s < 16; ++s) {
      const float2 v0 = b0[s * NL];
      if (HRES == 0) {
        const float2 v1 = b1[s * NL];
        hr[s] = fmaf(a, v1.x - v0.x, v0.x);
        hi[s] = fmaf(a, v1.y - v0.y, v0.y);
      } else {
        hr[s] = v0.x;
        hi[s] = v0.y;
      }
    }
  }
  if (nq < 4) {  // wave-uniform: only fewer than 64 antennas need masking
    if (!qv) {  // antenna groups past NR contribute nothing
#pragma unroll
      for (int s = 0; s < 16; ++s) hr[s] = hi[s] = 0.f;
    }
  }

  // ---- 3. Gram on the matrix cores ---------------------------------------------------------
  // FP32: two real products, P = Hr^T Hi and D = (Hr - Hi)^T (Hr - Hi) = Hr^T Hr + Hi^T Hi -
  // P - P^T, so that Re G = D + (P + P^T) and Im G = P - P^T (P^T from the LDS transpose
  // below).  16-bit inputs: acc_g = Hr^T Hr + Hi^T Hi and P directly (no difference of the
  // rounded operands).
  floatx4 acc_g = {0.f, 0.f, 0.f, 0.f}, acc_p = acc_g, z_r = acc_g, z_i = acc_g;
  using LV = typename Lowp<PREC>::V;
  using LE = typename Lowp<PREC>::E;
  LowpH<LV> hh, hl;      // 16-bit channel operands and (refined modes) their remainders
  floatx4 dg_r = acc_g, dg_i = acc_g;  // refined modes: H_hi^H H_lo + H_lo^H H_hi
  int eh = 0;            // FP16: the channel operands' power-of-two scale
  if constexpr (PREC == kPrecF32) {
#pragma unroll
    for (int s = 0; s < 16; ++s) {
      const float hd = hr[s] - hi[s];
      acc_g = mfma(hd, hd, acc_g);
      acc_p = mfma(hr[s], hi[s], acc_p);
    }
  } else {
    if constexpr (Lowp<PREC>::half) {
      eh = f16_scale_exp<Lowp<PREC>::refine>(wave_absmax(hr, hi));
      if (eh != 0) {
#pragma unroll
        for (int s = 0; s < 16; ++s) {
          hr[s] = ldexpf(hr[s], eh);
          hi[s] = ldexpf(hi[s], eh);
        }
      }
    }
    hh = pack_h<LV, LE>(hr, hi);
    gram_lowp(hh, acc_g, acc_p);
    if constexpr (Lowp<PREC>::refine) hl = pack_h_lo<LV, LE>(hr, hi);
    if (eh != 0) {
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        acc_g[v] = ldexpf(acc_g[v], -2 * eh);
        acc_p[v] = ldexpf(acc_p[v], -2 * eh);
      }
    }
  }

  // ---- 4. G = Re + j (P - P^T) + s2 I, padded layers -> identity; invert in place ---------
  float* __restrict__ tp = lds_t[wave];
#pragma unroll
  for (int v = 0; v < 4; ++v) tp[(4 * q + v) * 17 + c] = acc_p[v];
  // Only this wave reads what it wrote: order the LDS accesses within the wave.
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  float ar[4], ai[4];
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    const int i = 4 * q + v;
    const bool in = (i < NL) && (c < NL);
    const float pt = tp[c * 17 + i];  // P[c][i]
    // P[i][c] + P[c][i] is the same sum for (i, c) and (c, i), so Re G stays symmetric
    const float re = PREC == kPrecF32 ? acc_g[v] + (acc_p[v] + pt) : acc_g[v];
    ar[v] = in ? re + ((i == c) ? s2 : 0.f) : ((i == c) ? 1.f : 0.f);
    ai[v] = in ? acc_p[v] - pt : 0.f;
  }
  int thb[16];
  {
    float th[4];
#pragma unroll
    for (int v = 0; v < 4; ++v) th[v] = PivotRel<float>::v * ar[v];
    read_thresholds<0>(th, thb);
  }
  bool ok = true;
  float scale = 1.f;
  unsigned pmin = 0xFFFFFFFFu, pmax = 0u;
  gj_all<0>(ar, ai, scale, q, c, NL, thb, ok, pmin, pmax);
  // Subcarriers whose system is too ill-conditioned for FP32 (or not numerically positive
  // definite in FP32) are solved again in FP64 once the FP32 solution is done (the decision
  // is uniform over the wave; placed after the FP32 route, the FP64 route's registers do not
  // compete with it).
  const bool f64 = !ok || __uint_as_float(pmax) > kCondMax * __uint_as_float(pmin);
  float xo[8], vo[4];
  {
    // Apply the deferred column scales: lane (q, c) now holds G^-1[4q+v][c].
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      ar[v] *= scale;
      ai[v] *= scale;
    }
    // Keep the matched filter (the first use of the received samples) after the inversion.
    __builtin_amdgcn_sched_barrier(0);

    // ---- 5. matched filter Z = H^H Y on the matrix cores ----------------------------------
    {
      float yr[16], yi[16];
      if constexpr (RXF == 0) {
#pragma unroll
        for (int i = 0; i < 8; ++i) {
          yr[2 * i] = yv[i].x;
          yi[2 * i] = yv[i].y;
          yr[2 * i + 1] = yv[i].z;
          yi[2 * i + 1] = yv[i].w;
        }
      } else {
        bfp_decode<0>(yw, yr, yi);
      }
      if constexpr (PREC == kPrecF32) {
        // Three real products (conj(a) b, a = hr + j hi, b = yr + j yi):
        //   m1 = hr yr,  m2 = hi yi,  m3 = (hr + hi)(yr - yi);  Re = m1 + m2,  Im = m1 - m2 - m3.
        // (hr + hi rather than the Gram's hr - hi: nothing of the Gram's operands stays live
        // across the inversion.)
        floatx4 acc_m1 = acc_g, acc_m2 = acc_g, acc_m3 = acc_g;
#pragma unroll
        for (int v = 0; v < 4; ++v) acc_m1[v] = acc_m2[v] = acc_m3[v] = 0.f;
#pragma unroll
        for (int s = 0; s < 16; ++s) {
          acc_m1 = mfma(hr[s], yr[s], acc_m1);
          acc_m2 = mfma(hi[s], yi[s], acc_m2);
          acc_m3 = mfma(hr[s] + hi[s], yr[s] - yi[s], acc_m3);
        }
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          z_r[v] = acc_m1[v] + acc_m2[v];
          z_i[v] = acc_m1[v] - acc_m2[v] - acc_m3[v];
        }
      } else {
        int ey = 0;  // FP16: the samples' power-of-two scale
        if constexpr (Lowp<PREC>::half) {
          ey = f16_scale_exp<Lowp<PREC>::refine>(wave_absmax(yr, yi));
          if (ey != 0) {
#pragma unroll
            for (int s = 0; s < 16; ++s) {
              yr[s] = ldexpf(yr[s], ey);
              yi[s] = ldexpf(yi[s], ey);
            }
          }
        }
        // One K step at a time (8 antennas per lane), so that few packed samples are live.
        // Refined modes: H^H y of the FP32 operands to first order, Z~ + H_hi^H y_lo +
        // H_lo^H y_hi.
        floatx4 zi_n = z_i;
#pragma unroll
        for (int t = 0; t < 2; ++t) {
          const LV br = pack8<LV, LE>(yr + 8 * t, 1.f);
          const LV bi = pack8<LV, LE>(yi + 8 * t, 1.f);
          mf_step(hh, t, br, bi, z_r, z_i, zi_n);
          if constexpr (Lowp<PREC>::refine) {
            mf_step(hh, t, pack8_lo<LV, LE>(yr + 8 * t), pack8_lo<LV, LE>(yi + 8 * t), z_r, z_i,
                    zi_n);
            mf_step(hl, t, br, bi, z_r, z_i, zi_n);
          }
        }
#pragma unroll
        for (int v = 0; v < 4; ++v) z_i[v] -= zi_n[v];
        if (eh + ey != 0) {
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            z_r[v] = ldexpf(z_r[v], -(eh + ey));
            z_i[v] = ldexpf(z_i[v], -(eh + ey));
          }
        }
        if constexpr (Lowp<PREC>::refine) {
          // The Gram of the FP32 operands to first order: H^H H = G~ + dG + (H_lo^H H_lo)
          // (formed here rather than before the inversion: fewer registers live across it).
          floatx4 dg_n = dg_i;
          herm_cross(hh, hl, dg_r, dg_i, dg_n);
          herm_cross(hl, hh, dg_r, dg_i, dg_n);
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            // padded layers (copies of layer NL-1) carry an identity block: no correction
            const bool in = (4 * q + v < NL) && (c < NL);
            dg_r[v] = in ? ldexpf(dg_r[v], -2 * eh) : 0.f;
            dg_i[v] = in ? ldexpf(dg_i[v] - dg_n[v], -2 * eh) : 0.f;
          }
        }
      }
    }

    // ---- 6. X_hat = G^-1 Z on the matrix cores (G^-1 Hermitian) --------------------------
    floatx4 acc_xr, acc_xi;
    herm_mul(ar, ai, z_r, z_i, acc_xr, acc_xi);

    // ---- 7. unbias: lane (q, d = c) holds layers 4q .. 4q+3 of data symbol d ------------
    float dl[4];
#pragma unroll
    for (int v = 0; v < 4; ++v) dl[v] = lane_read(ar[v], 16 * q + 4 * q + v);  // G^-1[4q+v][4q+v]
    if constexpr (Lowp<PREC>::refine) {
      // One refinement step.  With G~ the 16-bit Gram (+ s2 I) that was inverted and
      // G = G~ + dG the Gram of the FP32 operands, the residual of x^ = G~^-1 Z is
      // Z - G x^ = -dG x^ (Z already the FP32 matched filter to first order), so
      //   x^ <- x^ - G~^-1 dG x^   and, to the same order,   diag(G^-1) = diag(G~^-1) -
      //   diag(G~^-1 dG G~^-1).   With N = dG G~^-1 (dG Hermitian), G~^-1 dG = N^H.
      floatx4 nr, ni, cr, ci;
      float dgr[4], dgi[4], nrr[4], nri[4];
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        dgr[v] = dg_r[v];
        dgi[v] = dg_i[v];
      }
      floatx4 gr, gi;
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        gr[v] = ar[v];
        gi[v] = ai[v];
      }
      herm_mul(dgr, dgi, gr, gi, nr, ni);
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        nrr[v] = nr[v];
        nri[v] = ni[v];
      }
      herm_mul(nrr, nri, acc_xr, acc_xi, cr, ci);
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        acc_xr[v] -= cr[v];
        acc_xi[v] -= ci[v];
      }
      // diag(N^H G~^-1)[l] = sum_n conj(N[n][l]) G~^-1[n][l]: column l of both, which lanes
      // (q, c = l) hold in rows 4q..4q+3; summed over the four row groups.
      float part = 0.f;
#pragma unroll
      for (int v = 0; v < 4; ++v) part = fmaf(nrr[v], ar[v], fmaf(nri[v], ai[v], part));
      part += lane_read(part, lane ^ 32);
      part += lane_read(part, lane ^ 16);
#pragma unroll
      for (int v = 0; v < 4; ++v) dl[v] -= lane_read(part, 16 * q + 4 * q + v);
    }
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const float sd = s2 * dl[v];
      const float im = __builtin_amdgcn_rcpf(1.f - sd);
      xo[2 * v] = acc_xr[v] * im;
      xo[2 * v + 1] = acc_xi[v] * im;
      vo[v] = sd * im;
    }
  }
  if (f64) solve_f64<HRES, NL, RXF>(g, lds_h, jlo, k0, k, slot, rx, s2, q, c, xo, vo);
  const int d = c;
  const bool mine = live && d < ND && 4 * q < NL;
  const int64_t o = ((int64_t)(slot * ND + (d < ND ? d : 0)) * g.n_sc + k) * NL;
  // Layers 4q .. 4q+3 of one RE: 32 contiguous bytes of x, 16 of nv.
  if (mine && x != nullptr) {
    if (NL % 4 == 0) {
      float4* __restrict__ xd = reinterpret_cast<float4*>(x + o + 4 * q);
      xd[0] = make_float4(xo[0], xo[1], xo[2], xo[3]);
      xd[1] = make_float4(xo[4], xo[5], xo[6], xo[7]);
      *reinterpret_cast<float4*>(nv + o + 4 * q) = make_float4(vo[0], vo[1], vo[2], vo[3]);
    } else {
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        if (4 * q + v < NL) {
          x[o + 4 * q + v] = make_float2(xo[2 * v], xo[2 * v + 1]);
          nv[o + 4 * q + v] = vo[v];
        }
      }
    }
  }
  if (llr != nullptr) {  // demapping fused into the detector (qm and the branch block-uniform)
    constexpr int kStage = kRows * kMaxRx * NL / 2;  // floats: a quarter of lds_h
    constexpr bool kStaged = PREC != kPrecF32;
    float* stage = reinterpret_cast<float*>(lds_h) + wave * kStage;
    const int64_t seg0 = ((int64_t)slot * ND * g.n_sc + k) * NL;  // RE (slot, d = 0, k)
    const int64_t dstride = (int64_t)g.n_sc * NL;                  // REs between symbols
    switch (g.qm) {
      case 2: emit_llr<2, NL, kStage, kStaged>(llr, stage, seg0, dstride, o, xo, vo, q, c, ND, mine, live); break;
      case 4: emit_llr<4, NL, kStage, kStaged>(llr, stage, seg0, dstride, o, xo, vo, q, c, ND, mine, live); break;
      case 6: emit_llr<6, NL, kStage, kStaged>(llr, stage, seg0, dstride, o, xo, vo, q, c, ND, mine, live); break;
      default: emit_llr<8, NL, kStage, kStaged>(llr, stage, seg0, dstride, o, xo, vo, q, c, ND, mine, live); break;
    }
  }
}

// pil != NULL: the pilot-resolution estimate is formed inside the detector (LSF = 1).
template <int HRES, int NL, int PREC>
void launch_one(const Geom& g, dim3 grid, const float2* rx, bool bfp, const float2* h,
                const float2* pil, const float* nvar, float2* x, float* nv, float* llr,
                hipStream_t s) {
  if constexpr (HRES == 0 && PREC == kPrecF32) {  // the one-launch chain is FP32 only
    if (pil != nullptr) {
      if (bfp)
        hipLaunchKernelGGL((mmse_mfma_kernel<0, NL, PREC, 1, 1>), grid, dim3(256), 0, s, g, rx,
                           h, pil, nvar, x, nv, llr);
      else
        hipLaunchKernelGGL((mmse_mfma_kernel<0, NL, PREC, 0, 1>), grid, dim3(256), 0, s, g, rx,
                           h, pil, nvar, x, nv, llr);
      return;
    }
  }
  if (bfp)
    hipLaunchKernelGGL((mmse_mfma_kernel<HRES, NL, PREC, 1, 0>), grid, dim3(256), 0, s, g, rx, h,
                       pil, nvar, x, nv, llr);
  else
    hipLaunchKernelGGL((mmse_mfma_kernel<HRES, NL, PREC, 0, 0>), grid, dim3(256), 0, s, g, rx, h,
                       pil, nvar, x, nv, llr);
}

template <int HRES, int PREC>
void launch_nl(const Geom& g, dim3 grid, const float2* rx, bool bfp, const float2* h,
               const float2* pil, const float* nvar, float2* x, float* nv, float* llr,
               hipStream_t s) {
  switch (g.n_layers) {
    case 5: launch_one<HRES, 5, PREC>(g, grid, rx, bfp, h, pil, nvar, x, nv, llr, s); break;
    case 6: launch_one<HRES, 6, PREC>(g, grid, rx, bfp, h, pil, nvar, x, nv, llr, s); break;
    case 7: launch_one<HRES, 7, PREC>(g, grid, rx, bfp, h, pil, nvar, x, nv, llr, s); break;
    case 8: launch_one<HRES, 8, PREC>(g, grid, rx, bfp, h, pil, nvar, x, nv, llr, s); break;
    case 9: launch_one<HRES, 9, PREC>(g, grid, rx, bfp, h, pil, nvar, x, nv, llr, s); break;
    case 10: launch_one<HRES, 10, PREC>(g, grid, rx, bfp, h, pil, nvar, x, nv, llr, s); break;
    case 11: launch_one<HRES, 11, PREC>(g, grid, rx, bfp, h, pil, nvar, x, nv, llr, s); break;
    case 12: launch_one<HRES, 12, PREC>(g, grid, rx, bfp, h, pil, nvar, x, nv, llr, s); break;
    case 13: launch_one<HRES, 13, PREC>(g, grid, rx, bfp, h, pil, nvar, x, nv, llr, s); break;
    case 14: launch_one<HRES, 14, PREC>(g, grid, rx, bfp, h, pil, nvar, x, nv, llr, s); break;
    case 15: launch_one<HRES, 15, PREC>(g, grid, rx, bfp, h, pil, nvar, x, nv, llr, s); break;
    default: launch_one<HRES, 16, PREC>(g, grid, rx, bfp, h, pil, nvar, x, nv, llr, s); break;
  }
}

template <int PREC>
void launch_prec(const Geom& g, dim3 grid, const float2* rx, bool bfp, const float2* h,
                 const float2* pil, int h_res, const float* nvar, float2* x, float* nv,
                 float* llr, hipStream_t s) {
  if (h_res == 0) launch_nl<0, PREC>(g, grid, rx, bfp, h, pil, nvar, x, nv, llr, s);
  else launch_nl<1, PREC>(g, grid, rx, bfp, h, pil, nvar, x, nv, llr, s);
}

}  // namespace

bool mmse_mfma_eligible(const Geom& g, const void* rx, const void* h, const void* x,
                        const void* nv, const void* llr) {
  // 16-byte aligned buffers: 16-byte loads of the received grid and channel rows, 16-byte
  // stores of x, nv and LLRs (absent outputs are NULL, which is aligned).
  const uintptr_t mis =
      ((uintptr_t)rx | (uintptr_t)h | (uintptr_t)x | (uintptr_t)nv | (uintptr_t)llr) & 15u;
  return mis == 0 && g.n_occ == 1 && g.n_layers >= 5 && g.n_layers <= 16 &&
         g.n_rx % 16 == 0 && g.n_rx <= 64 && g.n_dsym <= 16;
}

hipError_t launch_mmse_mfma(const Geom& g, const float2* rx, bool bfp, const float2* h,
                            const float2* pil, int h_res, const float* nvar, float2* x,
                            float* nv, float* llr, int prec, hipStream_t s) {
  const int64_t waves = (int64_t)g.n_slots * g.n_sc;
  const int64_t blocks = (waves + 3) / 4;
  const dim3 grid((unsigned)((blocks + kXcds - 1) / kXcds * kXcds));
  if (pil != nullptr && prec != kPrecF32) return hipErrorInvalidValue;  // one launch: FP32 only
  switch (prec) {
    case kPrecF32: launch_prec<kPrecF32>(g, grid, rx, bfp, h, pil, h_res, nvar, x, nv, llr, s); break;
    case kPrecF16: launch_prec<kPrecF16>(g, grid, rx, bfp, h, pil, h_res, nvar, x, nv, llr, s); break;
    case kPrecBF16: launch_prec<kPrecBF16>(g, grid, rx, bfp, h, pil, h_res, nvar, x, nv, llr, s); break;
    case kPrecF16R: launch_prec<kPrecF16R>(g, grid, rx, bfp, h, pil, h_res, nvar, x, nv, llr, s); break;
    case kPrecBF16R: launch_prec<kPrecBF16R>(g, grid, rx, bfp, h, pil, h_res, nvar, x, nv, llr, s); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace ranphy
