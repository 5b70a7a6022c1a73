// Learned refinement of the pilot-resolution channel estimate: a 4-layer residual CNN
// (channel estimation is the PHY block the paper names besides MIMO detection, abstract and
// Sec. III-B; the network itself is this library's addition).
//
// One image is the estimate of one (receive antenna, layer) pair over the pilot grid: rows
// are DMRS occasions, columns the port's pilot index j, two channels (real, imaginary).  A
// pilot-resolution estimate h[slot][occ][j][rx][layer] is therefore already an image stack
// [group = slot][pixel = occ * J + j][image = rx * Nl + layer][channel], and the kernels keep
// every tensor in that order, [group][pixel][image][channel], with 32 BF16 channels per
// activation (the 2-channel input and output padded with zeros):
//   a0 = x;  a_{l+1} = max(conv3x3(a_l; W_l, b_l), 0)  (l = 0, 1, 2);  out = x + conv3x3(a_3; W_3, b_3)
// conv3x3 is a correlation with zero padding, tap t = 3 (dy + 1) + (dx + 1) reading pixel
// (row + dy, col + dx).  Training minimises sum((out - target)^2) / out.size with Adam.
// With a per-group noise variance s2_g the network works on noise-normalised estimates: it
// sees x / sigma_g (unit noise variance at every SNR, the channel's amplitude telling the
// SNR) and refines x into x + sigma_g y; training then compares x / sigma_g + y with
// target / sigma_g, which weighs every SNR alike.
//
// Convolutions run on v_mfma_f32_16x16x32_bf16: one wave computes 16 images x 4 pixels x 32
// output channels; per valid tap the A operand is the 16 images' 32 input channels at the
// neighbouring pixel (a contiguous 1 KB row block) and the B operand the tap's 32 x 32
// weights.  The input-gradient pass is the same kernel on the mirrored, transposed weights;
// the weight gradients are FP32 partial sums per (group, 16-pixel, 64-image) block, reduced
// in a second pass (deterministic, no atomics).
#include <stdint.h>

#include "geom.h"

namespace ranphy {

constexpr int kCnnCh = 32;       // padded channel count
constexpr int kCnnTaps = 9;
constexpr int kCnnLayers = 4;
constexpr int kCnnLayerParams = kCnnTaps * kCnnCh * kCnnCh + kCnnCh;  // W[t][ci][co], b[co]
constexpr int kCnnParams = kCnnLayers * kCnnLayerParams;
// real input / output channels of each layer (the rest are zero padding)
const int kCnnCin[kCnnLayers] = {2, 32, 32, 32};
const int kCnnCout[kCnnLayers] = {32, 32, 32, 2};
constexpr int kWgradPx = 16, kWgradImg = 64;  // pixels x images of one weight-gradient block

namespace {

typedef float floatx4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

struct Grid2 {
  int rows, cols, npx, nimg, ngrp;
};

// Noise normalisation of group g: r = 1 / sigma (0 when s2 <= 0), sigma = sqrt(s2).
__device__ __forceinline__ float inv_sigma(const float* nv, int64_t g) {
  if (nv == nullptr) return 1.f;
  const float v = nv[g];
  return v > 0.f ? rsqrtf(v) : 0.f;
}

// Packed BF16 weights of one layer, [t][out][in], in forward and in input-gradient form.
__global__ void cnn_pack_kernel(const float* __restrict__ params, __bf16* __restrict__ wf,
                                __bf16* __restrict__ wb) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;  // [l][t][o][i]
  if (e >= kCnnLayers * kCnnTaps * kCnnCh * kCnnCh) return;
  const int i = e % kCnnCh;
  const int o = (e / kCnnCh) % kCnnCh;
  const int t = (e / (kCnnCh * kCnnCh)) % kCnnTaps;
  const int l = e / (kCnnTaps * kCnnCh * kCnnCh);
  const float* W = params + l * kCnnLayerParams;  // W[t][ci][co]
  // forward: out = co, in = ci
  wf[e] = (__bf16)W[(t * kCnnCh + i) * kCnnCh + o];
  // input gradient: d a[q][ci] = sum_t sum_co dz[q - t][co] W[t][ci][co], a correlation of
  // dz with taps t' = mirror(t) = 8 - t: out = ci, in = co (training only)
  if (wb != nullptr) wb[e] = (__bf16)W[((kCnnTaps - 1 - t) * kCnnCh + o) * kCnnCh + i];
}

// x [group][pixel][image][2] FP32 -> a0 [group][pixel][image][32] BF16 (zero padded).
__global__ void cnn_input_kernel(const float* __restrict__ x, __bf16* __restrict__ a0,
                                 int64_t n, int64_t per_group, const float* __restrict__ nv) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;  // n = groups * per_group
  if (e >= n * 4) return;
  const int64_t q = e >> 2;  // (group, pixel, image)
  const int part = (int)(e & 3);  // 8 channels each
  bf16x8 v;
#pragma unroll
  for (int c = 0; c < 8; ++c) v[c] = (__bf16)0.f;
  if (part == 0) {
    const float r = inv_sigma(nv, q / per_group);
    v[0] = (__bf16)(x[2 * q] * r);
    v[1] = (__bf16)(x[2 * q + 1] * r);
  }
  reinterpret_cast<bf16x8*>(a0 + q * kCnnCh)[part] = v;
}

// One 3x3 layer.  MODE 0: out_b = max(conv + b, 0) [* (mask > 0)]; MODE 1: out_b = conv * (mask
// > 0) (input gradient: no bias); MODE 2, channels 0 and 1 to out_f[..][2], with y = conv + b
// and r = 1 / sigma of the group (1 without noise variances): res + y / r (refinement), or
// r res + y (training, normalised units, norm_out); groups with gate_nv < gate_min (or no
// positive noise variance) keep res, and in MODE 0 (given noise variances only for
// inference) such groups are skipped.
template <int MODE>
__global__ void __launch_bounds__(256) cnn_conv_kernel(Grid2 gd, const __bf16* __restrict__ in,
                                                       const __bf16* __restrict__ w,
                                                       const float* __restrict__ bias,
                                                       const __bf16* __restrict__ mask,
                                                       __bf16* __restrict__ out_b,
                                                       const float* __restrict__ res,
                                                       float* __restrict__ out_f,
                                                       const float* __restrict__ nv,
                                                       float gate_min, int norm_out) {
  const int lane = threadIdx.x & 63;
  const int64_t wave = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  const int nquad = (gd.npx + 3) >> 2;
  const int nib = (gd.nimg + 15) >> 4;
  const int64_t total = (int64_t)gd.ngrp * nquad * nib;
  if (wave >= total) return;  // wave-uniform
  const int ib = (int)(wave % nib);
  const int64_t rest = wave / nib;
  const int quad = (int)(rest % nquad);
  const int64_t grp = rest / nquad;
  const int p0 = quad * 4;
  const int r16 = lane & 15;   // A row (image) / B column (output channel)
  const int kg = lane >> 4;    // K chunk: channels 8 kg .. 8 kg + 7
  const int img_a = ib * 16 + r16;
  const bool img_ok = img_a < gd.nimg;
  const int64_t gbase = grp * gd.npx;
  // MODE 2: groups whose noise variance is below gate_min keep their input (out = res)
  const float r = inv_sigma(nv, grp);
  const bool keep = nv == nullptr || (nv[grp] >= gate_min && r > 0.f);
  // Inference: a group that keeps its input needs no hidden activations (MODE 0 is given the
  // noise variances only then) and no products in the last layer.
  if (MODE == 0 && !keep) return;  // wave-uniform
  const bool work = MODE != 2 || norm_out || keep;

  floatx4 acc[4][2];
#pragma unroll
  for (int pp = 0; pp < 4; ++pp)
#pragma unroll
    for (int tt = 0; tt < 2; ++tt) acc[pp][tt] = floatx4{0.f, 0.f, 0.f, 0.f};

  int prow[4], pcol[4];
#pragma unroll
  for (int pp = 0; pp < 4; ++pp) {
    prow[pp] = (p0 + pp) / gd.cols;
    pcol[pp] = (p0 + pp) - prow[pp] * gd.cols;
  }
  for (int t = 0; t < (work ? kCnnTaps : 0); ++t) {
    const int dy = t / 3 - 1, dx = t % 3 - 1;
    bool any = false;
#pragma unroll
    for (int pp = 0; pp < 4; ++pp) {
      const int r = prow[pp] + dy, c = pcol[pp] + dx;
      any = any || (p0 + pp < gd.npx && r >= 0 && r < gd.rows && c >= 0 && c < gd.cols);
    }
    if (!any) continue;  // uniform: e.g. the dy = +-1 taps of a one-row grid
    const bf16x8 b0 = reinterpret_cast<const bf16x8*>(w + (t * kCnnCh + r16) * kCnnCh)[kg];
    // the last layer has two output channels: its second tile of 16 is never read
    const bf16x8* w1 = reinterpret_cast<const bf16x8*>(w + (t * kCnnCh + 16 + r16) * kCnnCh);
    const bf16x8 b1 = MODE == 2 ? b0 : w1[kg];
#pragma unroll
    for (int pp = 0; pp < 4; ++pp) {
      const int r = prow[pp] + dy, c = pcol[pp] + dx;
      if (p0 + pp < gd.npx && r >= 0 && r < gd.rows && c >= 0 && c < gd.cols) {
        bf16x8 a;
        if (img_ok) {
          a = reinterpret_cast<const bf16x8*>(
              in + ((gbase + r * gd.cols + c) * gd.nimg + img_a) * kCnnCh)[kg];
        } else {
#pragma unroll
          for (int e = 0; e < 8; ++e) a[e] = (__bf16)0.f;
        }
        acc[pp][0] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b0, acc[pp][0], 0, 0, 0);
        if (MODE != 2) acc[pp][1] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b1, acc[pp][1], 0, 0, 0);
      }
    }
  }
  // D[i][j] = acc[..][v] of lane j + 16 (i / 4): image ib * 16 + 4 kg + v, channel 16 tt + r16
#pragma unroll
  for (int pp = 0; pp < 4; ++pp) {
    const int p = p0 + pp;
    if (p >= gd.npx) continue;
#pragma unroll
    for (int tt = 0; tt < (MODE == 2 ? 1 : 2); ++tt) {
      const int o = 16 * tt + r16;
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int img = ib * 16 + 4 * kg + v;
        if (img >= gd.nimg) continue;
        const int64_t q = (gbase + p) * gd.nimg + img;
        float val = acc[pp][tt][v];
        if (MODE == 2) {
          if (o < 2) {
            const float y = val + bias[o];
            out_f[q * 2 + o] = norm_out ? r * res[q * 2 + o] + y
                                        : (keep ? res[q * 2 + o] + y / r : res[q * 2 + o]);
          }
        } else {
          if (MODE == 0) val = fmaxf(val + bias[o], 0.f);
          if (mask != nullptr && !((float)mask[q * kCnnCh + o] > 0.f)) val = 0.f;
          out_b[q * kCnnCh + o] = (__bf16)val;
        }
      }
    }
  }
}

// Loss terms and the output gradient: dz = 2 (out - target) / n_el on channels 0, 1.
__global__ void cnn_loss_kernel(const float* __restrict__ out, const float* __restrict__ target,
                                __bf16* __restrict__ dz, float* __restrict__ partial, int64_t n,
                                float scale, int64_t per_group, const float* __restrict__ nv) {
  __shared__ float red[256];  // n = groups * per_group (pixels * images)
  const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  float s = 0.f;
  if (q < n) {
    const float r = inv_sigma(nv, q / per_group);  // target in the output's (normalised) units
    const float d0 = out[2 * q] - r * target[2 * q];
    const float d1 = out[2 * q + 1] - r * target[2 * q + 1];
    s = d0 * d0 + d1 * d1;
    bf16x8 v;
#pragma unroll
    for (int c = 0; c < 8; ++c) v[c] = (__bf16)0.f;
    v[0] = (__bf16)(2.f * scale * d0);
    v[1] = (__bf16)(2.f * scale * d1);
    bf16x8* dst = reinterpret_cast<bf16x8*>(dz + q * kCnnCh);
    dst[0] = v;
#pragma unroll
    for (int c = 0; c < 8; ++c) v[c] = (__bf16)0.f;
    dst[1] = v;
    dst[2] = v;
    dst[3] = v;
  }
  red[threadIdx.x] = s;
  __syncthreads();
  for (int k = 128; k > 0; k >>= 1) {
    if (threadIdx.x < k) red[threadIdx.x] += red[threadIdx.x + k];
    __syncthreads();
  }
  if (threadIdx.x == 0) partial[blockIdx.x] = red[0];
}

// Sums the loss partials in a fixed order: loss = scale * sum.
__global__ void cnn_loss_reduce_kernel(const float* __restrict__ partial, int n, float scale,
                                       float* __restrict__ loss) {
  __shared__ float red[256];
  float s = 0.f;
  for (int i = threadIdx.x; i < n; i += 256) s += partial[i];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int k = 128; k > 0; k >>= 1) {
    if (threadIdx.x < k) red[threadIdx.x] += red[threadIdx.x + k];
    __syncthreads();
  }
  if (threadIdx.x == 0) *loss = red[0] * scale;
}

// Weight and bias gradient partial sums of one layer over one (group, 16-pixel, 64-image)
// block: part[blk][t][ci][co] = sum x[p + t][img][ci] dz[p][img][co] (t < 9) and
// part[blk][9][0][co] = sum dz[p][img][co].  Thread (ci, 4 output channels).
__global__ void __launch_bounds__(256) cnn_wgrad_kernel(Grid2 gd, const __bf16* __restrict__ x,
                                                        const __bf16* __restrict__ dz,
                                                        float* __restrict__ part) {
  const int npc = (gd.npx + kWgradPx - 1) / kWgradPx;
  const int nic = (gd.nimg + kWgradImg - 1) / kWgradImg;
  const int blk = blockIdx.x;
  const int ic = blk % nic;
  const int pc = (blk / nic) % npc;
  const int64_t grp = blk / (nic * npc);
  const int ci = threadIdx.x >> 3;
  const int co = (threadIdx.x & 7) * 4;
  float acc[kCnnTaps + 1][4];
#pragma unroll
  for (int t = 0; t <= kCnnTaps; ++t)
#pragma unroll
    for (int k = 0; k < 4; ++k) acc[t][k] = 0.f;
  const int64_t gbase = grp * gd.npx;
  const int i0 = ic * kWgradImg, i1 = min(gd.nimg, i0 + kWgradImg);
  for (int pi = 0; pi < kWgradPx; ++pi) {
    const int p = pc * kWgradPx + pi;
    if (p >= gd.npx) break;
    const int r = p / gd.cols, c = p - r * gd.cols;
    int nb[kCnnTaps];
#pragma unroll
    for (int t = 0; t < kCnnTaps; ++t) {
      const int rr = r + t / 3 - 1, cc = c + t % 3 - 1;
      nb[t] = (rr >= 0 && rr < gd.rows && cc >= 0 && cc < gd.cols) ? rr * gd.cols + cc : -1;
    }
    for (int img = i0; img < i1; ++img) {
      const __bf16* d = dz + ((gbase + p) * gd.nimg + img) * kCnnCh + co;
      const float d0 = (float)d[0], d1 = (float)d[1], d2 = (float)d[2], d3 = (float)d[3];
#pragma unroll
      for (int t = 0; t < kCnnTaps; ++t) {
        if (nb[t] < 0) continue;  // uniform over the block
        const float xv = (float)x[((gbase + nb[t]) * gd.nimg + img) * kCnnCh + ci];
        acc[t][0] = fmaf(xv, d0, acc[t][0]);
        acc[t][1] = fmaf(xv, d1, acc[t][1]);
        acc[t][2] = fmaf(xv, d2, acc[t][2]);
        acc[t][3] = fmaf(xv, d3, acc[t][3]);
      }
      acc[kCnnTaps][0] += d0;
      acc[kCnnTaps][1] += d1;
      acc[kCnnTaps][2] += d2;
      acc[kCnnTaps][3] += d3;
    }
  }
  float* dst = part + (int64_t)blk * (kCnnTaps + 1) * kCnnCh * kCnnCh;
#pragma unroll
  for (int t = 0; t <= kCnnTaps; ++t)
#pragma unroll
    for (int k = 0; k < 4; ++k) dst[(t * kCnnCh + ci) * kCnnCh + co + k] = acc[t][k];
}

// grad (one layer, params layout W[t][ci][co], b[co]) = sum over blocks, in block order.
__global__ void cnn_wgrad_reduce_kernel(const float* __restrict__ part, int nblk,
                                        float* __restrict__ grad, int layer, int cin,
                                        int cout) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;  // [t][ci][co], t <= 9
  if (e >= (kCnnTaps + 1) * kCnnCh * kCnnCh) return;
  const int t = e / (kCnnCh * kCnnCh);
  const int ci = (e / kCnnCh) % kCnnCh;
  const int co = e % kCnnCh;
  if (t == kCnnTaps && ci != 0) return;
  float s = 0.f;
  for (int b = 0; b < nblk; ++b) s += part[(int64_t)b * (kCnnTaps + 1) * kCnnCh * kCnnCh + e];
  // padded channels carry no gradient (their inputs or outputs are zero by construction)
  const bool real = (t == kCnnTaps || ci < cin) && co < cout;
  float* g = grad + layer * kCnnLayerParams;
  if (t < kCnnTaps) g[e] = real ? s : 0.f;
  else g[kCnnTaps * kCnnCh * kCnnCh + co] = real ? s : 0.f;
}

__global__ void cnn_adam_kernel(float* __restrict__ p, const float* __restrict__ g,
                                float* __restrict__ m, float* __restrict__ v, int n, float lr,
                                float b1, float b2, float eps, float c1, float c2) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n) return;
  const float gg = g[e];
  const float mm = b1 * m[e] + (1.f - b1) * gg;
  const float vv = b2 * v[e] + (1.f - b2) * gg * gg;
  m[e] = mm;
  v[e] = vv;
  p[e] -= lr * (mm / c1) / (sqrtf(vv / c2) + eps);
}

// ---- inference on one-row grids: the four layers in one kernel ----------------------------
// A one-row grid (one DMRS occasion) makes every layer a 1 x 3 correlation along the pilots
// (the dy = +-1 taps read the zero padding).  One wave holds kFuseSeg consecutive pixels of
// 16 images in registers, one B operand (bf16x8) per pixel, and runs the four layers there:
// layer l computes pixels l + 1 .. kFuseSeg - 2 - l of the segment, so the last writes the
// kFuseOut pixels 4 .. kFuseSeg - 5.  Products are transposed relative to cnn_conv_kernel:
// A = the tap's weights (rows = 16 output channels), B = activations (columns = 16 images,
// K = 32 input channels), so a lane's accumulators (image l & 15, output channels 4 (l >> 4)
// + v of each 16-channel tile) are, after bias and ReLU, exactly its B operand for the next
// layer when the K slots 8 q + e of lane group q hold input channels 4 q + e (e < 4) and
// 16 + 4 q + e - 4 (e >= 4).  Pixels outside the image are zero at every layer's input.
constexpr int kFuseSeg = 24;
constexpr int kFuseOut = kFuseSeg - 2 * kCnnLayers;
constexpr int kFuseW = kCnnTaps * kCnnCh * kCnnCh;  // packed weights of one layer
typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
typedef __bf16 bf16x4 __attribute__((ext_vector_type(4)));

// x [g][p][img][2] FP32 -> xn [g][p][img][2] BF16, divided by sigma of the group; groups the
// gate keeps plain are skipped (the fused kernel copies them).
// Group g0 + blockIdx.y, elements blockIdx.x * 256 + threadIdx.x of its per_group.
__global__ void cnn_norm_kernel(const float2* __restrict__ x, bf16x2* __restrict__ xn, int64_t g0,
                                int per_group, const float* __restrict__ nv, float gate_min) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= per_group) return;
  const int64_t g = g0 + blockIdx.y;
  const float r = inv_sigma(nv, g);
  if (!(nv == nullptr || (nv[g] >= gate_min && r > 0.f))) return;
  const int64_t e = g * per_group + i;
  const float2 v = x[e];
  bf16x2 o;
  o[0] = (__bf16)(v.x * r);
  o[1] = (__bf16)(v.y * r);
  xn[e] = o;
}

// The A operand of one output channel's packed row wf[t][o][0 .. 31] for lane group q.
__device__ __forceinline__ bf16x8 fused_w(const __bf16* row, int q) {
  const bf16x4 lo = *reinterpret_cast<const bf16x4*>(row + 4 * q);
  const bf16x4 hi = *reinterpret_cast<const bf16x4*>(row + 16 + 4 * q);
  bf16x8 r;
#pragma unroll
  for (int e = 0; e < 4; ++e) {
    r[e] = lo[e];
    r[4 + e] = hi[e];
  }
  return r;
}

// relu(lo), relu(hi) as two BF16 in one word: round to nearest even, then the ReLU as a
// 16-bit integer max with 0 (a BF16 is negative exactly when its sign bit is set, and the
// order of non-negative BF16 bit patterns is that of their values).
__device__ __forceinline__ unsigned relu_bf16x2(float lo, float hi) {
  typedef float floatx2 __attribute__((ext_vector_type(2)));
  typedef short shortx2 __attribute__((ext_vector_type(2)));
  const bf16x2 v = __builtin_convertvector((floatx2){lo, hi}, bf16x2);
  const shortx2 m = __builtin_elementwise_max(__builtin_bit_cast(shortx2, v), (shortx2){0, 0});
  return __builtin_bit_cast(unsigned, m);
}

// Hidden layer L (0..2) in place: act[p] <- relu(b + sum_dx W[3 + dx] act[p - 1 + dx]) for
// p = L + 1 .. kFuseSeg - 2 - L (the bias seeds the accumulators); pixel p sits at column
// pos0 + p, and pixels outside the image are zeroed afterwards.
template <int L>
__device__ __forceinline__ void fused_hidden(bf16x8 (&act)[kFuseSeg], const __bf16* __restrict__ wf,
                                             const float* __restrict__ params, int pos0, int cols,
                                             int j, int q) {
  typedef unsigned uintx4 __attribute__((ext_vector_type(4)));
  const __bf16* wl = wf + L * kFuseW;
  bf16x8 wa[3][2];
#pragma unroll
  for (int dx = 0; dx < 3; ++dx)
#pragma unroll
    for (int tt = 0; tt < 2; ++tt)
      wa[dx][tt] = fused_w(wl + ((3 + dx) * kCnnCh + 16 * tt + j) * kCnnCh, q);
  const float* bias = params + L * kCnnLayerParams + kFuseW;
  floatx4 b0, b1;
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    b0[v] = bias[4 * q + v];
    b1[v] = bias[16 + 4 * q + v];
  }
  constexpr int lo = L + 1, hi = kFuseSeg - 1 - L;
  bf16x8 held;
#pragma unroll
  for (int p = lo; p < hi; ++p) {
    floatx4 a0 = b0, a1 = b1;
#pragma unroll
    for (int dx = 0; dx < 3; ++dx) {
      a0 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(wa[dx][0], act[p - 1 + dx], a0, 0, 0, 0);
      a1 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(wa[dx][1], act[p - 1 + dx], a1, 0, 0, 0);
    }
    const uintx4 o = {relu_bf16x2(a0[0], a0[1]), relu_bf16x2(a0[2], a0[3]),
                      relu_bf16x2(a1[0], a1[1]), relu_bf16x2(a1[2], a1[3])};
    if (p > lo) act[p - 1] = held;  // pixel p - 1's input was last read just above
    held = __builtin_bit_cast(bf16x8, o);
  }
  act[hi - 1] = held;
  if (pos0 + lo < 0 || pos0 + hi > cols) {  // wave-uniform: a segment at an image edge
#pragma unroll
    for (int p = lo; p < hi; ++p)
      if ((unsigned)(pos0 + p) >= (unsigned)cols) act[p] = bf16x8{};
  }
}

// out = x + sigma y for the groups the gate refines, out = x for the others; out may alias x
// (each lane reads x only at the pixels it writes; the halo comes from xn).
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2, 2))) cnn_fused1_kernel(Grid2 gd, const __bf16* __restrict__ wf,
                                                         const float* __restrict__ params,
                                                         const bf16x2* __restrict__ xn,
                                                         const float2* x, float2* out,
                                                         const float* __restrict__ nv,
                                                         float gate_min) {
  const int lane = threadIdx.x & 63;
  const int64_t wave = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  const int nseg = (gd.cols + kFuseOut - 1) / kFuseOut;
  const int nib = (gd.nimg + 15) >> 4;
  if (wave >= (int64_t)gd.ngrp * nseg * nib) return;  // wave-uniform
  const int ib = (int)(wave % nib);
  const int64_t rest = wave / nib;
  const int seg = (int)(rest % nseg);
  const int64_t grp = rest / nseg;
  const int j = lane & 15, q = lane >> 4;
  const int img = ib * 16 + j;
  const bool mine = q == 0 && img < gd.nimg;  // the lanes that own image img's two channels
  const int c0 = seg * kFuseOut;
  const int pos0 = c0 - kCnnLayers;           // column of segment pixel 0
  const int64_t gbase = grp * gd.npx;
  const float r = inv_sigma(nv, grp);
  const bool keep = nv == nullptr || (nv[grp] >= gate_min && r > 0.f);
  // The residual x at the wave's output pixels is loaded in full before any store: out may
  // alias x, so a load placed after a store could not be issued before that store completes.
  float2 res[kFuseOut];
  auto load_res = [&]() {
#pragma unroll
    for (int p = 0; p < kFuseOut; ++p) {
      res[p] = make_float2(0.f, 0.f);
      if (mine && c0 + p < gd.cols) res[p] = x[(gbase + c0 + p) * gd.nimg + img];
    }
  };
  if (!keep) {  // wave-uniform: the plain estimate (nothing to do in place)
    if (out != x) {
      load_res();
#pragma unroll
      for (int p = 0; p < kFuseOut; ++p)
        if (mine && c0 + p < gd.cols) out[(gbase + c0 + p) * gd.nimg + img] = res[p];
    }
    return;
  }
  bf16x8 act[kFuseSeg];
#pragma unroll
  for (int p = 0; p < kFuseSeg; ++p) {
    bf16x8 a;
#pragma unroll
    for (int e = 0; e < 8; ++e) a[e] = (__bf16)0.f;
    const int pos = pos0 + p;
    if (mine && (unsigned)pos < (unsigned)gd.cols) {
      const bf16x2 v = xn[(gbase + pos) * gd.nimg + img];
      a[0] = v[0];
      a[1] = v[1];
    }
    act[p] = a;
  }
  fused_hidden<0>(act, wf, params, pos0, gd.cols, j, q);
  fused_hidden<1>(act, wf, params, pos0, gd.cols, j, q);
  fused_hidden<2>(act, wf, params, pos0, gd.cols, j, q);
  // last layer: output channels 0 and 1 (tile 0, lanes q = 0, registers 0 and 1)
  const __bf16* wl = wf + 3 * kFuseW;
  bf16x8 wa[3];
#pragma unroll
  for (int dx = 0; dx < 3; ++dx) wa[dx] = fused_w(wl + ((3 + dx) * kCnnCh + j) * kCnnCh, q);
  load_res();
  const float* bias = params + 3 * kCnnLayerParams + kFuseW;
  const floatx4 b3 = {bias[0], bias[1], 0.f, 0.f};
  const float sigma = 1.f / r;
#pragma unroll
  for (int p = kCnnLayers; p < kFuseSeg - kCnnLayers; ++p) {
    floatx4 a0 = b3;
#pragma unroll
    for (int dx = 0; dx < 3; ++dx)
      a0 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(wa[dx], act[p - 1 + dx], a0, 0, 0, 0);
    const int pos = pos0 + p;
    if (mine && pos < gd.cols) {
      const float2 xr = res[p - kCnnLayers];
      out[(gbase + pos) * gd.nimg + img] =
          make_float2(fmaf(a0[0], sigma, xr.x), fmaf(a0[1], sigma, xr.y));
    }
  }
}

// Workspace carving (every piece 256-byte aligned).
struct CnnWs {
  __bf16* wf;     // [4][9][32][32]
  __bf16* wb;     // [4][9][32][32]
  __bf16* act[4]; // a0 .. a3
  __bf16* xn;     // one-row inference: [g][p][img][2] normalised BF16 input
  __bf16* dz[2];
  float* out;     // [g][p][img][2]
  float* part;    // weight-gradient partials
  float* lpart;   // loss partials
  int64_t bytes;
};

int64_t align256(int64_t b) { return (b + 255) & ~int64_t(255); }

CnnWs carve(void* base, const Grid2& gd, bool train) {
  CnnWs w{};
  char* p = static_cast<char*>(base);
  int64_t off = 0;
  auto take = [&](int64_t b) {  // an empty piece is a null pointer
    char* r = (p != nullptr && b > 0) ? p + off : nullptr;
    off += align256(b);
    return r;
  };
  const int64_t nq = (int64_t)gd.ngrp * gd.npx * gd.nimg;
  const int64_t wsz = (int64_t)kCnnLayers * kCnnTaps * kCnnCh * kCnnCh * 2;
  w.wf = reinterpret_cast<__bf16*>(take(wsz));
  w.wb = reinterpret_cast<__bf16*>(take(train ? wsz : 0));
  const bool fused = !train && gd.rows == 1;  // inference on one-row grids: one kernel
  const int nact = train ? 4 : (fused ? 0 : 2);
  for (int i = 0; i < 4; ++i)
    w.act[i] = i < nact ? reinterpret_cast<__bf16*>(take(nq * kCnnCh * 2)) : nullptr;
  w.xn = reinterpret_cast<__bf16*>(take(fused ? nq * 2 * 2 : 0));
  for (int i = 0; i < 2; ++i)
    w.dz[i] = train ? reinterpret_cast<__bf16*>(take(nq * kCnnCh * 2)) : nullptr;
  w.out = reinterpret_cast<float*>(take(train ? nq * 2 * 4 : 0));
  const int64_t nblk = (int64_t)gd.ngrp * ((gd.npx + kWgradPx - 1) / kWgradPx) *
                       ((gd.nimg + kWgradImg - 1) / kWgradImg);
  w.part = reinterpret_cast<float*>(take(train ? nblk * (kCnnTaps + 1) * kCnnCh * kCnnCh * 4 : 0));
  w.lpart = reinterpret_cast<float*>(take(train ? ((nq + 255) / 256) * 4 : 0));
  w.bytes = off;
  return w;
}

template <int MODE>
hipError_t conv(const Grid2& gd, const __bf16* in, const __bf16* w, const float* bias,
                const __bf16* mask, __bf16* out_b, const float* res, float* out_f,
                hipStream_t s, const float* nv = nullptr, float gate_min = 0.f,
                int norm_out = 0) {
  const int64_t waves = (int64_t)gd.ngrp * ((gd.npx + 3) / 4) * ((gd.nimg + 15) / 16);
  const dim3 grid((unsigned)((waves + 3) / 4));
  hipLaunchKernelGGL((cnn_conv_kernel<MODE>), grid, dim3(256), 0, s, gd, in, w, bias, mask,
                     out_b, res, out_f, nv, gate_min, norm_out);
  return hipGetLastError();
}

const int64_t kWsz = (int64_t)kCnnTaps * kCnnCh * kCnnCh;  // one layer of packed weights

hipError_t forward(const Grid2& gd, const float* params, const float* x, float* out,
                   const CnnWs& w, bool keep, hipStream_t s, const float* nv, float gate_min) {
  const int64_t nq = (int64_t)gd.ngrp * gd.npx * gd.nimg;
  hipLaunchKernelGGL(cnn_pack_kernel, dim3((kCnnLayers * kWsz + 255) / 256), dim3(256), 0, s,
                     params, w.wf, w.wb);
  if (w.xn != nullptr) {  // inference on a one-row grid
    const int per_group = gd.npx * gd.nimg;
    for (int g0 = 0; g0 < gd.ngrp; g0 += 65535) {
      const int ng = gd.ngrp - g0 < 65535 ? gd.ngrp - g0 : 65535;
      hipLaunchKernelGGL(cnn_norm_kernel, dim3((unsigned)((per_group + 255) / 256), ng), dim3(256),
                         0, s, reinterpret_cast<const float2*>(x), reinterpret_cast<bf16x2*>(w.xn),
                         (int64_t)g0, per_group, nv, gate_min);
    }
    const int64_t waves = (int64_t)gd.ngrp * ((gd.cols + kFuseOut - 1) / kFuseOut) *
                          ((gd.nimg + 15) / 16);
    hipLaunchKernelGGL(cnn_fused1_kernel, dim3((unsigned)((waves + 3) / 4)), dim3(256), 0, s, gd,
                       w.wf, params, reinterpret_cast<const bf16x2*>(w.xn),
                       reinterpret_cast<const float2*>(x), reinterpret_cast<float2*>(out), nv,
                       gate_min);
    return hipGetLastError();
  }
  hipLaunchKernelGGL(cnn_input_kernel, dim3((unsigned)((nq * 4 + 255) / 256)), dim3(256), 0, s,
                     x, w.act[0], nq, (int64_t)gd.npx * gd.nimg, nv);
  // training keeps a0 .. a3; inference ping-pongs between two buffers
  __bf16* a[4] = {w.act[0], w.act[1], keep ? w.act[2] : w.act[0], keep ? w.act[3] : w.act[1]};
  for (int l = 0; l < 3; ++l) {  // inference skips the groups the gate keeps plain
    const hipError_t e = conv<0>(gd, a[l], w.wf + l * kWsz, params + l * kCnnLayerParams + kWsz,
                                 nullptr, a[l + 1], nullptr, nullptr, s, keep ? nullptr : nv,
                                 gate_min);
    if (e != hipSuccess) return e;
  }
  // training (keep) writes the output in normalised units for the loss
  return conv<2>(gd, a[3], w.wf + 3 * kWsz, params + 3 * kCnnLayerParams + kWsz, nullptr,
                 nullptr, x, out, s, nv, gate_min, keep ? 1 : 0);
}

}  // namespace

int64_t cnn_param_count() { return kCnnParams; }

int64_t cnn_workspace_bytes(int rows, int cols, int nimg, int ngrp, bool train) {
  const Grid2 gd{rows, cols, rows * cols, nimg, ngrp};
  return carve(nullptr, gd, train).bytes;
}

hipError_t cnn_forward(int rows, int cols, int nimg, int ngrp, const float* params,
                       const float* x, float* out, void* ws, hipStream_t s, const float* nv,
                       float gate_min) {
  const Grid2 gd{rows, cols, rows * cols, nimg, ngrp};
  const CnnWs w = carve(ws, gd, false);
  return forward(gd, params, x, out, w, false, s, nv, gate_min);
}

hipError_t cnn_grad(int rows, int cols, int nimg, int ngrp, const float* params, const float* x,
                    const float* target, const float* nv, float* grad, float* loss, void* ws,
                    hipStream_t s) {
  const Grid2 gd{rows, cols, rows * cols, nimg, ngrp};
  const CnnWs w = carve(ws, gd, true);
  hipError_t e = forward(gd, params, x, w.out, w, true, s, nv, 0.f);
  if (e != hipSuccess) return e;
  const int64_t nq = (int64_t)gd.ngrp * gd.npx * gd.nimg;
  const float scale = 1.f / (float)(nq * 2);
  const int nlb = (int)((nq + 255) / 256);
  hipLaunchKernelGGL(cnn_loss_kernel, dim3(nlb), dim3(256), 0, s, w.out, target, w.dz[0],
                     w.lpart, nq, scale, (int64_t)gd.npx * gd.nimg, nv);
  hipLaunchKernelGGL(cnn_loss_reduce_kernel, dim3(1), dim3(256), 0, s, w.lpart, nlb, scale, loss);
  const int nblk = gd.ngrp * ((gd.npx + kWgradPx - 1) / kWgradPx) *
                   ((gd.nimg + kWgradImg - 1) / kWgradImg);
  const int nred = (kCnnTaps + 1) * kCnnCh * kCnnCh;
  int cur = 0;
  for (int l = kCnnLayers - 1; l >= 0; --l) {
    hipLaunchKernelGGL(cnn_wgrad_kernel, dim3(nblk), dim3(256), 0, s, gd, w.act[l], w.dz[cur],
                       w.part);
    hipLaunchKernelGGL(cnn_wgrad_reduce_kernel, dim3((nred + 255) / 256), dim3(256), 0, s,
                       w.part, nblk, grad, l, kCnnCin[l], kCnnCout[l]);
    if (l == 0) break;
    // dz_{l-1} = (sum_t dz_l[q - t] W_l[t]^T) * (a_l > 0)
    e = conv<1>(gd, w.dz[cur], w.wb + l * kWsz, nullptr, w.act[l], w.dz[cur ^ 1], nullptr,
                nullptr, s);
    if (e != hipSuccess) return e;
    cur ^= 1;
  }
  return hipGetLastError();
}

hipError_t cnn_adam(float* params, const float* grad, float* m, float* v, int step, float lr,
                    hipStream_t s) {
  const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
  const float c1 = 1.f - powf(b1, (float)step), c2 = 1.f - powf(b2, (float)step);
  hipLaunchKernelGGL(cnn_adam_kernel, dim3((kCnnParams + 255) / 256), dim3(256), 0, s, params,
                     grad, m, v, kCnnParams, lr, b1, b2, eps, c1, c2);
  return hipGetLastError();
}

}  // namespace ranphy
