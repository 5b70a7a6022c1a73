/*
 * ranphy.h — C ABI of libranphy, the MI355X (gfx950) uplink receive hot path.
 *
 * The three calls are the data-parallel steps of a software-defined DU's uplink PHY that
 * the paper accelerates with SIMD (Sec. III-B: channel estimation and MIMO detection;
 * Sec. IV and Fig. 4: LMMSE detection built from a factorisation of the covariance and
 * forward/backward substitution):
 *
 *   ranphy_chest_ls     DMRS least-squares channel estimate (+ frequency interpolation)
 *   ranphy_mmse_detect  channel interpolation, Gram H^H H + s2 I, Cholesky factorisation,
 *                       matched filter, forward/back substitution, unbiasing
 *   ranphy_llr_demap    max-log LLR soft demapping, QPSK .. 256QAM
 *
 * Conventions shared by every call
 *   - Complex values are interleaved float pairs (re, im) ("complex64"); every buffer is
 *     row-major with the slot index outermost.
 *   - All buffers are device memory allocated by the caller, at least 8-byte aligned
 *     (256-byte alignment recommended).  The library allocates nothing, keeps no pointer
 *     after returning and holds no global mutable state: calls are thread-safe.
 *   - Work is enqueued on `stream` (a hipStream_t; NULL = the null stream) and is
 *     asynchronous: the call returns once the kernels are launched.
 *   - The descriptor and sizes are validated on the host before any launch; invalid input
 *     returns a negative status and touches no memory.  Nothing throws across the ABI.
 *   - Per-element numerical failure is not an error: where the regularised Gram matrix is
 *     not numerically positive definite (possible only with s2 = 0 and a rank-deficient
 *     channel) the detector writes NaN symbols and +inf post-equalisation variance for
 *     that resource element.
 *
 * DMRS structure (the paper gives none; the 3GPP NR shape is used): port p occupies
 * subcarriers k = (p mod C) + C j of every DMRS symbol, j < ceil(n_sc / C); occasion o spans
 * symbols dmrs_sym0[o] .. dmrs_sym0[o] + T - 1, T in {1, 2}; with T = 2, ports p and p + C
 * share a comb offset and are separated by a time cover code contained in the pilot values
 * the caller passes.  Layers map one-to-one onto ports 0 .. n_layers-1, so n_layers <= C T.
 * Symbols of a DMRS occasion carry no data; "dsym" enumerates the remaining symbols in
 * ascending order.
 */
#ifndef RANPHY_H
#define RANPHY_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define RANPHY_ABI_VERSION 1

#if defined(__GNUC__) || defined(__clang__)
#define RANPHY_API __attribute__((visibility("default")))
#else
#define RANPHY_API
#endif

/* Shape of a batch of slots; every slot in the batch has the same shape. */
typedef struct ranphy_slot_desc {
  int32_t n_prb;        /* resource blocks, 1..275; n_sc = 12 n_prb subcarriers       */
  int32_t n_symb;       /* OFDM symbols per slot, 1..14                                */
  int32_t n_rx;         /* receive antennas, 1..64                                     */
  int32_t n_layers;     /* layers, 1..16, <= n_rx and <= dmrs_comb * dmrs_td          */
  int32_t qm;           /* bits per symbol: 2 QPSK, 4 16QAM, 6 64QAM, 8 256QAM        */
  int32_t dmrs_comb;    /* comb C: 2, 4 or 8                                           */
  int32_t dmrs_td;      /* symbols per DMRS occasion T: 1 or 2                         */
  int32_t n_occ;        /* DMRS occasions, 1..4                                        */
  int32_t dmrs_sym0[4]; /* first symbol of each occasion, ascending, non-overlapping  */
  int32_t n_slots;      /* slots in the batch, >= 0 (0 is a no-op)                     */
} ranphy_slot_desc;

/* Resolution of a channel-estimate buffer. */
enum {
  RANPHY_H_PILOT = 0, /* [slot][occ][j][rx][layer], j < ceil(n_sc / C): the estimate on the
                         layer's own pilot subcarrier (p mod C) + C j; unused tail entries
                         (j past the layer's last pilot) are written as 0 and never read  */
  RANPHY_H_FULL = 1   /* [slot][occ][sc][rx][layer]: interpolated to every subcarrier     */
};

/* Status codes. */
enum {
  RANPHY_OK = 0,
  RANPHY_ERR_INVALID = -1,     /* NULL or misaligned pointer, bad descriptor field      */
  RANPHY_ERR_UNSUPPORTED = -2, /* well-formed but outside the supported shapes          */
  RANPHY_ERR_LAUNCH = -3       /* the HIP runtime refused a launch (no device, ...)     */
};

/* Input precision of the Gram and matched-filter products in ranphy_mmse_detect_prec.
 * Accumulation, inversion, solve and unbiasing are FP32 in every mode.  FP16 operands are
 * scaled per subcarrier by a power of two into the FP16 range before rounding and the
 * products scaled back exactly, so any FP32 input magnitude works; within [2^-2, 2^14) no
 * scaling happens (none is needed there).
 * The refined modes add one step of iterative refinement (Sec. III-A: 16-bit components with
 * the accuracy kept; the residual in FP32): each operand is also split into its 16-bit
 * value and 16-bit remainder, the remainders give the FP32 Gram G and matched filter z to
 * first order (G = G~ + dG, z = z~ + dz, products of 16-bit values accumulated in FP32), and
 * the solution of the inverted 16-bit system G~ is corrected once with the FP32 residual,
 * x^ <- x^ + G~^-1 (z - G x^); diag(G^-1), which the unbiasing uses, is corrected to the
 * same order.  Their results approach the FP32 mode's (the remainders carry 22 bits in
 * FP16, 16 in BF16). */
enum {
  RANPHY_PREC_FP32 = 0,         /* FP32 inputs (the plain path; ranphy_mmse_detect)        */
  RANPHY_PREC_FP16 = 1,         /* inputs rounded to FP16, FP32 accumulation (matrix cores) */
  RANPHY_PREC_BF16 = 2,         /* inputs rounded to BF16, FP32 accumulation (matrix cores) */
  RANPHY_PREC_FP16_REFINED = 3, /* FP16 products plus one refinement step                   */
  RANPHY_PREC_BF16_REFINED = 4  /* BF16 products plus one refinement step                   */
};

/* Buffer identifiers for ranphy_buffer_floats. */
enum {
  RANPHY_BUF_RX = 0,        /* [slot][symb][sc][rx]           complex64 */
  RANPHY_BUF_PILOTS = 1,    /* [slot][occ][t][j][layer]       complex64 */
  RANPHY_BUF_H = 2,         /* see RANPHY_H_PILOT / RANPHY_H_FULL        */
  RANPHY_BUF_NOISE_VAR = 3, /* [slot]                         float     */
  RANPHY_BUF_X = 4,         /* [slot][dsym][sc][layer]        complex64 */
  RANPHY_BUF_NV = 5,        /* [slot][dsym][sc][layer]        float     */
  RANPHY_BUF_LLR = 6        /* [slot][dsym][sc][layer][qm]    float     */
};

/* ABI version the library was built with (RANPHY_ABI_VERSION). */
RANPHY_API int ranphy_abi_version(void);

/* Static description of a status code; never NULL. */
RANPHY_API const char* ranphy_status_str(int status);

/* Number of floats (a complex value counts 2) in buffer `buf` for descriptor `d`
 * (h_res matters only for RANPHY_BUF_H); a negative status if `d` is invalid. */
RANPHY_API int64_t ranphy_buffer_floats(const ranphy_slot_desc* d, int buf, int h_res);

/*
 * DMRS least-squares channel estimate (Sec. III-B names channel estimation as a block
 * suited to data-parallel execution; the estimator is the standard LS one).
 *   h(o, j, r, p) = (1/T) sum_{t<T} rx(dmrs_sym0[o] + t, k, r) conj(pilots(o, t, j, p)),
 *   k = (p mod C) + C j.
 * With h_res = RANPHY_H_FULL the estimate is interpolated linearly in frequency between the
 * layer's consecutive pilots and held at the nearest pilot outside the first/last one.
 *   rx      in  [slot][symb][sc][rx] complex64
 *   pilots  in  [slot][occ][t][j][layer] complex64 (unit modulus, cover code included)
 *   h       out per h_res, complex64
 */
RANPHY_API int ranphy_chest_ls(const ranphy_slot_desc* d, const float* rx, const float* pilots, float* h,
                    int h_res, void* stream);

/*
 * Linear MMSE detection per data resource element (Sec. IV, Fig. 4: LMMSE detection with a
 * triangular factorisation of the covariance and forward/backward substitution; here the
 * layer-domain covariance G = H^H H + s2 I, factorised by Cholesky).
 *   H      channel at (sc, symbol): frequency interpolation of h (PILOT) or h itself (FULL),
 *          then linear interpolation in the symbol index between occasion centres
 *          dmrs_sym0[o] + (T-1)/2, held outside them (a single occasion is held).
 *   x_hat  = G^-1 H^H y,  mu_l = 1 - s2 (G^-1)_ll,
 *   x      = x_hat / mu (unbiased),  nv = (1 - mu) / mu  (post-equalisation noise plus
 *          interference variance of the unbiased estimate, unit-energy layers).
 *   rx         in  [slot][symb][sc][rx] complex64
 *   h          in  per h_res, complex64
 *   noise_var  in  [slot] float, s2 >= 0 (noise variance per receive antenna and RE)
 *   x          out [slot][dsym][sc][layer] complex64
 *   nv         out [slot][dsym][sc][layer] float
 */
RANPHY_API int ranphy_mmse_detect(const ranphy_slot_desc* d, const float* rx, const float* h, int h_res,
                       const float* noise_var, float* x, float* nv, void* stream);

/*
 * ranphy_mmse_detect with a choice of input precision for the two contractions over the
 * receive antennas (the Gram H^H H and the matched filter H^H y): the paper's point that
 * reduced precision keeps detection accuracy (Sec. III-A: 16-bit real/imaginary parts are
 * often enough; Sec. IV, Fig. 5(a): single precision matches double), taken to 16-bit
 * matrix-core inputs.  Same arguments, layouts and outputs as ranphy_mmse_detect.
 * The 16-bit modes (RANPHY_PREC_FP16, _BF16 and their refined forms) run only on the
 * matrix-core detector: one DMRS
 * occasion, 5..16 layers, n_rx a multiple of 16, rx / h / x / nv 16-byte aligned; other
 * shapes return RANPHY_ERR_UNSUPPORTED.  RANPHY_PREC_FP32 accepts every shape.
 */
RANPHY_API int ranphy_mmse_detect_prec(const ranphy_slot_desc* d, const float* rx,
                                       const float* h, int h_res, const float* noise_var,
                                       float* x, float* nv, int precision, void* stream);

/*
 * Detection and demapping in one pass: ranphy_mmse_detect_prec followed by ranphy_llr_demap,
 * with the demapping done by the detector as it produces each symbol, so the symbols and
 * variances need not travel through HBM.  x and nv are optional outputs: both NULL (only
 * LLRs are written) or both given (written exactly as ranphy_mmse_detect_prec writes them).
 * Same shapes as the reduced-precision modes (one DMRS occasion, 5..16 layers, n_rx a
 * multiple of 16, every buffer 16-byte aligned); others return RANPHY_ERR_UNSUPPORTED.
 *   llr  out [slot][dsym][sc][layer][qm] float, as ranphy_llr_demap.
 */
RANPHY_API int ranphy_mmse_llr(const ranphy_slot_desc* d, const float* rx, const float* h,
                               int h_res, const float* noise_var, float* x, float* nv,
                               float* llr, int precision, void* stream);

/*
 * Max-log LLRs of Gray square QAM (3GPP NR mapping structure: bits b0, b2, .. on the
 * in-phase axis, b1, b3, .. on the quadrature axis), unit average energy:
 *   llr_b = (min_{s: b=1} |x - s|^2 - min_{s: b=0} |x - s|^2) / nv,  positive favours 0.
 *   x    in  [slot][dsym][sc][layer] complex64
 *   nv   in  [slot][dsym][sc][layer] float (> 0; 0 gives +-inf, NaN on a tie)
 *   llr  out [slot][dsym][sc][layer][qm] float
 */
RANPHY_API int ranphy_llr_demap(const ranphy_slot_desc* d, const float* x, const float* nv, float* llr,
                     void* stream);

/* ---------------------------------------------------------------------------------------
 * Learned refinement of the pilot-resolution channel estimate (a library addition beside
 * the paper's method: channel estimation is the PHY block the paper names besides MIMO
 * detection, abstract and Sec. III-B).
 *
 * Network: 4 layers of 3x3 correlation with zero padding over an image grid of `rows` x `cols`
 * pixels, channels 2 -> 32 -> 32 -> 32 -> 2, ReLU after the first three, last layer y.  Tap
 * t = 3 (dy + 1) + (dx + 1) reads pixel (row + dy, col + dx).  BF16 operands, FP32
 * accumulation.
 * Noise normalisation: with a noise variance s2_g > 0 per group (noise_var, device, may be
 * NULL: s2 = 1 for every group) the network sees x / sigma_g, sigma_g = sqrt(s2_g), and the
 * refined tensor is x + sigma_g y; training measures (x / sigma_g + y - target / sigma_g)^2,
 * summed and divided by the number of values, so that every SNR weighs alike.
 *
 * Parameters: one FP32 vector of ranphy_cnn_param_count() floats, per layer l = 0..3:
 * W_l[9][32 in][32 out] then b_l[32]; channels beyond a layer's real ones (2 inputs of layer
 * 0, 2 outputs of layer 3) must be zero and stay zero.
 * Tensors: x, target, out [group][pixel = row * cols + col][image][2] FP32 (real, imaginary).
 * A pilot-resolution estimate h[slot][occ][j][rx][layer] is such a tensor with
 * group = slot, rows = occasions, cols = pilots, image = rx * n_layers + layer.
 * Limits: rows * cols <= 2^20 pixels, n_img <= 2^20 and rows * cols * n_img <= 2^30 per group
 * (else RANPHY_ERR_UNSUPPORTED).
 * Workspace: device memory of ranphy_cnn_workspace_bytes(..) bytes, 256-byte aligned,
 * owned by the caller; its contents need not be initialised.  Inference on a one-row grid
 * runs the four layers in one kernel and needs only the packed weights and a BF16 copy of
 * the input; other grids and training keep every layer's activations.  Errors as above.
 * ------------------------------------------------------------------------------------- */
RANPHY_API int64_t ranphy_cnn_param_count(void);
/* Workspace bytes for a forward pass (train = 0) or a gradient pass (train = 1). */
RANPHY_API int64_t ranphy_cnn_workspace_bytes(int rows, int cols, int n_img, int n_groups,
                                              int train);
/* out = x + sigma y (x + y without noise variances); groups whose noise variance is below
 * min_noise_var, or not positive, keep out = x.  out may be x itself (in place); it must not
 * otherwise overlap x. */
RANPHY_API int ranphy_cnn_forward(const float* params, const float* x, const float* noise_var,
                                  float min_noise_var, float* out, int rows, int cols,
                                  int n_img, int n_groups, void* workspace,
                                  int64_t workspace_bytes, void* stream);
/* loss (one float, device) and its gradient with respect to every parameter (grad: same
 * layout as params; zero on the padded channels).  Every group's noise variance must be
 * positive. */
RANPHY_API int ranphy_cnn_grad(const float* params, const float* x, const float* target,
                               const float* noise_var, float* grad, float* loss, int rows,
                               int cols, int n_img, int n_groups, void* workspace,
                               int64_t workspace_bytes, void* stream);
/* One Adam step (beta1 0.9, beta2 0.999, eps 1e-8) of step number `step` >= 1 on params with
 * first and second moments m, v (zero before step 1). */
RANPHY_API int ranphy_cnn_adam(float* params, const float* grad, float* m, float* v, int step,
                               float lr, void* stream);
/* The network applied to a pilot-resolution estimate (ranphy_chest_ls with RANPHY_H_PILOT),
 * h_out in the same layout (it may be h_in itself, but must not otherwise overlap it).  Slots
 * whose noise variance noise_var[slot] (device, as for ranphy_mmse_detect; may be NULL: every
 * slot refined) is below min_noise_var keep the plain estimate: above the SNR where validation
 * shows the refinement no longer helps, plain interpolation of the LS estimate is the better
 * one.  Processed in as
 * many slots per pass as the workspace holds (at least ranphy_cnn_workspace_bytes(n_occ,
 * ceil(n_sc / C), n_rx * n_layers, 1, 0) bytes). */
RANPHY_API int ranphy_cnn_denoise(const ranphy_slot_desc* d, const float* params,
                                  const float* noise_var, float min_noise_var,
                                  const float* h_in, float* h_out, void* workspace,
                                  int64_t workspace_bytes, void* stream);

/* For callers that cannot allocate device memory (code under HIP graph capture, tight serving
 * loops, harnesses that forbid hipMalloc): ranphy_cnn_denoise without a workspace argument.
 * Its workspace is the library's own array of RANPHY_NOALLOC_SCRATCH_BYTES bytes in the
 * device memory of each GPU it runs on, held until the process ends; the call allocates
 * nothing (no hipMalloc, no allocating library routine).  The array belongs to the device of
 * `stream` (the current device for the null stream); its device address is looked up once
 * per device, on that device's first call.  Every call on one GPU shares the array, so calls
 * whose executions overlap on one GPU (different streams, or graphs replayed concurrently)
 * race and give undefined results; calls ordered on one stream do not.  Same arguments,
 * semantics and results (bit for bit) as ranphy_cnn_denoise; slots are processed as many per
 * pass as the array holds.  RANPHY_ERR_UNSUPPORTED when one slot needs more than the array
 * (ranphy_cnn_workspace_bytes(n_occ, ceil(n_sc / C), n_rx * n_layers, 1, 0) >
 * RANPHY_NOALLOC_SCRATCH_BYTES; e.g. one 64 x 16 slot of 273 PRB at comb 8 needs 1.7 MB, a
 * two-occasion 64-image slot 12.9 MB), checked before anything runs on the GPU. */
#define RANPHY_NOALLOC_SCRATCH_BYTES (32LL << 20)
RANPHY_API int ranphy_cnn_denoise_noalloc(const ranphy_slot_desc* d, const float* params,
                                          const float* noise_var, float min_noise_var,
                                          const float* h_in, float* h_out, void* stream);

/*
 * The whole chain in one launch for up to 8 layers: LS estimation at the pilots (abstract,
 * Sec. III-B), interpolation, LMMSE detection by Cholesky factorisation and substitution
 * (Sec. IV, Fig. 4), unbiasing and max-log demapping, computed tile by tile with the pilot
 * estimates of each tile of subcarriers held on chip, so only the received grid, the pilots
 * and the LLRs travel through device memory.  Same results as ranphy_chest_ls (pilot
 * resolution) -> ranphy_mmse_detect -> ranphy_llr_demap up to rounding order.
 *   rx, pilots, noise_var as for ranphy_chest_ls / ranphy_mmse_detect;
 *   llr out [slot][dsym][sc][layer][qm] float.
 * More than 8 layers run on the matrix-core detector, each block forming the pilot estimates
 * it needs itself with ranphy_chest_ls's arithmetic, so the LLRs equal ranphy_chest_ls ->
 * ranphy_mmse_llr bit for bit; this needs that detector's shapes (one DMRS occasion, n_rx a
 * multiple of 16, rx and llr 16-byte aligned), else RANPHY_ERR_UNSUPPORTED.
 */
RANPHY_API int ranphy_receive(const ranphy_slot_desc* d, const float* rx, const float* pilots,
                              const float* noise_var, float* llr, void* stream);

/*
 * Block floating point (BFP) compression of the received grid, for the fronthaul of
 * distributed MIMO (Sec. VI-A proposes it and fixes no format; the format here is a reading):
 *   - the grid rx [slot][symb][sc][rx] complex64 is cut into blocks of B consecutive antennas
 *     of one resource element, B = 16 when n_rx is a multiple of 16, else B = n_rx (< 16);
 *     any other antenna count returns RANPHY_ERR_UNSUPPORTED;
 *   - a block's 2B real values v_i (I and Q interleaved, antenna order) share the exponent e,
 *     the smallest integer with max |v_i| <= 255 * 2^e (0 for an all-zero block); each is
 *     stored as the 9-bit two's complement mantissa m_i = round-half-even(v_i / 2^e), and
 *     decompresses to m_i * 2^e, so the error is at most 2^(e-1) per value;
 *   - a block is one 32-bit word holding e (two's complement), then ceil(18 B / 32) words of
 *     mantissas, a little-endian bit stream with m_i in bits 9 i .. 9 i + 8 (unused high bits
 *     zero); blocks follow the grid's resource elements, then antenna groups.
 * For 16-antenna blocks that is 10 words for 128 bytes of FP32 samples (3.2x smaller).
 *
 * ranphy_bfp_words: the 32-bit words of the compressed grid of `d`, or a negative status.
 * ranphy_bfp_compress: rx (device, 8-byte aligned) -> packed (device, 4-byte aligned,
 *   ranphy_bfp_words(d) words).  Values must be finite.
 * ranphy_bfp_decompress: packed -> rx; rx then holds exactly what the receive calls expect.
 * The words and the samples must not overlap.
 * Both are asynchronous on `stream`; host validation as for the other calls.
 */
RANPHY_API int64_t ranphy_bfp_words(const ranphy_slot_desc* d);
RANPHY_API int ranphy_bfp_compress(const ranphy_slot_desc* d, const float* rx, uint32_t* packed,
                                   void* stream);
RANPHY_API int ranphy_bfp_decompress(const ranphy_slot_desc* d, const uint32_t* packed,
                                     float* rx, void* stream);
/*
 * The decompression fused into the loads of the receive path (the fronthaul delivers the
 * words, the grid is never expanded in device memory):
 * ranphy_chest_ls_bfp: ranphy_chest_ls with the received grid given as BFP words (packed:
 *   device, 4-byte aligned, ranphy_bfp_words(d) words); every sample is decoded where the
 *   estimator reads it.  Antenna counts without a block width: RANPHY_ERR_UNSUPPORTED.
 * ranphy_mmse_llr_bfp: ranphy_mmse_llr with the received grid given as BFP words (packed:
 *   8-byte aligned); its shapes (n_rx a multiple of 16, so one lane's 16 antennas of one
 *   symbol are one block), each block decoded in registers inside the detector.
 * Both give bit for bit what the FP32 calls give on ranphy_bfp_decompress's output.
 */
RANPHY_API int ranphy_chest_ls_bfp(const ranphy_slot_desc* d, const uint32_t* packed,
                                   const float* pilots, float* h, int h_res, void* stream);
RANPHY_API int ranphy_mmse_llr_bfp(const ranphy_slot_desc* d, const uint32_t* packed,
                                   const float* h, int h_res, const float* noise_var, float* x,
                                   float* nv, float* llr, int precision, void* stream);
/* ranphy_receive with the received grid given as BFP words (packed: 4-byte aligned), every
 * sample decoded where the one-launch chain loads it; antenna counts without a block width:
 * RANPHY_ERR_UNSUPPORTED.  Bit for bit ranphy_receive on ranphy_bfp_decompress's output. */
RANPHY_API int ranphy_receive_bfp(const ranphy_slot_desc* d, const uint32_t* packed,
                                  const float* pilots, const float* noise_var, float* llr,
                                  void* stream);

/* ---------------------------------------------------------------------------------------
 * Many UEs of uneven allocations in one persistent launch (the scheduling and divergence
 * costs of SIMT processing the paper weighs in Sec. V): for every UE, LS estimation at the
 * pilots, interpolation, LMMSE detection and max-log demapping, LLRs out.
 *
 * ranphy_batch_plan builds, on the host, a plan of the batch (per UE its geometry and
 * buffers, and work items of about `tile_re` resource elements each: tiles of consecutive
 * subcarriers, grouped by (layers, modulation, antennas) class, heaviest first) and copies it
 * synchronously into `plan`, device memory of ranphy_batch_plan_bytes(..) bytes, 256-byte
 * aligned, owned by the caller.  The UE buffers must stay valid while the plan is used; their
 * contents may change between runs.  ranphy_batch_run clears the plan's work counter and
 * launches `n_blocks` persistent blocks of 256 threads on `stream` that take items until none
 * is left (both launches can be captured into a HIP graph; runs of one plan must not
 * overlap).  Per UE: one slot (desc.n_slots = 1), 1..8 layers; LLRs as ranphy_llr_demap.
 * ------------------------------------------------------------------------------------- */
typedef struct {
  ranphy_slot_desc desc;  /* the UE's allocation, n_slots = 1 */
  const float* rx;        /* [symb][sc][rx] complex64 */
  const float* pilots;    /* [occ][t][j][layer] complex64 */
  const float* noise_var; /* one float */
  float* llr;             /* [dsym][sc][layer][qm] float */
} ranphy_ue;

RANPHY_API int64_t ranphy_batch_plan_bytes(const ranphy_ue* ues, int n_ue, int tile_re);
RANPHY_API int ranphy_batch_plan(const ranphy_ue* ues, int n_ue, int tile_re, void* plan,
                                 int64_t plan_bytes);
RANPHY_API int ranphy_batch_run(void* plan, int n_blocks, void* stream);

#ifdef __cplusplus
}
#endif
#endif
