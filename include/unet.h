/* unet.h -- C ABI of the learned warm start's network kernels (gfx950).
 *
 * A U-Net on periodic lattice fields predicts a later density field from an initial
 * one; the lattice solver (lbm.h) starts from the prediction.  These calls are the
 * network's building blocks: 3x3 convolutions on bfloat16 activations with FP32
 * accumulation on the matrix cores, their two gradients, 2x2 max pooling, nearest
 * 2x upsampling, the 1x1 output head with the mean-squared-error loss, and the Adam
 * update (Kingma & Ba, 2015).
 *
 * Conventions shared by every call:
 *  - Activations are NHWC, bfloat16 (raw 16-bit patterns, round to nearest even),
 *    unless a call says FP32.  A tensor argument comes with `ld` (elements between
 *    consecutive pixels, >= its channel count) and `off` (channel offset), so one
 *    buffer can hold the channel concatenation of two tensors.  ld and off must be
 *    multiples of 8 and the base pointer 16-byte aligned (16-bit tensors).
 *  - H and W are powers of two (>= 2; the pooled and upsampled sizes follow); the
 *    3x3 convolutions wrap around (periodic padding), matching the lattice.
 *  - 3x3 weights are [C_out][3][3][C_in] (tap (ky, kx) reads offset (ky-1, kx-1)).
 *  - Every pointer is device memory owned by the caller; nothing is allocated.
 *    Calls are asynchronous on `stream` (a hipStream_t; NULL = null stream).
 *  - Returns 0 on success, UNET_EINVAL (-1) for a bad argument (checked before any
 *    launch), UNET_ESHAPE (-2) when a fused call does not cover valid arguments of that
 *    shape (nothing launched; the separate calls it replaces do), UNET_EHIP (-3) when a
 *    launch fails; unet_last_error() explains.
 */
#ifndef UNET_H
#define UNET_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define UNET_OK 0
#define UNET_EINVAL (-1)
#define UNET_ESHAPE (-2)
#define UNET_EHIP (-3)

/* y = epilogue(conv3x3(x, w) + bias): y[n,p,o] = bias[o] + sum_{t,i} w[o,t,i] x[n,p+off_t,i].
 * flags: UNET_RELU applies max(., 0); UNET_OUT_F32 stores FP32 (else bfloat16).
 * mask (nullable, bfloat16, [N,H,W] x C_out with its own ld/off): the result is
 * zeroed where mask <= 0 (the ReLU gradient gate of a backward pass).
 * bias may be NULL (no bias).  C_in % 8 == 0, C_out % 16 == 0. */
#define UNET_RELU 1
#define UNET_OUT_F32 2
int unet_conv3x3_fwd(const void* x, int32_t ldx, int32_t offx, const void* w, const float* bias,
                     void* y, int32_t ldy, int32_t offy, const void* mask, int32_t ldm, int32_t offm,
                     int32_t N, int32_t H, int32_t W, int32_t C_in, int32_t C_out, int32_t flags,
                     void* stream);

/* The same convolution with its input the channel concatenation of two tensors and its
 * output split between two, without either being stored whole: the U-Net decoder's
 * [upsample2(lower level) | skip connection] input, and its input gradient, whose two
 * channel ranges go back to the two branches.  Input channels [0, C_x) come from x,
 * which is [N,H,W] x C_x, or with half != 0 [N,H/2,W/2] x C_x read through the nearest
 * 2x upsampling (pixel (Y, X) reads (Y/2, X/2)); channels [C_x, C_in) come from x2
 * ([N,H,W] x (C_in - C_x); NULL when C_x = C_in).  Output channels [0, C_y) go to y,
 * [C_y, C_out) to y2 (NULL when C_y = C_out), each with its own ld/off; the mask, if
 * any, is one [N,H,W] x C_out tensor.  C_x and C_y are multiples of 8 in [8, C_in] and
 * [8, C_out], and C_x a multiple of 32 when C_in is.  Results are bitwise those of unet_conv3x3_fwd on the concatenated input
 * with the output stored whole.  unet_conv3x3_fwd(...) is this call with C_x = C_in,
 * half = 0, x2 = NULL, C_y = C_out, y2 = NULL. */
int unet_conv3x3_fwd_cat(const void* x, int32_t ldx, int32_t offx, int32_t C_x, int32_t half,
                         const void* x2, int32_t ldx2, int32_t offx2, const void* w, const float* bias,
                         void* y, int32_t ldy, int32_t offy, int32_t C_y, void* y2, int32_t ldy2,
                         int32_t offy2, const void* mask, int32_t ldm, int32_t offm, int32_t N, int32_t H,
                         int32_t W, int32_t C_in, int32_t C_out, int32_t flags, void* stream);

/* unet_conv3x3_fwd (bfloat16 output, no mask) followed by unet_maxpool2_fwd of its
 * output, in one pass: y as unet_conv3x3_fwd stores it and yp ([N,H/2,W/2] x C_out, its
 * own ld/off) bitwise as the pooling call computes it from y (the encoder's convolution
 * before the U-Net's 2x2 max pooling).  UNET_ESHAPE unless H, W >= 16 and C_in, C_out
 * are multiples of 32; UNET_EINVAL for UNET_OUT_F32. */
int unet_conv3x3_fwd_pool(const void* x, int32_t ldx, int32_t offx, const void* w, const float* bias,
                          void* y, int32_t ldy, int32_t offy, void* yp, int32_t ldyp, int32_t offyp,
                          int32_t N, int32_t H, int32_t W, int32_t C_in, int32_t C_out, int32_t flags,
                          void* stream);

/* Input gradient of the U-Net decoder's convolution, whose input is [upsample2(low) |
 * skip], through to the lower level: dx = conv3x3(g, wf) (C_g -> C_in channels, wf the
 * flipped weights); channels [C_low, C_in) are the skip branch's gradient, stored in
 * dskip ([N,H,W] x (C_in - C_low)); channels [0, C_low) go through the upsampling's
 * gradient and the lower level's ReLU: the sum over each 2x2 block, zeroed where
 * low <= 0, stored in dlow ([N,H/2,W/2] x C_low; low the same shape).  Bitwise the
 * result of unet_conv3x3_fwd_cat with the output split at C_low followed by
 * unet_upsample2_bwd, without the full-size gradient of the upsampled branch ever
 * being stored.  UNET_ESHAPE unless H, W >= 16, C_g and C_in are multiples of 32 and
 * C_low a multiple of the kernel's output-channel width (64 when C_g != 32 and
 * C_in % 64 == 0, else 32). */
int unet_conv3x3_bwd_upcat(const void* g, int32_t ldg, int32_t offg, const void* wf, void* dlow,
                           int32_t lddl, int32_t offdl, const void* low, int32_t ldlow, int32_t offlow,
                           int32_t C_low, void* dskip, int32_t ldds, int32_t offds, int32_t N, int32_t H,
                           int32_t W, int32_t C_g, int32_t C_in, void* stream);

/* wf[i][t][o] = w[o][8-t][i]: the weights of the input-gradient convolution
 * (dx = conv3x3_fwd(g, wf) with C_in and C_out exchanged). */
int unet_flip_weights(const void* w, void* wf, int32_t C_out, int32_t C_in, void* stream);

/* The same for n <= 64 layers in one launch: w[l], wf[l] (device, bfloat16, 16-byte
 * aligned) with C_out[l], C_in[l] >= 1; the four arrays are host memory, read before
 * the call returns.  UNET_EINVAL for n outside [1, 64] or a bad entry (nothing is
 * launched then). */
int unet_flip_weights_many(const void* const* w, void* const* wf, const int32_t* C_out, const int32_t* C_in,
                           int32_t n, void* stream);

/* Weight and bias gradients: dw[o,t,i] = sum_{n,p} g[n,p,o] x[n,p+off_t,i] and
 * db[o] = sum g[n,p,o] (FP32, overwritten).  The pixel sum is split over slabs whose
 * FP32 partial sums go to `partials` and are then added in a fixed order
 * (deterministic).  unet_wgrad_partial_bytes() gives the partials size. */
int unet_wgrad_partial_bytes(int32_t N, int32_t H, int32_t W, int32_t C_in, int32_t C_out, size_t* bytes);
int unet_conv3x3_wgrad(const void* x, int32_t ldx, int32_t offx, const void* g, int32_t ldg, int32_t offg,
                       float* dw, float* db, void* partials, size_t partial_bytes, int32_t N, int32_t H,
                       int32_t W, int32_t C_in, int32_t C_out, void* stream);

/* The same gradients with the layer input the concatenation of two tensors, as in
 * unet_conv3x3_fwd_cat (x: channels [0, C_x), at half size when half != 0; x2: channels
 * [C_x, C_in), NULL when C_x = C_in).  Results are bitwise those of unet_conv3x3_wgrad
 * on the concatenated input; the partials size is unet_wgrad_partial_bytes(C_in, C_out). */
int unet_conv3x3_wgrad_cat(const void* x, int32_t ldx, int32_t offx, int32_t C_x, int32_t half,
                           const void* x2, int32_t ldx2, int32_t offx2, const void* g, int32_t ldg,
                           int32_t offg, float* dw, float* db, void* partials, size_t partial_bytes,
                           int32_t N, int32_t H, int32_t W, int32_t C_in, int32_t C_out, void* stream);

/* The same weight and bias gradients for callers that cannot allocate device memory
 * (code under HIP graph capture, serving loops, harnesses that forbid hipMalloc): the
 * partial sums go to a static device array of UNET_WGRAD_SCRATCH_BYTES that the library
 * holds on each GPU it runs on until the process ends, and nothing is allocated.  The
 * caller still owns x, g, dw and db.  Results are bitwise those of unet_conv3x3_wgrad
 * (same split and summation order).  UNET_EINVAL when the shape needs more partials than
 * the array holds (unet_wgrad_partial_bytes() > UNET_WGRAD_SCRATCH_BYTES; every layer of
 * the 32/64/128/256 network at 256x256 x 16 fits), UNET_EHIP when the array's device
 * address cannot be looked up.  Every call on one GPU uses that GPU's one array: calls
 * that overlap on one GPU (other streams, other host threads) race and must be ordered
 * by the caller; calls on one stream are ordered by the stream. */
#define UNET_WGRAD_SCRATCH_BYTES ((size_t)48 << 20)
int unet_conv3x3_wgrad_noalloc(const void* x, int32_t ldx, int32_t offx, const void* g, int32_t ldg, int32_t offg,
                               float* dw, float* db, int32_t N, int32_t H, int32_t W, int32_t C_in,
                               int32_t C_out, void* stream);

/* 2x2 max pooling with stride 2: y[n,Y,X,c] = max of x over rows 2Y..2Y+1, cols 2X..2X+1.
 * The four 2x2 calls take C a multiple of 8 and need N * H * W * C / 8 < 2^31, with
 * H, W the full-resolution sizes (UNET_EINVAL otherwise). */
int unet_maxpool2_fwd(const void* x, int32_t ldx, int32_t offx, void* y, int32_t ldy, int32_t offy,
                      int32_t N, int32_t H, int32_t W, int32_t C, void* stream);

/* Pooling gradient: dx = route(dy) + add, gated by x > 0 when gate_relu != 0, where
 * route sends each window's dy to its first maximum in row-major window order.
 * add (nullable) is a full-size tensor.  H, W are the input (unpooled) sizes. */
int unet_maxpool2_bwd(const void* x, int32_t ldx, int32_t offx, const void* dy, int32_t lddy, int32_t offdy,
                      const void* add, int32_t lda, int32_t offa, void* dx, int32_t lddx, int32_t offdx,
                      int32_t gate_relu, int32_t N, int32_t H, int32_t W, int32_t C, void* stream);

/* Nearest 2x upsampling: y[n,2Y+a,2X+b,c] = x[n,Y,X,c].  H, W are the input sizes. */
int unet_upsample2_fwd(const void* x, int32_t ldx, int32_t offx, void* y, int32_t ldy, int32_t offy,
                       int32_t N, int32_t H, int32_t W, int32_t C, void* stream);

/* Upsampling gradient: dx[n,Y,X,c] = sum over the 2x2 block of dy, zeroed where
 * gate <= 0 (gate nullable, same shape as dx).  H, W are the output (small) sizes. */
int unet_upsample2_bwd(const void* dy, int32_t lddy, int32_t offdy, const void* gate, int32_t ldgt,
                       int32_t offgt, void* dx, int32_t lddx, int32_t offdx, int32_t N, int32_t H, int32_t W,
                       int32_t C, void* stream);

/* Network input from the fields of a lattice state: x[n,p,0] = (rho - rho_v[n]) /
 * (rho_l[n] - rho_v[n]), x[n,p,1] = cond[n], x[n,p,2] = (T / T0[n] - 1) / theta_scale
 * (0 when T is NULL), channels 3..7 zero (x is [N,H,W,8] bfloat16).  rin (FP32,
 * [2][N,H,W]) receives channels 0 and 2 unrounded: the residual the head adds.  rho
 * and T are FP64 [N,H,W]; x or rin may be NULL, not both. */
int unet_prepare_input(const double* rho, const double* T, const double* rho_v, const double* rho_l,
                       const double* T0, const double* cond, double theta_scale, void* x, float* rin,
                       int32_t N, int32_t H, int32_t W, void* stream);

/* Fields from the K normalised output planes (FP32 [K][N,H,W]): rho = rho_v + (rho_l -
 * rho_v) out[0]; T (nullable) = T0 (1 + theta_scale out[1]) (T0 when K = 1). */
int unet_output_fields(const float* out, int32_t K, const double* rho_v, const double* rho_l,
                       const double* T0, double theta_scale, double* rho, double* T, int32_t N, int32_t H,
                       int32_t W, void* stream);

/* Output head, K <= 4 outputs: out[k][n,p] = sum_c hw[k][c] d[n,p,c] + hb[k] + rin[k][n,p]
 * (FP32 planes).  With target (nullable, [K][N,H,W]) also the loss over all K N H W
 * values: dout = 2 (out - target) / (K N H W) and the mean squared error in loss[0]
 * (the sum uses per-block partials in `partials`, >= unet_head_partial_bytes(),
 * added in a fixed order). */
int unet_head_partial_bytes(int32_t N, int32_t H, int32_t W, int32_t C, int32_t K, size_t* bytes);
int unet_head_fwd(const void* d, int32_t ldd, const float* hw, const float* hb, const float* rin,
                  const float* target, float* out, float* dout, float* loss, void* partials,
                  size_t partial_bytes, int32_t N, int32_t H, int32_t W, int32_t C, int32_t K, void* stream);

/* Head gradient: g[n,p,c] = sum_k dout[k][n,p] hw[k][c] (gated by d > 0), dhw[k][c] =
 * sum dout[k] d[.,c], dhb[k] = sum dout[k] (FP32, deterministic block partials).
 * C / 8 must divide 256 (C in {8, 16, 32, 64, 128, 256}); UNET_EINVAL otherwise. */
int unet_head_bwd(const void* d, int32_t ldd, const float* hw, const float* dout, void* g, float* dhw,
                  float* dhb, void* partials, size_t partial_bytes, int32_t N, int32_t H, int32_t W,
                  int32_t C, int32_t K, void* stream);

/* unet_head_fwd with a target followed by unet_head_bwd, in one pass over d (training):
 * out, dout, loss, g, dhw and dhb as those two calls define them, with the same
 * partials size.  The K outputs of a pixel are summed in another order (8 channels per
 * lane, then across lanes), so out and what follows from it may differ from the two
 * calls in the last bits of FP32.  C / 8 must be a power of two dividing 256. */
int unet_head_train(const void* d, int32_t ldd, const float* hw, const float* hb, const float* rin,
                    const float* target, float* out, float* dout, float* loss, void* g, float* dhw,
                    float* dhb, void* partials, size_t partial_bytes, int32_t N, int32_t H, int32_t W,
                    int32_t C, int32_t K, void* stream);

/* Adam step t >= 1 on n FP32 parameters: m = b1 m + (1-b1) g; v = b2 v + (1-b2) g^2;
 * p -= lr (m / (1-b1^t)) / (sqrt(v / (1-b2^t)) + eps).  p16 (nullable) receives the
 * bfloat16 rounding of the updated p. */
int unet_adam(float* p, const float* g, float* m, float* v, void* p16, size_t n, float lr, float b1,
              float b2, float eps, int32_t t, void* stream);

/* bfloat16 <-> FP32 copies of n values (round to nearest even). */
int unet_to_bf16(const float* src, void* dst, size_t n, void* stream);
int unet_to_f32(const void* src, float* dst, size_t n, void* stream);

const char* unet_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* UNET_H */
