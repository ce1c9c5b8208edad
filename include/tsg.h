/*
 * tsg.h -- C ABI of the tactile surrogate's training and inference kernels
 * (gfx950, BF16 MFMA with FP32 accumulation).
 *
 * The surrogate is a convolutional encoder-decoder that maps the indenter's
 * height field over the sensor plus the press depth to the displacement field
 * of the elastomer's contact surface; it is trained on displacement fields
 * produced by the MLS-MPM simulation of tacchi.h, which stays its fallback
 * and error judge. These calls are its building blocks; the network is
 * sequenced by the caller.
 *
 * Conventions
 *  - Activations are NHWC bfloat16 (uint16 storage). A tensor view is
 *    (pointer, N, H, W, ld, off): element (n, h, w, c) is at
 *    ((n*H + h)*W + w)*ld + off + c, so channel slices of a wider buffer
 *    (skip concatenation) are addressed without copies. ld, off and channel
 *    counts used by convolutions must be multiples of 8 and pointers 16-byte
 *    aligned.
 *  - Convolution weights: FP32 master copy [Cout][taps][Cin] (taps = 9 for
 *    3x3 with tap = 3*kh + kw, taps = 1 for 1x1), bias [Cout]. The kernels use
 *    BF16 packs made by tsg_pack_weights.
 *  - All calls enqueue on `stream` (a hipStream_t, NULL = legacy default) and
 *    return 0, or -1 for invalid arguments / -3 for a failed launch (message in
 *    tsg_last_error()). The caller owns all memory.
 */
#ifndef TSG_H
#define TSG_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t tsg_status;

enum { TSG_EPI_BIAS = 0,      /* out = acc + bias (bf16) */
       TSG_EPI_BIAS_GELU = 1, /* z = acc + bias stored to zbuf (bf16), out = GELU(z) (bf16) */
       TSG_EPI_DGELU = 2,     /* out = acc * GELU'(z), z read from zbuf (bf16); backward through GELU */
       TSG_EPI_F32 = 3        /* out32 = acc + bias (fp32, dense [N*H*W][Cout]) */ };

/* Padded row length of a BF16 weight pack: K = taps * Cin_p rounded up to 32. */
int32_t tsg_pack_k(int32_t taps, int32_t cin_p);

/* BF16 packs of an FP32 master weight [Cout][taps][Cin]:
 *   wf [Cout][Kf]   forward:  wf[co][tap*Cin_p + ci] = w[co][tap][ci]
 *   wt [Cin_p][Kt]  backward (input gradient): the kernel flipped in space and
 *                   transposed, wt[ci][tap*Cout_p + co] = w[co][taps-1-tap][ci]
 * with Kf = tsg_pack_k(taps, Cin_p), Kt = tsg_pack_k(taps, Cout_p); padding is
 * zero. Either output may be NULL. */
tsg_status tsg_pack_weights(const float *w, int32_t cout, int32_t cin, int32_t cin_p, int32_t cout_p,
                            int32_t taps, uint16_t *wf, uint16_t *wt, void *stream);

/* Convolution as an implicit GEMM on MFMA (3x3 with zero padding 1, or 1x1):
 * acc[n,h,w,co] = sum_{tap,ci} in[n, h+dh(tap), w+dw(tap), ci] * W[co][tap][ci],
 * with the epilogue chosen by `epi` (see TSG_EPI_*). With wt packs and
 * TSG_EPI_DGELU this computes the input gradient of a forward convolution.
 * in: view with cin_p channels; wpack: [cout rows][tsg_pack_k(taps, cin_p)];
 * bias: [cout] or NULL; out: view with cout channels (or out32 for F32);
 * zbuf: view of the pre-activation (BIAS_GELU writes it, DGELU reads it). */
tsg_status tsg_conv(const uint16_t *in, int32_t n, int32_t h, int32_t w, int32_t in_ld, int32_t in_off,
                    int32_t cin_p, const uint16_t *wpack, const float *bias, int32_t cout, int32_t taps,
                    int32_t epi, uint16_t *out, int32_t out_ld, int32_t out_off, uint16_t *zbuf,
                    int32_t z_ld, int32_t z_off, float *out32, void *stream);

/* Weight gradient of a convolution: dw[co][tap][ci] (FP32, [cout][taps][cin])
 * = sum over n,h,w of dout[n,h,w,co] * in[n, h+dh(tap), w+dw(tap), ci], and
 * db[co] = sum of dout[n,h,w,co] (db may be NULL). Split over pixel ranges
 * whose partial sums go to `scratch` and are reduced in a fixed order
 * (deterministic); scratch needs tsg_wgrad_scratch_bytes(...) bytes. */
size_t tsg_wgrad_scratch_bytes(int32_t n, int32_t h, int32_t w, int32_t cin_p, int32_t cout, int32_t taps);
tsg_status tsg_conv_wgrad(const uint16_t *in, int32_t n, int32_t h, int32_t w, int32_t in_ld, int32_t in_off,
                          int32_t cin, int32_t cin_p, const uint16_t *dout, int32_t d_ld, int32_t d_off,
                          int32_t cout, int32_t taps, float *dw, float *db, float *scratch, size_t scratch_bytes,
                          void *stream);

/* Same as tsg_conv_wgrad for a 1x1 convolution with a dense FP32 output
 * gradient [n*h*w][cout] (the head's gradient from the loss); dw is
 * [cout][cin], db [cout] (both required); cout*(cin+1) <= 1024; scratch needs
 * tsg_head_scratch_bytes(cout, cin) bytes. */
size_t tsg_head_scratch_bytes(int32_t cout, int32_t cin);
tsg_status tsg_conv_wgrad_f32(const uint16_t *in, int32_t n, int32_t h, int32_t w, int32_t in_ld,
                              int32_t in_off, int32_t cin, int32_t cin_p, const float *dout, int32_t cout,
                              float *dw, float *db, float *scratch, size_t scratch_bytes, void *stream);

/* Input gradient of the 1x1 head from its dense FP32 output gradient:
 * din[n,h,w,ci] = sum_co dout[n,h,w,co] * w[co][ci], times GELU'(z) of the
 * head's input when zbuf is given. */
tsg_status tsg_head_dgrad(const float *dout, int32_t npix, int32_t cout, const float *w, int32_t cin,
                          uint16_t *din, int32_t din_ld, int32_t din_off, const uint16_t *zbuf, int32_t z_ld,
                          int32_t z_off, void *stream);

/* 2x2 average pooling (h, w even) and its gradient; nearest-neighbour x2
 * upsampling and its gradient (sum of the 4 children). c channels. */
tsg_status tsg_avgpool2(const uint16_t *in, int32_t n, int32_t h, int32_t w, int32_t c, int32_t in_ld,
                        int32_t in_off, uint16_t *out, int32_t out_ld, int32_t out_off, void *stream);
tsg_status tsg_avgpool2_bwd(const uint16_t *dout, int32_t n, int32_t h, int32_t w, int32_t c, int32_t d_ld,
                            int32_t d_off, uint16_t *din, int32_t din_ld, int32_t din_off, int32_t accumulate,
                            void *stream);
tsg_status tsg_upsample2(const uint16_t *in, int32_t n, int32_t h, int32_t w, int32_t c, int32_t in_ld,
                         int32_t in_off, uint16_t *out, int32_t out_ld, int32_t out_off, void *stream);
tsg_status tsg_upsample2_bwd(const uint16_t *dout, int32_t n, int32_t h, int32_t w, int32_t c, int32_t d_ld,
                             int32_t d_off, uint16_t *din, int32_t din_ld, int32_t din_off, void *stream);

/* The two gradients above followed by the backward through the GELU that
 * produced the forward input of the pooling (or the upsampled tensor): din is
 * then (its pooling / upsampling gradient, plus din's old value when
 * accumulate) times GELU'(z), z the GELU's pre-activation in din's layout
 * (own stride and offset), in one pass; equal to the plain call followed by
 * tsg_dgelu up to one BF16 rounding of the intermediate. */
tsg_status tsg_avgpool2_bwd_dgelu(const uint16_t *dout, int32_t n, int32_t h, int32_t w, int32_t c, int32_t d_ld,
                                  int32_t d_off, uint16_t *din, int32_t din_ld, int32_t din_off, int32_t accumulate,
                                  const uint16_t *z, int32_t z_ld, int32_t z_off, void *stream);
tsg_status tsg_upsample2_bwd_dgelu(const uint16_t *dout, int32_t n, int32_t h, int32_t w, int32_t c, int32_t d_ld,
                                   int32_t d_off, uint16_t *din, int32_t din_ld, int32_t din_off, const uint16_t *z,
                                   int32_t z_ld, int32_t z_off, void *stream);

/* Elementwise on views of npix pixels x c channels:
 * tsg_add_inplace: a <- a + b (gradients meeting at a skip connection);
 * tsg_dgelu: d <- d * GELU'(z) (backward through GELU where it cannot be
 * fused into the next convolution's input gradient). GELU is the exact
 * z/2 (1 + erf(z/sqrt 2)). */
tsg_status tsg_add_inplace(uint16_t *a, int32_t a_ld, int32_t a_off, const uint16_t *b, int32_t b_ld,
                           int32_t b_off, int32_t npix, int32_t c, void *stream);
tsg_status tsg_dgelu(uint16_t *d, int32_t d_ld, int32_t d_off, const uint16_t *z, int32_t z_ld, int32_t z_off,
                     int32_t npix, int32_t c, void *stream);

/* Mean squared error over count = npix*c values of pred (fp32) against
 * target (fp32): *loss = mean((pred - target)^2) (fp32 scalar on device,
 * summed in a fixed order) and dpred = 2 (pred - target) / count (fp32). */
tsg_status tsg_mse(const float *pred, const float *target, int64_t count, float *loss, float *dpred,
                   float *scratch, void *stream);

/* AdamW (Loshchilov and Hutter, decoupled weight decay) on n FP32 values:
 * m = b1 m + (1-b1) g; v = b2 v + (1-b2) g^2;
 * p -= lr * (m / (1 - b1^t) / (sqrt(v / (1 - b2^t)) + eps) + wd * p), t = step >= 1. */
tsg_status tsg_adamw(float *p, const float *g, float *m, float *v, int64_t n, float lr, float b1, float b2,
                     float eps, float wd, int32_t step, void *stream);

/* FP32 [npix][c] -> BF16 view with channel padding to cp (zeros). */
tsg_status tsg_to_bf16(const float *src, int32_t npix, int32_t c, uint16_t *dst, int32_t cp, void *stream);

/* Nearest-neighbour distance: for each of nq query vectors (dim d, fp32),
 * dist2[i] = min_j |q_i - t_j|^2 over nt reference vectors, index[i] = argmin
 * (lowest index on ties). */
tsg_status tsg_nn_dist(const float *q, int32_t nq, const float *t, int32_t nt, int32_t d, float *dist2,
                       int32_t *index, void *stream);

/* Router features of n gap fields [n][h][w] (fp32): out[k] (row length
 * (h/f)(w/f) + 1) holds the f x f box means of field k in row-major order
 * followed by depth[k] * depth_scale. h and w must be multiples of f. */
tsg_status tsg_features(const float *gap, int32_t n, int32_t h, int32_t w, int32_t f, const float *depth,
                        float depth_scale, float *out, void *stream);

/* Per-sample mean squared difference of channel ch of two [n][npix][c] fp32
 * arrays: out[k] = mean_p (a[k][p][ch] - b[k][p][ch])^2 (fixed-order sum). */
tsg_status tsg_channel_mse(const float *a, const float *b, int32_t n, int32_t npix, int32_t c, int32_t ch,
                           float *out, void *stream);

/* Symmetry copies of n samples (x [n][res][res][2], y [n][res][res][3], fp32,
 * row = y index, column = x index): sample k is transformed by ops[k] (device
 * int32): bit 2 transposes x <-> y, bit 0 mirrors x, bit 1 mirrors y, applied
 * in that order; the target's (ux, uy) components are turned with the field
 * (swapped by the transpose, negated by the mirror of their axis). Outputs
 * must not alias the inputs. The elastomer block, its lattice and grid are
 * symmetric under these eight maps, so each copy is again a valid sample. */
tsg_status tsg_augment(const float *x, const float *y, int32_t n, int32_t res, const int32_t *ops, float *x_out,
                       float *y_out, void *stream);

/* Contact term of the surrogate's output, added in FP32 after the head:
 * out[p][2] += scale * min(x[p][0], 0) for p < npix, with out the head's
 * [npix][3] output and x the FP32 input [npix][2] (channel 0 the gap field).
 * Where the indenter is below the undeformed face, the sticking surface
 * follows it, so this term carries the large part of u_z exactly and the
 * network (BF16 storage) only learns the smooth remainder. */
tsg_status tsg_contact_residual(float *out, const float *x, int64_t npix, float scale, void *stream);

const char *tsg_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* TSG_H */
