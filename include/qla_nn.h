/*
 * qla_nn.h -- C ABI of the convolutional surrogate kernels in libqla.
 *
 * The surrogate learns the map (Q(t), n) -> Q(t + K) of the qubit lattice
 * algorithm (K whole steps of Eq. (23) or Eq. (28) of Vahala et al.,
 * arXiv:2301.13601) on periodic lattices. It is a convolutional U-net built
 * from the primitives below; the network itself (layer list, buffers,
 * training loop) is orchestrated by paper_2301_13601_amd/surrogate.py.
 *
 * Conventions:
 *  - Activations are NHWC: element (b, y, x, c) of a tensor with C channels
 *    is at ((b * H + y) * W + x) * C + c. Spatial indices wrap periodically
 *    (the lattice is periodic).
 *  - BF16 tensors are raw 16-bit bfloat16 words (uint16_t); accumulation is
 *    FP32; FP32 tensors are float.
 *  - 3x3 weights are [C_out][9][C_in], tap t = (dy + 1) * 3 + (dx + 1) for
 *    the input offset (dy, dx) in {-1, 0, 1}^2.
 *  - All pointers are device pointers owned by the caller; nothing is
 *    allocated. Work is enqueued on hip_stream (NULL: default stream) and
 *    is asynchronous. Each call returns 0 on success, QNN_EINVAL (-1) for
 *    bad sizes or null pointers, QNN_EDEVICE (-3) on a launch error; the
 *    message is available from qla_last_error().
 */
#ifndef QLA_NN_H
#define QLA_NN_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum { QNN_OK = 0, QNN_EINVAL = -1, QNN_EDEVICE = -3 };
enum { QNN_ACT_NONE = 0, QNN_ACT_LEAKY = 1 };   /* leaky ReLU, negative slope 1/8 */

/*
 * y = act(bias + conv3x3(x, w)), circular padding, on B images of H x W.
 *   x      BF16 [B*H*W][c_in], c_in a multiple of 16, 16-byte aligned
 *   w      BF16 [c_out][9][c_in], c_out a multiple of 32, 16-byte aligned
 *   bias   FP32 [c_out] or NULL
 *   y      [B*H*W][y_ld], BF16 (y_fp32 = 0) or FP32 (y_fp32 = 1); channels
 *          >= c_store are not written (c_store <= c_out, c_store <= y_ld)
 * MFMA (32x32x16 BF16) implicit GEMM: M = B*H*W pixels, N = c_out,
 * K = 9*c_in; FP32 accumulation of 16-channel MFMA products. B*H*W*max(c_in,
 * y_ld) must stay below 2^31 (QNN_EINVAL otherwise). The tiled kernels run
 * for W a multiple of 16 with c_in = 32 or 48 and c_out = 32, or with c_in =
 * 32 or 64, c_out = 64 and 256 or more tiles of 256 pixels, and otherwise
 * for W = 16, 32 or a multiple of 64; they sum the input channels 16 at a
 * time in increasing order, the nine taps in order within each 16, and give
 * bitwise the same result as each other. Other widths take a per-pixel
 * kernel that sums taps outer, channels inner (the last bits may differ).
 * All are fastest with BF16 output when c_store = c_out, y_ld is a multiple
 * of 8 and y is 16-byte aligned (else the per-pixel kernel runs).
 */
int qnn_conv3x3_fwd(int32_t B, int32_t H, int32_t W, const uint16_t *x, int32_t c_in,
                    const uint16_t *w, const float *bias, int32_t c_out, int32_t act,
                    void *y, int32_t y_fp32, int32_t y_ld, int32_t c_store, void *hip_stream);

/*
 * The forward convolution with its U-net neighbours folded in, for
 * inference (the training pass keeps the intermediate tensors, which its
 * backward pass reads):
 *   y = act(bias + conv3x3(U(x), w)) + add
 *   up = 1: x is BF16 [B*(H/2)*(W/2)][c_in] and U(x) its 2x nearest
 *           upsampling (qnn_upsample2), never stored; H and W even
 *   up = 0: x is BF16 [B*H*W][c_in] and U(x) = x
 *   add     BF16 [B*H*W][y_ld] or NULL, added to the rounded BF16 result
 *           and rounded again: bitwise qnn_conv3x3_fwd followed by qnn_add
 *   y       BF16 [B*H*W][y_ld], all c_out channels written
 * W must be 16, 32 or a multiple of 64; y_ld >= c_out, a multiple of 8; x,
 * w, add and y 16-byte aligned; otherwise QNN_EINVAL (and nothing runs).
 */
int qnn_conv3x3_fwd_fused(int32_t B, int32_t H, int32_t W, const uint16_t *x, int32_t c_in,
                          int32_t up, const uint16_t *w, const float *bias, int32_t c_out,
                          int32_t act, const uint16_t *add, uint16_t *y, int32_t y_ld,
                          void *hip_stream);

/*
 * The network's output layer and the unpacking of its result in one pass,
 * for inference:
 *   q[b][c][y][x] = scale[b] * act(bias + conv3x3(x, w))[b, y, x, c],
 *   c < n_planes
 *   x      BF16 [B*H*W][c_in], c_in = 32 or 48, 16-byte aligned
 *   w      BF16 [32][9][c_in] (c_out = 32), 16-byte aligned
 *   bias   FP32 [32] or NULL; scale FP32 [B]
 *   q      FP32 [B][n_planes][H][W], 1 <= n_planes <= 32
 * W must be a multiple of 16 and B*H*W*c_in below 2^31; otherwise QNN_EINVAL
 * (and nothing runs). Bitwise qnn_conv3x3_fwd with FP32 output followed by
 * qnn_unpack_output (n_planes = 6), without the intermediate tensor.
 */
int qnn_conv3x3_fwd_planes(int32_t B, int32_t H, int32_t W, const uint16_t *x, int32_t c_in,
                           const uint16_t *w, const float *bias, int32_t c_out, int32_t act,
                           const float *scale, int32_t n_planes, float *q, void *hip_stream);

/*
 * A convolution and the 2x2 average pooling of its result, for an encoder
 * level in inference:
 *   y     = act(bias + conv3x3(x, w))   BF16 [B*H*W][c_out]
 *   pool  = avgpool2(y)                 BF16 [B*(H/2)*(W/2)][c_out]
 * bitwise qnn_conv3x3_fwd (BF16, y_ld = c_store = c_out) followed by
 * qnn_avgpool2; where the convolution runs on the resident-weight tiles
 * (see qnn_conv3x3_fwd) the pooling is done as the tiles are stored, else the
 * two calls are made in turn. H and W even; x, w, y and pool 16-byte aligned;
 * c_in a multiple of 16, c_out of 32; B*H*W*max(c_in, c_out) below 2^31;
 * otherwise QNN_EINVAL (and nothing runs).
 */
int qnn_conv3x3_fwd_pool(int32_t B, int32_t H, int32_t W, const uint16_t *x, int32_t c_in,
                         const uint16_t *w, const float *bias, int32_t c_out, int32_t act,
                         uint16_t *y, uint16_t *pool, void *hip_stream);

/* wt = the weights of the adjoint convolution: wt[ci][8 - t][co] = w[co][t][ci]
 * (the data gradient of a circular 3x3 convolution is a 3x3 convolution of
 * the output gradient with the flipped, transposed kernel). */
int qnn_conv3x3_flip(const uint16_t *w, int32_t c_out, int32_t c_in, uint16_t *wt,
                     void *hip_stream);

/*
 * Weight and bias gradients of y = conv3x3(x, w) + bias:
 *   dw[co][t][ci] = sum_p dy[p][co] * x[p + offset(t)][ci]      (FP32)
 *   dbias[co]     = sum_p dy[p][co]                               (FP32, if non-NULL)
 *   x BF16 [P][c_in], dy BF16 [P][c_out]; c_in a multiple of 16, c_out a
 *   multiple of 32; P * max(c_in, c_out) < 2^31 (QNN_EINVAL otherwise).
 *   Any H, W; with x and dy 16-byte aligned and W a multiple of 8 the
 *   staged MFMA kernel runs, otherwise a slower one reading 2-byte elements.
 *   work FP32 scratch of qnn_wgrad_work_floats(...) floats (0 for sizes the
 *   call would reject); it holds one partial dW (and dbias) per pixel range
 *   until the call's kernels have run.
 * Deterministic: the pixel ranges' partial sums are folded in a fixed order,
 * so repeated calls give bitwise equal results.
 */
int64_t qnn_wgrad_work_floats(int32_t B, int32_t H, int32_t W, int32_t c_in, int32_t c_out);
int qnn_conv3x3_wgrad(int32_t B, int32_t H, int32_t W, const uint16_t *x, int32_t c_in,
                      const uint16_t *dy, int32_t c_out, float *dw, float *dbias, float *work,
                      void *hip_stream);

/* dz = dy * (y > 0 ? 1 : 1/8), the leaky ReLU backward from its output y
 * (in place allowed: dz may equal dy). n elements, BF16. */
int qnn_leaky_bwd(int64_t n, const uint16_t *y, const uint16_t *dy, uint16_t *dz, void *hip_stream);

/* y = a + b (BF16, n elements; y may alias a or b). */
int qnn_add(int64_t n, const uint16_t *a, const uint16_t *b, uint16_t *y, void *hip_stream);

/* 2x2 average pooling H x W -> H/2 x W/2 (H, W even), and its backward:
 * dx[b,y,x,c] (+)= dy[b,y/2,x/2,c] / 4 (accumulate = 1 adds into dx). */
int qnn_avgpool2(int32_t B, int32_t H, int32_t W, int32_t C, const uint16_t *x, uint16_t *y,
                 void *hip_stream);
int qnn_avgpool2_bwd(int32_t B, int32_t H, int32_t W, int32_t C, const uint16_t *dy,
                     uint16_t *dx, int32_t accumulate, void *hip_stream);

/* Nearest-neighbour 2x upsampling h x w -> 2h x 2w, and its backward
 * dx[b,y,x,c] = sum of the four dy it was copied to. */
int qnn_upsample2(int32_t B, int32_t h, int32_t w, int32_t C, const uint16_t *x, uint16_t *y,
                  void *hip_stream);
int qnn_upsample2_bwd(int32_t B, int32_t h, int32_t w, int32_t C, const uint16_t *dy,
                      uint16_t *dx, void *hip_stream);

/*
 * Per-sample scale for the network input: scale[b] = max |q| over the 6
 * planes of lattice sample idx[b] (1 if that maximum is 0).
 *   q FP32 [N][6][H][W]; idx int32 [B] (NULL: sample b is idx b); scale FP32 [B].
 */
int qnn_absmax(int32_t B, int32_t H, int32_t W, const float *q, const int32_t *idx, float *scale,
               void *hip_stream);

/*
 * Network input from lattice fields: for sample b, with s = idx_q[b] and
 * m = idx_n[b] (NULL: identity), Q = q[s] / scale[b]:
 *   channels  0..5   Q(y, x)
 *   channels  6..8   (n[m](y, x) - n_shift) / n_scale
 *   channels  9..14  Q(y, x - d)     (content displaced by +d along x)
 *   channels 15..20  Q(y, x + d)     (displaced by -d along x)
 *   channels 21..26  Q(y - d, x)     (displaced by +d along y)
 *   channels 27..32  Q(y + d, x)     (displaced by -d along y)
 *   channels 33..47  0
 * with periodic wrap; d = shift is the distance a vacuum wave travels over
 * the surrogate's jump, so each displaced copy lines up with the waves
 * that moved along one axis.
 *   q FP32 [N][6][H][W], n FP32 [M][3][H][W], scale FP32 [B],
 *   x BF16 [B*H*W][48], 16-byte aligned (-1 otherwise).
 */
int qnn_pack_input(int32_t B, int32_t H, int32_t W, const float *q, const int32_t *idx_q,
                   const float *n, const int32_t *idx_n, const float *scale, float n_shift,
                   float n_scale, int32_t shift, uint16_t *x, void *hip_stream);

/* Lattice fields from the network output: q[b][c][y][x] = y[b,y,x,c] * scale[b]
 * for c < 6 (y FP32 [B*H*W][y_ld]). */
int qnn_unpack_output(int32_t B, int32_t H, int32_t W, const float *y, int32_t y_ld,
                      const float *scale, float *q, void *hip_stream);

/*
 * Relative L2 loss over B samples and its gradient, against the lattice
 * fields target[idx_t[b]] / scale[b] (idx_t NULL: identity):
 *   loss = (1/B) sum_b |pred_b - t_b|^2 / |t_b|^2
 *   dpred (BF16 [P][d_ld], may be NULL; channels >= 6 set to 0) = d loss / d pred
 *   pred FP32 [P][pred_ld] (first 6 channels used), target FP32 [N][6][H][W].
 *   loss_out: FP64 device scalar; per_sample (FP64 [B], may be NULL) gets
 *   the relative errors |pred_b - t_b| / |t_b|.
 *   work: FP64 scratch of 64 * B doubles. B <= 1024.
 */
int qnn_rel_l2(int32_t B, int32_t H, int32_t W, const float *pred, int32_t pred_ld,
               const float *target, const int32_t *idx_t, const float *scale, uint16_t *dpred,
               int32_t d_ld, double *loss_out, double *per_sample, double *work, void *hip_stream);

/*
 * One Adam step (decoupled weight decay 0) on n parameters:
 *   m = b1 m + (1-b1) g;  v = b2 v + (1-b2) g^2
 *   p -= lr * (m / (1 - b1^t)) / (sqrt(v / (1 - b2^t)) + eps)
 * p, m, v, g FP32; p_bf16 receives the rounded parameters (may be NULL).
 */
int qnn_adam(int64_t n, float *p, float *m, float *v, const float *g, uint16_t *p_bf16, float lr,
             float b1, float b2, float eps, int32_t t, void *hip_stream);

/* FP64 values of device workspace qnn_compare needs for B samples. */
int64_t qnn_compare_work_doubles(int32_t B);

/* Per-sample comparison of B FP32 tensors of m values each (sample b at
 * offset b*m): rel[b] = |a_b - r_b| / |r_b| and en[b] = | |a_b|^2 - |r_b|^2 |
 * / |r_b|^2, accumulated in FP64. rel, en: FP64 device arrays of B; work:
 * caller-owned FP64 device scratch of qnn_compare_work_doubles(B) values.
 * B at most 65535. */
int qnn_compare(int32_t B, int64_t m, const float *a, const float *r, double *rel, double *en,
                double *work, void *hip_stream);

/* y = bf16(x) for n FP32 values (round to nearest even). */
int qnn_to_bf16(int64_t n, const float *x, uint16_t *y, void *hip_stream);

#ifdef __cplusplus
}
#endif

#endif /* QLA_NN_H */
