/*
 * surrogate.h -- C ABI of the operators of the learned surrogate: a 3-level 3-D convolutional
 * encoder-decoder that maps coarse-grained phase and velocity fields of the lattice
 * Boltzmann method to the same fields a fixed number of steps later.
 *
 * All tensors are device pointers in channels-last layout, [n][d][h][w][c] with c fastest;
 * activations and weights are BF16 (uint16_t bit patterns), accumulation is FP32 on the
 * matrix cores (v_mfma_f32_32x32x16_bf16).  Convolutions are 3x3x3, stride 1, zero padding 1;
 * weights are [27][cout][cin] with tap = (dz+1)*9 + (dy+1)*3 + (dx+1).  Channel counts:
 * cin in {8, 16, 32, 64, 128} for the forward convolution (a multiple of 8 for the weight
 * gradient), cout a multiple of 32.  Every call enqueues work on `stream` (a
 * hipStream_t or NULL) and returns 0, or a negative value for invalid sizes (nothing is
 * launched then).  The caller owns all memory; scratch buffers are passed in and their
 * required sizes are given by the *_scratch_bytes calls.
 */
#ifndef SURROGATE_H_
#define SURROGATE_H_

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* out = act(conv(in, w) + bias); act = max(0, .) if relu != 0.  in: [n][d][h][w][cin],
 * out: [n][d][h][w][cout] BF16 (out_f32 != NULL: written as FP32 there instead). */
int surr_conv3d_fwd(const uint16_t *in, const uint16_t *w, const float *bias, uint16_t *out, float *out_f32, int n,
                    int d, int h, int wd, int cin, int cout, int relu, void *stream);

/* Gradient of the input: din = conv_transpose(dout, w), i.e. the forward convolution with the
 * taps mirrored and the channel roles swapped (w_t: [27][cin][cout], made by
 * surr_conv3d_flip_weights).  cin a multiple of 32 here.  With relu_y (the ReLU output that
 * produced the layer's input, [n][d][h][w][cin]) not NULL, din is 0 where relu_y is not
 * positive: the gradient of the pre-activation, as surr_relu_bwd would give. */
int surr_conv3d_flip_weights(const uint16_t *w, uint16_t *w_t, int cin, int cout, void *stream);
int surr_conv3d_dgrad(const uint16_t *dout, const uint16_t *w_t, const uint16_t *relu_y, uint16_t *din, int n, int d,
                      int h, int wd, int cin, int cout, void *stream);

/* Gradient of the weights and bias: dw[27][cout][cin] = sum_v dout[v][co] in[v + tap][ci],
 * dbias[co] = sum_v dout[v][co], FP32, reduced in a fixed order through `scratch`. */
size_t surr_conv3d_wgrad_scratch_bytes(int n, int d, int h, int wd, int cin, int cout);
int surr_conv3d_wgrad(const uint16_t *in, const uint16_t *dout, float *dw, float *dbias, void *scratch, int n, int d,
                      int h, int wd, int cin, int cout, void *stream);

/* dx = dy where y > 0, else 0 (y: the ReLU output). count elements; dx may alias dy. */
int surr_relu_bwd(const uint16_t *y, const uint16_t *dy, uint16_t *dx, long long count, void *stream);

/* 2x2x2 average pooling [n][d][h][w][c] -> [n][d/2][h/2][w/2][c] (d, h, w even) and its
 * gradient; (d, h, w) are the dimensions of the fine tensor (in, din).  Nearest 2x
 * upsampling with an added skip tensor, out = up(in) + skip, and its gradient with respect to
 * in (the gradient of skip is dout itself); (d, h, w) are the dimensions of the coarse tensor
 * (in, din), out and skip being 2d x 2h x 2w.  c a multiple of 8 and every pointer 16-byte
 * aligned (8 channels move per access), else -1.  surr_up_bwd with relu_y (shaped as din) not
 * NULL gives 0 where relu_y is not positive. */
int surr_pool_fwd(const uint16_t *in, uint16_t *out, int n, int d, int h, int wd, int c, void *stream);
int surr_pool_bwd(const uint16_t *dout, uint16_t *din, int n, int d, int h, int wd, int c, void *stream);
int surr_up_add_fwd(const uint16_t *in, const uint16_t *skip, uint16_t *out, int n, int d, int h, int wd, int c,
                    void *stream);
int surr_up_bwd(const uint16_t *dout, const uint16_t *relu_y, uint16_t *din, int n, int d, int h, int wd, int c,
                void *stream);

/* Mean-squared error over the first `used` of `stride` channels of pred (FP32) against
 * target (FP32, `used` channels): dpred = 2 (pred - target) / (count * used) written as
 * BF16 with zeros in the unused channels; the per-block partial sums of the squared error
 * go to loss_part (ceil(count / 256) floats), summed by the caller.  count voxels; stride a
 * multiple of 8 and dpred 16-byte aligned. */
int surr_mse(const float *pred, const float *target, uint16_t *dpred, float *loss_part, long long count, int stride,
             int used, void *stream);

/* One Adam step on FP32 master weights, refreshing their BF16 copy: m, v moments,
 * t the 1-based step count. */
int surr_adam(float *w, uint16_t *w_bf16, const float *g, float *m, float *v, long long count, float lr, float beta1,
              float beta2, float eps, int t, void *stream);

/* out = a + b element-wise in BF16 (FP32 sum, rounded); out may alias a or b.  With relu_y not
 * NULL, out is 0 where relu_y is not positive. */
int surr_add(const uint16_t *a, const uint16_t *b, const uint16_t *relu_y, uint16_t *out, long long count,
             void *stream);

/* FP32 <-> BF16 conversion (round to nearest even). */
int surr_to_bf16(const float *x, uint16_t *y, long long count, void *stream);
int surr_to_f32(const uint16_t *x, float *y, long long count, void *stream);

/* Network input: y[v][c] = bf16(x[v][c]) for c < c_src and 0 for c_src <= c < c_dst
 * (x: [nvox][c_src] FP32, y: [nvox][c_dst] BF16). */
int surr_pack_input(const float *x, uint16_t *y, long long nvox, int c_src, int c_dst, void *stream);

#ifdef __cplusplus
}
#endif

#endif /* SURROGATE_H_ */
