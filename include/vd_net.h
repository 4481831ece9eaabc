/*
 * vd_net.h -- C-ABI of the learned warm start of the lattice solver.
 *
 * Not part of the paper.  A small 3-D convolutional encoder-decoder predicts,
 * for every node of the finest lattice, the change of its displacement over
 * the coming frame; vd_solve_frame (vd.h) can start from that prediction and
 * keeps it only when it lowers the energy of eq. (1) against the plain
 * initialisation (the previous frame's state), so the plain flip-flop solve of
 * Sec. 7 always runs after it and judges it.
 *
 * Network (channels 16-32-64, 3x3x3 kernels, zero padding, ReLU, stride-2
 * convolutions down, nearest x2 up-sampling, skip concatenation):
 *   e0a = relu(conv(x, 8->16))           e0 = relu(conv(e0a, 16->16))
 *   e1a = relu(conv_s2(e0, 16->32))      e1 = relu(conv(e1a, 32->32))
 *   e2a = relu(conv_s2(e1, 32->64))      e2 = relu(conv(e2a, 64->64))
 *   u1  = relu(conv(up(e2), 64->32))     d1 = relu(conv([u1, e1], 64->32))
 *   u0  = relu(conv(up(d1), 32->16))     d0 = relu(conv([u0, e0], 32->16))
 *   out = conv(d0, 16->3)
 * A stride-2 convolution reads input position 2*o + tap - 1 (an axis of n
 * nodes becomes ceil(n/2)); up-sampling reads node j/2 and is cropped to the
 * skip tensor's size.  Training minimises the mean over nodes of
 * ||out - target||^2 with Adam (Kingma & Ba, bias-corrected).
 *
 * Arithmetic: bfloat16 operands on the matrix cores with float32
 * accumulation; activations and activation gradients are stored as bfloat16
 * (round to nearest even), the output, the loss, the parameter gradients and
 * the Adam state are float32.
 *
 * Layouts:
 *   - Input features x: [batch][nz][ny][nx][8] bfloat16 bit patterns
 *     (uint16), node (a,b,c) at a + nx*(b + ny*c) as in vd.h.  Channels:
 *     0-2 displacement t - t_hat of the previous frame, 3-5 its change from
 *     the frame before, 6 the weight-normalised point-to-plane residual
 *     splatted to the nodes, 7 validity (1 where a sample touches the node)
 *     -- all lengths in units of the finest spacing (see vd_warm_features).
 *   - Output and training target: [batch][3][N] float32 (x block, y block,
 *     z block per sample), the displacement change in units of the spacing.
 *   - Parameters: one float32 vector, layer by layer in the order above; per
 *     layer the weights W[c_out][c_in][dz][dy][dx] then the bias[c_out].  The
 *     input channels of a concatenation list the up-sampled branch first.
 *
 * Conventions (status codes, `mem`, streams, ownership) are those of vd.h.
 */
#ifndef VD_NET_H
#define VD_NET_H

#include <stdint.h>

#include "vd.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct vd_net vd_net;

/* Number of float32 parameters (weights and biases of all 11 layers). */
int64_t vd_net_param_count(void);

/* Create a network for grids of nx*ny*nz nodes (each >= 1) and up to
 * max_batch samples per call.  Allocates activations, gradients and the Adam
 * state; the parameters start at zero (call vd_net_set_params). */
int vd_net_create(int32_t nx, int32_t ny, int32_t nz, int32_t max_batch, void* stream,
                  vd_net** out);

/* Free the network.  NULL is a no-op. */
int vd_net_destroy(vd_net* n);

/* Load the float32 parameters (vd_net_param_count values), reset the Adam
 * moments and step count.  VD_EINVAL on a non-finite value. */
int vd_net_set_params(vd_net* n, const float* params, int32_t mem);

/* Copy the float32 parameters out.  Waits for the stream. */
int vd_net_get_params(vd_net* n, float* params, int32_t mem);

/* Inference: out = net(x) for `batch` samples (1 .. max_batch).  With
 * VD_MEM_DEVICE the call is asynchronous on the stream; with VD_MEM_HOST it
 * waits. */
int vd_net_forward(vd_net* n, const uint16_t* x, int32_t batch, float* out, int32_t mem);

/* Loss and parameter gradients (same layout as the parameters) at the current
 * parameters, without an update.  loss may be NULL.  Waits for the stream. */
int vd_net_gradients(vd_net* n, const uint16_t* x, const float* target, int32_t batch,
                     float* grad, double* loss, int32_t mem);

/* One training step: forward, loss, backward, one Adam update with step
 * size lr (beta1 0.9, beta2 0.999, eps 1e-8).  loss (may be NULL) receives the
 * loss before the update, which makes the call wait for the stream; without
 * it the step is asynchronous. */
int vd_net_train_step(vd_net* n, const uint16_t* x, const float* target, int32_t batch,
                      float lr, int32_t mem, double* loss);

/* Input features of the lattice's finest level for the coming frame, from
 * the current state (taken as the previous frame's solution, t^{k-1}), the
 * displacement prev2 of the frame before ([3][N] x/y/z blocks, world units,
 * NULL: no change) and the correspondences last given to
 * vd_set_constraints.  Channels 0-2 are d/h for the current displacement d,
 * channels 3-5 (d - prev2)/h (0 when prev2 is NULL).  Channel 6 at node i is
 *   sum_c alpha_ci w_c r_c / sum_c alpha_ci w_c,   r_c = n_c . (S(p_hat_c) - p_c)
 * over the dense samples c whose cell has node i as a corner (alpha the
 * trilinear weights of Sec. 4, S the warp at the current state, w_c the
 * sample weight times w_d), channel 7 is 1 where the denominator is > 0.
 * x receives [nz][ny][nx][8] bfloat16 bits.  VD_ESTATE without
 * constraints. */
int vd_warm_features(vd_lattice* l, const float* prev2, uint16_t* x, int32_t mem);

#ifdef __cplusplus
}
#endif

#endif /* VD_NET_H */
