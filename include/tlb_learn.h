/*
 * tlb_learn.h -- learned correction of a coarsened torus step (an extension of the method of
 * arXiv:1904.10070; the paper itself has no learned part).
 *
 * A coarse grid, k times coarser than a fine one in each angle, takes one time step of the
 * ordinary scheme (tlb_step_n; its time step is usually k times the fine one).  A small
 * periodic convolutional network then reads the coarse state's moments and the metric factor
 * and predicts how the state should change to follow the fine solution; the correction is
 * applied to the populations through the equilibrium, which keeps the hydrodynamic moments
 * consistent:
 *
 *   network   five 3x3 convolutions, periodic in theta and phi, widths
 *             6 -> 32 -> 32 -> 32 -> 32 -> 4, ReLU between layers.  Input channels per node:
 *             (phi - s0) c0, (n - s1) c1, (u_theta - s2) c2, (u_phi - s3) c3 (shift s and scale
 *             c of the descriptor), r, and the metric factor J = R + r cos theta (eq. torus,
 *             appendix A).  Output z, whose channels times out_scale are the corrections
 *             (dphi, dn, du_theta, du_phi).  Tap t = 3 (dy + 1) + (dx + 1) reads node
 *             (theta_{q+dy}, phi_{s+dx}).
 *   numerics  products on the matrix cores in bfloat16 with FP32 accumulation: the input
 *             features, the weights as used, the hidden activations and the back-propagated
 *             error signals are rounded to bfloat16 (nearest, ties to even); biases, the last
 *             layer's output, the loss, the gradients and the Adam state are FP32 (gradient
 *             sums over blocks in FP64).
 *   correct   dphi and dn lose their area-weighted means (so mass and the J-weighted sum of
 *             phi are unchanged), then f += f_eq(n + dn, u + du) - f_eq(n, u) with the
 *             equilibrium of eq. feq, and phi += dphi.  In the learned step, corrections
 *             outside the descriptor's apply_mask are zero.
 *   train     loss L = sum_c w_c (z_c - y_c / out_scale_c)^2 / (4 N n_theta n_phi) over a
 *             batch of N samples, y the target corrections; its gradient with respect to the
 *             FP32 weights (through the bfloat16 rounding unchanged); Adam (Kingma & Ba).
 *
 * Parameters are one flat FP32 vector of TLB_CNN_PARAMS values, layer by layer:
 * W[c_out][9][c_in] then b[c_out].
 *
 * Data layouts (device memory, caller-owned unless stated):
 *   moment samples  float[n_samples][n_theta][n_phi][4] = (phi, n, u_theta, u_phi)
 *   target samples  float[n_samples][n_theta][n_phi][4] = (dphi, dn, du_theta, du_phi)
 *   corrections     float[n_theta][n_phi][4], physical units
 *   sample indices  int32_t[n] (device): batch slot i reads sample idx[i]; NULL = 0..n-1.
 *
 * Streams.  A network handle enqueues its work on the stream given at its creation, except
 * tlb_learned_step_n, which uses the grid's stream; the caller orders the two streams when
 * they differ.  Functions that return host values (loss, gradient, parameters, statistics)
 * wait for their stream.  Errors as in tlb.h (tlb_last_error).
 */
#ifndef TLB_LEARN_H
#define TLB_LEARN_H

#include "tlb.h"

#ifdef __cplusplus
extern "C" {
#endif

#define TLB_CNN_WIDTH 32
#define TLB_CNN_LAYERS 5
#define TLB_CNN_PARAMS 30660

typedef struct tlb_cnn tlb_cnn;

/* Descriptor of a network: the torus and grid it runs on (n_theta x n_phi nodes, radii r < R
 * for the J input), the largest batch of samples a call may pass (sizes the workspace:
 * about 420 bytes per node and sample), which corrections the learned step applies, the
 * input normalisation, the output scale and the loss weights.                             */
typedef struct {
  double r, R;
  int32_t n_theta, n_phi;
  int32_t max_batch;
  uint32_t apply_mask; /* bit c set: correction c is applied (0 = all four)             */
  float in_shift[4], in_scale[4];
  float out_scale[4];
  float loss_weight[4];
} tlb_cnn_desc;

/* Adam hyper-parameters of one update; step counts from 1 (bias correction 1 - beta^step). */
typedef struct {
  float lr, beta1, beta2, eps;
  int32_t step;
} tlb_adam;

/* Create a network with zero weights; load weights with tlb_cnn_set_params.  The handle owns
 * its device workspaces: bf16 activations, error signals and outputs of max_batch samples
 * (416 B per node and sample), the weights, gradients and Adam moments, and 28 MB of
 * per-workgroup partial gradients; freed by tlb_cnn_destroy.  Errors: TLB_EINVAL (sizes,
 * radii, non-finite or zero scales), TLB_ENOMEM, TLB_EHIP.                                  */
int32_t tlb_cnn_create(const tlb_cnn_desc* desc, void* hip_stream, tlb_cnn** out);
void tlb_cnn_destroy(tlb_cnn* net);

/* Copy TLB_CNN_PARAMS FP32 values from / to host memory (synchronous).  set_params also
 * clears the Adam moments.                                                                 */
int32_t tlb_cnn_set_params(tlb_cnn* net, const float* host_params);
int32_t tlb_cnn_get_params(tlb_cnn* net, float* host_params);

/* Corrections for n samples: out[i] = z(moments[idx[i]]) * out_scale, float[n][nt][np][4]. */
int32_t tlb_cnn_forward(tlb_cnn* net, const float* moments, const int32_t* idx, int32_t n,
                        float* out);

/* Loss (host double, may be NULL) and its gradient with respect to the weights (host float
 * array of TLB_CNN_PARAMS, may be NULL) on a batch, weights unchanged.                     */
int32_t tlb_cnn_gradient(tlb_cnn* net, const float* moments, const float* targets,
                         const int32_t* idx, int32_t n, double* loss, float* host_grad);

/* One training step: forward, loss, backward, Adam update of the weights.  loss (host, may
 * be NULL; then nothing waits) receives the loss before the update.                        */
int32_t tlb_cnn_train_step(tlb_cnn* net, const float* moments, const float* targets,
                           const int32_t* idx, int32_t n, const tlb_adam* adam, double* loss);

/* Sums of x and x^2 of each of the 4 channels of float[count][4] data (device), in FP64
 * with a fixed order: out[c] = sum x_c, out[4 + c] = sum x_c^2 (host array of 8).  For
 * choosing in_shift / in_scale / out_scale.  Waits for the stream.  The partial sums go to
 * a 33 KB workspace per device that the first call on the device allocates and the process
 * keeps (later calls allocate nothing).                                                    */
int32_t tlb_learn_stats(const float* data, int64_t count, void* hip_stream, double out[8]);

/* Restrict the state of `fine` onto `coarse` (overwriting its state): fine n_theta and n_phi
 * must be k times the coarse ones for one even k >= 2, same radii, flags and precision.  Every
 * population and phi is averaged with the full-weighting stencil of width 2k + 1 (weight 1/2
 * at its two ends), weighted by J along theta, so that the J-weighted totals carry over.
 * Enqueued on the coarse grid's stream (the caller orders it after the fine grid's work).  */
int32_t tlb_restrict(const tlb_grid* fine, tlb_grid* coarse);

/* Moments (phi, n, u_theta, u_phi) of a grid's state into float[nt][np][4] (device).
 * With `truth` non-NULL (same sizes and precision), also targets = moments(truth) -
 * moments(grid) into float[nt][np][4]; moments are summed and differenced in FP64 before
 * rounding to float.  Enqueued on the grid's stream.                                      */
int32_t tlb_learn_pair(const tlb_grid* grid, const tlb_grid* truth, float* moments,
                       float* targets);

/* Apply corrections float[nt][np][4] (device, physical units) to a grid's state as
 * described above.  Enqueued on the grid's stream; does not wait and allocates nothing (its
 * per-row sums use a workspace made with the grid).                                        */
int32_t tlb_apply_correction(tlb_grid* grid, const float* corrections);

/* n_steps learned coarse steps: each is one tlb_step_n step of the grid followed by the
 * network's correction of the result.  The grid must match the network's n_theta, n_phi.
 * The network of a step runs as one launch that forms the moments itself (tiles with a
 * five-node halo, activations on chip); the corrections it applies are bit for bit those of
 * tlb_cnn_forward on the moments from tlb_learn_pair.  Runs of 32 steps replay a prebuilt
 * graph unless the grid has TLB_NO_GRAPH.                                                  */
int32_t tlb_learned_step_n(tlb_grid* grid, tlb_cnn* net, int64_t n_steps);

#ifdef __cplusplus
}
#endif

#endif /* TLB_LEARN_H */
