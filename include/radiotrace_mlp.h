/*
 * radiotrace -- learned surrogate for emitter -> receiver solves on MI355X.
 *
 * A multilayer perceptron maps a source/receiver pair and the firn profile
 * to the launch angles, travel times, path lengths and amplitudes of its
 * direct and surface-reflected rays, plus whether each exists.  It is
 * trained on solutions of the tracer (radiotrace_solve.h) and used only as a
 * seed: every prediction is verified by shooting (raytrace_solve_seeded),
 * and the tracer's full solve is the fallback.  The paper has no surrogate;
 * this is an accelerator of the receiver/emitter set-ups it supports
 * (section 2, paragraph after the Fig. 1 example).
 *
 * Network (fixed): inputs x (RT_MLP_IN = 5 features) -> 4 hidden layers of
 * RT_MLP_WIDTH = 256 units with SiLU, s(z) = z / (1 + exp(-z)) -> RT_MLP_OUT
 * = 10 outputs.  Layer l computes z = W_l a + b_l with W_l of shape
 * [n_out][n_in] (row-major).  Arithmetic: BF16 operands (weights and
 * activations rounded to nearest even), FP32 accumulation on the matrix
 * cores, FP32 bias, activation, loss and optimiser.
 *
 * Parameters are one FP32 device array of rt_mlp_param_count() values:
 * for l = 0..4, W_l (n_out * n_in values) then b_l (n_out values), with
 * (n_in, n_out) = (5, 256), (256, 256) x 3, (256, 10).
 *
 * Features, targets and the loss are defined by the caller's normalisation
 * (the Python surrogate module documents the one it uses).  The loss is
 *   L = 1/B sum_b [ sum_f m_bf sum_q (y_b,4f+q - t_b,4f+q)^2
 *                   + sum_f BCE(y_b,8+f ; m_bf) ]
 * over a batch of B rows, families f = 0, 1, regression outputs q = 0..3,
 * targets t (8 per row), masks m (2 per row, 0 or 1), and
 * BCE(y; m) = log(1 + exp(y)) - m y (outputs 8, 9 are logits).
 *
 * Conventions of radiotrace.h hold: device arrays owned by the caller,
 * asynchronous on 'stream', no allocation (scratch = caller workspace),
 * kernel launches only (graph-capturable).
 */
#ifndef RADIOTRACE_MLP_H
#define RADIOTRACE_MLP_H

#include "radiotrace.h"

#ifdef __cplusplus
extern "C" {
#endif

#define RT_MLP_IN 5
#define RT_MLP_WIDTH 256
#define RT_MLP_HIDDEN 4
#define RT_MLP_OUT 10
#define RT_MLP_TARGETS 8

/* Number of FP32 parameters (201,482). */
int64_t rt_mlp_param_count(void);

/* Workspace bytes for batches of up to 'batch' rows; training != 0 adds the
 * buffers of the backward pass.  The workspace also holds the BF16 copies
 * of the weights written by rt_mlp_pack / rt_mlp_adam. */
rt_status rt_mlp_workspace_bytes(int64_t batch, int32_t training, size_t* bytes);

/* Round the FP32 parameters to the BF16 copies the matrix kernels read. */
rt_status rt_mlp_pack(const float* params, void* workspace, size_t workspace_bytes,
                      void* stream);

/* y[B][10] = network(x[B][5]) with the packed weights; biases are read from
 * 'params'.  1 <= batch <= the workspace's batch. */
rt_status rt_mlp_forward(const float* params, const float* x, int64_t batch, float* y,
                         void* workspace, size_t workspace_bytes, void* stream);

/* Forward and backward pass of the loss above: grad[rt_mlp_param_count()]
 * receives dL/dparams (overwritten), *loss (device, one float) the loss.
 * targets [B][8], mask [B][2].  Needs a training workspace. */
rt_status rt_mlp_gradients(const float* params, const float* x, const float* targets,
                           const float* mask, int64_t batch, float* grad, float* loss,
                           void* workspace, size_t workspace_bytes, void* stream);

typedef struct {
  float lr, beta1, beta2, eps;
} rt_adam;

/* One Adam step (Kingma & Ba) on every parameter, 'step' = 1, 2, ...:
 * m = b1 m + (1 - b1) g; v = b2 v + (1 - b2) g^2;
 * p -= lr (m / (1 - b1^step)) / (sqrt(v / (1 - b2^step)) + eps);
 * then the BF16 copies are re-packed. */
rt_status rt_mlp_adam(float* params, float* m, float* v, const float* grad, int64_t step,
                      const rt_adam* hp, void* workspace, size_t workspace_bytes,
                      void* stream);

#ifdef __cplusplus
}
#endif
#endif /* RADIOTRACE_MLP_H */
