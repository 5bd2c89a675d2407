/*
 * radiotrace -- learned surrogate for emitter -> receiver solves on MI355X.
 *
 * A multilayer perceptron maps a source/receiver pair and the firn profile
 * to the launch angles, travel times, path lengths and amplitudes of its
 * direct and surface-reflected rays, plus whether each exists and whether
 * its family has more than one ray to the receiver.  It is
 * trained on solutions of the tracer (radiotrace_solve.h) and used only as a
 * seed: every prediction is verified by shooting (raytrace_solve_seeded),
 * and the tracer's full solve is the fallback.  The paper has no surrogate;
 * this is an accelerator of the receiver/emitter set-ups it supports
 * (section 2, paragraph after the Fig. 1 example).
 *
 * Network (fixed): inputs x (RT_MLP_IN = 5 features) -> 4 hidden layers of
 * RT_MLP_WIDTH = 256 units with SiLU, s(z) = z / (1 + exp(-z)) -> RT_MLP_OUT
 * = 12 outputs.  Layer l computes z = W_l a + b_l with W_l of shape
 * [n_out][n_in] (row-major).  Arithmetic: BF16 operands (weights and
 * activations rounded to nearest even), FP32 accumulation on the matrix
 * cores, FP32 bias, activation, loss and optimiser.
 *
 * Parameters are one FP32 device array of rt_mlp_param_count() values:
 * for l = 0..4, W_l (n_out * n_in values) then b_l (n_out values), with
 * (n_in, n_out) = (5, 256), (256, 256) x 3, (256, 12).
 *
 * Features, targets and the loss are defined by the caller's normalisation
 * (the Python surrogate module documents the one it uses).  The loss is
 *   L = 1/B sum_b [ sum_f m_bf sum_q (y_b,4f+q - t_b,4f+q)^2
 *                   + sum_f BCE(y_b,8+f ; m_bf) + sum_f BCE(y_b,10+f ; r_bf) ]
 * over a batch of B rows, families f = 0, 1, regression outputs q = 0..3,
 * targets t (8 per row), labels (4 per row, 0 or 1: m_b0, m_b1, r_b0,
 * r_b1), and BCE(y; m) = log(1 + exp(y)) - m y (outputs 8 .. 11 are
 * logits).
 *
 * Conventions of radiotrace.h hold: device arrays owned by the caller,
 * asynchronous on 'stream', no allocation (scratch = caller workspace),
 * kernel launches only (graph-capturable).
 */
#ifndef RADIOTRACE_MLP_H
#define RADIOTRACE_MLP_H

#include "radiotrace.h"
#include "radiotrace_solve.h"

#ifdef __cplusplus
extern "C" {
#endif

#define RT_MLP_IN 5
#define RT_MLP_WIDTH 256
#define RT_MLP_HIDDEN 4
#define RT_MLP_OUT 12
#define RT_MLP_TARGETS 8
#define RT_MLP_LABELS 4

/* The surrogate network has no counterpart in the paper: it accelerates the
 * receiver/emitter set-ups of section 2 by seeding the shooting solver, and
 * every solution it seeds is verified by a trace (or solved by the tracer).
 * Number of FP32 parameters (201,996). */
int64_t rt_mlp_param_count(void);

/* Workspace bytes for batches of up to 'batch' rows; training != 0 adds the
 * buffers of the backward pass.  The workspace also holds the BF16 copies
 * of the weights written by rt_mlp_pack / rt_mlp_adam. */
rt_status rt_mlp_workspace_bytes(int64_t batch, int32_t training, size_t* bytes);

/* Round the FP32 parameters to the BF16 copies the matrix kernels read. */
rt_status rt_mlp_pack(const float* params, void* workspace, size_t workspace_bytes,
                      void* stream);

/* y[B][12] = network(x[B][5]) with the packed weights; biases are read from
 * 'params'.  1 <= batch <= the workspace's batch.  One launch for the whole
 * network (the activations of a tile of 128 rows stay on chip between the
 * layers). */
rt_status rt_mlp_forward(const float* params, const float* x, int64_t batch, float* y,
                         void* workspace, size_t workspace_bytes, void* stream);

/* Plumbing: the same forward as one matrix-core launch per layer, the
 * activations going through the workspace; results equal rt_mlp_forward's
 * bit for bit (the same products in the same order). */
rt_status rt_mlp_forward_layers(const float* params, const float* x, int64_t batch, float* y,
                                void* workspace, size_t workspace_bytes, void* stream);

/* Forward and backward pass of the loss above: grad[rt_mlp_param_count()]
 * receives dL/dparams (overwritten), *loss (device, one float) the loss.
 * targets [B][8], labels [B][4].  Needs a training workspace. */
rt_status rt_mlp_gradients(const float* params, const float* x, const float* targets,
                           const float* labels, int64_t batch, float* grad, float* loss,
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

/* ------------------------------------------------------------------------
 * Surrogate-seeded solves.
 *
 * Normalisation of the network's inputs and outputs (the definition the
 * feature, target and decode kernels implement):
 *   features  x0 = (zs - 1025)/975, x1 = (zr - 100)/100,
 *             x2 = (dist - 1505)/1495, x3 = (z0 - 80)/40,
 *             x4 = (dn - 0.425)/0.075
 *             (z0, dn: scale depth and index contrast of the firn profile
 *             n = a - dn exp(-z/z0); the ranges map to [-1, 1])
 *   targets   per family f (outputs 4f .. 4f+3):
 *             theta / (pi/2) - 1, c0 t / 3000 m - 1, s / 3000 m - 1,
 *             2 A - 1 with A = sqrt((|A_s|^2 + |A_p|^2) / 2);
 *   labels    m_f = 1 where the tracer found the solution, r_f = 1 where it
 *             found more than one root (roots >= 2)
 *   logits    outputs 8 + f: existence of family f's solution;
 *             outputs 10 + f: more than one root in family f.
 *
 * Seeded secant of one (pair, family) entry: shot at the seed theta0, then
 * at theta0 + dseed (theta0 - dseed if that leaves (0, pi)), then secant
 * steps theta_{k+1} = theta_k - m_k (theta_k - theta_{k-1}) / (m_k -
 * m_{k-1}); the entry is solved by the first shot that meets the receiver
 * plane with |miss| <= verify_tol (that shot is its verification), and
 * fails at a shot that does not meet the receiver plane, a step outside
 * (0, pi), or after max_shots shots. */
typedef struct {
  double z0, dn;       /* profile features of the medium */
  double verify_tol;   /* |miss| of the verifying shot (m), > 0 */
  double dseed;        /* second shot offset (rad), > 0 */
  int32_t max_shots;   /* shots per seeded entry, 2..64 */
  float absent_logit;  /* existence logit at or below which an entry is not
                          seeded (the tracer solves it) */
  float multi_logit;   /* several-roots logit above which an entry is not
                          seeded (the tracer picks its first arrival); a
                          low value such as -10 sends every family the
                          network is unsure of to the tracer */
} rt_surrogate_params;

/* How each entry [2 pair + family] of a surrogate solve was decided. */
enum {
  RT_PATH_SURROGATE = 0, /* network seed, verified by a shot */
  RT_PATH_TRACER = 1     /* the tracer's full solve of the entry's family */
};

/* Seeded secant (above) of every entry [2 n] with seed_try != 0: results
 * into out (found = verified; the other fields those of the verifying
 * shot), verify[2 n] = 1 (verified) or 0 (not) for the tried entries,
 * untouched otherwise.  Workspace: 4 KiB. */
rt_status raytrace_solve_seeded(const rt_field* field, const rt_boundaries* boundaries,
                                double tol, const rt_step_limits* limits,
                                const rt_pairs* pairs, const double* seed,
                                const int32_t* seed_try, const rt_surrogate_params* sp,
                                rt_solve_outputs* out, int32_t* verify, void* workspace,
                                size_t workspace_bytes, void* stream, const rt_tuning* tuning);

/* Features [n][5] (FP32) of the pairs in the profile (z0, dn). */
rt_status rt_surrogate_features(const rt_pairs* pairs, double z0, double dn, float* x,
                                void* stream);

/* Training targets [n][8] and labels [n][4] (FP32) from solve results. */
rt_status rt_surrogate_targets(const rt_solve_outputs* solved, int64_t n, float* targets,
                               float* labels, void* stream);

/* Workspace bytes of raytrace_solve_surrogate for n_pairs pairs. */
rt_status rt_surrogate_workspace_bytes(const rt_field* field, int64_t n_pairs,
                                       const rt_solve_params* fallback, size_t* bytes);

/* Solve every pair with the network as seed: features -> network
 * (mlp_params, FP32 device array) -> per entry, the seeded secant when the
 * network predicts one root (existence logit > absent_logit, several-roots
 * logit <= multi_logit); every entry that is not seeded or whose seed is not
 * verified is solved by the tracer's full solve of its family (raytrace_solve
 * with 'fallback'), so the network never decides that an entry has no
 * solution.  On the device (no host synchronisation).  Results in out as
 * for raytrace_solve; path [2 n] (device) receives RT_PATH_*;
 * *fallback_pairs (device, one int64) the number of pairs with an entry
 * solved by the tracer; out->stats the shots and steps of the seeded phase
 * plus the fallback solve.  tuning (may be NULL): block size and refill
 * threshold of the seeded phase and of the tracer's solve, whose scan
 * interleave and fused launch it also sets (results do not depend on it);
 * its events are not recorded. */
rt_status raytrace_solve_surrogate(const rt_field* field, const rt_boundaries* boundaries,
                                   double tol, const rt_step_limits* limits,
                                   const rt_pairs* pairs, const rt_solve_params* fallback,
                                   const rt_surrogate_params* sp, const float* mlp_params,
                                   rt_solve_outputs* out, int32_t* path,
                                   int64_t* fallback_pairs, void* workspace,
                                   size_t workspace_bytes, void* stream,
                                   const rt_tuning* tuning);

#ifdef __cplusplus
}
#endif
#endif /* RADIOTRACE_MLP_H */
