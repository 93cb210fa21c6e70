/*
 * byo_selector.h -- learned edgeMap-variant selector (not part of the paper).
 *
 * The paper's API study (Section 6.3, Table api-components-avg) shows that
 * which map variants are available changes running time but never results.
 * This selector exploits that freedom: a small MLP predicts, per level, the
 * log2 time of every edgeMap variant (byo_variant) from a 12-value feature
 * vector, and the level runs the variant with the smallest prediction. The
 * threshold heuristic (dense iff |U| + sum(deg(U)) > m / 20) is the fallback
 * whenever no valid weights are loaded or a prediction is not finite.
 *
 * Network: F = 12 inputs -> 32 ReLU -> 32 ReLU -> K = 6 outputs, FP32.
 * Parameters are one packed float array, row-major [fan_in][fan_out]:
 *   W1[F*H] b1[H] W2[H*H] b2[H] W3[H*K] b3[K]   (BYO_MLP_PARAMS floats).
 * Training loss: masked mean squared error sum(M*(out-Y)^2) / max(sum(M), 1);
 * optimiser: Adam (Kingma and Ba 2015) with bias correction.
 * All d_ buffers are device FP32 arrays owned by the caller.
 */
#ifndef BYO_SELECTOR_H_
#define BYO_SELECTOR_H_

#include <stdint.h>

#include "byo.h"
#include "byo_trace.h"

#ifdef __cplusplus
extern "C" {
#endif

#define BYO_MLP_F 12
#define BYO_MLP_H 32
#define BYO_MLP_K 6
#define BYO_MLP_PARAMS (BYO_MLP_F * BYO_MLP_H + BYO_MLP_H + BYO_MLP_H * BYO_MLP_H + BYO_MLP_H + \
                        BYO_MLP_H * BYO_MLP_K + BYO_MLP_K)

/* Raw (unnormalised) features of a level, host-side and pure (CPU-callable):
 *   [0] log2(1+k)   [1] log2(1+sum deg(U))   [2] log2(1+unvisited)   [3] log2(1+n)
 *   [4] log2(1+m)   [5] (k + sum deg(U))/(m+1)   [6] k/(n+1)   [7] log2(1+max degree)
 *   [8] degree coefficient of variation   [9] log2(1 + sum deg(U)/(k+1))
 *   [10] unvisited/(n+1)   [11] 1 if the frontier is held only as a bitmap, else 0
 * The device inference computes the same values from its level counters. */
byo_status byo_selector_features(const byo_level_record *rec, float *out);

/* The threshold rule the selector falls back to (pure host function).
 * Dense (pull) when |U| + sum deg(U) > m / dense_divisor (the sparse/dense
 * cutoff that Section 6.3 takes from Ligra and GBBS); otherwise a push whose
 * load-balancing scheme is set by the frontier's lists: with max_deg_u, the
 * largest degree in U, known (>= 0), edge-balanced when a list is longer than
 * 512 or sum deg(U) >= 65536, one lane per list when every list is at most 8
 * long, else a wavefront per list; with max_deg_u = -1, edge-balanced when the
 * graph's largest degree max_deg >= t_block or sum deg(U) >= 65536, else by
 * the average list length against t_wave. The pull scheme uses max_deg and cv. */
int32_t byo_heuristic_choice(int64_t k, int64_t degsum, int64_t m, int64_t max_deg, double cv, const byo_opts *opts,
                             int32_t allow_pull, int64_t max_deg_u);

/* out[N][K] = MLP(X[N][F]) (no normalisation applied; X is already normalised). */
byo_status byo_mlp_forward(const float *d_params, const float *d_X, int32_t N, float *d_out, void *stream);
/* grad[BYO_MLP_PARAMS] = d loss / d params; *d_loss = loss. Y, M are [N][K]. */
byo_status byo_mlp_loss_grad(const float *d_params, const float *d_X, const float *d_Y, const float *d_M, int32_t N,
                             float *d_grad, float *d_loss, void *stream);
/* One Adam step at step index t (1-based), in place on params, m, v. */
byo_status byo_mlp_adam(float *d_params, const float *d_grad, float *d_m, float *d_v, int32_t t, float lr,
                        float beta1, float beta2, float eps, void *stream);
/* `steps` full-batch Adam steps from the given params (moments start at zero);
 * d_losses[steps] receives the loss before each step (nullable). */
byo_status byo_mlp_train(float *d_params, const float *d_X, const float *d_Y, const float *d_M, int32_t N,
                         int32_t steps, float lr, float *d_losses, void *stream);

/* Install selector weights (host arrays: params, per-feature mean and standard
 * deviation used to normalise). BYO_EINVAL (and nothing installed) if any value
 * is not finite or a deviation is <= 0. */
byo_status byo_selector_set(const float *h_params, const float *h_mu, const float *h_sd);
byo_status byo_selector_clear(void);
byo_status byo_selector_loaded(int32_t *out);
/* Predict with the installed weights on the device: raw features in,
 * per-variant predictions out (nullable) and the chosen variant (pull variants
 * excluded unless allow_pull; -1 if a prediction is not finite). BYO_ESTATE if
 * no weights are installed. Syncs. Traversals with BYO_SEL_MLP make the same
 * float computation on the host, from the level counters they read back. */
byo_status byo_selector_predict(const float *h_features, int32_t allow_pull, float *h_pred, int32_t *variant);

/* Timing collection for training: run BFS from src (algo BYO_ALGO_BFS) or
 * connectivity (BYO_ALGO_CC), and at every level time each of the
 * BYO_NUM_VARIANTS variants from the same saved state (best of `repeats`),
 * then continue with the fastest. One record per (level, variant) goes to the
 * trace buffer (byo_trace_read), with the trial's time in `ms`. Results of the
 * run are left in d_out (depth for BFS, labels for CC). */
byo_status byo_selector_collect(byo_graph *g, int32_t algo, int64_t src, int32_t repeats, int32_t *d_out,
                                const byo_opts *opts, void *stream);

#ifdef __cplusplus
}
#endif
#endif /* BYO_SELECTOR_H_ */
