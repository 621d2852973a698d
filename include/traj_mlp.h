/*
 * traj_mlp.h -- learned warm start for the batched trajectory optimizer of
 * traj.h (MI355X, gfx950).
 *
 * Algorithm 1 of arXiv 2109.10392 may start from any iterate (Remark 4). The
 * warm start predicts, from 64 features of a scene, the iterate (c, lambda) of
 * the scene's 256 template goals (4 lanes x 64 longitudinal slots, lane-major):
 * per goal c_x, c_y, c_psi, lambda_x, lambda_y, lambda_psi, 11 values each, i.e.
 * 16,896 outputs. The network is a multilayer perceptron 64 -> 256 -> 256 ->
 * 256 -> 16,896 with ReLU on the hidden layers, BF16 weights, FP32 biases and
 * FP32 accumulation. It is trained by regression on the optimizer's own
 * solutions (standardised per output), forward and backward on the GPU.
 *
 * Conventions as in traj.h: return TRAJ_OK or a negative TRAJ_E_* code (message
 * in traj_last_error()); device pointers are caller-owned HIP device memory;
 * every call only enqueues kernels on `stream` (no allocation, no host
 * synchronisation). BF16 values are stored as uint16_t bit patterns.
 *
 * Rounding points (the definition the kernels follow): each layer input is
 * rounded to BF16 (nearest, ties to even); the products sum BF16 x BF16 terms
 * in FP32; the bias is added in FP32; ReLU; the output layer stays FP32. In the
 * backward pass dy and every hidden-layer gradient are rounded to BF16 before
 * their products; the ReLU derivative is (stored activation > 0).
 */
#ifndef TRAJ_MLP_H
#define TRAJ_MLP_H

#include <stdint.h>

#include "traj.h"

#ifdef __cplusplus
extern "C" {
#endif

#define TRAJ_N_FEAT 64 /* features per scene */

typedef struct {
  int32_t n_in;     /* features, multiple of 8 (64) */
  int32_t n_hidden; /* width of the hidden layers, multiple of 8 (256) */
  int32_t n_layers; /* hidden layers, 1..8 (3) */
  int32_t n_out;    /* outputs, multiple of 8 (16,896 = 256 goals x 66) */
} traj_mlp_dims;

/* Parameters, packed in one array (the same offsets for the FP32 master copy, the
 * BF16 copy, the gradient and the two Adam moments): for each layer l = 1 .. n_layers
 * + 1, W_l [fan_in][fan_out] row-major, then b_l [fan_out]. */
typedef struct {
  traj_mlp_dims dims;
  float *params;          /* device, FP32 master parameters */
  uint16_t *params_bf16;  /* device, BF16 copy (the weight blocks are what the products read) */
  float *grad;            /* device, gradient (backward writes it; may be NULL for inference) */
  float *adam_m, *adam_v; /* device, Adam moments (training only; may be NULL otherwise) */
} traj_mlp;

/* traj_mlp_param_count -- number of packed parameters (host-only).
 * Errors: TRAJ_E_INVAL (NULL, sizes not multiples of 8, n_layers outside 1..8). */
int traj_mlp_param_count(const traj_mlp_dims *dims, int64_t *count);

/* traj_mlp_sync_bf16 -- params_bf16 = bf16(params) (after loading master weights). */
int traj_mlp_sync_bf16(const traj_mlp *net, void *stream);

/*
 * traj_features -- 64 features of every scene of a batch (a scene's obstacles
 * and ego state at t = 0): f[0] = v0 / 30 m/s; then for the 10 obstacles nearest
 * to the ego (squared distance in FP32, computed without fused multiply-add; ties
 * by index) in increasing distance: (x - x0, y - y0) / 100 m and (vx - vx0,
 * vy - vy0) / 30 m/s; the rest zero.
 *   feat: device [n_scenes][64]. Scenes with more than 64 obstacles: TRAJ_E_INVAL
 *   is not detected on the host; such scenes get NaN features.
 */
int traj_features(const traj_batch *batch, float *feat, void *stream);

/*
 * traj_mlp_forward -- y = network(x) for `batch` rows.
 *   x: device [batch][n_in] FP32. acts: device BF16, batch * (n_in + n_layers * n_hidden)
 *   entries: the rounded input of every layer one after another, a0 [batch][n_in],
 *   then a1 .. a_L [batch][n_hidden] (kept for the backward pass).
 *   y: device [batch][n_out] FP32.
 */
int traj_mlp_forward(const traj_mlp *net, const float *x, int batch, uint16_t *acts, float *y, void *stream);

/*
 * traj_mlp_loss -- mean squared error of y against the standardised targets
 * (target - mean) / stdv over all batch x n_out entries, and its gradient.
 *   dy: device BF16 [batch][n_out], bf16(2 (y - t) / (batch n_out)).
 *   row_loss: device [batch] scratch; loss: device [1], the mean.
 */
int traj_mlp_loss(const traj_mlp_dims *dims, const float *y, const float *target, const float *mean,
                  const float *stdv, int batch, uint16_t *dy, float *row_loss, float *loss, void *stream);

/*
 * traj_mlp_backward -- gradient of the loss with respect to every parameter into
 * net->grad, from the stored activations and dy (both as written above).
 *   work: device BF16 scratch of 2 * batch * n_hidden entries.
 */
int traj_mlp_backward(const traj_mlp *net, const uint16_t *acts, const uint16_t *dy, int batch, uint16_t *work,
                      void *stream);

/*
 * traj_mlp_adam -- one Adam step (Kingma and Ba 2015, bias-corrected, step >= 1)
 * on every parameter from net->grad; refreshes params_bf16.
 */
int traj_mlp_adam(const traj_mlp *net, int step, float lr, float beta1, float beta2, float eps, void *stream);

/*
 * traj_colstats -- per-column mean and standard deviation (population, FP64
 * sums) of rows [n_rows][n_cols]; a column whose deviation is below
 * 1e-5 max(1, |mean|) gets stdv = 1 (constant outputs such as x(0) = 0).
 */
int traj_colstats(const float *rows, int n_rows, int n_cols, float *mean, float *stdv, void *stream);

/*
 * traj_state_rows -- gather the iterate of every scene into one row per scene:
 * rows[s][66 * i + 11 q + k] = (q < 3 ? c : lam)[q mod 3][k][goal_off[s] + i] for the
 * scene's goals i < goals_per_scene. A scene with another goal count gets NaN.
 *   rows: device [n_scenes][66 * goals_per_scene].
 */
int traj_state_rows(const traj_batch *batch, const traj_state *state, int goals_per_scene, float *rows,
                    void *stream);

/*
 * traj_rows_state -- the inverse, de-standardising: value = y * stdv + mean, written
 * into state c and lam of the scene's goals (scenes with another goal count are
 * left unchanged).
 */
int traj_rows_state(const traj_batch *batch, traj_state *state, int goals_per_scene, const float *y,
                    const float *mean, const float *stdv, void *stream);

/*
 * traj_gemm_bf16 -- the product the network runs on, exposed for verification:
 * C[M][N] = op(A) op(B) (+ bias[N], ReLU if relu), A and B BF16, FP32 sums on the
 * matrix cores. ta: A stored [K][M] (else [M][K]); tb: B stored [N][K] (else
 * [K][N]); row-major, M, N, K multiples of 8. C: device FP32 [M][N]; bias may be NULL.
 */
int traj_gemm_bf16(int ta, int tb, int M, int N, int K, const uint16_t *A, const uint16_t *B, const float *bias,
                   int relu, float *C, void *stream);

#ifdef __cplusplus
}
#endif

#endif /* TRAJ_MLP_H */
