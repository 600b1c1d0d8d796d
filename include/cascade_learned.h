/* Learned setup for cascading smoothers on MI355X (gfx950).
 *
 * The Frobenius setup (Sec. 2.1, Alg. 2) costs O(k_l n^3) per block and level
 * and dominates construction on fine levels (Sec. 2.5).  This interface
 * replaces it on the finest level by a multilayer perceptron that maps local
 * features of the coefficient field around a block to the block's prescaled
 * cascade blocks Lambda~_1..Lambda~_nu; the library unscales them as in
 * Sec. 2.3 (Lambda = W Lambda~ W) and keeps the Frobenius fit on the coarser
 * levels.  The paper contains no learned component: this is the extension its
 * setup-cost discussion motivates, and measured convergence factors (Sec. 3.1)
 * decide whether the learned blocks are used.
 *
 * Network: y = W3 silu(W2 silu(W1 x + b1) + b2) + b3, silu(z) = z/(1+e^-z),
 * FP32, weights (out, in) row-major.  Parameters are one FP32 vector in the
 * order W1, b1, W2, b2, W3, b3.  Training minimises the mean squared error
 * against targets standardised per output with the network's output scaling
 * (mean, std); cs_mlp_forward returns y * std + mean.
 *
 * Pointers named *_dev are device pointers; the others are host pointers.
 * All calls return CS_EINVAL for bad sizes or null pointers and CS_EDEVICE
 * for HIP failures, with the message in cs_mlp_last_error.
 */
#ifndef CASCADE_LEARNED_H
#define CASCADE_LEARNED_H

#include "cascade.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct cs_mlp_s *cs_mlp;

/* Network n_in -> width -> width -> n_out on HIP device `device`, issuing work
 * on `stream` (hipStream_t or NULL).  Parameters start at zero; the output
 * scaling at mean 0, std 1. */
cs_status cs_mlp_create(cs_mlp *out, int32_t device, void *stream, int32_t n_in, int32_t width, int32_t n_out);
void cs_mlp_destroy(cs_mlp m);
const char *cs_mlp_last_error(cs_mlp m);
cs_status cs_mlp_param_count(cs_mlp m, int64_t *count);
/* Replace the parameters (host FP32 [count]); clears the Adam moments and step. */
cs_status cs_mlp_set_params(cs_mlp m, const float *params);
cs_status cs_mlp_get_params(cs_mlp m, float *params);
/* Output scaling, host FP32 [n_out] each; std entries must be > 0. */
cs_status cs_mlp_set_scaling(cs_mlp m, const float *mean, const float *std);
cs_status cs_mlp_get_scaling(cs_mlp m, float *mean, float *std);
/* Set the output scaling to the per-output mean and population standard
 * deviation (zero deviations become 1) of the target rows rows_dev[0..n) of
 * T_dev [*][n_out] (rows_dev NULL: rows 0..n-1). */
cs_status cs_mlp_fit_scaling(cs_mlp m, const float *T_dev, const int32_t *rows_dev, int64_t n);

/* Loss and gradient (host FP32 [count]) of the MSE over the rows
 * rows_dev[0..n) of X_dev [*][n_in] and T_dev [*][n_out] (rows_dev NULL: rows
 * 0..n-1).  No parameter changes. */
cs_status cs_mlp_gradient(cs_mlp m, const float *X_dev, const float *T_dev, const int32_t *rows_dev, int64_t n,
                          float *grad, double *loss);
/* Mean squared error over the given rows (evaluation; no gradient). */
cs_status cs_mlp_loss(cs_mlp m, const float *X_dev, const float *T_dev, const int32_t *rows_dev, int64_t n,
                      double *loss);
/* Adam training (beta1 0.9, beta2 0.999, eps 1e-8) with a cosine learning
 * rate from lr0 to lr_min over all steps.  order_dev [epochs][n_train] lists,
 * per epoch, the rows of X_dev/T_dev in the order they are visited (the
 * caller draws the shuffles); each epoch takes ceil(n_train/batch) steps, the
 * last one shorter.  epoch_loss (host, may be NULL) receives each epoch's
 * mean batch loss. */
cs_status cs_mlp_train(cs_mlp m, const float *X_dev, const float *T_dev, const int32_t *order_dev, int64_t n_train,
                       int32_t epochs, int32_t batch, double lr0, double lr_min, double *epoch_loss);
/* Y_dev [n][n_out] = prediction in target units for the rows of X_dev [n][n_in]. */
cs_status cs_mlp_forward(cs_mlp m, const float *X_dev, int64_t n, float *Y_dev);

/* Features of the 2x2x2 node blocks of a trilinear (Q1) hexahedral mesh with
 * n^3 hexes (n even), blocks (I, J, K) lexicographic with x fastest:
 * log10mu_dev [n][n][n] (index [k][j][i]) -> X_dev [(n/2)^3][1464]:
 *   [0, 729)     (log10 mu - m) / 3 over the 9^3 hexes (2I-4+u, 2J-4+v, 2K-4+w),
 *                u + 9v + 81w, m the mean over the patch hexes inside the
 *                mesh; 0 outside;
 *   [729, 1458)  1 for patch hexes inside the mesh, 0 outside;
 *   [1458, 1464) min(d, 4)/4 for the block distances d to the faces
 *                x=0, x=1, y=0, y=1, z=0, z=1.
 * The 9^3 patch is the region the second cascade level of a 2x2x2 node block
 * depends on for a 27-point stencil (two applications of A around the block). */
cs_status cs_fe_block_features(void *stream, const double *log10mu_dev, int32_t n, float *X_dev);

/* Prescaled smoother blocks of a level after cs_setup:
 * out_dev [n_blocks][depth][nb][nb] FP32 with Lambda~ = W^-1 Lambda W^-1
 * (W = diag(a_kk^-1/2), Sec. 2.3) - the training targets of the network. */
cs_status cs_get_prescaled_blocks(cs_ctx ctx, int32_t level, float *out_dev);

/* Setup with the network on the finest level: its prediction for X_dev
 * [n_blocks][n_in] is read as Lambda~ [n_blocks][depth][nb][nb] (n_out must
 * equal depth*nb*nb), unscaled with W and used as the level-0 cascade; every
 * coarser level gets the Frobenius fit of cs_setup.  Replaces any previous
 * setup; cs_info.setup_ms then times this call (features excluded). */
cs_status cs_setup_learned(cs_ctx ctx, const cs_options *opt, cs_mlp m, const float *X_dev);

#ifdef __cplusplus
}
#endif

#endif
