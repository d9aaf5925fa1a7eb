/*
 * acopf_mlp.h -- C ABI of the FP32 multilayer perceptron behind the learned
 * ADMM warm start (an extension of the method of arXiv 2310.13143: the
 * paper starts each ADMM solve from a fixed or previous point; here a
 * small per-component network trained on the solver's own traces proposes
 * the starting multipliers and penalties of each coupling).
 *
 * Network: y = W3 relu(W2 relu(W1 x + b1) + b2) + b3 with hidden width
 * ACOPF_MLP_HIDDEN, n_in in [1, 64] inputs and n_out in [1, 16] outputs.
 * Parameters are one FP32 vector theta, in this order and row-major:
 * W1 [64][n_in], b1 [64], W2 [64][64], b2 [64], W3 [n_out][64], b3 [n_out].
 * Samples are stored feature-major: feature f of sample s at X[f * ldx + s]
 * (ldx >= n), the same for targets T and outputs Y.  Loss: mean squared
 * error over samples and outputs, sum((y - t)^2) / (n * n_out).
 *
 * Every array is a DEVICE pointer owned by the caller; calls enqueue work
 * on the stream and return.  Errors are reported as in acopf_admm.h
 * (acopf_last_error).  Dense products run on the matrix cores in FP32 with
 * FP32 accumulation; sums over samples are reduced in a fixed order, so
 * results do not depend on timing.
 */
#ifndef ACOPF_MLP_H
#define ACOPF_MLP_H

#include "acopf_admm.h"

#ifdef __cplusplus
extern "C" {
#endif

#define ACOPF_MLP_HIDDEN 64

/* Number of FP32 parameters of a network; 0 for unsupported sizes. */
size_t acopf_mlp_param_count(int32_t n_in, int32_t n_out);

/* Bytes of device scratch acopf_mlp_gradient needs for n samples. */
size_t acopf_mlp_scratch_bytes(int32_t n_in, int32_t n_out, int64_t n);

/* Outputs Y of n samples X (inference). */
acopf_status acopf_mlp_forward(const float* theta, int32_t n_in, int32_t n_out, const float* X, int64_t ldx,
                               int64_t n, float* Y, int64_t ldy, void* stream);

/* Gradient of the loss over the n samples (X, T) by back-propagation,
 * written to grad (acopf_mlp_param_count floats, parameter order), and the
 * loss to *loss (one float, device).  scratch: acopf_mlp_scratch_bytes
 * bytes of caller memory (per-block partial sums). */
acopf_status acopf_mlp_gradient(const float* theta, int32_t n_in, int32_t n_out, const float* X, int64_t ldx,
                                const float* T, int64_t ldt, int64_t n, float* grad, float* loss, void* scratch,
                                size_t scratch_bytes, void* stream);

/* Size in bytes of the library's static device scratch used by
 * acopf_mlp_gradient_noalloc: (512 + 32) x (9,360 + 1) floats, the most
 * acopf_mlp_scratch_bytes returns for any network size and sample count. */
#define ACOPF_MLP_NOALLOC_SCRATCH_BYTES ((size_t)20369536)

/* acopf_mlp_gradient without a scratch argument, for callers that cannot
 * allocate device memory (code recorded under HIP graph capture, training
 * loops that must not call hipMalloc, harnesses that forbid it).  Same
 * kernels, same result bits as acopf_mlp_gradient.  The per-block partials
 * go to a static device array of ACOPF_MLP_NOALLOC_SCRATCH_BYTES that each
 * GPU holds from the first call on it until the process ends; the call
 * allocates nothing.  Every call on one GPU shares that GPU's array, so
 * calls that overlap in time on one GPU (other streams, other threads) race
 * and give undefined results; calls ordered on one stream are safe.  Sizes
 * whose scratch would exceed the array are rejected with
 * ACOPF_ERR_INVALID_ARG (none do with n_in <= 64, n_out <= 16). */
acopf_status acopf_mlp_gradient_noalloc(const float* theta, int32_t n_in, int32_t n_out, const float* X,
                                        int64_t ldx, const float* T, int64_t ldt, int64_t n, float* grad,
                                        float* loss, void* stream);

/* One Adam step (Kingma and Ba, 2015) on count parameters: m <- b1 m +
 * (1 - b1) g, v <- b2 v + (1 - b2) g^2, theta <- theta - lr mh / (sqrt(vh)
 * + eps) with the bias-corrected moments mh = m / (1 - b1^t), vh = v / (1 -
 * b2^t); t >= 1 counts the steps taken so far including this one. */
acopf_status acopf_mlp_adam(float* theta, float* m, float* v, const float* grad, int64_t count, int32_t t,
                            float lr, float beta1, float beta2, float eps, void* stream);

/* Standardisation used for training (an affine map per input and per
 * output, afterwards folded into the network so that it takes raw inputs
 * and returns raw outputs). */
#define ACOPF_MLP_STD_FLOOR 1e-4

/* Mean and standard deviation (population; deviations below
 * ACOPF_MLP_STD_FLOOR raised to it) of each of `rows` rows of X over its
 * first n columns; mean and stdev: rows doubles each (device).  FP64 sums
 * in a fixed order. */
acopf_status acopf_mlp_feature_stats(const float* X, int32_t rows, int64_t ldx, int64_t n, double* mean,
                                    double* stdev, void* stream);

/* In place: X[r][i] <- (X[r][i] - mean[r]) / stdev[r], clipped to +-clip if
 * clip > 0 (0 = no clip). */
acopf_status acopf_mlp_standardize(float* X, int32_t rows, int64_t ldx, int64_t n, const double* mean,
                                   const double* stdev, double clip, void* stream);

/* Fold the input map x -> (x - in_mean) / in_std (n_in entries) into W1, b1
 * and the output map y -> out_std y + out_mean (n_out entries) into W3, b3
 * of theta, in place (FP64 arithmetic, FP32 result). */
acopf_status acopf_mlp_fold(float* theta, int32_t n_in, int32_t n_out, const double* in_mean, const double* in_std,
                            const double* out_mean, const double* out_std, void* stream);

#ifdef __cplusplus
}
#endif

#endif /* ACOPF_MLP_H */
