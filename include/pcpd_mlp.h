/*
 * pcpd_mlp.h -- C ABI of the density surrogate in libpcpd: a perceptron
 * (log10 of the particle density as a function of p, d and t) trained on the
 * GPU by hand-written HIP kernels (bfloat16 MFMA products, float32
 * accumulation), used to propose where to run the simulation when searching
 * for the critical annihilation rate p_c of paper Sec. 2 (active phase for
 * p < p_c, inactive for p > p_c; p_c depends on d).
 *
 * Network: three inputs per row; the p_c search feeds ((p - 0.16) / 0.07, d,
 * log10(t) / 6), which puts one cell of its p grid above the bfloat16
 * resolution of the first products. Layers 3 -> 128 -> 128 -> 128 -> 1 with
 * tanh-form GELU after each hidden layer; output log10(rho).
 * Parameters: one float32 vector of PCPD_MLP_PARAMS values, in the order
 *   W1[128][3], b1[128], W2[128][128], b2[128], W3[128][128], b3[128],
 *   w4[128], b4[1]          (weights output-major, W[o][i]).
 * Arithmetic: both operands of every matrix product are rounded to bfloat16
 * (nearest, ties to even) and accumulated in float32; biases, activations,
 * loss and gradients are float32. Loss: mean squared error over rows whose
 * mask is nonzero. Optimiser: Adam (beta1 0.9, beta2 0.999, eps 1e-8) on a
 * float32 master copy.
 *
 * Conventions as in pcpd.h: status returns, no exceptions; x, y, target and
 * mask pointers are DEVICE pointers (float32, row-major [N][3] for x, [N]
 * for the others) borrowed for the call; host parameter/gradient buffers are
 * borrowed for the call. Work is enqueued on the given stream; calls that
 * return values to the host synchronise.
 */
#ifndef PCPD_MLP_H
#define PCPD_MLP_H

#include <stddef.h>
#include <stdint.h>

#include "pcpd.h"

#ifdef __cplusplus
extern "C" {
#endif

#define PCPD_MLP_PARAMS 33665
/* Rows of one predict / loss call, and of one gradient / training call. A
 * gradient call keeps the pre-activations of every row on the device
 * (1.5 KiB per row: 1.6 GB at the limit) plus at most 512 gradient partials
 * (69 MB) whatever N; predict and loss keep 8 bytes per 64 rows. */
#define PCPD_MLP_MAX_ROWS (1u << 24)
#define PCPD_MLP_MAX_TRAIN_ROWS (1u << 20)

typedef struct pcpd_mlp pcpd_mlp;

/* Create a network with uniform(-1/sqrt(fan_in), 1/sqrt(fan_in)) parameters
 * drawn from Philox-4x32-10 keyed by `seed`. dev->hip_stream selects the
 * stream (NULL = null stream); dev->dev_buf is unused. */
PCPD_API int pcpd_mlp_init(pcpd_mlp **out, uint32_t seed, const pcpd_device *dev);

/* Copy the float32 master parameters to / from the host. Setting resets the
 * Adam moments and step count. */
PCPD_API int pcpd_mlp_get_params(pcpd_mlp *net, float *host_params);
PCPD_API int pcpd_mlp_set_params(pcpd_mlp *net, const float *host_params);

/* y_dev[r] = network(x_dev[r]) for r < N (N <= PCPD_MLP_MAX_ROWS). Asynchronous. */
PCPD_API int pcpd_mlp_predict(pcpd_mlp *net, const float *x_dev, uint32_t N, float *y_dev);

/* Masked mean squared error of the network on N rows (N <= PCPD_MLP_MAX_ROWS),
 * forward pass only; the outputs go to y_dev[N]. mask_dev may be NULL (all
 * rows). Synchronises. */
PCPD_API int pcpd_mlp_loss(pcpd_mlp *net, const float *x_dev, const float *target_dev,
                           const float *mask_dev, uint32_t N, float *y_dev, float *loss_out);

/* Loss and gradient (host, PCPD_MLP_PARAMS floats) of the masked mean squared
 * error at the current parameters (N <= PCPD_MLP_MAX_TRAIN_ROWS); mask_dev may
 * be NULL (all rows). Synchronises. */
PCPD_API int pcpd_mlp_grads(pcpd_mlp *net, const float *x_dev, const float *target_dev,
                            const float *mask_dev, uint32_t N, float *host_grads,
                            float *loss_out);

/* One Adam step on the masked mean squared error of this batch
 * (N <= PCPD_MLP_MAX_TRAIN_ROWS). If loss_out is
 * not NULL the loss before the step is returned (this synchronises). */
PCPD_API int pcpd_mlp_train_step(pcpd_mlp *net, const float *x_dev, const float *target_dev,
                                 const float *mask_dev, uint32_t N, float lr, float *loss_out);

PCPD_API int pcpd_mlp_free(pcpd_mlp *net);

#ifdef __cplusplus
}
#endif

#endif /* PCPD_MLP_H */
