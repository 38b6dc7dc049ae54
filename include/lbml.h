/*
 * lbml — the warm-start network of lbnlm: a fully connected network with SiLU
 * hidden layers whose GEMMs run on the gfx950 matrix cores (BF16 operands,
 * FP32 accumulation), trained with Adam on FP32 master weights.
 *
 * It predicts steady channel profiles of the nlM fluid from the channel
 * parameters so that lb_set_profile can start a run close to its steady
 * state; the lattice-Boltzmann solver stays the judge of the result. The
 * paper itself has no such network: this is an added component.
 *
 * C ABI: plain pointers and sizes; device pointers are marked dev_. Every
 * call returns an lbml_status (0 = OK) and leaves a message for
 * lbml_last_error() on failure. A handle is bound to one HIP stream and is
 * not thread safe.
 *
 * Parameter layout (FP32, flat): for each layer l = 0..n_layers-1 with
 * in = dims[l], out = dims[l+1]: the weight matrix W_l[out][in] (row major),
 * then the bias b_l[out]. Gradients and the Adam moments use the same layout.
 * Layer l computes z = x W_l^T + b_l, followed by SiLU(z) = z / (1 + e^-z) on
 * every layer except the last.
 */
#ifndef LBNLM_LBML_H
#define LBNLM_LBML_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct lbml_net lbml_net;
typedef int32_t lbml_status; /* 0 ok, -1 invalid argument, -2 workspace too small, -3 HIP error, -5 state */

/* Bytes of device workspace for a network with n_layers layers of widths
 * dims[0..n_layers] and batches of at most max_batch rows. */
lbml_status lbml_workspace_bytes(int32_t n_layers, const int32_t *dims, int32_t max_batch, size_t *bytes);

/* Number of FP32 parameters (weights and biases of all layers). */
lbml_status lbml_param_count(int32_t n_layers, const int32_t *dims, size_t *count);

/* Creates a network in caller-owned device memory (aligned to 256 bytes,
 * kept alive until lbml_destroy). Parameters are zero until lbml_set_params;
 * the Adam moments start at zero. hip_stream: the stream every call of this
 * handle runs on; NULL is the default (null) stream. The caller orders its own
 * producers and consumers of dev_ buffers with that stream (passing the
 * stream those run on is the simple way). */
lbml_status lbml_create(int32_t n_layers, const int32_t *dims, int32_t max_batch, void *dev_workspace,
                        size_t ws_bytes, void *hip_stream, lbml_net **out);
lbml_status lbml_destroy(lbml_net *net);

/* Copies n FP32 parameters from/to host memory (n must equal the count);
 * setting them also refreshes the BF16 copies of the weights. Synchronous. */
lbml_status lbml_set_params(lbml_net *net, const float *host_params, size_t n);
lbml_status lbml_get_params(lbml_net *net, float *host_params, size_t n);

/* Forward pass of `batch` rows (1 <= batch <= max_batch): dev_x[batch][dims[0]]
 * FP32 in, dev_y[batch][dims[n_layers]] FP32 out. The activations (and a BF16
 * copy of the input) are kept for lbml_backward. Asynchronous. */
lbml_status lbml_forward(lbml_net *net, const float *dev_x, int32_t batch, float *dev_y);

/* Mean-squared error of dev_y against dev_target (both [batch][dims[n_layers]],
 * mean over all entries) and its gradient d loss / d y into dev_dy. If
 * host_loss is not NULL the loss is returned there (synchronises). */
lbml_status lbml_mse(lbml_net *net, const float *dev_y, const float *dev_target, int32_t batch, float *dev_dy,
                     double *host_loss);

/* Backward pass for the last forward: gradients of the loss with respect to
 * all parameters (overwritten, not accumulated) from dev_dy. Asynchronous. */
lbml_status lbml_backward(lbml_net *net, const float *dev_dy, int32_t batch);

/* Copies the parameter gradients of the last backward pass to host memory. */
lbml_status lbml_get_grads(lbml_net *net, float *host_grads, size_t n);

/* One Adam update of the FP32 master parameters with the current gradients
 * (t = 1, 2, ... the update count, for bias correction), then refreshes the
 * BF16 weights. Asynchronous. */
lbml_status lbml_adam_step(lbml_net *net, float lr, float beta1, float beta2, float eps, int32_t t);
/* One training step on a minibatch gathered on the device: rows
 * dev_idx[0..batch) (int32, caller-owned; each in [0, n), not checked) of
 * the inputs dev_X[n][dims[0]] and the targets dev_Y[n][dims[n_layers]] (FP32,
 * caller-owned), then the forward pass, the mean-squared error, the backward
 * pass and one Adam update (t as in lbml_adam_step); the same arithmetic as
 * those calls on the gathered rows, in one call. If host_loss is not NULL
 * the batch loss before the update is returned there (synchronises);
 * asynchronous otherwise. The gradients remain readable with lbml_get_grads. */
lbml_status lbml_train_step(lbml_net *net, const float *dev_X, const float *dev_Y, const int32_t *dev_idx,
                            int32_t batch, float lr, float beta1, float beta2, float eps, int32_t t,
                            double *host_loss);

const char *lbml_last_error(const lbml_net *net);

#ifdef __cplusplus
}
#endif

#endif /* LBNLM_LBML_H */
