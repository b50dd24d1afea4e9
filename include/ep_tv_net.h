/*
 * ep_tv_net.h -- C ABI of the learned warm start for EP-TV (gfx950).
 *
 * A 6-layer 3x3 convolutional network, channels 1 -> 32 -> 32 -> 32 -> 32 -> 32
 * -> 2, ReLU after layers 1..5, zero padding, maps the normalised observation
 * x0 = (y - m) / s of an image (m = mean of y, s = population standard
 * deviation, floored at 1e-6) to o = (o0, o1); the prediction is
 *   mu_hat = m + s * o0,   var_hat = xi * exp(o1)     (xi = noise variance).
 * Trained on pairs (y, converged EP marginals) that the EP solver itself
 * produces, it only initialises the EP sites (ep_tv_init_warm in ep_tv.h); EP
 * then runs to convergence.  Loss for training: the mean over pixels of
 *   (o0 - (mu - m)/s)^2 + (o1 - log(v / xi))^2.
 * Optimiser: Adam (Kingma & Ba, 2015) with beta1 = 0.9, beta2 = 0.999,
 * eps = 1e-8 and bias correction.
 *
 * Parameters: one float32 vector of ep_tv_net_param_count() = 37,890 numbers,
 * owned by the caller (device memory), in the canonical order
 *   W1[3][3][1][32], b1[32], (W_l[3][3][32][32], b_l[32]) for l = 2..5,
 *   W6[3][3][32][2], b6[2]
 * (tap row a, tap column b, input channel, output channel); tap (a, b)
 * multiplies the input pixel (r + a - 1, c + b - 1).
 * Precision: weights, activations and activation gradients are stored as
 * bfloat16 (round to nearest even), sums accumulate in float32 (32 -> 32
 * layers on the matrix cores), weight-gradient partials are summed in float64;
 * master weights and Adam moments are float32.
 *
 * Images are batches of equal-size row-major float32 images (batch x h x w,
 * device pointers).  Status codes are the EP_TV_* codes of ep_tv.h.  All calls
 * enqueue on the stream given at creation and are asynchronous unless a host
 * output is requested.  A network object is not thread-safe.
 */
#ifndef EP_TV_NET_H
#define EP_TV_NET_H

#include <stddef.h>
#include <stdint.h>

#include "ep_tv.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct ep_tv_net ep_tv_net;

/* Number of float32 parameters (37890). */
int ep_tv_net_param_count(void);

/* Device workspace bytes for calls with batch <= max_batch, h <= max_h,
 * w <= max_w (activations of every layer for the backward pass, gradient
 * buffers, per-block partial sums, bfloat16 weight copies, Adam moments). */
int ep_tv_net_workspace_bytes(int32_t max_batch, int32_t max_h, int32_t max_w, size_t* bytes);

/* Create a network over caller-owned parameters d_params (device, float32,
 * param_count values, read by every call and updated in place by Adam steps)
 * and a caller-owned workspace (device, 256-byte aligned, at least
 * ep_tv_net_workspace_bytes bytes, used exclusively until destroy).
 * Derives the bfloat16 weight copies and zeroes the Adam state. */
int ep_tv_net_create(float* d_params, void* d_workspace, size_t ws_bytes, int32_t max_batch,
                     int32_t max_h, int32_t max_w, void* hip_stream, ep_tv_net** out);

/* After the caller has written new values into d_params: re-derive the
 * bfloat16 copies and zero the Adam state.  Asynchronous. */
int ep_tv_net_sync(ep_tv_net* net);

/* Predict (mu_hat, var_hat) for a batch of images.  d_y: batch*h*w floats;
 * d_mu_hat, d_var_hat: batch*h*w floats written.  noise_var = xi > 0.
 * Asynchronous. */
int ep_tv_net_infer(ep_tv_net* net, const float* d_y, int32_t batch, int32_t h, int32_t w,
                    double noise_var, float* d_mu_hat, float* d_var_hat);

/* Loss and its gradient with respect to the parameters for a batch with
 * targets (d_mu_t, d_var_t: batch*h*w floats, var > 0).  The gradient is kept
 * for ep_tv_net_adam_step and, if d_grad is not NULL, also copied there
 * (device, param_count floats, canonical order).  loss_out: host double or NULL
 * (non-NULL synchronises the stream). */
int ep_tv_net_loss_grad(ep_tv_net* net, const float* d_y, const float* d_mu_t, const float* d_var_t,
                        int32_t batch, int32_t h, int32_t w, double noise_var, float* d_grad,
                        double* loss_out);

/* One Adam step with the last computed gradient and learning rate lr > 0;
 * updates d_params in place and the bfloat16 copies.  Asynchronous. */
int ep_tv_net_adam_step(ep_tv_net* net, float lr);

/* ep_tv_net_loss_grad followed by ep_tv_net_adam_step. */
int ep_tv_net_train_step(ep_tv_net* net, const float* d_y, const float* d_mu_t, const float* d_var_t,
                         int32_t batch, int32_t h, int32_t w, double noise_var, float lr,
                         double* loss_out);

/* Adam steps taken since creation or the last sync (-1 for NULL). */
int ep_tv_net_adam_count(const ep_tv_net* net);

const char* ep_tv_net_last_error(const ep_tv_net* net);

/* Frees only what the library allocated (nothing the caller passed). */
void ep_tv_net_destroy(ep_tv_net* net);

#ifdef __cplusplus
}
#endif

#endif /* EP_TV_NET_H */
