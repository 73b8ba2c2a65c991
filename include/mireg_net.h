/*
 * mireg_net -- learned warm start for the Gauss-Newton-Krylov registration
 * solver of mireg.h, on one MI355X (gfx950).
 *
 * The solver starts each solve from a velocity (Sec. 3.6 of the paper uses
 * v = 0, or the previous solution while it continues in beta_v).  This
 * library predicts that starting velocity from the image pair with a small
 * convolutional network and trains the network on pairs the solver itself
 * produces.  The network is not part of the paper.
 *
 * Network on the periodic n^3 grid (channels c0..c3 at n, n/2, n/4, n/8):
 *   x  = (mT, mR)
 *   e0 = relu(C x),  e_l = relu(C P e_{l-1})            l = 1, 2, 3
 *   d2 = relu(C U e3 + e2), d1 = relu(C U d2 + e1), d0 = relu(C U d1 + e0)
 *   v  = Leray(H d0 + G_sigma U8 H3 e3)
 * C: periodic 3x3x3 convolution with bias (BF16 operands on the matrix cores,
 * FP32 accumulation), P: 2x2x2 mean, U: nearest upsampling by 2 (U8 by 8),
 * H, H3: pointwise 1x1x1 maps (FP32), G_sigma: spectral Gaussian of width
 * sigma cells, Leray: the projection onto divergence-free fields.
 * Loss of a pair: |v - v_target|^2 / (2 * 3 n^3).
 *
 * Parameters: one FP32 vector; per layer (enc0, enc1, enc2, enc3, dec2,
 * dec1, dec0, head, head3) the weights W[Cout][T][Cin] (T = 27 taps, or 1
 * for the heads; tap t = 9 (d1+1) + 3 (d2+1) + (d3+1) reads x + (d1,d2,d3))
 * then the biases b[Cout].
 *
 * Conventions as in mireg.h: field pointers are DEVICE pointers to FP32
 * arrays owned by the caller (scalars [n1][n2][n3], vectors [3][n1][n2][n3]);
 * parameter and gradient vectors are HOST arrays; all work runs on the
 * stream given at creation and every call returns after its results are
 * complete.  Errors are negative MIREG_E_* codes (mireg.h) with a message
 * from mireg_net_last_error.
 */
#ifndef MIREG_NET_H
#define MIREG_NET_H

#include "mireg.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct mireg_net mireg_net;

typedef struct {
    int n;              /* grid points per axis: power of two, 16..256 */
    int channels[4];    /* c0..c3, each 16, 32, 64 or 128 */
    double skip_sigma;  /* width (cells of the n^3 grid) of the skip's Gaussian, >= 0 */
} mireg_net_config;

/* Allocates the network's device memory (activations of one pair, their
 * gradients, packed BF16 weights, Adam moments).  Parameters start at zero.
 * MIREG_E_SHAPE / MIREG_E_ARG for an unsupported configuration. */
int mireg_net_create(const mireg_net_config *cfg, void *stream, mireg_net **out);
int mireg_net_destroy(mireg_net *net);
const char *mireg_net_last_error(const mireg_net *net);
/* Number of FP32 parameters. */
long long mireg_net_param_count(const mireg_net *net);
/* Copy the parameters in (host FP32, param_count values) or out; setting
 * them also clears the Adam moments and the step count. */
int mireg_net_set_params(mireg_net *net, const float *params);
int mireg_net_get_params(const mireg_net *net, float *params);

/* Predicted velocity v (device [3][n^3]) for the pair mT, mR (device [n^3]). */
int mireg_net_forward(mireg_net *net, const float *mT, const float *mR, float *v);

/* Loss of one pair and its gradient with respect to every parameter (host,
 * param_count values; not accumulated).  grad may be NULL. */
int mireg_net_loss_grad(mireg_net *net, const float *mT, const float *mR, const float *v_target, double *loss,
                        float *grad);

/* One Adam step (beta1 0.9, beta2 0.999, eps 1e-8) on the mean gradient of
 * `batch` pairs: mT[i], mR[i] (device [n^3]) and v_target[i] (device
 * [3][n^3]) are arrays of `batch` device pointers held on the host.
 * *loss = mean loss of the pairs before the step. */
int mireg_net_train_step(mireg_net *net, int batch, const float *const *mT, const float *const *mR,
                         const float *const *v_target, double lr, double *loss);

/* Training-data helper: a periodic Voronoi phantom on the n^3 grid of
 * [0, 2 pi)^3.  seeds (host, 3 ns values, positions in [0, 2 pi)) and
 * values (host, ns values); out (device [n^3]) receives the value of the
 * nearest seed under the periodic distance (ties: the lower seed index). */
int mireg_net_voronoi(mireg_net *net, int ns, const float *seeds, const float *values, float *out);

#ifdef __cplusplus
}
#endif

#endif /* MIREG_NET_H */
