/*
 * lbm_nn.h -- the learned warm start: a small BF16 network and the kernels that turn
 * its output into an initial lattice state.
 *
 * A multilayer perceptron evaluated per grid point maps features of the problem (the
 * relaxation time and the Fourier modes of the acceleration field, see
 * lbm_ws_features) to the steady velocity and density there.  Matrix products run on
 * the gfx950 matrix cores in BF16 with FP32 accumulation (hand-written kernels);
 * master weights, gradients and the Adam moments are FP32.  Hidden layers use the
 * tanh form of GELU, the output layer is linear.  The lattice is then started from
 * the predicted fields (lbm_reset_fields: force-corrected equilibrium of (rho, u), the
 * same state lbm_init builds), and the converged lattice-Boltzmann solution remains the
 * judge of the prediction's error.  The plain start (rest, rho0) stays the fallback.
 *
 * Device arrays (float*, row-major, one row per point) are caller-owned device memory;
 * host arrays are copied during the call.  Work is enqueued on the stream given at
 * creation; calls returning host data synchronise it.  Status codes as in lbm.h.
 */
#ifndef LBM_NN_H
#define LBM_NN_H

#include <stddef.h>
#include <stdint.h>

#include "lbm.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct lbm_mlp lbm_mlp;

/* widths[0] inputs, widths[nlayers] outputs, nlayers >= 1, every width in 1..4096.
 * Parameters start at zero (set them with lbm_mlp_set_params).  max_rows bounds the
 * rows of every later forward / backward call (activations are kept for backward). */
int lbm_mlp_create(const int32_t *widths, int32_t nlayers, int64_t max_rows, void *hip_stream,
                   lbm_mlp **out);
int lbm_mlp_num_params(const lbm_mlp *m, int64_t *n);

/* Parameters in the order W_0 (widths[1] x widths[0], row-major), b_0, W_1, b_1, ...
 * (FP32 on the host).  set also refreshes the BF16 copies and clears Adam's moments. */
int lbm_mlp_set_params(lbm_mlp *m, const float *host, int64_t n);
int lbm_mlp_get_params(lbm_mlp *m, float *host, int64_t n);
int lbm_mlp_get_grads(lbm_mlp *m, float *host, int64_t n);

/* y (rows x outputs, FP32 device) = network(x (rows x inputs, FP32 device)); x is
 * rounded to BF16.  Keeps what backward needs. */
int lbm_mlp_forward(lbm_mlp *m, const float *x_dev, int64_t rows, float *y_dev);

/* Weighted mean-square loss of the last forward's output against target (rows x
 * outputs, device): L = sum_{r,c} w_c (y - t)^2 / (rows * outputs), w = channel_weight
 * (host, outputs entries, NULL = 1).  Accumulates dL/dparams into the gradients (call
 * lbm_mlp_zero_grads first) and returns L in *loss (may be NULL). */
int lbm_mlp_loss_backward(lbm_mlp *m, const float *target_dev, const float *channel_weight,
                          double *loss);

/* Accumulate the gradients of sum(dy * y) for a given dL/dy (rows x outputs, device)
 * of the last forward. */
int lbm_mlp_backward(lbm_mlp *m, const float *dy_dev);
int lbm_mlp_zero_grads(lbm_mlp *m);

/* One Adam step (t >= 1 is the step number for the bias corrections). */
int lbm_mlp_adam(lbm_mlp *m, double lr, double beta1, double beta2, double eps, int64_t t);
int lbm_mlp_free(lbm_mlp *m);

/* Fourier forcing g(x) = sum_j amp_j p_j sin(2 pi k_j . x / box + phase_j) on a periodic
 * box^3 lattice with viscosity nu = (tau2 - 1/2)/3. */
typedef struct {
  double tau2;
  int32_t nmodes;           /* 1..8 */
  double k[8][3];           /* integer wavevectors (as doubles) */
  double p[8][3];           /* unit polarisations, perpendicular to k */
  double amp[8];
  double phase[8];
} lbm_ws_problem;

#define LBM_WS_FEATURES 34  /* features per point (8 per mode for 4 modes + 2) */

/* Per-point network inputs on an n^3 grid spanning the box (point (i,j,l) sits at lattice
 * position (i, j, l) * box / n), rows in x-fastest order.  Needs nmodes == 4.  Also
 * returns the velocity scale U of the problem (outputs are velocity / U and
 * (rho - 1) / U^2).  Features per mode j, with K_j = 2 pi |k_j| / box and
 * s_j = amp_j / (nu K_j^2): p_j sin(theta_j) (3), p_j cos(theta_j) (3), s_j / U,
 * K_j; then tau2 - 1/2 and the Reynolds number U / (nu K_min). */
int lbm_ws_features(const lbm_ws_problem *p, int32_t n, int32_t box, float *x_dev,
                    double *U_out, void *hip_stream);

/* Periodic trilinear upsampling of nchan fields (channel-major planes, nc^3 each, x
 * fastest) to nf^3 (nf a multiple of nc): fine point x takes the coarse grid at x nc/nf. */
int lbm_upsample_periodic(const float *coarse_dev, int32_t nc, int32_t nchan, float *fine_dev,
                          int32_t nf, void *hip_stream);

/* Restart lattice c from device fields: rho (N floats) and u (D x N floats, component
 * planes), or from the network's point-major output (N x (D+1): u / U then
 * (rho - 1) / U^2, when point_major != 0, scaled by U).  The state becomes the
 * force-corrected equilibrium of those fields (as lbm_init), time 0. */
int lbm_reset_fields(lbm_ctx *c, const float *fields_dev, int32_t point_major, double U);

#ifdef __cplusplus
}
#endif
#endif /* LBM_NN_H */
