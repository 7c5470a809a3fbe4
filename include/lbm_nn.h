/*
 * lbm_nn.h -- the warm start of the steady forced lattice: the lattice's own steady state
 * expanded in the forcing amplitude, a small BF16 network that resums that expansion,
 * and the kernels that set the state.
 *
 * The start is the sum over orders n = 1..4 of the population waves W_n of the steady
 * state's expansion about rest (lbm_ws_lattice_waves_ordered), each order scaled by a
 * factor c_n = 1 + sigma y_n (lbm_ws_scale_orders), where sigma is the expansion's own
 * ratio and y the output of a multilayer perceptron of problem-level inputs
 * (lbm_ws_resum_features); the waves are synthesised on the device by lbm_set_waves.
 * The network's matrix products run on the gfx950 matrix cores in BF16 with FP32
 * accumulation (hand-written kernels); master weights, gradients and the Adam moments
 * are FP32; hidden layers use the tanh form of GELU, the output layer is linear.  The
 * converged lattice-Boltzmann solution stays the reference: the start only shortens the
 * run to it, and the plain start (rest, rho0) is the fallback.  Earlier stages of the
 * same pipeline remain available: per-point analytic base fields (lbm_ws_features),
 * each mode's exact linear response (lbm_ws_lattice_response) and the consistent
 * restart from (rho, u) fields (lbm_reset_fields).
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

/* y (rows x outputs, FP32 device) = scale * network(x (rows x inputs, FP32 device)) +
 * addend (rows x outputs, FP32 device; NULL = none: the network then learns the residual
 * over a given field); scale per output channel (lbm_mlp_set_output_scale, default 1);
 * x is rounded to BF16.  Keeps what backward needs. */
int lbm_mlp_forward(lbm_mlp *m, const float *x_dev, int64_t rows, const float *addend_dev,
                    float *y_dev);

/* Weighted mean-square loss of the last forward's output against target (rows x
 * outputs, device): L = sum_{r,c} w_c (y - t)^2 / (rows * outputs), w = channel_weight
 * (host, outputs entries, NULL = 1).  Accumulates dL/dparams into the gradients (call
 * lbm_mlp_zero_grads first) and returns L in *loss (may be NULL). */
int lbm_mlp_loss_backward(lbm_mlp *m, const float *target_dev, const float *channel_weight,
                          double *loss);

/* Output scale per channel (host, outputs entries, each > 0): lets the last layer work
 * at unit scale when the targets are small.  Applies to later forward / backward calls. */
int lbm_mlp_set_output_scale(lbm_mlp *m, const float *scale);

/* The same weighted mean-square loss for any y (rows x outputs, device, rows >= 1)
 * against target: L into *loss (may be NULL) and dL/dy into dy_dev (device).  Does not
 * touch the network's gradients (for a loss on a field derived from the output). */
int lbm_mlp_loss_grad(lbm_mlp *m, const float *y_dev, const float *target_dev,
                      const float *channel_weight, int64_t rows, float *dy_dev, double *loss);

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

#define LBM_WS_FEATURES 46  /* features per point (11 per mode for 4 modes + 2) */

/* Per-point network inputs on an n^3 grid spanning the box (point (i,j,l) sits at lattice
 * position (i, j, l) * box / n), rows in x-fastest order.  Needs nmodes == 4.  Also
 * returns the velocity scale U = sum_j |s_j| of the problem (the network's outputs are
 * velocity / U and (rho - rho0) / (U rho_scale)).  Features per mode j, with K_j = 2 pi |k_j| / box,
 * s_j = amp_j / (nu K_j^2) and theta_j = 2 pi k_j . x / box + phase_j:
 * p_j sin(theta_j) (3), p_j cos(theta_j) (3), s_j / U, K_j, k_j / |k_j| (3); then
 * tau2 - 1/2 and the Reynolds number U / (nu K_min).
 * base_dev (rows x 4, may be NULL) receives the perturbative steady solution of the
 * incompressible equations in the same units (rho0 = 1; rho_scale > 0 is used only
 * here):
 *   base_order 1: the Stokes superposition u1 = sum_j s_j p_j sin(theta_j), density 0
 *     (each mode alone, with advection dropped, is steady there);
 *   base_order 2: plus u2 and its pressure, nu lap u2 = (u1 . grad) u1 + grad p2 / rho0,
 *     solved exactly: every pair i != j forces the waves theta_i +- theta_j with
 *     A = s_i s_j (p_i . k_j) p_j / 2, giving u2 = -P_q A / (nu |q|^2) sin(.) (P_q the
 *     projection normal to q = k_i +- k_j, q = 0 skipped) and
 *     rho - rho0 = 3 p2 = 3 (q . A) / |q|^2 cos(.). */
int lbm_ws_features(const lbm_ws_problem *p, int32_t n, int32_t box, float *x_dev,
                    float *base_dev, int32_t base_order, double rho_scale,
                    const float *mode_coef_dev, double *U_out, void *hip_stream);
/* x_dev may be NULL when base_dev is not (the base alone, e.g. on the full lattice).
 * mode_coef_dev (device, 4 x 8, may be NULL) corrects each mode's own response in the
 * base: u_j = s_j ((p_j + c_0..2) sin(theta_j) + c_3..5 cos(theta_j)) and
 * rho_j - rho0 = s_j (c_6 sin(theta_j) + c_7 cos(theta_j)) (the network's output). */

/* Each mode's exact linear steady response on the periodic lattice, as mode_coef
 * coefficients (host, nmodes x 8, binary64): the steady state of the step linearised
 * about rest under the forcing g = p_j sin(theta_j), relative to the Stokes amplitude
 * s_j = 1/(nu K_j^2) per unit amp_j, nu = (tau[2] - 1/2)/3, K_j = 2 pi |k_j| / box.  It
 * is what mode_coef approaches at small Reynolds numbers, independent of amp_j and
 * phase_j.  params gives the lattice, collision and rates (with tau_bulk, tau_31,
 * max_order, force_order) and rho0 (0 = 1); its sizes, storage, boundaries, force and
 * solid fields are ignored.  Method: the collision's Jacobians in the populations and in
 * g at rest, by central differences of this library's step on a one-node periodic
 * lattice in binary64 (there the pull streaming is the identity); then per mode the Q x Q
 * complex system (I - S J) f = S G g_hat with S = diag(exp(-i kappa . e_i)),
 * kappa = 2 pi k_j / box, g_hat = -i p_j.  Uses the device (a few tiny contexts).
 * Errors: LBM_EINVAL (NULL, box < 1, nmodes outside 1..8, k_j = 0, a D2Q9 mode off the
 * x-y plane, invalid params as for lbm_init, a singular system). */
int lbm_ws_lattice_response(const lbm_params *params, const lbm_ws_problem *p, int32_t box,
                            double *coef);

/* The steady state of the forced periodic lattice expanded in the forcing amplitude to
 * order 1 to 4 about rest, as population waves for lbm_set_waves (the state is
 * w_i rho0 + sum_w Re[A_wi exp(i theta_w)]).  C(f, g) below is the collision of one node
 * as this library's step computes it, and a_j = amp_j e^{i phase_j} (f_j, -i p_j) the
 * direction of mode j in (populations, g).
 *   Order 1: one wave per mode (k_j, phase_j, A = amp_j f_j), f_j the linear response of
 *     lbm_ws_lattice_response, (I - S J) f_j = S G g_hat.
 *   Order 2 adds, for every pair i <= j, the waves k_i + k_j and k_i - k_j: the steady
 *     responses (I - S J) f = S s to the sources D2(a_i, a_j) / 2 and D2(a_i, conj a_j) / 2
 *     (1/4 instead of 1/2 when i = j) of the collision's second derivative D2.
 *   Order 3 adds the waves of the cross term D2(a_j, b_w) / 2 and D2(a_j, conj b_w) / 2
 *     (b_w the second-order waves, at k_j +- q_w) and of the cubic term: per unordered
 *     triple of signed modes, m D3(a_c1, a_c2, a_c3) / 24 at k_c1 + k_c2 + k_c3 (m its
 *     orderings, a_c = a_j or conj a_j for k_c = +-k_j; each triple counted once with its
 *     all-flipped conjugate).  Sources at one wavevector are summed, one wave each.
 *   Order 4 adds the waves of D2(delta1, delta3) + D2(delta2, delta2) / 2 +
 *     D3(delta1, delta1, delta2) / 2 + D4(delta1, delta1, delta1, delta1) / 24, delta_n the
 *     order-n field written as its conjugate-closed components (k, b/2), (-k, conj b/2),
 *     tuples within one delta taken as multisets times their orderings.
 * A wave of zero wavevector (a mean part) solves (I - J) f = s with the mean's mass and
 * momentum held at zero.  Waves of order 2 and 3 carry their phase in A (phase 0).  J, G
 * and the derivatives D2, D3 along directions are central differences of the library's
 * step on binary64 lattices, extended multilinearly (no conjugation) to complex
 * directions; all evaluations of one order run as one step of an n x 1 x 1 lattice.
 * params, box and the problem are as for lbm_ws_lattice_response (forcing
 * g = sum_j amp_j p_j sin(2 pi k_j . x / box + phase_j), integer k_j).  Outputs (host):
 * k_out max_waves x 3, phase_out max_waves, amp_out max_waves x Q x 2 ((re, im) of A_wi
 * at 2 (w Q + i)), count = the waves written; max_waves must be at least
 * lbm_ws_max_waves(nmodes, order).  Uses the device (small contexts).  Errors: those of
 * lbm_ws_lattice_response, and LBM_EINVAL for an order outside 1..4, max_waves below the
 * bound, a non-integer k or a NULL output. */
int lbm_ws_lattice_waves(const lbm_params *params, const lbm_ws_problem *p, int32_t box,
                         int32_t order, int32_t max_waves, int32_t *k_out, double *phase_out,
                         double *amp_out, int32_t *count);

/* lbm_ws_lattice_waves with the boundaries of the orders: order_end[n - 1] (4 entries) is
 * the number of waves of orders 1..n, so order n's waves are [order_end[n - 2],
 * order_end[n - 1]) (from 0 for n = 1); entries beyond `order` equal the count. */
int lbm_ws_lattice_waves_ordered(const lbm_params *params, const lbm_ws_problem *p,
                                 int32_t box, int32_t order, int32_t max_waves, int32_t *k_out,
                                 double *phase_out, double *amp_out, int32_t *count,
                                 int32_t *order_end);

/* The learned resummation of the expansion.  The steady state is approximated by
 * sum_n c_n W_n, W_n the order-n waves of lbm_ws_lattice_waves_ordered (order 4), with
 * c_n = 1 + sigma y_n, where sigma = a_3 / sqrt(a_2 a_1) (a_n the root-sum-square of the
 * order-n amplitudes: the expansion's ratio, which vanishes as the series converges) and
 * y (4 values) is the network's output.
 * lbm_ws_resum_features writes the network's LBM_WS_RESUM_FEATURES inputs and sigma from
 * a problem (nmodes 4) and its order-4 waves (amp: nwaves x Q x 2, order_end as above):
 * tau2 - 1/2; log10 sigma; log10 (a_2/a_1), (a_3/a_1), (a_4/a_1); log10 of the summed
 * Stokes amplitude U = sum_j s_j (s_j = amp_j / (nu K_j^2), K_j = 2 pi |k_j| / box) and of
 * the largest Reynolds number Re_j = amp_j / (nu^2 K_j^3); then per mode, by decreasing
 * s_j: s_j / U, K_j, log10 Re_j.  Host only.  Errors: LBM_EINVAL (NULL, nmodes != 4, an
 * order without waves). */
#define LBM_WS_RESUM_FEATURES 19
int lbm_ws_resum_features(const lbm_ws_problem *p, int32_t box, int32_t Q, const double *amp,
                          const int32_t *order_end, float *feat, double *sigma);

/* amp (waves x Q x 2, in place) of each order n scaled by c[n - 1] (4 entries).  Host. */
int lbm_ws_scale_orders(double *amp, int32_t Q, const int32_t *order_end, const double *c);

/* An upper bound on the waves lbm_ws_lattice_waves writes for nmodes modes (1..8) to
 * order 1..4 (0 for arguments outside those ranges). */
int32_t lbm_ws_max_waves(int32_t nmodes, int32_t order);

#define LBM_WS_MODE_FEATURES 13
/* Per-mode network inputs (rows nmodes x 13, device, copied before return): the phase
 * advance per lattice link kappa_a = 2 pi k_a / box (3), sin(kappa_a) (3),
 * 1 - cos(kappa_a) (3), p_j (3), tau2 - 1/2 -- what a single mode's linear lattice
 * response depends on (the lattice sees a wave through its values on the links). */
int lbm_ws_mode_features(const lbm_ws_problem *p, int32_t box, float *out_dev,
                         void *hip_stream);

/* Restart lattice c from device fields (N nodes, D velocity components):
 *   layout 0: planes rho (N), then u (D x N) (U and R unused);
 *   layout 1: the network's point-major rows (N x (D+1)): u / U, then (rho - rho0) / R;
 *   layout 2: the same quantities as channel-major planes ((D+1) x N).
 * flags (bits) transform the fields, in binary64 and in this order, before the state is
 * built:
 *   LBM_RESET_FILTER: along every periodic axis, the 7-point low-pass filter
 *     (11/16, 15/64, -3/32, 1/64 at offsets 0, +-1, +-2, +-3), transfer 1 - sin^6(k/2),
 *     which removes the wavenumber pi.  The linearised step of every velocity set here
 *     has an eigenvalue -1 at k = (pi, 0, 0) (and its permutations), a checkerboard
 *     along one axis that never decays, so a start with content there never becomes
 *     steady;
 *   LBM_RESET_MASS: adds one constant to rho so that sum rho = N rho0 (the mass of the
 *     plain start);
 *   LBM_RESET_MOMENTUM: subtracts one constant vector from u so that sum rho u = 0.
 *     With no walls the dynamics conserve total mass and momentum (the forcing sums to
 *     zero over the periodic box), so a start that differs from the plain start in
 *     them ends in a different, drifting state.
 * The state becomes the force-corrected equilibrium of the fields (as lbm_init), time 0,
 * and with
 *   LBM_RESET_NONEQ: plus the non-equilibrium second moment the velocity gradient implies
 *     to leading order, Pi = -c_s^2 tau2 rho (grad u + grad u^T) (tau2 = tau[2]; central
 *     differences, one-sided at walls), as the Hermite term w_i (e_i e_i - c_s^2 I) : Pi /
 *     (2 c_s^4).  Without it the start carries no stress; the jump relaxes within a few
 *     steps but launches pressure waves that hold the per-step residual up for many. */
#define LBM_RESET_MASS 1
#define LBM_RESET_MOMENTUM 2
#define LBM_RESET_FILTER 4
#define LBM_RESET_NONEQ 8
int lbm_reset_fields(lbm_ctx *c, const float *fields_dev, int32_t layout, double U, double R,
                     int32_t flags);

#ifdef __cplusplus
}
#endif
#endif /* LBM_NN_H */
