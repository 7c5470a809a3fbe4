/*
 * lbm_batch.h -- many independent lattice-Boltzmann domains stepped together.
 *
 * Each domain is its own instance of the forced discrete-velocity Boltzmann problem of
 * lbm.h (Li, Duan & Shan, arXiv 2212.07494, Sec. II.A eq:dv; the step is eq:evolution
 * with the BGK update eq:explict_eq or the SMRT update of Sec. II.C): its own size,
 * walls, relaxation times and acceleration field.  All domains share one lattice,
 * collision model and storage mode, and all are advanced by ONE persistent kernel
 * launch per time step: a fixed grid of workgroups walks a flattened table of
 * equal-sized tiles (one tile = one workgroup's worth of nodes of one domain), so
 * uneven domains load-balance.  lbm_batch_run captures K steps plus the convergence
 * monitors as one HIP graph and replays it; per-domain convergence is decided on the
 * device, and the tiles of converged domains are skipped.
 *
 * Conventions are those of lbm.h: status codes, lbm_last_error(), node order
 * n = (z ny + y) nx + x within a domain, population order, host arrays copied during
 * the call, device work on the stream given at init.
 */
#ifndef LBM_BATCH_H
#define LBM_BATCH_H

#include <stddef.h>
#include <stdint.h>

#include "lbm.h"

#ifdef __cplusplus
extern "C" {
#endif

/* One domain.
 *   nx, ny, nz : size (nz = 1 on D2Q9).
 *   bc[3]      : lbm_bc per axis.
 *   tau[5]     : tau-hat per Hermite order as in lbm_params (BGK: tau[2]; SMRT:
 *                tau[2], tau[3], tau[4] == 1).
 *   g_kind     : LBM_G_UNIFORM (g_uniform), LBM_G_PROFILE (g_axis, g_data: 3 x n_axis
 *                doubles, component-major) or LBM_G_FIELD (g_data: 3 x N doubles).
 *   rho_init, u_init : optional initial density (N) and velocity (D x N) fields, NULL
 *                for rho0 and rest. */
typedef struct {
  int32_t nx, ny, nz;
  int32_t bc[3];
  double tau[5];
  int32_t g_kind, g_axis;
  double g_uniform[3];
  const double *g_data;
  const double *rho_init;
  const double *u_init;
} lbm_domain;

/* Per-domain status after lbm_batch_run. */
typedef enum {
  LBM_DOM_RUNNING = 0,   /* still stepping (max_steps reached first) */
  LBM_DOM_CONVERGED = 1, /* resid < tol at a check */
  LBM_DOM_FLOOR = 2,     /* resid stopped decreasing and is noise: round-off floor (below) */
  LBM_DOM_NONFINITE = 3  /* NaN/Inf seen; the domain was stopped */
} lbm_domain_status;

typedef struct lbm_batch lbm_batch;

/* Create ndom >= 1 domains (lattice, collision, storage as in lbm_params; rho0 as in
 * lbm_params) and set each to its force-corrected equilibrium, as lbm_init does.
 * Errors: LBM_EINVAL (any domain invalid: message names it), LBM_ENOMEM, LBM_EDEVICE. */
int lbm_batch_init(const lbm_domain *domains, int32_t ndom, int32_t lattice, int32_t collision,
                   int32_t storage, double rho0, void *hip_stream, lbm_batch **out);

/* Advance every still-active domain by n steps (no convergence checks).  Enqueues only. */
int lbm_batch_advance(lbm_batch *b, int64_t n);

/* Step until every domain has converged (resid < tol), hit its round-off floor, or
 * max_steps steps were taken.  resid is the per-domain relative per-step change of the
 * physical velocity, sqrt(sum |u(t) - u(t-1)|^2 / sum |u(t)|^2), checked every
 * check_every steps (even, >= 2).  A domain is stopped as LBM_DOM_FLOOR when for
 * stall_checks consecutive checks its resid has not dropped below 0.99 of its best value
 * and its change is noise rather than a drift: over a window of stall_checks checks, the
 * change of the velocity divided by the window's steps is below 3% of the last
 * step's change (a state still converging, however slowly, drifts steadily and is not
 * stopped; round-off noise does not accumulate over the window).  Each
 * check_every steps with the monitor pass run as one replay of a captured HIP graph.
 * Outputs (ndom entries each, any may be NULL): steps taken, last resid, status.
 * Synchronises the stream once per replay. */
int lbm_batch_run(lbm_batch *b, int64_t max_steps, double tol, int32_t check_every,
                  int32_t stall_checks, int64_t *steps_out, double *resid_out,
                  int32_t *status_out);

/* The batched step of the problem statement (eq:dv per domain, advanced by eq:evolution):
 * step every domain until its residual (as in lbm_batch_run) is below tol, it reaches its
 * round-off floor, or max_steps steps were taken; the same as lbm_batch_run with
 * check_every = LBM_BATCH_CHECK_EVERY and stall_checks = LBM_BATCH_STALL_CHECKS.
 * steps_out, resid_out: ndom entries each, or NULL.  The per-domain outcome is read with
 * lbm_batch_status.  Errors as lbm_batch_run. */
#define LBM_BATCH_CHECK_EVERY 100
#define LBM_BATCH_STALL_CHECKS 10
int lbm_batch_step(lbm_batch *b, int64_t max_steps, double tol, int64_t *steps_out,
                   double *resid_out);

/* Per-domain lbm_domain_status after the last run (ndom entries).  Synchronises. */
int lbm_batch_status(lbm_batch *b, int32_t *status_out);

/* Density and physical velocity of domain dom (as lbm_moments, force scale 1). */
int lbm_batch_moments(lbm_batch *b, int32_t dom, double *rho, double *u);

/* Pre-collision populations of domain dom, values as stored (as lbm_get_populations). */
int lbm_batch_get_populations(lbm_batch *b, int32_t dom, double *f);

/* Replace domain dom's state (Q x N doubles as stored); it becomes active again. */
int lbm_batch_set_populations(lbm_batch *b, int32_t dom, const double *f);

/* Launch configuration: tile policy (tile_bx 64, 128, 256: tiles of that width and
 * 256/tile_bx rows; 0: per domain the smallest of those covering nx; 1: linear tiles
 * of 256 consecutive nodes of a layer, every lane busy whatever the width), persistent
 * workgroups per compute unit (1..32; 0: one workgroup per tile instead of a persistent
 * grid) and the memory variant of lbm_tuning.  Results do not depend on it. */
typedef struct {
  int32_t tile_bx;
  int32_t blocks_per_cu;
  int32_t variant;
} lbm_batch_tuning;

int lbm_batch_set_tuning(lbm_batch *b, const lbm_batch_tuning *t);
int lbm_batch_get_tuning(const lbm_batch *b, lbm_batch_tuning *t);

/* Time every launch configuration for `steps` steps on a saved copy of the state and
 * keep the fastest (the state is restored).  best / best_ms (per step) may be NULL. */
int lbm_batch_autotune(lbm_batch *b, int32_t steps, lbm_batch_tuning *best, double *best_ms);

/* Total nodes, tiles and device bytes of the batch (any pointer may be NULL). */
int lbm_batch_info(const lbm_batch *b, int64_t *nodes, int64_t *tiles, size_t *bytes);

int lbm_batch_free(lbm_batch *b);

#ifdef __cplusplus
}
#endif
#endif /* LBM_BATCH_H */
