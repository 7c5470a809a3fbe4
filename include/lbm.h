/*
 * lbm.h -- C ABI of the MI355X (gfx950) forced lattice-Boltzmann library.
 *
 * The library advances the discrete-velocity Boltzmann equation with a body force,
 * d f_i/dt + e_i . grad f_i = Omega_i + F_i (Li, Duan & Shan, arXiv 2212.07494,
 * Sec. II.A, eq:dv), discretised in space and time by the second-order (trapezoidal)
 * rule of Sec. II.B: the stored variable is f-bar_i = f_i - Omega_i/2 - F_i/2
 * (eq:newf) and one step is f-bar_i(x + e_i, t+1) = f-bar_i + Omega_i + F_i
 * (eq:evolution), implemented as one fused pull-streaming + collision kernel.
 *
 *   collision  BGK   : eq:explict_eq with the second-order truncated equilibrium and
 *                      the second-order (Guo-form) force term (Sec. II.B).
 *              SMRT  : relaxation of central Hermite moments per order (eq:domg,
 *                      eq:RHS), force entering through the first central moment only,
 *                      back-transform of eq:bbd1 to order 4, reconstruction with the
 *                      lattice's exact inverse Hermite transform (Sec. II.C), or on
 *                      D3Q39 with the paper's Hermite sum to order 4 itself.
 *   lattice    D2Q9, D3Q19, D3Q27 (lattice units, c_s^2 = 1/3, quadrature degree 5) and
 *              the high-order lattice D3Q39 (c_s^2 = 2/3, degree 7; periodic boxes).
 *   force      g(x, t) = g(x) s(t): an acceleration; the force density is rho g.
 *   walls      halfway bounce-back (stationary no-slip wall midway between the last
 *              fluid node and the next) on both faces of an axis, or periodic.
 *
 * Conventions for every entry point
 *   - Returns LBM_OK (0), a negative lbm_status (an error) or the positive warning
 *     LBM_WMACH; never aborts or throws.  After a failure or warning lbm_last_error()
 *     returns a thread-local message.
 *   - Node index n = (z * ny + y) * nx + x (x fastest); N = nx * ny * nz (nz = 1 in 2-D).
 *   - Host arrays passed in are read during the call only; the caller keeps them.
 *     Output arrays are caller-allocated host memory.
 *   - All device work is enqueued on the HIP stream given at init, in call order.
 *     Calls that return host data (lbm_moments, lbm_get_populations, lbm_monitors)
 *     synchronise that stream; lbm_step and lbm_set_populations do not.
 *   - A context is not thread-safe; distinct contexts are independent.
 *
 * Population order (shared with any external consumer of lbm_get_populations):
 *   i = 0 rest, then pairs (e, -e):
 *   D2Q9 : (1,0) (-1,0) (0,1) (0,-1) (1,1) (-1,-1) (1,-1) (-1,1)
 *   D3Q19: +-x, +-y, +-z, +-(1,1,0), +-(1,-1,0), +-(1,0,1), +-(1,0,-1), +-(0,1,1), +-(0,1,-1)
 *   D3Q27: D3Q19 then +-(1,1,1), +-(1,1,-1), +-(1,-1,1), +-(1,-1,-1)
 *   D3Q39: +-x, +-y, +-z, +-(1,1,1), +-(1,1,-1), +-(1,-1,1), +-(1,-1,-1), +-(2,0,0),
 *          +-(0,2,0), +-(0,0,2), +-(2,2,0), +-(2,-2,0), +-(2,0,2), +-(2,0,-2), +-(0,2,2),
 *          +-(0,2,-2), +-(3,0,0), +-(0,3,0), +-(0,0,3)
 */
#ifndef LBM_H
#define LBM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  LBM_OK = 0,
  LBM_WMACH = 1,       /* warning, the call did its work: a monitor record showed
                          max |u| > mach_limit c_s (see lbm_params.mach_limit) */
  LBM_EINVAL = -1,     /* invalid argument or parameter combination */
  LBM_ENOMEM = -2,     /* device or host allocation failed */
  LBM_EDEVICE = -3,    /* a HIP call failed; message in lbm_last_error() */
  LBM_ENONFINITE = -4, /* the monitors saw a NaN or Inf; the state is kept for inspection */
  LBM_ESTATE = -5      /* NULL or wrong-kind context */
} lbm_status;

/* LBM_D3Q39: the degree-7 quadrature of speed shells |e|^2 = 0, 1, 3, 4, 8, 9 with
 * weights 1/12, 1/12, 1/27, 2/135, 1/432, 1/1620 and c_s^2 = 2/3 (viscosity
 * (2/3)(tau[2] - 1/2)).  It carries every Hermite moment of order <= 4 (35 of them; on
 * its 39 velocities they span 29 dimensions); SMRT and RMRT rebuild the post-collision
 * populations from those moments with the Hermite sum to order 4 (the reconstruction
 * after eq:bbd1), which keeps the moments of orders 0 to 3 exactly and drops what the
 * moments do not describe.  Periodic boxes only, every extent >= 3, no solid nodes, no
 * tau_31 (it carries D_aaa); not in the batched engine or the warm-start expansion. */
typedef enum { LBM_D2Q9 = 0, LBM_D3Q19 = 1, LBM_D3Q27 = 2, LBM_D3Q39 = 3 } lbm_lattice;
/* LBM_BGK: single relaxation time with the second-order force term (eq:explict_eq).
 * LBM_SMRT: central-moment relaxation per Hermite order with the force in the first
 * central moment (Sec. II.C).  LBM_RMRT: the raw-moment MRT of the paper's appendix
 * (eq:RHS_a, explicit form, raw force moments a_F^(n) of eq:bbd1): same rates and the
 * same trimming of order 4 as SMRT; differs from it at order 3. */
typedef enum { LBM_BGK = 0, LBM_SMRT = 1, LBM_RMRT = 2 } lbm_collision;

/* Storage of the populations in HBM and the arithmetic of the step.
 *   LBM_F64          binary64 values of f-bar_i, binary64 arithmetic (reference mode).
 *   LBM_F32          binary32 values of f-bar_i, binary32 arithmetic.
 *   LBM_F32_SHIFTED  binary32 deviations f-bar_i - w_i rho0, binary32 arithmetic.
 *   LBM_F16_SHIFTED  binary16 deviations f-bar_i - w_i rho0, binary32 arithmetic.
 * Stores round to nearest-even.  Bytes per node and step: 2 Q sizeof(storage). */
typedef enum { LBM_F64 = 0, LBM_F32 = 1, LBM_F32_SHIFTED = 2, LBM_F16_SHIFTED = 3 } lbm_storage;

typedef enum { LBM_PERIODIC = 0, LBM_WALLS = 1 } lbm_bc;

/* Acceleration field g(x):
 *   LBM_G_UNIFORM  g_uniform[3] everywhere.
 *   LBM_G_PROFILE  g depends on one coordinate: g_axis in {0,1,2}; g_data holds
 *                  3 x n_axis doubles, component-major (gx[0..n), gy[0..n), gz[0..n)).
 *   LBM_G_FIELD    g_data holds 3 x N doubles, component planes (gx[N], gy[N], gz[N]).
 * 2-D lattices ignore the z component. */
typedef enum { LBM_G_UNIFORM = 0, LBM_G_PROFILE = 1, LBM_G_FIELD = 2 } lbm_force_kind;

/* Optional device allocator (e.g. a framework's caching allocator).  alloc returns
 * device memory of at least `bytes` bytes aligned to 256 bytes, or NULL. */
typedef struct {
  void *(*alloc)(size_t bytes, void *user);
  void (*free)(void *ptr, void *user);
  void *user;
} lbm_allocator;

typedef struct {
  int32_t lattice;     /* lbm_lattice */
  int32_t collision;   /* lbm_collision */
  int32_t storage;     /* lbm_storage */
  int32_t nx, ny, nz;  /* nz must be 1 for D2Q9 */
  int32_t bc[3];       /* lbm_bc per axis (both faces of the axis) */
  /* tau-hat per Hermite order n (tau-hat = tau + 1/2 of Sec. II.B, omega_n = 1/tau-hat_n,
   * viscosity c_s^2 (tau[2] - 1/2)).  BGK uses tau[2] only.  SMRT and RMRT relax order 2 with
   * tau[2] and order 3 with tau[3]; order 4 is trimmed, which is tau[4] == 1 (required).
   * tau[0], tau[1] are ignored (mass and momentum are conserved).  Each used value > 1/2. */
  double tau[5];
  double rho0;         /* reference density: the shift of *_SHIFTED storage; default rho */
  int32_t g_kind;      /* lbm_force_kind */
  int32_t g_axis;      /* for LBM_G_PROFILE */
  double g_uniform[3]; /* for LBM_G_UNIFORM */
  const double *g_data;         /* host array, copied at init (see lbm_force_kind) */
  int32_t monitor_every;        /* K >= 1: lbm_step updates the monitors every K steps; 0 = never */
  const lbm_allocator *allocator; /* NULL: hipMalloc / hipFree */
  /* Force content of the SMRT collision (Sec. II.C): 1 (or 0) = first order only, the
   * paper's choice when the non-equilibrium parts are neglected (d_F^(n) = 0, n >= 2);
   * 3 = also d_F^(3) = 3 g d^(2) (eq:Frc at theta = 1), with d^(2) the non-equilibrium
   * central second moment of f itself, the mean of the moments before and after the
   * collision (eq:newf, eq:evolution; the trace at tau_bulk where that is set), added to
   * the relaxed third-order central moments as (1 - 1/(2 tau[3])) d_F^(3), on the
   * lattice's third-order index set; 4 = also the fourth-order term of eq:Frc,
   * d_F^(4) = 4 g d^(3) with d^(3) likewise the mean of order 3, entering the trimmed
   * order 4 with 1 - omega_4/2 = 1/2 (not on D3Q39, whose fourth-order moments are not
   * independent on its 39 velocities, and not with max_order 6).  BGK and RMRT: 0 or 1. */
  int32_t force_order;
  /* Solid nodes: host array of N bytes (nonzero = solid), copied at init; NULL = none.
   * A fluid node whose pull source x - e_i is solid takes halfway bounce-back from its
   * own node, f-bar_i(x, t+1) = f-bar*_opp(i)(x, t), as at a wall face (a stationary wall
   * halfway between the two nodes).  Solid nodes are not stepped; lbm_moments reports
   * rho = 0 and u = 0 there, the monitors sum over fluid nodes only, and populations
   * stored at solid nodes are unspecified.  At least one node must be fluid. */
  const uint8_t *solid;
  /* SMRT only: relaxation time (tau-hat) of the trace of the second-order moment, the
   * irreducible component S^(2,0) of eq:domg (bulk viscosity (2/D) c_s^2 (tau_bulk - 1/2));
   * the traceless part keeps tau[2] (shear).  0 = tau[2] (one rate for order 2). */
  double tau_bulk;
  /* SMRT on D3Q19 / D3Q27 only: relaxation time of the third-order trace S^(3,1) of
   * eq:domg, the vector sum_b D_abb of the central third moment; the lattices carry it as
   * D_abb + D_acc (b, c the other two axes; D_aaa is not carried).  The traceless rest
   * (the differences D_abb - D_acc and D_xyz) keeps tau[3].  0 = tau[3].  Not with
   * force_order 3 or 4. */
  double tau_31;
  /* Highest Hermite order carried after the collision.  0 or 4: raw moments above order
   * 4 are set to zero (the reconstruction sums to order 4, as the paper does).  6 (SMRT on
   * D3Q27 only): orders 5 and 6 are carried as rho u^m plus the back-shift of the
   * relaxed central moments, their own central parts trimmed to zero like order 4. */
  int32_t max_order;
  /* Mach guard: if > 0, a monitor record whose max |u| exceeds mach_limit c_s (c_s^2 =
   * 1/3) makes the call that reads it return the warning LBM_WMACH (the low-Mach
   * expansion behind the truncated equilibrium loses accuracy there).  0 = off. */
  double mach_limit;
  /* Debug pass: 1 = before every step, fill the buffer the step writes with NaN, so a
   * value that the next step pulls but this step did not write shows up as NaN in the
   * results (every slot a step pulls is written by the step before it).  0 = off. */
  int32_t debug_poison;
} lbm_params;

/* Monitor record (binary64, summed on the device in a fixed order).
 *   mass = sum rho, mom = sum rho u (physical u of eq:half_F), j = sum_x sum_i f-bar_i e_i
 *   (= sum rho u-bar: the stored first moment, mom - sum F/2), umax = max |u|,
 *   resid = sqrt(sum |u(t) - u(t-1)|^2 / sum |u(t)|^2) over the nodes,
 *   nonfinite = number of nodes whose rho or u is NaN or Inf.
 * step is the time t the fields belong to (-1: never computed). */
typedef struct {
  int64_t step;
  double mass, mom[3], j[3], umax, resid;
  int64_t nonfinite;
} lbm_monitors;

typedef struct lbm_ctx lbm_ctx; /* opaque, owned by the library */

/* Create a lattice of the given parameters and set its state to the force-corrected
 * equilibrium f-bar_i = f_eq_i(rho, u) - F_i(rho, u, g(x, 0))/2 (eq:newf with Omega = 0),
 * whose density and physical velocity are exactly rho and u.
 *   rho_init : N doubles, or NULL for rho0 everywhere.
 *   u_init   : D x N doubles (component planes, D = 2 or 3), or NULL for rest.
 *   hip_stream: a hipStream_t (NULL = the default stream).
 * Errors: LBM_EINVAL (tau <= 1/2, SMRT with tau[4] != 1, nz != 1 on D2Q9, unknown
 * enum, non-positive size, node count >= 2^31, missing g_data, rho0 <= 0, D3Q39 with
 * walls, solid nodes, tau_31 or an extent below 3, force_order 3 or 4 without SMRT,
 * force_order 4 on D3Q39 or with max_order 6, tau_31 with force_order 3 or 4),
 * LBM_ENOMEM, LBM_EDEVICE.  On error *out is NULL. */
int lbm_init(const lbm_params *p, const double *rho_init, const double *u_init,
             void *hip_stream, lbm_ctx **out);

/* Advance n >= 0 steps.  g_scale: NULL (s(t) = 1) or n host doubles, the factor s(t)
 * of g(x) for each step.  Enqueues work only (no synchronisation), except as below.
 * Small lattices (N <= 2^21 nodes), where launch overhead dominates: when n covers at
 * least two chunks of 64 steps and neither monitor_every nor debug_poison is set, the
 * chunks are replayed from a HIP graph captured once per buffer parity (the factors s(t)
 * are then staged in pinned host memory, uploaded asynchronously and read on the device;
 * the call waits only for the previous call's upload to have completed); the remainder
 * runs as single launches.  The results are identical to single launches.
 * Monitors in the step: if monitor_every is K > 0, after every step whose time t is a
 * multiple of K the monitor record of time t is computed on the device (with the
 * residual against time t - 1, whose velocity is recorded one step earlier; K = 1
 * compares every step) and copied to host memory without blocking.  lbm_step and every
 * call that synchronises the stream read the latest such record once it is complete:
 *   - non-finite nodes: the call returns LBM_ENONFINITE, lbm_step refuses to advance
 *     (the state is kept for inspection) until the state is replaced (lbm_set_populations,
 *     lbm_set_waves, lbm_reset_fields, lbm_load);
 *   - max |u| above the Mach limit: LBM_WMACH (warning; the call did its work).
 * lbm_monitors_get at such a time t returns that record as computed in the step. */
int lbm_step(lbm_ctx *c, int64_t n, const double *g_scale);

/* Density and physical velocity u = j/rho + g s/2 (eq:half_F) of the current state,
 * evaluated with acceleration g(x) * g_scale.  rho: N doubles or NULL; u: D x N doubles
 * (component planes) or NULL.  Synchronises the stream.  May return LBM_ENONFINITE or
 * LBM_WMACH from an in-step monitor record (see lbm_step); the outputs are written. */
int lbm_moments(lbm_ctx *c, double g_scale, double *rho, double *u);

/* Return the monitor record of the current time t: the one computed in lbm_step at t
 * if monitor_every made one, else a fresh one (force scale of the last step, 1 before
 * any step).  resid compares with the state one step earlier when that was recorded,
 * else 0.  Returns LBM_ENONFINITE if any node is not finite, LBM_WMACH if max |u|
 * exceeds the Mach limit (the record is filled either way).  Synchronises the stream. */
int lbm_monitors_get(lbm_ctx *c, lbm_monitors *mon);

/* Pre-collision populations f-bar_i(x, t) of the current state, values as stored
 * (f-bar_i - w_i rho0 for *_SHIFTED storage) converted exactly to binary64.
 *   nodes: nnodes node indices, or NULL for all N nodes in order (then nnodes == N).
 *   out  : Q x nnodes doubles, population-major.  Synchronises the stream. */
int lbm_get_populations(lbm_ctx *c, int64_t nnodes, const int64_t *nodes, double *out);

/* For callers that cannot allocate device memory (code under HIP graph capture, tight
 * serving loops, harnesses that forbid hipMalloc): lbm_get_populations staging through a
 * fixed device array of LBM_NOALLOC_SCRATCH_BYTES instead of memory it allocates on
 * demand.  Same arguments and results as lbm_get_populations, for nnodes with
 * (Q + 1) * 8 * nnodes <= LBM_NOALLOC_SCRATCH_BYTES (Q * 8 * N with nodes NULL); larger
 * requests fail with LBM_EINVAL.  Calls no allocating routine.  Every context on a
 * device shares that device's array (set up by lbm_init, kept until the process ends):
 * calls that overlap on one device race; calls on one stream, or synchronised, do not. */
#define LBM_NOALLOC_SCRATCH_BYTES (4 << 20)
int lbm_get_populations_noalloc(lbm_ctx *c, int64_t nnodes, const int64_t *nodes, double *out);

/* Replace the state by the given pre-collision populations (Q x N doubles, as stored,
 * population-major), rounded to the storage type (nearest-even). */
int lbm_set_populations(lbm_ctx *c, const double *f);

/* Replace the state by a sum of Fourier waves about rest, synthesised on the device:
 *   f-bar_i(x) = w_i rho0 + sum_w Re[A_wi exp(i theta_w(x))],
 *   theta_w(x) = 2 pi (k_w0 x / nx + k_w1 y / ny + k_w2 z / nz) + phase_w,
 * at every fluid node, evaluated in binary64 and rounded once to the storage type (for
 * *_SHIFTED storage the stored value is f-bar_i - w_i rho0).  The populations are the
 * pre-collision f-bar of Sec. II.B, as lbm_set_populations takes them; w_i rho0 is the
 * unforced rest state.  Arguments (host, read before return): k: nwaves x 3 int32
 * wavevectors (any integers; k_wa x_a is reduced modulo n_a), phase: nwaves binary64,
 * amp: nwaves x Q x 2 binary64, the (re, im) pairs of A_wi at 2 (w Q + i).  nwaves = 0
 * gives the rest state.  Resets the time to 0, like lbm_set_populations; values at solid
 * nodes are unspecified.  Errors: LBM_EINVAL (nwaves outside 0..LBM_MAX_WAVES, a NULL
 * array with nwaves > 0, a non-finite amplitude or phase), LBM_ESTATE, LBM_EDEVICE. */
#define LBM_MAX_WAVES 4096
int lbm_set_waves(lbm_ctx *c, int32_t nwaves, const int32_t *k, const double *phase,
                  const double *amp);

/* Simulation time t (number of steps taken since init or the last set_populations). */
int lbm_time(const lbm_ctx *c, int64_t *t);

/* Bytes of device memory the context holds. */
int lbm_device_bytes(const lbm_ctx *c, size_t *bytes);

int lbm_free(lbm_ctx *c);

/* Checkpoint / resume.  lbm_save writes the state as stored (populations in the storage
 * format and the library's slot layout), the time, and a hash of everything the dynamics
 * depend on (lattice, collision, storage, sizes, boundaries, rates, rho0, force content
 * and the force table as uploaded); it synchronises the stream.  lbm_load restores time
 * and state into a context created with the same parameters (LBM_EINVAL with a message
 * if the file is not a checkpoint, is truncated or does not match; the context is then
 * unchanged).  Running n steps, saving, loading into a fresh context and running n more
 * gives the same state bit for bit as 2n steps.  The residual monitor restarts (it
 * needs a previous record).  Files are for this library version and machine byte order. */
int lbm_save(lbm_ctx *c, const char *path);
int lbm_load(lbm_ctx *c, const char *path);

/* Launch configuration of the step kernel: block shape bx x by (bx in {64, 128, 256},
 * bx * by <= 256) and variant 0..59, whose base b = variant % 12 selects the memory
 * access b % 3 (0 plain loads and stores, 1 non-temporal stores, 2 non-temporal loads and
 * stores); (b / 3) odd also lets workgroups that cannot bounce back (no solid nodes, away
 * from wall faces) address each population plane through a scalar base and 32-bit
 * offsets; b >= 6 places the blocks XCD-contiguously (each of the chip's 8 XCDs, with its
 * own L2, steps one contiguous stretch of the lattice, so the lines neighbouring blocks
 * share stay in one L2) instead of in dispatch order.  variant / 12 = 1, 2, 3, 4 holds the
 * step's workgroups to at most 5, 4, 3, 2 waves per SIMD (each reserves LDS it does not
 * use, so fewer fit on a CU; fewer concurrent streams of populations can use HBM better);
 * 0 leaves as many as the kernel's registers allow, as does a cap the block shape cannot
 * express.  Results are identical for every configuration; only the speed differs. */
typedef struct {
  int32_t bx, by;
  int32_t variant;
} lbm_tuning;

int lbm_set_tuning(lbm_ctx *c, const lbm_tuning *t);
int lbm_get_tuning(const lbm_ctx *c, lbm_tuning *t);

/* Time every block shape with the variants 0..11 for `steps` steps (>= 1), then the
 * fastest of those with each wave cap (variant + 12 k, k = 1..4), and keep the fastest
 * of all.  The state is saved before and restored after, so the simulation is
 * unchanged.  best and
 * best_ms (time per step of the winner) may be NULL.  Synchronises the stream and
 * temporarily needs one extra population buffer of device memory. */
int lbm_autotune(lbm_ctx *c, int32_t steps, lbm_tuning *best, double *best_ms);

/* Stream-copy probe: dst = src for `bytes` bytes (multiple of 16) of device memory,
 * enqueued `reps` times on hip_stream with the block size `block` (64..1024, multiple
 * of 64; 0 = 256).  variant: 0 grid-stride 16-byte vectors, 1 one 16-byte vector per
 * thread, 2 as 1 with non-temporal loads and stores, 3 four vectors per thread.  The
 * best read + write bandwidth over variants is the practical HBM roofline the step is
 * compared against. */
int lbm_copy_probe(const void *src, void *dst, size_t bytes, int32_t reps, int32_t block,
                   int32_t variant, void *hip_stream);

const char *lbm_strerror(int status);
const char *lbm_last_error(void);
int lbm_version(void); /* 100 * major + minor */

/* The velocity set of a lattice in the population order above: D, Q, the velocities
 * (e: Q x 3 int32, x y z) and the weights (w: Q binary64); any output may be NULL.  Host
 * only (no device, no context).  Errors: LBM_EINVAL (unknown lattice). */
int lbm_lattice_info(int32_t lattice, int32_t *D, int32_t *Q, int32_t *e, double *w);

#ifdef __cplusplus
}
#endif
#endif /* LBM_H */
