// Internal interface between the C-ABI runtime (lbm_runtime.hip) and the per-lattice
// kernel units (lbm_d2q9.hip, lbm_d3q19.hip, lbm_d3q27.hip, lbm_d3q39.hip), which are compiled
// separately so the heavily unrolled kernels build in parallel.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace lbm {

// Slots of a monitor record (binary64), per block partial and after finalisation: mass,
// momentum of the physical velocity sum rho u (x, y, z), sum j = sum f-bar e (x, y, z),
// sum |u(t) - u(t-1)|^2, sum |u|^2, max |u|, non-finite node count.
enum {
  MON_MASS = 0, MON_MX, MON_MY, MON_MZ, MON_JX, MON_JY, MON_JZ, MON_DU2, MON_U2, MON_UMAX,
  MON_BAD, MON_SLOTS
};

// Solid mask word: bit i = the pull source of population i is solid; this bit = the
// node itself is solid.
constexpr uint32_t SOLID_NODE = 1u << 31;

struct GeomDesc {
  int nx, ny, nz, N;
  int64_t ps;  // plane stride (elements between population planes), >= nx ny
  int wall[3];
  const uint32_t *smask;  // device, per-node solid mask words (NULL: no solid nodes)
};

// One launch of a lattice kernel.  Coefficients are binary64 on the host and are
// rounded once to the arithmetic type of the storage mode.
struct LaunchDesc {
  int coll;      // 0 BGK, 1 SMRT with one rate per order, 2 RMRT; SMRT whose traces may
                 // relax at rates of their own: 7, 3 carrying orders 5-6 (D3Q27), and with
                 // the non-equilibrium force content 4 to order 3, 5 to order 4, 6 to
                 // order 3 carrying orders 5-6
  int storage;   // lbm_storage
  int gk;        // 0 profile/uniform table, 1 full field
  const void *fin;
  void *fout;
  GeomDesc geo;
  const void *gtab;  // force table in the arithmetic type
  int g_axis, g_n;
  double gscale;
  double shift;
  double c0, c1;
  double c2;         // SMRT: coefficient of the third-order force term (0 = off); RMRT: h2
  double c3;         // RMRT: h3 = 1 - omega_3 / 2; SMRT: (q_bulk - q2)/D (0 = one rate)
  double c4;         // SMRT: (q_31 - q3)/2 for the third-order trace pairs (0 = one rate)
  int bx, by;        // block shape (bx * by <= 256, bx a multiple of 64)
  int variant;       // memory-access variant of the step kernel (MEM_*)
  int fast_ok;       // 1: blocks that cannot bounce back may take the scalar-base path
  int xcd;           // 1: XCD-contiguous block placement, 0: dispatch order
  // Dynamic LDS a workgroup of the step kernel reserves and never touches (0: none): it
  // caps the workgroups resident on a CU, and so the waves per SIMD, below what the
  // kernel's registers allow.
  unsigned lds_pad;
  // Force factor from device memory (steps replayed from a captured graph): when gs_dev
  // is set, s(t) = gs_dev[*gs_ctr + gs_j] instead of gscale.
  const double *gs_dev;
  const int64_t *gs_ctr;
  int gs_j;
};

// One launch of the batched engine's persistent kernels.
struct BatchLaunch {
  int coll, storage, variant;
  const void *fin;
  void *fout;
  const void *gbuf;
  const void *doms;   // device BatchDom[ndom]
  const void *tiles;  // device BatchTile[ntiles]
  const int *active;
  int ntiles;
  int grid;           // persistent workgroups
  double shift;
  void *urec;         // monitor: recorded velocities (the step before a check)
  void *uchk;         // monitor: velocities at the start of the coherence window
  const void *state;  // monitor: per-domain DomState (which checks start a window)
  int window;         // monitor: checks per coherence window
  int mode;           // monitor: 2 record, 4 compare + record
  double *partials;   // monitor: BATCH_PARTIALS per tile
};

// Per-tile slots of the batched monitor: sum |u(t) - u(t-1)|^2, sum |u|^2, non-finite
// count, sum |u(t) - u(start of the coherence window)|^2.
enum { BP_DU2 = 0, BP_U2, BP_BAD, BP_DUK2, BATCH_PARTIALS };

struct LatticeOps {
  int D, Q;
  const int *E;     // host: the Q velocities, Q x 3 (x, y, z)
  const double *W;  // host: the Q weights
  hipError_t (*step)(const LaunchDesc &, hipStream_t);
  // pi: optional non-equilibrium second moment, 6 binary64 planes (xx, yy, zz, xy, xz, yz)
  hipError_t (*init)(const LaunchDesc &, const double *rho, const double *u, double rho0,
                     const double *pi, hipStream_t);
  hipError_t (*gather)(const LaunchDesc &, const int64_t *nodes, int64_t nn, double *out,
                       hipStream_t);
  // Host: per-node solid mask words from a byte mask (bit i: the pull source of
  // population i is solid, periodic wrap, sources across a wall face not marked; bit 31:
  // the node is solid).
  void (*solid_words)(const uint8_t *solid, int nx, int ny, int nz, const int wall[3],
                      uint32_t *out);
  hipError_t (*scatter)(const LaunchDesc &, const double *in, hipStream_t);
  // State from nw Fourier waves about the rest state of density base (waves_kernel;
  // device arrays k: nw x 3, phase: nw, amp: nw x Q x 2)
  hipError_t (*waves)(const LaunchDesc &, int nw, const int *k, const double *phase,
                      const double *amp, double base, hipStream_t);
  hipError_t (*moments)(const LaunchDesc &, double *rho, double *u, void *uprev, int mode,
                        double *partials, hipStream_t);
  hipError_t (*batch_step)(const BatchLaunch &, hipStream_t);
  hipError_t (*batch_monitor)(const BatchLaunch &, hipStream_t);
};

// Per-domain convergence state of the batched engine (device array, one per domain).
struct DomState {
  int64_t steps;
  double resid, best;
  int status, stall;
  int nchk;           // checks since the state was set
  int64_t win_steps;  // steps at the start of the current coherence window (-1: none)
  double coherence;   // last full window: drift per step over it / the last step's change
};

// lbm_aux.hip
hipError_t decide_domains(const int *tile_begin, const int *tile_end, const double *partials,
                          void *state, int *active, int *n_active, int ndom, double tol,
                          int stall_checks, int steps, hipStream_t s);
hipError_t add_domain_steps(const int *active, void *state, int ndom, int64_t n, hipStream_t s);

const LatticeOps &ops_d2q9();
const LatticeOps &ops_d3q19();
const LatticeOps &ops_d3q27();
const LatticeOps &ops_d3q39();

// Launcher table of an lbm_lattice value (0 D2Q9, 1 D3Q19, 3 D3Q39, else D3Q27).
inline const LatticeOps &ops_for(int lattice) {
  switch (lattice) {
    case 0: return ops_d2q9();
    case 1: return ops_d3q19();
    case 3: return ops_d3q39();
    default: return ops_d3q27();
  }
}

// Error reporting shared by the runtime units (lbm_runtime.hip): records the message
// for lbm_last_error() and returns status.
int set_error(int status, const char *fmt, ...);

inline dim3 grid_of(const LaunchDesc &d) {
  return dim3((d.geo.nx + d.bx - 1) / d.bx, (d.geo.ny + d.by - 1) / d.by, d.geo.nz);
}

}  // namespace lbm
