// Internal interface between the C-ABI runtime (lbm_runtime.hip) and the per-lattice
// kernel units (lbm_d2q9.hip, lbm_d3q19.hip, lbm_d3q27.hip), which are compiled
// separately so the heavily unrolled kernels build in parallel.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace lbm {

struct GeomDesc {
  int nx, ny, nz, N;
  int wall[3];
};

// One launch of a lattice kernel.  Coefficients are binary64 on the host and are
// rounded once to the arithmetic type of the storage mode.
struct LaunchDesc {
  int coll;      // 0 BGK, 1 SMRT
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
  int bx, by;        // block shape (bx * by <= 256, bx a multiple of 64)
  int variant;       // memory-access variant of the step kernel (MEM_*)
};

struct LatticeOps {
  int D, Q;
  hipError_t (*step)(const LaunchDesc &, hipStream_t);
  hipError_t (*init)(const LaunchDesc &, const double *rho, const double *u, double rho0,
                     hipStream_t);
  hipError_t (*gather)(const LaunchDesc &, const int64_t *nodes, int64_t nn, double *out,
                       hipStream_t);
  hipError_t (*scatter)(const LaunchDesc &, const double *in, hipStream_t);
  hipError_t (*moments)(const LaunchDesc &, double *rho, double *u, void *uprev, int mode,
                        double *partials, hipStream_t);
};

const LatticeOps &ops_d2q9();
const LatticeOps &ops_d3q19();
const LatticeOps &ops_d3q27();

inline dim3 grid_of(const LaunchDesc &d) {
  return dim3((d.geo.nx + d.bx - 1) / d.bx, (d.geo.ny + d.by - 1) / d.by, d.geo.nz);
}

}  // namespace lbm
