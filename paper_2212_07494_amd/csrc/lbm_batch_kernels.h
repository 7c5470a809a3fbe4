// Kernels of the batched engine: many independent domains, one persistent launch per
// step.
//
// Layout: the domains' populations are packed one domain after another in each of the
// two population buffers (domain d occupies Q N_d values starting at element base_d, in
// the single-lattice layout of pop_slot); velocities recorded for the residual are packed the same way (D
// planes per domain); force tables / fields are packed into one table buffer.
//
// Work decomposition: a flattened table of tiles, each tile = one 256-thread workgroup
// of one domain (tbx x tby nodes of one z slice, tbx = 64, 128 or 256).  A fixed grid of
// workgroups (a few per compute unit) walks the table with a stride of the grid size,
// so domains of any size share the machine evenly; tiles of inactive (converged)
// domains are skipped after reading one flag.
#pragma once

#include "lbm_kernels.h"

namespace lbm {

struct BatchDom {
  int64_t base;   // population offset (elements) of plane 0, on a 128-byte boundary
  int64_t ps;     // plane stride: nx ny rounded up to 128 bytes
  int64_t ubase;  // offset of the recorded-velocity planes
  int64_t goff;   // offset of the force table / field in the table buffer
  int nx, ny, nz, N;
  int wall[3];
  int gaxis;      // 0, 1, 2: profile along that axis; -1: uniform (3 values); 3: full field
  int gn;         // profile length
  int tbx_log2;   // tile width 2^tbx_log2, height 256 >> tbx_log2; -1: linear tiles
  int tile_begin, tile_end;
  double c0, c1;  // collision coefficients (see StepArgs)
};

// A tile: the block of nodes (x0.., y0..) of layer z, or for linear tiles (tbx_log2 -1)
// the 256 nodes from offset x0 within layer z.
struct BatchTile {
  int dom, x0, y0, z;
};

// This lane's node of a tile; false if it lies beyond the domain.
__device__ __forceinline__ bool tile_xy(const BatchTile &t, const BatchDom &dm, int &x, int &y) {
  if (dm.tbx_log2 < 0) {
    const int r = t.x0 + (int)threadIdx.x;
    if (r >= dm.nx * dm.ny) return false;
    y = r / dm.nx;
    x = r - y * dm.nx;
    return true;
  }
  x = t.x0 + (threadIdx.x & ((1 << dm.tbx_log2) - 1));
  y = t.y0 + (threadIdx.x >> dm.tbx_log2);
  return x < dm.nx && y < dm.ny;
}

// Whether no node of the tile can bounce back (fast_block over the rows it covers).
template <class S>
__device__ __forceinline__ bool tile_fast(const BatchTile &t, const BatchDom &dm,
                                          const Geom &geo) {
  if (dm.tbx_log2 < 0) {
    const int last = min(t.x0 + 255, dm.nx * dm.ny - 1);
    return fast_block<S>(geo, 0, dm.nx - 1, t.x0 / dm.nx, last / dm.nx, t.z);
  }
  return fast_block<S>(geo, t.x0, t.x0 + (1 << dm.tbx_log2) - 1, t.y0,
                       t.y0 + (256 >> dm.tbx_log2) - 1, t.z);
}

template <class T>
__device__ __forceinline__ void batch_force(const T *__restrict__ gbuf, const BatchDom &dm, int x,
                                            int y, int z, int node, int D, T (&g)[3]) {
  const T *tab = gbuf + dm.goff;
  if (dm.gaxis == 3) {
    for (int a = 0; a < 3; ++a) g[a] = (a < D) ? tab[(int64_t)a * dm.N + node] : T(0);
  } else {
    const int c = dm.gaxis == 0 ? x : (dm.gaxis == 1 ? y : (dm.gaxis == 2 ? z : 0));
    for (int a = 0; a < 3; ++a) g[a] = (a < D) ? tab[a * dm.gn + c] : T(0);
  }
}

// The tiles a persistent workgroup walks.  Workgroups are dispatched to the chip's
// XCDs round-robin (workgroup b on XCD b mod kXcds) and each XCD has its own L2, while
// neighbouring tiles share cache lines through their +-1 pulls: so each XCD takes one
// contiguous part of the tile table (equal counts), which its own workgroups walk in turn.
// A grid that is not a multiple of kXcds falls back to a plain stride over the table.
struct TileWalk {
  int t, end, stride;
};
__device__ __forceinline__ TileWalk tile_walk(int ntiles) {
  const int G = gridDim.x, b = blockIdx.x;
  if (G % kXcds) return {b, ntiles, G};
  const int x = b % kXcds;
  const int lo = (int)((int64_t)ntiles * x / kXcds);
  const int hi = (int)((int64_t)ntiles * (x + 1) / kXcds);
  return {lo + b / kXcds, hi, G / kXcds};
}

__device__ __forceinline__ Geom batch_geom(const BatchDom &dm) {
  Geom geo;
  geo.nx = dm.nx;
  geo.ny = dm.ny;
  geo.nz = dm.nz;
  geo.N = dm.N;
  geo.ps = dm.ps;
  for (int a = 0; a < 3; ++a) geo.wall[a] = dm.wall[a];
  geo.smask = nullptr;  // batched domains have no solid nodes
  return geo;
}

template <class L, int COLL, class S, class T, int MEM>
__global__ void __launch_bounds__(256)
    batch_step_kernel(const S *__restrict__ fin, S *__restrict__ fout, const T *__restrict__ gbuf,
                      const BatchDom *__restrict__ doms, const BatchTile *__restrict__ tiles,
                      const int *__restrict__ active, int ntiles, T shift) {
  for (TileWalk w = tile_walk(ntiles); w.t < w.end; w.t += w.stride) {
    const int t = w.t;
    const BatchTile tile = tiles[t];
    if (!active[tile.dom]) continue;
    const BatchDom dm = doms[tile.dom];
    int x, y;
    const int z = tile.z;
    if (!tile_xy(tile, dm, x, y)) continue;
    const Geom geo = batch_geom(dm);
    const int node = (z * dm.ny + y) * dm.nx + x;
    T g[3];
    batch_force<T>(gbuf, dm, x, y, z, node, L::D, g);
    const bool fast = tile_fast<S>(tile, dm, geo);
    step_node<L, COLL, S, T, MEM>(fin + dm.base, fout + dm.base, geo, x, y, z, 0u, fast, g,
                                  shift, T(dm.c0), T(dm.c1));
  }
}

// Residual monitor over the tiles of active domains: physical u(t) of the current state
// (pulled), compared with the recorded u (mode 4) and/or recorded (modes 2 and 4).  At a
// check (mode 4) u(t) is also compared with uchk, the velocity at the start of the
// domain's coherence window; at a check that starts a window (every `window` checks)
// uchk takes u(t).  Writes per tile the BATCH_PARTIALS slots (lbm_internal.h).
template <class L, class S, class T>
__global__ void __launch_bounds__(256)
    batch_monitor_kernel(const S *__restrict__ f, const T *__restrict__ gbuf,
                         const BatchDom *__restrict__ doms, const BatchTile *__restrict__ tiles,
                         const int *__restrict__ active, int ntiles, T shift,
                         T *__restrict__ urec, T *__restrict__ uchk,
                         const DomState *__restrict__ st, int window, int mode,
                         double *__restrict__ partials) {
  __shared__ double red[4][BATCH_PARTIALS];
  for (TileWalk w = tile_walk(ntiles); w.t < w.end; w.t += w.stride) {
    const int t = w.t;
    const BatchTile tile = tiles[t];
    if (!active[tile.dom]) continue;
    const BatchDom dm = doms[tile.dom];
    int x = 0, y = 0;
    const int z = tile.z;
    double v[BATCH_PARTIALS] = {0.0, 0.0, 0.0, 0.0};
    if (tile_xy(tile, dm, x, y)) {
      const Geom geo = batch_geom(dm);
      const int node = (z * dm.ny + y) * dm.nx + x;
      T d[L::Q];
      const S *fd = f + dm.base;
      static_for<L::Q>([&](auto I) {
        constexpr int i = decltype(I)::value;
        d[i] = T(fd[pull_slot<L, i>(x, y, z, geo, 0u)]);
      });
      T g[3];
      batch_force<T>(gbuf, dm, x, y, z, node, L::D, g);
      const Macro<T> M = macroscopic<L>(d, shift, g);
      T *ur = urec + dm.ubase;
      T *uk = uchk + dm.ubase;
      const bool starts = st[tile.dom].nchk % window == 0;
      for (int c = 0; c < L::D; ++c) {
        const int64_t o = (int64_t)c * dm.N + node;
        const double uc = double(M.u[c]);
        v[BP_U2] += uc * uc;
        if (mode & MOM_COMPARE) {
          const double dd = uc - double(ur[o]);
          v[BP_DU2] += dd * dd;
          const double dk = uc - double(uk[o]);
          v[BP_DUK2] += dk * dk;
          if (starts) uk[o] = M.u[c];
        }
        ur[o] = M.u[c];
      }
      v[BP_BAD] = (isfinite(v[BP_U2]) && isfinite(double(M.rho))) ? 0.0 : 1.0;
    }
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    for (int s = 0; s < BATCH_PARTIALS; ++s) {
      const double r = wave_sum(v[s]);
      if (lane == 0) red[wave][s] = r;
    }
    __syncthreads();
    if (threadIdx.x < BATCH_PARTIALS) {
      const int s = threadIdx.x;
      partials[(int64_t)t * BATCH_PARTIALS + s] =
          ((red[0][s] + red[1][s]) + red[2][s]) + red[3][s];
    }
    __syncthreads();
  }
}

}  // namespace lbm
