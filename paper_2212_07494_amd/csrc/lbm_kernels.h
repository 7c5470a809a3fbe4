// Kernels of the forced lattice-Boltzmann library (gfx950).
//
// Memory layout in HBM: one slab per z layer, each holding that layer's Q population
// planes of nx ny values back to back (pop_slot; node index n = (z ny + y) nx + x,
// x fastest).  Two such buffers alternate between steps.  The buffer a step writes
// holds, at slot (i, x), the post-collision population f*_i(x, t); the next step pulls
// slot (i, x - e_i) into node x (or, when x - e_i lies beyond a wall or is solid, slot
// (opp(i), x): halfway bounce-back).  Reads of each population plane are therefore
// row-contiguous with a one-element x offset, writes are aligned and contiguous: every
// wavefront moves 64 consecutive values per plane in each direction.
//
// A thread owns one node.  Blocks tile (x, y) rows with blockDim = (bx, by), one z
// slice per blockIdx.z.  Each node is read and written once per step and no value is
// reused by another block, so the block order carries no cache locality to exploit.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "lbm_internal.h"
#include "lbm_node.h"

namespace lbm {

enum { GK_PROFILE = 0, GK_FIELD = 1 };

// Workgroups are dispatched to the chip's XCDs round-robin (workgroup b on XCD b mod
// kXcds), and each XCD has its own L2.
constexpr int kXcds = 8;

// XCD-contiguous placement of a grid's nb blocks: block b (in dispatch order) takes the
// logical block start(XCD) + b / kXcds, so each XCD works through one contiguous stretch
// of the lattice (whole row segments, rows and layers), and the lines that neighbouring
// blocks share -- the x-shifted pulls across a block's edges, the rows and layers beside
// it -- are fetched into one L2 rather than two.  The XCDs take nb / kXcds blocks each,
// the first nb mod kXcds one more: a bijection of [0, nb) for any nb.
__device__ __forceinline__ int64_t xcd_block(int64_t b, int64_t nb) {
  const int64_t q = nb / kXcds, r = nb % kXcds, x = b % kXcds;
  return x * q + (x < r ? x : r) + b / kXcds;
}

struct Geom {
  int nx, ny, nz, N;
  int64_t ps;  // plane stride: elements from one population plane to the next (>= nx ny)
  int wall[3];
  // Solid nodes (NULL: none): per node, bit i = the pull source of population i is solid,
  // bit 31 = the node itself is solid.  Lattices of more than 31 populations (D3Q39) run
  // without solid nodes.
  const uint32_t *smask;
};

__device__ __forceinline__ uint32_t node_mask(const Geom &G, int node) {
  return G.smask ? G.smask[node] : 0u;
}

template <class T>
struct ForceRef {
  const T *tab;  // profile: 3 x n (component-major); field: 3 planes of N
  int axis;      // profile: 0, 1, 2, or -1 (uniform, n = 1)
  int n;
  T scale;       // s(t)
  // s(t) from device memory instead (graph replays): sdev[*sctr + sj], rounded to T as
  // the host value would be
  const double *sdev;
  const int64_t *sctr;
  int sj;
};

// Memory-access variants of the step (chosen at run time by the tuner):
//   MEM_PLAIN  ordinary loads and stores;
//   MEM_NTST   non-temporal stores (the written buffer is not re-read this step);
//   MEM_NTALL  non-temporal loads and stores.
enum { MEM_PLAIN = 0, MEM_NTST = 1, MEM_NTALL = 2, MEM_VARIANTS = 3 };

template <class S, class T>
__device__ __forceinline__ T load_as(const S *p) {
  return T(*p);
}
template <class S, class T>
__device__ __forceinline__ S store_as(T v) {
  return S(v);
}
template <int MEM, class S, class T>
__device__ __forceinline__ T load_v(const S *p) {
  if constexpr (MEM == MEM_NTALL)
    return T(__builtin_nontemporal_load(p));
  else
    return T(*p);
}
template <int MEM, class S, class T>
__device__ __forceinline__ void store_v(S *p, T v) {
  if constexpr (MEM == MEM_NTST || MEM == MEM_NTALL)
    __builtin_nontemporal_store(S(v), p);
  else
    *p = S(v);
}

// Storage slot of population i at node (x, y, z).  Layout: one slab per z layer holding
// the layer's Q planes back to back, slot = (z Q + i) ps + y nx + x, with the plane stride
// ps = nx ny for a single lattice and nx ny rounded up to 128 bytes in the batched
// engine (so every plane of every domain starts on a cache line).  Compared with Q
// planes of the whole grid it keeps every access of a workgroup (its layer and the two
// beside it) inside 3 Q nx ny contiguous values (a probe of the access pattern alone
// streamed 5% faster this way).
template <class L>
__device__ __forceinline__ int64_t pop_slot(int i, int x, int y, int z, const Geom &G) {
  return ((int64_t)z * L::Q + i) * G.ps + (y * G.nx + x);
}

// Start of population i's plane in layer z.  z comes from blockIdx.z, so the address is
// the same across the workgroup and lives in scalar registers.
template <class L, class S>
__device__ __forceinline__ S *plane_ptr(S *f, int i, int z, const Geom &G) {
  return f + ((int64_t)z * L::Q + i) * G.ps;
}

// Element o of a plane through a 32-bit byte offset (the scalar-base + vector-offset
// form of the memory instructions); needs nx ny sizeof(S) < 2^32 (fast_block).
template <class S>
__device__ __forceinline__ S *at_offset(S *plane, uint32_t o) {
  using B = std::conditional_t<std::is_const_v<S>, const char, char>;
  return reinterpret_cast<S *>(reinterpret_cast<B *>(plane) + o * (uint32_t)sizeof(S));
}

// Whether no pull of a workgroup covering x0..x1, y0..y1 of layer z can bounce back (no
// solid nodes, and the block keeps off the first and last index of every walled axis)
// and a plane's bytes fit 32 bits: then its pulls need no bounce-back test (any wrap is
// periodic) and address through at_offset.  Uniform across the workgroup.
template <class S>
__device__ __forceinline__ bool fast_block(const Geom &G, int x0, int x1, int y0, int y1,
                                           int z) {
  if (G.smask != nullptr || (uint64_t)G.ps * sizeof(S) >= (1ull << 32)) return false;
  if (G.wall[0] && (x0 == 0 || x1 >= G.nx - 1)) return false;
  if (G.wall[1] && (y0 == 0 || y1 >= G.ny - 1)) return false;
  if (G.wall[2] && (z == 0 || z >= G.nz - 1)) return false;
  return true;
}

// The pull of population i where no bounce-back can occur (fast_block): (i, x - e_i),
// wrapped periodically (one wrap: every extent is at least max |e_ia|).
template <class L, int i, class S>
__device__ __forceinline__ const S *pull_ptr_periodic(const S *f, int x, int y, int z,
                                                      const Geom &G) {
  constexpr int ex = L::E[i][0], ey = L::E[i][1], ez = L::E[i][2];
  int xs = x - ex, ys = y - ey, zs = z - ez;
  if constexpr (ex != 0) xs = (xs < 0) ? xs + G.nx : ((xs >= G.nx) ? xs - G.nx : xs);
  if constexpr (ey != 0) ys = (ys < 0) ? ys + G.ny : ((ys >= G.ny) ? ys - G.ny : ys);
  if constexpr (ez != 0) zs = (zs < 0) ? zs + G.nz : ((zs >= G.nz) ? zs - G.nz : zs);
  return at_offset(plane_ptr<L>(f, i, zs, G), (uint32_t)(ys * G.nx + xs));
}

// Slot that node (x, y, z) pulls population i from: (i, x - e_i) with periodic wrap,
// or (opp(i), x) when x - e_i crosses a wall face or is a solid node (halfway
// bounce-back); sm is the node's solid mask word.
template <class L, int i>
__device__ __forceinline__ int64_t pull_slot(int x, int y, int z, const Geom &G, uint32_t sm) {
  constexpr int ex = L::E[i][0], ey = L::E[i][1], ez = L::E[i][2];
  int xs = x - ex, ys = y - ey, zs = z - ez;
  bool bounce = false;
  if constexpr (i < 31) bounce = (sm >> i) & 1u;  // the source node is solid
  if constexpr (ex != 0) {
    const bool o = (xs < 0) | (xs >= G.nx);
    bounce |= o & (G.wall[0] != 0);
    xs = (xs < 0) ? xs + G.nx : ((xs >= G.nx) ? xs - G.nx : xs);
  }
  if constexpr (ey != 0) {
    const bool o = (ys < 0) | (ys >= G.ny);
    bounce |= o & (G.wall[1] != 0);
    ys = (ys < 0) ? ys + G.ny : ((ys >= G.ny) ? ys - G.ny : ys);
  }
  if constexpr (ez != 0) {
    const bool o = (zs < 0) | (zs >= G.nz);
    bounce |= o & (G.wall[2] != 0);
    zs = (zs < 0) ? zs + G.nz : ((zs >= G.nz) ? zs - G.nz : zs);
  }
  return bounce ? pop_slot<L>(L::OPP[i], x, y, z, G) : pop_slot<L>(i, xs, ys, zs, G);
}

template <class T, int GK>
__device__ __forceinline__ void load_force(const ForceRef<T> &F, int x, int y, int z, int node,
                                           int N, int D, T (&g)[3]) {
  const T scale = F.sdev ? T(F.sdev[*F.sctr + F.sj]) : F.scale;
  if constexpr (GK == GK_FIELD) {
    for (int a = 0; a < 3; ++a) g[a] = (a < D) ? F.tab[(int64_t)a * N + node] * scale : T(0);
  } else {
    const int c = F.axis == 0 ? x : (F.axis == 1 ? y : (F.axis == 2 ? z : 0));
    for (int a = 0; a < 3; ++a) g[a] = (a < D) ? F.tab[a * F.n + c] * scale : T(0);
  }
}

template <class T>
struct StepArgs {
  const void *fin;
  void *fout;
  Geom geo;
  ForceRef<T> force;
  T shift;
  T c0, c1;  // BGK: omega, 1 - omega/2;  SMRT: q2, q3
  T c2;      // SMRT: coefficient of the third-order force term (0 = off); RMRT: h2
  T c3;      // RMRT: h3; SMRT: (q_bulk - q2)/D (0 = one rate at order 2)
  T c4;      // SMRT: (q_31 - q3)/2 (0 = one rate at order 3)
  int fast_ok;  // 1: fast_block workgroups take the scalar-base path
  int xcd;      // 1: XCD-contiguous block placement (xcd_block), 0: dispatch order
};

// One node of the fused step: pull the populations (periodic wrap or halfway
// bounce-back), collide with the force, store at the node's own slots.
template <class L, int COLL, class S, class T, int MEM>
__device__ __forceinline__ void step_node(const S *__restrict__ fin, S *__restrict__ fout,
                                          const Geom &geo, int x, int y, int z,
                                          uint32_t sm, bool fast, const T (&g)[3], T shift,
                                          T c0, T c1, T c2 = T(0), T c3 = T(0), T c4 = T(0)) {
  T d[L::Q];
  if (fast) {
    static_for<L::Q>([&](auto I) {
      constexpr int i = decltype(I)::value;
      d[i] = load_v<MEM, S, T>(pull_ptr_periodic<L, i>(fin, x, y, z, geo));
    });
  } else {
    static_for<L::Q>([&](auto I) {
      constexpr int i = decltype(I)::value;
      d[i] = load_v<MEM, S, T>(fin + pull_slot<L, i>(x, y, z, geo, sm));
    });
  }
  if constexpr (COLL == 0) {
    collide_bgk<L>(d, shift, g, BGKCoef<T>{c0, c1});
  } else {
    const SMRTCoef<T> sc{c0, c1, c2, c3, c4};
    if constexpr (COLL == 1)
      collide_smrt<L, false, T, 0, false>(d, shift, g, sc);
    else if constexpr (COLL == 7)
      collide_smrt<L, false, T, 0>(d, shift, g, sc);
    else if constexpr (COLL == 3)
      collide_smrt<L, true, T, 0>(d, shift, g, sc);
    else if constexpr (COLL == 4)
      collide_smrt<L, false, T, 3>(d, shift, g, sc);
    else if constexpr (COLL == 5)
      collide_smrt<L, false, T, 4>(d, shift, g, sc);
    else if constexpr (COLL == 6)
      collide_smrt<L, true, T, 3>(d, shift, g, sc);
    else
      collide_rmrt<L>(d, shift, g, RMRTCoef<T>{c0, c1, c2, c3});
  }
  if (fast) {
    const uint32_t o = (uint32_t)(y * geo.nx + x);
    static_for<L::Q>([&](auto I) {
      constexpr int i = decltype(I)::value;
      store_v<MEM, S, T>(at_offset(plane_ptr<L>(fout, i, z, geo), o), d[i]);
    });
  } else {
    static_for<L::Q>([&](auto I) {
      constexpr int i = decltype(I)::value;
      store_v<MEM, S, T>(fout + pop_slot<L>(i, x, y, z, geo), d[i]);
    });
  }
}

template <class L, int COLL, class S, class T, int GK, int MEM>
__global__ void __launch_bounds__(256) step_kernel(StepArgs<T> a) {
  // the block's place in the lattice (uniform across the workgroup)
  int bxi = blockIdx.x, byi = blockIdx.y, bzi = blockIdx.z;
  if (a.xcd) {
    const int64_t nxy = (int64_t)gridDim.x * gridDim.y;
    const int64_t b = blockIdx.x + (int64_t)gridDim.x * blockIdx.y + nxy * blockIdx.z;
    const int64_t t = xcd_block(b, nxy * gridDim.z);
    bzi = (int)(t / nxy);
    byi = (int)((t % nxy) / gridDim.x);
    bxi = (int)(t % gridDim.x);
  }
  const int x = bxi * blockDim.x + threadIdx.x;
  const int y = byi * blockDim.y + threadIdx.y;
  const int z = bzi;
  if (x >= a.geo.nx || y >= a.geo.ny) return;
  const int node = (z * a.geo.ny + y) * a.geo.nx + x;
  const uint32_t sm = node_mask(a.geo, node);
  if (sm & SOLID_NODE) return;  // no fluid here: nothing pulls from its slots
  T g[3];
  load_force<T, GK>(a.force, x, y, z, node, a.geo.N, L::D, g);
  const int x0 = bxi * blockDim.x, y0 = byi * blockDim.y;
  const bool fast = a.fast_ok && fast_block<S>(a.geo, x0, x0 + (int)blockDim.x - 1, y0,
                                               y0 + (int)blockDim.y - 1, z);
  step_node<L, COLL, S, T, MEM>(static_cast<const S *>(a.fin), static_cast<S *>(a.fout), a.geo,
                                x, y, z, sm, fast, g, a.shift, a.c0, a.c1, a.c2, a.c3,
                                a.c4);
}

// Initial state: compute f-bar(x, 0) at every node and place each population in the
// slot the first step will pull it from.
template <class L, int COLL, class S, class T, int GK>
__global__ void __launch_bounds__(256) init_kernel(StepArgs<T> a, const double *rho,
                                                   const double *u, int has_rho, int has_u,
                                                   T rho0, const double *pi) {
  const int x = blockIdx.x * blockDim.x + threadIdx.x;
  const int y = blockIdx.y * blockDim.y + threadIdx.y;
  const int z = blockIdx.z;
  if (x >= a.geo.nx || y >= a.geo.ny) return;
  const int node = (z * a.geo.ny + y) * a.geo.nx + x;
  const uint32_t sm = node_mask(a.geo, node);
  if (sm & SOLID_NODE) return;
  const int N = a.geo.N;
  T r = has_rho ? T(rho[node]) : rho0;
  T uu[3];
  for (int c = 0; c < 3; ++c) uu[c] = (has_u && c < L::D) ? T(u[(int64_t)c * N + node]) : T(0);
  T g[3];
  load_force<T, GK>(a.force, x, y, z, node, N, L::D, g);
  T out[L::Q];
  init_node<L, T, COLL>(r, uu, g, a.shift, out);
  if (pi) {
    // A non-equilibrium second moment Pi (planes xx, yy, zz, xy, xz, yz): the Hermite
    // term w_i (e_i e_i - c_s^2 I) : Pi / (2 c_s^4), which has no mass or momentum.
    T P[6];
    for (int c = 0; c < 6; ++c) P[c] = T(pi[(int64_t)c * N + node]);
    const T c2 = T(L::CS2N) / T(L::CS2D);
    static_for<L::Q>([&](auto I) {
      constexpr int i = decltype(I)::value;
      constexpr int ex = L::E[i][0], ey = L::E[i][1], ez = L::E[i][2];
      const T q = ((T(ex * ex) - c2) * P[0] + (T(ey * ey) - c2) * P[1] +
                   (T(ez * ez) - c2) * P[2]) +
                  T(2) * ((T(ex * ey) * P[3] + T(ex * ez) * P[4]) + T(ey * ez) * P[5]);
      out[i] = out[i] + Tab<L, T>::w(i) * (T(0.5 * L::ICS2 * L::ICS2) * q);
    });
  }
  S *__restrict__ f = static_cast<S *>(a.fout);
  static_for<L::Q>([&](auto I) {
    constexpr int i = decltype(I)::value;
    f[pull_slot<L, i>(x, y, z, a.geo, sm)] = store_as<S, T>(out[i]);
  });
}

// Pre-collision populations at selected nodes (or all nodes), as stored, in binary64.
template <class L, class S>
__global__ void __launch_bounds__(256) gather_kernel(const S *__restrict__ f, Geom geo,
                                                     const int64_t *nodes, int64_t nn,
                                                     double *__restrict__ out) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= nn) return;
  const int node = nodes ? (int)nodes[j] : (int)j;
  const int x = node % geo.nx;
  const int y = (node / geo.nx) % geo.ny;
  const int z = node / (geo.nx * geo.ny);
  const uint32_t sm = node_mask(geo, node);
  static_for<L::Q>([&](auto I) {
    constexpr int i = decltype(I)::value;
    out[(int64_t)i * nn + j] = double(f[pull_slot<L, i>(x, y, z, geo, sm)]);
  });
}

template <class L, class S>
__global__ void __launch_bounds__(256) scatter_kernel(S *__restrict__ f, Geom geo,
                                                      const double *__restrict__ in) {
  const int64_t node = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (node >= geo.N) return;
  const int n = (int)node;
  const int x = n % geo.nx;
  const int y = (n / geo.nx) % geo.ny;
  const int z = n / (geo.nx * geo.ny);
  const uint32_t sm = node_mask(geo, n);
  if (sm & SOLID_NODE) return;
  static_for<L::Q>([&](auto I) {
    constexpr int i = decltype(I)::value;
    const double v = in[(int64_t)i * geo.N + n];
    if constexpr (std::is_same<S, double>::value)
      f[pull_slot<L, i>(x, y, z, geo, sm)] = v;
    else
      f[pull_slot<L, i>(x, y, z, geo, sm)] = S(float(v));
  });
}

// State from a sum of Fourier waves about rest: f-bar_i(x) = w_i rho0 + sum_w
// Re[A_wi e^{i theta_w(x)}], theta_w(x) = 2 pi sum_a k_wa x_a / n_a + phase_w, stored as
// f-bar_i - w_i shift, rounded once from binary64.  k_wa x_a is reduced modulo n_a in
// integers first, so the angle stays within a few periods at any size.  amp holds the
// (re, im) pairs of wave w's Q amplitudes at 2 (w Q + i).
template <class L, class S>
__global__ void __launch_bounds__(256) waves_kernel(S *__restrict__ f, Geom geo, int nw,
                                                    const int *__restrict__ k,
                                                    const double *__restrict__ phase,
                                                    const double *__restrict__ amp,
                                                    double base) {
  const int64_t node = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (node >= geo.N) return;
  const int n = (int)node;
  const int x = n % geo.nx;
  const int y = (n / geo.nx) % geo.ny;
  const int z = n / (geo.nx * geo.ny);
  const uint32_t sm = node_mask(geo, n);
  if (sm & SOLID_NODE) return;
  const double two_pi = 6.283185307179586;
  double acc[L::Q];
  for (int i = 0; i < L::Q; ++i) acc[i] = 0.0;
  for (int w = 0; w < nw; ++w) {
    const int mx = (int)(((int64_t)k[3 * w] * x) % geo.nx);
    const int my = (int)(((int64_t)k[3 * w + 1] * y) % geo.ny);
    const int mz = (int)(((int64_t)k[3 * w + 2] * z) % geo.nz);
    const double t = (double(mx) / geo.nx + double(my) / geo.ny) + double(mz) / geo.nz;
    double s, c;
    sincos(two_pi * t + phase[w], &s, &c);
    const double *a = amp + (int64_t)2 * L::Q * w;
    static_for<L::Q>([&](auto I) {
      constexpr int i = decltype(I)::value;
      acc[i] = acc[i] + (a[2 * i] * c - a[2 * i + 1] * s);
    });
  }
  static_for<L::Q>([&](auto I) {
    constexpr int i = decltype(I)::value;
    f[pull_slot<L, i>(x, y, z, geo, sm)] = S(Tab<L, double>::w(i) * base + acc[i]);
  });
}

// ---- monitors -------------------------------------------------------------------------
// Block partials use the monitor slots of lbm_internal.h (MON_*).
enum { MOM_WRITE = 1, MOM_RECORD = 2, MOM_COMPARE = 4 };

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}
__device__ __forceinline__ double wave_max(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
  return v;
}

// Density and physical velocity of the current state (pulled), optionally written out
// (binary64), recorded into uprev, and reduced into per-block monitor partials.
template <class L, class S, class T, int GK>
__global__ void __launch_bounds__(256) moments_kernel(StepArgs<T> a, double *rho_out,
                                                      double *u_out, T *uprev, int mode,
                                                      double *partials) {
  const int x = blockIdx.x * blockDim.x + threadIdx.x;
  const int y = blockIdx.y * blockDim.y + threadIdx.y;
  const int z = blockIdx.z;
  const bool inside = (x < a.geo.nx) && (y < a.geo.ny);
  const int node = (z * a.geo.ny + y) * a.geo.nx + x;
  const uint32_t sm = inside ? node_mask(a.geo, node) : 0u;
  const bool live = inside && !(sm & SOLID_NODE);
  double v[MON_SLOTS];
  for (int s = 0; s < MON_SLOTS; ++s) v[s] = 0.0;
  if (inside && !live && (mode & MOM_WRITE)) {  // solid node: no fluid
    if (rho_out) rho_out[node] = 0.0;
    if (u_out)
      for (int c = 0; c < L::D; ++c) u_out[(int64_t)c * a.geo.N + node] = 0.0;
  }
  if (live) {
    const int N = a.geo.N;
    const S *__restrict__ fin = static_cast<const S *>(a.fin);
    T d[L::Q];
    static_for<L::Q>([&](auto I) {
      constexpr int i = decltype(I)::value;
      d[i] = load_as<S, T>(fin + pull_slot<L, i>(x, y, z, a.geo, sm));
    });
    T g[3];
    load_force<T, GK>(a.force, x, y, z, node, N, L::D, g);
    const Macro<T> M = macroscopic<L>(d, a.shift, g);
    if (mode & MOM_WRITE) {
      if (rho_out) rho_out[node] = double(M.rho);
      if (u_out)
        for (int c = 0; c < L::D; ++c) u_out[(int64_t)c * N + node] = double(M.u[c]);
    }
    const double r = double(M.rho);
    double u2 = 0, du2 = 0;
    for (int c = 0; c < L::D; ++c) {
      const double uc = double(M.u[c]);
      u2 += uc * uc;
      v[MON_MX + c] = r * uc;
      v[MON_JX + c] = double(M.j[c]);
      if (mode & MOM_COMPARE) {
        const double dd = uc - double(uprev[(int64_t)c * N + node]);
        du2 += dd * dd;
      }
      if (mode & (MOM_RECORD | MOM_COMPARE)) uprev[(int64_t)c * N + node] = M.u[c];
    }
    v[MON_MASS] = r;
    v[MON_DU2] = du2;
    v[MON_U2] = u2;
    v[MON_UMAX] = sqrt(u2);
    const bool bad = !isfinite(r) || !isfinite(u2);
    v[MON_BAD] = bad ? 1.0 : 0.0;
    if (bad) v[MON_UMAX] = 0;
  }
  if (!partials) return;
  __shared__ double red[4][MON_SLOTS];
  const int tid = threadIdx.y * blockDim.x + threadIdx.x;
  const int wave = tid >> 6, lane = tid & 63;
  for (int s = 0; s < MON_SLOTS; ++s) {
    const double t = (s == MON_UMAX) ? wave_max(v[s]) : wave_sum(v[s]);
    if (lane == 0) red[wave][s] = t;
  }
  __syncthreads();
  if (tid < MON_SLOTS) {
    const int nw = (blockDim.x * blockDim.y + 63) >> 6;
    double acc = red[0][tid];
    for (int w = 1; w < nw; ++w) acc = (tid == MON_UMAX) ? fmax(acc, red[w][tid]) : acc + red[w][tid];
    const int64_t b = ((int64_t)blockIdx.z * gridDim.y + blockIdx.y) * gridDim.x + blockIdx.x;
    partials[b * MON_SLOTS + tid] = acc;
  }
}

}  // namespace lbm
