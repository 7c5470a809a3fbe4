// Launchers of one lattice's kernels; included once per lattice unit with LBM_LAT set
// to the lattice struct (D2Q9, D3Q19, D3Q27, D3Q39) and LBM_OPS to the exported table
// name.  The batched engine is built for the lattices of at most 27 populations.
#pragma once

#include "lbm_batch_kernels.h"
#include "lbm_internal.h"
#include "lbm_kernels.h"

namespace lbm {
namespace impl {

template <class T>
inline StepArgs<T> make_args(const LaunchDesc &d) {
  StepArgs<T> a;
  a.fin = d.fin;
  a.fout = d.fout;
  a.geo.nx = d.geo.nx;
  a.geo.ny = d.geo.ny;
  a.geo.nz = d.geo.nz;
  a.geo.N = d.geo.N;
  a.geo.ps = d.geo.ps;
  for (int c = 0; c < 3; ++c) a.geo.wall[c] = d.geo.wall[c];
  a.geo.smask = d.geo.smask;
  a.force.tab = static_cast<const T *>(d.gtab);
  a.force.axis = d.g_axis;
  a.force.n = d.g_n;
  a.force.scale = T(d.gscale);
  a.force.sdev = d.gs_dev;
  a.force.sctr = d.gs_ctr;
  a.force.sj = d.gs_j;
  a.shift = T(d.shift);
  a.c0 = T(d.c0);
  a.c1 = T(d.c1);
  a.c2 = T(d.c2);
  a.c3 = T(d.c3);
  a.c4 = T(d.c4);
  a.fast_ok = d.fast_ok;
  a.xcd = d.xcd;
  return a;
}

inline Geom geom_of(const LaunchDesc &d) {
  Geom g;
  g.nx = d.geo.nx;
  g.ny = d.geo.ny;
  g.nz = d.geo.nz;
  g.N = d.geo.N;
  g.ps = d.geo.ps;
  for (int c = 0; c < 3; ++c) g.wall[c] = d.geo.wall[c];
  g.smask = d.geo.smask;
  return g;
}

// storage mode -> (storage type S, arithmetic type T)
template <class F>
inline hipError_t with_types(int storage, F &&f) {
  switch (storage) {
    case 0: return f((double *)nullptr, (double *)nullptr);
    case 1:
    case 2: return f((float *)nullptr, (float *)nullptr);
    case 3: return f((_Float16 *)nullptr, (float *)nullptr);
    default: return hipErrorInvalidValue;
  }
}

template <class L>
struct Ops {
  template <int COLL, class S, class T, int GK, int MEM>
  static hipError_t step_m(const LaunchDesc &d, hipStream_t s) {
    hipLaunchKernelGGL((step_kernel<L, COLL, S, T, GK, MEM>), grid_of(d), dim3(d.bx, d.by),
                       d.lds_pad, s, make_args<T>(d));
    return hipGetLastError();
  }
  template <int COLL, class S, class T, int GK>
  static hipError_t step_t(const LaunchDesc &d, hipStream_t s) {
    switch (d.variant) {
      case MEM_PLAIN: return step_m<COLL, S, T, GK, MEM_PLAIN>(d, s);
      case MEM_NTST: return step_m<COLL, S, T, GK, MEM_NTST>(d, s);
      case MEM_NTALL: return step_m<COLL, S, T, GK, MEM_NTALL>(d, s);
      default: return hipErrorInvalidValue;
    }
  }
  static hipError_t step(const LaunchDesc &d, hipStream_t s) {
    return with_types(d.storage, [&](auto *sp, auto *tp) -> hipError_t {
      using S = std::remove_pointer_t<decltype(sp)>;
      using T = std::remove_pointer_t<decltype(tp)>;
      if (d.coll == 0)
        return d.gk ? step_t<0, S, T, GK_FIELD>(d, s) : step_t<0, S, T, GK_PROFILE>(d, s);
      if (d.coll == 2)
        return d.gk ? step_t<2, S, T, GK_FIELD>(d, s) : step_t<2, S, T, GK_PROFILE>(d, s);
      if constexpr (L::ORD[L::NM - 1] > 4) {
        if (d.coll == 3)
          return d.gk ? step_t<3, S, T, GK_FIELD>(d, s) : step_t<3, S, T, GK_PROFILE>(d, s);
        if (d.coll == 6)
          return d.gk ? step_t<6, S, T, GK_FIELD>(d, s) : step_t<6, S, T, GK_PROFILE>(d, s);
      }
      if (d.coll == 4)
        return d.gk ? step_t<4, S, T, GK_FIELD>(d, s) : step_t<4, S, T, GK_PROFILE>(d, s);
      if (d.coll == 7)
        return d.gk ? step_t<7, S, T, GK_FIELD>(d, s) : step_t<7, S, T, GK_PROFILE>(d, s);
      if constexpr (L::NM == L::Q) {
        if (d.coll == 5)
          return d.gk ? step_t<5, S, T, GK_FIELD>(d, s) : step_t<5, S, T, GK_PROFILE>(d, s);
      }
      return d.gk ? step_t<1, S, T, GK_FIELD>(d, s) : step_t<1, S, T, GK_PROFILE>(d, s);
    });
  }
  template <int COLL, class S, class T, int GK>
  static hipError_t init_t(const LaunchDesc &d, const double *rho, const double *u,
                           double rho0, const double *pi, hipStream_t s) {
    hipLaunchKernelGGL((init_kernel<L, COLL, S, T, GK>), grid_of(d), dim3(d.bx, d.by), 0, s,
                       make_args<T>(d), rho, u, rho != nullptr, u != nullptr, T(rho0), pi);
    return hipGetLastError();
  }
  static hipError_t init(const LaunchDesc &d, const double *rho, const double *u, double rho0,
                         const double *pi, hipStream_t s) {
    return with_types(d.storage, [&](auto *sp, auto *tp) -> hipError_t {
      using S = std::remove_pointer_t<decltype(sp)>;
      using T = std::remove_pointer_t<decltype(tp)>;
      if (d.coll == 0)
        return d.gk ? init_t<0, S, T, GK_FIELD>(d, rho, u, rho0, pi, s)
                    : init_t<0, S, T, GK_PROFILE>(d, rho, u, rho0, pi, s);
      return d.gk ? init_t<1, S, T, GK_FIELD>(d, rho, u, rho0, pi, s)
                  : init_t<1, S, T, GK_PROFILE>(d, rho, u, rho0, pi, s);
    });
  }
  static void solid_words(const uint8_t *solid, int nx, int ny, int nz, const int wall[3],
                          uint32_t *out) {
    const int dims[3] = {nx, ny, nz};
    for (int z = 0; z < nz; ++z)
      for (int y = 0; y < ny; ++y)
        for (int x = 0; x < nx; ++x) {
          const int64_t n = ((int64_t)z * ny + y) * nx + x;
          uint32_t w = solid[n] ? SOLID_NODE : 0u;
          for (int i = 0; i < L::Q && i < 31; ++i) {
            int c[3] = {x - L::E[i][0], y - L::E[i][1], z - L::E[i][2]};
            bool across_wall = false;
            for (int a = 0; a < 3; ++a) {
              if (c[a] >= 0 && c[a] < dims[a]) continue;
              if (wall[a]) across_wall = true;
              c[a] = (c[a] + dims[a]) % dims[a];
            }
            if (!across_wall && solid[((int64_t)c[2] * ny + c[1]) * nx + c[0]]) w |= 1u << i;
          }
          out[n] = w;
        }
  }
  static hipError_t gather(const LaunchDesc &d, const int64_t *nodes, int64_t nn, double *out,
                           hipStream_t s) {
    if (nn <= 0) return hipSuccess;
    return with_types(d.storage, [&](auto *sp, auto *) -> hipError_t {
      using S = std::remove_pointer_t<decltype(sp)>;
      const unsigned blocks = (unsigned)((nn + 255) / 256);
      hipLaunchKernelGGL((gather_kernel<L, S>), dim3(blocks), dim3(256), 0, s,
                         static_cast<const S *>(d.fin), geom_of(d), nodes, nn, out);
      return hipGetLastError();
    });
  }
  static hipError_t scatter(const LaunchDesc &d, const double *in, hipStream_t s) {
    return with_types(d.storage, [&](auto *sp, auto *) -> hipError_t {
      using S = std::remove_pointer_t<decltype(sp)>;
      const unsigned blocks = (unsigned)((d.geo.N + 255) / 256);
      hipLaunchKernelGGL((scatter_kernel<L, S>), dim3(blocks), dim3(256), 0, s,
                         static_cast<S *>(d.fout), geom_of(d), in);
      return hipGetLastError();
    });
  }
  static hipError_t waves(const LaunchDesc &d, int nw, const int *k, const double *phase,
                          const double *amp, double base, hipStream_t s) {
    return with_types(d.storage, [&](auto *sp, auto *) -> hipError_t {
      using S = std::remove_pointer_t<decltype(sp)>;
      const unsigned blocks = (unsigned)((d.geo.N + 255) / 256);
      hipLaunchKernelGGL((waves_kernel<L, S>), dim3(blocks), dim3(256), 0, s,
                         static_cast<S *>(d.fout), geom_of(d), nw, k, phase, amp, base);
      return hipGetLastError();
    });
  }
  template <class S, class T, int GK>
  static hipError_t moments_t(const LaunchDesc &d, double *rho, double *u, void *uprev, int mode,
                              double *partials, hipStream_t s) {
    hipLaunchKernelGGL((moments_kernel<L, S, T, GK>), grid_of(d), dim3(d.bx, d.by), 0, s,
                       make_args<T>(d), rho, u, static_cast<T *>(uprev), mode, partials);
    return hipGetLastError();
  }
  static hipError_t moments(const LaunchDesc &d, double *rho, double *u, void *uprev, int mode,
                            double *partials, hipStream_t s) {
    return with_types(d.storage, [&](auto *sp, auto *tp) -> hipError_t {
      using S = std::remove_pointer_t<decltype(sp)>;
      using T = std::remove_pointer_t<decltype(tp)>;
      return d.gk ? moments_t<S, T, GK_FIELD>(d, rho, u, uprev, mode, partials, s)
                  : moments_t<S, T, GK_PROFILE>(d, rho, u, uprev, mode, partials, s);
    });
  }
  template <int COLL, class S, class T, int MEM>
  static hipError_t batch_step_t(const BatchLaunch &b, hipStream_t s) {
    hipLaunchKernelGGL((batch_step_kernel<L, COLL, S, T, MEM>), dim3(b.grid), dim3(256), 0, s,
                       static_cast<const S *>(b.fin), static_cast<S *>(b.fout),
                       static_cast<const T *>(b.gbuf), static_cast<const BatchDom *>(b.doms),
                       static_cast<const BatchTile *>(b.tiles), b.active, b.ntiles, T(b.shift));
    return hipGetLastError();
  }
  static hipError_t batch_step(const BatchLaunch &b, hipStream_t s) {
    if constexpr (L::Q > 27) return hipErrorInvalidValue;
    else return with_types(b.storage, [&](auto *sp, auto *tp) -> hipError_t {
      using S = std::remove_pointer_t<decltype(sp)>;
      using T = std::remove_pointer_t<decltype(tp)>;
      switch (b.variant + 3 * b.coll) {
        case 0: return batch_step_t<0, S, T, MEM_PLAIN>(b, s);
        case 1: return batch_step_t<0, S, T, MEM_NTST>(b, s);
        case 2: return batch_step_t<0, S, T, MEM_NTALL>(b, s);
        case 3: return batch_step_t<1, S, T, MEM_PLAIN>(b, s);
        case 4: return batch_step_t<1, S, T, MEM_NTST>(b, s);
        case 5: return batch_step_t<1, S, T, MEM_NTALL>(b, s);
        default: return hipErrorInvalidValue;
      }
    });
  }
  static hipError_t batch_monitor(const BatchLaunch &b, hipStream_t s) {
    if constexpr (L::Q > 27) return hipErrorInvalidValue;
    else return with_types(b.storage, [&](auto *sp, auto *tp) -> hipError_t {
      using S = std::remove_pointer_t<decltype(sp)>;
      using T = std::remove_pointer_t<decltype(tp)>;
      hipLaunchKernelGGL((batch_monitor_kernel<L, S, T>), dim3(b.grid), dim3(256), 0, s,
                         static_cast<const S *>(b.fin), static_cast<const T *>(b.gbuf),
                         static_cast<const BatchDom *>(b.doms),
                         static_cast<const BatchTile *>(b.tiles), b.active, b.ntiles, T(b.shift),
                         static_cast<T *>(b.urec), static_cast<T *>(b.uchk),
                         static_cast<const DomState *>(b.state), b.window, b.mode, b.partials);
      return hipGetLastError();
    });
  }
};

}  // namespace impl

// Host function returning the launcher table (a host-only definition, so the device
// compilation pass never references host launchers).
const LatticeOps &LBM_OPS() {
  static const LatticeOps ops = {LBM_LAT::D,
                                 LBM_LAT::Q,
                                 &LBM_LAT::E[0][0],
                                 &LBM_LAT::W[0],
                                 &impl::Ops<LBM_LAT>::step,
                                 &impl::Ops<LBM_LAT>::init,
                                 &impl::Ops<LBM_LAT>::gather,
                                 &impl::Ops<LBM_LAT>::solid_words,
                                 &impl::Ops<LBM_LAT>::scatter,
                                 &impl::Ops<LBM_LAT>::waves,
                                 &impl::Ops<LBM_LAT>::moments,
                                 &impl::Ops<LBM_LAT>::batch_step,
                                 &impl::Ops<LBM_LAT>::batch_monitor};
  return ops;
}

}  // namespace lbm
