// Monitor finalisation and the stream-copy probe.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "lbm_internal.h"

namespace lbm {
namespace {

constexpr int kSlots = MON_SLOTS;  // the monitor record's slots (lbm_internal.h)
constexpr int kUmax = MON_UMAX;

// Sum the per-block partials in a fixed order (one block of 256 threads): thread k
// folds blocks k, k + 256, ... in turn, then a fixed binary tree combines the threads.
// The result is deterministic for a given block count.
__global__ void __launch_bounds__(256) finalize_kernel(const double *partials, int64_t nb,
                                                       double *out) {
  __shared__ double red[256];
  for (int s = 0; s < kSlots; ++s) {
    double acc = 0.0;
    for (int64_t b = threadIdx.x; b < nb; b += 256) {
      const double t = partials[b * kSlots + s];
      acc = (s == kUmax) ? fmax(acc, t) : acc + t;
    }
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
      if ((int)threadIdx.x < o)
        red[threadIdx.x] = (s == kUmax) ? fmax(red[threadIdx.x], red[threadIdx.x + o])
                                        : red[threadIdx.x] + red[threadIdx.x + o];
      __syncthreads();
    }
    if (threadIdx.x == 0) out[s] = red[0];
    __syncthreads();
  }
}

// Copy variants (16-byte vectors):
// 0: grid-stride loop;  1: one vector per thread;  2: one vector per thread,
// non-temporal;  3: four vectors per thread, block-strided (all loads before stores).
__global__ void copy_stride(const float4 *__restrict__ src, float4 *__restrict__ dst, int64_t n) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride)
    dst[i] = src[i];
}
__global__ void copy_one(const float4 *__restrict__ src, float4 *__restrict__ dst, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) dst[i] = src[i];
}
typedef float v4f __attribute__((ext_vector_type(4)));
__global__ void copy_one_nt(const float4 *__restrict__ src, float4 *__restrict__ dst, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const v4f *s = reinterpret_cast<const v4f *>(src);
  v4f *d = reinterpret_cast<v4f *>(dst);
  if (i < n) __builtin_nontemporal_store(__builtin_nontemporal_load(s + i), d + i);
}
__global__ void copy_four(const float4 *__restrict__ src, float4 *__restrict__ dst, int64_t n) {
  const int64_t base = (int64_t)blockIdx.x * blockDim.x * 4 + threadIdx.x;
  float4 v[4];
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const int64_t i = base + (int64_t)k * blockDim.x;
    if (i < n) v[k] = src[i];
  }
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const int64_t i = base + (int64_t)k * blockDim.x;
    if (i < n) dst[i] = v[k];
  }
}

// Every byte of a buffer set to 0xff: a quiet NaN in binary16, binary32 and binary64 alike
// (the debug pass that poisons the buffer a step is about to write).  16 bytes a thread,
// then the tail byte by byte.
__global__ void fill_ff_kernel(uint4 *__restrict__ p, int64_t n16, unsigned char *__restrict__ tail,
                               int ntail) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n16) p[i] = make_uint4(~0u, ~0u, ~0u, ~0u);
  if (i < ntail) tail[i] = 0xff;
}

// Below this window coherence a stalled residual counts as the round-off floor.
constexpr double kFloorCoherence = 0.03;

// Per-domain convergence decision after a compare pass (one thread per domain).
__global__ void decide_kernel(const int *__restrict__ tile_begin, const int *__restrict__ tile_end,
                              const double *__restrict__ partials, DomState *__restrict__ st,
                              int *__restrict__ active, int *__restrict__ n_active, int ndom,
                              double tol, int stall_checks, int steps) {
  const int d = blockIdx.x * blockDim.x + threadIdx.x;
  if (d >= ndom || !active[d]) return;
  double du2 = 0.0, u2 = 0.0, bad = 0.0, duk2 = 0.0;
  for (int t = tile_begin[d]; t < tile_end[d]; ++t) {
    du2 += partials[(int64_t)t * BATCH_PARTIALS + BP_DU2];
    u2 += partials[(int64_t)t * BATCH_PARTIALS + BP_U2];
    bad += partials[(int64_t)t * BATCH_PARTIALS + BP_BAD];
    duk2 += partials[(int64_t)t * BATCH_PARTIALS + BP_DUK2];
  }
  DomState s = st[d];
  s.steps += steps;
  const double r = u2 > 0.0 ? sqrt(du2 / u2) : (du2 > 0.0 ? INFINITY : 0.0);
  s.resid = r;
  // Coherence over a window of stall_checks checks: the drift per step since the window
  // started against the change of the last step.  A state still converging, however
  // slowly, drifts steadily (coherence near 1); at the round-off floor the per-step
  // changes are noise, which the long window does not accumulate (coherence near 0).
  // The monitor pass of a check that starts a window stored the window's first velocity.
  const bool window_end = s.nchk % stall_checks == 0;  // this check also starts the next
  if (window_end) {
    const int64_t gap = s.win_steps >= 0 ? s.steps - s.win_steps : 0;
    if (gap > 0) s.coherence = du2 > 0.0 ? sqrt(duk2 / du2) / (double)gap : 0.0;
    s.win_steps = s.steps;
  }
  s.nchk += 1;
  int stop = 0;
  if (bad > 0.0 || !isfinite(r)) {
    s.status = 3;
    stop = 1;
  } else if (r < tol) {
    s.status = 1;
    stop = 1;
  } else {
    if (r < 0.99 * s.best) {
      s.best = r;
      s.stall = 0;
    } else if (++s.stall >= stall_checks && window_end && s.coherence < kFloorCoherence) {
      // no progress for a whole window, and its change is noise, not a drift
      s.status = 2;
      stop = 1;
    }
  }
  st[d] = s;
  if (stop) {
    active[d] = 0;
    atomicSub(n_active, 1);
  }
}

// Steps taken by eager advances of the active domains.
__global__ void add_steps_kernel(const int *__restrict__ active, DomState *__restrict__ st,
                                 int ndom, int64_t n) {
  const int d = blockIdx.x * blockDim.x + threadIdx.x;
  if (d < ndom && active[d]) st[d].steps += n;
}

}  // namespace

hipError_t decide_domains(const int *tile_begin, const int *tile_end, const double *partials,
                          void *state, int *active, int *n_active, int ndom, double tol,
                          int stall_checks, int steps, hipStream_t s) {
  hipLaunchKernelGGL(decide_kernel, dim3((ndom + 255) / 256), dim3(256), 0, s, tile_begin,
                     tile_end, partials, static_cast<DomState *>(state), active, n_active, ndom,
                     tol, stall_checks, steps);
  return hipGetLastError();
}

hipError_t add_domain_steps(const int *active, void *state, int ndom, int64_t n, hipStream_t s) {
  hipLaunchKernelGGL(add_steps_kernel, dim3((ndom + 255) / 256), dim3(256), 0, s, active,
                     static_cast<DomState *>(state), ndom, n);
  return hipGetLastError();
}

// The force-factor counter of graph replays: *ctr = set ? add : *ctr + add.
__global__ void counter_kernel(int64_t *ctr, int64_t add, int set) {
  if (threadIdx.x == 0 && blockIdx.x == 0) *ctr = set ? add : *ctr + add;
}

hipError_t graph_counter(int64_t *ctr, int64_t add, int set, hipStream_t s) {
  hipLaunchKernelGGL(counter_kernel, dim3(1), dim3(64), 0, s, ctr, add, set);
  return hipGetLastError();
}

hipError_t fill_nan(void *p, size_t bytes, hipStream_t s) {
  const int64_t n16 = (int64_t)(bytes / 16);
  const int ntail = (int)(bytes % 16);
  const int64_t n = n16 > ntail ? n16 : ntail;
  if (n == 0) return hipSuccess;
  unsigned char *tail = static_cast<unsigned char *>(p) + (size_t)n16 * 16;
  hipLaunchKernelGGL(fill_ff_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s,
                     static_cast<uint4 *>(p), n16, tail, ntail);
  return hipGetLastError();
}

hipError_t finalize_monitors(const double *partials, int64_t nb, double *out, hipStream_t s) {
  hipLaunchKernelGGL(finalize_kernel, dim3(1), dim3(256), 0, s, partials, nb, out);
  return hipGetLastError();
}

hipError_t copy_probe(const void *src, void *dst, size_t bytes, int reps, int block, int variant,
                      hipStream_t s) {
  const int64_t n = (int64_t)(bytes / 16);
  if (n == 0) return hipSuccess;
  const float4 *a = static_cast<const float4 *>(src);
  float4 *b = static_cast<float4 *>(dst);
  for (int r = 0; r < reps; ++r) {
    if (variant == 0) {
      int64_t blocks = (n + (int64_t)block * 4 - 1) / ((int64_t)block * 4);
      if (blocks > 65536) blocks = 65536;
      hipLaunchKernelGGL(copy_stride, dim3((unsigned)blocks), dim3(block), 0, s, a, b, n);
    } else if (variant == 1 || variant == 2) {
      const int64_t blocks = (n + block - 1) / block;
      if (variant == 1)
        hipLaunchKernelGGL(copy_one, dim3((unsigned)blocks), dim3(block), 0, s, a, b, n);
      else
        hipLaunchKernelGGL(copy_one_nt, dim3((unsigned)blocks), dim3(block), 0, s, a, b, n);
    } else {
      const int64_t blocks = (n + (int64_t)block * 4 - 1) / ((int64_t)block * 4);
      hipLaunchKernelGGL(copy_four, dim3((unsigned)blocks), dim3(block), 0, s, a, b, n);
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

}  // namespace lbm
