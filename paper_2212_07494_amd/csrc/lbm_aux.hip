// Monitor finalisation and the stream-copy probe.
#include <hip/hip_runtime.h>

#include <cstdint>

namespace lbm {
namespace {

constexpr int kSlots = 8;   // mass, mom x/y/z, sum |du|^2, sum |u|^2, max |u|, non-finite
constexpr int kUmax = 6;

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

}  // namespace

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
