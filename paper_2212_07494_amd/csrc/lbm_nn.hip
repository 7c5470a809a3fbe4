// The warm-start network (include/lbm_nn.h): BF16 matrix-core products with FP32
// accumulation, GELU, mean-square loss, Adam; per-point problem features; periodic
// trilinear upsampling.
//
// Matrix product.  C(m, n) = sum_k A(m, k) B(n, k) with A(m, k) = A[m sam + k sak] and
// B(n, k) = B[n sbn + k sbk] in BF16, accumulated in FP32 by
// v_mfma_f32_16x16x32_bf16.  A 256-thread workgroup computes a 64 x 64 tile; each of
// its four wavefronts a 32 x 32 sub-tile (2 x 2 instructions of 16 x 16 x 32).  K advances
// 32 at a time through LDS (rows padded to 40 elements so the 16-byte fragment reads of
// a wavefront spread over the banks).  Fragment layout: lane l supplies row l % 16 of A
// (column l % 16 of B) and 8 consecutive K values starting at 8 (l / 16); A and B use
// the same K assignment, so the sum over K is exact whatever order the unit takes; the
// 16 x 16 result sits in lane l, register r at row 4 (l / 16) + r, column l % 16.
// Long reductions (the weight gradients sum over every grid point) split K across
// blockIdx.z into FP32 partials that a second kernel sums in a fixed order.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <cstring>
#include <new>
#include <vector>

#include "lbm.h"
#include "lbm_internal.h"
#include "lbm_nn.h"

namespace {

using lbm::set_error;

#define HIP_TRY(expr)                                                                       \
  do {                                                                                      \
    hipError_t e_ = (expr);                                                                 \
    if (e_ != hipSuccess)                                                                   \
      return set_error(LBM_EDEVICE, "%s: %s (%s:%d)", #expr, hipGetErrorString(e_), __FILE__, \
                       __LINE__);                                                           \
  } while (0)

typedef __bf16 bf16;
typedef bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int BM = 64, BN = 64, BK = 32, LDSK = BK + 8;

struct GemmArgs {
  const bf16 *A;
  int64_t sam, sak;
  const bf16 *B;
  int64_t sbn, sbk;
  int M, N, K;
  int kchunk;           // reduction length per blockIdx.z (multiple of BK)
  float *C;             // C(m, n) at C[z * zstride + m * ldc + n]
  int64_t ldc, zstride;
};

__device__ __forceinline__ void load_tile(bf16 (*S)[LDSK], const bf16 *P, int64_t s_row,
                                          int64_t s_k, int row0, int rows, int k0, int kend,
                                          int tid) {
  const int r = tid >> 2, kk = (tid & 3) * 8;
  const int row = row0 + r;
  const int k = k0 + kk;
  if (s_k == 1 && (s_row % 8) == 0 && row < rows && k + 8 <= kend &&
      ((reinterpret_cast<uintptr_t>(P + (int64_t)row * s_row + k) & 15) == 0)) {
    const bf16x8 v = *reinterpret_cast<const bf16x8 *>(P + (int64_t)row * s_row + k);
    *reinterpret_cast<bf16x8 *>(&S[r][kk]) = v;
  } else {
    for (int j = 0; j < 8; ++j) {
      const int kj = k + j;
      S[r][kk + j] = (row < rows && kj < kend) ? P[(int64_t)row * s_row + (int64_t)kj * s_k]
                                               : bf16(0.0f);
    }
  }
}

__global__ void __launch_bounds__(256) gemm_bf16_kernel(GemmArgs g) {
  __shared__ __attribute__((aligned(16))) bf16 As[BM][LDSK];
  __shared__ __attribute__((aligned(16))) bf16 Bs[BN][LDSK];
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int m0 = blockIdx.y * BM, n0 = blockIdx.x * BN;
  const int kbeg = blockIdx.z * g.kchunk;
  const int kend = min(g.K, kbeg + g.kchunk);
  const int wm = (wave >> 1) * 32, wn = (wave & 1) * 32;
  f32x4 acc[2][2];
  for (int i = 0; i < 2; ++i)
    for (int j = 0; j < 2; ++j) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};
  for (int k0 = kbeg; k0 < kend; k0 += BK) {
    load_tile(As, g.A, g.sam, g.sak, m0, g.M, k0, kend, tid);
    load_tile(Bs, g.B, g.sbn, g.sbk, n0, g.N, k0, kend, tid);
    __syncthreads();
    for (int mi = 0; mi < 2; ++mi) {
      const bf16x8 a = *reinterpret_cast<const bf16x8 *>(&As[wm + mi * 16 + (lane & 15)][(lane >> 4) * 8]);
      for (int ni = 0; ni < 2; ++ni) {
        const bf16x8 b =
            *reinterpret_cast<const bf16x8 *>(&Bs[wn + ni * 16 + (lane & 15)][(lane >> 4) * 8]);
        acc[mi][ni] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, acc[mi][ni], 0, 0, 0);
      }
    }
    __syncthreads();
  }
  float *C = g.C + (int64_t)blockIdx.z * g.zstride;
  for (int mi = 0; mi < 2; ++mi)
    for (int ni = 0; ni < 2; ++ni)
      for (int r = 0; r < 4; ++r) {
        const int m = m0 + wm + mi * 16 + (lane >> 4) * 4 + r;
        const int n = n0 + wn + ni * 16 + (lane & 15);
        if (m < g.M && n < g.N) C[(int64_t)m * g.ldc + n] = acc[mi][ni][r];
      }
}

// out[i] (+)= sum_z P[z][i] in order z = 0, 1, ...
__global__ void splitk_reduce_kernel(const float *P, int64_t zstride, int nz, int64_t n,
                                     float *out, int accumulate) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  float s = P[i];
  for (int z = 1; z < nz; ++z) s += P[(int64_t)z * zstride + i];
  out[i] = accumulate ? out[i] + s : s;
}

__device__ __forceinline__ float gelu(float z) {
  const float c = 0.7978845608028654f;  // sqrt(2 / pi)
  return 0.5f * z * (1.0f + tanhf(c * (z + 0.044715f * z * z * z)));
}
__device__ __forceinline__ float gelu_grad(float z) {
  const float c = 0.7978845608028654f;
  const float t = tanhf(c * (z + 0.044715f * z * z * z));
  return 0.5f * (1.0f + t) + 0.5f * z * (1.0f - t * t) * c * (1.0f + 3.0f * 0.044715f * z * z);
}

// Z += bias (per column); act: X_next = bf16(gelu(Z)) or, for the output layer,
// y = scale_c Z (+ addend, a field the network's output is added to).
__global__ void bias_act_kernel(float *Z, const float *bias, int64_t rows, int cols,
                                bf16 *x_next, float *y_out, const float *oscale,
                                const float *addend) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= rows * cols) return;
  const int c = (int)(i % cols);
  const float z = Z[i] + bias[c];
  Z[i] = z;
  if (x_next) x_next[i] = bf16(gelu(z));
  if (y_out) {
    const float y = oscale[c] * z;
    y_out[i] = addend ? y + addend[i] : y;
  }
}

// dZ = dA * gelu'(Z) for hidden layers, dZ = scale_c dA for the output layer; also the
// BF16 copy.
__global__ void act_back_kernel(const float *dA, const float *Z, int64_t n, int cols,
                                const float *oscale, float *dZ, bf16 *dZb) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float d = oscale ? dA[i] * oscale[i % cols] : dA[i] * gelu_grad(Z[i]);
  dZ[i] = d;
  dZb[i] = bf16(d);
}

// db[c] += sum over rows of dZ[r, c] (one workgroup per column, fixed order).
__global__ void __launch_bounds__(256) colsum_kernel(const float *dZ, int64_t rows, int cols,
                                                     float *db) {
  __shared__ float red[256];
  const int c = blockIdx.x;
  float s = 0.f;
  for (int64_t r = threadIdx.x; r < rows; r += 256) s += dZ[r * cols + c];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) db[c] += red[0];
}

__global__ void to_bf16_kernel(const float *x, int64_t n, bf16 *y) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) y[i] = bf16(x[i]);
}

// dY = 2 w_c (y - t) / (rows * cols); per-block partial losses (FP64).
__global__ void __launch_bounds__(256) mse_kernel(const float *y, const float *t, const float *w,
                                                  int64_t rows, int cols, float *dy,
                                                  double *partial) {
  __shared__ double red[256];
  const int64_t n = rows * cols;
  const double inv = 1.0 / (double)n;
  double s = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    const int c = (int)(i % cols);
    const float d = y[i] - t[i];
    dy[i] = (float)(2.0 * w[c] * d * inv);
    s += (double)w[c] * d * d;
  }
  red[threadIdx.x] = s;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) partial[blockIdx.x] = red[0] * inv;
}

__global__ void adam_kernel(float *w, const float *g, float *m, float *v, int64_t n, float lr,
                            float b1, float b2, float eps, float c1, float c2) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float gi = g[i];
  const float mi = b1 * m[i] + (1.f - b1) * gi;
  const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  w[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

unsigned blocks_for(int64_t n) { return (unsigned)((n + 255) / 256); }

}  // namespace

struct lbm_mlp {
  uint32_t magic = 0x4c424e31u;  // "LBN1"
  int L = 0;
  std::vector<int> w;
  int64_t max_rows = 0, rows = 0, nparams = 0;
  hipStream_t stream = nullptr;
  std::vector<int64_t> woff, boff;  // offsets into the parameter vector
  float *params = nullptr, *grads = nullptr, *m1 = nullptr, *m2 = nullptr;
  bf16 *wb = nullptr;               // BF16 copy of the parameter vector
  std::vector<bf16 *> X;            // X[l]: rows x w[l] (BF16 inputs of layer l)
  std::vector<float *> Z;           // Z[l]: rows x w[l+1] (FP32 pre-activations)
  float *dA = nullptr, *dZ = nullptr;
  bf16 *dZb = nullptr;
  float *part = nullptr;            // split-K partials
  int64_t part_elems = 0;
  double *lossp = nullptr;
  float *dy = nullptr, *cw = nullptr;
  float *oscale = nullptr;          // output scale per channel (device)
  std::vector<float> cw_host, oscale_host;  // stay valid while copies are in flight
  float *last_y = nullptr;
  std::vector<void *> owned;

  int alloc(void **p, size_t n) {
    hipError_t e = hipMalloc(p, n ? n : 256);
    if (e != hipSuccess) {
      *p = nullptr;
      return set_error(LBM_ENOMEM, "hipMalloc(%zu): %s", n, hipGetErrorString(e));
    }
    owned.push_back(*p);
    return LBM_OK;
  }
};

namespace {

bool valid(const lbm_mlp *m) { return m && m->magic == 0x4c424e31u; }

// C (rows x cols, FP32) = A . B^T with the given strides; split-K when the reduction is
// long.  accumulate: add into C instead of overwriting (only through the partials).
int gemm(lbm_mlp *m, const bf16 *A, int64_t sam, int64_t sak, const bf16 *B, int64_t sbn,
         int64_t sbk, int M, int N, int K, float *C, int64_t ldc, bool accumulate) {
  GemmArgs g{A, sam, sak, B, sbn, sbk, M, N, K, K, C, ldc, 0};
  const int mt = (M + BM - 1) / BM, nt = (N + BN - 1) / BN;
  int splits = 1;
  if ((int64_t)mt * nt < 512 && K > 4 * BK) {
    splits = (int)std::min<int64_t>((K + 1023) / 1024, 256);
    while (splits > 1 && (int64_t)splits * M * N > m->part_elems) --splits;
  }
  if (splits == 1 && !accumulate) {
    hipLaunchKernelGGL(gemm_bf16_kernel, dim3(nt, mt, 1), dim3(256), 0, m->stream, g);
    HIP_TRY(hipGetLastError());
    return LBM_OK;
  }
  if ((int64_t)splits * M * N > m->part_elems)
    return set_error(LBM_EINVAL, "gemm partials too small");
  int chunk = (K + splits - 1) / splits;
  chunk = (chunk + BK - 1) / BK * BK;
  splits = (K + chunk - 1) / chunk;
  g.kchunk = chunk;
  g.C = m->part;
  g.ldc = N;
  g.zstride = (int64_t)M * N;
  hipLaunchKernelGGL(gemm_bf16_kernel, dim3(nt, mt, splits), dim3(256), 0, m->stream, g);
  HIP_TRY(hipGetLastError());
  if (ldc != N) return set_error(LBM_EINVAL, "split-K output must be dense");
  hipLaunchKernelGGL(splitk_reduce_kernel, dim3(blocks_for((int64_t)M * N)), dim3(256), 0,
                     m->stream, m->part, (int64_t)M * N, splits, (int64_t)M * N, C,
                     accumulate ? 1 : 0);
  HIP_TRY(hipGetLastError());
  return LBM_OK;
}

int refresh_bf16(lbm_mlp *m) {
  hipLaunchKernelGGL(to_bf16_kernel, dim3(blocks_for(m->nparams)), dim3(256), 0, m->stream,
                     m->params, m->nparams, m->wb);
  HIP_TRY(hipGetLastError());
  return LBM_OK;
}

}  // namespace

extern "C" {

int lbm_mlp_create(const int32_t *widths, int32_t nlayers, int64_t max_rows, void *hip_stream,
                   lbm_mlp **out) {
  if (!out) return set_error(LBM_EINVAL, "out is NULL");
  *out = nullptr;
  if (!widths || nlayers < 1 || nlayers > 16) return set_error(LBM_EINVAL, "invalid layer count");
  for (int l = 0; l <= nlayers; ++l)
    if (widths[l] < 1 || widths[l] > 4096) return set_error(LBM_EINVAL, "invalid width %d", widths[l]);
  if (max_rows < 1 || max_rows > (int64_t(1) << 26)) return set_error(LBM_EINVAL, "invalid max_rows");
  lbm_mlp *m = new (std::nothrow) lbm_mlp();
  if (!m) return set_error(LBM_ENOMEM, "host allocation failed");
  m->L = nlayers;
  m->w.assign(widths, widths + nlayers + 1);
  m->max_rows = max_rows;
  m->stream = static_cast<hipStream_t>(hip_stream);
  int64_t off = 0, widest = 0;
  for (int l = 0; l < nlayers; ++l) {
    m->woff.push_back(off);
    off += (int64_t)m->w[l + 1] * m->w[l];
    m->boff.push_back(off);
    off += m->w[l + 1];
  }
  for (int v : m->w) widest = std::max<int64_t>(widest, v);
  m->nparams = off;
  int64_t maxwk = 0;
  for (int l = 0; l < nlayers; ++l) maxwk = std::max<int64_t>(maxwk, (int64_t)m->w[l + 1] * m->w[l]);
  m->part_elems = std::max<int64_t>(maxwk * 64, 1 << 20);
  auto fail_free = [&](int rc) {
    for (void *p : m->owned) (void)hipFree(p);
    delete m;
    return rc;
  };
  int rc;
  if ((rc = m->alloc((void **)&m->params, off * 4)) || (rc = m->alloc((void **)&m->grads, off * 4)) ||
      (rc = m->alloc((void **)&m->m1, off * 4)) || (rc = m->alloc((void **)&m->m2, off * 4)) ||
      (rc = m->alloc((void **)&m->wb, off * 2)) ||
      (rc = m->alloc((void **)&m->dA, max_rows * widest * 4)) ||
      (rc = m->alloc((void **)&m->dZ, max_rows * widest * 4)) ||
      (rc = m->alloc((void **)&m->dZb, max_rows * widest * 2)) ||
      (rc = m->alloc((void **)&m->part, m->part_elems * 4)) ||
      (rc = m->alloc((void **)&m->lossp, 1024 * 8)) ||
      (rc = m->alloc((void **)&m->dy, max_rows * m->w[nlayers] * 4)) ||
      (rc = m->alloc((void **)&m->cw, 4096 * 4)) ||
      (rc = m->alloc((void **)&m->oscale, 4096 * 4)))
    return fail_free(rc);
  m->X.resize(nlayers);
  m->Z.resize(nlayers);
  for (int l = 0; l < nlayers; ++l) {
    if ((rc = m->alloc((void **)&m->X[l], max_rows * m->w[l] * 2)) ||
        (rc = m->alloc((void **)&m->Z[l], max_rows * m->w[l + 1] * 4)))
      return fail_free(rc);
  }
  hipStream_t s = m->stream;
  if (hipMemsetAsync(m->params, 0, off * 4, s) != hipSuccess ||
      hipMemsetAsync(m->grads, 0, off * 4, s) != hipSuccess ||
      hipMemsetAsync(m->m1, 0, off * 4, s) != hipSuccess ||
      hipMemsetAsync(m->m2, 0, off * 4, s) != hipSuccess ||
      hipMemsetAsync(m->wb, 0, off * 2, s) != hipSuccess)
    return fail_free(set_error(LBM_EDEVICE, "clearing the parameters failed"));
  m->oscale_host.assign(m->w[nlayers], 1.0f);
  if (hipMemcpyAsync(m->oscale, m->oscale_host.data(), m->w[nlayers] * 4, hipMemcpyHostToDevice,
                     s) != hipSuccess ||
      hipStreamSynchronize(s) != hipSuccess)
    return fail_free(set_error(LBM_EDEVICE, "setting the output scale failed"));
  *out = m;
  return LBM_OK;
}

int lbm_mlp_num_params(const lbm_mlp *m, int64_t *n) {
  if (!valid(m)) return set_error(LBM_ESTATE, "invalid network");
  if (!n) return set_error(LBM_EINVAL, "n is NULL");
  *n = m->nparams;
  return LBM_OK;
}

int lbm_mlp_set_params(lbm_mlp *m, const float *host, int64_t n) {
  if (!valid(m)) return set_error(LBM_ESTATE, "invalid network");
  if (!host || n != m->nparams) return set_error(LBM_EINVAL, "expected %lld parameters", (long long)m->nparams);
  HIP_TRY(hipMemcpyAsync(m->params, host, n * 4, hipMemcpyHostToDevice, m->stream));
  HIP_TRY(hipMemsetAsync(m->m1, 0, n * 4, m->stream));
  HIP_TRY(hipMemsetAsync(m->m2, 0, n * 4, m->stream));
  int rc = refresh_bf16(m);
  if (rc) return rc;
  HIP_TRY(hipStreamSynchronize(m->stream));
  return LBM_OK;
}

int lbm_mlp_get_params(lbm_mlp *m, float *host, int64_t n) {
  if (!valid(m)) return set_error(LBM_ESTATE, "invalid network");
  if (!host || n != m->nparams) return set_error(LBM_EINVAL, "expected %lld parameters", (long long)m->nparams);
  HIP_TRY(hipMemcpyAsync(host, m->params, n * 4, hipMemcpyDeviceToHost, m->stream));
  HIP_TRY(hipStreamSynchronize(m->stream));
  return LBM_OK;
}

int lbm_mlp_get_grads(lbm_mlp *m, float *host, int64_t n) {
  if (!valid(m)) return set_error(LBM_ESTATE, "invalid network");
  if (!host || n != m->nparams) return set_error(LBM_EINVAL, "expected %lld parameters", (long long)m->nparams);
  HIP_TRY(hipMemcpyAsync(host, m->grads, n * 4, hipMemcpyDeviceToHost, m->stream));
  HIP_TRY(hipStreamSynchronize(m->stream));
  return LBM_OK;
}

int lbm_mlp_zero_grads(lbm_mlp *m) {
  if (!valid(m)) return set_error(LBM_ESTATE, "invalid network");
  HIP_TRY(hipMemsetAsync(m->grads, 0, m->nparams * 4, m->stream));
  return LBM_OK;
}

int lbm_mlp_forward(lbm_mlp *m, const float *x_dev, int64_t rows, const float *addend_dev,
                    float *y_dev) {
  if (!valid(m)) return set_error(LBM_ESTATE, "invalid network");
  if (!x_dev || !y_dev) return set_error(LBM_EINVAL, "NULL device array");
  if (rows < 1 || rows > m->max_rows) return set_error(LBM_EINVAL, "rows %lld out of range", (long long)rows);
  hipStream_t s = m->stream;
  hipLaunchKernelGGL(to_bf16_kernel, dim3(blocks_for(rows * m->w[0])), dim3(256), 0, s, x_dev,
                     rows * m->w[0], m->X[0]);
  HIP_TRY(hipGetLastError());
  for (int l = 0; l < m->L; ++l) {
    const int K = m->w[l], N = m->w[l + 1];
    int rc = gemm(m, m->X[l], K, 1, m->wb + m->woff[l], K, 1, (int)rows, N, K, m->Z[l], N, false);
    if (rc) return rc;
    const bool last = l == m->L - 1;
    hipLaunchKernelGGL(bias_act_kernel, dim3(blocks_for(rows * N)), dim3(256), 0, s, m->Z[l],
                       m->params + m->boff[l], rows, N, last ? nullptr : m->X[l + 1],
                       last ? y_dev : nullptr, m->oscale, last ? addend_dev : nullptr);
    HIP_TRY(hipGetLastError());
  }
  m->rows = rows;
  m->last_y = y_dev;
  return LBM_OK;
}

int lbm_mlp_backward(lbm_mlp *m, const float *dy_dev) {
  if (!valid(m)) return set_error(LBM_ESTATE, "invalid network");
  if (!dy_dev || m->rows < 1) return set_error(LBM_EINVAL, "backward needs a forward first");
  hipStream_t s = m->stream;
  const int64_t rows = m->rows;
  const float *dA = dy_dev;
  for (int l = m->L - 1; l >= 0; --l) {
    const int K = m->w[l], N = m->w[l + 1];
    const bool last = l == m->L - 1;
    hipLaunchKernelGGL(act_back_kernel, dim3(blocks_for(rows * N)), dim3(256), 0, s, dA, m->Z[l],
                       rows * N, N, last ? m->oscale : nullptr, m->dZ, m->dZb);
    HIP_TRY(hipGetLastError());
    hipLaunchKernelGGL(colsum_kernel, dim3(N), dim3(256), 0, s, m->dZ, rows, N,
                       m->grads + m->boff[l]);
    HIP_TRY(hipGetLastError());
    // dW (N x K) += dZ^T X : A(n, r) = dZ[r N + n], B(k, r) = X[r K + k]
    int rc = gemm(m, m->dZb, 1, N, m->X[l], 1, K, N, K, (int)rows, m->grads + m->woff[l], K, true);
    if (rc) return rc;
    if (l > 0) {
      // dA_l (rows x K) = dZ W : A(r, n) = dZ[r N + n], B(k, n) = W[n K + k]
      rc = gemm(m, m->dZb, N, 1, m->wb + m->woff[l], 1, K, (int)rows, K, N, m->dA, K, false);
      if (rc) return rc;
      dA = m->dA;
    }
  }
  return LBM_OK;
}

int lbm_mlp_set_output_scale(lbm_mlp *m, const float *scale) {
  if (!valid(m)) return set_error(LBM_ESTATE, "invalid network");
  if (!scale) return set_error(LBM_EINVAL, "scale is NULL");
  const int C = m->w[m->L];
  for (int c = 0; c < C; ++c)
    if (!(std::isfinite(scale[c]) && scale[c] > 0))
      return set_error(LBM_EINVAL, "output scale %d must be positive", c);
  HIP_TRY(hipStreamSynchronize(m->stream));  // earlier copies from oscale_host are done
  m->oscale_host.assign(scale, scale + C);
  HIP_TRY(hipMemcpyAsync(m->oscale, m->oscale_host.data(), C * 4, hipMemcpyHostToDevice,
                         m->stream));
  return LBM_OK;
}

// Weighted mean-square loss of y against target and its gradient dy (device, rows x C).
static int mse_grad(lbm_mlp *m, const float *y, const float *target, const float *channel_weight,
                    int64_t rows, float *dy, double *loss) {
  const int C = m->w[m->L];
  HIP_TRY(hipStreamSynchronize(m->stream));  // earlier copies from cw_host are done
  m->cw_host.assign(C, 1.0f);
  if (channel_weight)
    for (int c = 0; c < C; ++c) m->cw_host[c] = channel_weight[c];
  HIP_TRY(hipMemcpyAsync(m->cw, m->cw_host.data(), C * 4, hipMemcpyHostToDevice, m->stream));
  const int nb = 1024;
  hipLaunchKernelGGL(mse_kernel, dim3(nb), dim3(256), 0, m->stream, y, target, m->cw, rows, C, dy,
                     m->lossp);
  HIP_TRY(hipGetLastError());
  if (loss) {
    std::vector<double> h(nb);
    HIP_TRY(hipMemcpyAsync(h.data(), m->lossp, nb * 8, hipMemcpyDeviceToHost, m->stream));
    HIP_TRY(hipStreamSynchronize(m->stream));
    double s = 0;
    for (double v : h) s += v;
    *loss = s;
  }
  return LBM_OK;
}

int lbm_mlp_loss_grad(lbm_mlp *m, const float *y_dev, const float *target_dev,
                      const float *channel_weight, int64_t rows, float *dy_dev, double *loss) {
  if (!valid(m)) return set_error(LBM_ESTATE, "invalid network");
  if (!y_dev || !target_dev || !dy_dev) return set_error(LBM_EINVAL, "NULL device array");
  if (rows < 1) return set_error(LBM_EINVAL, "rows must be positive");
  return mse_grad(m, y_dev, target_dev, channel_weight, rows, dy_dev, loss);
}

int lbm_mlp_loss_backward(lbm_mlp *m, const float *target_dev, const float *channel_weight,
                          double *loss) {
  if (!valid(m)) return set_error(LBM_ESTATE, "invalid network");
  if (!target_dev || m->rows < 1) return set_error(LBM_EINVAL, "loss needs a forward first");
  int rc = mse_grad(m, m->last_y, target_dev, channel_weight, m->rows, m->dy, nullptr);
  if (rc) return rc;
  rc = lbm_mlp_backward(m, m->dy);
  if (rc) return rc;
  if (loss) {
    std::vector<double> h(1024);
    HIP_TRY(hipMemcpyAsync(h.data(), m->lossp, 1024 * 8, hipMemcpyDeviceToHost, m->stream));
    HIP_TRY(hipStreamSynchronize(m->stream));
    double s = 0;
    for (double v : h) s += v;
    *loss = s;
  }
  return LBM_OK;
}

int lbm_mlp_adam(lbm_mlp *m, double lr, double beta1, double beta2, double eps, int64_t t) {
  if (!valid(m)) return set_error(LBM_ESTATE, "invalid network");
  if (t < 1 || !(lr >= 0) || !(beta1 >= 0 && beta1 < 1) || !(beta2 >= 0 && beta2 < 1) || !(eps > 0))
    return set_error(LBM_EINVAL, "invalid Adam parameters");
  const float c1 = (float)(1.0 - std::pow(beta1, (double)t));
  const float c2 = (float)(1.0 - std::pow(beta2, (double)t));
  hipLaunchKernelGGL(adam_kernel, dim3(blocks_for(m->nparams)), dim3(256), 0, m->stream, m->params,
                     m->grads, m->m1, m->m2, m->nparams, (float)lr, (float)beta1, (float)beta2,
                     (float)eps, c1, c2);
  HIP_TRY(hipGetLastError());
  return refresh_bf16(m);
}

int lbm_mlp_free(lbm_mlp *m) {
  if (!valid(m)) return set_error(LBM_ESTATE, "invalid network");
  (void)hipStreamSynchronize(m->stream);
  for (void *p : m->owned) (void)hipFree(p);
  m->magic = 0;
  delete m;
  return LBM_OK;
}

}  // extern "C"

// ---- problem features and upsampling -------------------------------------------------------

namespace {

struct ModeDev {
  float k[3], p[3], s, K, phase;
};

__global__ void features_kernel(ModeDev m0, ModeDev m1, ModeDev m2, ModeDev m3, int n, float step,
                                float inv_box2pi, float tau_m, float re, float invU, float U,
                                int order, float inv_rho_scale,
                                const float *__restrict__ mode_coef, float *__restrict__ x,
                                float *__restrict__ base) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t N = (int64_t)n * n * n;
  if (idx >= N) return;
  const float px = (float)(idx % n) * step;
  const float py = (float)((idx / n) % n) * step;
  const float pz = (float)(idx / ((int64_t)n * n)) * step;
  float tmp[LBM_WS_FEATURES];
  float *o = x ? x + idx * LBM_WS_FEATURES : tmp;
  const ModeDev ms[4] = {m0, m1, m2, m3};
  float th[4];
  float ub[3] = {0.0f, 0.0f, 0.0f};
  float rmode = 0.0f;
  for (int j = 0; j < 4; ++j) {
    const ModeDev &m = ms[j];
    // theta = 2 pi k . x / box + phase
    th[j] = (m.k[0] * px + m.k[1] * py + m.k[2] * pz) * inv_box2pi + m.phase;
    const float sn = sinf(th[j]), cs = cosf(th[j]);
    const float a_j = m.s * invU;
    const float kn = m.K / inv_box2pi;  // |k_j| in integer units
    for (int a = 0; a < 3; ++a) {
      o[11 * j + a] = m.p[a] * sn;
      o[11 * j + 3 + a] = m.p[a] * cs;
      o[11 * j + 8 + a] = m.k[a] / kn;
      ub[a] += a_j * (m.p[a] * sn);
    }
    if (mode_coef) {
      // the mode's own response corrected: a_j ((p_j + c_0..2) sin + c_3..5 cos), density
      // a_j (c_6 sin + c_7 cos)
      const float *cj = mode_coef + 8 * j;
      for (int a = 0; a < 3; ++a) ub[a] += a_j * (cj[a] * sn + cj[3 + a] * cs);
      rmode += a_j * (cj[6] * sn + cj[7] * cs);
    }
    o[11 * j + 6] = a_j;
    o[11 * j + 7] = m.K;
  }
  o[44] = tau_m;
  o[45] = re;
  if (!base) return;
  float rb = rmode;
  if (order >= 2) {
    // (u1 . grad) u1 = sum_{i != j} s_i s_j (p_i . k_j) p_j sin(theta_i) cos(theta_j): each
    // product is half a wave at theta_i + theta_j and half at theta_i - theta_j.  Its
    // solenoidal part is balanced by viscosity, the rest by the pressure 3 rho0 delta-rho.
    const float nu = tau_m / 3.0f;
    for (int i = 0; i < 4; ++i) {
      for (int j = 0; j < 4; ++j) {
        if (i == j) continue;
        const ModeDev &mi = ms[i], &mj = ms[j];
        const float pk = (mi.p[0] * mj.k[0] + mi.p[1] * mj.k[1] + mi.p[2] * mj.k[2]) * inv_box2pi;
        if (pk == 0.0f) continue;
        const float c = 0.5f * (mi.s * invU) * (mj.s * invU) * U * pk;  // |A| / U
        for (int sg = -1; sg <= 1; sg += 2) {
          float q[3];
          for (int a = 0; a < 3; ++a) q[a] = (mi.k[a] + sg * mj.k[a]) * inv_box2pi;
          const float q2 = q[0] * q[0] + q[1] * q[1] + q[2] * q[2];
          if (q2 == 0.0f) continue;
          const float qA = c * (q[0] * mj.p[0] + q[1] * mj.p[1] + q[2] * mj.p[2]);
          const float ph = th[i] + sg * th[j];
          const float sn = sinf(ph), cs = cosf(ph);
          for (int a = 0; a < 3; ++a) ub[a] -= (c * mj.p[a] - q[a] * qA / q2) / (nu * q2) * sn;
          rb += 3.0f * qA / q2 * cs;
        }
      }
    }
  }
  float *b = base + idx * 4;
  b[0] = ub[0];
  b[1] = ub[1];
  b[2] = ub[2];
  b[3] = rb * inv_rho_scale;
}

}  // namespace

extern "C" {

int lbm_ws_features(const lbm_ws_problem *p, int32_t n, int32_t box, float *x_dev,
                    float *base_dev, int32_t base_order, double rho_scale,
                    const float *mode_coef_dev, double *U_out, void *hip_stream) {
  if (!p || (!x_dev && !base_dev)) return set_error(LBM_EINVAL, "NULL argument");
  if (p->nmodes != 4) return set_error(LBM_EINVAL, "the feature layout needs 4 modes");
  if (n < 1 || box < 1 || n > 1024) return set_error(LBM_EINVAL, "invalid grid");
  if (!(p->tau2 > 0.5)) return set_error(LBM_EINVAL, "tau2 must exceed 1/2");
  if (base_dev && base_order != 1 && base_order != 2)
    return set_error(LBM_EINVAL, "base_order must be 1 or 2");
  if (base_dev && !(std::isfinite(rho_scale) && rho_scale > 0))
    return set_error(LBM_EINVAL, "rho_scale must be positive");
  const double nu = (p->tau2 - 0.5) / 3.0;
  const double two_pi = 6.283185307179586;
  ModeDev md[4];
  double U = 0, Kmin = 1e300;
  for (int j = 0; j < 4; ++j) {
    const double kk = std::sqrt(p->k[j][0] * p->k[j][0] + p->k[j][1] * p->k[j][1] +
                                p->k[j][2] * p->k[j][2]);
    if (!(kk > 0)) return set_error(LBM_EINVAL, "mode %d has a zero wavevector", j);
    const double K = two_pi * kk / box;
    const double s = p->amp[j] / (nu * K * K);
    U += std::fabs(s);
    Kmin = std::min(Kmin, K);
    for (int a = 0; a < 3; ++a) {
      md[j].k[a] = (float)p->k[j][a];
      md[j].p[a] = (float)p->p[j][a];
    }
    md[j].s = (float)s;
    md[j].K = (float)K;
    md[j].phase = (float)p->phase[j];
  }
  if (!(U > 0)) return set_error(LBM_EINVAL, "zero forcing");
  const double re = U / (nu * Kmin);
  const int64_t N = (int64_t)n * n * n;
  hipLaunchKernelGGL(features_kernel, dim3((unsigned)((N + 255) / 256)), dim3(256), 0,
                     static_cast<hipStream_t>(hip_stream), md[0], md[1], md[2], md[3], n,
                     (float)box / (float)n, (float)(two_pi / box), (float)(p->tau2 - 0.5),
                     (float)re, (float)(1.0 / U), (float)U, (int)base_order,
                     base_dev ? (float)(1.0 / rho_scale) : 1.0f, mode_coef_dev, x_dev,
                     base_dev);
  HIP_TRY(hipGetLastError());
  if (U_out) *U_out = U;
  return LBM_OK;
}

int lbm_ws_mode_features(const lbm_ws_problem *p, int32_t box, float *out_dev,
                         void *hip_stream) {
  if (!p || !out_dev) return set_error(LBM_EINVAL, "NULL argument");
  if (p->nmodes < 1 || p->nmodes > 8) return set_error(LBM_EINVAL, "nmodes must be 1..8");
  if (box < 1) return set_error(LBM_EINVAL, "invalid box");
  if (!(p->tau2 > 0.5)) return set_error(LBM_EINVAL, "tau2 must exceed 1/2");
  const double two_pi = 6.283185307179586;
  std::vector<float> h((size_t)p->nmodes * LBM_WS_MODE_FEATURES);
  for (int j = 0; j < p->nmodes; ++j) {
    const double kk = std::sqrt(p->k[j][0] * p->k[j][0] + p->k[j][1] * p->k[j][1] +
                                p->k[j][2] * p->k[j][2]);
    if (!(kk > 0)) return set_error(LBM_EINVAL, "mode %d has a zero wavevector", j);
    float *o = h.data() + (size_t)j * LBM_WS_MODE_FEATURES;
    for (int a = 0; a < 3; ++a) {
      const double ka = two_pi * p->k[j][a] / box;  // phase advance per lattice link
      o[a] = (float)ka;
      o[3 + a] = (float)std::sin(ka);
      o[6 + a] = (float)(1.0 - std::cos(ka));
      o[9 + a] = (float)p->p[j][a];
    }
    o[12] = (float)(p->tau2 - 0.5);
  }
  hipStream_t s = static_cast<hipStream_t>(hip_stream);
  HIP_TRY(hipMemcpyAsync(out_dev, h.data(), h.size() * sizeof(float), hipMemcpyHostToDevice, s));
  HIP_TRY(hipStreamSynchronize(s));  // h is released on return
  return LBM_OK;
}

}  // extern "C"
