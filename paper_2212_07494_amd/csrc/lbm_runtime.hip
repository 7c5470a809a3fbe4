// C-ABI runtime of the forced lattice-Boltzmann library: parameter validation, device
// memory, dispatch to the per-lattice kernels, monitors and data transfer.
// The declarations and their contracts are in include/lbm.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "lbm.h"
#include "lbm_internal.h"
#include "lbm_nn.h"

namespace {

thread_local std::string g_last_error;

int fail(int status, const char *fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_last_error = buf;
  return status;
}

}  // namespace

int lbm::set_error(int status, const char *fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_last_error = buf;
  return status;
}

namespace {

#define HIP_TRY(expr)                                                                     \
  do {                                                                                    \
    hipError_t e_ = (expr);                                                               \
    if (e_ != hipSuccess)                                                                 \
      return fail(LBM_EDEVICE, "%s: %s (%s:%d)", #expr, hipGetErrorString(e_), __FILE__, \
                  __LINE__);                                                              \
  } while (0)

constexpr uint32_t kMagic = 0x4c424d31u;  // "LBM1"

size_t storage_bytes(int s) { return s == LBM_F64 ? 8 : (s == LBM_F16_SHIFTED ? 2 : 4); }

// FNV-1a, 64-bit (Fowler, Noll and Vo): identity of the parameters a checkpoint needs.
uint64_t fnv1a(uint64_t h, const void *data, size_t n) {
  const unsigned char *b = static_cast<const unsigned char *>(data);
  for (size_t i = 0; i < n; ++i) {
    h ^= b[i];
    h *= 0x100000001b3ull;
  }
  return h;
}
// Memory-access variants of the step (plain, non-temporal stores, non-temporal loads and
// stores); a tuning variant v has the base b = v % kBaseVariants, which selects
// b % kMemVariants, for (b / kMemVariants) odd the scalar-base addressing path where no
// bounce-back can occur, and for b >= 2 kMemVariants the XCD-contiguous placement of the
// blocks; v / kBaseVariants indexes kWaveCaps, the waves per SIMD the step's workgroups
// are held to (0: as many as the registers allow).
constexpr int kMemVariants = 3;
constexpr int kBaseVariants = 4 * kMemVariants;
constexpr int kWaveCaps[] = {0, 5, 4, 3, 2};
constexpr int kNumCaps = sizeof(kWaveCaps) / sizeof(kWaveCaps[0]);

// Dynamic LDS bytes that leave room for at most (4 SIMDs x cap) / (waves of a block)
// blocks of bx x by threads on a CU with lds_cu bytes of LDS, at most lds_block of them
// to one block: a size strictly between lds_cu / (n + 1) and lds_cu / n, taken at the
// middle of that interval on a 256-byte grid so that allocation granularity cannot move
// it out; 0 where no cap is asked for or none is possible.
unsigned lds_for_cap(int cap, int bx, int by, int lds_cu, int lds_block) {
  if (cap <= 0 || lds_cu <= 0 || lds_block <= 0) return 0;
  const int wpb = (bx * by + 63) / 64;
  const int n = (4 * cap) / wpb;
  if (n < 1) return 0;
  const long lo = (long)lds_cu / (n + 1) + 1;
  const long hi = std::min<long>((long)lds_cu / n, lds_block);
  if (lo > hi) return 0;
  long pad = ((lo + hi) / 2) & ~255L;
  if (pad < lo) pad = hi;
  return (unsigned)pad;
}
constexpr uint64_t kFnvBasis = 0xcbf29ce484222325ull;
size_t arith_bytes(int s) { return s == LBM_F64 ? 8 : 4; }
bool shifted(int s) { return s == LBM_F32_SHIFTED || s == LBM_F16_SHIFTED; }

using lbm::ops_for;

// Block shape: 64-wide rows (one wavefront per row segment), up to 256 threads.
void block_shape(int nx, int &bx, int &by) {
  bx = nx >= 256 ? 256 : (nx >= 128 ? 128 : 64);
  by = 256 / bx;
}

}  // namespace

// Staging memory of lbm_get_populations_noalloc, which allocates nothing: node indices and
// gathered values.  Each device holds its own copy for the life of the process.  In host
// code this name is not a device address: its address on each device is taken once, with
// that device current, by noalloc_scratch_setup (called from lbm_init), and only that
// address is passed to kernels and copies.
static __device__ __align__(256) unsigned char lbm_noalloc_scratch[LBM_NOALLOC_SCRATCH_BYTES];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_noalloc_mu;
void *g_noalloc_ptr[kMaxDevices] = {};

// The device address of lbm_noalloc_scratch on the current device, kept per device.
int noalloc_scratch_setup(int device) {
  if (device < 0 || device >= kMaxDevices)
    return fail(LBM_EDEVICE, "device %d beyond the library's table of %d", device, kMaxDevices);
  std::lock_guard<std::mutex> lock(g_noalloc_mu);
  if (g_noalloc_ptr[device]) return LBM_OK;
  void *ptr = nullptr;
  const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(lbm_noalloc_scratch));
  if (e != hipSuccess || !ptr)
    return fail(LBM_EDEVICE, "hipGetSymbolAddress of the no-alloc scratch: %s",
                hipGetErrorString(e));
  g_noalloc_ptr[device] = ptr;
  return LBM_OK;
}

void *noalloc_scratch_of(int device) {
  if (device < 0 || device >= kMaxDevices) return nullptr;
  std::lock_guard<std::mutex> lock(g_noalloc_mu);
  return g_noalloc_ptr[device];
}

}  // namespace

struct lbm_ctx {
  uint32_t magic = kMagic;
  int device = 0;  // the device current at lbm_init
  lbm_params p{};
  const lbm::LatticeOps *ops = nullptr;
  int D = 0, Q = 0;
  int64_t N = 0;
  hipStream_t stream = nullptr;
  lbm_allocator alloc{};
  bool own_alloc = true;
  void *buf[2] = {nullptr, nullptr};
  int cur = 0;
  void *gtab = nullptr;
  int g_n = 1, g_axis = -1, gk = 0;
  uint64_t g_hash = 0;  // FNV-1a of the force table as uploaded (checkpoint identity)
  uint32_t *smask = nullptr;              // device solid mask words (NULL: none)
  std::vector<uint32_t> smask_host;       // the same on the host (upload source, identity)
  void *uprev = nullptr;
  int64_t uprev_time = -2;
  double *partials = nullptr;
  int64_t nblocks = 0, nblocks_cap = 0;  // blocks of the current grid; partials' capacity
  double *mon_dev = nullptr;
  // In-step monitor checks (monitor_every > 0): the device record of time dev_step (-1:
  // none) and its mode; the latest check's copy in pinned host memory (mon_host) with the
  // event that completes it, read once without blocking (check_pending); a non-finite
  // record stops the stepping until the state is replaced.
  int64_t dev_step = -1;
  int dev_mode = 0;
  double *mon_host = nullptr;
  hipEvent_t mon_ev = nullptr;
  bool check_pending = false;
  int64_t check_step = -1;
  int check_mode = 0;
  bool nonfinite_seen = false;
  int64_t nonfinite_step = -1;
  // Steps replayed from captured graphs (small lattices, where launches dominate): a
  // chunk of kGraphChunk steps captured on a private stream, one graph per (buffer
  // parity, device force factors or not); the factors are uploaded to gs_dev and read at
  // the device counter gs_ctr, which each replay advances.
  hipStream_t cap = nullptr;
  hipGraphExec_t gexec[2][2] = {{nullptr, nullptr}, {nullptr, nullptr}};
  double *gs_dev = nullptr;
  size_t gs_cap = 0;
  int64_t *gs_ctr = nullptr;
  // pinned staging of the factors (the upload is asynchronous) and the event of the last
  // upload, waited on before the staging buffer is written again
  double *gs_host = nullptr;
  size_t gs_host_cap = 0;
  hipEvent_t gs_ev = nullptr;
  void drop_graphs() {
    for (auto &row : gexec)
      for (auto &e : row) {
        if (e) (void)hipGraphExecDestroy(e);
        e = nullptr;
      }
  }
  void *scratch = nullptr;
  size_t scratch_bytes = 0;
  size_t bytes = 0;
  int64_t t = 0;
  double last_scale = 1.0;
  double c0 = 0, c1 = 0, c2 = 0, c3 = 0, c4 = 0, shift = 0;
  int bx = 64, by = 4, variant = 0;
  int lds_cu = 0, lds_block = 0;  // LDS bytes of a CU and the most one workgroup may take
  lbm_monitors mon{};

  int dalloc(void **ptr, size_t n) {
    *ptr = nullptr;
    if (n == 0) n = 256;
    if (alloc.alloc) {
      *ptr = alloc.alloc(n, alloc.user);
      if (!*ptr) return fail(LBM_ENOMEM, "allocator returned NULL for %zu bytes", n);
    } else {
      hipError_t e = hipMalloc(ptr, n);
      if (e != hipSuccess) {
        *ptr = nullptr;
        return fail(e == hipErrorOutOfMemory ? LBM_ENOMEM : LBM_EDEVICE, "hipMalloc(%zu): %s", n,
                    hipGetErrorString(e));
      }
    }
    bytes += n;
    return LBM_OK;
  }
  void dfree(void *ptr) {
    if (!ptr) return;
    if (alloc.free)
      alloc.free(ptr, alloc.user);
    else if (!alloc.alloc)
      (void)hipFree(ptr);
  }
  int need_scratch(size_t n) {
    if (n <= scratch_bytes) return LBM_OK;
    // the stream may still use the old scratch
    HIP_TRY(hipStreamSynchronize(stream));
    dfree(scratch);
    bytes -= scratch_bytes;
    scratch = nullptr;
    scratch_bytes = 0;
    int rc = dalloc(&scratch, n);
    if (rc) return rc;
    scratch_bytes = n;
    return LBM_OK;
  }
  lbm::LaunchDesc desc(double gscale) const {
    lbm::LaunchDesc d{};
    d.coll = p.collision;
    if (p.collision == LBM_SMRT) {
      const bool hi = p.max_order == 6;
      if (p.force_order == 4) d.coll = 5;
      else if (p.force_order == 3) d.coll = hi ? 6 : 4;
      else if (hi) d.coll = 3;
      else if (c3 != 0 || c4 != 0) d.coll = 7;  // split trace rates
    }
    d.storage = p.storage;
    d.gk = gk;
    d.fin = buf[cur];
    d.fout = buf[cur ^ 1];
    d.geo.nx = p.nx;
    d.geo.ny = p.ny;
    d.geo.nz = p.nz;
    d.geo.N = (int)N;
    d.geo.ps = (int64_t)p.nx * p.ny;
    for (int a = 0; a < 3; ++a) d.geo.wall[a] = p.bc[a] == LBM_WALLS;
    d.geo.smask = smask;
    d.gtab = gtab;
    d.g_axis = g_axis;
    d.g_n = g_n;
    d.gscale = gscale;
    d.shift = shift;
    d.c0 = c0;
    d.c1 = c1;
    d.c2 = c2;
    d.c3 = c3;
    d.c4 = c4;
    d.bx = bx;
    d.by = by;
    const int base = variant % kBaseVariants;
    d.variant = base % kMemVariants;
    d.fast_ok = (base / kMemVariants) % 2;
    d.xcd = base / (2 * kMemVariants);
    d.lds_pad = lds_for_cap(kWaveCaps[variant / kBaseVariants], bx, by, lds_cu, lds_block);
    return d;
  }
};

namespace {

bool valid(const lbm_ctx *c) { return c && c->magic == kMagic; }

// c_s^2 = num / 3 of a lattice: 1/3, or 2/3 on D3Q39.
double cs2_num(int lattice) { return lattice == LBM_D3Q39 ? 2.0 : 1.0; }

int validate(const lbm_params *p) {
  if (!p) return fail(LBM_EINVAL, "params is NULL");
  if (p->lattice < LBM_D2Q9 || p->lattice > LBM_D3Q39)
    return fail(LBM_EINVAL, "unknown lattice %d", p->lattice);
  if (p->collision != LBM_BGK && p->collision != LBM_SMRT && p->collision != LBM_RMRT)
    return fail(LBM_EINVAL, "unknown collision %d", p->collision);
  if (p->storage < LBM_F64 || p->storage > LBM_F16_SHIFTED)
    return fail(LBM_EINVAL, "unknown storage %d", p->storage);
  if (p->nx <= 0 || p->ny <= 0 || p->nz <= 0)
    return fail(LBM_EINVAL, "sizes must be positive (%d, %d, %d)", p->nx, p->ny, p->nz);
  if (p->lattice == LBM_D2Q9 && p->nz != 1) return fail(LBM_EINVAL, "D2Q9 needs nz == 1");
  if (p->lattice == LBM_D3Q39) {
    // links of up to three nodes: one periodic wrap needs every extent >= 3; no wall or
    // solid-node rule is defined for populations that cross more than one node
    if (p->nx < 3 || p->ny < 3 || p->nz < 3)
      return fail(LBM_EINVAL, "D3Q39 needs every extent >= 3 (%d, %d, %d)", p->nx, p->ny, p->nz);
    if (p->bc[0] != LBM_PERIODIC || p->bc[1] != LBM_PERIODIC || p->bc[2] != LBM_PERIODIC)
      return fail(LBM_EINVAL, "D3Q39 runs periodic boxes only (no wall rule for its long links)");
    if (p->solid) return fail(LBM_EINVAL, "D3Q39 runs without solid nodes");
  }
  if (p->ny > 65535 || p->nz > 65535) return fail(LBM_EINVAL, "ny and nz must be <= 65535");
  const int64_t N = (int64_t)p->nx * p->ny * p->nz;
  if (N >= (int64_t(1) << 31)) return fail(LBM_EINVAL, "node count %lld >= 2^31", (long long)N);
  for (int a = 0; a < 3; ++a)
    if (p->bc[a] != LBM_PERIODIC && p->bc[a] != LBM_WALLS)
      return fail(LBM_EINVAL, "unknown boundary kind %d on axis %d", p->bc[a], a);
  if (!(p->tau[2] > 0.5) || !std::isfinite(p->tau[2]))
    return fail(LBM_EINVAL, "tau[2] = %g must exceed 1/2", p->tau[2]);
  if (p->collision == LBM_SMRT || p->collision == LBM_RMRT) {
    if (!(p->tau[3] > 0.5) || !std::isfinite(p->tau[3]))
      return fail(LBM_EINVAL, "tau[3] = %g must exceed 1/2", p->tau[3]);
    if (p->tau[4] != 1.0)
      return fail(LBM_EINVAL, "SMRT trims order 4: tau[4] must be 1 (got %g)", p->tau[4]);
  }
  if (p->force_order != 0 && p->force_order != 1 && p->force_order != 3 && p->force_order != 4)
    return fail(LBM_EINVAL, "force_order must be 1, 3 or 4 (got %d)", p->force_order);
  if (p->force_order >= 3 && p->collision != LBM_SMRT)
    return fail(LBM_EINVAL, "force_order %d needs the SMRT collision", p->force_order);
  if (p->force_order == 4 && p->lattice == LBM_D3Q39)
    return fail(LBM_EINVAL,
                "force_order 4 needs independent fourth-order moments, which D3Q39 lacks");
  if (p->force_order == 4 && p->max_order == 6)
    return fail(LBM_EINVAL, "force_order 4 is not combined with max_order 6");
  if (p->tau_bulk != 0) {
    if (p->collision != LBM_SMRT)
      return fail(LBM_EINVAL, "tau_bulk needs the SMRT collision");
    if (!(p->tau_bulk > 0.5) || !std::isfinite(p->tau_bulk))
      return fail(LBM_EINVAL, "tau_bulk = %g must exceed 1/2 (or be 0)", p->tau_bulk);
  }
  if (p->max_order != 0 && p->max_order != 4) {
    if (p->max_order != 6)
      return fail(LBM_EINVAL, "max_order = %d: 4 (default) or 6", (int)p->max_order);
    if (p->collision != LBM_SMRT || p->lattice != LBM_D3Q27)
      return fail(LBM_EINVAL, "max_order 6 needs SMRT on D3Q27 (the lattice with orders 5-6)");
  }
  if (p->tau_31 != 0) {
    if (p->collision != LBM_SMRT)
      return fail(LBM_EINVAL, "tau_31 needs the SMRT collision");
    if (p->lattice == LBM_D2Q9)
      return fail(LBM_EINVAL, "tau_31: D2Q9 carries no traceless third-order component");
    if (p->lattice == LBM_D3Q39)
      return fail(LBM_EINVAL, "tau_31 is defined on D3Q19/D3Q27 (D3Q39 carries D_aaa)");
    if (p->force_order >= 3)
      return fail(LBM_EINVAL, "tau_31 is not combined with force_order %d", p->force_order);
    if (!(p->tau_31 > 0.5) || !std::isfinite(p->tau_31))
      return fail(LBM_EINVAL, "tau_31 = %g must exceed 1/2 (or be 0)", p->tau_31);
  }
  if (!(p->rho0 > 0) || !std::isfinite(p->rho0))
    return fail(LBM_EINVAL, "rho0 = %g must be positive", p->rho0);
  if (p->g_kind < LBM_G_UNIFORM || p->g_kind > LBM_G_FIELD)
    return fail(LBM_EINVAL, "unknown force kind %d", p->g_kind);
  if (p->g_kind == LBM_G_PROFILE && (p->g_axis < 0 || p->g_axis > 2))
    return fail(LBM_EINVAL, "profile axis %d", p->g_axis);
  if (p->g_kind != LBM_G_UNIFORM && !p->g_data)
    return fail(LBM_EINVAL, "g_data is NULL for a profile or field force");
  if (p->monitor_every < 0) return fail(LBM_EINVAL, "monitor_every must be >= 0");
  if (!(p->mach_limit >= 0) || !std::isfinite(p->mach_limit))
    return fail(LBM_EINVAL, "mach_limit = %g must be >= 0 (0 = off)", p->mach_limit);
  if (p->debug_poison != 0 && p->debug_poison != 1)
    return fail(LBM_EINVAL, "debug_poison must be 0 or 1");
  if (p->allocator && (!p->allocator->alloc || !p->allocator->free))
    return fail(LBM_EINVAL, "allocator needs both alloc and free");
  return LBM_OK;
}

template <class T>
void convert(const double *src, size_t n, std::vector<unsigned char> &out) {
  out.resize(n * sizeof(T));
  T *o = reinterpret_cast<T *>(out.data());
  for (size_t i = 0; i < n; ++i) o[i] = static_cast<T>(src[i]);
}

void release(lbm_ctx *c) {
  if (!c) return;
  (void)hipStreamSynchronize(c->stream);
  c->dfree(c->buf[0]);
  c->dfree(c->buf[1]);
  c->dfree(c->gtab);
  c->dfree(c->uprev);
  c->dfree(c->smask);
  c->dfree(c->partials);
  c->dfree(c->mon_dev);
  c->dfree(c->scratch);
  if (c->mon_host) (void)hipHostFree(c->mon_host);
  if (c->mon_ev) (void)hipEventDestroy(c->mon_ev);
  c->drop_graphs();
  c->dfree(c->gs_dev);
  c->dfree(c->gs_ctr);
  if (c->gs_host) (void)hipHostFree(c->gs_host);
  if (c->gs_ev) (void)hipEventDestroy(c->gs_ev);
  if (c->cap) (void)hipStreamDestroy(c->cap);
  c->magic = 0;
  delete c;
}

}  // namespace

// Monitor finalisation, the NaN fill and the stream-copy probe (lbm_aux.hip).
namespace lbm {
hipError_t finalize_monitors(const double *partials, int64_t nb, double *out, hipStream_t s);
hipError_t fill_nan(void *p, size_t bytes, hipStream_t s);
hipError_t graph_counter(int64_t *ctr, int64_t add, int set, hipStream_t s);
hipError_t copy_probe(const void *src, void *dst, size_t bytes, int reps, int block,
                      int variant, hipStream_t s);
}  // namespace lbm

namespace {

int refresh_monitors(lbm_ctx *c, int mode) {
  lbm::LaunchDesc d = c->desc(c->last_scale);
  HIP_TRY(c->ops->moments(d, nullptr, nullptr, c->uprev, mode, c->partials, c->stream));
  HIP_TRY(lbm::finalize_monitors(c->partials, c->nblocks, c->mon_dev, c->stream));
  return LBM_OK;
}

// A monitor record from the finalised slots h (lbm_internal.h MON_*) of time t; the
// residual exists only if the pass compared with a recorded previous step (mode 4).
lbm_monitors record_of(const double *h, int64_t t, int mode) {
  lbm_monitors m{};
  m.step = t;
  m.mass = h[lbm::MON_MASS];
  for (int a = 0; a < 3; ++a) {
    m.mom[a] = h[lbm::MON_MX + a];
    m.j[a] = h[lbm::MON_JX + a];
  }
  m.resid = (mode == 4 && h[lbm::MON_U2] > 0) ? std::sqrt(h[lbm::MON_DU2] / h[lbm::MON_U2]) : 0.0;
  m.umax = h[lbm::MON_UMAX];
  m.nonfinite = (int64_t)h[lbm::MON_BAD];
  return m;
}

// What a monitor record reports: LBM_ENONFINITE (sticky until the state is replaced),
// the warning LBM_WMACH, or LBM_OK.
int judge_record(lbm_ctx *c, const lbm_monitors &m) {
  if (m.nonfinite) {
    c->nonfinite_seen = true;
    c->nonfinite_step = m.step;
    return fail(LBM_ENONFINITE, "%lld nodes are not finite at step %lld",
                (long long)m.nonfinite, (long long)m.step);
  }
  const double cs = std::sqrt(cs2_num(c->p.lattice) / 3.0);
  if (c->p.mach_limit > 0 && m.umax > c->p.mach_limit * cs)
    return fail(LBM_WMACH, "max |u| = %g at step %lld exceeds the Mach limit %g c_s", m.umax,
                (long long)m.step, c->p.mach_limit);
  return LBM_OK;
}

// The in-step check at the current time t (a multiple of monitor_every): the record of
// time t on the device, compared with t - 1 when that was recorded, and its copy to the
// pinned host record behind an event.
int in_step_check(lbm_ctx *c) {
  const int mode = (c->uprev_time == c->t - 1) ? 4 : 2;
  int rc = refresh_monitors(c, mode);
  if (rc) return rc;
  c->uprev_time = c->t;
  c->dev_step = c->t;
  c->dev_mode = mode;
  HIP_TRY(hipMemcpyAsync(c->mon_host, c->mon_dev, lbm::MON_SLOTS * sizeof(double),
                         hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(hipEventRecord(c->mon_ev, c->stream));
  c->check_pending = true;
  c->check_step = c->t;
  c->check_mode = mode;
  return LBM_OK;
}

// Read the latest in-step record once it is complete (wait: block until it is).  A
// non-finite state seen before keeps returning LBM_ENONFINITE.
int poll_checks(lbm_ctx *c, bool wait) {
  if (c->nonfinite_seen)
    return fail(LBM_ENONFINITE, "the state had non-finite nodes at step %lld",
                (long long)c->nonfinite_step);
  if (!c->check_pending) return LBM_OK;
  const hipError_t e = wait ? hipEventSynchronize(c->mon_ev) : hipEventQuery(c->mon_ev);
  if (e == hipErrorNotReady) return LBM_OK;
  if (e != hipSuccess)
    return fail(LBM_EDEVICE, "monitor check: %s", hipGetErrorString(e));
  c->check_pending = false;
  const lbm_monitors m = record_of(c->mon_host, c->check_step, c->check_mode);
  c->mon = m;
  return judge_record(c, m);
}

// The state was replaced: no record, residual or non-finite flag carries over.
void state_replaced(lbm_ctx *c) {
  c->uprev_time = -2;
  c->dev_step = -1;
  c->check_pending = false;
  c->nonfinite_seen = false;
  c->mon.step = -1;
}

}  // namespace

namespace {

// Fields -> binary64 planes for the init kernel.  layout 0: planes rho, u; 1: the
// network's point-major rows (u / U, (rho - rho0) / R); 2: the same as planes.
__global__ void fields_to_planes_kernel(const float *in, int layout, int64_t N, int D, double U,
                                        double R, double rho0, double *rho, double *u) {
  const int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (n >= N) return;
  if (layout == 1) {
    const float *row = in + n * (D + 1);
    rho[n] = rho0 + R * (double)row[D];
    for (int c = 0; c < D; ++c) u[c * N + n] = U * (double)row[c];
  } else if (layout == 2) {
    rho[n] = rho0 + R * (double)in[D * N + n];
    for (int c = 0; c < D; ++c) u[c * N + n] = U * (double)in[c * N + n];
  } else {
    rho[n] = (double)in[n];
    for (int c = 0; c < D; ++c) u[c * N + n] = (double)in[N + c * N + n];
  }
}

// Totals for the conservation projection: per block, sum rho, sum rho u_a, sum u_a
// (1 + 2D slots), then one block reduces the partials in block order and writes the
// density shift delta and the velocity shift c_a.
constexpr int CONS_BLOCKS = 512;
constexpr int CONS_SLOTS = 7;

__global__ void __launch_bounds__(256) conserve_partials_kernel(const double *rho, const double *u,
                                                                int64_t N, int D, double *part) {
  double v[CONS_SLOTS] = {-0.0, -0.0, -0.0, -0.0, -0.0, -0.0, -0.0};
  for (int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; n < N;
       n += (int64_t)gridDim.x * blockDim.x) {
    const double r = rho[n];
    v[0] += r;
    for (int a = 0; a < D; ++a) {
      const double ua = u[a * N + n];
      v[1 + a] += r * ua;
      v[1 + D + a] += ua;
    }
  }
  __shared__ double red[CONS_SLOTS][4];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  for (int k = 0; k < 1 + 2 * D; ++k) {
    double w = v[k];
    for (int o = 32; o > 0; o >>= 1) w += __shfl_xor(w, o, 64);
    if (lane == 0) red[k][wave] = w;
  }
  __syncthreads();
  if (threadIdx.x < 1 + 2 * D) {
    const int k = threadIdx.x;
    part[(int64_t)blockIdx.x * CONS_SLOTS + k] = ((red[k][0] + red[k][1]) + red[k][2]) + red[k][3];
  }
}

// shift[0] = delta, shift[1 + a] = c_a such that rho' = rho + delta, u' = u - c give
// sum rho' = N rho0 (mass) and sum rho' u' = 0 (momentum), each only if requested.
__global__ void conserve_finalize_kernel(const double *part, int nb, int64_t N, int D,
                                         double rho0, int flags, double *shift) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  double t[CONS_SLOTS] = {-0.0, -0.0, -0.0, -0.0, -0.0, -0.0, -0.0};
  for (int b = 0; b < nb; ++b)
    for (int k = 0; k < 1 + 2 * D; ++k) t[k] += part[(int64_t)b * CONS_SLOTS + k];
  const double delta = (flags & LBM_RESET_MASS) ? ((double)N * rho0 - t[0]) / (double)N : 0.0;
  shift[0] = delta;
  const double mass = t[0] + (double)N * delta;
  for (int a = 0; a < D; ++a)
    shift[1 + a] = (flags & LBM_RESET_MOMENTUM) ? (t[1 + a] + delta * t[1 + D + a]) / mass : 0.0;
}

// One pass of the periodic 7-point low-pass filter (transfer 1 - sin^6(k/2)) along one
// axis of nplanes planes nx x ny x nz (x fastest); the offsets are summed in a fixed
// order, each wrapped periodically (any axis length, also below 7).
__global__ void filter_axis_kernel(const double *in, double *out, int nx, int ny, int nz,
                                   int axis, int nplanes) {
  const int64_t N = (int64_t)nx * ny * nz;
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= N * nplanes) return;
  const int64_t pl = idx / N, n = idx - pl * N;
  const int x = (int)(n % nx), y = (int)((n / nx) % ny), z = (int)(n / ((int64_t)nx * ny));
  const int len = axis == 0 ? nx : axis == 1 ? ny : nz;
  const int pos = axis == 0 ? x : axis == 1 ? y : z;
  const int64_t stride = axis == 0 ? 1 : axis == 1 ? nx : (int64_t)nx * ny;
  const double *src = in + pl * N + (n - (int64_t)pos * stride);
  const double c[4] = {11.0 / 16.0, 15.0 / 64.0, -3.0 / 32.0, 1.0 / 64.0};
  double acc = c[0] * src[(int64_t)pos * stride];
  for (int o = 1; o <= 3; ++o) {
    const int lo = ((pos - o) % len + len) % len, hi = (pos + o) % len;
    acc += c[o] * (src[(int64_t)lo * stride] + src[(int64_t)hi * stride]);
  }
  out[idx] = acc;
}

// Non-equilibrium second moment of a start state, to leading (Chapman-Enskog) order:
// Pi_ab = -c_s^2 tau2 rho (d_a u_b + d_b u_a), planes xx, yy, zz, xy, xz, yz.  Central
// differences of unit spacing, one-sided at the faces of walled axes, zero along axes of
// length 1.
__global__ void strain_kernel(const double *rho, const double *u, int nx, int ny, int nz, int D,
                              int wx, int wy, int wz, double coef, double *pi) {
  const int64_t N = (int64_t)nx * ny * nz;
  const int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (n >= N) return;
  const int p[3] = {(int)(n % nx), (int)((n / nx) % ny), (int)(n / ((int64_t)nx * ny))};
  const int len[3] = {nx, ny, nz};
  const int wall[3] = {wx, wy, wz};
  const int64_t stride[3] = {1, nx, (int64_t)nx * ny};
  double g[3][3];  // g[a][b] = d_b u_a
  for (int b = 0; b < 3; ++b) {
    int lo = p[b] - 1, hi = p[b] + 1;
    double h = 0.5;
    if (len[b] == 1) {
      for (int a = 0; a < 3; ++a) g[a][b] = 0.0;
      continue;
    }
    if (wall[b]) {
      if (lo < 0) { lo = p[b]; h = 1.0; }
      if (hi >= len[b]) { hi = p[b]; h = 1.0; }
    } else {
      lo = (lo + len[b]) % len[b];
      hi = hi % len[b];
    }
    const int64_t nl = n + (int64_t)(lo - p[b]) * stride[b];
    const int64_t nh = n + (int64_t)(hi - p[b]) * stride[b];
    for (int a = 0; a < 3; ++a)
      g[a][b] = a < D ? h * (u[a * N + nh] - u[a * N + nl]) : 0.0;
  }
  const double c = coef * rho[n];
  pi[0 * N + n] = c * (g[0][0] + g[0][0]);
  pi[1 * N + n] = c * (g[1][1] + g[1][1]);
  pi[2 * N + n] = c * (g[2][2] + g[2][2]);
  pi[3 * N + n] = c * (g[0][1] + g[1][0]);
  pi[4 * N + n] = c * (g[0][2] + g[2][0]);
  pi[5 * N + n] = c * (g[1][2] + g[2][1]);
}

__global__ void conserve_apply_kernel(double *rho, double *u, int64_t N, int D,
                                      const double *shift) {
  const int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (n >= N) return;
  rho[n] += shift[0];
  for (int a = 0; a < D; ++a) u[a * N + n] -= shift[1 + a];
}

}  // namespace

extern "C" {

int lbm_version(void) { return 100; }

int lbm_lattice_info(int32_t lattice, int32_t *D, int32_t *Q, int32_t *e, double *w) {
  if (lattice < LBM_D2Q9 || lattice > LBM_D3Q39)
    return fail(LBM_EINVAL, "unknown lattice %d", (int)lattice);
  const lbm::LatticeOps &ops = lbm::ops_for(lattice);
  if (D) *D = ops.D;
  if (Q) *Q = ops.Q;
  for (int i = 0; i < ops.Q; ++i) {
    if (e)
      for (int a = 0; a < 3; ++a) e[3 * i + a] = ops.E[3 * i + a];
    if (w) w[i] = ops.W[i];
  }
  return LBM_OK;
}

const char *lbm_strerror(int status) {
  switch (status) {
    case LBM_OK: return "ok";
    case LBM_WMACH: return "warning: max |u| exceeds the Mach limit";
    case LBM_EINVAL: return "invalid argument";
    case LBM_ENOMEM: return "out of memory";
    case LBM_EDEVICE: return "device error";
    case LBM_ENONFINITE: return "non-finite value in the state";
    case LBM_ESTATE: return "invalid context";
    default: return "unknown status";
  }
}

const char *lbm_last_error(void) { return g_last_error.c_str(); }

int lbm_init(const lbm_params *p, const double *rho_init, const double *u_init, void *hip_stream,
             lbm_ctx **out) {
  if (!out) return fail(LBM_EINVAL, "out is NULL");
  *out = nullptr;
  int rc = validate(p);
  if (rc) return rc;
  int device = 0;
  if (hipGetDevice(&device) != hipSuccess) return fail(LBM_EDEVICE, "no current HIP device");
  if ((rc = noalloc_scratch_setup(device))) return rc;
  lbm_ctx *c = new (std::nothrow) lbm_ctx();
  if (!c) return fail(LBM_ENOMEM, "host allocation of the context failed");
  c->device = device;
  if (hipDeviceGetAttribute(&c->lds_cu, hipDeviceAttributeMaxSharedMemoryPerMultiprocessor,
                            device) != hipSuccess ||
      hipDeviceGetAttribute(&c->lds_block, hipDeviceAttributeMaxSharedMemoryPerBlock, device) !=
          hipSuccess) {
    c->lds_cu = 0;  // no occupancy caps
    c->lds_block = 0;
  }
  c->p = *p;
  c->p.g_data = nullptr;
  if (p->allocator) c->alloc = *p->allocator;
  c->ops = &ops_for(p->lattice);
  c->D = c->ops->D;
  c->Q = c->ops->Q;
  c->N = (int64_t)p->nx * p->ny * p->nz;
  c->stream = static_cast<hipStream_t>(hip_stream);
  c->shift = shifted(p->storage) ? p->rho0 : 0.0;
  if (p->collision == LBM_BGK) {
    const double om = 1.0 / p->tau[2];
    c->c0 = om;
    c->c1 = 1.0 - 0.5 * om;
  } else {
    c->c0 = 1.0 - 1.0 / p->tau[2];
    c->c1 = 1.0 - 1.0 / p->tau[3];
    if (p->collision == LBM_RMRT) {
      c->c2 = 1.0 - 0.5 / p->tau[2];
      c->c3 = 1.0 - 0.5 / p->tau[3];
    } else {
      if (p->force_order >= 3) c->c2 = 1.0 - 0.5 / p->tau[3];
      if (p->tau_bulk != 0 && p->tau_bulk != p->tau[2])
        c->c3 = ((1.0 - 1.0 / p->tau_bulk) - (1.0 - 1.0 / p->tau[2])) / c->D;
      if (p->tau_31 != 0 && p->tau_31 != p->tau[3])
        c->c4 = ((1.0 - 1.0 / p->tau_31) - (1.0 - 1.0 / p->tau[3])) / 2;
    }
  }
  block_shape(p->nx, c->bx, c->by);
  const dim3 grid((p->nx + c->bx - 1) / c->bx, (p->ny + c->by - 1) / c->by, p->nz);
  c->nblocks = (int64_t)grid.x * grid.y * grid.z;
  c->nblocks_cap = c->nblocks;

  const size_t pop_bytes = (size_t)c->Q * (size_t)c->N * storage_bytes(p->storage);
  const size_t ab = arith_bytes(p->storage);
  // force table, in the arithmetic type
  std::vector<double> gh;
  if (p->g_kind == LBM_G_UNIFORM) {
    c->g_axis = -1;
    c->g_n = 1;
    gh.assign(p->g_uniform, p->g_uniform + 3);
  } else if (p->g_kind == LBM_G_PROFILE) {
    c->g_axis = p->g_axis;
    c->g_n = p->g_axis == 0 ? p->nx : (p->g_axis == 1 ? p->ny : p->nz);
    gh.assign(p->g_data, p->g_data + 3 * (size_t)c->g_n);
  } else {
    c->gk = 1;
    c->g_axis = -1;
    c->g_n = (int)c->N;
    gh.assign(p->g_data, p->g_data + 3 * (size_t)c->N);
  }
  for (double v : gh)
    if (!std::isfinite(v)) {
      delete c;
      return fail(LBM_EINVAL, "non-finite acceleration value");
    }
  std::vector<unsigned char> gconv;
  if (ab == 8)
    convert<double>(gh.data(), gh.size(), gconv);
  else
    convert<float>(gh.data(), gh.size(), gconv);
  c->g_hash = fnv1a(kFnvBasis, gconv.data(), gconv.size());
  if (p->solid) {
    const int walls[3] = {p->bc[0] == LBM_WALLS, p->bc[1] == LBM_WALLS, p->bc[2] == LBM_WALLS};
    c->smask_host.resize((size_t)c->N);
    c->ops->solid_words(p->solid, p->nx, p->ny, p->nz, walls, c->smask_host.data());
    int64_t fluid = 0;
    for (uint32_t w : c->smask_host) fluid += (w & lbm::SOLID_NODE) ? 0 : 1;
    if (fluid == 0) {
      delete c;
      return fail(LBM_EINVAL, "every node is solid");
    }
  }

  if ((rc = c->dalloc(&c->buf[0], pop_bytes)) || (rc = c->dalloc(&c->buf[1], pop_bytes)) ||
      (rc = c->dalloc(&c->gtab, gconv.size())) ||
      (p->solid && (rc = c->dalloc((void **)&c->smask, (size_t)c->N * sizeof(uint32_t)))) ||
      (rc = c->dalloc(&c->uprev, 3 * (size_t)c->N * ab)) ||
      (rc = c->dalloc((void **)&c->partials,
                      (size_t)c->nblocks * lbm::MON_SLOTS * sizeof(double))) ||
      (rc = c->dalloc((void **)&c->mon_dev, lbm::MON_SLOTS * sizeof(double)))) {
    std::string msg = g_last_error;
    release(c);
    return fail(rc, "%s", msg.c_str());
  }
  if (p->monitor_every > 0) {
    if (hipHostMalloc((void **)&c->mon_host, lbm::MON_SLOTS * sizeof(double),
                      hipHostMallocDefault) != hipSuccess) {
      c->mon_host = nullptr;
      release(c);
      return fail(LBM_ENOMEM, "pinned host memory for the monitor record");
    }
    if (hipEventCreateWithFlags(&c->mon_ev, hipEventDisableTiming) != hipSuccess) {
      c->mon_ev = nullptr;
      release(c);
      return fail(LBM_EDEVICE, "creating the monitor event failed");
    }
  }
  auto bail = [&](int code) {
    std::string msg = g_last_error;
    release(c);
    return fail(code, "%s", msg.c_str());
  };
  if (hipMemcpyAsync(c->gtab, gconv.data(), gconv.size(), hipMemcpyHostToDevice, c->stream) !=
      hipSuccess)
    return bail(fail(LBM_EDEVICE, "uploading the force table failed"));
  if (c->smask &&
      hipMemcpyAsync(c->smask, c->smask_host.data(), c->smask_host.size() * sizeof(uint32_t),
                     hipMemcpyHostToDevice, c->stream) != hipSuccess)
    return bail(fail(LBM_EDEVICE, "uploading the solid mask failed"));
  // upload initial fields
  const size_t fld = (size_t)c->N * sizeof(double);
  if ((rho_init || u_init) && (rc = c->need_scratch(fld * (1 + c->D)))) return bail(rc);
  double *rho_d = nullptr, *u_d = nullptr;
  if (rho_init) {
    for (int64_t n = 0; n < c->N; ++n)
      if (!(rho_init[n] > 0) || !std::isfinite(rho_init[n]))
        return bail(fail(LBM_EINVAL, "rho_init[%lld] = %g is not a positive finite density",
                         (long long)n, rho_init[n]));
    rho_d = static_cast<double *>(c->scratch);
    if (hipMemcpyAsync(rho_d, rho_init, fld, hipMemcpyHostToDevice, c->stream) != hipSuccess)
      return bail(fail(LBM_EDEVICE, "uploading rho_init failed"));
  }
  if (u_init) {
    for (int64_t n = 0; n < (int64_t)c->D * c->N; ++n)
      if (!std::isfinite(u_init[n])) return bail(fail(LBM_EINVAL, "non-finite u_init value"));
    u_d = reinterpret_cast<double *>(static_cast<char *>(c->scratch) + fld);
    if (hipMemcpyAsync(u_d, u_init, fld * c->D, hipMemcpyHostToDevice, c->stream) != hipSuccess)
      return bail(fail(LBM_EDEVICE, "uploading u_init failed"));
  }
  lbm::LaunchDesc d = c->desc(1.0);
  d.fout = c->buf[0];
  if (c->ops->init(d, rho_d, u_d, p->rho0, nullptr, c->stream) != hipSuccess)
    return bail(fail(LBM_EDEVICE, "init kernel launch failed"));
  if (hipStreamSynchronize(c->stream) != hipSuccess)
    return bail(fail(LBM_EDEVICE, "init failed: %s", hipGetErrorString(hipGetLastError())));
  c->cur = 0;
  c->t = 0;
  c->mon.step = -1;
  *out = c;
  return LBM_OK;
}

namespace {

constexpr int kGraphChunk = 64;             // steps per captured graph (even)
constexpr int64_t kGraphMaxNodes = 1 << 21;  // larger lattices are not launch-bound

// Whether n steps of c run as graph replays: a small lattice, at least two chunks, no
// in-step monitors or poison pass.
bool graph_steps(const lbm_ctx *c, int64_t n) {
  return c->N <= kGraphMaxNodes && n >= 2 * kGraphChunk && c->p.monitor_every == 0 &&
         !c->p.debug_poison;
}

// The graph of one chunk from the current buffer, with device force factors (scaled) or
// s(t) = 1; captured once per (parity, scaled).
int chunk_graph(lbm_ctx *c, bool scaled, hipGraphExec_t *out) {
  hipGraphExec_t &e = c->gexec[c->cur][scaled];
  if (e) {
    *out = e;
    return LBM_OK;
  }
  if (!c->cap) HIP_TRY(hipStreamCreateWithFlags(&c->cap, hipStreamNonBlocking));
  if (!c->gs_ctr) {
    int rc = c->dalloc((void **)&c->gs_ctr, sizeof(int64_t));
    if (rc) return rc;
  }
  HIP_TRY(hipStreamBeginCapture(c->cap, hipStreamCaptureModeThreadLocal));
  hipError_t err = hipSuccess;
  int cur = c->cur;
  for (int j = 0; j < kGraphChunk && err == hipSuccess; ++j) {
    const int saved = c->cur;
    c->cur = cur;
    lbm::LaunchDesc d = c->desc(1.0);
    c->cur = saved;
    if (scaled) {
      d.gs_dev = c->gs_dev;
      d.gs_ctr = c->gs_ctr;
      d.gs_j = j;
    }
    err = c->ops->step(d, c->cap);
    cur ^= 1;
  }
  if (err == hipSuccess && scaled) err = lbm::graph_counter(c->gs_ctr, kGraphChunk, 0, c->cap);
  hipGraph_t g = nullptr;
  const hipError_t ec = hipStreamEndCapture(c->cap, &g);
  if (err == hipSuccess) err = ec;
  if (err == hipSuccess) err = hipGraphInstantiate(&e, g, nullptr, nullptr, 0);
  if (g) (void)hipGraphDestroy(g);
  if (err != hipSuccess) {
    e = nullptr;
    return fail(LBM_EDEVICE, "capturing the step graph: %s", hipGetErrorString(err));
  }
  *out = e;
  return LBM_OK;
}

// n >= 2 kGraphChunk steps as graph replays plus the remainder launched one by one.
int graph_run(lbm_ctx *c, int64_t n, const double *g_scale) {
  const bool scaled = g_scale != nullptr;
  if (scaled) {
    const size_t need = (size_t)n * sizeof(double);
    if (need > c->gs_cap) {
      HIP_TRY(hipStreamSynchronize(c->stream));  // the old table may still be read
      c->drop_graphs();                          // the graphs hold its address
      c->dfree(c->gs_dev);
      c->bytes -= c->gs_cap;
      c->gs_dev = nullptr;
      c->gs_cap = 0;
      int rc = c->dalloc((void **)&c->gs_dev, need);
      if (rc) return rc;
      c->gs_cap = need;
    }
    // stage the factors in pinned memory and upload them without blocking: the copy is
    // ordered after the replays of earlier calls that read gs_dev, and the staging buffer
    // is rewritten only after the previous upload from it has completed
    if (!c->gs_ev) HIP_TRY(hipEventCreateWithFlags(&c->gs_ev, hipEventDisableTiming));
    else HIP_TRY(hipEventSynchronize(c->gs_ev));
    if (need > c->gs_host_cap) {
      if (c->gs_host) HIP_TRY(hipHostFree(c->gs_host));
      c->gs_host = nullptr;
      c->gs_host_cap = 0;
      if (hipHostMalloc((void **)&c->gs_host, need, hipHostMallocDefault) != hipSuccess) {
        c->gs_host = nullptr;
        return fail(LBM_ENOMEM, "pinned staging of %zu bytes of force factors", need);
      }
      c->gs_host_cap = need;
    }
    std::memcpy(c->gs_host, g_scale, need);
    HIP_TRY(hipMemcpyAsync(c->gs_dev, c->gs_host, need, hipMemcpyHostToDevice, c->stream));
    HIP_TRY(hipEventRecord(c->gs_ev, c->stream));
  }
  hipGraphExec_t e = nullptr;
  int rc = chunk_graph(c, scaled, &e);
  if (rc) return rc;
  if (scaled) HIP_TRY(lbm::graph_counter(c->gs_ctr, 0, 1, c->stream));
  const int64_t reps = n / kGraphChunk;
  for (int64_t r = 0; r < reps; ++r) HIP_TRY(hipGraphLaunch(e, c->stream));
  c->t += reps * kGraphChunk;  // kGraphChunk is even: the current buffer is unchanged
  int64_t s = reps * kGraphChunk;
  for (; s < n; ++s) {
    const double sc = scaled ? g_scale[s] : 1.0;
    HIP_TRY(c->ops->step(c->desc(sc), c->stream));
    c->cur ^= 1;
    c->t += 1;
  }
  c->last_scale = scaled ? g_scale[n - 1] : 1.0;
  return LBM_OK;
}

}  // namespace

int lbm_step(lbm_ctx *c, int64_t n, const double *g_scale) {
  if (!valid(c)) return fail(LBM_ESTATE, "invalid context");
  if (n < 0) return fail(LBM_EINVAL, "negative step count");
  if (g_scale)
    for (int64_t s = 0; s < n; ++s)
      if (!std::isfinite(g_scale[s]))
        return fail(LBM_EINVAL, "g_scale[%lld] is not finite", (long long)s);
  // a completed in-step record: a non-finite state stops here, a Mach warning is
  // returned after the steps are enqueued
  const int seen = poll_checks(c, false);
  if (seen < 0) return seen;
  if (graph_steps(c, n)) {
    const int rc = graph_run(c, n, g_scale);
    return rc ? rc : seen;
  }
  const int K = c->p.monitor_every;
  const size_t pop_bytes = (size_t)c->Q * c->N * storage_bytes(c->p.storage);
  for (int64_t s = 0; s < n; ++s) {
    const double sc = g_scale ? g_scale[s] : 1.0;
    if (c->p.debug_poison) HIP_TRY(lbm::fill_nan(c->buf[c->cur ^ 1], pop_bytes, c->stream));
    lbm::LaunchDesc d = c->desc(sc);
    HIP_TRY(c->ops->step(d, c->stream));
    c->cur ^= 1;
    c->t += 1;
    c->last_scale = sc;
    if (K > 0) {
      if (c->t % K == 0) {
        int rc = in_step_check(c);
        if (rc) return rc;
      } else if ((c->t + 1) % K == 0) {
        // the velocity of the step before a check, for its residual
        int rc = refresh_monitors(c, 2 /* record */);
        if (rc) return rc;
        c->uprev_time = c->t;
      }
    }
  }
  return seen;
}

int lbm_monitors_get(lbm_ctx *c, lbm_monitors *mon) {
  if (!valid(c)) return fail(LBM_ESTATE, "invalid context");
  if (!mon) return fail(LBM_EINVAL, "mon is NULL");
  int mode;
  if (c->dev_step == c->t) {
    // the in-step check of this time holds the record (refreshing it now would compare
    // the state with itself)
    mode = c->dev_mode;
  } else {
    mode = (c->uprev_time == c->t - 1) ? 4 : 2;
    int rc = refresh_monitors(c, mode);
    if (rc) return rc;
    c->uprev_time = c->t;
    c->dev_step = c->t;
    c->dev_mode = mode;
  }
  double h[lbm::MON_SLOTS];
  HIP_TRY(hipMemcpyAsync(h, c->mon_dev, sizeof(h), hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(hipStreamSynchronize(c->stream));
  c->check_pending = false;  // this record is the latest
  const lbm_monitors m = record_of(h, c->t, mode);
  c->mon = m;
  *mon = m;
  return judge_record(c, m);
}

int lbm_moments(lbm_ctx *c, double g_scale, double *rho, double *u) {
  if (!valid(c)) return fail(LBM_ESTATE, "invalid context");
  if (!std::isfinite(g_scale)) return fail(LBM_EINVAL, "g_scale is not finite");
  const size_t fld = (size_t)c->N * sizeof(double);
  int rc = c->need_scratch(fld * (1 + c->D));
  if (rc) return rc;
  double *rho_d = static_cast<double *>(c->scratch);
  double *u_d = reinterpret_cast<double *>(static_cast<char *>(c->scratch) + fld);
  lbm::LaunchDesc d = c->desc(g_scale);
  HIP_TRY(c->ops->moments(d, rho_d, u_d, nullptr, 1, nullptr, c->stream));
  if (rho) HIP_TRY(hipMemcpyAsync(rho, rho_d, fld, hipMemcpyDeviceToHost, c->stream));
  if (u) HIP_TRY(hipMemcpyAsync(u, u_d, fld * c->D, hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(hipStreamSynchronize(c->stream));
  return poll_checks(c, true);
}

int lbm_get_populations(lbm_ctx *c, int64_t nnodes, const int64_t *nodes, double *out) {
  if (!valid(c)) return fail(LBM_ESTATE, "invalid context");
  if (!out) return fail(LBM_EINVAL, "out is NULL");
  if (!nodes && nnodes != c->N) return fail(LBM_EINVAL, "nodes NULL requires nnodes == N");
  if (nnodes < 0) return fail(LBM_EINVAL, "negative node count");
  if (nnodes == 0) return LBM_OK;
  if (nodes)
    for (int64_t j = 0; j < nnodes; ++j)
      if (nodes[j] < 0 || nodes[j] >= c->N)
        return fail(LBM_EINVAL, "node index %lld out of range", (long long)nodes[j]);
  const size_t outb = (size_t)c->Q * nnodes * sizeof(double);
  const size_t idxb = nodes ? (size_t)nnodes * sizeof(int64_t) : 0;
  int rc = c->need_scratch(outb + idxb);
  if (rc) return rc;
  double *out_d = static_cast<double *>(c->scratch);
  int64_t *idx_d = nodes ? reinterpret_cast<int64_t *>(static_cast<char *>(c->scratch) + outb)
                         : nullptr;
  if (nodes) HIP_TRY(hipMemcpyAsync(idx_d, nodes, idxb, hipMemcpyHostToDevice, c->stream));
  lbm::LaunchDesc d = c->desc(1.0);
  HIP_TRY(c->ops->gather(d, idx_d, nnodes, out_d, c->stream));
  HIP_TRY(hipMemcpyAsync(out, out_d, outb, hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(hipStreamSynchronize(c->stream));
  return poll_checks(c, true);
}

int lbm_get_populations_noalloc(lbm_ctx *c, int64_t nnodes, const int64_t *nodes, double *out) {
  if (!valid(c)) return fail(LBM_ESTATE, "invalid context");
  if (!out) return fail(LBM_EINVAL, "out is NULL");
  if (!nodes && nnodes != c->N) return fail(LBM_EINVAL, "nodes NULL requires nnodes == N");
  if (nnodes < 0) return fail(LBM_EINVAL, "negative node count");
  if (nnodes == 0) return LBM_OK;
  const size_t outb = (size_t)c->Q * (size_t)nnodes * sizeof(double);
  const size_t idxb = nodes ? (size_t)nnodes * sizeof(int64_t) : 0;
  if ((uint64_t)nnodes > (uint64_t)LBM_NOALLOC_SCRATCH_BYTES / sizeof(double) ||
      outb + idxb > (size_t)LBM_NOALLOC_SCRATCH_BYTES)
    return fail(LBM_EINVAL,
                "%lld nodes need %zu bytes of staging, beyond the %d bytes of the no-alloc "
                "scratch (at most %lld nodes of this lattice)",
                (long long)nnodes, outb + idxb, LBM_NOALLOC_SCRATCH_BYTES,
                (long long)(LBM_NOALLOC_SCRATCH_BYTES / ((c->Q + 1) * sizeof(double))));
  if (nodes)
    for (int64_t j = 0; j < nnodes; ++j)
      if (nodes[j] < 0 || nodes[j] >= c->N)
        return fail(LBM_EINVAL, "node index %lld out of range", (long long)nodes[j]);
  char *base = static_cast<char *>(noalloc_scratch_of(c->device));
  if (!base) return fail(LBM_ESTATE, "no-alloc scratch not set up on device %d", c->device);
  double *out_d = reinterpret_cast<double *>(base);
  int64_t *idx_d = nodes ? reinterpret_cast<int64_t *>(base + outb) : nullptr;
  if (nodes) HIP_TRY(hipMemcpyAsync(idx_d, nodes, idxb, hipMemcpyHostToDevice, c->stream));
  lbm::LaunchDesc d = c->desc(1.0);
  HIP_TRY(c->ops->gather(d, idx_d, nnodes, out_d, c->stream));
  HIP_TRY(hipMemcpyAsync(out, out_d, outb, hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(hipStreamSynchronize(c->stream));
  return poll_checks(c, true);
}

int lbm_set_populations(lbm_ctx *c, const double *f) {
  if (!valid(c)) return fail(LBM_ESTATE, "invalid context");
  if (!f) return fail(LBM_EINVAL, "f is NULL");
  const size_t inb = (size_t)c->Q * c->N * sizeof(double);
  int rc = c->need_scratch(inb);
  if (rc) return rc;
  HIP_TRY(hipMemcpyAsync(c->scratch, f, inb, hipMemcpyHostToDevice, c->stream));
  lbm::LaunchDesc d = c->desc(1.0);
  d.fout = c->buf[c->cur];
  HIP_TRY(c->ops->scatter(d, static_cast<const double *>(c->scratch), c->stream));
  // the host array may be released once this returns
  HIP_TRY(hipStreamSynchronize(c->stream));
  c->t = 0;
  state_replaced(c);
  return LBM_OK;
}

int lbm_set_waves(lbm_ctx *c, int32_t nwaves, const int32_t *k, const double *phase,
                  const double *amp) {
  if (!valid(c)) return fail(LBM_ESTATE, "invalid context");
  if (nwaves < 0 || nwaves > LBM_MAX_WAVES)
    return fail(LBM_EINVAL, "nwaves = %d must be in 0..%d", (int)nwaves, LBM_MAX_WAVES);
  if (nwaves > 0 && (!k || !phase || !amp)) return fail(LBM_EINVAL, "k, phase or amp is NULL");
  for (int64_t j = 0; j < (int64_t)2 * c->Q * nwaves; ++j)
    if (!std::isfinite(amp[j])) return fail(LBM_EINVAL, "amp[%lld] is not finite", (long long)j);
  for (int w = 0; w < nwaves; ++w)
    if (!std::isfinite(phase[w])) return fail(LBM_EINVAL, "phase[%d] is not finite", w);
  // device copies: amp (binary64), phase, then k (int32)
  const size_t ab = (size_t)2 * c->Q * nwaves * sizeof(double);
  const size_t pb = (size_t)nwaves * sizeof(double);
  const size_t kb = (size_t)3 * nwaves * sizeof(int32_t);
  int rc = c->need_scratch(ab + pb + kb + 8);
  if (rc) return rc;
  char *base = static_cast<char *>(c->scratch);
  double *amp_d = reinterpret_cast<double *>(base);
  double *phase_d = reinterpret_cast<double *>(base + ab);
  int32_t *k_d = reinterpret_cast<int32_t *>(base + ab + pb);
  if (nwaves > 0) {
    HIP_TRY(hipMemcpyAsync(amp_d, amp, ab, hipMemcpyHostToDevice, c->stream));
    HIP_TRY(hipMemcpyAsync(phase_d, phase, pb, hipMemcpyHostToDevice, c->stream));
    HIP_TRY(hipMemcpyAsync(k_d, k, kb, hipMemcpyHostToDevice, c->stream));
  }
  lbm::LaunchDesc d = c->desc(1.0);
  d.fout = c->buf[c->cur];
  HIP_TRY(c->ops->waves(d, nwaves, k_d, phase_d, amp_d, c->p.rho0 - c->shift, c->stream));
  // the host arrays may be released once this returns
  HIP_TRY(hipStreamSynchronize(c->stream));
  c->t = 0;
  state_replaced(c);
  return LBM_OK;
}

int lbm_reset_fields(lbm_ctx *c, const float *fields_dev, int32_t layout, double U, double R,
                     int32_t flags) {
  if (!valid(c)) return fail(LBM_ESTATE, "invalid context");
  if (!fields_dev) return fail(LBM_EINVAL, "fields_dev is NULL");
  if (layout < 0 || layout > 2) return fail(LBM_EINVAL, "unknown field layout %d", layout);
  if (layout && !(std::isfinite(U) && U > 0 && std::isfinite(R) && R > 0))
    return fail(LBM_EINVAL, "U and R must be positive");
  if (flags & ~(LBM_RESET_MASS | LBM_RESET_MOMENTUM | LBM_RESET_FILTER | LBM_RESET_NONEQ))
    return fail(LBM_EINVAL, "unknown reset flags 0x%x", (unsigned)flags);
  const int nplanes = 1 + c->D;
  const int64_t N = c->N;
  const bool filter = flags & LBM_RESET_FILTER;
  const bool conserve = flags & (LBM_RESET_MASS | LBM_RESET_MOMENTUM);
  const bool noneq = flags & LBM_RESET_NONEQ;
  // scratch (binary64): planes A (rho, u), the filter's second copy B, the
  // non-equilibrium moment (6 planes), the conservation partials and shifts
  const size_t nA = (size_t)nplanes * N, nB = filter ? nA : 0, nP = noneq ? (size_t)6 * N : 0;
  const size_t nC = conserve ? (size_t)(CONS_BLOCKS + 1) * CONS_SLOTS : 0;
  int rc = c->need_scratch((nA + nB + nP + nC) * sizeof(double));
  if (rc) return rc;
  double *A = static_cast<double *>(c->scratch);
  double *B = A + nA;
  double *P = B + nB;
  double *part = P + nP;
  const unsigned grid = (unsigned)((N + 255) / 256);
  hipLaunchKernelGGL(fields_to_planes_kernel, dim3(grid), dim3(256), 0, c->stream, fields_dev,
                     layout, N, c->D, U, R, c->p.rho0, A, A + N);
  HIP_TRY(hipGetLastError());
  double *cur = A;
  if (filter) {
    const int dims[3] = {c->p.nx, c->p.ny, c->p.nz};
    const unsigned fgrid = (unsigned)((N * nplanes + 255) / 256);
    for (int axis = 0; axis < 3; ++axis) {
      if (c->p.bc[axis] != LBM_PERIODIC || dims[axis] == 1) continue;
      double *dst = cur == A ? B : A;
      hipLaunchKernelGGL(filter_axis_kernel, dim3(fgrid), dim3(256), 0, c->stream, cur, dst,
                         c->p.nx, c->p.ny, c->p.nz, axis, nplanes);
      HIP_TRY(hipGetLastError());
      cur = dst;
    }
  }
  double *rho_d = cur, *u_d = cur + N;
  if (conserve) {
    double *shift = part + (size_t)CONS_BLOCKS * CONS_SLOTS;
    hipLaunchKernelGGL(conserve_partials_kernel, dim3(CONS_BLOCKS), dim3(256), 0, c->stream, rho_d,
                       u_d, N, c->D, part);
    hipLaunchKernelGGL(conserve_finalize_kernel, dim3(1), dim3(64), 0, c->stream, part,
                       CONS_BLOCKS, N, c->D, c->p.rho0, (int)flags, shift);
    hipLaunchKernelGGL(conserve_apply_kernel, dim3(grid), dim3(256), 0, c->stream, rho_d, u_d, N,
                       c->D, shift);
    HIP_TRY(hipGetLastError());
  }
  if (noneq) {
    hipLaunchKernelGGL(strain_kernel, dim3(grid), dim3(256), 0, c->stream, rho_d, u_d, c->p.nx,
                       c->p.ny, c->p.nz, c->D, c->p.bc[0] == LBM_WALLS, c->p.bc[1] == LBM_WALLS,
                       c->p.bc[2] == LBM_WALLS, -(c->p.tau[2] * cs2_num(c->p.lattice)) / 3.0, P);
    HIP_TRY(hipGetLastError());
  }
  c->cur = 0;
  lbm::LaunchDesc d = c->desc(1.0);
  d.fout = c->buf[0];
  HIP_TRY(c->ops->init(d, rho_d, u_d, c->p.rho0, noneq ? P : nullptr, c->stream));
  c->t = 0;
  state_replaced(c);
  return LBM_OK;
}

int lbm_time(const lbm_ctx *c, int64_t *t) {
  if (!valid(c)) return fail(LBM_ESTATE, "invalid context");
  if (!t) return fail(LBM_EINVAL, "t is NULL");
  *t = c->t;
  return LBM_OK;
}

int lbm_device_bytes(const lbm_ctx *c, size_t *bytes) {
  if (!valid(c)) return fail(LBM_ESTATE, "invalid context");
  if (!bytes) return fail(LBM_EINVAL, "bytes is NULL");
  *bytes = c->bytes;
  return LBM_OK;
}

int lbm_free(lbm_ctx *c) {
  if (!valid(c)) return fail(LBM_ESTATE, "invalid context");
  release(c);
  return LBM_OK;
}

namespace {

constexpr char kCkptMagic[8] = {'L', 'B', 'M', 'C', 'K', 'P', 'T', '1'};
constexpr uint32_t kCkptVersion = 2;  // 2: z-slab population layout

// Everything the dynamics of a context depend on, besides its state and time.
uint64_t params_hash(const lbm_ctx *c) {
  const lbm_params &p = c->p;
  uint64_t h = kFnvBasis;
  const int32_t ints[] = {p.lattice, p.collision, p.storage, p.nx,     p.ny,     p.nz,
                          p.bc[0],   p.bc[1],     p.bc[2],   p.g_kind, p.g_axis,
                          p.force_order >= 3 ? p.force_order : 1, p.max_order == 6 ? 6 : 4};
  h = fnv1a(h, ints, sizeof(ints));
  const double reals[] = {p.tau[2], p.tau[3], p.tau[4], p.rho0,
                          p.tau_bulk == 0 ? p.tau[2] : p.tau_bulk,
                          p.tau_31 == 0 ? p.tau[3] : p.tau_31};
  h = fnv1a(h, reals, sizeof(reals));
  h = fnv1a(h, c->smask_host.data(), c->smask_host.size() * sizeof(uint32_t));
  return fnv1a(h, &c->g_hash, sizeof(c->g_hash));
}

struct CkptHeader {
  char magic[8];
  uint32_t version;
  int32_t lattice, collision, storage, nx, ny, nz;
  int64_t t;
  uint64_t hash, payload;
};

bool write_all(FILE *f, const void *p, size_t n) { return fwrite(p, 1, n, f) == n; }
bool read_all(FILE *f, void *p, size_t n) { return fread(p, 1, n, f) == n; }

bool write_header(FILE *f, const CkptHeader &h) {
  return write_all(f, h.magic, 8) && write_all(f, &h.version, 4) &&
         write_all(f, &h.lattice, 4) && write_all(f, &h.collision, 4) &&
         write_all(f, &h.storage, 4) && write_all(f, &h.nx, 4) && write_all(f, &h.ny, 4) &&
         write_all(f, &h.nz, 4) && write_all(f, &h.t, 8) && write_all(f, &h.hash, 8) &&
         write_all(f, &h.payload, 8);
}
bool read_header(FILE *f, CkptHeader &h) {
  return read_all(f, h.magic, 8) && read_all(f, &h.version, 4) && read_all(f, &h.lattice, 4) &&
         read_all(f, &h.collision, 4) && read_all(f, &h.storage, 4) && read_all(f, &h.nx, 4) &&
         read_all(f, &h.ny, 4) && read_all(f, &h.nz, 4) && read_all(f, &h.t, 8) &&
         read_all(f, &h.hash, 8) && read_all(f, &h.payload, 8);
}

}  // namespace

int lbm_save(lbm_ctx *c, const char *path) {
  if (!valid(c)) return fail(LBM_ESTATE, "invalid context");
  if (!path) return fail(LBM_EINVAL, "path is NULL");
  const size_t bytes = (size_t)c->Q * c->N * storage_bytes(c->p.storage);
  std::vector<unsigned char> host(bytes);
  HIP_TRY(hipMemcpyAsync(host.data(), c->buf[c->cur], bytes, hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(hipStreamSynchronize(c->stream));
  CkptHeader h{};
  memcpy(h.magic, kCkptMagic, 8);
  h.version = kCkptVersion;
  h.lattice = c->p.lattice;
  h.collision = c->p.collision;
  h.storage = c->p.storage;
  h.nx = c->p.nx;
  h.ny = c->p.ny;
  h.nz = c->p.nz;
  h.t = c->t;
  h.hash = params_hash(c);
  h.payload = bytes;
  FILE *f = fopen(path, "wb");
  if (!f) return fail(LBM_EINVAL, "cannot open %s for writing", path);
  const bool ok = write_header(f, h) && write_all(f, host.data(), bytes);
  const bool closed = fclose(f) == 0;
  if (!ok || !closed) return fail(LBM_EINVAL, "writing %s failed", path);
  return LBM_OK;
}

int lbm_load(lbm_ctx *c, const char *path) {
  if (!valid(c)) return fail(LBM_ESTATE, "invalid context");
  if (!path) return fail(LBM_EINVAL, "path is NULL");
  FILE *f = fopen(path, "rb");
  if (!f) return fail(LBM_EINVAL, "cannot open %s", path);
  CkptHeader h{};
  if (!read_header(f, h) || memcmp(h.magic, kCkptMagic, 8) != 0) {
    fclose(f);
    return fail(LBM_EINVAL, "%s is not a checkpoint of this library", path);
  }
  if (h.version != kCkptVersion) {
    fclose(f);
    return fail(LBM_EINVAL, "checkpoint version %u, expected %u", h.version, kCkptVersion);
  }
  const size_t bytes = (size_t)c->Q * c->N * storage_bytes(c->p.storage);
  if (h.lattice != c->p.lattice || h.collision != c->p.collision || h.storage != c->p.storage ||
      h.nx != c->p.nx || h.ny != c->p.ny || h.nz != c->p.nz || h.payload != bytes) {
    fclose(f);
    return fail(LBM_EINVAL, "checkpoint lattice, collision, storage or size differ");
  }
  if (h.hash != params_hash(c)) {
    fclose(f);
    return fail(LBM_EINVAL, "checkpoint parameters (rates, walls, force) differ");
  }
  std::vector<unsigned char> host(bytes);
  const bool ok = read_all(f, host.data(), bytes);
  fclose(f);
  if (!ok) return fail(LBM_EINVAL, "%s is truncated", path);
  HIP_TRY(hipMemcpyAsync(c->buf[0], host.data(), bytes, hipMemcpyHostToDevice, c->stream));
  HIP_TRY(hipStreamSynchronize(c->stream));  // host is released on return
  c->cur = 0;
  c->t = h.t;
  state_replaced(c);
  return LBM_OK;
}

int lbm_copy_probe(const void *src, void *dst, size_t bytes, int32_t reps, int32_t block,
                   int32_t variant, void *hip_stream) {
  if (!src || !dst) return fail(LBM_EINVAL, "NULL buffer");
  if (bytes % 16) return fail(LBM_EINVAL, "bytes must be a multiple of 16");
  if (reps < 0) return fail(LBM_EINVAL, "negative repetition count");
  if (variant < 0 || variant > 3) return fail(LBM_EINVAL, "copy variant %d", variant);
  if (block == 0) block = 256;
  if (block < 64 || block > 1024 || block % 64) return fail(LBM_EINVAL, "block %d", block);
  if (bytes / 16 / (size_t)block >= (size_t(1) << 31))
    return fail(LBM_EINVAL, "copy of %zu bytes needs too many blocks", bytes);
  HIP_TRY(lbm::copy_probe(src, dst, bytes, reps, block, variant,
                          static_cast<hipStream_t>(hip_stream)));
  return LBM_OK;
}

namespace {
// memory access x addressing x placement x wave cap
constexpr int kVariants = kBaseVariants * kNumCaps;
bool tuning_ok(const lbm_tuning *t) {
  return t && (t->bx == 64 || t->bx == 128 || t->bx == 256) && t->by >= 1 &&
         t->bx * t->by <= 256 && t->variant >= 0 && t->variant < kVariants;
}
}  // namespace

int lbm_set_tuning(lbm_ctx *c, const lbm_tuning *t) {
  if (!valid(c)) return fail(LBM_ESTATE, "invalid context");
  if (!tuning_ok(t)) return fail(LBM_EINVAL, "invalid tuning");
  if (t->by > 65535) return fail(LBM_EINVAL, "invalid tuning");
  // the monitor partials are sized by the block grid: a larger buffer is allocated
  // before anything changes, so a failure leaves the context as it was
  const int64_t nb = (int64_t)((c->p.nx + t->bx - 1) / t->bx) * ((c->p.ny + t->by - 1) / t->by) *
                     c->p.nz;
  if (nb > c->nblocks_cap) {
    double *grown = nullptr;
    int rc = c->dalloc((void **)&grown, (size_t)nb * lbm::MON_SLOTS * sizeof(double));
    if (rc) return rc;
    HIP_TRY(hipStreamSynchronize(c->stream));  // the stream may still read the old one
    c->dfree(c->partials);
    c->bytes -= (size_t)c->nblocks_cap * lbm::MON_SLOTS * sizeof(double);
    c->partials = grown;
    c->nblocks_cap = nb;
  }
  if (c->bx != t->bx || c->by != t->by || c->variant != t->variant) {
    HIP_TRY(hipStreamSynchronize(c->stream));  // a replay may still be in flight
    c->drop_graphs();
  }
  c->bx = t->bx;
  c->by = t->by;
  c->variant = t->variant;
  c->nblocks = nb;
  return LBM_OK;
}

int lbm_get_tuning(const lbm_ctx *c, lbm_tuning *t) {
  if (!valid(c)) return fail(LBM_ESTATE, "invalid context");
  if (!t) return fail(LBM_EINVAL, "t is NULL");
  t->bx = c->bx;
  t->by = c->by;
  t->variant = c->variant;
  return LBM_OK;
}

int lbm_autotune(lbm_ctx *c, int32_t steps, lbm_tuning *best, double *best_ms) {
  if (!valid(c)) return fail(LBM_ESTATE, "invalid context");
  if (steps < 1) return fail(LBM_EINVAL, "steps must be >= 1");
  const size_t pop_bytes = (size_t)c->Q * c->N * storage_bytes(c->p.storage);
  int rc = c->need_scratch(pop_bytes);
  if (rc) return rc;
  // graphs hold a launch configuration: the trials change it
  HIP_TRY(hipStreamSynchronize(c->stream));
  c->drop_graphs();
  // save the state; trials ping-pong between the two buffers
  HIP_TRY(hipMemcpyAsync(c->scratch, c->buf[c->cur], pop_bytes, hipMemcpyDeviceToDevice,
                         c->stream));
  const lbm_tuning start = {c->bx, c->by, c->variant};
  lbm_tuning win = start;
  float win_ms = -1.0f;
  hipEvent_t e0, e1;
  HIP_TRY(hipEventCreate(&e0));
  HIP_TRY(hipEventCreate(&e1));
  const int cur0 = c->cur;
  int status = LBM_OK;
  // one timed trial of a launch configuration; false on a device error (status set)
  auto trial = [&](int bx, int by, int v) -> bool {
    c->bx = bx;
    c->by = by;
    c->variant = v;
    // warm-up launch, then the timed ones
    lbm::LaunchDesc d = c->desc(1.0);
    hipError_t e = c->ops->step(d, c->stream);
    c->cur ^= 1;
    if (e == hipSuccess) e = hipEventRecord(e0, c->stream);
    for (int s = 0; s < steps && e == hipSuccess; ++s) {
      d = c->desc(1.0);
      e = c->ops->step(d, c->stream);
      c->cur ^= 1;
    }
    if (e == hipSuccess) e = hipEventRecord(e1, c->stream);
    if (e == hipSuccess) e = hipEventSynchronize(e1);
    float ms = 0;
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
    if (e != hipSuccess) {
      status = fail(LBM_EDEVICE, "autotune trial failed: %s", hipGetErrorString(e));
      return false;
    }
    ms /= steps;
    if (win_ms < 0 || ms < win_ms) {
      win_ms = ms;
      win = {bx, by, v};
    }
    return true;
  };
  // block shapes x base variants, every workgroup resident that the registers allow ...
  for (int bx : {64, 128, 256}) {
    if (bx > 64 && bx >= 2 * c->p.nx) continue;  // mostly idle lanes
    for (int by : {1, 2, 4}) {
      if (bx * by > 256) continue;
      for (int v = 0; v < kBaseVariants && !status; ++v) trial(bx, by, v);
      if (status) break;
    }
    if (status) break;
  }
  // ... then the winner held to fewer waves per SIMD
  const lbm_tuning stage1 = win;
  for (int k = 1; k < kNumCaps && !status; ++k)
    if (lds_for_cap(kWaveCaps[k], stage1.bx, stage1.by, c->lds_cu, c->lds_block))
      trial(stage1.bx, stage1.by, stage1.variant % kBaseVariants + k * kBaseVariants);
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  // restore the state into the buffer it came from
  c->cur = cur0;
  HIP_TRY(hipMemcpyAsync(c->buf[c->cur], c->scratch, pop_bytes, hipMemcpyDeviceToDevice,
                         c->stream));
  HIP_TRY(hipStreamSynchronize(c->stream));
  if (status) {
    lbm_set_tuning(c, &start);
    return status;
  }
  rc = lbm_set_tuning(c, &win);
  if (rc) return rc;
  if (best) *best = win;
  if (best_ms) *best_ms = win_ms;
  return LBM_OK;
}

}  // extern "C"
