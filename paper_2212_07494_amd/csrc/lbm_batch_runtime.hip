// Host side of the batched engine (include/lbm_batch.h): validation, packing of the
// domains, the tile table, graph capture and replay, per-domain transfers, the tuner.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <limits>
#include <new>
#include <string>
#include <vector>

#include "lbm.h"
#include "lbm_batch.h"
#include "lbm_batch_kernels.h"
#include "lbm_internal.h"

namespace {

using lbm::set_error;

#define HIP_TRY(expr)                                                                       \
  do {                                                                                      \
    hipError_t e_ = (expr);                                                                 \
    if (e_ != hipSuccess)                                                                   \
      return set_error(LBM_EDEVICE, "%s: %s (%s:%d)", #expr, hipGetErrorString(e_), __FILE__, \
                       __LINE__);                                                           \
  } while (0)

constexpr uint32_t kMagic = 0x4c424231u;  // "LBB1"

size_t storage_bytes(int s) { return s == LBM_F64 ? 8 : (s == LBM_F16_SHIFTED ? 2 : 4); }
size_t arith_bytes(int s) { return s == LBM_F64 ? 8 : 4; }

using lbm::ops_for;

void block_shape(int nx, int &bx, int &by) {
  bx = nx >= 256 ? 256 : (nx >= 128 ? 128 : 64);
  by = 256 / bx;
}

// Tile policy 1: linear tiles of 256 consecutive nodes (any domain width).
constexpr int kLinearTiles = 1;

int tile_width(int policy, int nx) {
  if (policy) return policy;
  return nx > 128 ? 256 : (nx > 64 ? 128 : 64);
}

int log2i(int v) {
  int l = 0;
  while ((1 << l) < v) ++l;
  return l;
}

}  // namespace

struct lbm_batch {
  uint32_t magic = kMagic;
  int lattice = 0, coll = 0, storage = 0;
  double rho0 = 1.0, shift = 0.0;
  const lbm::LatticeOps *ops = nullptr;
  int D = 0, Q = 0;
  hipStream_t stream = nullptr;
  hipStream_t cap = nullptr;  // private stream the check interval is captured on
  int ndom = 0;
  int64_t nodes = 0;
  int64_t pop_elems = 0;  // elements of one population buffer (planes padded to lines)
  std::vector<lbm::BatchDom> dom;
  std::vector<int> gk;  // per domain: 1 if full field
  void *buf[2] = {nullptr, nullptr};
  int cur = 0;
  void *gbuf = nullptr, *urec = nullptr, *uchk = nullptr;
  void *doms_d = nullptr, *tiles_d = nullptr;
  int *tile_begin_d = nullptr, *tile_end_d = nullptr;
  int ntiles = 0, max_tiles = 0;
  double *partials = nullptr;
  int *active_d = nullptr, *n_active_d = nullptr;
  lbm::DomState *state_d = nullptr;
  void *scratch = nullptr;
  size_t scratch_bytes = 0;
  size_t bytes = 0;
  lbm_batch_tuning tune{0, 8, 1};
  int ncu = 256;
  // captured graph of one check interval
  hipGraphExec_t exec = nullptr;
  hipGraph_t graph = nullptr;
  int g_K = 0, g_stall = 0, g_cur = -1;
  double g_tol = 0;
  bool g_valid = false;

  int dalloc(void **p, size_t n) {
    *p = nullptr;
    if (n == 0) n = 256;
    hipError_t e = hipMalloc(p, n);
    if (e != hipSuccess) {
      *p = nullptr;
      return set_error(e == hipErrorOutOfMemory ? LBM_ENOMEM : LBM_EDEVICE, "hipMalloc(%zu): %s",
                       n, hipGetErrorString(e));
    }
    bytes += n;
    return LBM_OK;
  }
  int need_scratch(size_t n) {
    if (n <= scratch_bytes) return LBM_OK;
    HIP_TRY(hipStreamSynchronize(stream));
    if (scratch) (void)hipFree(scratch);
    bytes -= scratch_bytes;
    scratch = nullptr;
    scratch_bytes = 0;
    int rc = dalloc(&scratch, n);
    if (rc) return rc;
    scratch_bytes = n;
    return LBM_OK;
  }
  void drop_graph() {
    if (exec) (void)hipGraphExecDestroy(exec);
    if (graph) (void)hipGraphDestroy(graph);
    exec = nullptr;
    graph = nullptr;
    g_valid = false;
  }
  // per-domain launch descriptor for the single-domain kernels (init, moments, transfers)
  lbm::LaunchDesc desc(int d) const {
    const lbm::BatchDom &m = dom[d];
    const size_t sb = storage_bytes(storage), ab = arith_bytes(storage);
    lbm::LaunchDesc L{};
    L.coll = coll;
    L.storage = storage;
    L.gk = gk[d];
    L.fin = static_cast<const char *>(buf[cur]) + (size_t)m.base * sb;
    L.fout = static_cast<char *>(buf[cur]) + (size_t)m.base * sb;
    L.geo.nx = m.nx;
    L.geo.ny = m.ny;
    L.geo.nz = m.nz;
    L.geo.N = m.N;
    L.geo.ps = m.ps;
    for (int a = 0; a < 3; ++a) L.geo.wall[a] = m.wall[a];
    L.gtab = static_cast<const char *>(gbuf) + (size_t)m.goff * ab;
    L.g_axis = m.gaxis == 3 ? -1 : m.gaxis;
    L.g_n = m.gaxis == 3 ? m.N : m.gn;
    L.gscale = 1.0;
    L.shift = shift;
    L.c0 = m.c0;
    L.c1 = m.c1;
    block_shape(m.nx, L.bx, L.by);
    L.variant = 0;
    return L;
  }
  lbm::BatchLaunch launch(int from) const {
    lbm::BatchLaunch b{};
    b.coll = coll;
    b.storage = storage;
    b.variant = tune.variant;
    b.fin = buf[from];
    b.fout = buf[from ^ 1];
    b.gbuf = gbuf;
    b.doms = doms_d;
    b.tiles = tiles_d;
    b.active = active_d;
    b.ntiles = ntiles;
    // blocks_per_cu 0: one workgroup per tile (a multiple of the XCD count, so the
    // XCD-contiguous tile walk applies); else a persistent grid walking the table
    b.grid = tune.blocks_per_cu ? tune.blocks_per_cu * ncu : (ntiles + 7) / 8 * 8;
    b.shift = shift;
    b.urec = urec;
    b.uchk = uchk;
    b.state = state_d;
    b.window = 1;  // set by the monitor passes of a check interval
    b.partials = partials;
    return b;
  }
};

namespace {

bool valid(const lbm_batch *b) { return b && b->magic == kMagic; }

int validate_domain(const lbm_domain &d, int idx, int lattice, int coll) {
  if (d.nx <= 0 || d.ny <= 0 || d.nz <= 0)
    return set_error(LBM_EINVAL, "domain %d: sizes must be positive", idx);
  if (lattice == LBM_D2Q9 && d.nz != 1)
    return set_error(LBM_EINVAL, "domain %d: D2Q9 needs nz == 1", idx);
  if ((int64_t)d.nx * d.ny * d.nz >= (int64_t(1) << 31))
    return set_error(LBM_EINVAL, "domain %d: too many nodes", idx);
  for (int a = 0; a < 3; ++a)
    if (d.bc[a] != LBM_PERIODIC && d.bc[a] != LBM_WALLS)
      return set_error(LBM_EINVAL, "domain %d: unknown boundary kind", idx);
  if (!(d.tau[2] > 0.5) || !std::isfinite(d.tau[2]))
    return set_error(LBM_EINVAL, "domain %d: tau[2] = %g must exceed 1/2", idx, d.tau[2]);
  if (coll == LBM_SMRT) {
    if (!(d.tau[3] > 0.5) || !std::isfinite(d.tau[3]))
      return set_error(LBM_EINVAL, "domain %d: tau[3] = %g must exceed 1/2", idx, d.tau[3]);
    if (d.tau[4] != 1.0)
      return set_error(LBM_EINVAL, "domain %d: SMRT trims order 4: tau[4] must be 1", idx);
  }
  if (d.g_kind < LBM_G_UNIFORM || d.g_kind > LBM_G_FIELD)
    return set_error(LBM_EINVAL, "domain %d: unknown force kind", idx);
  if (d.g_kind == LBM_G_PROFILE && (d.g_axis < 0 || d.g_axis > 2))
    return set_error(LBM_EINVAL, "domain %d: profile axis %d", idx, d.g_axis);
  if (d.g_kind != LBM_G_UNIFORM && !d.g_data)
    return set_error(LBM_EINVAL, "domain %d: g_data is NULL", idx);
  return LBM_OK;
}

// Build the tile table for the current tuning and upload it.
int build_tiles(lbm_batch *b) {
  std::vector<lbm::BatchTile> tiles;
  std::vector<int> tb(b->ndom), te(b->ndom);
  for (int d = 0; d < b->ndom; ++d) {
    lbm::BatchDom &m = b->dom[d];
    m.tile_begin = (int)tiles.size();
    if (b->tune.tile_bx == kLinearTiles) {
      // 256 consecutive nodes of one z layer per tile: x0 is the first node's offset in
      // the layer, every lane busy except in a layer's last tile
      m.tbx_log2 = -1;
      for (int z = 0; z < m.nz; ++z)
        for (int r0 = 0; r0 < m.nx * m.ny; r0 += 256) tiles.push_back({d, r0, 0, z});
    } else {
      const int tbx = tile_width(b->tune.tile_bx, m.nx);
      const int tby = 256 / tbx;
      m.tbx_log2 = log2i(tbx);
      for (int z = 0; z < m.nz; ++z)
        for (int y0 = 0; y0 < m.ny; y0 += tby)
          for (int x0 = 0; x0 < m.nx; x0 += tbx) tiles.push_back({d, x0, y0, z});
    }
    m.tile_end = (int)tiles.size();
    tb[d] = m.tile_begin;
    te[d] = m.tile_end;
  }
  if ((int)tiles.size() > b->max_tiles)
    return set_error(LBM_EINVAL, "tile table larger than allocated");
  b->ntiles = (int)tiles.size();
  HIP_TRY(hipMemcpyAsync(b->tiles_d, tiles.data(), tiles.size() * sizeof(lbm::BatchTile),
                         hipMemcpyHostToDevice, b->stream));
  HIP_TRY(hipMemcpyAsync(b->doms_d, b->dom.data(), b->dom.size() * sizeof(lbm::BatchDom),
                         hipMemcpyHostToDevice, b->stream));
  HIP_TRY(hipMemcpyAsync(b->tile_begin_d, tb.data(), tb.size() * sizeof(int),
                         hipMemcpyHostToDevice, b->stream));
  HIP_TRY(hipMemcpyAsync(b->tile_end_d, te.data(), te.size() * sizeof(int), hipMemcpyHostToDevice,
                         b->stream));
  HIP_TRY(hipStreamSynchronize(b->stream));
  b->drop_graph();
  return LBM_OK;
}

// Largest tile count over the tile-width policies (tbx x 256/tbx tiles).
int max_tile_count(const std::vector<lbm::BatchDom> &dom) {
  int64_t best = 0;
  for (int policy : {0, 1, 64, 128, 256}) {
    int64_t n = 0;
    for (const auto &m : dom) {
      if (policy == kLinearTiles) {
        n += (int64_t)m.nz * (((int64_t)m.nx * m.ny + 255) / 256);
        continue;
      }
      const int tbx = tile_width(policy, m.nx), tby = 256 / tbx;
      n += (int64_t)m.nz * ((m.ny + tby - 1) / tby) * ((m.nx + tbx - 1) / tbx);
    }
    if (n > best) best = n;
  }
  return (int)best;
}

void release(lbm_batch *b) {
  if (!b) return;
  (void)hipStreamSynchronize(b->stream);
  b->drop_graph();
  if (b->cap) (void)hipStreamDestroy(b->cap);
  void *ptrs[] = {b->buf[0], b->buf[1], b->gbuf,     b->urec,         b->uchk,  b->doms_d,
                  b->tiles_d, b->tile_begin_d, b->tile_end_d, b->partials, b->active_d,
                  b->n_active_d, b->state_d, b->scratch};
  for (void *p : ptrs)
    if (p) (void)hipFree(p);
  b->magic = 0;
  delete b;
}

int reset_states(lbm_batch *b) {
  std::vector<int> act(b->ndom, 1);
  std::vector<lbm::DomState> st(b->ndom);
  for (auto &s : st) {
    s.steps = 0;
    s.resid = 0;
    s.best = std::numeric_limits<double>::infinity();
    s.status = LBM_DOM_RUNNING;
    s.stall = 0;
    s.nchk = 0;
    s.win_steps = -1;
    s.coherence = 1.0;
  }
  int n = b->ndom;
  HIP_TRY(hipMemcpyAsync(b->active_d, act.data(), act.size() * sizeof(int), hipMemcpyHostToDevice,
                         b->stream));
  HIP_TRY(hipMemcpyAsync(b->state_d, st.data(), st.size() * sizeof(lbm::DomState),
                         hipMemcpyHostToDevice, b->stream));
  HIP_TRY(hipMemcpyAsync(b->n_active_d, &n, sizeof(int), hipMemcpyHostToDevice, b->stream));
  HIP_TRY(hipStreamSynchronize(b->stream));
  return LBM_OK;
}

// Enqueue one check interval on stream s: K-1 steps, record u, one step, compare +
// record, decide.
int enqueue_interval(lbm_batch *b, int K, double tol, int stall, hipStream_t s) {
  int from = b->cur;
  for (int k = 0; k < K; ++k) {
    if (k == K - 1) {
      lbm::BatchLaunch m = b->launch(from);
      m.mode = 2;
      m.window = stall;
      HIP_TRY(b->ops->batch_monitor(m, s));
    }
    HIP_TRY(b->ops->batch_step(b->launch(from), s));
    from ^= 1;
  }
  lbm::BatchLaunch m = b->launch(from);
  m.mode = 4;
  m.window = stall;
  HIP_TRY(b->ops->batch_monitor(m, s));
  HIP_TRY(lbm::decide_domains(b->tile_begin_d, b->tile_end_d, b->partials, b->state_d,
                              b->active_d, b->n_active_d, b->ndom, tol, stall, K, s));
  return LBM_OK;
}

}  // namespace

extern "C" {

int lbm_batch_init(const lbm_domain *domains, int32_t ndom, int32_t lattice, int32_t collision,
                   int32_t storage, double rho0, void *hip_stream, lbm_batch **out) {
  if (!out) return set_error(LBM_EINVAL, "out is NULL");
  *out = nullptr;
  if (!domains || ndom < 1) return set_error(LBM_EINVAL, "need at least one domain");
  if (lattice < LBM_D2Q9 || lattice > LBM_D3Q27)
    return set_error(LBM_EINVAL, "unknown lattice (the batched engine covers D2Q9, D3Q19, D3Q27)");
  if (collision != LBM_BGK && collision != LBM_SMRT)
    return set_error(LBM_EINVAL, "unknown collision");
  if (storage < LBM_F64 || storage > LBM_F16_SHIFTED)
    return set_error(LBM_EINVAL, "unknown storage");
  if (!(rho0 > 0) || !std::isfinite(rho0)) return set_error(LBM_EINVAL, "rho0 must be positive");
  for (int d = 0; d < ndom; ++d) {
    int rc = validate_domain(domains[d], d, lattice, collision);
    if (rc) return rc;
  }
  lbm_batch *b = new (std::nothrow) lbm_batch();
  if (!b) return set_error(LBM_ENOMEM, "host allocation failed");
  b->lattice = lattice;
  b->coll = collision;
  b->storage = storage;
  b->rho0 = rho0;
  b->shift = (storage == LBM_F32_SHIFTED || storage == LBM_F16_SHIFTED) ? rho0 : 0.0;
  b->ops = &ops_for(lattice);
  b->D = b->ops->D;
  b->Q = b->ops->Q;
  b->stream = static_cast<hipStream_t>(hip_stream);
  b->ndom = ndom;
  int dev = 0;
  hipDeviceProp_t prop;
  if (hipGetDevice(&dev) == hipSuccess && hipGetDeviceProperties(&prop, dev) == hipSuccess)
    b->ncu = prop.multiProcessorCount > 0 ? prop.multiProcessorCount : 256;

  // pack the domains
  const size_t ab = arith_bytes(storage);
  std::vector<double> gh;
  int64_t base = 0, ubase = 0;
  b->dom.resize(ndom);
  b->gk.resize(ndom);
  for (int d = 0; d < ndom; ++d) {
    const lbm_domain &s = domains[d];
    lbm::BatchDom &m = b->dom[d];
    m.nx = s.nx;
    m.ny = s.ny;
    m.nz = s.nz;
    m.N = s.nx * s.ny * s.nz;
    for (int a = 0; a < 3; ++a) m.wall[a] = s.bc[a] == LBM_WALLS;
    // every population plane on a 128-byte boundary: a plane stride of whole cache lines
    // and a domain base on a line, so no line is shared by two planes or two domains
    const int64_t line = 128 / (int64_t)storage_bytes(storage);
    m.ps = ((int64_t)m.nx * m.ny + line - 1) / line * line;
    base = (base + line - 1) / line * line;
    m.base = base;
    m.ubase = ubase;
    base += (int64_t)b->Q * m.nz * m.ps;
    ubase += (int64_t)b->D * m.N;
    m.goff = (int64_t)gh.size();
    if (s.g_kind == LBM_G_UNIFORM) {
      m.gaxis = -1;
      m.gn = 1;
      gh.insert(gh.end(), s.g_uniform, s.g_uniform + 3);
    } else if (s.g_kind == LBM_G_PROFILE) {
      m.gaxis = s.g_axis;
      m.gn = s.g_axis == 0 ? s.nx : (s.g_axis == 1 ? s.ny : s.nz);
      gh.insert(gh.end(), s.g_data, s.g_data + 3 * (size_t)m.gn);
    } else {
      m.gaxis = 3;
      m.gn = m.N;
      gh.insert(gh.end(), s.g_data, s.g_data + 3 * (size_t)m.N);
    }
    b->gk[d] = s.g_kind == LBM_G_FIELD;
    if (collision == LBM_BGK) {
      const double om = 1.0 / s.tau[2];
      m.c0 = om;
      m.c1 = 1.0 - 0.5 * om;
    } else {
      m.c0 = 1.0 - 1.0 / s.tau[2];
      m.c1 = 1.0 - 1.0 / s.tau[3];
    }
  }
  for (double v : gh)
    if (!std::isfinite(v)) {
      delete b;
      return set_error(LBM_EINVAL, "non-finite acceleration value");
    }
  b->nodes = ubase / b->D;
  b->pop_elems = base;
  std::vector<unsigned char> gconv(gh.size() * ab);
  for (size_t k = 0; k < gh.size(); ++k) {
    if (ab == 8)
      reinterpret_cast<double *>(gconv.data())[k] = gh[k];
    else
      reinterpret_cast<float *>(gconv.data())[k] = static_cast<float>(gh[k]);
  }
  b->max_tiles = max_tile_count(b->dom);
  if (hipStreamCreateWithFlags(&b->cap, hipStreamNonBlocking) != hipSuccess) {
    b->cap = nullptr;
    release(b);
    return set_error(LBM_EDEVICE, "creating the capture stream failed");
  }
  const size_t pop = (size_t)base * storage_bytes(storage);
  int rc;
  if ((rc = b->dalloc(&b->buf[0], pop)) || (rc = b->dalloc(&b->buf[1], pop)) ||
      (rc = b->dalloc(&b->gbuf, gconv.size())) || (rc = b->dalloc(&b->urec, (size_t)ubase * ab)) ||
      (rc = b->dalloc(&b->uchk, (size_t)ubase * ab)) ||
      (rc = b->dalloc(&b->doms_d, ndom * sizeof(lbm::BatchDom))) ||
      (rc = b->dalloc(&b->tiles_d, (size_t)b->max_tiles * sizeof(lbm::BatchTile))) ||
      (rc = b->dalloc((void **)&b->tile_begin_d, ndom * sizeof(int))) ||
      (rc = b->dalloc((void **)&b->tile_end_d, ndom * sizeof(int))) ||
      (rc = b->dalloc((void **)&b->partials,
                      (size_t)b->max_tiles * lbm::BATCH_PARTIALS * sizeof(double))) ||
      (rc = b->dalloc((void **)&b->active_d, ndom * sizeof(int))) ||
      (rc = b->dalloc((void **)&b->n_active_d, sizeof(int))) ||
      (rc = b->dalloc((void **)&b->state_d, ndom * sizeof(lbm::DomState)))) {
    std::string msg = lbm_last_error();
    release(b);
    return set_error(rc, "%s", msg.c_str());
  }
  auto bail = [&](int code) {
    std::string msg = lbm_last_error();
    release(b);
    return set_error(code, "%s", msg.c_str());
  };
  if (hipMemcpyAsync(b->gbuf, gconv.data(), gconv.size(), hipMemcpyHostToDevice, b->stream) !=
      hipSuccess)
    return bail(set_error(LBM_EDEVICE, "uploading force tables failed"));
  if ((rc = build_tiles(b))) return bail(rc);
  if ((rc = reset_states(b))) return bail(rc);
  // initial states, one domain at a time
  for (int d = 0; d < ndom; ++d) {
    const lbm_domain &s = domains[d];
    const lbm::BatchDom &m = b->dom[d];
    const size_t fld = (size_t)m.N * sizeof(double);
    double *rho_d = nullptr, *u_d = nullptr;
    if (s.rho_init || s.u_init) {
      if ((rc = b->need_scratch(fld * (1 + b->D)))) return bail(rc);
      if (s.rho_init) {
        for (int n = 0; n < m.N; ++n)
          if (!(s.rho_init[n] > 0) || !std::isfinite(s.rho_init[n]))
            return bail(set_error(LBM_EINVAL, "domain %d: invalid rho_init", d));
        rho_d = static_cast<double *>(b->scratch);
        if (hipMemcpyAsync(rho_d, s.rho_init, fld, hipMemcpyHostToDevice, b->stream) != hipSuccess)
          return bail(set_error(LBM_EDEVICE, "upload failed"));
      }
      if (s.u_init) {
        for (int64_t n = 0; n < (int64_t)b->D * m.N; ++n)
          if (!std::isfinite(s.u_init[n]))
            return bail(set_error(LBM_EINVAL, "domain %d: non-finite u_init", d));
        u_d = reinterpret_cast<double *>(static_cast<char *>(b->scratch) + fld);
        if (hipMemcpyAsync(u_d, s.u_init, fld * b->D, hipMemcpyHostToDevice, b->stream) !=
            hipSuccess)
          return bail(set_error(LBM_EDEVICE, "upload failed"));
      }
    }
    lbm::LaunchDesc L = b->desc(d);
    if (b->ops->init(L, rho_d, u_d, rho0, nullptr, b->stream) != hipSuccess)
      return bail(set_error(LBM_EDEVICE, "init kernel failed for domain %d", d));
    if ((s.rho_init || s.u_init) && hipStreamSynchronize(b->stream) != hipSuccess)
      return bail(set_error(LBM_EDEVICE, "init failed for domain %d", d));
  }
  if (hipStreamSynchronize(b->stream) != hipSuccess)
    return bail(set_error(LBM_EDEVICE, "init failed"));
  *out = b;
  return LBM_OK;
}

int lbm_batch_advance(lbm_batch *b, int64_t n) {
  if (!valid(b)) return set_error(LBM_ESTATE, "invalid batch");
  if (n < 0) return set_error(LBM_EINVAL, "negative step count");
  for (int64_t s = 0; s < n; ++s) {
    HIP_TRY(b->ops->batch_step(b->launch(b->cur), b->stream));
    b->cur ^= 1;
  }
  if (n) HIP_TRY(lbm::add_domain_steps(b->active_d, b->state_d, b->ndom, n, b->stream));
  return LBM_OK;
}

int lbm_batch_run(lbm_batch *b, int64_t max_steps, double tol, int32_t check_every,
                  int32_t stall_checks, int64_t *steps_out, double *resid_out,
                  int32_t *status_out) {
  if (!valid(b)) return set_error(LBM_ESTATE, "invalid batch");
  if (check_every < 2 || check_every % 2)
    return set_error(LBM_EINVAL, "check_every must be even and >= 2");
  if (max_steps < 0 || !(tol >= 0) || stall_checks < 1)
    return set_error(LBM_EINVAL, "invalid max_steps / tol / stall_checks");
  const int K = check_every;
  if (!b->g_valid || b->g_K != K || b->g_tol != tol || b->g_stall != stall_checks ||
      b->g_cur != b->cur) {
    b->drop_graph();
    HIP_TRY(hipStreamSynchronize(b->stream));
    // captured on the private stream (capture is not allowed on the legacy default
    // stream); the graph is then launched on the caller's stream
    HIP_TRY(hipStreamBeginCapture(b->cap, hipStreamCaptureModeThreadLocal));
    int rc = enqueue_interval(b, K, tol, stall_checks, b->cap);
    hipGraph_t g = nullptr;
    hipError_t e = hipStreamEndCapture(b->cap, &g);
    if (rc) {
      if (g) (void)hipGraphDestroy(g);
      return rc;
    }
    if (e != hipSuccess) return set_error(LBM_EDEVICE, "graph capture: %s", hipGetErrorString(e));
    b->graph = g;
    HIP_TRY(hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0));
    b->g_valid = true;
    b->g_K = K;
    b->g_tol = tol;
    b->g_stall = stall_checks;
    b->g_cur = b->cur;
  }
  int n_active = 0;
  HIP_TRY(hipMemcpyAsync(&n_active, b->n_active_d, sizeof(int), hipMemcpyDeviceToHost,
                         b->stream));
  HIP_TRY(hipStreamSynchronize(b->stream));
  for (int64_t taken = 0; taken < max_steps && n_active > 0; taken += K) {
    HIP_TRY(hipGraphLaunch(b->exec, b->stream));
    HIP_TRY(hipMemcpyAsync(&n_active, b->n_active_d, sizeof(int), hipMemcpyDeviceToHost,
                           b->stream));
    HIP_TRY(hipStreamSynchronize(b->stream));
  }
  // K is even: the current buffer is unchanged after every replay
  std::vector<lbm::DomState> st(b->ndom);
  HIP_TRY(hipMemcpyAsync(st.data(), b->state_d, st.size() * sizeof(lbm::DomState),
                         hipMemcpyDeviceToHost, b->stream));
  HIP_TRY(hipStreamSynchronize(b->stream));
  for (int d = 0; d < b->ndom; ++d) {
    if (steps_out) steps_out[d] = st[d].steps;
    if (resid_out) resid_out[d] = st[d].resid;
    if (status_out) status_out[d] = st[d].status;
  }
  return LBM_OK;
}

int lbm_batch_step(lbm_batch *b, int64_t max_steps, double tol, int64_t *steps_out,
                   double *resid_out) {
  return lbm_batch_run(b, max_steps, tol, LBM_BATCH_CHECK_EVERY, LBM_BATCH_STALL_CHECKS,
                       steps_out, resid_out, nullptr);
}

int lbm_batch_status(lbm_batch *b, int32_t *status_out) {
  if (!valid(b)) return set_error(LBM_ESTATE, "invalid batch");
  if (!status_out) return set_error(LBM_EINVAL, "status_out is NULL");
  std::vector<lbm::DomState> st(b->ndom);
  HIP_TRY(hipMemcpyAsync(st.data(), b->state_d, st.size() * sizeof(lbm::DomState),
                         hipMemcpyDeviceToHost, b->stream));
  HIP_TRY(hipStreamSynchronize(b->stream));
  for (int d = 0; d < b->ndom; ++d) status_out[d] = st[d].status;
  return LBM_OK;
}

int lbm_batch_moments(lbm_batch *b, int32_t dom, double *rho, double *u) {
  if (!valid(b)) return set_error(LBM_ESTATE, "invalid batch");
  if (dom < 0 || dom >= b->ndom) return set_error(LBM_EINVAL, "domain %d out of range", dom);
  const size_t fld = (size_t)b->dom[dom].N * sizeof(double);
  int rc = b->need_scratch(fld * (1 + b->D));
  if (rc) return rc;
  double *rho_d = static_cast<double *>(b->scratch);
  double *u_d = reinterpret_cast<double *>(static_cast<char *>(b->scratch) + fld);
  HIP_TRY(b->ops->moments(b->desc(dom), rho_d, u_d, nullptr, 1, nullptr, b->stream));
  if (rho) HIP_TRY(hipMemcpyAsync(rho, rho_d, fld, hipMemcpyDeviceToHost, b->stream));
  if (u) HIP_TRY(hipMemcpyAsync(u, u_d, fld * b->D, hipMemcpyDeviceToHost, b->stream));
  HIP_TRY(hipStreamSynchronize(b->stream));
  return LBM_OK;
}

int lbm_batch_get_populations(lbm_batch *b, int32_t dom, double *f) {
  if (!valid(b)) return set_error(LBM_ESTATE, "invalid batch");
  if (dom < 0 || dom >= b->ndom) return set_error(LBM_EINVAL, "domain %d out of range", dom);
  if (!f) return set_error(LBM_EINVAL, "f is NULL");
  const int64_t N = b->dom[dom].N;
  const size_t outb = (size_t)b->Q * N * sizeof(double);
  int rc = b->need_scratch(outb);
  if (rc) return rc;
  HIP_TRY(b->ops->gather(b->desc(dom), nullptr, N, static_cast<double *>(b->scratch), b->stream));
  HIP_TRY(hipMemcpyAsync(f, b->scratch, outb, hipMemcpyDeviceToHost, b->stream));
  HIP_TRY(hipStreamSynchronize(b->stream));
  return LBM_OK;
}

int lbm_batch_set_populations(lbm_batch *b, int32_t dom, const double *f) {
  if (!valid(b)) return set_error(LBM_ESTATE, "invalid batch");
  if (dom < 0 || dom >= b->ndom) return set_error(LBM_EINVAL, "domain %d out of range", dom);
  if (!f) return set_error(LBM_EINVAL, "f is NULL");
  const size_t inb = (size_t)b->Q * b->dom[dom].N * sizeof(double);
  int rc = b->need_scratch(inb);
  if (rc) return rc;
  HIP_TRY(hipMemcpyAsync(b->scratch, f, inb, hipMemcpyHostToDevice, b->stream));
  HIP_TRY(b->ops->scatter(b->desc(dom), static_cast<const double *>(b->scratch), b->stream));
  // reactivate the domain
  std::vector<int> act(b->ndom);
  std::vector<lbm::DomState> st(b->ndom);
  HIP_TRY(hipMemcpyAsync(act.data(), b->active_d, act.size() * sizeof(int),
                         hipMemcpyDeviceToHost, b->stream));
  HIP_TRY(hipMemcpyAsync(st.data(), b->state_d, st.size() * sizeof(lbm::DomState),
                         hipMemcpyDeviceToHost, b->stream));
  HIP_TRY(hipStreamSynchronize(b->stream));
  act[dom] = 1;
  st[dom].steps = 0;
  st[dom].resid = 0;
  st[dom].best = std::numeric_limits<double>::infinity();
  st[dom].status = LBM_DOM_RUNNING;
  st[dom].stall = 0;
  st[dom].nchk = 0;
  st[dom].win_steps = -1;
  st[dom].coherence = 1.0;
  int n = 0;
  for (int a : act) n += a != 0;
  HIP_TRY(hipMemcpyAsync(b->active_d, act.data(), act.size() * sizeof(int), hipMemcpyHostToDevice,
                         b->stream));
  HIP_TRY(hipMemcpyAsync(b->state_d, st.data(), st.size() * sizeof(lbm::DomState),
                         hipMemcpyHostToDevice, b->stream));
  HIP_TRY(hipMemcpyAsync(b->n_active_d, &n, sizeof(int), hipMemcpyHostToDevice, b->stream));
  HIP_TRY(hipStreamSynchronize(b->stream));
  return LBM_OK;
}

int lbm_batch_set_tuning(lbm_batch *b, const lbm_batch_tuning *t) {
  if (!valid(b)) return set_error(LBM_ESTATE, "invalid batch");
  if (!t || !(t->tile_bx == 0 || t->tile_bx == kLinearTiles || t->tile_bx == 64 ||
              t->tile_bx == 128 || t->tile_bx == 256) ||
      t->blocks_per_cu < 0 || t->blocks_per_cu > 32 || t->variant < 0 || t->variant > 2)
    return set_error(LBM_EINVAL, "invalid batch tuning");
  b->tune = *t;
  return build_tiles(b);
}

int lbm_batch_get_tuning(const lbm_batch *b, lbm_batch_tuning *t) {
  if (!valid(b)) return set_error(LBM_ESTATE, "invalid batch");
  if (!t) return set_error(LBM_EINVAL, "t is NULL");
  *t = b->tune;
  return LBM_OK;
}

int lbm_batch_autotune(lbm_batch *b, int32_t steps, lbm_batch_tuning *best, double *best_ms) {
  if (!valid(b)) return set_error(LBM_ESTATE, "invalid batch");
  if (steps < 1) return set_error(LBM_EINVAL, "steps must be >= 1");
  const size_t pop = (size_t)b->pop_elems * storage_bytes(b->storage);
  int rc = b->need_scratch(pop);
  if (rc) return rc;
  HIP_TRY(hipMemcpyAsync(b->scratch, b->buf[b->cur], pop, hipMemcpyDeviceToDevice, b->stream));
  const int cur0 = b->cur;
  const lbm_batch_tuning start = b->tune;
  lbm_batch_tuning win = start;
  float win_ms = -1.0f;
  hipEvent_t e0, e1;
  HIP_TRY(hipEventCreate(&e0));
  HIP_TRY(hipEventCreate(&e1));
  int status = LBM_OK;
  for (int tbx : {0, kLinearTiles, 64, 128, 256}) {
    for (int bpc : {0, 2, 4, 8, 16}) {
      for (int v = 0; v < 3 && !status; ++v) {
        lbm_batch_tuning t{tbx, bpc, v};
        if ((status = lbm_batch_set_tuning(b, &t))) break;
        hipError_t e = b->ops->batch_step(b->launch(b->cur), b->stream);
        b->cur ^= 1;
        if (e == hipSuccess) e = hipEventRecord(e0, b->stream);
        for (int s = 0; s < steps && e == hipSuccess; ++s) {
          e = b->ops->batch_step(b->launch(b->cur), b->stream);
          b->cur ^= 1;
        }
        if (e == hipSuccess) e = hipEventRecord(e1, b->stream);
        if (e == hipSuccess) e = hipEventSynchronize(e1);
        float ms = 0;
        if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
        if (e != hipSuccess) {
          status = set_error(LBM_EDEVICE, "batch autotune trial: %s", hipGetErrorString(e));
          break;
        }
        ms /= steps;
        if (win_ms < 0 || ms < win_ms) {
          win_ms = ms;
          win = t;
        }
      }
      if (status) break;
    }
    if (status) break;
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  b->cur = cur0;
  HIP_TRY(hipMemcpyAsync(b->buf[b->cur], b->scratch, pop, hipMemcpyDeviceToDevice, b->stream));
  HIP_TRY(hipStreamSynchronize(b->stream));
  rc = lbm_batch_set_tuning(b, status ? &start : &win);
  if (status) return status;
  if (rc) return rc;
  if (best) *best = win;
  if (best_ms) *best_ms = win_ms;
  return LBM_OK;
}

int lbm_batch_info(const lbm_batch *b, int64_t *nodes, int64_t *tiles, size_t *bytes) {
  if (!valid(b)) return set_error(LBM_ESTATE, "invalid batch");
  if (nodes) *nodes = b->nodes;
  if (tiles) *tiles = b->ntiles;
  if (bytes) *bytes = b->bytes;
  return LBM_OK;
}

int lbm_batch_free(lbm_batch *b) {
  if (!valid(b)) return set_error(LBM_ESTATE, "invalid batch");
  release(b);
  return LBM_OK;
}

}  // extern "C"
