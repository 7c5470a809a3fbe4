// Steady response of the forced periodic lattice to Fourier forcing modes, order by order
// in the forcing amplitude (lbm_ws_lattice_response: first order, as mode coefficients;
// lbm_ws_lattice_waves: up to fourth order, as population waves).  Host code driving the
// library's own step: the collision's derivatives about rest are central differences of
// that step, and every wave of the response is one Q x Q complex solve.
//
// All collision evaluations of one stage run together as one step of an n x 1 x 1
// periodic lattice with a per-node acceleration field: there the pull streaming moves
// population i from node p to node p + e_ix (mod n) and leaves the other axes alone, so
// the state after the step holds C(f_p, g_p)_i at node p + e_ix.
#include <algorithm>
#include <array>
#include <cmath>
#include <complex>
#include <map>
#include <memory>
#include <vector>

#include "lbm.h"
#include "lbm_internal.h"
#include "lbm_nn.h"

namespace {

using cplx = std::complex<double>;
using cvec = std::vector<cplx>;
using rvec = std::vector<double>;
using gvec = std::array<double, 3>;
using gcvec = std::array<cplx, 3>;
using kvec = std::array<int, 3>;

// Gaussian elimination with partial pivoting on an n x n row-major system; x overwrites b.
bool solve_complex(int n, std::vector<cplx> &A, std::vector<cplx> &b) {
  for (int c = 0; c < n; ++c) {
    int piv = c;
    for (int r = c + 1; r < n; ++r)
      if (std::abs(A[r * n + c]) > std::abs(A[piv * n + c])) piv = r;
    if (std::abs(A[piv * n + c]) == 0.0) return false;
    if (piv != c) {
      for (int j = 0; j < n; ++j) std::swap(A[c * n + j], A[piv * n + j]);
      std::swap(b[c], b[piv]);
    }
    for (int r = c + 1; r < n; ++r) {
      const cplx f = A[r * n + c] / A[c * n + c];
      if (f == cplx(0.0)) continue;
      for (int j = c; j < n; ++j) A[r * n + j] -= f * A[c * n + j];
      b[r] -= f * b[c];
    }
  }
  for (int r = n - 1; r >= 0; --r) {
    cplx s = b[r];
    for (int j = r + 1; j < n; ++j) s -= A[r * n + j] * b[j];
    b[r] = s / A[r * n + r];
  }
  return true;
}

// A direction of the expansion in (populations, acceleration).
struct Dir {
  cvec f;
  gcvec g{};
};
struct RDir {
  rvec f;
  gvec g{};
};

Dir conj(const Dir &d) {
  Dir c = d;
  for (auto &v : c.f) v = std::conj(v);
  for (auto &v : c.g) v = std::conj(v);
  return c;
}
Dir scaled(const Dir &d, cplx s) {
  Dir c = d;
  for (auto &v : c.f) v *= s;
  for (auto &v : c.g) v *= s;
  return c;
}
RDir part(const Dir &d, bool imag) {
  RDir r;
  r.f.resize(d.f.size());
  for (size_t i = 0; i < d.f.size(); ++i) r.f[i] = imag ? d.f[i].imag() : d.f[i].real();
  for (int a = 0; a < 3; ++a) r.g[a] = imag ? d.g[a].imag() : d.g[a].real();
  return r;
}
double max_abs(const RDir &r) {
  double m = 0;
  for (double v : r.f) m = std::max(m, std::abs(v));
  for (double v : r.g) m = std::max(m, std::abs(v));
  return m;
}

// Collision evaluation points, run together (see the file comment).  The points are kept
// population-major as they are added, which is the layout lbm_set_populations takes.
class CollisionBatch {
 public:
  CollisionBatch(const lbm_params &q, int Q, const int *E)
      : q_(q), Q_(Q), E_(E), f_(Q), g_(3) {}
  int size() const { return n_; }
  int add(const rvec &f, const gvec &g) {
    for (int i = 0; i < Q_; ++i) f_[i].push_back(f[i]);
    for (int a = 0; a < 3; ++a) g_[a].push_back(g[a]);
    return n_++;
  }
  int run() {
    if (n_ == 0) return LBM_OK;
    const size_t n = (size_t)n_;
    std::unique_ptr<double[]> gplanes(new double[3 * n]), pop(new double[Q_ * n]);
    for (int a = 0; a < 3; ++a) std::copy(g_[a].begin(), g_[a].end(), gplanes.get() + a * n);
    for (int i = 0; i < Q_; ++i) std::copy(f_[i].begin(), f_[i].end(), pop.get() + i * n);
    next_.reset(new double[Q_ * n]);
    lbm_params q = q_;
    q.nx = n_;
    q.ny = q.nz = 1;
    q.g_kind = LBM_G_FIELD;
    q.g_data = gplanes.get();
    lbm_ctx *c = nullptr;
    int rc = lbm_init(&q, nullptr, nullptr, nullptr, &c);
    if (rc) return rc;
    const double one = 1.0;
    rc = lbm_set_populations(c, pop.get());
    if (!rc) rc = lbm_step(c, 1, &one);
    if (!rc) rc = lbm_get_populations(c, n_, nullptr, next_.get());
    lbm_free(c);
    return rc;
  }
  // After run(): C(f_p, g_p)_i, which the step left at node p + e_ix.
  double value(int p, int i) const {
    int dst = p + E_[3 * i];
    dst = dst < 0 ? dst + n_ : (dst >= n_ ? dst - n_ : dst);
    return next_[(size_t)i * n_ + dst];
  }

 private:
  lbm_params q_;
  int Q_;
  const int *E_;
  int n_ = 0;
  std::vector<rvec> f_, g_;
  std::unique_ptr<double[]> next_;
};

// The collision expanded about rest: J = dC/d f-bar (Q x Q) and G = dC/dg (Q x 3) by
// central differences, the second and third derivatives along directions by mixed
// central differences (planned into a batch, then read out), and the steady periodic
// waves they drive.
class Expansion {
 public:
  explicit Expansion(const lbm_params &q)
      : q_(q), Q(lbm::ops_for(q.lattice).Q), D(lbm::ops_for(q.lattice).D),
        E(lbm::ops_for(q.lattice).E) {}

  CollisionBatch batch() const { return CollisionBatch(q_, Q, E); }

  int build() {
    // rest: the start of a one-node context of zero acceleration
    lbm_ctx *c = nullptr;
    int rc = lbm_init(&q_, nullptr, nullptr, nullptr, &c);
    if (rc) return rc;
    f0_.assign(Q, 0.0);
    rc = lbm_get_populations(c, 1, nullptr, f0_.data());
    lbm_free(c);
    if (rc) return rc;
    const double h = 1e-6;
    CollisionBatch B = batch();
    rvec f;
    const gvec zero = {0, 0, 0};
    for (int col = 0; col < Q; ++col)
      for (double s : {1.0, -1.0}) {
        f = f0_;
        f[col] += s * h;
        B.add(f, zero);
      }
    for (int a = 0; a < D; ++a)
      for (double s : {1.0, -1.0}) {
        gvec g = zero;
        g[a] = s * h;
        B.add(f0_, g);
      }
    if ((rc = B.run())) return rc;
    J_.assign((size_t)Q * Q, 0.0);
    G_.assign((size_t)Q * 3, 0.0);
    for (int col = 0; col < Q; ++col)
      for (int i = 0; i < Q; ++i)
        J_[(size_t)i * Q + col] = (B.value(2 * col, i) - B.value(2 * col + 1, i)) / (2 * h);
    for (int a = 0; a < D; ++a)
      for (int i = 0; i < Q; ++i)
        G_[(size_t)i * 3 + a] =
            (B.value(2 * Q + 2 * a, i) - B.value(2 * Q + 2 * a + 1, i)) / (2 * h);
    return LBM_OK;
  }

  // A real mixed derivative of order m (2 to 4) along m real directions, planned as the
  // 2^m points f0 + h sum_k s_k x_k / |x_k| (s_k = +-1) and read out as
  // sum s_1..s_m C / (2^m h^m) times the directions' scales.  A zero direction makes it 0.
  struct RealJob {
    int base = -1;
    double scale = 0;
    int m = 0;
  };
  RealJob plan_real(CollisionBatch &B, const RDir *const *x, int m) const {
    RealJob j;
    j.m = m;
    double norm[4];
    for (int k = 0; k < m; ++k) {
      norm[k] = max_abs(*x[k]);
      if (norm[k] == 0) return j;
    }
    const double h = m == 2 ? 1e-4 : (m == 3 ? 5e-4 : 2e-3);
    rvec f(Q);
    for (int s = 0; s < (1 << m); ++s) {
      gvec g = {0, 0, 0};
      for (int i = 0; i < Q; ++i) f[i] = f0_[i];
      for (int k = 0; k < m; ++k) {
        const double c = ((s >> k) & 1 ? -h : h) / norm[k];
        for (int i = 0; i < Q; ++i) f[i] += c * x[k]->f[i];
        for (int a = 0; a < 3; ++a) g[a] += c * x[k]->g[a];
      }
      const int id = B.add(f, g);
      if (s == 0) j.base = id;
    }
    double sc = 1.0;
    for (int k = 0; k < m; ++k) sc *= norm[k] / (2 * h);
    j.scale = sc;
    return j;
  }
  void read_real(const RealJob &j, const CollisionBatch &B, double sign, cvec &acc,
                 bool imag) const {
    if (j.base < 0) return;
    for (int s = 0; s < (1 << j.m); ++s) {
      int par = 0;
      for (int k = 0; k < j.m; ++k) par ^= (s >> k) & 1;
      const double w = (par ? -1.0 : 1.0) * sign * j.scale;
      for (int i = 0; i < Q; ++i) {
        const double v = w * B.value(j.base + s, i);
        acc[i] += imag ? cplx(0.0, v) : cplx(v, 0.0);
      }
    }
  }

  // The multilinear extension to complex directions (no conjugation): each direction
  // splits into real and imaginary parts; a term with k imaginary parts carries i^k.
  struct ComplexJob {
    std::vector<RealJob> jobs;
    std::vector<int> ipow;  // k of each job
  };
  ComplexJob plan_complex(CollisionBatch &B, const Dir *const *d, int m) const {
    ComplexJob cj;
    RDir parts[4][2];
    for (int k = 0; k < m; ++k) {
      parts[k][0] = part(*d[k], false);
      parts[k][1] = part(*d[k], true);
    }
    for (int s = 0; s < (1 << m); ++s) {
      const RDir *x[4];
      int k_im = 0;
      for (int k = 0; k < m; ++k) {
        const int im = (s >> k) & 1;
        x[k] = &parts[k][im];
        k_im += im;
      }
      cj.jobs.push_back(plan_real(B, x, m));
      cj.ipow.push_back(k_im);
    }
    return cj;
  }
  cvec read_complex(const ComplexJob &cj, const CollisionBatch &B) const {
    cvec acc(Q, cplx(0.0));
    for (size_t t = 0; t < cj.jobs.size(); ++t) {
      const int k = cj.ipow[t] & 3;  // i^k: 1, i, -1, -i
      read_real(cj.jobs[t], B, (k == 2 || k == 3) ? -1.0 : 1.0, acc, k & 1);
    }
    return acc;
  }

  // The steady wave f at the integer wavevector k (period box) under the per-step source
  // s added after the collision: f = S (J f + s), S = diag(exp(-i kappa . e_i)),
  // kappa = 2 pi k / box (the pull moves node x - e_i's value to x).
  bool steady(const kvec &k, int box, const cvec &s, cvec &f) const {
    const double two_pi = 2.0 * std::acos(-1.0);
    std::vector<cplx> A((size_t)Q * Q);
    f.assign(Q, cplx(0.0));
    for (int i = 0; i < Q; ++i) {
      double ph = 0;
      for (int a = 0; a < 3; ++a) ph += two_pi * k[a] / box * E[3 * i + a];
      const cplx sh = std::polar(1.0, -ph);
      f[i] = sh * s[i];
      for (int col = 0; col < Q; ++col)
        A[(size_t)i * Q + col] =
            (i == col ? cplx(1.0) : cplx(0.0)) - sh * J_[(size_t)i * Q + col];
    }
    return solve_complex(Q, A, f);
  }

  // The steady mean (zero wavevector) under the constant source s, with the mean's mass
  // and momentum held at zero: there (I - J) is singular on the conserved moments M
  // (rows 1, e_x, e_y, e_z), so solve (I - J + B M) f = s - B (M B)^-1 M s with
  // B = f0 M^T; multiplying by M, which J leaves unchanged, gives M f = 0 and then
  // (I - J) f = s once s has no conserved part (any such part would be a drift, not a
  // steady state, and is dropped).
  bool steady_mean(const cvec &s, cvec &f) const {
    const int nc = D + 1;
    auto mrow = [&](int r, int i) { return r == 0 ? 1.0 : double(E[3 * i + (r - 1)]); };
    std::vector<cplx> MB((size_t)nc * nc, cplx(0.0));
    cvec Ms(nc, cplx(0.0));
    for (int r = 0; r < nc; ++r) {
      for (int i = 0; i < Q; ++i) Ms[r] += mrow(r, i) * s[i];
      for (int c = 0; c < nc; ++c)
        for (int i = 0; i < Q; ++i) MB[(size_t)r * nc + c] += mrow(r, i) * f0_[i] * mrow(c, i);
    }
    if (!solve_complex(nc, MB, Ms)) return false;  // Ms = (M B)^-1 M s
    std::vector<cplx> A((size_t)Q * Q);
    f.assign(Q, cplx(0.0));
    for (int i = 0; i < Q; ++i) {
      f[i] = s[i];
      for (int c = 0; c < nc; ++c) f[i] -= f0_[i] * mrow(c, i) * Ms[c];
      for (int col = 0; col < Q; ++col) {
        double bm = 0;
        for (int c = 0; c < nc; ++c) bm += f0_[i] * mrow(c, i) * mrow(c, col);
        A[(size_t)i * Q + col] = (i == col ? 1.0 : 0.0) - J_[(size_t)i * Q + col] + bm;
      }
    }
    return solve_complex(Q, A, f);
  }

  bool solve_wave(const kvec &k, int box, const cvec &s, cvec &f) const {
    return (k[0] == 0 && k[1] == 0 && k[2] == 0) ? steady_mean(s, f) : steady(k, box, s, f);
  }

  // First-order wave of the unit forcing g = p sin(theta) = Re[(-i p) e^{i theta}]: the
  // source is G (-i p).
  bool first(const kvec &k, const double p[3], int box, cvec &f) const {
    cvec s(Q, cplx(0.0));
    for (int i = 0; i < Q; ++i)
      for (int a = 0; a < 3; ++a) s[i] += G_[(size_t)i * 3 + a] * cplx(0.0, -p[a]);
    return steady(k, box, s, f);
  }

 private:
  lbm_params q_;
  rvec f0_, J_, G_;

 public:
  const int Q, D;
  const int *E;
};

// The one-node periodic binary64 lattice of params' collision and rates, at rest.
lbm_params one_node_params(const lbm_params &params) {
  lbm_params q = params;
  q.storage = LBM_F64;
  q.nx = q.ny = q.nz = 1;
  for (int a = 0; a < 3; ++a) q.bc[a] = LBM_PERIODIC;
  q.g_kind = LBM_G_UNIFORM;
  q.g_uniform[0] = q.g_uniform[1] = q.g_uniform[2] = 0.0;
  q.g_data = nullptr;
  q.solid = nullptr;
  q.monitor_every = 0;
  q.mach_limit = 0.0;
  q.debug_poison = 0;
  if (q.rho0 == 0) q.rho0 = 1.0;
  return q;
}

int check_problem(const lbm_params *params, const lbm_ws_problem *p, int box) {
  using lbm::set_error;
  if (!params || !p) return set_error(LBM_EINVAL, "NULL argument");
  if (box < 1) return set_error(LBM_EINVAL, "box = %d must be positive", box);
  if (p->nmodes < 1 || p->nmodes > 8)
    return set_error(LBM_EINVAL, "nmodes = %d must be in 1..8", (int)p->nmodes);
  if (params->lattice == LBM_D3Q39)
    return set_error(LBM_EINVAL, "the expansion covers D2Q9, D3Q19 and D3Q27");
  const bool two_d = params->lattice == LBM_D2Q9;
  for (int j = 0; j < p->nmodes; ++j) {
    const double *k = p->k[j];
    for (int a = 0; a < 3; ++a)
      if (!(std::abs(k[a]) <= 1e6) || k[a] != std::nearbyint(k[a]))
        return set_error(LBM_EINVAL, "mode %d: k must be integers", j);
    if (k[0] == 0 && k[1] == 0 && k[2] == 0)
      return set_error(LBM_EINVAL, "mode %d has k = 0", j);
    if (two_d && (k[2] != 0 || p->p[j][2] != 0))
      return set_error(LBM_EINVAL, "mode %d: a D2Q9 mode must lie in the x-y plane", j);
  }
  return LBM_OK;
}

kvec kint(const double k[3]) {
  return {(int)std::lround(k[0]), (int)std::lround(k[1]), (int)std::lround(k[2])};
}
kvec add(const kvec &a, const kvec &b, int sb) {
  return {a[0] + sb * b[0], a[1] + sb * b[1], a[2] + sb * b[2]};
}
// A wave Re[X e^{i k.x}] equals Re[conj(X) e^{-i k.x}]: the canonical wavevector has its
// first nonzero component positive.
bool flip(const kvec &k) {
  for (int a = 0; a < 3; ++a)
    if (k[a] != 0) return k[a] < 0;
  return false;
}

}  // namespace

extern "C" int lbm_ws_lattice_response(const lbm_params *params, const lbm_ws_problem *p,
                                       int32_t box, double *coef) {
  using lbm::set_error;
  if (!coef) return set_error(LBM_EINVAL, "NULL argument");
  int rc = check_problem(params, p, box);
  if (rc) return rc;
  const lbm_params q = one_node_params(*params);
  Expansion X(q);
  if ((rc = X.build())) return rc;
  const double nu = (params->tau[2] - 0.5) / 3.0;
  const double two_pi = 2.0 * std::acos(-1.0);
  for (int j = 0; j < p->nmodes; ++j) {
    const double *k = p->k[j];
    const double *pol = p->p[j];
    const double K = two_pi * std::sqrt(k[0] * k[0] + k[1] * k[1] + k[2] * k[2]) / box;
    cvec f;
    if (!X.first(kint(k), pol, box, f))
      return set_error(LBM_EINVAL, "mode %d: the linearised step is singular", j);
    // density and physical velocity u = j/rho + g/2 to first order about rest
    cplx rho = 0, u[3] = {0, 0, 0};
    for (int i = 0; i < X.Q; ++i) {
      rho += f[i];
      for (int a = 0; a < 3; ++a) u[a] += double(X.E[3 * i + a]) * f[i];
    }
    const double s = 1.0 / (nu * K * K);  // Stokes amplitude per unit forcing
    double *c = coef + (size_t)8 * j;
    for (int a = 0; a < 3; ++a) {
      const cplx ua = u[a] / q.rho0 + 0.5 * cplx(0.0, -pol[a]);
      // Re[ua e^{i theta}] = Re(ua) cos(theta) - Im(ua) sin(theta)
      c[a] = -ua.imag() / s - pol[a];
      c[3 + a] = ua.real() / s;
    }
    c[6] = -rho.imag() / s;
    c[7] = rho.real() / s;
  }
  return LBM_OK;
}

namespace {

// The waves of orders 1..order, emitted order by order; ends (may be NULL) receives after
// each order n the number of waves written so far (ends[n - 1]).
int lattice_waves(const lbm_params *params, const lbm_ws_problem *p, int32_t box,
                  int32_t order, int32_t max_waves, int32_t *k_out, double *phase_out,
                  double *amp_out, int32_t *count, int32_t *ends) {
  using lbm::set_error;
  if (!k_out || !phase_out || !amp_out || !count) return set_error(LBM_EINVAL, "NULL argument");
  int rc = check_problem(params, p, box);
  if (rc) return rc;
  if (order < 1 || order > 4) return set_error(LBM_EINVAL, "order = %d must be 1 to 4", order);
  const int n = p->nmodes;
  const int need = lbm_ws_max_waves(n, order);
  if (max_waves < need)
    return set_error(LBM_EINVAL, "max_waves = %d is below %d", (int)max_waves, need);
  const lbm_params q = one_node_params(*params);
  Expansion X(q);
  if ((rc = X.build())) return rc;
  const int Q = X.Q;
  int w = 0;
  auto emit = [&](const kvec &k, double phase, const cvec &amp, cplx scale) {
    if (w >= max_waves) return;  // cannot happen: max_waves covers the bound
    for (int a = 0; a < 3; ++a) k_out[3 * w + a] = k[a];
    phase_out[w] = phase;
    for (int i = 0; i < Q; ++i) {
      const cplx v = scale * amp[i];
      amp_out[((size_t)w * Q + i) * 2] = v.real();
      amp_out[((size_t)w * Q + i) * 2 + 1] = v.imag();
    }
    ++w;
  };
  // First order: each mode's own wave.  a_j = amp_j e^{i phase_j} (f_j, -i p_j) is the
  // mode's direction of the expansion in (populations, g) with its phase folded in, so
  // the first-order state is sum_j Re[a_j e^{i kappa_j . x}].
  std::vector<Dir> a1(n);
  std::vector<kvec> k1(n);
  for (int j = 0; j < n; ++j) {
    k1[j] = kint(p->k[j]);
    cvec f;
    if (!X.first(k1[j], p->p[j], box, f))
      return set_error(LBM_EINVAL, "mode %d: the linearised step is singular", j);
    emit(k1[j], p->phase[j], f, p->amp[j]);
    Dir d;
    d.f = f;
    for (int a = 0; a < 3; ++a) d.g[a] = cplx(0.0, -p->p[j][a]);
    a1[j] = scaled(d, std::polar(p->amp[j], p->phase[j]));
  }
  if (ends) ends[0] = w;
  if (order == 1) {
    *count = w;
    return LBM_OK;
  }
  struct Item {
    kvec k;
    double c;
    Expansion::ComplexJob job;
  };
  // Second order: the Taylor term D2(delta, delta) / 2 of the collision with
  // delta = sum_j Re[a_j e^{i theta_j}].  By Re[a e^{i alpha}] Re[b e^{i beta}] =
  // (Re[a b e^{i(alpha+beta)}] + Re[a conj(b) e^{i(alpha-beta)}]) / 2, each pair i <= j
  // drives the wave k_i + k_j with source D2(a_i, a_j) / 2 and the wave k_i - k_j with
  // source D2(a_i, conj a_j) / 2, each 1/4 instead when i = j (the orderings (i, j) and
  // (j, i) coincide).  A wave of zero wavevector (the mean part, always present for
  // i = j) is the steady mean.
  struct Wave {
    kvec k;
    cvec f;  // population amplitude, phase folded in
  };
  std::vector<Wave> w2, w3;
  const kvec zero_k = {0, 0, 0};
  {
    CollisionBatch B = X.batch();
    std::vector<Item> items;
    std::vector<Dir> ac(n);
    for (int j = 0; j < n; ++j) ac[j] = conj(a1[j]);
    for (int i = 0; i < n; ++i)
      for (int j = i; j < n; ++j)
        for (int sgn : {1, -1}) {
          const Dir *d[2] = {&a1[i], sgn > 0 ? &a1[j] : &ac[j]};
          items.push_back({add(k1[i], k1[j], sgn), i == j ? 0.25 : 0.5,
                           X.plan_complex(B, d, 2)});
        }
    if ((rc = B.run())) return rc;
    for (const Item &it : items) {
      cvec src = X.read_complex(it.job, B), f2;
      for (auto &v : src) v *= it.c;
      if (!X.solve_wave(it.k, box, src, f2))
        return set_error(LBM_EINVAL, "a second-order wave: the linearised step is singular");
      emit(it.k, 0.0, f2, 1.0);
      w2.push_back({it.k, f2});
    }
  }
  if (ends) ends[1] = w;
  if (order == 2) {
    *count = w;
    return LBM_OK;
  }
  // Third order: the cross term D2(delta1, delta2) of the second-order Taylor term (the
  // first-order directions a_j against the second-order population waves b_w, which
  // carry no acceleration) and the cubic term D3(delta1, delta1, delta1) / 6.
  //   cross: each (j, w) drives k_j + q_w with D2(a_j, b_w) / 2 and k_j - q_w with
  //     D2(a_j, conj b_w) / 2;
  //   cubic: with delta1 = sum over the 2n signed components c of (a_c e^{i k_c . x}) / 2
  //     (a_c = a_j or conj a_j, k_c = +-k_j), the term is
  //     sum over ordered triples D3(a_c1, a_c2, a_c3) e^{i (k_c1 + k_c2 + k_c3) . x} / 48;
  //     an unordered triple M with m orderings and its conjugate M* (every sign flipped,
  //     never equal to M) together give Re[m D3(...) / 24 e^{i k_M . x}].
  // Sources at the same wavevector are summed (a wave at -k as the conjugate at k) and
  // solved once per wavevector.
  {
    CollisionBatch B = X.batch();
    std::vector<Item> items;
    std::vector<Dir> b2(w2.size()), b2c(w2.size());
    for (size_t v = 0; v < w2.size(); ++v) {
      b2[v].f = w2[v].f;
      b2c[v] = conj(b2[v]);
    }
    for (int j = 0; j < n; ++j)
      for (size_t v = 0; v < w2.size(); ++v)
        for (int sgn : {1, -1}) {
          const Dir *d[2] = {&a1[j], sgn > 0 ? &b2[v] : &b2c[v]};
          items.push_back({add(k1[j], w2[v].k, sgn), 0.5, X.plan_complex(B, d, 2)});
        }
    std::vector<Dir> comp(2 * n);  // signed component c = 2 j + (sign < 0)
    for (int j = 0; j < n; ++j) {
      comp[2 * j] = a1[j];
      comp[2 * j + 1] = conj(a1[j]);
    }
    auto ck = [&](int c) { return (c & 1) ? add(zero_k, k1[c >> 1], -1) : k1[c >> 1]; };
    for (int c1 = 0; c1 < 2 * n; ++c1)
      for (int c2 = c1; c2 < 2 * n; ++c2)
        for (int c3 = c2; c3 < 2 * n; ++c3) {
          const std::array<int, 3> m = {c1, c2, c3};
          std::array<int, 3> mc = {c1 ^ 1, c2 ^ 1, c3 ^ 1};
          std::sort(mc.begin(), mc.end());
          if (!(m < mc)) continue;  // one of each conjugate pair
          const int orderings = (c1 == c2 && c2 == c3) ? 1 : (c1 == c2 || c2 == c3) ? 3 : 6;
          const Dir *d[3] = {&comp[c1], &comp[c2], &comp[c3]};
          items.push_back({add(add(ck(c1), ck(c2), 1), ck(c3), 1), orderings / 24.0,
                           X.plan_complex(B, d, 3)});
        }
    if ((rc = B.run())) return rc;
    std::map<kvec, cvec> src;
    for (const Item &it : items) {
      const cvec s = X.read_complex(it.job, B);
      kvec k = it.k;
      const bool fl = flip(k);
      if (fl) k = {-k[0], -k[1], -k[2]};
      cvec &acc = src[k];
      if (acc.empty()) acc.assign(Q, cplx(0.0));
      for (int i = 0; i < Q; ++i) acc[i] += it.c * (fl ? std::conj(s[i]) : s[i]);
    }
    for (const auto &kv : src) {
      cvec f3;
      if (!X.solve_wave(kv.first, box, kv.second, f3))
        return set_error(LBM_EINVAL, "a third-order wave: the linearised step is singular");
      emit(kv.first, 0.0, f3, 1.0);
      w3.push_back({kv.first, f3});
    }
  }
  if (ends) ends[2] = w;
  if (order == 3) {
    *count = w;
    return LBM_OK;
  }
  // Fourth order: D2(delta1, delta3) + D2(delta2, delta2) / 2 + D3(delta1, delta1, delta2) / 2
  // + D4(delta1, delta1, delta1, delta1) / 24 (the fourth-order part of the Taylor series
  // of the collision).  Each delta_n is written as its conjugate-closed components
  // c = (k_c, v_c): (k, b / 2) and (-k, conj b / 2) for a wave Re[b e^{i k.x}], so a
  // multilinear term is a sum over tuples of components of D(v_c1, ...) e^{i (k_c1 + ...).x}.
  // Tuples drawn from one delta are taken as unordered multisets times their number of
  // orderings (the derivatives are symmetric).  The total at -k is the conjugate of that
  // at k, so only tuples whose wavevector is canonical or zero are evaluated; a canonical
  // k then carries 2 X_k and the mean X_0.
  {
    struct Comp {
      kvec k;
      Dir v;
    };
    auto comps = [&](const std::vector<Wave> &ws, std::vector<Comp> &out) {
      for (const Wave &wv : ws) {
        Dir d;
        d.f = wv.f;
        out.push_back({wv.k, scaled(d, 0.5)});
        out.push_back({add(zero_k, wv.k, -1), scaled(conj(d), 0.5)});
      }
    };
    std::vector<Comp> c1, c2, c3;
    for (int j = 0; j < n; ++j) {
      c1.push_back({k1[j], scaled(a1[j], 0.5)});
      c1.push_back({add(zero_k, k1[j], -1), scaled(conj(a1[j]), 0.5)});
    }
    comps(w2, c2);
    comps(w3, c3);
    CollisionBatch B = X.batch();
    std::vector<Item> items;
    auto plan = [&](std::initializer_list<const Comp *> cs, double coef) {
      kvec k = zero_k;
      const Dir *d[4];
      int m = 0;
      for (const Comp *c : cs) {
        k = add(k, c->k, 1);
        d[m++] = &c->v;
      }
      if (flip(k)) return;
      items.push_back({k, coef, X.plan_complex(B, d, m)});
    };
    auto orderings = [](std::initializer_list<int> idx) {
      // m! / prod(multiplicity!) for a sorted multiset of at most four indices
      std::vector<int> v(idx);
      int fact[5] = {1, 1, 2, 6, 24}, den = 1, run = 1;
      for (size_t t = 1; t <= v.size(); ++t) {
        if (t < v.size() && v[t] == v[t - 1]) {
          ++run;
        } else {
          den *= fact[run];
          run = 1;
        }
      }
      return fact[v.size()] / den;
    };
    for (const Comp &a : c1)
      for (const Comp &b : c3) plan({&a, &b}, 1.0);
    for (size_t i = 0; i < c2.size(); ++i)
      for (size_t j = i; j < c2.size(); ++j)
        plan({&c2[i], &c2[j]}, 0.5 * orderings({(int)i, (int)j}));
    for (size_t i = 0; i < c1.size(); ++i)
      for (size_t j = i; j < c1.size(); ++j)
        for (const Comp &c : c2) plan({&c1[i], &c1[j], &c}, 0.5 * orderings({(int)i, (int)j}));
    for (size_t i = 0; i < c1.size(); ++i)
      for (size_t j = i; j < c1.size(); ++j)
        for (size_t k = j; k < c1.size(); ++k)
          for (size_t l = k; l < c1.size(); ++l)
            plan({&c1[i], &c1[j], &c1[k], &c1[l]},
                 orderings({(int)i, (int)j, (int)k, (int)l}) / 24.0);
    if ((rc = B.run())) return rc;
    std::map<kvec, cvec> src;
    for (const Item &it : items) {
      const cvec s4 = X.read_complex(it.job, B);
      cvec &acc = src[it.k];
      if (acc.empty()) acc.assign(Q, cplx(0.0));
      for (int i = 0; i < Q; ++i) acc[i] += it.c * s4[i];
    }
    for (auto &kv : src) {
      const bool mean = kv.first == zero_k;
      if (!mean)
        for (auto &v : kv.second) v *= 2.0;
      cvec f4;
      if (!X.solve_wave(kv.first, box, kv.second, f4))
        return set_error(LBM_EINVAL, "a fourth-order wave: the linearised step is singular");
      emit(kv.first, 0.0, f4, 1.0);
    }
  }
  if (ends) ends[3] = w;
  *count = w;
  return LBM_OK;
}

}  // namespace

extern "C" int lbm_ws_lattice_waves(const lbm_params *params, const lbm_ws_problem *p,
                                    int32_t box, int32_t order, int32_t max_waves,
                                    int32_t *k_out, double *phase_out, double *amp_out,
                                    int32_t *count) {
  return lattice_waves(params, p, box, order, max_waves, k_out, phase_out, amp_out, count,
                       nullptr);
}

extern "C" int lbm_ws_lattice_waves_ordered(const lbm_params *params, const lbm_ws_problem *p,
                                            int32_t box, int32_t order, int32_t max_waves,
                                            int32_t *k_out, double *phase_out,
                                            double *amp_out, int32_t *count,
                                            int32_t *order_end) {
  if (!order_end) return lbm::set_error(LBM_EINVAL, "order_end is NULL");
  for (int n = 0; n < 4; ++n) order_end[n] = 0;
  int rc = lattice_waves(params, p, box, order, max_waves, k_out, phase_out, amp_out, count,
                         order_end);
  if (rc) return rc;
  for (int n = order; n < 4; ++n) order_end[n] = *count;
  return LBM_OK;
}

extern "C" int lbm_ws_resum_features(const lbm_ws_problem *p, int32_t box, int32_t Q,
                                     const double *amp, const int32_t *order_end,
                                     float *feat, double *sigma) {
  using lbm::set_error;
  if (!p || !amp || !order_end || !feat || !sigma) return set_error(LBM_EINVAL, "NULL argument");
  if (p->nmodes != 4) return set_error(LBM_EINVAL, "nmodes = %d: the features need 4", p->nmodes);
  if (box < 1 || Q < 1) return set_error(LBM_EINVAL, "box and Q must be positive");
  if (!(p->tau2 > 0.5)) return set_error(LBM_EINVAL, "tau2 must exceed 1/2");
  // root-sum-square amplitude of each order's waves
  double a[4];
  int lo = 0;
  for (int n = 0; n < 4; ++n) {
    const int hi = order_end[n];
    if (hi < lo) return set_error(LBM_EINVAL, "order_end must not decrease");
    double s = 0.0;
    for (int64_t j = (int64_t)lo * Q * 2; j < (int64_t)hi * Q * 2; ++j) s += amp[j] * amp[j];
    a[n] = std::sqrt(s);
    lo = hi;
  }
  if (!(a[0] > 0) || !(a[1] > 0) || !(a[2] > 0) || !(a[3] > 0))
    return set_error(LBM_EINVAL, "the features need waves of all four orders");
  // sigma^2 = a3^2 / (a2 a1): the series' ratio applied once more, relative to order 1
  *sigma = a[2] / std::sqrt(a[1] * a[0]);
  const double nu = (p->tau2 - 0.5) / 3.0;
  struct M {
    double s, K, Re;
  };
  M m[4];
  double U = 0.0, Remax = 0.0;
  for (int j = 0; j < 4; ++j) {
    double kk = 0.0;
    for (int c = 0; c < 3; ++c) kk += p->k[j][c] * p->k[j][c];
    const double K = 2.0 * M_PI * std::sqrt(kk) / box;
    m[j] = {p->amp[j] / (nu * K * K), K, p->amp[j] / (nu * nu * K * K * K)};
    U += m[j].s;
    Remax = std::max(Remax, m[j].Re);
  }
  // modes by decreasing Stokes amplitude (ties keep their order)
  int ord[4] = {0, 1, 2, 3};
  for (int i = 1; i < 4; ++i)
    for (int j = i; j > 0 && m[ord[j]].s > m[ord[j - 1]].s; --j) std::swap(ord[j], ord[j - 1]);
  int f = 0;
  feat[f++] = (float)(p->tau2 - 0.5);
  feat[f++] = (float)std::log10(*sigma);
  feat[f++] = (float)std::log10(a[1] / a[0]);
  feat[f++] = (float)std::log10(a[2] / a[0]);
  feat[f++] = (float)std::log10(a[3] / a[0]);
  feat[f++] = (float)std::log10(U);
  feat[f++] = (float)std::log10(Remax);
  for (int i = 0; i < 4; ++i) {
    const M &q = m[ord[i]];
    feat[f++] = (float)(q.s / U);
    feat[f++] = (float)q.K;
    feat[f++] = (float)std::log10(q.Re);
  }
  return f == LBM_WS_RESUM_FEATURES ? LBM_OK : set_error(LBM_EINVAL, "feature count");
}

extern "C" int lbm_ws_scale_orders(double *amp, int32_t Q, const int32_t *order_end,
                                   const double *c) {
  if (!amp || !order_end || !c || Q < 1) return lbm::set_error(LBM_EINVAL, "bad argument");
  int lo = 0;
  for (int n = 0; n < 4; ++n) {
    const int hi = order_end[n];
    if (hi < lo) return lbm::set_error(LBM_EINVAL, "order_end must not decrease");
    if (!std::isfinite(c[n])) return lbm::set_error(LBM_EINVAL, "c[%d] is not finite", n);
    for (int64_t j = (int64_t)lo * Q * 2; j < (int64_t)hi * Q * 2; ++j) amp[j] *= c[n];
    lo = hi;
  }
  return LBM_OK;
}

extern "C" int32_t lbm_ws_max_waves(int32_t nmodes, int32_t order) {
  if (nmodes < 1 || nmodes > 8 || order < 1 || order > 4) return 0;
  const int64_t n = nmodes;
  auto multisets = [](int64_t m, int64_t r) {  // C(m + r - 1, r)
    int64_t c = 1;
    for (int64_t t = 1; t <= r; ++t) c = c * (m + t - 1) / t;
    return c;
  };
  const int64_t n2 = n * (n + 1);                                  // second order
  const int64_t n3 = 2 * n * n2 + multisets(2 * n, 3);             // third order
  int64_t c = n;                                                   // first order
  if (order >= 2) c += n2;  // a sum and a difference per pair i <= j
  if (order >= 3) c += n3;  // at most one wavevector per planned item
  if (order >= 4)
    c += 2 * n * 2 * n3 + multisets(2 * n2, 2) + multisets(2 * n, 2) * 2 * n2 +
         multisets(2 * n, 4);
  return (int32_t)c;
}
