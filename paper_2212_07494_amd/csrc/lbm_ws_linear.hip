// Steady response of the forced periodic lattice to Fourier forcing modes, order by order
// in the forcing amplitude (lbm_ws_lattice_response: first order, as mode coefficients;
// lbm_ws_lattice_waves: first and second order, as population waves).  Host code: the
// collision's first and second derivatives about rest are taken by central differences
// of the library's own step on one-node periodic lattices, where the pull streaming maps
// every population onto itself, so one step is one collision.  Each wave of the response
// is then one Q x Q complex solve.
#include <array>
#include <cmath>
#include <complex>
#include <map>
#include <tuple>
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

// The collision of one node, C(f, g), as the library computes it: one step of a one-node
// periodic binary64 lattice of uniform acceleration g (a context per distinct g, made on
// first use and kept until destruction).
class NodeCollision {
 public:
  explicit NodeCollision(const lbm_params &q) : q_(q) {}
  ~NodeCollision() {
    for (auto &kv : ctx_) lbm_free(kv.second);
  }
  NodeCollision(const NodeCollision &) = delete;
  NodeCollision &operator=(const NodeCollision &) = delete;

  // Rest populations (the start of a context of zero acceleration).
  int rest(rvec &f0) {
    lbm_ctx *c = nullptr;
    const int rc = context({0.0, 0.0, 0.0}, &c);
    if (rc) return rc;
    f0.assign(lbm::ops_for(q_.lattice).Q, 0.0);
    return lbm_get_populations(c, 1, nullptr, f0.data());
  }
  int operator()(const rvec &f, const gvec &g, rvec &out) {
    lbm_ctx *c = nullptr;
    int rc = context(g, &c);
    if (rc) return rc;
    out.assign(f.size(), 0.0);
    const double one = 1.0;
    rc = lbm_set_populations(c, f.data());
    if (!rc) rc = lbm_step(c, 1, &one);
    if (!rc) rc = lbm_get_populations(c, 1, nullptr, out.data());
    return rc;
  }

 private:
  int context(const gvec &g, lbm_ctx **out) {
    const auto key = std::make_tuple(g[0], g[1], g[2]);
    auto it = ctx_.find(key);
    if (it != ctx_.end()) {
      *out = it->second;
      return LBM_OK;
    }
    lbm_params q = q_;
    for (int a = 0; a < 3; ++a) q.g_uniform[a] = g[a];
    lbm_ctx *c = nullptr;
    const int rc = lbm_init(&q, nullptr, nullptr, nullptr, &c);
    if (rc) return rc;
    ctx_[key] = c;
    *out = c;
    return LBM_OK;
  }
  lbm_params q_;
  std::map<std::tuple<double, double, double>, lbm_ctx *> ctx_;
};

// The collision expanded about rest: J = dC/d f-bar (Q x Q), G = dC/dg (Q x 3), and the
// second derivative along two directions; and the steady periodic waves they drive.
class Expansion {
 public:
  explicit Expansion(const lbm_params &q)
      : C_(q), Q(lbm::ops_for(q.lattice).Q), D(lbm::ops_for(q.lattice).D),
        E(lbm::ops_for(q.lattice).E) {}

  int build() {
    int rc = C_.rest(f0_);
    if (rc) return rc;
    const double h = 1e-6;
    const gvec zero = {0, 0, 0};
    J_.assign((size_t)Q * Q, 0.0);
    G_.assign((size_t)Q * 3, 0.0);
    rvec fp, fm, cp, cm;
    for (int col = 0; col < Q; ++col) {
      fp = f0_;
      fm = f0_;
      fp[col] += h;
      fm[col] -= h;
      if ((rc = C_(fp, zero, cp)) || (rc = C_(fm, zero, cm))) return rc;
      for (int i = 0; i < Q; ++i) J_[(size_t)i * Q + col] = (cp[i] - cm[i]) / (2 * h);
    }
    for (int a = 0; a < D; ++a) {
      gvec gp = {0, 0, 0}, gm = {0, 0, 0};
      gp[a] = h;
      gm[a] = -h;
      if ((rc = C_(f0_, gp, cp)) || (rc = C_(f0_, gm, cm))) return rc;
      for (int i = 0; i < Q; ++i) G_[(size_t)i * 3 + a] = (cp[i] - cm[i]) / (2 * h);
    }
    return LBM_OK;
  }

  // Mixed second derivative of C along the real directions (a, ga) and (b, gb).
  int d2(const rvec &a, const gvec &ga, const rvec &b, const gvec &gb, rvec &out) {
    const double h = 1e-4;
    const double sa[4] = {1, 1, -1, -1}, sb[4] = {1, -1, 1, -1};
    rvec f(Q), c[4];
    for (int t = 0; t < 4; ++t) {
      gvec g;
      for (int i = 0; i < Q; ++i) f[i] = f0_[i] + h * (sa[t] * a[i] + sb[t] * b[i]);
      for (int k = 0; k < 3; ++k) g[k] = h * (sa[t] * ga[k] + sb[t] * gb[k]);
      const int rc = C_(f, g, c[t]);
      if (rc) return rc;
    }
    out.assign(Q, 0.0);
    for (int i = 0; i < Q; ++i)
      out[i] = ((c[0][i] - c[1][i]) - (c[2][i] - c[3][i])) / (4 * h * h);
    return LBM_OK;
  }

  // Its bilinear extension to complex directions (no conjugation).
  int d2c(const cvec &a, const gcvec &ga, const cvec &b, const gcvec &gb, cvec &out) {
    rvec ar(Q), ai(Q), br(Q), bi(Q), rr, ii, ri, ir;
    gvec gar, gai, gbr, gbi;
    for (int i = 0; i < Q; ++i) {
      ar[i] = a[i].real();
      ai[i] = a[i].imag();
      br[i] = b[i].real();
      bi[i] = b[i].imag();
    }
    for (int k = 0; k < 3; ++k) {
      gar[k] = ga[k].real();
      gai[k] = ga[k].imag();
      gbr[k] = gb[k].real();
      gbi[k] = gb[k].imag();
    }
    int rc;
    if ((rc = d2(ar, gar, br, gbr, rr)) || (rc = d2(ai, gai, bi, gbi, ii)) ||
        (rc = d2(ar, gar, bi, gbi, ri)) || (rc = d2(ai, gai, br, gbr, ir)))
      return rc;
    out.assign(Q, cplx(0.0));
    for (int i = 0; i < Q; ++i) out[i] = cplx(rr[i] - ii[i], ri[i] + ir[i]);
    return LBM_OK;
  }

  // The steady wave f at the integer wavevector k (period box) under the per-step source
  // s added after the collision: f = S (J f + s), S = diag(exp(-i kappa . e_i)),
  // kappa = 2 pi k / box (the pull moves node x - e_i's value to x).
  bool steady(const double k[3], int box, const cvec &s, cvec &f) const {
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

  // First-order wave of the unit forcing g = p sin(theta) = Re[(-i p) e^{i theta}]: the
  // source is G (-i p).
  bool first(const double k[3], const double p[3], int box, cvec &f) const {
    cvec s(Q, cplx(0.0));
    for (int i = 0; i < Q; ++i)
      for (int a = 0; a < 3; ++a) s[i] += G_[(size_t)i * 3 + a] * cplx(0.0, -p[a]);
    return steady(k, box, s, f);
  }

 private:
  NodeCollision C_;
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
  if (q.rho0 == 0) q.rho0 = 1.0;
  return q;
}

int check_problem(const lbm_params *params, const lbm_ws_problem *p, int box) {
  using lbm::set_error;
  if (!params || !p) return set_error(LBM_EINVAL, "NULL argument");
  if (box < 1) return set_error(LBM_EINVAL, "box = %d must be positive", box);
  if (p->nmodes < 1 || p->nmodes > 8)
    return set_error(LBM_EINVAL, "nmodes = %d must be in 1..8", (int)p->nmodes);
  const bool two_d = params->lattice == LBM_D2Q9;
  for (int j = 0; j < p->nmodes; ++j) {
    const double *k = p->k[j];
    if (k[0] == 0 && k[1] == 0 && k[2] == 0)
      return set_error(LBM_EINVAL, "mode %d has k = 0", j);
    if (two_d && (k[2] != 0 || p->p[j][2] != 0))
      return set_error(LBM_EINVAL, "mode %d: a D2Q9 mode must lie in the x-y plane", j);
  }
  return LBM_OK;
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
    if (!X.first(k, pol, box, f))
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

extern "C" int lbm_ws_lattice_waves(const lbm_params *params, const lbm_ws_problem *p,
                                    int32_t box, int32_t order, int32_t max_waves,
                                    int32_t *k_out, double *phase_out, double *amp_out,
                                    int32_t *count) {
  using lbm::set_error;
  if (!k_out || !phase_out || !amp_out || !count) return set_error(LBM_EINVAL, "NULL argument");
  int rc = check_problem(params, p, box);
  if (rc) return rc;
  if (order != 1 && order != 2) return set_error(LBM_EINVAL, "order = %d must be 1 or 2", order);
  const int n = p->nmodes;
  const int need = order == 1 ? n : n + n * (n + 1);
  if (max_waves < need)
    return set_error(LBM_EINVAL, "max_waves = %d is below %d", (int)max_waves, need);
  const lbm_params q = one_node_params(*params);
  Expansion X(q);
  if ((rc = X.build())) return rc;
  const int Q = X.Q;
  int w = 0;
  auto emit = [&](const double k[3], double phase, const cvec &amp, double scale) {
    for (int a = 0; a < 3; ++a) k_out[3 * w + a] = (int32_t)std::lround(k[a]);
    phase_out[w] = phase;
    for (int i = 0; i < Q; ++i) {
      amp_out[((size_t)w * Q + i) * 2] = scale * amp[i].real();
      amp_out[((size_t)w * Q + i) * 2 + 1] = scale * amp[i].imag();
    }
    ++w;
  };
  // first order: each mode's own wave; the direction of the expansion is (f1, -i p)
  std::vector<cvec> f1(n);
  std::vector<gcvec> g1(n);
  for (int j = 0; j < n; ++j) {
    if (!X.first(p->k[j], p->p[j], box, f1[j]))
      return set_error(LBM_EINVAL, "mode %d: the linearised step is singular", j);
    for (int a = 0; a < 3; ++a) g1[j][a] = cplx(0.0, -p->p[j][a]);
    emit(p->k[j], p->phase[j], f1[j], p->amp[j]);
  }
  // second order: the collision's second derivative on two first-order waves drives the
  // waves theta_i + theta_j and theta_i - theta_j (i <= j).  With
  // Re[a e^{i alpha}] Re[b e^{i beta}] = (Re[a b e^{i(alpha+beta)}] +
  // Re[a conj(b) e^{i(alpha-beta)}]) / 2 and the Taylor factor 1/2, the source of a sum
  // wave is a_i a_j D2(z_i, z_j) / 2 and that of a difference wave
  // a_i a_j D2(z_i, conj z_j) / 2, each 1/4 instead when i = j (the orderings (i, j) and
  // (j, i) coincide).  A wave of zero wavevector (the mean part, always present for
  // i = j) is the steady mean.
  if (order == 2)
    for (int i = 0; i < n; ++i)
      for (int j = i; j < n; ++j)
        for (int sgn : {1, -1}) {
          double kq[3];
          for (int a = 0; a < 3; ++a) kq[a] = p->k[i][a] + sgn * p->k[j][a];
          const bool mean = kq[0] == 0 && kq[1] == 0 && kq[2] == 0;
          cvec zb = f1[j];
          gcvec gb = g1[j];
          if (sgn < 0) {
            for (auto &v : zb) v = std::conj(v);
            for (auto &v : gb) v = std::conj(v);
          }
          cvec src, f2;
          if ((rc = X.d2c(f1[i], g1[i], zb, gb, src))) return rc;
          if (!(mean ? X.steady_mean(src, f2) : X.steady(kq, box, src, f2)))
            return set_error(LBM_EINVAL, "wave of modes (%d, %d): the linearised step is singular",
                             i, j);
          const double scale = p->amp[i] * p->amp[j] * (i == j ? 0.25 : 0.5);
          emit(kq, p->phase[i] + sgn * p->phase[j], f2, scale);
        }
  *count = w;
  return LBM_OK;
}
