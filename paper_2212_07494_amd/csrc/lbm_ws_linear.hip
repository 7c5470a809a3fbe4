// Exact linear steady response of the periodic lattice to one Fourier forcing mode
// (lbm_ws_lattice_response).  Host code: the collision's Jacobians at rest are taken by
// central differences of the library's own step on a one-node periodic lattice, where
// the pull streaming maps every population onto itself, so one step is one collision;
// each mode is then one Q x Q complex solve.
#include <cmath>
#include <complex>
#include <vector>

#include "lbm.h"
#include "lbm_internal.h"
#include "lbm_nn.h"

namespace {

using cplx = std::complex<double>;

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

// One collision of the populations f (Q values) with uniform acceleration g_scale * g of
// the context: set, step once, read back.
int collide_once(lbm_ctx *c, const std::vector<double> &f, double g_scale,
                 std::vector<double> &out) {
  int rc = lbm_set_populations(c, f.data());
  if (!rc) rc = lbm_step(c, 1, &g_scale);
  if (!rc) rc = lbm_get_populations(c, 1, nullptr, out.data());
  return rc;
}

struct CtxGuard {
  lbm_ctx *c = nullptr;
  ~CtxGuard() {
    if (c) lbm_free(c);
  }
};

}  // namespace

extern "C" int lbm_ws_lattice_response(const lbm_params *params, const lbm_ws_problem *p,
                                       int32_t box, double *coef) {
  using lbm::set_error;
  if (!params || !p || !coef) return set_error(LBM_EINVAL, "NULL argument");
  if (box < 1) return set_error(LBM_EINVAL, "box = %d must be positive", (int)box);
  if (p->nmodes < 1 || p->nmodes > 8)
    return set_error(LBM_EINVAL, "nmodes = %d must be in 1..8", (int)p->nmodes);
  // a one-node periodic lattice of the same collision, binary64, no force yet
  lbm_params q = *params;
  q.storage = LBM_F64;
  q.nx = q.ny = q.nz = 1;
  for (int a = 0; a < 3; ++a) q.bc[a] = LBM_PERIODIC;
  q.g_kind = LBM_G_UNIFORM;
  q.g_uniform[0] = q.g_uniform[1] = q.g_uniform[2] = 0.0;
  q.g_data = nullptr;
  q.solid = nullptr;
  q.monitor_every = 0;
  if (q.rho0 == 0) q.rho0 = 1.0;
  CtxGuard c0;
  int rc = lbm_init(&q, nullptr, nullptr, nullptr, &c0.c);
  if (rc) return rc;
  const int Q = lbm::ops_for(q.lattice).Q;
  const int D = lbm::ops_for(q.lattice).D;
  std::vector<double> f0(Q), fp(Q), fm(Q), cp(Q), cm(Q);
  if ((rc = lbm_get_populations(c0.c, 1, nullptr, f0.data()))) return rc;

  // J = d collide / d f-bar at rest (column q), G = d collide / d g (column a)
  const double h = 1e-6;
  std::vector<double> J((size_t)Q * Q), G((size_t)Q * 3, 0.0);
  for (int col = 0; col < Q; ++col) {
    fp = f0;
    fm = f0;
    fp[col] += h;
    fm[col] -= h;
    if ((rc = collide_once(c0.c, fp, 0.0, cp)) || (rc = collide_once(c0.c, fm, 0.0, cm)))
      return rc;
    for (int i = 0; i < Q; ++i) J[(size_t)i * Q + col] = (cp[i] - cm[i]) / (2 * h);
  }
  for (int a = 0; a < D; ++a) {
    lbm_params qa = q;
    qa.g_uniform[a] = h;
    CtxGuard ca;
    if ((rc = lbm_init(&qa, nullptr, nullptr, nullptr, &ca.c))) return rc;
    if ((rc = collide_once(ca.c, f0, 1.0, cp)) || (rc = collide_once(ca.c, f0, -1.0, cm)))
      return rc;
    for (int i = 0; i < Q; ++i) G[(size_t)i * 3 + a] = (cp[i] - cm[i]) / (2 * h);
  }

  const int *E = lbm::ops_for(q.lattice).E;
  const double nu = (params->tau[2] - 0.5) / 3.0;
  const double two_pi = 2.0 * std::acos(-1.0);
  for (int j = 0; j < p->nmodes; ++j) {
    const double *k = p->k[j];
    const double *pol = p->p[j];
    const double K = two_pi * std::sqrt(k[0] * k[0] + k[1] * k[1] + k[2] * k[2]) / box;
    if (K == 0) return set_error(LBM_EINVAL, "mode %d has k = 0", j);
    if (D == 2 && (k[2] != 0 || pol[2] != 0))
      return set_error(LBM_EINVAL, "mode %d: a D2Q9 mode must lie in the x-y plane", j);
    // g = p sin(theta) = Re[(-i p) e^{i theta}]; the state's perturbation is
    // Re[fhat e^{i theta}] with fhat = S (J fhat + G ghat), S_i = e^{-i kappa . e_i}
    std::vector<cplx> A((size_t)Q * Q), b(Q);
    for (int i = 0; i < Q; ++i) {
      double ph = 0;
      for (int a = 0; a < 3; ++a) ph += two_pi * k[a] / box * E[3 * i + a];
      const cplx s = std::polar(1.0, -ph);
      cplx gi = 0;
      for (int a = 0; a < 3; ++a) gi += G[(size_t)i * 3 + a] * cplx(0.0, -pol[a]);
      b[i] = s * gi;
      for (int col = 0; col < Q; ++col)
        A[(size_t)i * Q + col] = (i == col ? cplx(1.0) : cplx(0.0)) - s * J[(size_t)i * Q + col];
    }
    if (!solve_complex(Q, A, b))
      return set_error(LBM_EINVAL, "mode %d: the linearised step is singular", j);
    // density and physical velocity u = j/rho + g/2 to first order about rest
    cplx rho = 0, u[3] = {0, 0, 0};
    for (int i = 0; i < Q; ++i) {
      rho += b[i];
      for (int a = 0; a < 3; ++a) u[a] += double(E[3 * i + a]) * b[i];
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
