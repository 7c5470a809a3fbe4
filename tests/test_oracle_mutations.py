"""Planted mistakes in the oracle fail its pins (CPU only).

The oracle is pinned to the paper and to mathematics, not to itself, and the pins are
meant to be sharp enough that a plausible mistake anywhere in it fails one of them.  This
module checks that claim directly: each case copies ``oracle/`` into a temporary
directory, plants one mistake in the copy -- a dropped term, a wrong sign, factor or rate,
a transposed operand, a wrong index or pairing, a wrong streaming or bounce-back
direction -- builds the copy, and runs the pin modules against it in a child process
(the copy comes first on its import path).  Every planted mistake must make a pin fail
(an assertion, not an import or build error).  A control case runs the same harness on
an unplanted copy and must pass, and the child reports which ``oracle`` it imported.

Nothing here touches the product library or a GPU; the repository's oracle is never
modified.
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import re
import shutil
import subprocess
import sys
import tempfile

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
ORACLE = os.path.join(ROOT, "oracle")
T = os.path.join(ROOT, "tests")

# The pins, cheapest first (a caught mistake ends the child at its first failure).
PINS = [
    os.path.join(T, "test_oracle_trapezoid.py"),
    os.path.join(T, "test_oracle_collision.py"),
    os.path.join(T, "test_oracle_lattice.py"),
    os.path.join(T, "test_oracle_d3q39.py"),
    os.path.join(T, "test_oracle_flows.py") + "::test_uniform_force_momentum_balance",
    os.path.join(T, "test_oracle_flows.py") + "::test_uniform_state_accelerates_exactly",
    os.path.join(T, "test_oracle_flows.py") + "::test_equilibrium_is_fixed_point_without_force",
    os.path.join(T, "test_oracle_flows.py") + "::test_rotation_symmetry",
    os.path.join(T, "test_oracle_flows.py") + "::test_density_wave_moves_with_the_flow",
    os.path.join(T, "test_oracle_flows.py") + "::test_poiseuille_matches_closed_form",
    os.path.join(T, "test_oracle_flows.py") + "::test_kolmogorov_matches_discrete_closed_form",
    os.path.join(T, "test_oracle_flows.py") + "::test_solid_layers_equal_wall_faces",
]

C_SRC = "lbm_oracle.c"
PY_SRC = "__init__.py"
LAT_SRC = "lattice.py"

# name -> (file in oracle/, text, replacement); each text occurs exactly once.
MUTATIONS = {
    # macroscopic quantities (Sec. II.B)
    "velocity without the half-force shift":
        (C_SRC, "M->u[a] = M->j[a] / M->rho + (real)0.5 * g[a];",
         "M->u[a] = M->j[a] / M->rho;"),
    "momentum sum without the velocity's sign":
        (C_SRC, "if (ea != 0) ja = ja + (real)ea * f[i];", "if (ea != 0) ja = ja + f[i];"),
    "force density from the deviation mass":
        (C_SRC, "M->F[a] = M->rho * g[a];", "M->F[a] = M->drho * g[a];"),
    # BGK (eq:explict_eq, the force term below eq:Fr)
    "BGK equilibrium: sign of the u.u term":
        (C_SRC, "- (real)(0.5 * L->ics2) * usq;", "+ (real)(0.5 * L->ics2) * usq;"),
    "BGK force: (e.F)(e.u) over c_s^2 instead of c_s^4":
        (C_SRC, "(real)(L->ics2 * L->ics2) * (eF * eu)", "(real)L->ics2 * (eF * eu)"),
    "BGK force: (e - u).F replaced by e.F":
        (C_SRC, "(real)L->ics2 * (eF - uF)", "(real)L->ics2 * eF"),
    "BGK force term without 1 - omega/2":
        (C_SRC, "c[i] = P->hforce * Fi - P->omega * (f[i] - feq);",
         "c[i] = Fi - P->omega * (f[i] - feq);"),
    "BGK conserved-moment fix-up ignores the long links":
        (C_SRC, "if (ea > 1 || ea < -1) s = s + (real)ea * c[i];", ""),
    "BGK fix-up with the wrong sign":
        (C_SRC, "out[i] = f[i] + (c[i] + corr);", "out[i] = f[i] + (c[i] - corr);"),
    # SMRT (eq:domg, eq:RHS, eq:bbd1)
    "SMRT equilibrium moments from the deviation mass":
        (C_SRC, "E[k] = M.rho * U[k];", "E[k] = M.drho * U[k];"),
    "SMRT first-order non-equilibrium moment +F/2":
        (C_SRC, "N[k] = (real)-0.5 * M.F[a];", "N[k] = (real)0.5 * M.F[a];"),
    "SMRT relaxed first-order moment F/4":
        (C_SRC, "Pc[k] = (real)0.5 * M.F[a];", "Pc[k] = (real)0.25 * M.F[a];"),
    "SMRT shift to the moving frame without (-1)^|l|":
        (C_SRC, "S->cdown[k][t] = (mabs(l) % 2) ? -c : c;", "S->cdown[k][t] = c;"),
    "SMRT back-shift without the binomial":
        (C_SRC, "S->cup[k][t] = c;", "S->cup[k][t] = 1;"),
    "SMRT order 3 relaxed at the order-2 rate":
        (C_SRC, "Pc[k] = (n == 2 ? P->q2 : P->q3) * D;", "Pc[k] = P->q2 * D;"),
    "SMRT back-shift of the unrelaxed moments":
        (C_SRC, "R = fmar((real)S->cup[k][t] * U[S->kl[k][t]], Pc[km], R);",
         "R = fmar((real)S->cup[k][t] * U[S->kl[k][t]], N[km], R);"),
    "SMRT third-order force content without m_a":
        (C_SRC, "s = s + ((real)m[a] * g[a]) * ((real)0.5 * (D2[j] + Pc[j]));",
         "s = s + g[a] * ((real)0.5 * (D2[j] + Pc[j]));"),
    "third-order force content from the pre-collision second moment":
        (C_SRC, "((real)0.5 * (D2[j] + Pc[j]))", "D2[j]"),
    "third-order force content blind to the bulk rate":
        (C_SRC, "((real)0.5 * (D2[j] + Pc[j]))", "((real)0.5 * (D2[j] + P->q2 * D2[j]))"),
    "fourth-order force content without 1 - omega_4/2":
        (C_SRC, "Pc[k] = (real)0.5 * s;", "Pc[k] = s;"),
    "fourth-order force content from the pre-collision third moment":
        (C_SRC, "((real)0.5 * (D3[j] + Pc[j]))", "D3[j]"),
    "fourth-order force content left out of the back-shift":
        (C_SRC, "real R = (n <= 3 || (n == 4 && P->fo4)) ? Pc[k] : (real)-0.0;",
         "real R = (n <= 3) ? Pc[k] : (real)-0.0;"),
    "SMRT bulk rate over every second-order moment":
        (C_SRC, "if (mabs(m) == 2 && (m[0] == 2 || m[1] == 2 || m[2] == 2)) tr = tr + D2[k];",
         "if (mabs(m) == 2) tr = tr + D2[k];"),
    "SMRT third-order trace rate on the pair difference":
        (C_SRC, "const real s = D3[jb] + D3[jc];", "const real s = D3[jb] - D3[jc];"),
    "SMRT full reconstruction drops the mass":
        (C_SRC, "/* mass is unchanged */\n      dA[k] = full ? M.drho : 0;",
         "/* mass is unchanged */\n      dA[k] = 0;"),
    # the two operation orders of the transforms
    "twin projection: odd orders from the pair sums":
        (C_SRC, "if (h != 0) A = fmar(h, odd ? a[p] : s[p], A);",
         "if (h != 0) A = fmar(h, odd ? s[p] : a[p], A);"),
    "twin reconstruction: second member takes E + O":
        (C_SRC, "out[i + 1] = f[i + 1] + (ev - od);", "out[i + 1] = f[i + 1] + (ev + od);"),
    "plain projection skips the rest population":
        (C_SRC, "for (int i = 0; i < Q; ++i) P = P + L->H[k * Q + i] * f[i];",
         "for (int i = 1; i < Q; ++i) P = P + L->H[k * Q + i] * f[i];"),
    "plain reconstruction with the transposed inverse":
        (C_SRC, "for (int k = 0; k < NM; ++k) r = r + L->Minv[i * NM + k] * dA[k];",
         "for (int k = 0; k < NM; ++k) r = r + L->Minv[k * NM + i] * dA[k];"),
    # raw-moment MRT (appendix)
    "RMRT raw force moment without m_a":
        (C_SRC, "aF = aF + ((real)m[a] * U[j]) * M.F[a];", "aF = aF + U[j] * M.F[a];"),
    "RMRT order 3 force with the order-2 factor":
        (C_SRC, "t = t + P->h3 * aF;", "t = t + P->h2 * aF;"),
    "RMRT order 4 keeps the whole force moment":
        (C_SRC, "t = (real)0.5 * aF;", "t = aF;"),
    # initial state (eq:newf with Omega = 0)
    "BGK initial state with +F/2":
        (C_SRC, "out[i] = feq - (real)0.5 * Fi;", "out[i] = feq + (real)0.5 * Fi;"),
    "MRT initial state with +a_F/2":
        (C_SRC, "a[k] = rho * upow(m, u) - (real)0.5 * aF;",
         "a[k] = rho * upow(m, u) + (real)0.5 * aF;"),
    # streaming and walls (eq:evolution)
    "streaming against the velocity":
        (C_SRC, "d[a] = c[a] + L->e[3 * i + a];", "d[a] = c[a] - L->e[3 * i + a];"),
    "bounce-back without reversing the direction":
        (C_SRC, "fnew[(int64_t)L->opp[i] * N + n] = v;", "fnew[(int64_t)i * N + n] = v;"),
    # host-side rates and factors
    "third-order force factor at the order-2 rate":
        (PY_SRC, "fq3 = (1.0 - 0.5 / tau3) if force_order >= 3 else 0.0",
         "fq3 = (1.0 - 0.5 / tau2) if force_order >= 3 else 0.0"),
    "third-order force factor 1 - omega_3":
        (PY_SRC, "fq3 = (1.0 - 0.5 / tau3) if force_order >= 3 else 0.0",
         "fq3 = (1.0 - 1.0 / tau3) if force_order >= 3 else 0.0"),
    "bulk rate not divided by D":
        (PY_SRC, "dqb = (((1.0 - 1.0 / tau_bulk) - (1.0 - 1.0 / tau2)) / dim",
         "dqb = (((1.0 - 1.0 / tau_bulk) - (1.0 - 1.0 / tau2))"),
    "third-order trace rate not halved":
        (PY_SRC, "- (1.0 - 1.0 / tau3)) / 2 if tau_31", "- (1.0 - 1.0 / tau3)) if tau_31"),
    "BGK force factor 1 - omega":
        (PY_SRC, "hforce=1.0 - 0.5 * omega", "hforce=1.0 - omega"),
    "RMRT order-3 force factor at the order-2 rate":
        (PY_SRC, "h3=1.0 - 0.5 / tau3", "h3=1.0 - 0.5 / tau2"),
    # lattice tables
    "Hermite h3 = e^3 - c_s^2 e":
        (LAT_SRC, "return Fraction(e ** 3) - 3 * c2 * e", "return Fraction(e ** 3) - c2 * e"),
    "Hermite h4 constant c_s^4":
        (LAT_SRC, "+ 3 * c2 * c2", "+ c2 * c2"),
    "Hermite-sum reconstruction without m!":
        (LAT_SRC, "/ (mfact(m) * c2 ** sum(m))", "/ (c2 ** sum(m))"),
    "D3Q39 with c_s^2 = 1/3":
        (LAT_SRC, 'return Fraction(2, 3) if lat == "D3Q39" else CS2', "return CS2"),
}


def _child_env(copy_root: str) -> dict:
    env = dict(os.environ)
    env["PYTHONPATH"] = os.pathsep.join([copy_root, ROOT])
    env["OMP_NUM_THREADS"] = "1"
    env.pop("PYTEST_ADDOPTS", None)
    return env


def _make_copy(mutation) -> str:
    """A copy of oracle/ in a fresh directory with the mutation planted and built."""
    root = tempfile.mkdtemp(prefix="oracle_mut_")
    dst = os.path.join(root, "oracle")
    shutil.copytree(ORACLE, dst, ignore=shutil.ignore_patterns("__pycache__", "*.tmp"))
    rebuild = True
    if mutation is not None:
        fname, old, new = mutation
        path = os.path.join(dst, fname)
        with open(path) as fh:
            text = fh.read()
        if text.count(old) != 1:
            raise AssertionError(f"mutation anchor occurs {text.count(old)} times in {fname}")
        with open(path, "w") as fh:
            fh.write(text.replace(old, new))
        rebuild = fname == C_SRC
    if rebuild:
        for f in os.listdir(dst):
            if f.endswith(".so"):
                os.remove(os.path.join(dst, f))
        subprocess.run([sys.executable, "-c", "from oracle import build; build.build(force=True)"],
                       cwd=root, env=_child_env(root), check=True, capture_output=True)
    return root


def _run_pins(root: str, pins) -> tuple[int, str, str]:
    env = _child_env(root)
    where = subprocess.run([sys.executable, "-c", "import oracle; print(oracle.__file__)"],
                           cwd=root, env=env, capture_output=True, text=True, check=True)
    r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider",
                        "-p", "no:randomly", *pins],
                       cwd=root, env=env, capture_output=True, text=True)
    return r.returncode, where.stdout.strip(), r.stdout + r.stderr


def _case(name):
    root = _make_copy(None if name is None else MUTATIONS[name])
    try:
        return _run_pins(root, PINS if name is not None else PINS[:1])
    finally:
        shutil.rmtree(root, ignore_errors=True)


class _Outcomes(dict):
    """Outcome of each case, run on first use when not computed up front."""

    def __missing__(self, name):
        self[name] = out = _case(name)
        return out


@pytest.fixture(scope="module")
def outcomes():
    from oracle import build
    build.build(force=False)  # the copies start from built, current libraries
    out = _Outcomes()
    # Serially, every case runs up front on a thread pool.  Under pytest-xdist each worker
    # would repeat that for itself, so there each test runs its own case only.
    if not os.environ.get("PYTEST_XDIST_WORKER"):
        names = [None, *MUTATIONS]
        workers = max(1, min(8, os.cpu_count() or 1))
        with cf.ThreadPoolExecutor(workers) as ex:
            out.update(zip(names, ex.map(_case, names)))
    return out


def test_harness_imports_the_copy_and_passes_unplanted(outcomes):
    rc, where, out = outcomes[None]
    assert "oracle_mut_" in where, where
    assert rc == 0, out[-2000:]


@pytest.mark.parametrize("name", list(MUTATIONS))
def test_planted_mistake_fails_a_pin(outcomes, name):
    rc, where, out = outcomes[name]
    assert "oracle_mut_" in where, where
    summary = out.strip().splitlines()[-1] if out.strip() else ""
    assert rc == 1 and re.search(r"\b1 failed\b", summary) and "error" not in summary, \
        f"{name}: not caught (rc={rc}): {summary}\n{out[-3000:]}"
