"""Learned warm start for steady forced flows (orchestration; all compute is in liblbm).

Problem family: a periodic box^3 D3Q27 SMRT lattice driven by four seeded Fourier modes
(inputs.warmstart_problem).  The start is the second-order perturbative steady solution
of the modes (an analytic base, lbm_ws_features) with each mode's own response
corrected by a network (lbm.MLP, BF16 matrix-core kernels) that maps the mode's
wavevector, polarisation and tau2 to 8 amplitude coefficients.  The lattice is
restarted from that field on the full lattice (lbm_reset_fields: low-pass filtered,
projected onto the plain start's mass and momentum, with the non-equilibrium stress the
velocity gradient implies).  Training targets are projections of lattice-Boltzmann
solutions computed by the batched engine from the plain start; the parameters are
selected by the steps to steady state they give on validation problems.  The converged
lattice-Boltzmann solution decides the prediction's error; the plain start (rest, rho0)
remains the fallback.

With waves=True the start is instead the lattice's own steady state expanded to order
1-3 in the forcing amplitude (lbm_ws_lattice_waves), set directly as populations
(lbm_set_waves), with the network's per-mode output added as equilibrium waves.

torch supplies device buffers and the stream only.

CLI:  python -m paper_2212_07494_amd.warmstart --box 128 --train 80 --val 12 --test 16 --out <dir>
"""
from __future__ import annotations

import argparse
import json
import math
import os
import time

import numpy as np

from . import inputs
from . import lbm as L

WIDTHS = [L.WS_MODE_FEATURES, 576, 576, 576, 576, 8]  # 1.00M parameters
TAU3 = 1.0
BASE_ORDER = 2
NMODES = 4
# Waves start, order "auto": the fourth order is added when a3^2 / (a2 a1) exceeds this,
# a_n the norm of the order-n wave amplitudes (the expansion's ratio applied once more,
# relative to the first order).  Measured at 128^3: below about 1e-6 the third-order start
# is steady within 20-60 steps; above about 3e-6 it needs hundreds to thousands, which the
# fourth order (about 26 ms more on the host) cuts to 20-560.
AUTO_ORDER4 = 3e-6


def series_ratio(nmodes, amp):
    """a3^2 / (a2 a1) for third-order waves (lbm_ws_lattice_waves order 3 with nmodes
    modes: nmodes first-order waves, then nmodes (nmodes + 1) second-order ones, then the
    third order), a_n the root-sum-square of the order-n amplitudes."""
    n = nmodes
    n2 = n + n * (n + 1)
    a1, a2, a3 = (float(np.sqrt((np.abs(amp[lo:hi]) ** 2).sum()))
                  for lo, hi in ((0, n), (n, n2), (n2, len(amp))))
    return a3 * a3 / (a2 * a1) if a2 > 0 and a1 > 0 else 0.0


def domain_of(problem, box):
    shape = (box, box, box)
    g = inputs.fourier_force(shape, problem["modes"])
    return dict(shape=shape, walls=(0, 0, 0), tau=(problem["tau2"], TAU3, 1.0), g_field=g)


def mode_phases(problem, box):
    """theta_j(x) = 2 pi k_j . x / box + phase_j on the box^3 lattice, x fastest (nmodes x N)."""
    N = box ** 3
    n = np.arange(N)
    pos = np.stack([n % box, (n // box) % box, n // (box * box)]).astype(np.float64)
    return np.stack([2 * math.pi * (np.asarray(m["k"], np.float64) @ pos) / box + m["phase"]
                     for m in problem["modes"]])


def separable(problem):
    """Whether each mode's own wave can be told apart: no two wavevectors equal or
    opposite (their sine and cosine projections would mix)."""
    ks = [np.asarray(m["k"]) for m in problem["modes"]]
    for i in range(len(ks)):
        for j in range(i):
            if np.array_equal(ks[i], ks[j]) or np.array_equal(ks[i], -ks[j]):
                return False
    return True


def solve_batch(problems, box, tol, max_steps, storage="f64", check_every=200, stall=40,
                stream=None, fields=True):
    """Solve every problem from the plain start with the batched engine; returns
    steps, resid, status and (if fields) the converged (rho, u) per problem."""
    doms = [domain_of(p, box) for p in problems]
    with L.Batch(doms, "D3Q27", "smrt", storage, stream=stream) as b:
        steps, resid, status = b.run(max_steps, tol, check_every=check_every,
                                     stall_checks=stall)
        out = [b.moments(d) for d in range(len(doms))] if fields else None
    return steps, resid, status, out


class WarmStart:
    """The per-mode network plus the buffers to train and apply it.

    The start is the second-order perturbative steady solution of the forcing modes
    (lbm_ws_features) in which each mode's own response is corrected by the network:
    from the mode's phase advance per lattice link, polarisation and tau2
    (lbm_ws_mode_features) it predicts 8 coefficients -- the velocity amplitude's
    deviation from s_j p_j on sin(theta_j) (3) and on cos(theta_j) (3) and the density
    amplitudes (2), in units of s_j.  At small Reynolds numbers the steady state's error
    against the analytic base is mostly this per-mode lattice response, and a correction
    confined to the modes' own waves adds nothing to slowly decaying waves the solution
    does not have.  The output layer starts at zero (the untrained start is the base);
    per-channel output scales are the RMS targets.  The lattice is restarted with the
    low-pass filter, the plain start's mass and momentum and the non-equilibrium stress
    of the field (lbm_reset_fields)."""

    FLAGS = L.RESET_FILTER | L.RESET_MASS | L.RESET_MOMENTUM | L.RESET_NONEQ

    def __init__(self, box=128, widths=WIDTHS, seed=0, max_rows=4096, stream=None,
                 base_order=BASE_ORDER, flags=None, linear=False, waves=False,
                 waves_order="auto"):
        import torch
        self.torch = torch
        self.box = box
        # linear: add each mode's exact linear lattice response (lbm_ws_lattice_response)
        # to the correction; the network then predicts only what that misses
        self.linear = linear
        # waves: start from the lattice's own steady state to second order in the forcing
        # (lbm_ws_lattice_waves, set as populations by lbm_set_waves) instead of the
        # analytic base; the network's coefficients then correct each mode's own wave
        # relative to that start (correction_waves)
        self.waves = waves
        self.waves_order = waves_order
        self.velset = L.lbm_lattice_info("D3Q27") if waves else None
        self.widths = list(widths)
        self.stream = stream
        self.base_order = base_order
        self.flags = self.FLAGS if flags is None else flags
        self.scale = np.ones(self.widths[-1], np.float32)
        self.max_rows = max_rows
        self.net = L.MLP(self.widths, max_rows=max_rows, stream=stream)
        self.reset_params(seed)
        self.y = torch.empty((max_rows, self.widths[-1]), device="cuda")
        self.best_iter = None
        self.val_curve = []

    def reset_params(self, seed):
        p = inputs.mlp_init_params(self.widths, seed)
        nlast = self.widths[-1] * (self.widths[-2] + 1)
        p[-nlast:] = 0.0
        self.net.set_params(p.astype(np.float32))
        self.step = 0

    def set_scale(self, scale):
        """Output scales; channels far below the largest (round-off, e.g. amplitudes
        that vanish by symmetry) are floored at 1e-3 of it so their noise is not fitted."""
        scale = np.asarray(scale, np.float64)
        self.scale = np.maximum(scale, 1e-3 * max(float(scale.max()), 1e-30)).astype(np.float32)
        self.net.set_output_scale(self.scale)

    # -- data -------------------------------------------------------------------------
    def mode_features(self, problem, out=None):
        torch = self.torch
        out = out if out is not None else torch.empty((NMODES, self.widths[0]), device="cuda")
        L.lbm_ws_mode_features(problem, self.box, out, stream=self.stream)
        return out

    def lattice_response(self, problem):
        """Each mode's exact linear lattice response (nmodes x 8) as mode coefficients."""
        return L.lbm_ws_lattice_response(problem, self.box, tau3=TAU3)

    def lattice_waves(self, problem):
        """The problem's steady lattice state to order waves_order in the forcing (1 to 4;
        "auto": 3, or 4 where the series converges slowly, AUTO_ORDER4), as population
        waves (k, phase, complex amplitudes)."""
        if self.waves_order != "auto":
            return L.lbm_ws_lattice_waves(problem, self.box, order=int(self.waves_order),
                                          tau3=TAU3)
        k, ph, A = L.lbm_ws_lattice_waves(problem, self.box, order=3, tau3=TAU3)
        if series_ratio(len(problem["modes"]), A) > AUTO_ORDER4:
            return L.lbm_ws_lattice_waves(problem, self.box, order=4, tau3=TAU3)
        return k, ph, A

    def correction_waves(self, problem, coef):
        """Each mode's correction (coef: nmodes x 8, the network's output in units of
        s_j = amp_j / (nu K_j^2): velocity on sin(theta_j) (3) and cos(theta_j) (3),
        density on sin and cos) as the equilibrium wave it implies about rest (rho0 = 1):
        A_i = w_i (rho_hat + 3 e_i . u_hat), u_hat = s_j (c_3..5 - i c_0..2),
        rho_hat = s_j (c_7 - i c_6), since Re[(a - i b) e^{i theta}] = a cos + b sin."""
        e, w = self.velset
        nu = (problem["tau2"] - 0.5) / 3.0
        ks, phs, amps = [], [], []
        for j, m in enumerate(problem["modes"]):
            K = 2 * math.pi * np.linalg.norm(m["k"]) / self.box
            s = m["amp"] / (nu * K * K)
            uh = s * (coef[j, 3:6] - 1j * coef[j, 0:3])
            rh = s * (coef[j, 7] - 1j * coef[j, 6])
            ks.append(np.asarray(m["k"], np.int32))
            phs.append(m["phase"])
            amps.append(w * (rh + 3.0 * (e.astype(np.float64) @ uh)))
        return np.array(ks), np.array(phs), np.array(amps)

    def waves_targets(self, problem, rho, u):
        """The coefficients that correct the waves start towards a converged lattice state
        (rho, u): projections on sin(theta_j), cos(theta_j) of the state minus those of the
        start's own fields, in units of s_j."""
        dom = domain_of(problem, self.box)
        with L.Lattice("D3Q27", "smrt", "f64", dom["shape"], dom["walls"], dom["tau"],
                       g_field=dom["g_field"], stream=self.stream) as lat:
            lat.set_waves(*self.lattice_waves(problem))
            rho_s, u_s = lat.moments()
        N = self.box ** 3
        r = np.concatenate([u - u_s, (rho - rho_s)[None]])
        th = mode_phases(problem, self.box)
        nu = (problem["tau2"] - 0.5) / 3.0
        out = np.empty((NMODES, 8))
        for j, m in enumerate(problem["modes"]):
            K = 2 * math.pi * np.linalg.norm(m["k"]) / self.box
            a = m["amp"] / (nu * K * K)
            ps = 2.0 / N * (r @ np.sin(th[j]))
            pc = 2.0 / N * (r @ np.cos(th[j]))
            out[j, 0:3] = ps[:3] / a
            out[j, 3:6] = pc[:3] / a
            out[j, 6] = ps[3] / a
            out[j, 7] = pc[3] / a
        return out.astype(np.float32)

    def mode_targets(self, problem, rho, u):
        """The 8 coefficients per mode that make the base's own mode responses match a
        converged lattice state (rho, u on the box^3 lattice): projections on
        sin(theta_j), cos(theta_j) of the state minus the base's pair terms (in waves
        mode: minus the waves start's fields, waves_targets)."""
        if self.waves:
            return self.waves_targets(problem, rho, u)
        torch = self.torch
        N = self.box ** 3
        b1 = torch.empty((N, 4), device="cuda")
        b2 = torch.empty((N, 4), device="cuda")
        U = L.lbm_ws_features(problem, self.box, self.box, None, b1, 1, stream=self.stream)
        L.lbm_ws_features(problem, self.box, self.box, None, b2, 2, stream=self.stream)
        pair = (b2 - b1).double().cpu().numpy().T        # (4, N), units of U
        r = np.concatenate([u / U, (rho[None] - 1.0) / U]) - pair
        th = mode_phases(problem, self.box)
        sn, cs = np.sin(th), np.cos(th)
        nu = (problem["tau2"] - 0.5) / 3.0
        out = np.empty((NMODES, 8))
        for j, m in enumerate(problem["modes"]):
            K = 2 * math.pi * np.linalg.norm(m["k"]) / self.box
            a = m["amp"] / (nu * K * K) / U
            ps = 2.0 / N * (r @ sn[j])
            pc = 2.0 / N * (r @ cs[j])
            out[j, 0:3] = ps[:3] / a - np.asarray(m["p"])
            out[j, 3:6] = pc[:3] / a
            out[j, 6] = ps[3] / a
            out[j, 7] = pc[3] / a
        if self.linear:
            out -= self.lattice_response(problem)
        return out.astype(np.float32)

    def dataset(self, problems, fields, fit_scale=False):
        """Device tensors X (4n x 8 features), T (4n x 8 targets) from solved problems
        (those with separable modes); fit_scale sets the output scales from them."""
        torch = self.torch
        keep = [(p, f) for p, f in zip(problems, fields) if separable(p)]
        X = torch.empty((NMODES * len(keep), self.widths[0]), device="cuda")
        T = np.empty((NMODES * len(keep), self.widths[-1]), np.float32)
        for i, (p, (rho, u)) in enumerate(keep):
            self.mode_features(p, out=X[NMODES * i: NMODES * (i + 1)])
            T[NMODES * i: NMODES * (i + 1)] = self.mode_targets(p, rho, u)
        if fit_scale:
            self.set_scale(np.sqrt(np.mean(T.astype(np.float64) ** 2, axis=0)))
        return X, torch.from_numpy(T).cuda()

    # -- training ---------------------------------------------------------------------
    def train(self, X, T, iters=6000, batch=256, lr=1e-3, lr_min=1e-5, seed=1, log_every=0,
              val=None, eval_every=1000):
        """Adam with a cosine learning rate over random batches of modes, loss the mean
        square error in units of the output scales.  val, a callable returning a score
        (lower is better, e.g. validation_steps), selects the parameters: evaluated at the
        start and every eval_every iterations, the best are kept, so the result is never
        worse on it than the base (the zero correction training starts from).  The curve
        is left in self.val_curve as (iteration, score), the kept iteration in best_iter."""
        torch = self.torch
        n = X.shape[0]
        rng = np.random.default_rng(seed)
        batch = min(batch, n, self.max_rows)
        xb = torch.empty((batch, self.widths[0]), device="cuda")
        tb = torch.empty((batch, self.widths[-1]), device="cuda")
        w = (1.0 / self.scale.astype(np.float64) ** 2).astype(np.float32)
        self.val_curve = []
        self.best_iter = None
        best = None

        def check(it):
            nonlocal best
            if val is None:
                return
            score = float(val())
            self.val_curve.append((it, score))
            if best is None or score < best[0]:
                best = (score, self.net.params(), it)

        losses = []
        check(0)
        for it in range(iters):
            idx = torch.as_tensor(rng.choice(n, batch, replace=False))
            xb.copy_(X[idx])
            tb.copy_(T[idx])
            self.net.forward(xb, self.y[:batch])
            self.net.zero_grads()
            loss = self.net.loss_backward(tb, w)
            self.step += 1
            rate = lr_min + 0.5 * (lr - lr_min) * (1 + math.cos(math.pi * it / max(1, iters)))
            self.net.adam(rate, self.step)
            losses.append(loss)
            if log_every and it % log_every == 0:
                print(f"  iter {it} loss {loss:.3e}", flush=True)
            if (it + 1) % eval_every == 0 or it + 1 == iters:
                check(it + 1)
        if best is not None:
            self.net.set_params(best[1])
            self.best_iter = best[2]
        return losses

    def evaluate(self, X, T):
        """RMS error of the predicted coefficients in units of the output scales, and of
        the base (zero correction), over a set of modes."""
        self.net.forward(X, self.y[: X.shape[0]])
        y = self.y[: X.shape[0]].cpu().numpy().astype(np.float64)
        t = T.cpu().numpy().astype(np.float64)
        sc = self.scale.astype(np.float64)
        return (float(np.sqrt(np.mean(((y - t) / sc) ** 2))),
                float(np.sqrt(np.mean((t / sc) ** 2))))

    # -- inference ----------------------------------------------------------------------
    def predict(self, problem):
        """Start fields (box^3 x 4 rows, device: u / U, (rho - 1) / U) and U."""
        torch = self.torch
        x = self.mode_features(problem)
        coef = self.y[:NMODES]
        self.net.forward(x, coef)
        if self.linear:
            c = coef.cpu().numpy().astype(np.float64) + self.lattice_response(problem)
            coef = torch.from_numpy(c.astype(np.float32)).cuda()
        rows = torch.empty((self.box ** 3, 4), device="cuda")
        U = L.lbm_ws_features(problem, self.box, self.box, None, rows, self.base_order, 1.0,
                              mode_coef=coef, stream=self.stream)
        return rows, U

    def predict_waves(self, problem):
        """Waves mode: the second-order lattice waves plus the network's correction waves."""
        x = self.mode_features(problem)
        coef = self.y[:NMODES]
        self.net.forward(x, coef)
        c = coef.cpu().numpy().astype(np.float64)
        k, ph, A = self.lattice_waves(problem)
        kc, phc, Ac = self.correction_waves(problem, c)
        return (np.concatenate([k, kc]), np.concatenate([ph, phc]),
                np.concatenate([A, Ac]))

    def start(self, lattice, problem):
        """Restart `lattice` (a box^3 lbm.Lattice of this problem) from the prediction."""
        if self.waves:
            lattice.set_waves(*self.predict_waves(problem))
            return None
        rows, U = self.predict(problem)
        L.lbm_reset_fields(lattice.ctx, rows, 1, U, U, self.flags)
        return U

    def save(self, path):
        """Parameters (path + '.npy') and the settings (path + '.json')."""
        np.save(path + ".npy", self.net.params())
        with open(path + ".json", "w") as fh:
            json.dump(dict(widths=self.widths, box=self.box, base_order=self.base_order,
                           flags=self.flags, linear=self.linear, waves=self.waves,
                           waves_order=self.waves_order,
                           scale=self.scale.tolist()), fh)

    def load(self, path):
        with open(path + ".json") as fh:
            meta = json.load(fh)
        if meta["widths"] != self.widths:
            raise ValueError(f"saved widths {meta['widths']} differ from {self.widths}")
        self.base_order = meta["base_order"]
        self.flags = meta["flags"]
        self.linear = bool(meta.get("linear", False))
        self.waves = bool(meta.get("waves", False))
        self.waves_order = meta.get("waves_order", "auto")
        self.velset = L.lbm_lattice_info("D3Q27") if self.waves else None
        self.set_scale(meta["scale"])
        self.net.set_params(np.load(path + ".npy", allow_pickle=False))

    def close(self):
        self.net.close()


def run_to_steady(lattice, tol, check_every=200, max_steps=2_000_000):
    """Step until the per-step residual of the velocity drops below tol; returns
    (steps, resid)."""
    steps = 0
    resid = float("inf")
    while steps < max_steps:
        lattice.step(check_every - 1)
        lattice.monitors()              # records u(t)
        lattice.step(1)
        m = lattice.monitors()          # compares u(t + 1) with u(t)
        steps += check_every
        resid = m.resid
        if m.nonfinite:
            raise L.LBMError(L.LBM_ENONFINITE, "non-finite state")
        if resid < tol:
            break
    return steps, resid


def validation_steps(ws, problems, box, tol=1e-8, check_every=50, max_steps=2_000_000):
    """Total steps to resid < tol from ws's start over a set of problems (the score the
    training selects on: a smaller velocity error can still cost steps when the error
    sits in slowly decaying modes)."""
    total = 0
    for p in problems:
        dom = domain_of(p, box)
        with L.Lattice("D3Q27", "smrt", "f64", dom["shape"], dom["walls"], dom["tau"],
                       g_field=dom["g_field"], stream=ws.stream) as lat:
            ws.start(lat, p)
            total += run_to_steady(lat, tol, check_every, max_steps)[0]
    return total


def compare_starts(ws, problem, box, tol, storage="f64", check_every=200, max_steps=2_000_000,
                   reference=None, stream=None, plain=None, reference_u=None):
    """Steps and wall time to resid < tol from the plain start and from ws's start
    (inference, field evaluation and restart included in the warm time, and timed on
    their own as inference_s).  The plain run's final velocity is the reference for the true
    errors (initial_err, final_err) unless `reference` is given.  A plain record and its
    final velocity from an earlier call (plain, reference_u) skip the plain run."""
    torch = ws.torch
    dom = domain_of(problem, box)
    out = {}
    modes = ("warm",) if plain is not None else ("plain", "warm")
    if plain is not None:
        out["plain"] = plain
        reference = reference_u if reference is None else reference
    for mode in modes:
        with L.Lattice("D3Q27", "smrt", storage, dom["shape"], dom["walls"], dom["tau"],
                       g_field=dom["g_field"], stream=stream) as lat:
            torch.cuda.synchronize()
            t_inf = 0.0
            e0 = None
            if mode == "warm":
                t0 = time.perf_counter()
                ws.start(lat, problem)
                torch.cuda.synchronize()
                t_inf = time.perf_counter() - t0
                if reference is not None:  # outside the timed region
                    _, u0 = lat.moments()
                    e0 = float(np.linalg.norm(u0 - reference) / np.linalg.norm(reference))
            t0 = time.perf_counter()
            steps, resid = run_to_steady(lat, tol, check_every, max_steps)
            torch.cuda.synchronize()
            wall = t_inf + time.perf_counter() - t0
            _, u = lat.moments()
        rec = dict(steps=int(steps), resid=float(resid), wall_s=wall, inference_s=t_inf)
        if reference is not None:
            rec["final_err"] = float(np.linalg.norm(u - reference) / np.linalg.norm(reference))
        if e0 is not None:
            rec["initial_err"] = e0
        if mode == "plain":
            reference = u if reference is None else reference
            out["reference_u"] = u
        out[mode] = rec
    return out


def main():
    ap = argparse.ArgumentParser(description="train and evaluate the learned warm start")
    ap.add_argument("--box", type=int, default=128)
    ap.add_argument("--train", type=int, default=80)
    ap.add_argument("--val", type=int, default=12)
    ap.add_argument("--test", type=int, default=16)
    ap.add_argument("--iters", type=int, default=6000)
    ap.add_argument("--tol", type=float, default=1e-8)
    ap.add_argument("--data-tol", type=float, default=1e-10)
    ap.add_argument("--chunk", type=int, default=32, help="domains per batched data solve")
    ap.add_argument("--seed", type=int, default=2022)
    ap.add_argument("--out", default="warmstart_out")
    args = ap.parse_args()
    import torch
    os.makedirs(args.out, exist_ok=True)
    L.load()
    n_fit = args.train + args.val
    probs = [inputs.warmstart_problem(args.seed + i, box=args.box)
             for i in range(n_fit + args.test)]
    train_p, val_p, test_p = probs[:args.train], probs[args.train:n_fit], probs[n_fit:]
    ws = WarmStart(box=args.box, seed=args.seed)
    Xs, Ts = [], []
    t0 = time.time()
    data_steps = []
    for c0 in range(0, args.train, args.chunk):
        ps = train_p[c0:c0 + args.chunk]
        steps, _, status, fields = solve_batch(ps, args.box, args.data_tol, 3_000_000)
        if np.any((status != L.DOM_CONVERGED) & (status != L.DOM_FLOOR)):
            raise RuntimeError(f"data solve did not converge: {status.tolist()}")
        X, T = ws.dataset(ps, fields)
        Xs.append(X)
        Ts.append(T)
        data_steps += steps.tolist()
        del fields
        print(f"data: {c0 + len(ps)}/{args.train} solved, {time.time() - t0:.1f} s", flush=True)
    X, T = torch.cat(Xs), torch.cat(Ts)
    ws.set_scale(torch.sqrt(torch.mean(T.double() ** 2, 0)).cpu().numpy())
    t0 = time.time()
    losses = ws.train(X, T, iters=args.iters, log_every=1000,
                      val=lambda: validation_steps(ws, val_p, args.box, args.tol, 100))
    torch.cuda.synchronize()
    t_train = time.time() - t0
    print(f"train: {args.iters} iters, {t_train:.1f} s, final loss {losses[-1]:.3e}, "
          f"kept iteration {ws.best_iter}, validation steps {ws.val_curve}", flush=True)
    ws.save(os.path.join(args.out, "warmstart"))
    base = WarmStart(box=args.box, seed=args.seed,
                     flags=L.RESET_FILTER | L.RESET_MASS | L.RESET_MOMENTUM)
    results = []
    for i, p in enumerate(test_p):
        r = compare_starts(ws, p, args.box, args.tol, check_every=100)
        rb = compare_starts(base, p, args.box, args.tol, check_every=100, plain=r["plain"],
                            reference_u=r["reference_u"])
        r["base"] = rb["warm"]
        del r["reference_u"]
        r.update(tau2=p["tau2"], U=p["U"])
        results.append(r)
        print(f"test {i}: plain {r['plain']['steps']} steps {r['plain']['wall_s']:.2f} s | "
              f"base {r['base']['steps']} steps {r['base']['wall_s']:.2f} s | "
              f"learned {r['warm']['steps']} steps {r['warm']['wall_s']:.2f} s "
              f"(start {r['warm']['inference_s'] * 1e3:.1f} ms, error "
              f"{r['warm']['initial_err']:.1e} -> {r['warm']['final_err']:.1e})", flush=True)
    base.close()

    def med(key, field):
        return float(np.median([r[key][field] / r["plain"][field] for r in results]))

    summary = dict(box=args.box, train=args.train, val=args.val, test=args.test,
                   iters=args.iters, kept_iteration=ws.best_iter, val_curve=ws.val_curve,
                   train_seconds=t_train, final_loss=losses[-1], data_steps=data_steps,
                   scale=ws.scale.tolist(), results=results,
                   steps_ratio_median=med("warm", "steps"), wall_ratio_median=med("warm", "wall_s"),
                   base_steps_ratio_median=med("base", "steps"),
                   base_wall_ratio_median=med("base", "wall_s"))
    with open(os.path.join(args.out, "warmstart_summary.json"), "w") as fh:
        json.dump(summary, fh, indent=1)
    print(json.dumps({k: v for k, v in summary.items()
                      if k not in ("results", "data_steps", "val_curve")}))
    ws.close()


if __name__ == "__main__":
    main()
