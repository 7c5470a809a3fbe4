"""Learned warm start for steady forced flows (orchestration; all compute is in liblbm).

Problem family: a periodic box^3 D3Q27 SMRT lattice driven by four seeded Fourier modes
(inputs.warmstart_problem).  The start is the second-order perturbative steady solution
of the modes (an analytic base, lbm_ws_features) plus a learned correction: the network
(lbm.MLP, BF16 matrix-core kernels) maps per-point features of the problem to a vector
potential and a density residual on a coarse nc^3 grid, composed as (curl psi, r) so
that the velocity correction is divergence-free (lbm_ws_compose).  The correction is
interpolated to the lattice (lbm_upsample_periodic) and the lattice restarted from
base + correction (lbm_reset_fields, low-pass filtered and projected onto the plain
start's mass and momentum).  Training targets are lattice-Boltzmann solutions computed
by the batched engine from the plain start.  The converged lattice-Boltzmann solution
decides the prediction's error; the plain start (rest, rho0) remains the fallback.

torch supplies device buffers and the stream only.

CLI:  python -m paper_2212_07494_amd.warmstart --box 128 --train 80 --val 16 --test 16 --out <dir>
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

WIDTHS = [L.WS_FEATURES, 576, 576, 576, 576, 4]  # 1.02M parameters
TAU3 = 1.0
BASE_ORDER = 2


def domain_of(problem, box):
    shape = (box, box, box)
    g = inputs.fourier_force(shape, problem["modes"])
    return dict(shape=shape, walls=(0, 0, 0), tau=(problem["tau2"], TAU3, 1.0), g_field=g)


def coarse_targets(rho, u, box, nc, U, rho0=1.0):
    """Rows (nc^3 x 4) of (u / U, (rho - rho0) / U) sampled at lattice nodes
    (i, j, l) * box / nc, x fastest."""
    s = box // nc
    r = rho.reshape(box, box, box)[::s, ::s, ::s].ravel()
    uu = u.reshape(3, box, box, box)[:, ::s, ::s, ::s].reshape(3, -1)
    out = np.empty((nc ** 3, 4), np.float32)
    out[:, :3] = (uu / U).T
    out[:, 3] = (r - rho0) / U
    return out


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
    """The network plus the buffers to evaluate and train it.

    The start is base + (curl psi, r): base the second-order perturbative steady solution
    (lbm_ws_features), psi and r the network's outputs on the nc^3 grid, composed by
    lbm_ws_compose.  The velocity correction is a discrete curl, so it adds no
    compressive error (which would excite slowly damped sound); the output layer starts
    at zero, so the untrained start is the base.  Scales fitted on the training set: the
    density channel is carried in units of U * rho_scale and the potential in units of
    u_scale (the RMS residuals of the base), and the loss weighs the velocity channels
    by 1 / u_scale^2."""

    def __init__(self, nc=32, box=128, max_batch=4, widths=WIDTHS, seed=0, stream=None,
                 base_order=BASE_ORDER):
        import torch
        self.torch = torch
        self.nc, self.box = nc, box
        self.widths = list(widths)
        self.rows = nc ** 3
        self.stream = stream
        self.base_order = base_order
        self.rho_scale = 1.0
        self.u_scale = 1.0
        self.max_batch = max_batch
        self.net = L.MLP(self.widths, max_rows=self.rows * max_batch, stream=stream)
        self.reset_params(seed)
        shape = (self.rows * max_batch, self.widths[-1])
        self.y = torch.empty(shape, device="cuda")
        self.v = torch.empty(shape, device="cuda")

    def reset_params(self, seed):
        p = inputs.mlp_init_params(self.widths, seed)
        nlast = self.widths[-1] * (self.widths[-2] + 1)
        p[-nlast:] = 0.0
        self.net.set_params(p.astype(np.float32))
        self.step = 0

    def _set_scales(self, rho_scale, u_scale):
        self.rho_scale, self.u_scale = float(rho_scale), float(u_scale)
        self.net.set_output_scale([self.u_scale] * 3 + [1.0])

    def loss_weight(self):
        return np.array([1.0 / self.u_scale ** 2] * 3 + [1.0], np.float32)

    # -- data -------------------------------------------------------------------------
    def features(self, problem, x=None, base=None):
        """Features and base (device, rows x F and rows x 4) and the scale U."""
        torch = self.torch
        x = x if x is not None else torch.empty((self.rows, self.widths[0]), device="cuda")
        base = base if base is not None else torch.empty((self.rows, 4), device="cuda")
        U = L.lbm_ws_features(problem, self.nc, self.box, x, base, self.base_order,
                              self.rho_scale, stream=self.stream)
        return x, base, U

    def dataset(self, problems, fields, fit_scale=False):
        """Device tensors X (n x rows x F), B (n x rows x 4, base), T (n x rows x 4).
        fit_scale sets rho_scale and u_scale from these problems first."""
        torch = self.torch
        n = len(problems)
        if fit_scale:
            self._set_scales(1.0, 1.0)
        X = torch.empty((n, self.rows, self.widths[0]), device="cuda")
        B = torch.empty((n, self.rows, 4), device="cuda")
        T = torch.empty((n, self.rows, self.widths[-1]), device="cuda")
        for i, (p, (rho, u)) in enumerate(zip(problems, fields)):
            _, _, U = self.features(p, x=X[i], base=B[i])
            T[i] = torch.from_numpy(coarse_targets(rho, u, self.box, self.nc, U)).cuda()
        if fit_scale:
            r = (T[..., 3] - B[..., 3]).double()
            e = (T[..., :3] - B[..., :3]).double()
            self._set_scales(max(float(torch.sqrt(torch.mean(r * r))), 1e-12),
                             max(float(torch.sqrt(torch.mean(e * e))), 1e-12))
            B[..., 3] /= self.rho_scale
        T[..., 3] /= self.rho_scale
        return X, B, T

    # -- training ---------------------------------------------------------------------
    def train(self, X, B, T, iters=2000, batch=4, lr=1e-3, lr_min=1e-5, seed=1, log_every=0,
              val=None, eval_every=250):
        """Adam with a cosine learning rate over random batches of problems.  val, a
        callable returning a score (lower is better, e.g. validation_steps), selects
        the parameters: it is evaluated at the start and every eval_every iterations and
        the best parameters are kept, so the result is never worse on it than the base
        (the zero correction training starts from).  The curve is left in
        self.val_curve as (iteration, score) pairs, the kept iteration in best_iter."""
        torch = self.torch
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

        n = X.shape[0]
        rng = np.random.default_rng(seed)
        batch = min(batch, n, self.max_batch)
        rows = batch * self.rows
        xb = torch.empty((rows, self.widths[0]), device="cuda")
        bb = torch.empty((rows, 4), device="cuda")
        tb = torch.empty((rows, 4), device="cuda")
        dv = torch.empty((rows, 4), device="cuda")
        dy = torch.empty((rows, 4), device="cuda")
        w = self.loss_weight()
        losses = []
        check(0)
        for it in range(iters):
            idx = torch.as_tensor(rng.choice(n, batch, replace=False))
            xb.copy_(X[idx].reshape(rows, -1))
            bb.copy_(B[idx].reshape(rows, -1))
            tb.copy_(T[idx].reshape(rows, -1))
            self.net.forward(xb, self.y[:rows])
            L.lbm_ws_compose(self.y[:rows], bb, self.nc, batch, self.v[:rows], stream=self.stream)
            loss = self.net.loss_grad(self.v[:rows], tb, dv, w)
            L.lbm_ws_compose(dv, None, self.nc, batch, dy, stream=self.stream)
            self.net.zero_grads()
            self.net.backward(dy)
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

    def _compose(self, x, base, out):
        self.net.forward(x, self.y[: self.rows])
        L.lbm_ws_compose(self.y[: self.rows], base, self.nc, 1, out, stream=self.stream)

    def evaluate(self, X, B, T):
        """Relative L2 error of the velocity channels per problem, for the prediction and
        for the base alone."""
        errs, base_errs = [], []
        for i in range(X.shape[0]):
            self._compose(X[i], B[i], self.v[: self.rows])
            y = self.v[: self.rows].cpu().numpy()
            b = B[i].cpu().numpy()
            t = T[i].cpu().numpy()
            nt = np.linalg.norm(t[:, :3])
            errs.append(float(np.linalg.norm(y[:, :3] - t[:, :3]) / nt))
            base_errs.append(float(np.linalg.norm(b[:, :3] - t[:, :3]) / nt))
        return errs, base_errs

    # -- inference ----------------------------------------------------------------------
    def predict(self, problem):
        """The composed prediction rows (nc^3 x 4, device) and the problem's velocity scale."""
        x, base, U = self.features(problem)
        self._compose(x, base, self.v[: self.rows])
        return self.v[: self.rows], U

    def start(self, lattice, problem):
        """Restart `lattice` (a box^3 lbm.Lattice of this problem) from the prediction,
        low-pass filtered and projected onto the plain start's mass and momentum.  With
        nc < box only the network's correction is interpolated; the base is evaluated on
        the lattice itself."""
        torch = self.torch
        flags = L.RESET_FILTER | L.RESET_MASS | L.RESET_MOMENTUM
        if self.nc == self.box:
            v, U = self.predict(problem)
            L.lbm_reset_fields(lattice.ctx, v, 1, U, U * self.rho_scale, flags)
            return U
        x, _, U = self.features(problem)
        self.net.forward(x, self.y[: self.rows])
        corr = self.v[: self.rows]
        L.lbm_ws_compose(self.y[: self.rows], None, self.nc, 1, corr, stream=self.stream)
        fine_base = torch.empty((self.box ** 3, 4), device="cuda")
        L.lbm_ws_features(problem, self.box, self.box, None, fine_base, self.base_order,
                          self.rho_scale, stream=self.stream)
        fine = torch.empty((4, self.box ** 3), device="cuda")
        L.lbm_upsample_periodic(corr, self.nc, 4, fine, self.box, point_major_in=True,
                                addend=fine_base, stream=self.stream)
        L.lbm_reset_fields(lattice.ctx, fine, 2, U, U * self.rho_scale, flags)
        return U

    def save(self, path):
        """Parameters (path + '.npy') and the scales (path + '.json')."""
        np.save(path + ".npy", self.net.params())
        with open(path + ".json", "w") as fh:
            json.dump(dict(widths=self.widths, nc=self.nc, box=self.box,
                           base_order=self.base_order, rho_scale=self.rho_scale,
                           u_scale=self.u_scale), fh)

    def load(self, path):
        with open(path + ".json") as fh:
            meta = json.load(fh)
        if meta["widths"] != self.widths:
            raise ValueError(f"saved widths {meta['widths']} differ from {self.widths}")
        self.base_order = meta["base_order"]
        self._set_scales(meta["rho_scale"], meta["u_scale"])
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
    (inference, interpolation and restart included in the warm time, and timed on their
    own as inference_s).  The plain run's final velocity is the reference for the true
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
    ap.add_argument("--nc", type=int, default=32)
    ap.add_argument("--train", type=int, default=80)
    ap.add_argument("--val", type=int, default=16)
    ap.add_argument("--test", type=int, default=16)
    ap.add_argument("--iters", type=int, default=1500)
    ap.add_argument("--tol", type=float, default=1e-8)
    ap.add_argument("--data-tol", type=float, default=1e-8)
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
    ws = WarmStart(nc=args.nc, box=args.box, max_batch=8, seed=args.seed)
    parts = []
    t0 = time.time()
    data_steps = []
    for c0 in range(0, n_fit, args.chunk):
        ps = probs[c0:min(c0 + args.chunk, n_fit)]
        steps, _, status, fields = solve_batch(ps, args.box, args.data_tol, 3_000_000)
        if np.any(status != L.DOM_CONVERGED):
            raise RuntimeError(f"data solve did not converge: {status.tolist()}")
        parts.append(ws.dataset(ps, fields, fit_scale=(c0 == 0)))
        data_steps += steps.tolist()
        del fields
        print(f"data: {c0 + len(ps)}/{n_fit} solved, {time.time() - t0:.1f} s", flush=True)
    X, B, T = (torch.cat([p[k] for p in parts]) for k in range(3))
    del parts
    tr = slice(0, args.train)
    va = slice(args.train, n_fit)
    t0 = time.time()
    val_p = probs[args.train:n_fit]
    losses = ws.train(X[tr], B[tr], T[tr], iters=args.iters, batch=8, log_every=250,
                      val=lambda: validation_steps(ws, val_p, args.box, args.tol, 100))
    torch.cuda.synchronize()
    t_train = time.time() - t0
    print(f"train: {args.iters} iters, {t_train:.1f} s, final loss {losses[-1]:.3e}, "
          f"kept iteration {ws.best_iter}", flush=True)
    ws.save(os.path.join(args.out, "warmstart"))
    base = WarmStart(nc=args.nc, box=args.box, max_batch=1, seed=args.seed)
    base._set_scales(ws.rho_scale, ws.u_scale)
    results = []
    for i, p in enumerate(probs[n_fit:]):
        r = compare_starts(ws, p, args.box, args.tol, check_every=100)
        rb = compare_starts(base, p, args.box, args.tol, check_every=100,
                            reference=None, plain=r["plain"], reference_u=r["reference_u"])
        r["base"] = rb["warm"]
        del r["reference_u"]
        r.update(tau2=p["tau2"], U=p["U"])
        results.append(r)
        print(f"test {i}: plain {r['plain']['steps']} steps {r['plain']['wall_s']:.2f} s | "
              f"base {r['base']['steps']} steps {r['base']['wall_s']:.2f} s | "
              f"learned {r['warm']['steps']} steps {r['warm']['wall_s']:.2f} s", flush=True)

    def med(key, field):
        return float(np.median([r[key][field] / r["plain"][field] for r in results]))

    summary = dict(box=args.box, nc=args.nc, train=args.train, val=args.val, test=args.test,
                   iters=args.iters, kept_iteration=ws.best_iter, val_curve=ws.val_curve,
                   train_seconds=t_train, final_loss=losses[-1], data_steps=data_steps,
                   rho_scale=ws.rho_scale, u_scale=ws.u_scale, results=results,
                   steps_ratio_median=med("warm", "steps"), wall_ratio_median=med("warm", "wall_s"),
                   base_steps_ratio_median=med("base", "steps"),
                   base_wall_ratio_median=med("base", "wall_s"))
    with open(os.path.join(args.out, "warmstart_summary.json"), "w") as fh:
        json.dump(summary, fh, indent=1)
    print(json.dumps({k: v for k, v in summary.items()
                      if k not in ("results", "data_steps", "val_curve")}))


if __name__ == "__main__":
    main()
