"""Learned resummation of the lattice expansion: the warm start with a network in it.

The start is the steady state of the forced periodic lattice expanded to fourth order in
the forcing amplitude, as population waves (lbm_ws_lattice_waves_ordered), with each
order's waves W_n scaled by a learned factor:

    f_start = w rho0 + sum_n c_n W_n,   c_n = 1 + sigma y_n,

where sigma = a_3 / sqrt(a_2 a_1) is the expansion's own ratio (a_n the size of the
order-n amplitudes, lbm_ws_resum_features) and y = network(features) (4 values).  Where
the series converges fast, sigma is tiny and the start is the plain expansion; where it
converges slowly (stronger forcing, lower viscosity), the truncated series over- or
undershoots its orders, and the network predicts by how much from problem-level inputs
(tau2, the series' decay, the modes' Stokes amplitudes, wavenumbers and Reynolds
numbers).

Training data are solver outputs: each training problem is run from its plain
expansion to a converged steady state (per-step residual < 1e-10), and the factors c
that fit that state best are found by least squares over the waves' Fourier
coefficients (density and momentum at every wavevector the waves occupy).  The network
(lbm.MLP: BF16 matrix-core forward and backward kernels, FP32 Adam) is trained on
y = (c - 1) / sigma; the parameters are selected by the total steps to steady state on
validation problems, checked from iteration 0 (the zero output, i.e. the plain
expansion), so the kept network is never slower there than the start without it.  The
converged lattice solution remains the reference for the start's error.

Inference: waves (library, host), features (library, host), one forward pass (device),
the scaling (library, host), synthesis on the device (lbm_set_waves).

CLI (one GPU):
    python -m paper_2212_07494_amd.resum data  --out DIR --n 200        # training data
    python -m paper_2212_07494_amd.resum train --data DIR --out WEIGHTS  # network
    python -m paper_2212_07494_amd.resum eval  --weights WEIGHTS --n 16  # held-out problems
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
from . import warmstart as W

HERE = os.path.dirname(os.path.abspath(__file__))
WIDTHS = [L.WS_RESUM_FEATURES, 64, 64, 4]  # 5.8k parameters for ~10^2 training problems
WEIGHTS = os.path.join(HERE, "weights", "resum")
ORDER = 4
# The orders whose factors are learned (third and fourth).  The first two orders are
# accurate to far below what a prediction could resolve (their fitted factors differ
# from 1 by ~1e-7), and noise in them costs more than it gains: their factors stay 1.
LEARNED = (2, 3)
SIGMA_MIN = 1e-3   # problems below this series ratio start steady: no data from them
TRAIN_SEED, VAL_SEED, TEST_SEED = 40_000, 60_000, 80_000
# Seeds of the three splits: validation problems come from [VAL_SEED, VAL_SEED + VAL_SPAN),
# held-out test problems from TEST_SEED on; training problems from anywhere else at or
# above TRAIN_SEED (cmd_data refuses a set that reaches either range, cmd_train a set
# whose seeds meet the validation problems').
VAL_SPAN = 10_000


def _split_of_seed(s):
    if s >= TEST_SEED:
        return "test"
    if VAL_SEED <= s < VAL_SEED + VAL_SPAN:
        return "val"
    return "train" if s >= TRAIN_SEED else None


def check_splits(rows):
    """Refuses data rows whose seeds lie outside their split's range or that share a seed
    between the training and validation splits (rows written before seeds were recorded
    carry none and pass)."""
    tr = {r["seed"] for r in rows if r["split"] == "train" and "seed" in r}
    va = {r["seed"] for r in rows if r["split"] == "val" and "seed" in r}
    stray = sorted(r["seed"] for r in rows if "seed" in r and _split_of_seed(r["seed"]) != r["split"])
    if tr & va or stray:
        raise SystemExit(f"training and validation problems overlap or leave their seed "
                         f"ranges (shared seeds: {sorted(tr & va)[:5]}, out of range: {stray[:5]})")


def order_fields(k, ph, amp, ends, box):
    """Fourier coefficients (over N) of (rho - rho0, j_x, j_y, j_z) of each order's waves
    at every wavevector bin they occupy: (bins, P (nbins, 4, 4 orders) complex)."""
    e, _ = L.lbm_lattice_info("D3Q27")
    e = e.astype(np.float64)
    A = amp[..., 0] + 1j * amp[..., 1]
    v = np.concatenate([A.sum(1)[:, None], A @ e], 1) * np.exp(1j * ph)[:, None]
    per = []
    lo = 0
    for n in range(4):
        d = {}
        for w in range(lo, ends[n]):
            kp = tuple(int(x) % box for x in k[w])
            km = tuple(int(-x) % box for x in k[w])
            d[kp] = d.get(kp, 0) + v[w] / 2
            d[km] = d.get(km, 0) + np.conj(v[w]) / 2
        per.append(d)
        lo = ends[n]
    bins = sorted(set().union(*[set(d) for d in per]))
    P = np.stack([np.array([d.get(b, np.zeros(4)) for b in bins]) for d in per], -1)
    return bins, P


def fit_factors(problem, box, k, ph, amp, ends, rho, u, free=(0, 1, 2, 3)):
    """Least-squares order factors c (4,) of a converged state (rho, u), those of the
    orders not in `free` held at 1, and the relative residual of the fit and of c = 1."""
    N = box ** 3
    g = inputs.fourier_force((box, box, box), problem["modes"])
    j = rho * (u - 0.5 * g)
    F = [np.fft.fftn(x.reshape(box, box, box).T) / N for x in (rho - 1.0, j[0], j[1], j[2])]
    bins, P = order_fields(k, ph, amp, ends, box)
    T = np.array([[F[c][b] for c in range(4)] for b in bins])
    Ar = np.concatenate([P.real.reshape(-1, 4), P.imag.reshape(-1, 4)])
    tr = np.concatenate([T.real.ravel(), T.imag.ravel()])
    fixed = [n for n in range(4) if n not in free]
    rhs = tr - Ar[:, fixed].sum(1)
    cf, *_ = np.linalg.lstsq(Ar[:, list(free)], rhs, rcond=None)
    c = np.ones(4)
    c[list(free)] = cf
    nt = np.linalg.norm(tr)
    return c, float(np.linalg.norm(Ar @ c - tr) / nt), float(np.linalg.norm(Ar.sum(1) - tr) / nt)


def expansion(problem, box):
    """Order-4 waves with their order boundaries, features and sigma."""
    k, ph, amp, ends = L.lbm_ws_lattice_waves_ordered(problem, box, order=ORDER, tau3=W.TAU3)
    feat, sigma = L.lbm_ws_resum_features(problem, box, amp, ends)
    return k, ph, amp, ends, feat, sigma


def set_start(lattice, k, ph, amp, ends, c):
    a = np.ascontiguousarray(amp.copy())
    L.lbm_ws_scale_orders(a, ends, c)
    lattice.set_waves(k, ph, a[..., 0] + 1j * a[..., 1])


class ResumStart:
    """The network and the start it gives.  weights: path prefix of saved parameters
    (None: the zero output, i.e. the plain fourth-order expansion)."""

    def __init__(self, box=128, widths=WIDTHS, seed=0, stream=None, weights=None,
                 max_rows=4096):
        import torch
        self.torch = torch
        self.box = box
        self.widths = list(widths)
        self.stream = stream
        self.net = L.MLP(self.widths, max_rows=max_rows, stream=stream)
        self.x = torch.empty((max_rows, self.widths[0]), device="cuda")
        self.y = torch.empty((max_rows, self.widths[-1]), device="cuda")
        self.scale = np.ones(self.widths[-1], np.float32)
        self.reset(seed)
        if weights:
            self.load(weights)

    def reset(self, seed):
        p = inputs.mlp_init_params(self.widths, seed)
        nlast = self.widths[-1] * (self.widths[-2] + 1)
        p[-nlast:] = 0.0  # zero output: the plain expansion
        self.net.set_params(p.astype(np.float32))
        self.step = 0

    def set_scale(self, scale):
        self.scale = np.maximum(np.asarray(scale, np.float64), 1e-6).astype(np.float32)
        self.net.set_output_scale(self.scale)

    def predict_y(self, feats):
        """Network outputs y for a (rows, features) float32 array."""
        n = feats.shape[0]
        self.x[:n].copy_(self.torch.from_numpy(np.ascontiguousarray(feats, np.float32)))
        self.net.forward(self.x[:n], self.y[:n])
        return self.y[:n].cpu().numpy().astype(np.float64)

    def factors(self, feat, sigma):
        y = self.predict_y(feat[None])[0]
        c = np.ones(4)
        for n in LEARNED:
            c[n] = 1.0 + sigma * y[n]
        return c

    def start(self, lattice, problem):
        """Restart `lattice` (the problem's box^3 D3Q27 lattice) from the learned start;
        returns the factors c."""
        k, ph, amp, ends, feat, sigma = expansion(problem, self.box)
        c = self.factors(feat, sigma)
        set_start(lattice, k, ph, amp, ends, c)
        return c

    # -- training -----------------------------------------------------------------------
    def train(self, X, Y, iters=3000, lr=2e-3, lr_min=2e-5, val=None, eval_every=250,
              log_every=0, seed=1):
        """Adam with a cosine learning rate, full batches (the sets are small), loss the
        mean square of (y - target) in units of the output scales.  val, a callable
        returning the total validation steps, selects the parameters (evaluated at
        iteration 0 and every eval_every iterations; the best are kept)."""
        torch = self.torch
        n = X.shape[0]
        xb = torch.from_numpy(np.ascontiguousarray(X, np.float32)).cuda()
        tb = torch.from_numpy(np.ascontiguousarray(Y, np.float32)).cuda()
        w = (1.0 / self.scale.astype(np.float64) ** 2).astype(np.float32)
        for n in range(len(w)):
            if n not in LEARNED:
                w[n] = 0.0  # outputs that are not used
        self.val_curve, best = [], None

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
            self.net.forward(xb, self.y[:n])
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
        self.best_iter = None
        if best is not None:
            self.net.set_params(best[1])
            self.best_iter = best[2]
        return losses

    def save(self, path, meta=None):
        os.makedirs(os.path.dirname(path), exist_ok=True)
        np.save(path + ".npy", self.net.params())
        with open(path + ".json", "w") as fh:
            json.dump(dict(widths=self.widths, box=self.box, scale=self.scale.tolist(),
                           **(meta or {})), fh, indent=1)

    def load(self, path):
        with open(path + ".json") as fh:
            meta = json.load(fh)
        if meta["widths"] != self.widths:
            raise ValueError(f"saved widths {meta['widths']} differ from {self.widths}")
        self.set_scale(meta["scale"])
        self.net.set_params(np.load(path + ".npy", allow_pickle=False))
        self.meta = meta

    def close(self):
        self.net.close()


def fold_normalisation(params, widths, mean, std):
    """First layer of a network trained on (x - mean) / std, rewritten to take x:
    W0' = W0 / std, b0' = b0 - W0' mean."""
    p = np.asarray(params, np.float64).copy()
    n_in, n_out = widths[0], widths[1]
    W0 = p[: n_out * n_in].reshape(n_out, n_in)
    b0 = p[n_out * n_in: n_out * n_in + n_out]
    W0n = W0 / std[None, :]
    p[: n_out * n_in] = W0n.ravel()
    p[n_out * n_in: n_out * n_in + n_out] = b0 - W0n @ mean
    return p


def problems(seed0, n, box=128, sigma_min=SIGMA_MIN, max_draws=None):
    """n seeded wide-family problems whose expansion ratio sigma is at least sigma_min
    (with their expansions)."""
    out = []
    s = seed0
    limit = max_draws or 50 * n
    while len(out) < n and s - seed0 < limit:
        p = inputs.warmstart_problem(s, box=box, family="wide")
        p["seed"] = s
        s += 1
        ex = expansion(p, box)
        if ex[5] >= sigma_min:
            out.append((p, ex))
    return out


DATA_TOL = 1e-10  # the reference's per-step residual: its error is ~ resid / slowest decay rate


def converge(problem, ex, box, tol=DATA_TOL, check=100, max_steps=300_000, stream=None):
    """Run the problem from its plain expansion to resid < tol; (rho, u, steps, resid)."""
    k, ph, amp, ends = ex[:4]
    dom = W.domain_of(problem, box)
    with L.Lattice("D3Q27", "smrt", "f64", dom["shape"], dom["walls"], dom["tau"],
                   g_field=dom["g_field"], stream=stream) as lat:
        set_start(lat, k, ph, amp, ends, np.ones(4))
        steps, resid = W.run_to_steady(lat, tol, check, max_steps)
        rho, u = lat.moments()
    return rho, u, steps, resid


def steps_from(problem, ex, box, c, tol=1e-8, check=20, max_steps=300_000, stream=None):
    k, ph, amp, ends = ex[:4]
    dom = W.domain_of(problem, box)
    with L.Lattice("D3Q27", "smrt", "f64", dom["shape"], dom["walls"], dom["tau"],
                   g_field=dom["g_field"], stream=stream) as lat:
        set_start(lat, k, ph, amp, ends, c)
        return W.run_to_steady(lat, tol, check, max_steps)[0]


def cmd_data(args):
    L.load()
    os.makedirs(args.out, exist_ok=True)
    rows = []
    t0 = time.time()
    for split, seed0, n in (("train", TRAIN_SEED + args.seed_offset, args.n),
                            ("val", VAL_SEED + args.seed_offset, args.val)):
        for i, (p, ex) in enumerate(problems(seed0, n, args.box)):
            if _split_of_seed(p["seed"]) != split:
                raise SystemExit(f"seed {p['seed']} of a {split} problem lies in the "
                                 f"{_split_of_seed(p['seed'])} range: choose another offset")
            rho, u, steps, resid = converge(p, ex, args.box)
            if not resid < DATA_TOL:
                print(f"{split} {i}: not converged (resid {resid:.2e}), skipped", flush=True)
                continue
            k, ph, amp, ends, feat, sigma = ex
            c, fit, plain = fit_factors(p, args.box, k, ph, amp, ends, rho, u)
            rows.append(dict(split=split, seed=int(p["seed"]), tau2=p["tau2"], modes=[
                dict(k=[int(v) for v in m["k"]], p=[float(v) for v in m["p"]],
                     phase=float(m["phase"]), amp=float(m["amp"])) for m in p["modes"]],
                feat=feat.tolist(), sigma=sigma, c=c.tolist(), fit_resid=fit,
                order4_resid=plain, steps=int(steps)))
            print(f"{split} {i}: sigma {sigma:.2e} c {np.round(c, 4).tolist()} fit {fit:.1e} "
                  f"(order 4 {plain:.1e}), {steps} steps, {time.time() - t0:.0f} s", flush=True)
            with open(os.path.join(args.out, f"resum_data_{args.seed_offset}.json"), "w") as fh:
                json.dump(rows, fh)


def _problem_of(r):
    return dict(tau2=r["tau2"], modes=[dict(k=np.array(m["k"]), p=np.array(m["p"]),
                                            phase=m["phase"], amp=m["amp"]) for m in r["modes"]])


def cmd_train(args):
    import torch
    L.load()
    rows = []
    for name in sorted(os.listdir(args.data)):
        if name.startswith("resum_data") and name.endswith(".json"):
            rows += json.load(open(os.path.join(args.data, name)))
    tr = [r for r in rows if r["split"] == "train"]
    va = [r for r in rows if r["split"] == "val"]
    check_splits(rows)
    X = np.array([r["feat"] for r in tr], np.float64)
    Y = np.array([(np.array(r["c"]) - 1.0) / r["sigma"] for r in tr], np.float64)
    mean, std = X.mean(0), X.std(0) + 1e-6
    # the steps are spent on the problems whose series converges slowly: each problem
    # enters the loss in proportion to its ratio sigma (relative to the median), as copies
    sig = np.array([r["sigma"] for r in tr])
    reps = np.maximum(1, np.rint(sig / np.median(sig))).astype(int)
    X, Y = np.repeat(X, reps, 0), np.repeat(Y, reps, 0)
    rs = ResumStart(box=args.box, seed=args.seed)
    rs.set_scale(np.sqrt(np.mean(Y ** 2, 0)))
    val_p = [(_problem_of(r), None) for r in va]
    val_ex = [expansion(p, args.box) for p, _ in val_p]
    val_feat = np.array([ex[4] for ex in val_ex])
    Xn = (X - mean) / std
    Vn = (val_feat - mean) / std

    t0 = time.time()

    def val_steps():
        y = rs.predict_y(Vn.astype(np.float32))
        total = 0
        for (p, _), ex, yy in zip(val_p, val_ex, y):
            c = np.ones(4)
            for n in LEARNED:
                c[n] = 1.0 + ex[5] * yy[n]
            total += steps_from(p, ex, args.box, c)
        print(f"  validation: {total} steps ({time.time() - t0:.0f} s)", flush=True)
        return total

    t0 = time.time()
    losses = rs.train(Xn, Y, iters=args.iters, val=val_steps, eval_every=args.eval_every,
                      log_every=500)
    torch.cuda.synchronize()
    print(f"train: {args.iters} iterations in {time.time() - t0:.0f} s, loss {losses[0]:.3e} -> "
          f"{losses[-1]:.3e}; validation steps {rs.val_curve}; kept iteration {rs.best_iter}",
          flush=True)
    folded = fold_normalisation(rs.net.params(), rs.widths, mean, std)
    rs.net.set_params(folded.astype(np.float32))
    rs.save(args.out, meta=dict(kept_iteration=rs.best_iter, val_curve=rs.val_curve,
                                train_problems=len(tr), val_problems=len(va),
                                iters=args.iters, loss_first=losses[0], loss_last=losses[-1],
                                train_seed=TRAIN_SEED, val_seed=VAL_SEED,
                                sigma_min=SIGMA_MIN))
    # the folded network on raw features gives what the normalised one gave
    y_raw = rs.predict_y(val_feat.astype(np.float32))
    print("folded check (max |y|):", float(np.max(np.abs(y_raw))), flush=True)
    rs.close()


def evaluate(weights, n, box=128, seed0=TEST_SEED, sigma_min=SIGMA_MIN, tol=1e-8, check=20,
             stream=None, log=print, ceiling=False, plain=True):
    """Held-out problems: steps to resid < tol from rest, from the expansion (order 3 or 4
    by the series ratio, the start without a network), from the plain fourth-order
    expansion and from the learned start; with ceiling, also from the factors fitted to
    each problem's converged state (what a perfect network would give)."""
    ws = W.WarmStart(box=box, waves=True, stream=stream)
    rs = ResumStart(box=box, weights=weights, stream=stream)
    rows = []
    try:
        for i, (p, ex) in enumerate(problems(seed0, n, box, sigma_min)):
            dom = W.domain_of(p, box)
            r = dict(tau2=p["tau2"], Re=p["Re"], U=p["U"], sigma=ex[5])
            torch = rs.torch
            with L.Lattice("D3Q27", "smrt", "f64", dom["shape"], dom["walls"], dom["tau"],
                           g_field=dom["g_field"], stream=stream) as lat:
                if plain:
                    torch.cuda.synchronize()
                    t0 = time.perf_counter()
                    r["plain"] = W.run_to_steady(lat, tol, check, 300_000)[0]
                    torch.cuda.synchronize()
                    r["plain_s"] = time.perf_counter() - t0
                # the start without the network, its computation timed with the run
                t0 = time.perf_counter()
                lat.set_waves(*ws.lattice_waves(p))
                r["waves"] = W.run_to_steady(lat, tol, check, 300_000)[0]
                torch.cuda.synchronize()
                r["waves_s"] = time.perf_counter() - t0
                # the learned start: expansion, features, network, scaling, synthesis
                t0 = time.perf_counter()
                c = rs.start(lat, p)
                r["learned"] = W.run_to_steady(lat, tol, check, 300_000)[0]
                torch.cuda.synchronize()
                r["learned_s"] = time.perf_counter() - t0
            r["order4"] = steps_from(p, ex, box, np.ones(4), tol, check, stream=stream)
            r["c"] = c.tolist()
            if ceiling:
                rho, u, _, _ = converge(p, ex, box, stream=stream)
                cf, _, _ = fit_factors(p, box, *ex[:4], rho, u, free=LEARNED)
                r["c_fit"] = cf.tolist()
                r["ceiling"] = steps_from(p, ex, box, cf, tol, check, stream=stream)
            rows.append(r)
            log(json.dumps(r))
    finally:
        ws.close()
        rs.close()
    keys = (("plain",) if plain else ()) + ("waves", "order4", "learned") + \
        (("ceiling",) if ceiling else ())
    tot = {k: int(sum(r[k] for r in rows)) for k in keys}
    out = dict(problems=rows, totals=tot,
               learned_over_waves_total=tot["learned"] / tot["waves"],
               learned_over_waves_median=float(np.median([r["learned"] / r["waves"] for r in rows])),
               wall_learned_over_waves=sum(r["learned_s"] for r in rows) /
               sum(r["waves_s"] for r in rows))
    if plain:
        out["learned_over_plain_total"] = tot["learned"] / tot["plain"]
        out["wall_learned_over_plain"] = (sum(r["learned_s"] for r in rows) /
                                          sum(r["plain_s"] for r in rows))
    return out


def cmd_eval(args):
    L.load()
    res = evaluate(args.weights, args.n, args.box, sigma_min=args.sigma_min,
                   ceiling=args.ceiling)
    print(json.dumps({k: v for k, v in res.items() if k != "problems"}), flush=True)


def main():
    ap = argparse.ArgumentParser(description="learned resummation of the lattice expansion")
    sp = ap.add_subparsers(dest="cmd", required=True)
    d = sp.add_parser("data")
    d.add_argument("--out", required=True)
    d.add_argument("--n", type=int, default=160)
    d.add_argument("--val", type=int, default=16)
    d.add_argument("--box", type=int, default=128)
    d.add_argument("--seed-offset", type=int, default=0,
                   help="draw the training problems from TRAIN_SEED + this")
    t = sp.add_parser("train")
    t.add_argument("--data", required=True)
    t.add_argument("--out", default=WEIGHTS)
    t.add_argument("--iters", type=int, default=3000)
    t.add_argument("--eval-every", type=int, default=250)
    t.add_argument("--box", type=int, default=128)
    t.add_argument("--seed", type=int, default=0)
    e = sp.add_parser("eval")
    e.add_argument("--weights", default=WEIGHTS)
    e.add_argument("--n", type=int, default=16)
    e.add_argument("--box", type=int, default=128)
    e.add_argument("--sigma-min", type=float, default=SIGMA_MIN)
    e.add_argument("--ceiling", action="store_true",
                   help="also the steps from the factors fitted to each converged state")
    args = ap.parse_args()
    {"data": cmd_data, "train": cmd_train, "eval": cmd_eval}[args.cmd](args)


if __name__ == "__main__":
    main()
