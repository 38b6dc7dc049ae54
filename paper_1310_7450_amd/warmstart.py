"""Learned warm start of steady channel runs.

A network (``mlp.Net``: 5 -> 256 -> 256 -> 256 -> 192, SiLU, BF16 matrix-core
GEMMs with FP32 accumulation) maps the channel parameters
(log10 g, ny, eps, log10 tau0, G/eta_s) to the steady profiles of u_x,
sigma_xy and N1 = sigma_xx - sigma_yy at the 64 Chebyshev-Gauss points
d_k = cos(pi (2k+1)/128) across the channel (d = (y - y_c)/H). It is trained
on steady states the lattice-Boltzmann solver itself produces; at inference
the predicted u_x and N1 initialise new runs through ``lb_set_profile``. The
solver stays the judge: a warm run is kept only if its converged profile
agrees with a run from rest (else the rest run is the answer: fallback).

Targets are scaled to O(1): u_x by g H^2 / (2 eta_s), sigma_xy by g H and N1 by
G gamma_c^2 (lattice units, rho0 = 1).

Run the whole experiment with ``python -m paper_1310_7450_amd.warmstart``.
"""
import json
import math
import sys
import time

import numpy as np

from . import workloads
from .lbnlm import ChannelSpec, Solver
from .mlp import Net, init_params

DIMS = [5, 256, 256, 256, 192]
N_PTS = 64
CHEB = np.cos(np.pi * (2 * np.arange(N_PTS) + 1) / (2 * N_PTS))


def eta_s(spec):
    return (spec.tau_lb - 0.5) / 3.0


def features(specs):
    return np.array([[math.log10(c.force), c.ny, c.eps, math.log10(c.tau0), c.G / eta_s(c)] for c in specs])


def scales(spec):
    H = spec.ny / 2.0
    return (spec.force * H * H / (2.0 * eta_s(spec)), spec.force * H, max(spec.G * spec.gamma_c ** 2, 1e-300))


def sample_at_points(spec, ux, sxy, n1):
    """Row profiles -> values at the Chebyshev points (linear interpolation;
    u_x vanishes on the half-way walls, the stresses are extended linearly
    to them)."""
    ny = spec.ny
    H, yc = ny / 2.0, (ny - 1) / 2.0
    ys = yc + CHEB * H
    rows = np.arange(ny, dtype=np.float64)
    yw = np.concatenate([[-0.5], rows, [ny - 0.5]])

    def ext_lin(v):
        if ny == 1:
            return np.concatenate([[v[0]], v, [v[0]]])
        lo = v[0] - 0.5 * (v[1] - v[0])
        hi = v[-1] + 0.5 * (v[-1] - v[-2])
        return np.concatenate([[lo], v, [hi]])

    u = np.interp(ys, yw, np.concatenate([[0.0], ux, [0.0]]))
    s = np.interp(ys, yw, ext_lin(sxy))
    n = np.interp(ys, yw, ext_lin(n1))
    return u, s, n


def targets(specs, profiles):
    Y = np.zeros((len(specs), 3 * N_PTS))
    for i, (c, (ux, sxy, n1)) in enumerate(zip(specs, profiles)):
        u, s, n = sample_at_points(c, ux, sxy, n1)
        su, ss, sn = scales(c)
        Y[i] = np.concatenate([u / su, s / ss, n / sn])
    return Y


# Bounds put on a prediction before it initialises a run: the batch admits
# channels whose solvent Poiseuille velocity is at most U_SOLVENT_MAX (low
# Mach number), and the warm density 1 - (3/2) N1 must stay close to 1.
U_WARM_MAX = workloads.U_SOLVENT_MAX
N1_WARM_MAX = 1e-2


def solve_to_steady(specs, precision="fp32", max_steps=3_000_000, strip_rows=None, warm=None, tol=1e-9):
    """Runs every channel to its steady state (residual < tol) in one handle.
    ``warm`` optionally gives (u_x, N1) at the Chebyshev points per channel,
    clipped to the low-Mach range before use; ``strip_rows`` None takes the
    autotuner's choice for a run to steady state. A convergence check that
    sees NaN/Inf (LB_EUNSTABLE) restarts the offending channels from rest in
    the same handle; their wasted steps count with their run. Returns the row
    profiles (u_x, sigma_xy, N1), the steps each channel took, which channels
    froze, which were restarted from rest and the wall time."""
    from .lbnlm import LbError
    if strip_rows is None:
        from . import autotune
        strip_rows = autotune.tune_strip_rows(specs, precision, steps=200, to_steady=True)
    t0 = time.perf_counter()
    n = len(specs)
    restarted = np.zeros(n, dtype=bool)
    wasted = np.zeros(n, dtype=np.int64)
    with Solver(specs, precision=precision, obs_every=1000, steady_tol=tol, strip_rows=strip_rows) as s:
        if warm is not None:
            for i, (u, n1) in enumerate(warm):
                u = np.clip(np.asarray(u, dtype=np.float64), -U_WARM_MAX, U_WARM_MAX)
                n1 = np.clip(np.asarray(n1, dtype=np.float64), -N1_WARM_MAX, N1_WARM_MAX)
                s.set_profile(i, u, n1, points="chebyshev")
        done = 0
        while done < max_steps:
            try:
                s.step(max_steps - done)
                break
            except LbError as e:
                if e.status != -4:  # LB_EUNSTABLE
                    raise
                bad = [i for i in range(n) if s.observe(i, "nan") != 0.0]
                if not bad:
                    raise
                done = max(int(s.observe(i, "step")) + int(wasted[i]) for i in range(n))
                for i in bad:
                    c = specs[i]
                    t_i = int(s.observe(i, "step"))
                    wasted[i] += t_i
                    restarted[i] = True
                    s.set_state(i, np.broadcast_to(workloads.REST_WEIGHTS[:, None, None], (9, c.ny, c.nx)).copy(),
                                np.zeros((c.ny, c.nx)), 0)
        steps = np.array([int(s.observe(i, "step")) for i in range(n)]) + wasted
        frozen = np.array([s.observe(i, "active") == 0 for i in range(n)])
        prof = [(s.observe(i, "ux"), s.observe(i, "sxy"), s.observe(i, "n1")) for i in range(n)]
    return prof, steps, frozen, restarted, time.perf_counter() - t0


def generate(seeds, n_per_seed=256, verbose=True):
    specs = []
    for sd in seeds:
        specs += workloads.batched_sweep(seed=sd, n_channels=n_per_seed)["channels"]
    prof, steps, frozen, _, wall = solve_to_steady(specs)
    if verbose:
        print(f"warmstart: {len(specs)} training states, {frozen.sum()} steady, {wall:.1f} s", file=sys.stderr,
              flush=True)
    keep = np.nonzero(frozen)[0]
    specs = [specs[i] for i in keep]
    prof = [prof[i] for i in keep]
    return specs, features(specs), targets(specs, prof)


class Normaliser:
    def __init__(self, X):
        self.mu = X.mean(axis=0)
        sd = X.std(axis=0)
        self.sd = np.where(sd > 0, sd, 1.0)

    def __call__(self, X):
        return ((X - self.mu) / self.sd).astype(np.float32)


def train(X, Y, steps=4000, batch=256, lr=1e-3, seed=0, verbose=True):
    import torch
    norm = Normaliser(X)
    Xn = torch.from_numpy(norm(X)).cuda()
    Yd = torch.from_numpy(Y.astype(np.float32)).cuda()
    net = Net(DIMS, max_batch=batch)
    net.set_params(init_params(DIMS, seed=seed))
    rng = np.random.default_rng(seed)
    hist = []
    n = X.shape[0]
    # every minibatch's rows, drawn up front and copied once; the library
    # gathers them on the device (lbml_train_step)
    idx_all = torch.from_numpy(np.stack([rng.choice(n, batch, replace=n < batch) for _ in range(steps)])
                               .astype(np.int32)).cuda()
    for it in range(steps):
        want = (it % 500 == 0) or it == steps - 1
        # cosine decay of the learning rate
        loss = net.train_step(Xn, Yd, idx_all[it], lr=lr * 0.5 * (1 + math.cos(math.pi * it / steps)) + 1e-5,
                              want_loss=want)
        if want:
            hist.append((it, loss))
            if verbose and (it % 5000 == 0 or it == steps - 1):
                print(f"warmstart: train step {it} loss {loss:.4e}", file=sys.stderr, flush=True)
    return net, norm, hist


def predict(net, norm, specs):
    import torch
    X = torch.from_numpy(norm(features(specs))).cuda()
    out = []
    for i0 in range(0, len(specs), net.max_batch):
        xb = X[i0:i0 + net.max_batch].contiguous()
        out.append(net.forward(xb).cpu().numpy())
    Y = np.concatenate(out).astype(np.float64)
    res = []
    for c, y in zip(specs, Y):
        su, ss, sn = scales(c)
        res.append((y[:N_PTS] * su, y[N_PTS:2 * N_PTS] * ss, y[2 * N_PTS:] * sn))
    return res


def experiment(train_seeds=range(100, 116), test_seed=200, n_per_seed=256, train_steps=20000, train_lr=2e-3,
               train_batch=512, agree_tol=5e-3, n_test=None, verbose=True, details=False):
    """Trains on steady states of ``train_seeds`` and warm-starts the held-out
    ``test_seed`` batch (its first ``n_test`` channels, default all); returns
    a report of steps to steady, warm vs rest, and with ``details`` also the
    per-channel results."""
    t0 = time.perf_counter()
    specs, X, Y = generate(list(train_seeds), n_per_seed, verbose)
    t_gen = time.perf_counter() - t0
    net, norm, hist = train(X, Y, steps=train_steps, batch=train_batch, lr=train_lr, verbose=verbose)
    t_train = time.perf_counter() - t0 - t_gen
    test = workloads.batched_sweep(seed=test_seed, n_channels=n_per_seed)["channels"]
    if n_test is not None:
        test = test[:n_test]
    pred = predict(net, norm, test)
    prof_w, steps_w, frozen_w, restarted_w, wall_w = solve_to_steady(test, warm=[(u, n1) for u, _, n1 in pred])
    prof_r, steps_r, frozen_r, _, wall_r = solve_to_steady(test)
    # the solver judges: warm and rest converged profiles must agree (a run
    # stopped at residual R is up to about R / (slowest decay rate) from its
    # fixed point, 1e-4..1e-3 of u_x for the widest channels); a warm run the
    # solver had to restart from rest is a fallback too
    err = np.array([np.abs(pw[0] - pr[0]).max() / np.abs(pr[0]).max() for pw, pr in zip(prof_w, prof_r)])
    ok = (err <= agree_tol) & frozen_w & ~restarted_w
    used = np.where(ok, steps_w, steps_r + steps_w)  # a fallback pays for both runs
    pred_err = []
    for c, p, pr in zip(test, pred, prof_r):
        u, _, _ = sample_at_points(c, *pr)
        pred_err.append(np.abs(p[0] - u).max() / np.abs(u).max())
    ratio = steps_r / np.maximum(steps_w, 1)
    rep = {
        "train_states": int(X.shape[0]), "train_seeds": [int(s) for s in train_seeds], "test_seed": int(test_seed),
        "test_channels": len(test), "final_train_loss": hist[-1][1],
        "prediction_linf_rel_ux": {"median": float(np.median(pred_err)), "max": float(np.max(pred_err))},
        "steps_rest": {"median": int(np.median(steps_r)), "total": int(steps_r.sum())},
        "steps_warm": {"median": int(np.median(steps_w)), "total": int(steps_w.sum())},
        "steps_ratio_rest_over_warm": {"median": float(np.median(ratio)),
                                       "geomean": float(np.exp(np.mean(np.log(ratio))))},
        "steps_with_fallback_total": int(used.sum()),
        "fallbacks": int((~ok).sum()), "restarted_unstable": int(restarted_w.sum()), "agree_tol": agree_tol,
        "final_linf_rel_ux_warm_vs_rest": {"median": float(np.median(err)), "max": float(np.max(err))},
        "seconds": {"generate": round(t_gen, 1), "train": round(t_train, 1), "warm_run": round(wall_w, 1),
                    "rest_run": round(wall_r, 1)},
    }
    if details:
        return rep, {"test": test, "pred": pred, "prof_warm": prof_w, "prof_rest": prof_r, "steps_warm": steps_w,
                     "steps_rest": steps_r, "frozen_warm": frozen_w, "frozen_rest": frozen_r, "ok": ok,
                     "restarted_warm": restarted_w,
                     "err_warm_vs_rest": err}
    return rep


def time_training(steps=2000, batch=512, seed=0):
    """Wall time per training step of the network on seeded synthetic data
    (X ~ N(0, 1) of shape 4096 x 5, Y = sin(X A) with a seeded 5 x 192
    matrix A), after 50 warm-up steps: the cost of the training loop alone."""
    import torch
    rng = np.random.default_rng(seed)
    X = rng.standard_normal((4096, DIMS[0]))
    Y = np.sin(X @ rng.standard_normal((DIMS[0], DIMS[-1])))
    train(X, Y, steps=50, batch=batch, lr=2e-3, verbose=False)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    _, _, hist = train(X, Y, steps=steps, batch=batch, lr=2e-3, verbose=False)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    return {"steps": steps, "batch": batch, "seconds": round(dt, 4), "us_per_step": round(dt / steps * 1e6, 1),
            "final_loss": hist[-1][1]}


if __name__ == "__main__":
    import argparse
    ap = argparse.ArgumentParser(description="the learned warm-start experiment, or the training loop's timing")
    ap.add_argument("--time-training", type=int, default=0, metavar="STEPS",
                    help="time STEPS training steps on synthetic data instead of running the experiment")
    args = ap.parse_args()
    if args.time_training:
        print(json.dumps(time_training(args.time_training)), flush=True)
    else:
        print(json.dumps(experiment()), flush=True)
