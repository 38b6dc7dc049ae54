"""Throughput of the fused D2Q9 + inlM sweep on one MI355X.

One step is one lattice-Boltzmann time step of the whole 4096 x 1024
channel (every node pulled, stress evaluated, collided and stored). The
headline value is FP32-shifted MLUPS (million lattice-node updates per
second) with the state resident in HBM; the FP64 run of the same workload is
reported beside it, and the FP64 CPU oracle is timed on a bounded sample of
the same lattice on the host. Further legs: the batched channels to steady
state, the 16 x 8192 x 2048 start-up lattice, the same 4096 x 1024 lattice
with the time-integrated (viscoelastic) stress and with the stress as a force
density, and the learned warm start.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-fp64] [--no-cpu]
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "MLUPS + % HBM roofline (FP32 vs FP64); steps-to-steady, learned vs from-rest"
HBM_PEAK_GBS = 8000.0
# Algorithmic HBM bytes per node update: read 9 populations + the previous
# stress trace, write 9 populations + the new trace; the time-integrated
# (viscoelastic) model also reads and writes the three stress fields.
BYTES_PER_NODE = {"fp32": 80, "fp64": 160}
BYTES_PER_NODE_VE = {"fp32": 104, "fp64": 208}
# Stress as a force density (FP64, one fused kernel per step): u~ and
# Sigma^nN stay on chip, so a node update reads 9 populations and P and
# writes them (80 + 80 B), as the FP64 sweep does.
BYTES_PER_NODE_SAF = 160


def measured_traffic(key):
    """HBM bytes per sweep launch from the committed rocprofv3 counter
    summary (FETCH_SIZE and WRITE_SIZE, scaled by a copy of known size) for
    'fp32' / 'fp64' (4096 x 1024, two steps per launch), 'fp32_one' /
    'fp64_one' (one step per launch), 'transient_fp32' (16 x 8192 x 2048, two
    steps per launch) and the other legs' keys, or
    None when the kernel sources changed since the counters were taken."""
    path = os.path.join(ROOT, "profiles", "traffic_sweep_vec.json")
    if not os.path.exists(path):
        return None
    rec = json.load(open(path))
    h = hashlib.sha256()
    for f in ["lb_kernels.hip", "lb_runtime.hip", "lb_internal.h"]:
        h.update(open(os.path.join(ROOT, "paper_1310_7450_amd", "csrc", f), "rb").read())
    if h.hexdigest()[:16] != rec.get("source_hash"):
        return None
    k = rec["kernels"].get(key)
    return None if k is None else round(k["traffic_bytes"])


def time_solver(precision, wl, steps, warmup, strip_rows=0, viscoelastic=False, stress_force=False,
                steps_per_sweep=0):
    import torch
    from paper_1310_7450_amd import Solver
    spec = wl["channels"][0]
    nodes = spec.nx * spec.ny
    with Solver([spec], precision=precision, obs_every=1000, strip_rows=strip_rows, viscoelastic=viscoelastic,
                stress_force=stress_force, nn_pressure=not stress_force, steps_per_sweep=steps_per_sweep) as s:
        s.step(warmup)
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        t0 = time.perf_counter()
        e0.record(s.stream)
        s.step(steps)
        e1.record(s.stream)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        ms = e0.elapsed_time(e1)
        umid = s.observe(0, "umid")
        mass = s.observe(0, "mass")
    sec = ms / 1e3
    per_step = sec / steps
    mlups = nodes * steps / sec / 1e6
    bpn = BYTES_PER_NODE_SAF if stress_force else (BYTES_PER_NODE_VE if viscoelastic else BYTES_PER_NODE)[precision]
    achieved = bpn * nodes / per_step / 1e9
    return {"mlups": mlups, "ms_total": ms, "ms_per_step": ms / steps, "wall_s": wall,
            "achieved_GBs": achieved, "frac": achieved / HBM_PEAK_GBS, "umid": umid,
            "mass_rel_drift": (mass - nodes) / nodes}


def run_batched(max_steps=None, verbose=True):
    """The batched sweep: 256 ragged channels (nx = 8) in one handle, FP32
    shifted populations with FP64 reductions, each frozen once its steady
    residual is below 1e-9; strip rows from the autotuner. Whole-job
    throughput counts every node update of every channel until it froze."""
    import torch
    from paper_1310_7450_amd import Solver, autotune, workloads
    wl = workloads.batched_sweep()
    chans = wl["channels"]
    sr = autotune.tune_strip_rows(chans, "fp32", steps=200, verbose=verbose, to_steady=True)
    ms = wl["max_steps"] if max_steps is None else max_steps
    with Solver(chans, precision="fp32", obs_every=wl["obs_every"], steady_tol=wl["steady_tol"],
                strip_rows=sr) as s:
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        t0 = time.perf_counter()
        e0.record(s.stream)
        s.step(ms)
        e1.record(s.stream)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        steps = [int(s.observe(i, "step")) for i in range(len(chans))]
        active = [int(s.observe(i, "active")) for i in range(len(chans))]
        ref = batched_oracle_fixture()
        errs = {i: (linf_rel(s.observe(i, "ux"), u), linf_rel(s.observe(i, "sxy"), sx), steps[i] - t)
                for i, (t, u, sx) in ref.items()}
    sec = e0.elapsed_time(e1) / 1e3
    updates = sum(c.nx * c.ny * n for c, n in zip(chans, steps))
    import numpy as np
    st = np.array(steps)
    eu = np.array([e[0] for e in errs.values()])
    es = np.array([e[1] for e in errs.values()])
    return {"workload": wl["name"], "channels": len(chans), "nodes": sum(c.nx * c.ny for c in chans),
            "admitted": f"{len(chans)} of {wl['draws']} draws (seed {wl['seed']}; low-Mach rule only)",
            "stiff_split": f"{wl['stiff']} channels with G_inf tau > 0.3 run with visc_split 1/2, no delta-rho terms",
            "strip_rows": sr,
            "value": round(updates / sec / 1e6, 1), "unit": "MLUPS", "seconds": round(sec, 3),
            "wall_s": round(wall, 3), "converged": int(len(chans) - sum(active)),
            "steps_to_steady": {"median": int(np.median(st)), "max": int(st.max()), "min": int(st.min())},
            "precision": "fp32_shifted", "steady_tol": wl["steady_tol"],
            "error_vs_oracle": {
                "sample": f"{len(errs)} channels (three per width decile and the four widest), FP64 oracle steady "
                          "states from rest (tests/golden/batched_sweep_seed2_oracle.txt)",
                "linf_rel_ux": {"median": float(np.median(eu)), "max": float(eu.max())},
                "linf_rel_sxy": {"median": float(np.median(es)), "max": float(es.max())},
                "steps_minus_oracle": {"min": int(min(e[2] for e in errs.values())),
                                       "max": int(max(e[2] for e in errs.values()))}}}


def linf_rel(a, b):
    import numpy as np
    return float(np.abs(np.asarray(a) - np.asarray(b)).max() / np.abs(np.asarray(b)).max())


def batched_oracle_fixture():
    """The FP64 oracle's steady states of the batched sweep's width-stratified
    sample, stored by tests/golden/make_batched_oracle.py (oracle only)."""
    import importlib.util
    path = os.path.join(ROOT, "tests", "golden", "make_batched_oracle.py")
    spec = importlib.util.spec_from_file_location("make_batched_oracle", path)
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod.load()


def run_transient_scale(steps=200, warmup=100):
    """Throughput of the start-up/cessation workload at full size: 16
    channels of 8192 x 2048 (268M nodes), FP32 shifted, from rest with the
    force on. The protocol itself (250,000 steps, stopping times) runs on the
    x-reduced lattice in the tests."""
    import torch
    from paper_1310_7450_amd import Solver, workloads
    wl = workloads.transient_scale()
    chans = wl["channels"]
    nodes = sum(c.nx * c.ny for c in chans)
    # blocks of 100 steps, so that the timed steps are whole captured blocks
    # (two steps per pass)
    with Solver(chans, precision="fp32", obs_every=100) as s:
        s.step(warmup)
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(s.stream)
        s.step(steps)
        e1.record(s.stream)
        torch.cuda.synchronize()
        sec = e0.elapsed_time(e1) / 1e3
    achieved = BYTES_PER_NODE["fp32"] * nodes * steps / sec / 1e9
    return {"workload": wl["name"], "nodes": nodes, "steps": steps, "value": round(nodes * steps / sec / 1e6, 1),
            "unit": "MLUPS", "ms_per_step": round(sec * 1e3 / steps, 4),
            "roofline": two_step_roofline(achieved, nodes, sec / steps, measured_traffic("transient_fp32"))}


def copy_bandwidth(reps=5):
    """Measured device copy rate (GB/s, bytes read plus bytes written): a
    plain copy of 1 GiB, timed with HIP events after two untimed copies."""
    import torch
    n = 1 << 28
    a = torch.ones(n, device="cuda")
    b = torch.empty_like(a)
    for _ in range(2):
        b.copy_(a)
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        b.copy_(a)
    e1.record()
    torch.cuda.synchronize()
    sec = e0.elapsed_time(e1) / 1e3
    del a, b
    torch.cuda.empty_cache()
    return 2 * 4 * n * reps / sec / 1e9


def two_step_roofline(achieved, nodes, sec_per_step, traffic, precision="fp32", bpn=None):
    """Roofline of the two-step sweep (sweep_vec2_kernel): one launch
    performs two node updates per node, so at B bytes per node update (80 in
    FP32, 160 in FP64) its algorithmic bytes are 2 B per node and launch; the
    state itself is read and written once per launch (B per node), which
    state_GBs reports beside the counters' traffic per launch. The kernel is
    limited by instruction issue, not by HBM (state_frac)."""
    bpn = BYTES_PER_NODE[precision] if bpn is None else bpn
    state = bpn * nodes / (2 * sec_per_step) / 1e9
    out = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
           "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
           "traffic_unit": "bytes per launch (rocprofv3 FETCH_SIZE + WRITE_SIZE, copy-calibrated)",
           "kernel": "sweep_vec2_kernel", "node_updates_per_launch": 2 * nodes,
           "bytes_per_node_update": bpn, "algorithmic_bytes_per_launch": 2 * bpn * nodes,
           "state_bytes_per_launch": bpn * nodes, "state_GBs": round(state, 1),
           "state_frac": round(state / HBM_PEAK_GBS, 4)}
    if traffic is not None:
        out["traffic_GBs"] = round(traffic / (2 * sec_per_step) / 1e9, 1)
    return out


def run_viscoelastic(steps=2000, warmup=1000):
    """The same 4096 x 1024 workload with the time-integrated nonlinear
    Maxwell stress (three more fields per node read and written), FP32 and
    FP64."""
    from paper_1310_7450_amd import workloads
    wl = workloads.large_channel()
    out = {"workload": wl["name"] + "_viscoelastic", "steps": steps}
    nodes = wl["channels"][0].nx * wl["channels"][0].ny
    for prec in ("fp32", "fp64"):
        r = time_solver(prec, wl, steps, warmup, viscoelastic=True)
        one = time_solver(prec, wl, steps, warmup, viscoelastic=True, steps_per_sweep=1)
        out[prec] = {"value": round(r["mlups"], 1), "unit": "MLUPS", "ms_per_step": round(r["ms_per_step"], 5),
                     "bytes_per_node": BYTES_PER_NODE_VE[prec],
                     "roofline": two_step_roofline(r["achieved_GBs"], nodes, r["ms_per_step"] / 1e3,
                                                   measured_traffic("ve_" + prec), prec, BYTES_PER_NODE_VE[prec]),
                     "one_step_per_pass": {
                         "value": round(one["mlups"], 1), "unit": "MLUPS", "ms_per_step": round(one["ms_per_step"], 5),
                         "roofline": {"bound": "hbm", "achieved": round(one["achieved_GBs"], 1), "peak": HBM_PEAK_GBS,
                                      "unit": "GB/s", "frac": round(one["frac"], 4),
                                      "traffic": measured_traffic("ve_" + prec + "_one")}}}
    return out


def run_stress_force(steps=1000, warmup=1000):
    """The same 4096 x 1024 workload with the stress as a force density
    (FP64, no flow-induced density, one fused kernel per step)."""
    from paper_1310_7450_amd import workloads
    wl = workloads.large_channel()
    r = time_solver("fp64", wl, steps, warmup, stress_force=True)
    return {"workload": wl["name"] + "_stress_force", "steps": steps, "value": round(r["mlups"], 1),
            "unit": "MLUPS", "ms_per_step": round(r["ms_per_step"], 5), "bytes_per_node": BYTES_PER_NODE_SAF,
            "roofline": {"bound": "hbm", "achieved": round(r["achieved_GBs"], 1), "peak": HBM_PEAK_GBS,
                         "unit": "GB/s", "frac": round(r["frac"], 4), "traffic": measured_traffic("saf_fp64")}}


def run_warm_start(verbose=True):
    """Steps to steady state, learned warm start vs from rest: the network is
    trained on the GPU on 4096 solver steady states (seeds 100..115) and
    initialises the 256 held-out channels of seed 200."""
    from paper_1310_7450_amd import warmstart
    return warmstart.experiment(verbose=verbose)


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def _time_oracle(channel, budget_s):
    """Whole oracle steps of one channel for about budget_s seconds (at
    least one, after one warm-up step): (node updates, seconds, steps)."""
    channel.run(1)
    n = 0
    t0 = time.perf_counter()
    while True:
        channel.run(1)
        n += 1
        if time.perf_counter() - t0 > budget_s:
            break
    return channel.nx * channel.ny * n, time.perf_counter() - t0, n


def cpu_baseline(wl, budget_s=15.0):
    """The FP64 oracle as it stands, on the same lattice, for as many whole
    steps as fit in about budget_s seconds with every host thread, then for
    a fifth of that at one thread; and the batched sweep's channels, 1000
    steps each, for a fifth of the budget."""
    from oracle import core as orc
    from paper_1310_7450_amd import workloads
    spec = wl["channels"][0]

    def channel(c):
        return orc.Channel(c.nx, c.ny, c.force, tau_lb=c.tau_lb, G=c.G, tau0=c.tau0, gamma_c=c.gamma_c,
                           eps=c.eps, visc_split=c.visc_split, nn_pressure=c.resolved_nn_pressure())

    threads = orc.num_threads()
    upd, sec, n = _time_oracle(channel(spec), budget_s)
    orc.set_num_threads(1)
    upd1, sec1, n1 = _time_oracle(channel(spec), budget_s / 5)
    orc.set_num_threads(threads)
    # batched sweep: whole channels of 1000 steps until a fifth of the budget is spent
    b_upd, b_sec, b_ch = 0, 0.0, 0
    for c in workloads.batched_sweep()["channels"]:
        o = channel(c)
        t0 = time.perf_counter()
        o.run(1000)
        b_sec += time.perf_counter() - t0
        b_upd += c.nx * c.ny * 1000
        b_ch += 1
        if b_sec > budget_s / 5:
            break
    return {"value": upd / sec / 1e6, "unit": "MLUPS", "cores": threads, "kind": "oracle",
            "sample": f"{n} steps of the {spec.nx}x{spec.ny} lattice from rest (after 1 warm-up step), FP64, "
                      f"{threads} threads on {cpu_model()}",
            "single_thread": {"value": upd1 / sec1 / 1e6, "unit": "MLUPS", "cores": 1,
                              "sample": f"{n1} steps of the same lattice"},
            "batched": {"value": b_upd / b_sec / 1e6, "unit": "MLUPS", "cores": threads,
                        "sample": f"first {b_ch} channels of the batched sweep (nx = 8), 1000 steps each, FP64"}}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10000)
    ap.add_argument("--warmup", type=int, default=1000)
    ap.add_argument("--no-fp64", action="store_true")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--cpu-budget", type=float, default=15.0)
    ap.add_argument("--strip-rows", type=int, default=0, help="rows per wavefront strip (0: library default)")
    ap.add_argument("--tune", type=str, default="",
                    help="comma-separated strip_rows values to time (FP32 and FP64) instead of the JSON line")
    ap.add_argument("--no-batched", action="store_true", help="skip the batched-channel sweep")
    ap.add_argument("--no-transient", action="store_true", help="skip the 16 x 8192 x 2048 throughput leg")
    ap.add_argument("--no-warm", action="store_true", help="skip the learned warm-start experiment")
    ap.add_argument("--no-viscoelastic", action="store_true", help="skip the time-integrated stress leg")
    ap.add_argument("--no-stress-force", action="store_true", help="skip the stress-as-force leg")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain device copy of 1 GiB, 5 times (counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py: this build runs on one GPU only; multi-GPU runs are not part of it "
              f"(asked for --gpus {args.gpus})", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1310_7450_amd import workloads
    assert torch.cuda.is_available(), "bench.py needs the GPU"
    if args.copy_calibration:
        n = 1 << 28  # 2^28 float32 = 1 GiB read and 1 GiB written per copy
        a = torch.ones(n, device="cuda")
        b = torch.empty_like(a)
        for _ in range(5):
            b.copy_(a)
        torch.cuda.synchronize()
        print(f"copy calibration: 5 copies of {n * 4} bytes", flush=True)
        return
    wl = workloads.large_channel()
    if args.tune:
        for sr in [int(v) for v in args.tune.split(",")]:
            for prec in ["fp32", "fp64"]:
                r = time_solver(prec, wl, args.steps, args.warmup, sr)
                print(f"tune strip_rows={sr} {prec}: {r['mlups']:.0f} MLUPS {r['achieved_GBs']:.0f} GB/s "
                      f"({100 * r['frac']:.1f}%)", flush=True)
        return
    spec = wl["channels"][0]
    copy_gbs = copy_bandwidth()
    print(f"bench: device copy {copy_gbs:.0f} GB/s", file=sys.stderr, flush=True)
    print(f"bench: {wl['name']} g={spec.force:.3e} eps={spec.eps:+.4f}, fp32 {args.steps} steps",
          file=sys.stderr, flush=True)
    r32 = time_solver("fp32", wl, args.steps, args.warmup, args.strip_rows)
    print(f"bench: fp32 {r32['mlups']:.0f} MLUPS, {r32['achieved_GBs']:.0f} GB/s", file=sys.stderr, flush=True)
    r32one = time_solver("fp32", wl, min(args.steps, 4000), min(args.warmup, 1000), args.strip_rows,
                         steps_per_sweep=1)
    print(f"bench: fp32 one step per pass {r32one['mlups']:.0f} MLUPS", file=sys.stderr, flush=True)
    r64 = None
    if not args.no_fp64:
        r64 = time_solver("fp64", wl, args.steps, args.warmup, args.strip_rows)
        print(f"bench: fp64 {r64['mlups']:.0f} MLUPS, {r64['achieved_GBs']:.0f} GB/s", file=sys.stderr, flush=True)
        r64one = time_solver("fp64", wl, min(args.steps, 4000), min(args.warmup, 1000), args.strip_rows,
                             steps_per_sweep=1)
        print(f"bench: fp64 one step per pass {r64one['mlups']:.0f} MLUPS", file=sys.stderr, flush=True)
    batched = None
    if not args.no_batched:
        batched = run_batched()
        print(f"bench: batched {batched['value']:.0f} MLUPS, {batched['converged']}/{batched['channels']} steady "
              f"in {batched['seconds']:.1f} s", file=sys.stderr, flush=True)
    transient = None
    if not args.no_transient:
        transient = run_transient_scale()
        print(f"bench: transient_scale {transient['value']:.0f} MLUPS "
              f"({100 * transient['roofline']['frac']:.1f}% of HBM peak)", file=sys.stderr, flush=True)
    ve = None
    if not args.no_viscoelastic:
        ve = run_viscoelastic()
        print(f"bench: viscoelastic fp32 {ve['fp32']['value']:.0f} MLUPS "
              f"({100 * ve['fp32']['roofline']['frac']:.1f}%), fp64 {ve['fp64']['value']:.0f} MLUPS "
              f"({100 * ve['fp64']['roofline']['frac']:.1f}%)", file=sys.stderr, flush=True)
    saf = None
    if not args.no_stress_force:
        saf = run_stress_force()
        print(f"bench: stress force fp64 {saf['value']:.0f} MLUPS ({100 * saf['roofline']['frac']:.1f}% at "
              f"{BYTES_PER_NODE_SAF} B/node)", file=sys.stderr, flush=True)
    warm = None
    if not args.no_warm:
        warm = run_warm_start()
        print(f"bench: warm start cuts steps to steady by {warm['steps_ratio_rest_over_warm']['geomean']:.2f}x "
              f"(geomean), {warm['fallbacks']} fallbacks", file=sys.stderr, flush=True)
    cpu = None
    if not args.no_cpu:
        cpu = cpu_baseline(wl, args.cpu_budget)
        print(f"bench: cpu oracle {cpu['value']:.2f} MLUPS on {cpu['cores']} threads", file=sys.stderr, flush=True)

    out = {
        "metric": METRIC,
        "value": round(r32["mlups"], 1),
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(r32["ms_per_step"], 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": wl["name"], "nx": spec.nx, "ny": spec.ny, "seed": wl["seed"],
                   "force": spec.force, "eps": spec.eps, "tau_lb": spec.tau_lb, "G": spec.G,
                   "tau0": spec.tau0, "gamma_c": spec.gamma_c, "precision": "fp32_shifted",
                   "nn_pressure": 1, "start": "rest"},
        "roofline": dict(two_step_roofline(r32["achieved_GBs"], spec.nx * spec.ny, r32["ms_per_step"] / 1e3,
                                           measured_traffic("fp32")),
                         copy_GBs=round(copy_gbs, 1), frac_of_copy=round(r32["achieved_GBs"] / copy_gbs, 4)),
        "fp32_one_step_per_pass": {
            "value": round(r32one["mlups"], 1), "unit": "MLUPS", "ms_per_step": round(r32one["ms_per_step"], 5),
            "roofline": {"bound": "hbm", "achieved": round(r32one["achieved_GBs"], 1), "peak": HBM_PEAK_GBS,
                         "unit": "GB/s", "frac": round(r32one["frac"], 4), "traffic": measured_traffic("fp32_one"),
                         "kernel": "sweep_vec_kernel", "frac_of_copy": round(r32one["achieved_GBs"] / copy_gbs, 4)}},
        "fp64": None if r64 is None else {
            "value": round(r64["mlups"], 1), "unit": "MLUPS", "ms_per_step": round(r64["ms_per_step"], 5),
            "roofline": two_step_roofline(r64["achieved_GBs"], spec.nx * spec.ny, r64["ms_per_step"] / 1e3,
                                          measured_traffic("fp64"), "fp64"),
            "one_step_per_pass": {
                "value": round(r64one["mlups"], 1), "unit": "MLUPS", "ms_per_step": round(r64one["ms_per_step"], 5),
                "roofline": {"bound": "hbm", "achieved": round(r64one["achieved_GBs"], 1), "peak": HBM_PEAK_GBS,
                             "unit": "GB/s", "frac": round(r64one["frac"], 4),
                             "traffic": measured_traffic("fp64_one"), "kernel": "sweep_tile_kernel",
                             "frac_of_copy": round(r64one["achieved_GBs"] / copy_gbs, 4)}}},
        "batched": batched,
        "transient_scale": transient,
        "viscoelastic": ve,
        "stress_force": saf,
        "warm_start": warm,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
