"""Writes ``batched_sweep_seed2_oracle.txt``: the FP64 oracle's steady states
of a width-stratified sample of the batched sweep (seed 2), the expected
values of the batched tests and of the benchmark's per-channel error.

Calls only ``oracle/`` (and the seeded input recipe in
``paper_1310_7450_amd/workloads.py``, which holds no arithmetic of the
method). Each sampled channel runs on the oracle at nx = 1 (the flow from
rest stays x-uniform) from rest until the steady residual
R = max_y |ubar(t) - ubar(t - K)| / (K max_y |ubar(t)|), checked every
K = 1000 steps from the second check on, falls below 1e-9: the criterion
the solver applies. Run: ``python tests/golden/make_batched_oracle.py``
(about ten minutes on 8 cores).
"""
import multiprocessing as mp
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
OUT = os.path.join(HERE, "batched_sweep_seed2_oracle.txt")
K = 1000
TOL = 1e-9
CAP = 3_000_000


def steady(args):
    i, c = args
    sys.path.insert(0, ROOT)
    import numpy as np
    from oracle import core as orc
    orc.set_num_threads(1)
    o = orc.Channel(1, c.ny, c.force, tau_lb=c.tau_lb, G=c.G, tau0=c.tau0, gamma_c=c.gamma_c, eps=c.eps,
                    visc_split=c.visc_split, nn_pressure=c.nn_pressure)
    prev = None
    while o.t < CAP:
        o.run(K)
        u = o.profiles()["ux"]
        if prev is not None:
            R = np.abs(u - prev).max() / (K * np.abs(u).max())
            if R < TOL:
                break
        prev = u
    pr = o.profiles()
    return i, o.t, pr["ux"], pr["sxy"]


def main():
    sys.path.insert(0, ROOT)
    from paper_1310_7450_amd import workloads
    wl = workloads.batched_sweep(seed=2)
    chans = wl["channels"]
    idx = workloads.batched_sample(chans)
    jobs = sorted(((i, chans[i]) for i in idx), key=lambda a: -a[1].ny)
    with mp.get_context("spawn").Pool(os.cpu_count()) as pool:
        res = {}
        for i, t, u, s in pool.imap_unordered(steady, jobs):
            res[i] = (t, u, s)
            print(f"channel {i} (ny {chans[i].ny}): steady after {t} steps", flush=True)
    with open(OUT, "w") as f:
        f.write("# FP64 oracle steady states of the batched sweep (seed 2, 256 channels, nx = 8), width-stratified\n"
                "# sample (workloads.batched_sample). Written by tests/golden/make_batched_oracle.py from the oracle\n"
                "# alone (nx = 1, from rest, residual < 1e-9 checked every 1000 steps).\n"
                "# Per channel: a line 'channel <index> ny <ny> steps <steps>', then ny lines 'u_x sigma_xy'\n"
                "# for rows y = 0 .. ny-1.\n")
        for i in sorted(res):
            t, u, s = res[i]
            f.write(f"channel {i} ny {chans[i].ny} steps {t}\n")
            for a, b in zip(u, s):
                f.write(f"{a:.10e} {b:.10e}\n")
    print(f"wrote {OUT}")


def load(path=OUT):
    """{channel index: (steps, u_x[ny], sigma_xy[ny])} from the fixture."""
    import numpy as np
    out, cur = {}, None
    with open(path) as f:
        for line in f:
            if line.startswith("#"):
                continue
            if line.startswith("channel"):
                w = line.split()
                cur = int(w[1])
                out[cur] = (int(w[5]), [], [])
                continue
            a, b = line.split()
            out[cur][1].append(float(a))
            out[cur][2].append(float(b))
    return {k: (t, np.array(u), np.array(s)) for k, (t, u, s) in out.items()}


if __name__ == "__main__":
    main()
