"""Start-up and cessation protocol driver (Sec. III.C of the paper).

Host logic only: it steps a :class:`Solver` whose channels switch their
body force off at ``t_startup`` and records the centre-line velocity u_mid
every ``every`` steps, through ``lb_step`` and ``lb_observe``. The stopping
time at a threshold q is the first recorded t - t_startup with
u_mid(t) <= q u_mid(t_startup); with a finite Maxwell time the decay is
eventually exponential (Sec. III.C), so the time is reported at several
thresholds.
"""
import numpy as np


def startup_cessation(solver, startup, cessation_cap, every=1000, thresholds=(1e-2, 1e-3, 1e-4),
                      stop_fraction=None, channels=None, at_switch_off=None):
    """Runs ``startup`` steps with the force on, then up to ``cessation_cap``
    steps with it off (every channel of the solver must have
    t_startup == startup and start at t = 0). Cessation ends early once every
    listed channel has u_mid <= stop_fraction u_mid(startup) (default: the
    smallest threshold). Returns, per channel, the u_mid history (steps,
    values), u_mid at the switch-off and the stopping time at each threshold
    (None if not reached). ``at_switch_off(solver)`` is called once the
    start-up steps are done, before the first cessation step."""
    chans = list(range(len(solver.channels))) if channels is None else list(channels)
    for c in chans:
        if solver.channels[c].t_startup != startup:
            raise ValueError(f"channel {c} switches its force off at {solver.channels[c].t_startup}, not {startup}")
    if startup % every or cessation_cap % every:
        raise ValueError("startup and cessation_cap must be multiples of every")
    stop_fraction = min(thresholds) if stop_fraction is None else stop_fraction
    t_hist, u_hist = [0], [[solver.observe(c, "umid") for c in chans]]
    for t in range(every, startup + 1, every):
        solver.step(every)
        t_hist.append(t)
        u_hist.append([solver.observe(c, "umid") for c in chans])
    u_s = np.array(u_hist[-1])
    if at_switch_off is not None:
        at_switch_off(solver)
    for t in range(startup + every, startup + cessation_cap + 1, every):
        solver.step(every)
        t_hist.append(t)
        u = np.array([solver.observe(c, "umid") for c in chans])
        u_hist.append(list(u))
        if np.all(u <= stop_fraction * u_s):
            break
    t_arr, u_arr = np.array(t_hist), np.array(u_hist)
    out = []
    for j, c in enumerate(chans):
        after = t_arr >= startup
        stop = {}
        for q in thresholds:
            hit = np.nonzero(after & (u_arr[:, j] <= q * u_s[j]))[0]
            stop[q] = int(t_arr[hit[0]] - startup) if hit.size else None
        out.append({"channel": c, "t": t_arr, "umid": u_arr[:, j], "umid_startup": float(u_s[j]), "t_stop": stop})
    return out
