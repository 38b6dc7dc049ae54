"""Tile autotuner: picks the rows per wavefront strip of the sweep.

For a set of channels and a precision it times each candidate on a throwaway
handle (so the caller's state is untouched) with HIP events on the handle's
stream, keeps the fastest, and caches the choice in a JSON file keyed by the
device name, the precision and the shape of the batch (the width classes,
the node count and the row-count range).

For a batch run to steady state (``to_steady``) the time per step of the
whole batch alone is the wrong target. A channel relaxes over ~H^2/nu steps,
so the widest channels converge last and spend much of the run alone: with
widths spread evenly, about half the run has at most a quarter of the
channels active. The objective is then the mean time per step of the whole
batch, of its widest half and of its widest eighth.
"""
import json
import os
import sys
from typing import Iterable, Optional, Sequence

from .lbnlm import ChannelSpec, Solver

# 0: the library's own heights (for the narrow widths' two-step strips,
# chosen from the number of active channels)
DEFAULT_CANDIDATES = (0, 4, 8, 16, 24, 32, 64)
DEFAULT_CACHE = os.path.join(os.path.expanduser("~"), ".cache", "lbnlm_autotune.json")


def shape_key(channels: Sequence[ChannelSpec], precision: str) -> str:
    import torch
    nodes = sum(c.nx * c.ny for c in channels)
    widths = sorted({c.nx for c in channels})
    nys = [c.ny for c in channels]
    dev = torch.cuda.get_device_name(0)
    # node count rounded to two significant digits
    mag = 10 ** max(len(str(nodes)) - 2, 0)
    return f"{dev}|{precision}|nx={widths[:8]}|nodes~{round(nodes / mag) * mag}|ny={min(nys)}-{max(nys)}"


def time_candidate(channels, precision, strip_rows, steps, nn_pressure=True):
    import torch
    with Solver(channels, precision=precision, obs_every=max(2, (steps // 2) // 2 * 2),
                strip_rows=strip_rows, nn_pressure=nn_pressure) as s:
        s.step(s.opts.obs_every)  # captures the graph and warms the caches
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(s.stream)
        s.step(steps)
        e1.record(s.stream)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / steps


def widest(channels, fraction):
    """The widest ceil(fraction * n) channels (at least one)."""
    order = sorted(channels, key=lambda c: c.ny, reverse=True)
    return order[:max(1, int(-(-len(order) * fraction // 1)))]


def tune_strip_rows(channels: Sequence[ChannelSpec], precision: str = "fp32",
                    candidates: Iterable[int] = DEFAULT_CANDIDATES, steps: int = 200,
                    cache_path: Optional[str] = DEFAULT_CACHE, nn_pressure: bool = True,
                    verbose: bool = False, to_steady: bool = False) -> int:
    """Returns the fastest rows-per-strip for these channels (cached); with
    to_steady, fastest for a run of the batch to steady state."""
    key = shape_key(channels, precision) + ("|to_steady" if to_steady else "")
    cache = {}
    if cache_path and os.path.exists(cache_path):
        try:
            cache = json.load(open(cache_path))
        except (OSError, ValueError):
            cache = {}
    if key in cache:
        return int(cache[key]["strip_rows"])
    times = {}
    for sr in candidates:
        if to_steady:
            times[sr] = (time_candidate(channels, precision, sr, steps, nn_pressure) +
                         time_candidate(widest(channels, 0.5), precision, sr, steps, nn_pressure) +
                         time_candidate(widest(channels, 0.125), precision, sr, steps, nn_pressure)) / 3
        else:
            times[sr] = time_candidate(channels, precision, sr, steps, nn_pressure)
        if verbose:
            print(f"autotune {key}: strip_rows={sr} {times[sr] * 1e3:.1f} us/step", file=sys.stderr, flush=True)
    best = min(times, key=times.get)
    cache[key] = {"strip_rows": best, "ms_per_step": times}
    if cache_path:
        try:
            os.makedirs(os.path.dirname(cache_path), exist_ok=True)
            tmp = cache_path + ".tmp"
            json.dump(cache, open(tmp, "w"), indent=1)
            os.replace(tmp, cache_path)
        except OSError:
            pass
    return best
