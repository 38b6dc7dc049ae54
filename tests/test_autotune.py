"""The strip-height autotuner: the channel subsets its steady-state objective
times (CPU), and a tuning run with its cache (GPU)."""
import json

import pytest

from paper_1310_7450_amd import autotune, workloads
from paper_1310_7450_amd.lbnlm import ChannelSpec


def test_widest_subsets():
    """widest(f) keeps the ceil(f n) channels of largest ny, at least one."""
    chans = workloads.batched_sweep()["channels"]
    half, eighth = autotune.widest(chans, 0.5), autotune.widest(chans, 0.125)
    assert len(half) == 128 and len(eighth) == 32
    nys = sorted((c.ny for c in chans), reverse=True)
    assert sorted((c.ny for c in eighth), reverse=True) == nys[:32]
    assert min(c.ny for c in half) >= max(c.ny for c in chans if c not in half)
    assert len(autotune.widest(chans[:3], 0.125)) == 1


@pytest.mark.gpu
def test_tune_returns_a_candidate_and_caches(tmp_path):
    """A tuning run returns one of the candidates, stores it under the
    batch's key (with the steady-state objective marked), and a second call
    reads the cache."""
    chans = [ChannelSpec(nx=8, ny=ny, force=1e-6, tau_lb=1.0, G=1e-4, tau0=1e3, gamma_c=0.1)
             for ny in (32, 64, 128, 256)]
    cache = tmp_path / "tune.json"
    sr = autotune.tune_strip_rows(chans, "fp32", candidates=(8, 16), steps=20, cache_path=str(cache),
                                  to_steady=True)
    assert sr in (8, 16)
    rec = json.loads(cache.read_text())
    (key, val), = rec.items()
    assert key.endswith("|to_steady") and val["strip_rows"] == sr and set(val["ms_per_step"]) == {"8", "16"}
    val["strip_rows"] = 24  # a cached choice is returned without timing
    cache.write_text(json.dumps({key: val}))
    assert autotune.tune_strip_rows(chans, "fp32", candidates=(8, 16), steps=20, cache_path=str(cache),
                                    to_steady=True) == 24
