"""The autotuner times every candidate launch configuration of the ADR step
(two steps per launch or one, kernel variant, tile shape, cache policy) on
the lattice at hand, returns the fastest and caches it by lattice shape."""
import json

import numpy as np
import pytest

from workloads import make_workload

pytestmark = pytest.mark.gpu


def test_autotune_picks_a_candidate_and_caches_it(tmp_path):
    from paper_2109_04455_amd.autotune import DEFAULT_CANDIDATES, autotune
    w = make_workload("C1q")
    cache = tmp_path / "tune.json"
    best = autotune(w.node_type, w.k, real="f32", nspecies=3, tau_g=w.tau_g,
                    vel_scale=w.vel_scale, steps=40, cache_path=str(cache))
    assert tuple(best) in DEFAULT_CANDIDATES
    d = json.loads(cache.read_text())
    (key, entry), = d.items()
    assert tuple(entry["best"]) == tuple(best)
    timings = entry["timings_us"]
    assert len(timings) == len(DEFAULT_CANDIDATES)
    assert all(np.isfinite(v) and v > 0 for v in timings.values())
    assert timings[str(tuple(best))] == min(timings.values())
    # a second call answers from the cache
    assert tuple(autotune(w.node_type, w.k, real="f32", nspecies=3, tau_g=w.tau_g,
                          vel_scale=w.vel_scale, steps=40, cache_path=str(cache))) == tuple(best)
