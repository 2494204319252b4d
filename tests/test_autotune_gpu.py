"""The launch-geometry autotuner: it measures, caches, and what it picks
changes nothing in the results."""
import numpy as np
import pytest

from paper_2301_13601_amd import scenes

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def qla():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2301_13601_amd import qla as q
    q.lib()
    return q


def test_autotune_measures_caches_and_keeps_results(qla, tmp_path):
    from paper_2301_13601_amd import autotune

    n = scenes.object_profile(600, 300, "disk", (60,), (1.5, 2.0, 2.5), 6.0).astype(np.float32)
    q = scenes.random_state(600, 300, 3).astype(np.float32)
    cache = str(tmp_path / "tune.json")
    rec = autotune.tune([n], [0.3], cache_path=cache, steps=16)
    assert not rec["cached"] and len(rec["measured"]) >= 3
    assert rec["us_per_step"] == min(m["us_per_step"] for m in rec["measured"])
    again = autotune.tune([n], [0.3], cache_path=cache, steps=16)
    assert again["cached"] and again["launch"] == rec["launch"]

    ref = qla.Simulation(n, q, 0.3)
    ref.step(10)
    tuned = qla.Simulation(n, q, 0.3)
    autotune.apply(tuned, [n], [0.3], cache_path=cache)
    assert tuned.launch() == rec["launch"]
    tuned.step(10)
    assert np.array_equal(tuned.fields("Q"), ref.fields("Q"))
    ref.close()
    tuned.close()
