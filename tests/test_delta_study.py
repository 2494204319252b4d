"""The perturbation-parameter study harness: its scene is the 256 x 256 run
at delta = 0.3 (CPU), and a short run of the study logs what it promises
(GPU)."""
import numpy as np
import pytest

from paper_2301_13601_amd import delta_study, scenes


def test_scene_at_coarsest_delta_is_the_single_run():
    n, q = delta_study.scene(0.3, "Ez")
    sc = scenes.config_single()
    np.testing.assert_allclose(n, sc.n.astype(np.float32), rtol=0, atol=2e-6)
    np.testing.assert_allclose(q, sc.q.astype(np.float32), rtol=0, atol=2e-6)


def test_scene_scales_with_delta():
    n3, _ = delta_study.scene(0.3, "Ez")
    n1, _ = delta_study.scene(0.1, "Ez")
    assert n1.shape == (3, 768, 768)
    # the same physical points carry the same index
    np.testing.assert_allclose(n1[:, ::3, ::3], n3, rtol=0, atol=2e-5)


@pytest.mark.gpu
def test_short_study_runs_and_skew_conserves_energy():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    recs = delta_study.study(deltas=(0.3, 0.1), modes=("eq28",), pols=("Ez", "Ey"), forms=("printed", "skew"),
                             t_end=4.5, logs=2)
    assert len(recs) == 8
    for r in recs:
        assert len(r["log"]) == 2 and r["steps"] == round(4.5 / r["delta"] ** 2)
        key = "divB_ratio" if r["polarisation"] == "Ez" else "divD_ratio"
        assert all(key in e for e in r["log"])
        if r["v_form"] == "skew":
            assert abs(r["log"][-1]["energy_rel"]) < 1e-5
