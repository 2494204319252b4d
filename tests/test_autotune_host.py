"""Host logic of the launch autotuner (no device): the geometries it tries."""
from paper_2301_13601_amd import autotune


def test_two_step_candidates_are_single_pairs():
    c2 = autotune.candidates(152, 4096, steps_per_pass=2)
    assert c2 and all(c["waves_per_block"] == 1 and c["steps_per_pass"] == 2 for c in c2)
    c1 = autotune.candidates(152, 4096, steps_per_pass=1)
    assert {c["waves_per_block"] for c in c1} == {1, 2}


def test_candidate_segments_are_multiples_of_four_within_the_lattice():
    for spp in (1, 2):
        for default, ny in [(152, 4096), (512, 2048), (16, 16)]:
            for c in autotune.candidates(default, ny, steps_per_pass=spp):
                assert c["seg_rows"] % 4 == 0
                assert 8 <= c["seg_rows"] <= max(8, ny + 3) or c["seg_rows"] == default
    # one candidate replays no graph (every launch on its own)
    assert any(c["graph_steps"] == 1 for c in autotune.candidates(152, 4096, 2))
