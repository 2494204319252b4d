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


def test_two_step_candidates_try_both_cache_policies():
    c2 = autotune.candidates(152, 4096, steps_per_pass=2)
    assert {c["stream_loads"] for c in c2} == {1, 2}
    segs = {c["seg_rows"] for c in c2 if c["graph_steps"] == 32}
    for s in segs:
        assert {c["stream_loads"] for c in c2 if c["seg_rows"] == s and c["graph_steps"] == 32} == {1, 2}
    assert all(c["stream_loads"] == 2 for c in autotune.candidates(152, 4096, steps_per_pass=1))
