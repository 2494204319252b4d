"""Host-side logic of the surrogate (no GPU): how many lattices one
inference chunk takes."""
from paper_2301_13601_amd import surrogate as S

LIMIT = 2 ** 31     # the kernels index elements with 31-bit offsets


def test_widest_tensor_is_the_upsampled_level_one_output():
    assert S.widest_per_pixel() == 64


def test_default_chunk_stays_under_the_offset_limit():
    for side, want in ((256, 16), (1024, 16), (1536, 14), (2048, 7), (4096, 1), (8192, 1), (16384, 1)):
        c = S.default_chunk(side, side)
        assert c == want, (side, c)
        if c * side * side * 64 >= LIMIT:
            assert c == 1     # one lattice at least, even where that one alone does not fit
            continue
        # every tensor a layer reads or writes at its own level fits
        assert c * side * side * S.IN_CH < LIMIT
        for s in S.layer_specs():
            px = c * (side >> s.level) * (side >> s.level)
            assert px * max(s.c_in, s.c_out) < LIMIT, (side, s.name)
        assert c * side * side * S.OUT_LD < LIMIT
