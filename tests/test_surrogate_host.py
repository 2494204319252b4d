"""Host-side logic of the surrogate (no GPU): how many lattices one
inference chunk takes."""
from paper_2301_13601_amd import surrogate as S


def test_default_chunk_stays_under_the_offset_limit():
    for side, want in ((256, 16), (1024, 16), (2048, 10), (4096, 2), (8192, 1), (16384, 1)):
        c = S.default_chunk(side, side)
        assert c == want, (side, c)
        # the packed input of a chunk fits 31-bit element offsets (one
        # lattice at least, even where that one alone would not)
        assert c == 1 or c * side * side * S.IN_CH < 2 ** 31
