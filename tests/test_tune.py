"""Host logic of the tile-size / rank-cap autotuner (paper_1804_09137_amd/tune.py)."""
from paper_1804_09137_amd import tune as T


def test_candidates_are_valid_tile_sizes():
    c = T.candidates(102400)
    assert (800, 200) in c and (1024, 341) in c
    for nb, mr in c:
        assert nb % 16 == 0 and 32 <= nb <= 1024 and (102400 + nb - 1) // nb >= 4
        assert mr in (nb // 4, nb // 3)
    # few points: only tiles that still give 4 columns, else one fallback
    assert all((1500 + nb - 1) // nb >= 4 for nb, _ in T.candidates(1500))
    assert T.candidates(100) == [(32, 8)]


def test_choose_smallest_time_then_smaller_tile():
    assert T.choose({(800, 200): 5.0, (640, 160): 4.0, (1024, 256): 4.5}) == (640, 160)
    assert T.choose({(800, 200): 4.0, (640, 213): 4.0}) == (640, 213)
