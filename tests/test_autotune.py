"""Host-side checks of the schedule autotuner's search space."""
from paper_2211_12265_amd import autotune


def test_candidates_cover_speculation_range():
    for level, g in ((2, 16), (3, 12), (5, 9)):
        for waves in (1, 2, 4):
            assert autotune.slots_per_batch(level, waves) == waves * g
            c = autotune.candidates(level, 10000, 2048, waves)
            hm = {h for h, _ in c}
            assert 1 in hm and waves * g in hm and max(hm) == waves * g
            for h, grid in c:
                assert 1 <= grid <= 2048
                assert grid <= -(-10000 // h)


def test_candidates_small_batch():
    for waves in (1, 2, 4):
        c = autotune.candidates(2, 5, 2048, waves)
        assert all(grid <= 5 for _, grid in c)
        assert len(set(c)) == len(c)
