"""Host logic of the tuner: the choice rule of its coordinate descent."""
from paper_2002_05026_amd import tune


def test_pick_keeps_the_current_value_within_the_noise_margin():
    # 12 is 0.1% faster than the current 8: noise, 8 stays
    assert tune._pick({4: 100.0, 8: 99.7, 12: 99.6}, 8) == 8
    # 4 is 10% faster: it replaces the current value
    assert tune._pick({4: 90.0, 8: 100.0, 12: 101.0}, 8) == 4
    # exactly at the margin is not enough
    assert tune._pick({4: 100.0 * (1 - tune.MARGIN), 8: 100.0}, 8) == 8
    # a current value that was not timed: the fastest
    assert tune._pick({64: 3.0, 96: 2.0}, 128) == 96
