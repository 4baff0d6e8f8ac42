"""Host rules of the schedule autotuner (no GPU): padded widths, the compiled
schedule candidates of a kernel class and which schedules store the runs'
within-tile carries in their pre-pass (the library's rule: d <= 2, at least 2
columns per wave, runs of 8 to 32, at any width)."""
from paper_2508_01864_amd import autotune


def test_product_width_pads_to_the_column_block():
    assert [autotune.rhs_block(n) for n in (1, 2, 3, 4, 31, 32, 100)] == [1, 2, 2, 4, 4, 32, 32]
    assert [autotune.product_width(n) for n in (1, 2, 3, 5, 31, 32, 33)] == [1, 2, 4, 8, 32, 32, 64]


def test_run_carries_rule():
    assert autotune.stores_run_carries(2, 32, 16, 32, 1)       # the headline schedule
    assert autotune.stores_run_carries(2, 256, 16, 32, True)   # any width
    assert autotune.stores_run_carries(1, 4, 4, 16, 1)
    assert not autotune.stores_run_carries(2, 32, 16, 32, 0)   # declined by the schedule
    assert not autotune.stores_run_carries(3, 32, 16, 32, 1)   # d = 3: no room
    assert not autotune.stores_run_carries(2, 32, 32, 64, 1)   # runs longer than 32
    assert not autotune.stores_run_carries(2, 4, 1, 8, 1)      # one column per wave
    assert not autotune.stores_run_carries(2, 4, 4, 4, 1)      # runs of 4 keep their sums apart


def test_candidates_at_32_columns():
    c = autotune.schedule_candidates(2, 3, "product", 32)
    # the tuned d = 2, nu = 3/2 class offers both variants where run carries can be stored
    assert (16, 32, 1) in c and (16, 32, 0) in c
    assert (8, 32, 1) in c and (8, 32, 0) in c
    assert (32, 128, 1) in c and (32, 128, 0) not in c
    assert len(c) == len(set(c))
    # every candidate's column block divides the width
    assert all(32 % wb == 0 for wb, _, _ in c)


def test_candidates_by_class():
    # untuned classes get the base schedules only
    base = {(wb, e) for wb, e, _ in autotune.schedule_candidates(2, 1, "product", 32)}
    assert base == {(wb, e) for wb, e in autotune.BASE_SCHEDULES if 32 % wb == 0}
    # d = 3 never stores run carries
    assert all(rx == 1 for _, _, rx in autotune.schedule_candidates(3, 5, "product", 32))
    # width 4: blocks that do not divide it are left out
    c4 = autotune.schedule_candidates(2, 3, "product", 4)
    assert all(4 % wb == 0 for wb, _, _ in c4)
    assert (4, 16, 1) in c4 and (4, 16, 0) in c4 and (1, 4, 1) in c4
