"""Host logic of the BF16 launch planner (no GPU): wave counting over XCD
ranges and the main + thin-tail split, on synthetic full-wave times with
plans worked out by hand.

The planner costs a launch of T tiles of a shape as waves(T) x the shape's
full-wave time, where a ranged shape deals ceil(T / 8) tiles to each XCD and
runs grid / 8 workgroups there; a split adds a fixed 0.004 ms launch gap."""
import pytest

from paper_2404_14691_amd import sage as S

WAVES = {"ggemm6p_bf16_256x256": 0.100, "ggemm3t_bf16_32x32": 0.020}
BENCH_ROWS = [1105, 1004, 1008, 955]  # the sharing workload's four groups


def test_ragged_groups_split_off_the_one_small_tail():
    # unsplit: 17 row tiles x 16 = 272 tiles -> 34 per XCD range over 32
    # workgroups -> 2 waves = 0.200 ms.  Moving the 81-row tail of group 0
    # leaves 256 tiles (1 wave, 0.100) and adds 3 x 128 = 384 thin tiles
    # (48 per range over 64 workgroups: 1 wave, 0.020) + 0.004 = 0.124 ms;
    # moving the next tail too (187 rows) makes the thin launch 3 waves.
    plan, cost = S.sage_selftest_plan(4096, BENCH_ROWS, WAVES)
    assert plan == "ggemm6p_bf16_256x256:256+ggemm3t_bf16_32x32:384"
    assert cost == pytest.approx(0.124)


def test_full_wave_needs_no_split():
    plan, cost = S.sage_selftest_plan(4096, [1024] * 4, WAVES)
    assert plan == "ggemm6p_bf16_256x256:256"
    assert cost == pytest.approx(0.100)


def test_a_few_rows_take_the_thin_shape_alone():
    # 16 rows: the large tile is one 0.100 wave, the thin one 128 tiles in
    # one 0.020 wave; a "split" moving everything would add the launch gap
    plan, cost = S.sage_selftest_plan(4096, [16], WAVES)
    assert plan == "ggemm3t_bf16_32x32:128"
    assert cost == pytest.approx(0.020)


def test_no_split_when_the_large_tiles_fit_one_wave():
    # 8 groups of 255 rows: 8 x 16 = 128 large tiles, one 0.100 wave.  The
    # thin shape alone needs 8 x 8 x 128 = 8192 tiles (1024 per range over
    # 64: 16 waves, 0.320); moving tails only adds thin waves.
    plan, cost = S.sage_selftest_plan(4096, [255] * 8, WAVES)
    assert plan == "ggemm6p_bf16_256x256:128"
    assert cost == pytest.approx(0.100)
    # with a thin full wave of 0.001 ms the thin shape alone wins (0.016)
    plan, cost = S.sage_selftest_plan(4096, [255] * 8, {**WAVES, "ggemm3t_bf16_32x32": 0.001})
    assert plan == "ggemm3t_bf16_32x32:8192"
    assert cost == pytest.approx(0.016)


def test_wave_count_follows_xcd_ranges():
    # 2 x 2100 rows: 2 x 9 x 16 = 288 tiles -> 36 per range over 32: 2 waves
    # unsplit.  Tails of 52 rows each: moving one leaves 272 (34 per range, 2
    # waves); moving both leaves 256 (1 wave) + 2 x 2 x 128 = 512 thin tiles
    # (64 per range: 1 wave) -> 0.124
    plan, cost = S.sage_selftest_plan(4096, [2100, 2100], WAVES)
    assert plan == "ggemm6p_bf16_256x256:256+ggemm3t_bf16_32x32:512"
    assert cost == pytest.approx(0.124)


def test_shapes_not_listed_or_not_fitting_are_skipped():
    # width 128: the 256-wide tile does not fit; only the thin shape remains
    plan, _ = S.sage_selftest_plan(128, [40], WAVES)
    assert plan == "ggemm3t_bf16_32x32:8"
    with pytest.raises(S.SageError):
        S.sage_selftest_plan(4096, [40], {})
    with pytest.raises(S.SageError):
        S.sage_selftest_plan(4096, [40], {"no_such_shape": 1.0})
