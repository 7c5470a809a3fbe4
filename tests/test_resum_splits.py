"""The warm-start network's data splits: training, validation and held-out test problems
come from disjoint seed ranges, and the training step refuses data that mixes them."""
import pytest

from paper_2212_07494_amd import resum


def test_seed_ranges_are_disjoint():
    assert resum._split_of_seed(resum.TRAIN_SEED) == "train"
    assert resum._split_of_seed(resum.VAL_SEED - 1) == "train"
    assert resum._split_of_seed(resum.VAL_SEED) == "val"
    assert resum._split_of_seed(resum.VAL_SEED + resum.VAL_SPAN - 1) == "val"
    assert resum._split_of_seed(resum.VAL_SEED + resum.VAL_SPAN) == "train"
    assert resum._split_of_seed(resum.TEST_SEED - 1) == "train"
    assert resum._split_of_seed(resum.TEST_SEED) == "test"
    assert resum._split_of_seed(resum.TRAIN_SEED - 1) is None
    assert resum.VAL_SEED + resum.VAL_SPAN <= resum.TEST_SEED


def test_clean_rows_pass():
    resum.check_splits([dict(split="train", seed=40_000), dict(split="train", seed=75_000),
                        dict(split="val", seed=60_001), dict(split="train")])


@pytest.mark.parametrize("rows", [
    [dict(split="train", seed=60_005)],                     # a training seed in the val range
    [dict(split="train", seed=80_000)],                     # ... in the test range
    [dict(split="val", seed=45_000)],                       # a validation seed outside it
    [dict(split="train", seed=39_999)],                     # below every range
])
def test_mixed_rows_are_refused(rows):
    with pytest.raises(SystemExit):
        resum.check_splits(rows)
