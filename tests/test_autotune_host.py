"""Host-side parts of the autotuner (no GPU): workload signatures and the
candidate set."""
import numpy as np

from paper_2302_14801_amd import autotune


def test_signature_classes():
    a = autotune.signature([0, 1_000_000, 2_100_000, 3_000_000], 0)
    b = autotune.signature([0, 1_050_000, 2_000_000, 3_050_000], 0)
    assert a == b                      # same class: same count, similar sizes
    assert a != autotune.signature([0, 1_000_000, 2_100_000, 3_000_000], 1)
    assert autotune.signature([0, 0, 0], 0) == "empty/s0"
    # empty chunks are ignored
    assert autotune.signature([0, 10, 10, 20], 0) == autotune.signature([0, 10, 20], 0)


def test_candidates_are_valid_plans():
    assert (0, 0, 0) in autotune.CANDIDATES
    for e0, e1, ch in autotune.CANDIDATES:
        assert 0 <= e0 <= 4 and 0 <= e1 <= 4 and ch >= 0
    assert len(set(autotune.CANDIDATES)) == len(autotune.CANDIDATES)
