import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) and the built HIP library")
    config.addinivalue_line("markers", "slow: CPU test that takes more than a few seconds")


def _assert_same(got, want, what="results"):
    """Entry-by-entry equality of two result lists with a short message: a
    failed whole-list comparison of large integers makes pytest build a diff
    of the full lists, which takes minutes."""
    assert len(got) == len(want), f"{what}: {len(got)} entries, expected {len(want)}"
    bad = [i for i, (a, b) in enumerate(zip(got, want)) if a != b]
    assert not bad, f"{what}: {len(bad)} of {len(got)} entries differ, the first at index {bad[0]}"


@pytest.fixture
def assert_same():
    return _assert_same
