"""The allocation-free resultant entry point (snc_resultant_y_noalloc)
against the workspace entry point (snc_resultant_y) through the C ABI,
bit-exact: two calls in a row on the shared scratch array, the second with
a smaller input (the array keeps the first call's contents), a pair over
several register classes and point tiles, trivial results, and the
refusal of a pair whose plan exceeds the fixed array.
"""
import numpy as np
import pytest

import synth
from oracle import resultant as R

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def snc():
    import paper_1103_4697_amd as m
    return m


def test_two_calls_second_smaller(snc):
    rng = np.random.default_rng(7101)
    big = synth.random_pair(rng, 22, 18, 24, 20)      # y-degree 22 (register class 32), 35 primes, D = 396
    small = synth.config0()                             # degree 6/6, 7-bit
    got_big = snc.resultant_y_noalloc(*big)
    got_small = snc.resultant_y_noalloc(*small)
    assert got_big == snc.resultant_y(*big)
    assert got_small == snc.resultant_y(*small)
    assert got_small == R.resultant_y(*small)
    # and again in the other order, with the other entry point in between
    assert snc.resultant_y_noalloc(*small) == got_small
    assert snc.resultant_y_noalloc(*big) == got_big


def test_multilimb_and_classes(snc):
    rng = np.random.default_rng(7102)
    for df, dg, bits in ((40, 33, 32), (3, 12, 16)):
        f, g = synth.random_pair(rng, df, dg, bits, bits)
        assert snc.resultant_y_noalloc(f, g) == snc.resultant_y(f, g), (df, dg, bits)
    f, fy = synth.bigcoef_curve(rng, 9, 100)             # four-limb coefficients
    assert snc.resultant_y_noalloc(f, fy) == snc.resultant_y(f, fy)


def test_trivial_results(snc):
    f = [[3, 1]]          # constant in y
    g = [[2], [5]]        # y-degree 1
    assert snc.resultant_y_noalloc(f, g) == snc.resultant_y(f, g)
    assert snc.resultant_y_noalloc(f, [[7]]) == [1]
    assert snc.resultant_y_noalloc([[0]], g) == []


def test_oversized_refused_then_usable(snc):
    rng = np.random.default_rng(7103)
    f, g = synth.bigcoef_curve(rng, 45, 512)          # 1542 primes, D = 1980: about 75 MiB
    assert snc.resultant_plan(f, g).workspace_bytes > snc.NOALLOC_SCRATCH_BYTES
    with pytest.raises(snc.SncError) as ei:
        snc.resultant_y_noalloc(f, g)
    assert ei.value.status == snc.SNC_ENOMEM
    small = synth.config0()
    assert snc.resultant_y_noalloc(*small) == R.resultant_y(*small)
