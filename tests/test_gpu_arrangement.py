"""GPU parity of the arrangement batches (the projection phase of a set of
curves: contents in y, then res_y(p, p_y) of every primitive part and
res_y(p_i, p_j) of every pair) through the C ABI.

Exact integers, bit-identical comparisons:
* contents of many curves in one tree of batched gcds against the oracle's
  fold of exact gcds (random curves, circles, ellipses, graphs of rational
  functions, planted factors in x, one-row, integer-only and zero curves);
* every resultant of a 20-curve mixed set against the single-pair entry
  point on the oracle's primitive parts, exactly against the oracle's
  Sylvester determinant for the conics, and modulo a 61-bit prime at random
  points against the oracle's determinant for a sample of the rest;
* a 50-curve set of circles and ellipses (1275 resultants) exactly against
  the oracle.
"""
import random

import numpy as np
import pytest

import synth
from oracle import fastlift as FL
from oracle import gcd as G
from oracle import resultant as R
from oracle import zx

pytestmark = pytest.mark.gpu
Q61 = (1 << 61) - 1


@pytest.fixture(scope="module")
def snc():
    import paper_1103_4697_amd as m
    return m


def primitive_y(f, h):
    """f / h row by row (exact in Z[x]), trailing zero rows dropped."""
    if not h:
        return []
    rows = [zx.divexact(zx.trim(list(r)), h) if any(r) else [] for r in f]
    while rows and not rows[-1]:
        rows.pop()
    return rows


def as_rows(f):
    """Rows padded to a rectangle of Python ints (zero polynomial: [[0]])."""
    if not f:
        return [[0]]
    w = max(max(len(r), 1) for r in f)
    return [list(r) + [0] * (w - len(r)) for r in f]


def arrangement_pairs(prims):
    n = len(prims)
    pairs = [(p, FL.partial_y(p)) for p in prims]
    pairs += [(prims[i], prims[j]) for i in range(n) for j in range(i + 1, n)]
    return pairs


def test_content_batch_matches_oracle(snc):
    curves = synth.arrangement_set(np.random.default_rng(9101), 24)
    curves += [
        [[0]],                              # f = 0: content 0
        [[-3, 0, 3]],                       # one row: the row itself
        [[6, 4], [2]],                      # integer content only
        [[0, 0, 5], [0, 0, 0], [0, 0, -10]],  # content 5 x^2 with a zero row
        synth.bigcoef_curve(np.random.default_rng(9102), 6, 200)[0],  # multi-word, content 1
    ]
    got = snc.content_y_batch(curves)
    want = [G.content_y(f) for f in curves]
    assert got == want
    assert any(len(h) > 1 for h in want)    # planted factors in x were found


def test_arrangement_matches_single_calls_and_oracle(snc):
    curves = synth.arrangement_set(np.random.default_rng(9103), 20)
    A = snc.Arrangement(curves)
    A.run()
    conts, res = A.contents(), A.resultants()
    assert conts == [G.content_y(f) for f in curves]
    prims = [primitive_y(f, h) for f, h in zip(curves, conts)]
    pairs = arrangement_pairs(prims)
    assert len(res) == len(pairs) == 20 + 20 * 19 // 2
    for (a, b), r in zip(pairs, res):
        assert r == snc.resultant_y(as_rows(a), as_rows(b))
    rng = random.Random(9104)
    small = [i for i, (a, b) in enumerate(pairs) if len(a) <= 3 and len(b) <= 3]
    assert len(small) > 20
    for i in small:
        a, b = pairs[i]
        assert res[i] == R.resultant_y(as_rows(a), as_rows(b))
    for i in rng.sample(range(len(pairs)), 30):
        a, b = pairs[i]
        x0 = rng.randrange(Q61)
        assert zx.evaluate(res[i], x0) % Q61 == R.resultant_at_mod(as_rows(a), as_rows(b), x0, Q61)
    for _ in range(2):  # replays of the prepared batch
        A.run()
        assert A.resultants() == res
    A.close()


def test_arrangement_fifty_conics_exact(snc):
    curves = synth.arrangement_set(np.random.default_rng(9105), 50, kinds=("circle", "ellipse"))
    A = snc.Arrangement(curves)
    A.run()
    conts = A.contents()
    assert conts == [G.content_y(f) for f in curves]
    assert all(len(h) == 1 for h in conts)        # conics: integer contents only
    res = A.resultants()
    pairs = arrangement_pairs([primitive_y(f, h) for f, h in zip(curves, conts)])
    assert len(res) == 50 + 1225
    for (a, b), r in zip(pairs, res):
        assert r == R.resultant_y(a, b)
    A.close()
