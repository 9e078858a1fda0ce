"""GPU tests of the serving loop: requests of different kinds and sizes
submitted while others run are all answered, and each answer is identical
to the same request computed alone (tolerance 0) and to the oracle on the
small ones."""
import random

import numpy as np
import pytest

import synth
from oracle import gcd as G
from oracle import resultant as R
from oracle import zx

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def snc():
    import paper_1103_4697_amd as m
    return m


def mix(n, seed):
    rng = np.random.default_rng(seed)
    reqs = []
    for i in range(n):
        if i % 5 == 4:
            a, b, _ = synth.gcd_request(rng, 40, 200, 3, 12, 8, 24)
            reqs.append(("gcd", a, b))
        else:
            df, dg = int(rng.integers(3, 14)), int(rng.integers(3, 14))
            f, g = synth.random_pair(rng, df, dg, int(rng.integers(8, 40)), int(rng.integers(8, 40)))
            reqs.append(("res", f, g))
    return reqs


def test_mix_equals_alone_and_oracle(snc):
    reqs = mix(40, 11)
    srv = snc.Server(pool_bytes=256 << 20, max_slots=16, nstreams=3)
    tickets = []
    for kind, x, y in reqs:
        tickets.append(srv.submit_resultant(x, y) if kind == "res" else srv.submit_gcd(x, y))
    assert srv.wait(len(reqs), 60.0)
    got = [srv.poll(t) for t in tickets]
    for t in tickets:
        s, d = srv.times(t)
        assert d >= s
    srv.close()
    for (kind, x, y), r in zip(reqs, got):
        alone = snc.resultant_y(x, y) if kind == "res" else snc.gcd_z(x, y)
        assert r == alone
    # oracle on every gcd and on the small resultants
    for (kind, x, y), r in zip(reqs, got):
        if kind == "gcd":
            assert G.certify_gcd(x, y, r)
        elif R.degree_bound(x, y) <= 80:
            assert r == R.resultant_y_by_points(x, y)


def test_arrivals_while_running_and_small_pool(snc):
    # a pool that holds only a few requests at a time forces admission waits
    reqs = mix(24, 12)
    alone = [snc.resultant_y(x, y) if k == "res" else snc.gcd_z(x, y) for k, x, y in reqs]
    srv = snc.Server(pool_bytes=4 << 20, max_slots=4, nstreams=2)
    tickets = []
    rng = random.Random(3)
    import time
    for k, x, y in reqs:
        tickets.append(srv.submit_resultant(x, y) if k == "res" else srv.submit_gcd(x, y))
        time.sleep(rng.random() * 0.002)
    assert srv.wait(len(reqs), 60.0)
    assert [srv.poll(t) for t in tickets] == alone
    srv.close()


def test_oversized_request_refused(snc):
    srv = snc.Server(pool_bytes=1 << 16, max_slots=2, nstreams=1)
    f, g = synth.config1()
    with pytest.raises(snc.SncError):
        srv.submit_resultant(f, g)
    srv.close()


def test_pool_just_above_one_request(snc):
    """A pool a little larger than one request's own workspace (less than
    the headroom a joint batch reserves): the request is admitted alone and
    finishes, requests behind it follow one at a time, and a request larger
    than the pool is refused at submission -- nothing waits forever."""
    rng = np.random.default_rng(21)
    f, g = synth.random_pair(rng, 8, 7, 16, 16)
    need = snc.resultant_plan(f, g).workspace_bytes
    pool = (need + 255) // 256 * 256 + 1024
    srv = snc.Server(pool_bytes=pool, max_slots=4, nstreams=2)
    t = [srv.submit_resultant(f, g) for _ in range(3)]
    assert srv.wait(3, 30.0)
    want = snc.resultant_y(f, g)
    assert all(srv.poll(x) == want for x in t)
    big = synth.random_pair(rng, 20, 20, 32, 32)
    with pytest.raises(snc.SncError):
        srv.submit_resultant(*big)
    srv.close()
