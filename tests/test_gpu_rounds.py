"""Round counts of every primitive the library exposes, read from its
counters, against the paper's table of round complexities
(tests/golden/table1_rounds.json).  Addition, XOR and shifts are local and
have no library call."""
import json
import math
import os

import numpy as np
import pytest

import workloads
from tests.gpu_util import dev, say

pytestmark = pytest.mark.gpu

T1 = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "table1_rounds.json")))


@pytest.fixture(scope="module")
def m():
    import paper_2109_00984_amd as mod
    return mod


@pytest.fixture(scope="module")
def ctx(m):
    c = m.Context(device=0, seed=5)
    yield c
    c.close()


def rounds(ctx, call):
    before = ctx.stats()["opens"]
    call()
    ctx.sync()
    return ctx.stats()["opens"] - before


def test_arithmetic_two_parties(m, ctx):
    say("rounds: two-party arithmetic")
    n = 64
    x = ctx.share(dev(workloads.uniform_u64(1, (8, 8))), 0, 1)
    tm = ctx.dealer(m.TRIPLE_MUL, 1, 2, (n,))
    ts = ctx.dealer(m.TRIPLE_SQUARE, 1, 3, (n,))
    tmm = ctx.dealer(m.TRIPLE_MATMUL, 1, 4, (8, 8, 8))
    flat = m.SharedPair(x.s0.view(-1), x.s1.view(-1))
    mult = T1["arithmetic"]["multiplication"]
    assert rounds(ctx, lambda: ctx.beaver_mul(flat, flat, tm, 16)) == mult
    assert rounds(ctx, lambda: ctx.beaver_mul(flat, None, ts, 16)) == mult
    assert rounds(ctx, lambda: ctx.beaver_matmul(x, x, tmm, 16)) == mult
    assert rounds(ctx, lambda: ctx.truncate(x, 16)) == T1["arithmetic"]["truncation_two_parties"]
    assert rounds(ctx, lambda: ctx.reveal(x)) == 1  # each party sends its share once


def test_binary_and_conversions(m, ctx):
    say("rounds: binary sharing and conversions")
    n = 64
    x = dev(np.arange(n, dtype=np.uint64))
    b = ctx.bin_share(x, 0, 1)
    t = ctx.dealer_and(2, 1, ctx.A2B_TRIPLES * n)
    assert rounds(ctx, lambda: ctx.bin_and(b, b, t)) == T1["binary"]["and"]
    rb, ra = ctx.dealer_b2a(2, 2, n)
    assert rounds(ctx, lambda: ctx.b2a_bit(b, 5, rb, ra)) == T1["conversions"]["b2a"]
    # log2(P) * log2(L) doubling levels of the adder, plus the round of its
    # generate bits (a AND b) that the levels start from
    a2b = int(math.log2(2) * math.log2(T1["ring_bits"])) + 1
    assert rounds(ctx, lambda: ctx.a2b(ctx.share(x, 0, 2), 3, t)) == a2b


def test_arithmetic_three_parties(m, ctx):
    say("rounds: three-party arithmetic")
    n = 64
    s = ctx.mp_share(dev(np.arange(n, dtype=np.uint64)), 3, 0, 1)
    t = ctx.mp_dealer(3, m.TRIPLE_MUL, 3, 1, (n,))
    assert rounds(ctx, lambda: ctx.mp_beaver_mul(s, s, t)) == T1["arithmetic"]["multiplication"]
    r, th = ctx.mp_dealer_trunc(3, 3, 2, n)
    assert rounds(ctx, lambda: ctx.mp_truncate(s, 16, r, th)) == T1["arithmetic"]["truncation"]
