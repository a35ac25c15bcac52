"""GPU parity of the grouped element-wise Beaver product (section 5.2, batched
as in Section 6.1): many products and squares of uneven lengths in one
launch, each bit-identical to the CPU oracle and to one mpc_beaver_mul call
on the same shares and triple."""
import numpy as np
import pytest
import torch

import oracle
import workloads
from tests.gpu_util import dev, pair, say

pytestmark = pytest.mark.gpu

SEED = 4242
CHUNK = 1024
# lengths around the chunk size and tiny ones; (n, square?, offset view?)
CASES = [(1, False, False), (2, True, False), (3, False, True), (CHUNK - 1, False, False),
         (CHUNK, True, True), (CHUNK + 1, False, False), (100003, False, False),
         (5, True, True), (3 * CHUNK + 7, True, False), (65536, False, True)]


@pytest.fixture(scope="module")
def m():
    import paper_2109_00984_amd as mod
    return mod


def make_problem(m, c, i, n, sq, view):
    """Shares and triple of problem i; with `view`, every array is a view one
    element into a larger buffer (8-byte aligned only: the scalar path)."""
    x = workloads.uniform_u64(100 + i, (n,))
    y = workloads.uniform_u64(200 + i, (n,))
    off = 1 if view else 0

    def d(a):
        buf = torch.zeros(n + off, dtype=torch.int64, device=c.device)
        buf[off:] = dev(a)
        return buf[off:]

    xs = oracle.share(x, 0, SEED, 2 * i)
    ys = oracle.share(y, 1, SEED, 2 * i + 1)
    if sq:
        w = oracle.dealer_square(9, 30 + i, n)
        t = m.TripleShares(d(w.a[0]), d(w.a[1]), d(w.b[0]), d(w.b[1]))
        gy = None
    else:
        w = oracle.dealer_mul(9, 30 + i, n)
        t = m.TripleShares(*(d(v) for v in (w.a[0], w.a[1], w.b[0], w.b[1], w.c[0], w.c[1])))
        gy = m.SharedPair(d(ys[0]), d(ys[1]))
    gx = m.SharedPair(d(xs[0]), d(xs[1]))
    out = m.SharedPair(d(np.zeros(n, np.uint64)), d(np.zeros(n, np.uint64)))
    want = oracle.beaver_square(xs, w, 16) if sq else oracle.beaver_mul(xs, ys, w, 16)
    return (gx, gy, t), out, want


def test_grouped_mul_matches_oracle_and_single_calls(m):
    say("grouped beaver mul: mixed products and squares")
    c = m.Context(device=0, seed=SEED)
    probs, outs, wants = [], [], []
    for i, (n, sq, view) in enumerate(CASES):
        p, o, w = make_problem(m, c, i, n, sq, view)
        probs.append(p)
        outs.append(o)
        wants.append(w)
    before = c.stats()
    zs = c.beaver_mul_grouped(probs, 16, outs=outs)
    after = c.stats()
    assert after["launches"] - before["launches"] == 1
    assert after["opens"] - before["opens"] == len(CASES)
    for i, (z, w) in enumerate(zip(zs, wants)):
        g0, g1 = pair(c, z)
        assert np.array_equal(g0, w[0]) and np.array_equal(g1, w[1]), CASES[i]
        single = pair(c, c.beaver_mul(probs[i][0], probs[i][1], probs[i][2], 16))
        assert np.array_equal(single[0], g0) and np.array_equal(single[1], g1), CASES[i]
    c.close()


def test_grouped_mul_with_empty_products(m):
    # zero-length products and squares beside ordinary ones: they do nothing
    # and take no open; the others give the oracle's result
    say("grouped beaver mul: empty products")
    c = m.Context(device=0, seed=SEED)
    cases = [(0, False, False), (5, True, False), (0, True, True), (CHUNK + 3, False, True), (0, False, False)]
    probs, outs, wants = [], [], []
    for i, (n, sq, view) in enumerate(cases):
        p, o, w = make_problem(m, c, 40 + i, n, sq, view)
        probs.append(p)
        outs.append(o)
        wants.append(w)
    before = c.stats()
    zs = c.beaver_mul_grouped(probs, 16, outs=outs)
    after = c.stats()
    assert after["opens"] - before["opens"] == sum(1 for n, _, _ in cases if n)
    assert after["launches"] - before["launches"] == 1
    for (n, sq, view), z, w in zip(cases, zs, wants):
        g0, g1 = pair(c, z)
        assert g0.size == n and np.array_equal(g0, w[0]) and np.array_equal(g1, w[1]), (n, sq, view)
    # all empty: nothing is launched
    before = c.stats()
    c.beaver_mul_grouped([probs[0], probs[2]], 16, outs=[outs[0], outs[2]])
    assert c.stats()["launches"] == before["launches"]
    c.close()


def test_grouped_mul_graph_replay(m):
    say("grouped beaver mul: graph replay")
    side = torch.cuda.Stream()
    with torch.cuda.stream(side):
        c = m.Context(device=0, seed=SEED)
        probs, outs, wants = [], [], []
        for i, (n, sq, view) in enumerate(CASES[:6]):
            p, o, w = make_problem(m, c, i, n, sq, view)
            probs.append(p)
            outs.append(o)
            wants.append(w)
        c.graph_begin()
        c.beaver_mul_grouped(probs, 16, outs=outs)
        g = c.graph_end()
        try:
            for rep in range(3):
                for o in outs:
                    o.s0.zero_()
                    o.s1.zero_()
                c.graph_launch(g)
                for i, (o, w) in enumerate(zip(outs, wants)):
                    g0, g1 = pair(c, o)
                    assert np.array_equal(g0, w[0]) and np.array_equal(g1, w[1]), (rep, i)
                c.reveal(probs[0][0])  # eager work between replays
                c.sync()
        finally:
            m.Context.graph_destroy(g)
            c.close()


def test_grouped_mul_errors(m):
    c = m.Context(device=0, seed=SEED)
    (gx, gy, t), out, _ = make_problem(m, c, 0, 64, False, False)
    with pytest.raises(m.MPCError) as e:  # two products writing the same output
        c.beaver_mul_grouped([(gx, gy, t), (gx, gy, t)], 0, outs=[out, out])
    assert e.value.status == -3
    with pytest.raises(m.MPCError) as e:  # output aliases an input
        c.beaver_mul_grouped([(gx, gy, t)], 0, outs=[m.SharedPair(gx.s0, out.s1)])
    assert e.value.status == -3
    (hx, hy, ht), hout, _ = make_problem(m, c, 1, 64, False, False)
    with pytest.raises(m.MPCError) as e:  # one product writes another's input (they run concurrently)
        c.beaver_mul_grouped([(gx, gy, t), (hx, hy, ht)], 0, outs=[m.SharedPair(hx.s0, out.s1), hout])
    assert e.value.status == -3
    with pytest.raises(m.MPCError) as e:  # the same for grouped matmuls: output onto another's triple share c
        tm = c.dealer(m.TRIPLE_MATMUL, 3, 5, (8, 8, 8))
        tm2 = c.dealer(m.TRIPLE_MATMUL, 3, 6, (8, 8, 8))
        xs = c.share(torch.zeros((8, 8), dtype=torch.int64, device=c.device), 0, 7)
        ys = c.share(torch.zeros((8, 8), dtype=torch.int64, device=c.device), 1, 8)
        c.beaver_matmul_grouped([(xs, ys, tm), (xs, ys, tm2)], 0, "limb8",
                                outs=[m.SharedPair(tm2.c0, c.empty((8, 8))), m.SharedPair(c.empty((8, 8)), c.empty((8, 8)))])
    assert e.value.status == -3
    with pytest.raises(m.MPCError) as e:
        c.beaver_mul_grouped([(gx, gy, t)], 64)
    assert e.value.status == -1
    assert c.beaver_mul_grouped([], 16) == []
    c.close()
