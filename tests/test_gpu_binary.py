"""GPU parity of binary sharing (App. C.1.1): XOR sharing, bitwise AND with
Beaver triples, arithmetic-to-binary conversion, Algorithm 2 and ReLU, all
against the CPU oracle bit for bit on the same seeds."""
import numpy as np
import pytest

import oracle
import workloads
from tests.gpu_util import dev, host, pair, say

pytestmark = pytest.mark.gpu

SEED = 777
Q = 1 << 64
EDGE = np.array([0, 1, 2, Q - 1, 1 << 63, (1 << 63) - 1, (1 << 63) + 1, 0x5555555555555555], dtype=np.uint64)


@pytest.fixture(scope="module")
def m():
    import paper_2109_00984_amd as mod
    return mod


@pytest.fixture(scope="module")
def ctx(m):
    c = m.Context(device=0, seed=SEED)
    yield c
    c.close()


def dev_pair(m, a, b):
    return m.SharedPair(dev(a), dev(b))


def same_pair(ctx, got, want, what):
    g0, g1 = pair(ctx, got)
    assert np.array_equal(g0, want[0]), f"{what}: party 0 differs"
    assert np.array_equal(g1, want[1]), f"{what}: party 1 differs"


def oracle_triple(t_dev, ctx):
    a0, a1, b0, b1, c0, c1 = [host(ctx, v) for v in (t_dev.a0, t_dev.a1, t_dev.b0, t_dev.b1, t_dev.c0, t_dev.c1)]
    return oracle.Triple((a0, a1), (b0, b1), (c0, c1))


@pytest.mark.parametrize("n", [1, 1000, 100003])
@pytest.mark.parametrize("src", [0, 1])
def test_bin_share_reveal(m, ctx, n, src):
    say(f"bin share n={n} src={src}")
    x = workloads.uniform_u64(n + src, (n,))
    x[: min(n, EDGE.size)] = EDGE[: min(n, EDGE.size)]
    s = ctx.bin_share(dev(x), src, 3)
    same_pair(ctx, s, oracle.bin_share(x, src, SEED, 3), "bin share")
    assert np.array_equal(host(ctx, ctx.bin_reveal(s)), x)


@pytest.mark.parametrize("n", [1, 5003])
def test_dealer_and_and_bin_and(m, ctx, n):
    say(f"bin and n={n}")
    t = ctx.dealer_and(51, 2, n)
    w = oracle.dealer_and(51, 2, n)
    got = oracle_triple(t, ctx)
    for name in ("a", "b", "c"):
        for p in (0, 1):
            assert np.array_equal(getattr(got, name)[p], getattr(w, name)[p]), (name, p)
    x, y = workloads.uniform_u64(10, (n,)), workloads.uniform_u64(11, (n,))
    xs, ys = oracle.bin_share(x, 0, SEED, 4), oracle.bin_share(y, 1, SEED, 5)
    z = ctx.bin_and(dev_pair(m, *xs), dev_pair(m, *ys), t)
    same_pair(ctx, z, oracle.bin_and(xs, ys, w), "bin and")


@pytest.mark.parametrize("n", [1, 777, 65537])
def test_a2b(m, ctx, n):
    say(f"a2b n={n}")
    x = workloads.uniform_u64(20 + n, (n,))
    x[: min(n, EDGE.size)] = EDGE[: min(n, EDGE.size)]
    xs = oracle.share(x, 0, SEED, 6)
    t = ctx.dealer_and(52, 3, 12 * n)
    z = ctx.a2b(dev_pair(m, *xs), 7, t)
    want = oracle.a2b(xs, SEED, 7, oracle.dealer_and(52, 3, 12 * n))
    same_pair(ctx, z, want, "a2b")
    g0, g1 = pair(ctx, z)
    assert np.array_equal(g0 ^ g1, x)


@pytest.mark.parametrize("bit", [0, 17, 63])
def test_b2a_bit(m, ctx, bit):
    n = 9001
    say(f"b2a bit={bit}")
    x = workloads.uniform_u64(30 + bit, (n,))
    bs = oracle.bin_share(x, 1, SEED, 8)
    rb, ra = ctx.dealer_b2a(53, 4, n)
    wrb, wra = oracle.dealer_b2a(53, 4, n)
    same_pair(ctx, rb, wrb, "b2a <r>")
    same_pair(ctx, ra, wra, "b2a [r]")
    z = ctx.b2a_bit(dev_pair(m, *bs), bit, rb, ra)
    same_pair(ctx, z, oracle.b2a_bit(bs, bit, wrb, wra), "b2a")


@pytest.mark.parametrize("n", [1, 4096, 100001])
def test_relu(m, ctx, n):
    say(f"relu n={n}")
    v = np.random.default_rng(n).integers(-(1 << 40), 1 << 40, size=n, dtype=np.int64)
    v[: min(n, 3)] = [0, -1, 1][: min(n, 3)]
    xs = oracle.share(v.view(np.uint64), 0, SEED, 9)
    t = ctx.dealer_and(54, 5, 12 * n)
    rb, ra = ctx.dealer_b2a(54, 6, n)
    tm = ctx.dealer(m.TRIPLE_MUL, 54, 7, (n,))
    z = ctx.relu(dev_pair(m, *xs), 10, t, rb, ra, tm)
    want = oracle.relu(xs, SEED, 10, oracle.dealer_and(54, 5, 12 * n), *oracle.dealer_b2a(54, 6, n),
                       oracle.dealer_mul(54, 7, n))
    same_pair(ctx, z, want, "relu")
    g0, g1 = pair(ctx, z)
    assert np.array_equal((g0 + g1).view(np.int64), np.maximum(v, 0))


def test_binary_rounds_and_errors(m, ctx):
    n = 64
    x = dev(np.arange(n, dtype=np.uint64))
    s = ctx.bin_share(x, 0, 1)
    with pytest.raises(m.MPCError) as e:  # output aliases an input share
        ctx.bin_reveal(s, out=s.s0)
    assert e.value.status == -3
    rb, ra = ctx.dealer_b2a(1, 1, n)
    with pytest.raises(m.MPCError) as e:
        ctx.b2a_bit(s, 64, rb, ra)
    assert e.value.status == -1
    before = ctx.stats()["opens"]
    t = ctx.dealer_and(1, 2, 12 * n)
    ctx.a2b(ctx.share(x, 0, 2), 3, t)
    assert ctx.stats()["opens"] - before == 7


def test_binary_empty_inputs(m, ctx):
    # n = 0 through every binary call: nothing is launched and nothing opened
    say("binary empty inputs")
    e = dev(np.zeros(0, np.uint64))
    before = ctx.stats()
    s = ctx.bin_share(e, 0, 1)
    assert ctx.bin_reveal(s).numel() == 0
    t = ctx.dealer_and(1, 2, 0)
    assert ctx.bin_and(s, s, t).s0.numel() == 0
    a = ctx.share(e, 0, 2)
    assert ctx.a2b(a, 3, t).s0.numel() == 0
    rb, ra = ctx.dealer_b2a(1, 4, 0)
    assert ctx.b2a_bit(s, 0, rb, ra).s0.numel() == 0
    tm = ctx.dealer(m.TRIPLE_MUL, 1, 5, (0,))
    assert ctx.relu(a, 6, t, rb, ra, tm).s0.numel() == 0
    after = ctx.stats()
    assert after["opens"] == before["opens"] and after["launches"] == before["launches"]
