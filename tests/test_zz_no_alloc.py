"""mpc_beaver_matmul_noalloc (the entry point that allocates nothing; its
workspace is the library's static per-device array) through the C ABI: the
same shares, bit for bit, as mpc_beaver_matmul and the oracle, over several
calls in a row with smaller inputs after larger ones (the array keeps the last
call's contents), a K-chunked product, the one-launch small product, and its
refusals."""
import numpy as np
import pytest
import torch

import oracle
from tests.gpu_util import dev, pair, say

pytestmark = pytest.mark.gpu

SEED, DSEED = 2031, 3031


@pytest.fixture(scope="module")
def m():
    import paper_2109_00984_amd as mpc
    return mpc


def rnd(seed, shape):
    return np.random.default_rng(seed).integers(0, 2**64, size=shape, dtype=np.uint64)


def run(c, m, M, N, K, tag, form, trunc=16):
    X, Y = rnd(tag, (M, K)), rnd(tag + 1, (K, N))
    x, y = c.share(dev(X), 0, 2 * tag), c.share(dev(Y), 1, 2 * tag + 1)
    t = c.dealer(m.TRIPLE_MATMUL, DSEED, tag, (M, N, K))
    za = c.beaver_matmul_noalloc(x, y, t, trunc, form)
    zb = c.beaver_matmul(x, y, t, trunc, "limb8")
    ga, gb = pair(c, za), pair(c, zb)
    assert np.array_equal(ga[0], gb[0]) and np.array_equal(ga[1], gb[1]), (M, N, K, form)
    return X, Y, ga


@pytest.mark.parametrize("form", ["limb8", "auto"])
def test_noalloc_matches_beaver_matmul_and_oracle(m, form):
    say(f"no-alloc Beaver matmul, form {form}")
    c = m.Context(device=0, seed=SEED)
    # larger, then smaller (stale contents of the shared array must not leak
    # in), then a product whose 2K crosses the int32 chunk bound (two GEMM
    # launches), then the smallest again
    for i, (M, N, K) in enumerate([(300, 200, 700), (40, 24, 100), (70, 50, 9000), (3, 5, 7)]):
        say(f"  call {i}: {M}x{N}x{K}")
        X, Y, got = run(c, m, M, N, K, 10 + 4 * i, form)
        want = oracle.beaver_matmul(oracle.share(X, 0, SEED, 2 * (10 + 4 * i)),
                                    oracle.share(Y, 1, SEED, 2 * (10 + 4 * i) + 1),
                                    oracle.dealer_matmul(DSEED, 10 + 4 * i, M, N, K), 16)
        assert np.array_equal(got[0], want[0]) and np.array_equal(got[1], want[1]), (M, N, K)
    c.close()


def test_noalloc_small_product_auto(m):
    # the small workload's 64x128 @ 128x32 goes to the one-launch product
    say("no-alloc Beaver matmul, small product")
    c = m.Context(device=0, seed=SEED)
    X, Y, got = run(c, m, 64, 32, 128, 40, "auto")
    want = oracle.beaver_matmul(oracle.share(X, 0, SEED, 80), oracle.share(Y, 1, SEED, 81),
                                oracle.dealer_matmul(DSEED, 40, 64, 32, 128), 16)
    assert np.array_equal(got[0], want[0]) and np.array_equal(got[1], want[1])
    c.close()


def test_noalloc_refusals(m):
    say("no-alloc Beaver matmul, refusals")
    c = m.Context(device=0, seed=SEED)
    M = N = K = 2048  # packed operands 24 * (M*K + K*N) bytes > 64 MiB
    x = m.SharedPair(c.empty((M, K)), c.empty((M, K)))
    y = m.SharedPair(c.empty((K, N)), c.empty((K, N)))
    t = m.TripleShares(c.empty((M, K)), c.empty((M, K)), c.empty((K, N)), c.empty((K, N)),
                       c.empty((M, N)), c.empty((M, N)))
    with pytest.raises(m.MPCError) as e:
        c.beaver_matmul_noalloc(x, y, t, 16, "limb8")
    assert e.value.status == m.MPC_E_SHAPE
    xs = m.SharedPair(c.empty((8, 8)), c.empty((8, 8)))
    ts = c.dealer(m.TRIPLE_MATMUL, DSEED, 50, (8, 8, 8))
    for form, status in [("plain", m.MPC_E_UNSUPPORTED), ("fp64limb", m.MPC_E_UNSUPPORTED)]:
        with pytest.raises(m.MPCError) as e:
            c.beaver_matmul_noalloc(xs, xs, ts, 16, form)
        assert e.value.status == status
    c.sync()
    c.close()
