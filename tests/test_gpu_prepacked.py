"""Offline-packed matrix triples: mpc_dealer_triples_packed makes the same
triple as mpc_dealer_triples and packs a1, b0, b1; the online Beaver matmul
over it (single and grouped) gives the oracle's shares bit for bit."""
import numpy as np
import pytest
import torch

import oracle
from tests.gpu_util import dev, pair, say

pytestmark = pytest.mark.gpu

SEED, DSEED = 2041, 3041


@pytest.fixture(scope="module")
def m():
    import paper_2109_00984_amd as mpc
    return mpc


def rnd(seed, shape):
    return np.random.default_rng(seed).integers(0, 2**64, size=shape, dtype=np.uint64)


@pytest.mark.parametrize("M,N,K,trunc", [(64, 32, 128, 16), (200, 136, 70, 0), (1, 300, 33, 16), (513, 65, 260, 16),
                                         (96, 64, 9000, 16), (130, 260, 1100, 63)])
def test_prepacked_matmul_matches_oracle(m, M, N, K, trunc):
    say(f"prepacked Beaver matmul {M}x{N}x{K} trunc {trunc}")
    c = m.Context(device=0, seed=SEED)
    tag = M + 7 * N + 11 * K
    t, packed = c.dealer_packed(DSEED, tag, (M, N, K))
    tr = c.dealer(m.TRIPLE_MATMUL, DSEED, tag, (M, N, K))
    c.sync()
    for a, b in [(t.a0, tr.a0), (t.a1, tr.a1), (t.b0, tr.b0), (t.b1, tr.b1), (t.c0, tr.c0), (t.c1, tr.c1)]:
        assert torch.equal(a, b)
    X, Y = rnd(tag, (M, K)), rnd(tag + 1, (K, N))
    x, y = c.share(dev(X), 0, 1), c.share(dev(Y), 1, 2)
    z = c.beaver_matmul_prepacked(x, y, t, packed, trunc)
    zl = c.beaver_matmul(x, y, t, trunc, "limb8")
    got, ref = pair(c, z), pair(c, zl)
    want = oracle.beaver_matmul(oracle.share(X, 0, SEED, 1), oracle.share(Y, 1, SEED, 2),
                                oracle.dealer_matmul(DSEED, tag, M, N, K), trunc)
    for p in range(2):
        assert np.array_equal(got[p], want[p]) and np.array_equal(ref[p], want[p]), (M, N, K, p)
    c.close()


def test_prepacked_grouped_matches_oracle(m):
    say("prepacked grouped Beaver matmul")
    c = m.Context(device=0, seed=SEED)
    # thin in M, thin in N, and two regular products whose edges run as
    # strips (region offsets into the dealer's packed blocks)
    shapes = [(300, 120, 500), (17, 200, 300), (150, 20, 260), (40, 600, 64), (9, 5, 70), (200, 136, 70),
              (520, 65, 96)]
    probs, wants = [], []
    for i, (M, N, K) in enumerate(shapes):
        X, Y = rnd(100 + 2 * i, (M, K)), rnd(101 + 2 * i, (K, N))
        t, packed = c.dealer_packed(DSEED, 50 + i, (M, N, K))
        probs.append((c.share(dev(X), 0, 60 + 2 * i), c.share(dev(Y), 1, 61 + 2 * i), t, packed))
        wants.append(oracle.beaver_matmul(oracle.share(X, 0, SEED, 60 + 2 * i), oracle.share(Y, 1, SEED, 61 + 2 * i),
                                          oracle.dealer_matmul(DSEED, 50 + i, M, N, K), 16))
    for explicit in [None, 14, 15]:
        if explicit is not None:
            c.set_default_tile_config(explicit, 8, True)
        zs = c.beaver_matmul_grouped_prepacked(probs, 16)
        for (M, N, K), z, w in zip(shapes, zs, wants):
            got = pair(c, z)
            assert np.array_equal(got[0], w[0]) and np.array_equal(got[1], w[1]), (explicit, (M, N, K))
    c.close()


def test_prepacked_refusals(m):
    import ctypes
    say("prepacked refusals")
    c = m.Context(device=0, seed=SEED)
    M = N = K = 64
    t, packed = c.dealer_packed(DSEED, 77, (M, N, K))
    x = c.share(dev(rnd(1, (M, K))), 0, 1)
    y = c.share(dev(rnd(2, (K, N))), 1, 2)
    z = m.SharedPair(c.empty((M, N)), c.empty((M, N)))
    st = t.struct()
    lib = m._lib
    args = lambda pk, z0: (c._h, M, N, K, m._ptr(x.s0), m._ptr(x.s1), m._ptr(y.s0), m._ptr(y.s1), ctypes.byref(st),
                           pk, 16, z0, m._ptr(z.s1))
    assert lib.mpc_beaver_matmul_prepacked(*args(None, m._ptr(z.s0))) == m.MPC_E_INVAL
    assert lib.mpc_beaver_matmul_prepacked(*args(ctypes.c_void_p(packed.data_ptr() + 8), m._ptr(z.s0))) == m.MPC_E_INVAL
    # an output inside the packed buffer
    assert lib.mpc_beaver_matmul_prepacked(*args(m._ptr(packed), ctypes.c_void_p(packed.data_ptr()))) == m.MPC_E_ALIAS
    c.sync()
    c.close()
