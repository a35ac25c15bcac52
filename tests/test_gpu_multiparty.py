"""GPU parity of sharing among more than two parties (App. C.1.1) and of the
wrap-count truncation (Algorithm 1): every call against the CPU oracle on the
same seeds, bit for bit, for P from 2 to 16 parties."""
import numpy as np
import pytest
import torch

import oracle
import workloads
from tests.gpu_util import dev, say

pytestmark = pytest.mark.gpu

SEED = 4242
PARTIES = [2, 3, 5, 8, 16]


@pytest.fixture(scope="module")
def m():
    import paper_2109_00984_amd as mod
    return mod


@pytest.fixture(scope="module")
def ctx(m):
    c = m.Context(device=0, seed=SEED)
    yield c
    c.close()


def host(ctx, t):
    ctx.sync()
    return t.cpu().numpy().view(np.uint64)


def hosts(ctx, s):
    return [host(ctx, v) for v in s]


def to_dev_shared(m, arrs):
    return m.Shared([dev(a) for a in arrs])


def same(ctx, got, want, what):
    g = hosts(ctx, got)
    assert len(g) == len(want)
    for p, (a, b) in enumerate(zip(g, want)):
        assert np.array_equal(a.reshape(b.shape), b), f"{what}: party {p} differs"


@pytest.mark.parametrize("P", PARTIES)
@pytest.mark.parametrize("n", [1, 1000, 100003])
def test_mp_share_reveal(m, ctx, P, n):
    say(f"mp share/reveal P={P} n={n}")
    x = workloads.uniform_u64(P * 10 + n % 97, (n,))
    for src in (0, P - 1):
        s = ctx.mp_share(dev(x), P, src, 7)
        same(ctx, s, oracle.mp_share(x, P, src, SEED, 7), "share")
        assert np.array_equal(host(ctx, ctx.mp_reveal(s)), x)


@pytest.mark.parametrize("P", PARTIES)
@pytest.mark.parametrize("square", [False, True])
def test_mp_dealer_elementwise(m, ctx, P, square):
    n = 5001
    say(f"mp dealer P={P} square={square}")
    t = ctx.mp_dealer(P, m.TRIPLE_SQUARE if square else m.TRIPLE_MUL, 31, 2, (n,))
    w = oracle.mp_dealer_mul(31, 2, P, n, square=square)
    same(ctx, t.a, w.a, "a")
    same(ctx, t.b, w.b, "b")
    if not square:
        same(ctx, t.c, w.c, "c")


@pytest.mark.parametrize("P", [2, 3, 8])
@pytest.mark.parametrize("M,N,K", [(1, 1, 1), (37, 53, 70), (128, 96, 300), (300, 20, 17)])
def test_mp_dealer_matmul(m, ctx, P, M, N, K):
    say(f"mp dealer matmul P={P} {M}x{N}x{K}")
    t = ctx.mp_dealer(P, m.TRIPLE_MATMUL, 33, 4, (M, N, K))
    w = oracle.mp_dealer_matmul(33, 4, P, M, N, K)
    same(ctx, t.a, w.a, "a")
    same(ctx, t.b, w.b, "b")
    same(ctx, t.c, w.c, "c")


@pytest.mark.parametrize("P", PARTIES)
@pytest.mark.parametrize("square", [False, True])
def test_mp_beaver_mul(m, ctx, P, square):
    n = 4099
    say(f"mp beaver mul P={P} square={square}")
    X = oracle.encode(workloads.uniform(P + 1, (n,), -4, 4))
    Y = oracle.encode(workloads.uniform(P + 2, (n,), -4, 4))
    xs, ys = oracle.mp_share(X, P, 0, SEED, 11), oracle.mp_share(Y, P, P - 1, SEED, 12)
    kind = m.TRIPLE_SQUARE if square else m.TRIPLE_MUL
    t = ctx.mp_dealer(P, kind, 35, 6, (n,))
    z = ctx.mp_beaver_mul(to_dev_shared(m, xs), None if square else to_dev_shared(m, ys), t)
    w = oracle.mp_dealer_mul(35, 6, P, n, square=square)
    want = oracle.mp_beaver_mul(xs, None if square else ys, w)
    same(ctx, z, want, "beaver mul")


@pytest.mark.parametrize("P", [2, 3, 5])
@pytest.mark.parametrize("form", ["plain", "limb8"])
@pytest.mark.parametrize("M,N,K", [(1, 1, 1), (64, 32, 128), (37, 53, 70), (129, 65, 300)])
def test_mp_beaver_matmul(m, ctx, P, form, M, N, K):
    say(f"mp beaver matmul P={P} {form} {M}x{N}x{K}")
    xs = [workloads.uniform_u64(100 + p, (M, K)) for p in range(P)]
    ys = [workloads.uniform_u64(200 + p, (K, N)) for p in range(P)]
    t = ctx.mp_dealer(P, m.TRIPLE_MATMUL, 37, 8, (M, N, K))
    z = ctx.mp_beaver_matmul(to_dev_shared(m, xs), to_dev_shared(m, ys), t, form)
    want = oracle.mp_beaver_matmul(xs, ys, oracle.mp_dealer_matmul(37, 8, P, M, N, K))
    same(ctx, z, want, "beaver matmul")


def test_mp_beaver_matmul_k_chunked(m, ctx):
    # 2K = 20000 concatenated k: the limb form splits it over launches
    P, M, N, K = 3, 40, 24, 10000
    say("mp beaver matmul k-chunked")
    xs = [workloads.uniform_u64(300 + p, (M, K)) for p in range(P)]
    ys = [workloads.uniform_u64(400 + p, (K, N)) for p in range(P)]
    t = ctx.mp_dealer(P, m.TRIPLE_MATMUL, 39, 9, (M, N, K))
    w = oracle.mp_dealer_matmul(39, 9, P, M, N, K)
    want = oracle.mp_beaver_matmul(xs, ys, w)
    for form in ("limb8", "plain"):
        z = ctx.mp_beaver_matmul(to_dev_shared(m, xs), to_dev_shared(m, ys), t, form)
        same(ctx, z, want, f"beaver matmul {form}")


@pytest.mark.parametrize("P", PARTIES)
def test_mp_dealer_trunc(m, ctx, P):
    n = 3001
    say(f"mp dealer trunc P={P}")
    r, th = ctx.mp_dealer_trunc(P, 41, 3, n)
    wr, wt = oracle.mp_dealer_trunc(41, 3, P, n)
    same(ctx, r, wr, "r")
    same(ctx, th, wt, "theta_r")


@pytest.mark.parametrize("P", PARTIES)
@pytest.mark.parametrize("bits", [1, 16, 63])
def test_mp_truncate(m, ctx, P, bits):
    n = 20011
    say(f"mp truncate P={P} bits={bits}")
    rng = np.random.default_rng(P * 100 + bits)
    X = rng.integers(-(1 << 62), 1 << 62, size=n, dtype=np.int64)
    xs = oracle.mp_share(X, P, 0, SEED, 13)
    r, th = ctx.mp_dealer_trunc(P, 43, 5, n)
    wr, wt = oracle.mp_dealer_trunc(43, 5, P, n)
    g = to_dev_shared(m, xs)
    ctx.mp_truncate(g, bits, r, th)
    same(ctx, g, oracle.mp_truncate(xs, bits, wr, wt), "truncate")


def test_mp_layer_chain_plaintext(m, ctx):
    # three parties: X (64x128) @ W (128x32) with a 2^16 truncation, then a
    # square and truncation; the revealed values match float64 plaintext
    P, B, I, O = 3, 64, 128, 32
    Xr = workloads.uniform(7001, (B, I), -1, 1)
    Wr = workloads.uniform(7002, (I, O), -1, 1)
    x = ctx.mp_share(dev(oracle.encode(Xr)), P, 0, 21)
    w = ctx.mp_share(dev(oracle.encode(Wr)), P, 1, 22)
    t = ctx.mp_dealer(P, m.TRIPLE_MATMUL, 45, 1, (B, O, I))
    h = ctx.mp_beaver_matmul(x, w, t, "limb8")
    r, th = ctx.mp_dealer_trunc(P, 45, 2, B * O)
    flat = m.Shared([v.view(-1) for v in h])
    ctx.mp_truncate(flat, 16, r, th)
    sq_t = ctx.mp_dealer(P, m.TRIPLE_SQUARE, 45, 3, (B * O,))
    sq = ctx.mp_beaver_mul(flat, None, sq_t)
    r2, th2 = ctx.mp_dealer_trunc(P, 45, 4, B * O)
    ctx.mp_truncate(sq, 16, r2, th2)
    got = oracle.decode(host(ctx, ctx.mp_reveal(sq)).view(np.int64)).reshape(B, O)
    want = (Xr @ Wr) ** 2
    assert np.max(np.abs(got - want)) < 1e-2
    nmse = np.sum((got - want) ** 2) / np.sum(want ** 2)
    assert nmse < 4e-4


def test_mp_errors_and_counters(m, ctx):
    x = dev(np.arange(8, dtype=np.uint64))
    for P in (1, 17):
        with pytest.raises((m.MPCError, ValueError, IndexError, TypeError)):
            ctx.mp_share(x, P, 0, 1)
    s = ctx.mp_share(x, 3, 0, 1)
    r, th = ctx.mp_dealer_trunc(3, 1, 1, 8)
    with pytest.raises(m.MPCError) as e:
        ctx.mp_truncate(s, 0, r, th)
    assert e.value.status == -1
    with pytest.raises(m.MPCError) as e:  # output aliases an input
        ctx.mp_reveal(s, out=s.shares[1])
    assert e.value.status == -3
    before = ctx.stats()
    t = ctx.mp_dealer(3, m.TRIPLE_MUL, 1, 1, (8,))
    ctx.mp_beaver_mul(s, s, t)
    ctx.mp_truncate(s, 16, r, th)
    after = ctx.stats()
    assert after["opens"] - before["opens"] == 2
    assert after["truncations"] - before["truncations"] == 1


def test_mp_empty_inputs(m, ctx):
    # n = 0 and matrix products with no rows, no columns or no k among three
    # parties: the empty calls do nothing; k = 0 leaves each party its c share
    P = 3
    say("mp empty inputs")
    e = np.zeros(0, np.uint64)
    s = ctx.mp_share(dev(e), P, 0, 7)
    assert all(v.numel() == 0 for v in s.shares) and ctx.mp_reveal(s).numel() == 0
    t = ctx.mp_dealer(P, m.TRIPLE_MUL, 31, 30, (0,))
    assert ctx.mp_beaver_mul(s, s, t).shares[0].numel() == 0
    r, th = ctx.mp_dealer_trunc(P, 31, 31, 0)
    ctx.mp_truncate(s, 16, r, th)
    for i, (M, N, K) in enumerate([(0, 5, 3), (4, 0, 3), (4, 5, 0)]):
        xs = [workloads.uniform_u64(500 + p, (M, K)) for p in range(P)]
        ys = [workloads.uniform_u64(600 + p, (K, N)) for p in range(P)]
        t = ctx.mp_dealer(P, m.TRIPLE_MATMUL, 37, 40 + i, (M, N, K))
        w = oracle.mp_dealer_matmul(37, 40 + i, P, M, N, K)
        same(ctx, t.a, w.a, f"a {M}x{N}x{K}")
        same(ctx, t.b, w.b, f"b {M}x{N}x{K}")
        same(ctx, t.c, w.c, f"c {M}x{N}x{K}")
        for form in ("plain", "limb8"):
            z = ctx.mp_beaver_matmul(to_dev_shared(m, xs), to_dev_shared(m, ys), t, form)
            same(ctx, z, oracle.mp_beaver_matmul(xs, ys, w), f"beaver matmul {form} {M}x{N}x{K}")
