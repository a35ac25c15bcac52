"""GPU parity: every library call against the CPU oracle on identical seeded
inputs, bit for bit (ring results are exact, so the tolerance is zero)."""
import ctypes

import numpy as np
import pytest
import torch

import oracle
import workloads
from tests.gpu_util import dev, host, pair, say

pytestmark = pytest.mark.gpu

SEED = 2024
EDGE = np.array([0, 1, 2, (1 << 63) - 1, 1 << 63, (1 << 64) - 1, 0x7F7F7F7F7F7F7F80,
                 0x7F7F7F7F7F7F7F7F, 0x8080808080808080], dtype=np.uint64)


@pytest.fixture(scope="module")
def m():
    import paper_2109_00984_amd as mod
    return mod


@pytest.fixture(scope="module")
def ctx(m):
    c = m.Context(device=0, seed=SEED)
    yield c
    c.close()


def rnd(seed, shape):
    return workloads.uniform_u64(seed, shape)


def shares_dev(m, sh):
    return m.SharedPair(dev(sh[0]), dev(sh[1]))


def triple_dev(m, t):
    return m.TripleShares(dev(t.a[0]), dev(t.a[1]), dev(t.b[0]), dev(t.b[1]),
                          dev(t.c[0]) if t.c is not None else None,
                          dev(t.c[1]) if t.c is not None else None)


def assert_pair(ctx, got, want, what):
    g0, g1 = pair(ctx, got)
    assert np.array_equal(g0, want[0]), f"{what}: party 0 differs"
    assert np.array_equal(g1, want[1]), f"{what}: party 1 differs"


# ------------------------------------------------------------------ share / reveal / truncate
@pytest.mark.parametrize("n", [1, 9, 4096, 100003])
@pytest.mark.parametrize("src", [0, 1])
def test_share_reveal(m, ctx, n, src):
    say(f"share n={n} src={src}")
    x = np.concatenate([EDGE, rnd(n, n)])[:n]
    s = ctx.share(dev(x), src, tag=n + src)
    want = oracle.share(x, src, SEED, n + src)
    assert_pair(ctx, s, want, "share")
    r = ctx.reveal(s)
    assert np.array_equal(host(ctx, r), x)


@pytest.mark.parametrize("bits", [1, 16, 63])
def test_truncate(m, ctx, bits):
    say(f"truncate bits={bits}")
    a, b = np.concatenate([EDGE, rnd(1, 5000)]), np.concatenate([EDGE[::-1], rnd(2, 5000)])
    p = m.SharedPair(dev(a), dev(b))
    ctx.truncate(p, bits)
    assert_pair(ctx, p, (oracle.truncate(a, bits), oracle.truncate(b, bits)), "truncate")


def test_empty_inputs(m, ctx):
    say("empty")
    e = torch.empty(0, dtype=torch.int64, device="cuda")
    s = ctx.share(e, 0, 1)
    assert s.s0.numel() == 0
    assert ctx.reveal(s).numel() == 0
    ctx.truncate(s, 16)
    t = ctx.dealer(m.TRIPLE_MUL, 1, 1, (0,))
    z = ctx.beaver_mul(s, s, t, 16)
    assert z.s0.numel() == 0
    zt = ctx.dealer(m.TRIPLE_MATMUL, 1, 2, (0, 5, 3))
    x = m.SharedPair(ctx.empty((0, 3)), ctx.empty((0, 3)))
    y = m.SharedPair(ctx.empty((3, 5)), ctx.empty((3, 5)))
    y = ctx.share(dev(rnd(3, (3, 5))), 0, 3)
    assert ctx.beaver_matmul(x, y, zt, 16).s0.shape == (0, 5)
    ctx.sync()


@pytest.mark.parametrize("form", ["plain", "limb8"])
def test_zero_k(m, ctx, form):
    # k = 0: every product is the empty sum, so the dealer's c is 0 (shared as
    # c0, -c0) and each party's Beaver output is its c share, truncated
    M, N = 70, 9
    say(f"k = 0 ({form})")
    X, Y = np.zeros((M, 0), np.uint64), np.zeros((0, N), np.uint64)
    xs, ys = oracle.share(X, 0, SEED, 61), oracle.share(Y, 1, SEED, 62)
    w = oracle.dealer_matmul(3007, 63, M, N, 0)
    t = ctx.dealer(m.TRIPLE_MATMUL, 3007, 63, (M, N, 0))
    assert_pair(ctx, m.SharedPair(t.c0, t.c1), w.c, "dealer c at k = 0")
    gx, gy = ctx.share(dev(X), 0, 61), ctx.share(dev(Y), 1, 62)
    z = ctx.beaver_matmul(gx, gy, t, 16, form)
    assert_pair(ctx, z, oracle.beaver_matmul(xs, ys, w, 16), "Beaver matmul at k = 0")
    C = ctx.ring_gemm(gx.s0, gy.s0, form=form)
    assert not np.any(host(ctx, C))
    # a grouped call mixing k = 0 with an ordinary problem
    M2, N2, K2 = 33, 17, 40
    X2, Y2 = rnd(64, (M2, K2)), rnd(65, (K2, N2))
    gx2, gy2 = ctx.share(dev(X2), 0, 66), ctx.share(dev(Y2), 1, 67)
    t2 = ctx.dealer(m.TRIPLE_MATMUL, 3007, 68, (M2, N2, K2))
    zs = ctx.beaver_matmul_grouped([(gx, gy, t), (gx2, gy2, t2)], 16, form)
    assert_pair(ctx, zs[0], oracle.beaver_matmul(xs, ys, w, 16), "grouped, k = 0 problem")
    want2 = oracle.beaver_matmul(oracle.share(X2, 0, SEED, 66), oracle.share(Y2, 1, SEED, 67),
                                 oracle.dealer_matmul(3007, 68, M2, N2, K2), 16)
    assert_pair(ctx, zs[1], want2, "grouped, ordinary problem")


def test_argument_errors(m, ctx):
    say("errors")
    x = ctx.share(dev(rnd(1, 16)), 0, 1)
    with pytest.raises(m.MPCError):
        ctx.truncate(x, 64)
    with pytest.raises(m.MPCError):
        ctx.share(dev(rnd(1, 16)), 2, 1)
    t = ctx.dealer(m.TRIPLE_MUL, 1, 1, (16,))
    # output aliasing an input is refused
    with pytest.raises(m.MPCError):
        ctx.beaver_mul(x, x, t, 16, out=m.SharedPair(x.s0, t.c1.clone()))
    ctx.sync()


def test_oversized_shapes_refused(m, ctx):
    # element counts that no device holds (or whose products wrap 64 bits)
    # are refused before any work is issued, through the raw C ABI
    say("oversized shapes")
    L, p = m._lib, m._ptr
    buf = ctx.empty((64,))
    q = p(buf)
    big = 1 << 40
    assert L.mpc_ring_gemm(ctx._h, big, big, big, q, q, q, 0) == -2
    assert L.mpc_ring_gemm(ctx._h, 1 << 62, 4, 4, q, q, q, 1) == -2
    assert L.mpc_share(ctx._h, q, 1 << 50, 0, 1, q, q) == -2
    assert L.mpc_reveal(ctx._h, q, q, 1 << 62, q) == -2
    t = ctx.dealer(m.TRIPLE_MUL, 1, 1, (64,))
    st = t.struct()
    assert L.mpc_beaver_matmul(ctx._h, big, big, big, q, q, q, q, ctypes.byref(st), 0, 0, q, q) == -2
    dims = (m.I64 * 6)(big, big, big, 0, 0, 0)
    assert L.mpc_dealer_triples(ctx._h, m.TRIPLE_MATMUL, 1, 1, dims, ctypes.byref(st)) == -2
    shape = m.Conv1dShape(1 << 20, 1 << 20, 1 << 20, 4, 3, 1)
    assert L.mpc_beaver_conv1d(ctx._h, ctypes.byref(shape), q, q, q, q, ctypes.byref(st), 0, 0, q, q) == -2
    ctx.sync()


def test_binding_refuses_bad_tensors(m, ctx):
    # the library takes bare pointers: the binding checks device, dtype,
    # layout and element counts before any call
    say("binding argument checks")
    x = ctx.share(dev(rnd(81, 32)), 0, 81)
    t = ctx.dealer(m.TRIPLE_MUL, 1, 82, (32,))
    short = ctx.dealer(m.TRIPLE_MUL, 1, 83, (31,))
    with pytest.raises(ValueError):  # output on the host
        ctx.reveal(x, out=torch.empty(32, dtype=torch.int64))
    with pytest.raises(ValueError):  # output too small
        ctx.reveal(x, out=ctx.empty((31,)))
    with pytest.raises(ValueError):  # output of another dtype
        ctx.share(dev(rnd(84, 32)), 0, 84, out=m.SharedPair(ctx.empty((32,)), torch.empty(32, device="cuda")))
    with pytest.raises(ValueError):  # triple shorter than the operands
        ctx.beaver_mul(x, x, short, 16)
    with pytest.raises(ValueError):  # shares of different lengths
        ctx.beaver_mul(x, m.SharedPair(x.s0, ctx.empty((33,))), t, 16)
    with pytest.raises(ValueError):  # product without the triple's c
        ctx.beaver_mul(x, x, m.TripleShares(t.a0, t.a1, t.b0, t.b1), 16)
    with pytest.raises(ValueError):  # non-contiguous operand
        ctx.ring_gemm(ctx.empty((8, 16)).t(), ctx.empty((8, 4)))
    with pytest.raises(ValueError):  # matmul triple of the wrong shape
        ctx.beaver_matmul(m.SharedPair(ctx.empty((4, 8)), ctx.empty((4, 8))),
                          m.SharedPair(ctx.empty((8, 4)), ctx.empty((8, 4))),
                          ctx.dealer(m.TRIPLE_MATMUL, 1, 85, (4, 4, 4)), 16)
    with pytest.raises(ValueError):  # dealer into buffers too small for the shape
        ctx.dealer_into(m.TRIPLE_MATMUL, 1, 86, (4, 4, 8), ctx.dealer(m.TRIPLE_MATMUL, 1, 87, (4, 4, 4)))
    s3 = ctx.mp_share(dev(rnd(88, 32)), 3, 0, 88)
    t2 = ctx.mp_dealer(2, m.TRIPLE_MUL, 1, 89, (32,))
    with pytest.raises(ValueError):  # a 2-party triple for 3-party shares
        ctx.mp_beaver_mul(s3, s3, t2)
    ctx.sync()


def test_reveal_in_place_and_overlap(m, ctx):
    say("reveal in place / overlapping output")
    x = rnd(71, 100)
    buf = ctx.empty((202,))
    s0, s1 = buf[0:100], buf[101:201]
    s = ctx.share(dev(x), 1, 72, out=m.SharedPair(s0, s1))
    ctx.reveal(s, out=s1)  # in place
    assert np.array_equal(host(ctx, s1), x)
    with pytest.raises(m.MPCError) as e:  # one element past s0: overlaps it, not in place
        ctx.reveal(m.SharedPair(s0, s1), out=buf[1:101])
    assert e.value.status == -3


# ------------------------------------------------------------------ dealer
@pytest.mark.parametrize("n", [1, 4096, 65537])
def test_dealer_elementwise(m, ctx, n):
    say(f"dealer mul/square n={n}")
    t = ctx.dealer(m.TRIPLE_MUL, 77, 5, (n,))
    w = oracle.dealer_mul(77, 5, n)
    for g, e in [(t.a0, w.a[0]), (t.a1, w.a[1]), (t.b0, w.b[0]), (t.b1, w.b[1]), (t.c0, w.c[0]),
                 (t.c1, w.c[1])]:
        assert np.array_equal(host(ctx, g), e)
    s = ctx.dealer(m.TRIPLE_SQUARE, 78, 6, (n,))
    w = oracle.dealer_square(78, 6, n)
    for g, e in [(s.a0, w.a[0]), (s.a1, w.a[1]), (s.b0, w.b[0]), (s.b1, w.b[1])]:
        assert np.array_equal(host(ctx, g), e)


# the first four take the plain form, the rest the limb form (work >= 2^22),
# whose packs draw a and b from the PRG themselves
@pytest.mark.parametrize("M,N,K", [(1, 1, 1), (64, 32, 128), (37, 53, 70), (130, 70, 300),
                                   (200, 150, 300), (257, 33, 1000), (2048, 2049, 1), (64, 64, 1024)])
def test_dealer_matmul(m, ctx, M, N, K):
    say(f"dealer matmul {M}x{N}x{K}")
    t = ctx.dealer(m.TRIPLE_MATMUL, 3001, 7, (M, N, K))
    w = oracle.dealer_matmul(3001, 7, M, N, K)
    for g, e in [(t.a0, w.a[0]), (t.a1, w.a[1]), (t.b0, w.b[0]), (t.b1, w.b[1]), (t.c0, w.c[0]),
                 (t.c1, w.c[1])]:
        assert np.array_equal(host(ctx, g), e)


# ------------------------------------------------------------------ Beaver element-wise
@pytest.mark.parametrize("n", [1, 4096, 4099, 1 << 20])
@pytest.mark.parametrize("trunc", [0, 16])
def test_beaver_mul(m, ctx, n, trunc):
    say(f"beaver mul n={n} trunc={trunc}")
    x = oracle.encode(workloads.uniform(1001, n, -4, 4))
    y = oracle.encode(workloads.uniform(1002, n, -4, 4))
    xs, ys = oracle.share(x, 0, SEED, 1), oracle.share(y, 1, SEED, 2)
    gx = ctx.share(dev(x), 0, 1)
    gy = ctx.share(dev(y), 1, 2)
    assert_pair(ctx, gx, xs, "share x")
    t = ctx.dealer(m.TRIPLE_MUL, 3001, 9, (n,))
    z = ctx.beaver_mul(gx, gy, t, trunc)
    want = oracle.beaver_mul(xs, ys, oracle.dealer_mul(3001, 9, n), trunc)
    assert_pair(ctx, z, want, "beaver mul")


@pytest.mark.parametrize("n", [1, 4096, 70001])
def test_beaver_square(m, ctx, n):
    say(f"beaver square n={n}")
    x = np.concatenate([EDGE, rnd(5, n)])[:n]
    xs = oracle.share(x, 0, SEED, 3)
    t = ctx.dealer(m.TRIPLE_SQUARE, 11, 1, (n,))
    z = ctx.beaver_mul(ctx.share(dev(x), 0, 3), None, t, 16)
    want = oracle.beaver_square(xs, oracle.dealer_square(11, 1, n), 16)
    assert_pair(ctx, z, want, "beaver square")


# ------------------------------------------------------------------ ring GEMM and Beaver matmul
GEMM_SHAPES = [(1, 1, 1), (64, 32, 128), (37, 53, 70), (129, 65, 33), (256, 192, 160),
               (5, 300, 17)]


@pytest.mark.parametrize("form", ["plain", "limb8"])
@pytest.mark.parametrize("M,N,K", GEMM_SHAPES)
def test_ring_gemm(m, ctx, form, M, N, K):
    say(f"ring gemm {form} {M}x{N}x{K}")
    A, B = rnd(M * 7 + K, (M, K)), rnd(N * 11 + K, (K, N))
    A.ravel()[0] = 0x7F7F7F7F7F7F7F80
    B.ravel()[0] = 0x7F7F7F7F7F7F7F80
    C = ctx.ring_gemm(dev(A), dev(B), form=form)
    assert np.array_equal(host(ctx, C), oracle.ring_gemm(A, B))


@pytest.mark.parametrize("form", ["plain", "limb8"])
def test_ring_gemm_worst_case_limbs(m, ctx, form):
    # every limb -128: each int8 product is 2^14, the largest the bound allows
    say(f"ring gemm all -128 limbs {form}")
    M, N, K = 64, 64, 8192
    A = np.full((M, K), 0x7F7F7F7F7F7F7F80, dtype=np.uint64)
    B = np.full((K, N), 0x7F7F7F7F7F7F7F80, dtype=np.uint64)
    C = ctx.ring_gemm(dev(A), dev(B), form=form)
    assert np.array_equal(host(ctx, C), oracle.ring_gemm(A, B))


@pytest.mark.parametrize("form", ["plain", "limb8"])
@pytest.mark.parametrize("M,N,K", GEMM_SHAPES)
@pytest.mark.parametrize("trunc", [0, 16])
def test_beaver_matmul(m, ctx, form, M, N, K, trunc):
    say(f"beaver matmul {form} {M}x{N}x{K} trunc={trunc}")
    X = oracle.encode(workloads.uniform(M + 1, (M, K), -4, 4))
    Y = oracle.encode(workloads.uniform(N + 2, (K, N), -4, 4))
    xs, ys = oracle.share(X, 0, SEED, 21), oracle.share(Y, 1, SEED, 22)
    t = ctx.dealer(m.TRIPLE_MATMUL, 3001, 40, (M, N, K))
    z = ctx.beaver_matmul(ctx.share(dev(X), 0, 21), ctx.share(dev(Y), 1, 22), t, trunc, form)
    want = oracle.beaver_matmul(xs, ys, oracle.dealer_matmul(3001, 40, M, N, K), trunc)
    assert_pair(ctx, z, want, "beaver matmul")


@pytest.mark.parametrize("form", ["plain", "limb8"])
@pytest.mark.parametrize("trunc", [1, 63])
def test_beaver_matmul_truncation_extremes(m, ctx, form, trunc):
    # the fused truncation at its narrowest and widest shifts, on uniform ring
    # operands (every output's sign bit in play), split-K and one-launch sizes
    for (M, N, K) in [(130, 70, 300), (5, 7, 3000)]:
        say(f"beaver matmul {form} {M}x{N}x{K} trunc={trunc}")
        X, Y = rnd(M + 7, (M, K)), rnd(N + 9, (K, N))
        t = ctx.dealer(m.TRIPLE_MATMUL, 3011, 44, (M, N, K))
        z = ctx.beaver_matmul(ctx.share(dev(X), 0, 45), ctx.share(dev(Y), 1, 46), t, trunc, form)
        want = oracle.beaver_matmul(oracle.share(X, 0, SEED, 45), oracle.share(Y, 1, SEED, 46),
                                    oracle.dealer_matmul(3011, 44, M, N, K), trunc)
        assert_pair(ctx, z, want, f"beaver matmul trunc={trunc}")


@pytest.mark.parametrize("M,N,K", [(4096, 64, 1), (3, 5, 7), (2, 3, 1024), (64, 32, 128), (33, 7, 1000)])
@pytest.mark.parametrize("trunc", [0, 16])
def test_small_beaver_matmul_one_launch(m, ctx, M, N, K, trunc):
    # products of at most 2^18 ring MACs with k <= 1024 take the plain form's single fused launch
    say(f"small beaver matmul {M}x{N}x{K} trunc={trunc}")
    X, Y = rnd(M + 3, (M, K)), rnd(N + 5, (K, N))
    gx, gy = ctx.share(dev(X), 0, 41), ctx.share(dev(Y), 1, 42)
    t = ctx.dealer(m.TRIPLE_MATMUL, 3002, 43, (M, N, K))
    ctx.sync()
    before = ctx.stats()["launches"]
    z = ctx.beaver_matmul(gx, gy, t, trunc, "plain")
    assert ctx.stats()["launches"] - before == 1
    want = oracle.beaver_matmul(oracle.share(X, 0, SEED, 41), oracle.share(Y, 1, SEED, 42),
                                oracle.dealer_matmul(3002, 43, M, N, K), trunc)
    assert_pair(ctx, z, want, "small beaver matmul")


@pytest.mark.parametrize("form", ["plain", "limb8"])
def test_beaver_matmul_k_chunked(m, ctx, form):
    # 2K = 20000 concatenated k exceeds one limb launch's int32-safe range
    M, N, K = 40, 24, 10000
    say(f"beaver matmul k-chunked {form} {M}x{N}x{K}")
    X, Y = rnd(1, (M, K)), rnd(2, (K, N))
    xs, ys = oracle.share(X, 0, SEED, 31), oracle.share(Y, 0, SEED, 32)
    t = ctx.dealer(m.TRIPLE_MATMUL, 5, 41, (M, N, K))
    z = ctx.beaver_matmul(ctx.share(dev(X), 0, 31), ctx.share(dev(Y), 0, 32), t, 16, form)
    want = oracle.beaver_matmul(xs, ys, oracle.dealer_matmul(5, 41, M, N, K), 16)
    assert_pair(ctx, z, want, "beaver matmul chunked")


def test_forms_agree_and_reveal_is_product(m, ctx):
    say("forms agree")
    M, N, K = 96, 80, 200
    X = oracle.encode(workloads.uniform(7, (M, K), -4, 4))
    Y = oracle.encode(workloads.uniform(8, (K, N), -4, 4))
    gx, gy = ctx.share(dev(X), 0, 51), ctx.share(dev(Y), 0, 52)
    t = ctx.dealer(m.TRIPLE_MATMUL, 9, 50, (M, N, K))
    zp = ctx.beaver_matmul(gx, gy, t, 0, "plain")
    zl = ctx.beaver_matmul(gx, gy, t, 0, "limb8")
    assert_pair(ctx, zl, pair(ctx, zp), "limb vs plain")
    r = host(ctx, ctx.reveal(zl))
    assert np.array_equal(r, oracle.as_ring(X) @ oracle.as_ring(Y))


def test_round_counters(m, ctx):
    say("round counters")
    before = ctx.stats()
    x = ctx.share(dev(rnd(1, (8, 8))), 0, 61)
    t = ctx.dealer(m.TRIPLE_MATMUL, 1, 60, (8, 8, 8))
    ctx.beaver_matmul(x, x, t, 16)
    ctx.truncate(x, 16)
    after = ctx.stats()
    assert after["opens"] - before["opens"] == 1
    assert after["open_bytes_per_party"] - before["open_bytes_per_party"] == 8 * (64 + 64)
    assert after["truncations"] - before["truncations"] == 2


# ------------------------------------------------------------------ conv1d
CONV_SMALL = [(2, 3, 17, 4, 5, 2), (1, 40, 100, 16, 48, 2), (2, 8, 30, 8, 7, 1),
              (1, 16, 40, 32, 1, 1), (4, 16, 300, 64, 7, 1),
              # shorter than the kernel (no output), as long (one output
              # position), stride 3 with a ragged tail, one channel in and out
              (2, 3, 4, 5, 7, 1), (3, 2, 9, 5, 9, 1), (2, 5, 50, 3, 4, 3), (1, 1, 64, 1, 3, 2)]


@pytest.mark.parametrize("form", ["plain", "limb8", "fp64limb"])
@pytest.mark.parametrize("Bt,Cin,L,Cout,k,s", CONV_SMALL)
def test_beaver_conv1d(m, ctx, form, Bt, Cin, L, Cout, k, s):
    say(f"beaver conv1d {form} {(Bt, Cin, L, Cout, k, s)}")
    X = oracle.encode(workloads.uniform(L, (Bt, Cin, L), -2, 2))
    W = oracle.encode(workloads.uniform(k, (Cout, Cin, k), -2, 2))
    xs, ws = oracle.share(X, 0, SEED, 71), oracle.share(W, 1, SEED, 72)
    dims = (Bt, Cin, L, Cout, k, s)
    t = ctx.dealer(m.TRIPLE_CONV1D, 3004, 70, dims)
    wt = oracle.dealer_conv1d(3004, 70, *dims)
    for g, e in [(t.a0, wt.a[0]), (t.a1, wt.a[1]), (t.b0, wt.b[0]), (t.b1, wt.b[1]), (t.c0, wt.c[0]),
                 (t.c1, wt.c[1])]:
        assert np.array_equal(host(ctx, g), e)
    z = ctx.beaver_conv1d(ctx.share(dev(X), 0, 71), ctx.share(dev(W), 1, 72), t, s, 16, form)
    want = oracle.beaver_conv1d(xs, ws, wt, s, 16)
    assert_pair(ctx, z, want, "beaver conv1d")


# ------------------------------------------------------------------ graph capture
@pytest.mark.parametrize("M,N,K", [(96, 64, 160), (128, 64, 2048)])
def test_graph_replay_matches_eager(m, M, N, K):
    # capture needs a non-null stream for party 0: run this test on its own
    # stream.  The second shape has few tiles and a long k (split-K inside).
    say(f"graph replay {M}x{N}x{K}")
    side = torch.cuda.Stream()
    with torch.cuda.stream(side):
        c = m.Context(device=0, seed=SEED)
        X, Y = rnd(3, (M, K)), rnd(4, (K, N))
        gx, gy = c.share(dev(X), 0, 81), c.share(dev(Y), 0, 82)
        t = c.dealer(m.TRIPLE_MATMUL, 2, 80, (M, N, K))
        eager = pair(c, c.beaver_matmul(gx, gy, t, 16, "limb8"))
        out = m.SharedPair(c.empty((M, N)), c.empty((M, N)))
        c.beaver_matmul(gx, gy, t, 16, "limb8", out=out)  # sizes the workspace
        c.sync()
        c.graph_begin()
        c.beaver_matmul(gx, gy, t, 16, "limb8", out=out)
        c.truncate(gx, 0)  # a no-op call inside the capture
        g = c.graph_end()
        try:
            for rep in range(4):
                out.s0.zero_()
                out.s1.zero_()
                c.graph_launch(g)
                got = pair(c, out)
                assert np.array_equal(got[0], eager[0]), rep
                assert np.array_equal(got[1], eager[1]), rep
                # eager work between replays
                c.reveal(gx)
                c.sync()
        finally:
            m.Context.graph_destroy(g)
            c.close()


@pytest.mark.parametrize("M,N,K", [(64, 32, 128), (130, 70, 300)])
def test_graph_replay_plain_matches_eager(m, M, N, K):
    # the plain form from a graph: the single fused launch of a small product
    # (64x32x128), and the open + GEMM + split-K reduction of a larger one
    say(f"graph replay plain {M}x{N}x{K}")
    side = torch.cuda.Stream()
    with torch.cuda.stream(side):
        c = m.Context(device=0, seed=SEED)
        X, Y = rnd(5, (M, K)), rnd(6, (K, N))
        gx, gy = c.share(dev(X), 0, 83), c.share(dev(Y), 1, 84)
        t = c.dealer(m.TRIPLE_MATMUL, 2, 85, (M, N, K))
        eager = pair(c, c.beaver_matmul(gx, gy, t, 16, "plain"))
        want = oracle.beaver_matmul(oracle.share(X, 0, SEED, 83), oracle.share(Y, 1, SEED, 84),
                                    oracle.dealer_matmul(2, 85, M, N, K), 16)
        assert np.array_equal(eager[0], want[0]) and np.array_equal(eager[1], want[1])
        out = m.SharedPair(c.empty((M, N)), c.empty((M, N)))
        c.beaver_matmul(gx, gy, t, 16, "plain", out=out)  # sizes the workspace
        c.sync()
        c.graph_begin()
        c.beaver_matmul(gx, gy, t, 16, "plain", out=out)
        g = c.graph_end()
        try:
            for rep in range(4):
                out.s0.zero_()
                out.s1.zero_()
                c.graph_launch(g)
                got = pair(c, out)
                assert np.array_equal(got[0], eager[0]), rep
                assert np.array_equal(got[1], eager[1]), rep
                c.reveal(gx)  # eager work between replays
                c.sync()
        finally:
            m.Context.graph_destroy(g)
            c.close()


@pytest.mark.parametrize("n", [4096, 4097])
def test_beaver_mul_unaligned_views(m, ctx, n):
    # views starting one element in are only 8-byte aligned: the element-wise
    # kernels must take their scalar path and still match
    say(f"beaver mul/square on offset views n={n}")
    x = np.concatenate([EDGE, rnd(41, n + 1)])[: n + 1]
    y = rnd(42, n + 1)
    gx, gy = ctx.share(dev(x), 0, 91), ctx.share(dev(y), 1, 92)
    t = ctx.dealer(m.TRIPLE_MUL, 17, 93, (n + 1,))
    ts = m.TripleShares(*(v[1:] for v in (t.a0, t.a1, t.b0, t.b1, t.c0, t.c1)))
    xv = m.SharedPair(gx.s0[1:], gx.s1[1:])
    yv = m.SharedPair(gy.s0[1:], gy.s1[1:])
    out = m.SharedPair(ctx.empty((n + 1,))[1:], ctx.empty((n + 1,))[1:])
    z = ctx.beaver_mul(xv, yv, ts, 16, out=out)
    xs, ys = oracle.share(x, 0, SEED, 91), oracle.share(y, 1, SEED, 92)
    w = oracle.dealer_mul(17, 93, n + 1)
    sl = lambda p: (p[0][1:], p[1][1:])
    want = oracle.beaver_mul(sl(xs), sl(ys), oracle.Triple(sl(w.a), sl(w.b), sl(w.c)), 16)
    assert_pair(ctx, z, want, "beaver mul on views")
    sq = ctx.beaver_mul(xv, None, ts, 16, out=out)
    wsq = oracle.beaver_square(sl(xs), oracle.Triple(sl(w.a), sl(w.b)), 16)
    assert_pair(ctx, sq, wsq, "beaver square on views")


@pytest.mark.parametrize("variant", [0, 1, 2, 3, 4, 5, 6, 7, 8, 9, 10, 11, 12, 13, 14, 15])
@pytest.mark.parametrize("group_m,remap", [(1, False), (8, True)])
def test_limb_tile_variants(m, variant, group_m, remap):
    # every tile shape and schedule of the limb GEMM gives the oracle's result
    say(f"limb tile variant {variant} group_m={group_m} remap={remap}")
    c = m.Context(device=0, seed=SEED)
    c.set_default_tile_config(variant, group_m, remap)
    # the last shape's Beaver finish concatenates 2K = 18000 > 16320 (K chunks)
    # over few tiles (split-K)
    for (M, N, K) in [(200, 136, 70), (64, 64, 64), (1, 300, 33), (513, 65, 260), (130, 260, 1100),
                      (96, 64, 9000)]:
        A, B = rnd(M + variant, (M, K)), rnd(N + 7, (K, N))
        Cl = c.ring_gemm(dev(A), dev(B), "limb8")
        assert np.array_equal(host(c, Cl), oracle.ring_gemm(A, B)), (M, N, K)
        X, Y = rnd(M + 1, (M, K)), rnd(N + 2, (K, N))
        t = c.dealer(m.TRIPLE_MATMUL, 3, 9, (M, N, K))
        gx, gy = c.share(dev(X), 0, 1), c.share(dev(Y), 1, 2)
        zl = c.beaver_matmul(gx, gy, t, 16, "limb8")
        want = oracle.beaver_matmul(oracle.share(X, 0, SEED, 1), oracle.share(Y, 1, SEED, 2),
                                    oracle.dealer_matmul(3, 9, M, N, K), 16)
        got = pair(c, zl)
        assert np.array_equal(got[0], want[0]) and np.array_equal(got[1], want[1]), (M, N, K)
    c.close()


def test_autotune_grouped_and_cache(m, tmp_path):
    say("autotune grouped")
    c = m.Context(device=0, seed=SEED)
    shapes = [(300, 120, 500), (40, 600, 64), (128, 128, 128), (17, 33, 2000)]
    best = c.autotune_matmul(shapes)
    assert best["variant"] in m.TILE_VARIANTS.values() and best["ms"] > 0
    probs, outs_plain = [], []
    for i, (M, N, K) in enumerate(shapes):
        X, Y = rnd(3 * i, (M, K)), rnd(3 * i + 1, (K, N))
        x = c.share(dev(X), 0, 2 * i)
        y = c.share(dev(Y), 1, 2 * i + 1)
        t = c.dealer(m.TRIPLE_MATMUL, 5, i, (M, N, K))
        probs.append((x, y, t))
        want = oracle.beaver_matmul(oracle.share(X, 0, SEED, 2 * i), oracle.share(Y, 1, SEED, 2 * i + 1),
                                    oracle.dealer_matmul(5, i, M, N, K), 16)
        outs_plain.append(m.SharedPair(dev(want[0]), dev(want[1])))
    zs = c.beaver_matmul_grouped(probs, 16, "limb8")  # uses the tuned schedules
    c.sync()
    for z, zp in zip(zs, outs_plain):
        assert torch.equal(z.s0, zp.s0) and torch.equal(z.s1, zp.s1)
    path = tmp_path / "tuned.txt"
    c.autotune_save(path)
    # one line: the shape list's hash and three classes' (variant, group_m, remap)
    assert len(open(path).read().split()) == 10
    c2 = m.Context(device=0, seed=SEED)
    c2.autotune_load(path)
    zs2 = c2.beaver_matmul_grouped(probs, 16, "limb8")
    c2.sync()
    for z, zp in zip(zs2, outs_plain):
        assert torch.equal(z.s0, zp.s0) and torch.equal(z.s1, zp.s1)
    c2.close()
    c.close()


def test_grouped_tile_classes(m):
    # thin products take the thin tiles: untuned, every problem runs in one
    # launch of the classes schedule with its own tile class (64x64, 32x128,
    # 128x32); an explicit default schedule applies to every problem (the
    # classes schedules, one-shot and persistent, each problem in its own
    # class); the results are the oracle's either way
    say("grouped tile classes")
    c = m.Context(device=0, seed=SEED)
    shapes = [(300, 120, 500), (17, 200, 300), (150, 20, 260), (9, 5, 70)]  # regular, thin M, thin N, thin M
    probs, wants = [], []
    for i, (M, N, K) in enumerate(shapes):
        X, Y = rnd(50 + 2 * i, (M, K)), rnd(51 + 2 * i, (K, N))
        probs.append((c.share(dev(X), 0, 30 + 2 * i), c.share(dev(Y), 1, 31 + 2 * i),
                      c.dealer(m.TRIPLE_MATMUL, 6, i, (M, N, K))))
        wants.append(oracle.beaver_matmul(oracle.share(X, 0, SEED, 30 + 2 * i), oracle.share(Y, 1, SEED, 31 + 2 * i),
                                          oracle.dealer_matmul(6, i, M, N, K), 16))
    for explicit in [None, 5, 14, 15]:
        if explicit is not None:
            c.set_default_tile_config(explicit, 8, True)
        c.sync()
        c.profile(True)
        c.profile_read()
        zs = c.beaver_matmul_grouped(probs, 16, "limb8")
        c.sync()
        assert c.profile_read()["limb8"]["launches"] == 1, explicit
        c.profile(False)
        for z, w in zip(zs, wants):
            got = pair(c, z)
            assert np.array_equal(got[0], w[0]) and np.array_equal(got[1], w[1])
    c.close()


@pytest.mark.parametrize("form", ["plain", "limb8"])
def test_grouped_with_empty_products(m, form):
    # a grouped call holding products with no rows, no columns, or no k beside
    # a tiny one and ones whose edges run as strips: the empty ones do
    # nothing (their outputs are left as they were), the others give the
    # oracle's result, under the default and both classes schedules
    say(f"grouped with empty products ({form})")
    c = m.Context(device=0, seed=SEED)
    shapes = [(0, 17, 40), (33, 0, 40), (1, 1, 1), (200, 136, 70), (33, 17, 0), (520, 65, 96), (0, 0, 0)]
    probs, wants = [], []
    for i, (M, N, K) in enumerate(shapes):
        X, Y = rnd(80 + 2 * i, (M, K)), rnd(81 + 2 * i, (K, N))
        probs.append((c.share(dev(X), 0, 90 + 2 * i), c.share(dev(Y), 1, 91 + 2 * i),
                      c.dealer(m.TRIPLE_MATMUL, 9, i, (M, N, K))))
        wants.append(oracle.beaver_matmul(oracle.share(X, 0, SEED, 90 + 2 * i), oracle.share(Y, 1, SEED, 91 + 2 * i),
                                          oracle.dealer_matmul(9, i, M, N, K), 16))
    for explicit in ([None, 14, 15] if form == "limb8" else [None]):
        if explicit is not None:
            c.set_default_tile_config(explicit, 8, True)
        zs = c.beaver_matmul_grouped(probs, 16, form)
        for (M, N, K), z, w in zip(shapes, zs, wants):
            assert z.s0.shape == (M, N)
            got = pair(c, z)
            assert np.array_equal(got[0], w[0]) and np.array_equal(got[1], w[1]), (form, explicit, (M, N, K))
    c.close()


# ------------------------------------------------------------------ plain split-K
@pytest.mark.parametrize("form", ["plain", "limb8"])
@pytest.mark.parametrize("M,N,K", [(5, 7, 5000), (128, 10, 2048), (1, 1, 3000), (130, 70, 777),
                                   (128, 1024, 1568), (40, 24, 20000)])
def test_ring_gemm_split_k(m, ctx, form, M, N, K):
    # few output tiles and a long k: the launch splits k into slices
    say(f"ring gemm {form} split-k {M}x{N}x{K}")
    A, B = rnd(M + 3 * K, (M, K)), rnd(N + 5 * K, (K, N))
    C = ctx.ring_gemm(dev(A), dev(B), form=form)
    assert np.array_equal(host(ctx, C), oracle.ring_gemm(A, B))


@pytest.mark.parametrize("form", ["plain", "limb8"])
@pytest.mark.parametrize("trunc", [0, 16])
def test_beaver_matmul_split_k(m, ctx, form, trunc):
    # the MLP's last layer shape: 128 x 10 outputs over 2 x 1024 concatenated k
    M, N, K = 128, 10, 1024
    say(f"beaver matmul {form} split-k trunc={trunc}")
    X = oracle.encode(workloads.uniform(91, (M, K), -1, 1))
    Y = oracle.encode(workloads.uniform(92, (K, N), -1, 1))
    xs, ys = oracle.share(X, 0, SEED, 93), oracle.share(Y, 1, SEED, 94)
    t = ctx.dealer(m.TRIPLE_MATMUL, 3002, 95, (M, N, K))
    z = ctx.beaver_matmul(ctx.share(dev(X), 0, 93), ctx.share(dev(Y), 1, 94), t, trunc, form)
    want = oracle.beaver_matmul(xs, ys, oracle.dealer_matmul(3002, 95, M, N, K), trunc)
    assert_pair(ctx, z, want, f"beaver matmul {form} split-k")


def test_live_graph_pins_workspace(m):
    # while a captured graph exists the workspace cannot move: a call needing a
    # larger one is refused, and works again once the graph is destroyed
    say("graph pins workspace")
    side = torch.cuda.Stream()
    with torch.cuda.stream(side):
        c = m.Context(device=0, seed=SEED)
        try:
            M, N, K = 64, 64, 64
            gx = c.share(dev(rnd(5, (M, K))), 0, 1)
            gy = c.share(dev(rnd(6, (K, N))), 1, 2)
            t = c.dealer(m.TRIPLE_MATMUL, 2, 3, (M, N, K))
            out = m.SharedPair(c.empty((M, N)), c.empty((M, N)))
            # a large product's inputs (its dealer call grows the workspace a
            # little, less than the product itself will need)
            big = 1024
            bx = c.share(dev(rnd(7, (big, big))), 0, 4)
            by = c.share(dev(rnd(8, (big, big))), 1, 5)
            bt = c.dealer(m.TRIPLE_MATMUL, 2, 6, (big, big, big))
            c.beaver_matmul(gx, gy, t, 16, "limb8", out=out)
            c.sync()
            c.graph_begin()
            c.beaver_matmul(gx, gy, t, 16, "limb8", out=out)
            g = c.graph_end()
            with pytest.raises(m.MPCError) as e:
                c.beaver_matmul(bx, by, bt, 16, "limb8")
            assert e.value.status == -4
            c.graph_launch(g)
            m.Context.graph_destroy(g)
            z = c.beaver_matmul(bx, by, bt, 16, "limb8")
            c.sync()
            assert z.s0.shape == (big, big)
        finally:
            c.close()


def test_default_tile_config_roundtrip(m):
    c = m.Context(device=0, seed=SEED)
    assert c.default_tile_config() == {"variant": "lds64x64", "variant_id": 5, "group_m": 8, "xcd_remap": True}
    c.set_default_tile_config(1, 4, False)
    assert c.default_tile_config() == {"variant": "64x128", "variant_id": 1, "group_m": 4, "xcd_remap": False}
    for bad in (len(m.TILE_VARIANTS), -1):
        with pytest.raises(m.MPCError):
            c.set_default_tile_config(bad, 8, True)
    c.close()
