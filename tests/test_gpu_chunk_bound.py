"""Worst-case limbs at the int32 chunk bound of the limb form (section 5.3:
the ring product is exact only while every partial sum stays exact).

The value 0x7F7F7F7F7F7F7F80 has all eight signed 8-bit limbs equal to -128
and 0x7F7F7F7F7F7F7F7F all equal to +127.  With every limb -128, each of the
up to 8 limb products of a diagonal adds 2^14 per k, the largest possible
step, so a chunk of 16320 k brings a diagonal sum to 8 * 16320 * 2^14 =
2^31 - 2^21, just below the int32 limit.  Shapes are chosen with at least as
many output tiles as compute units, so the k range runs as consecutive
launches that add into the output (no split-K); a one-tile shape covers the
split-K path.  Expected values: all-equal operands give the closed form
C = K * v * w (mod 2^64) at every output; mixed operands are checked against
the oracle at sampled outputs."""
import numpy as np
import pytest
import torch

import oracle
import workloads
from tests.gpu_util import dev, host, say

pytestmark = pytest.mark.gpu
NEG = np.uint64(0x7F7F7F7F7F7F7F80)  # every limb -128
POS = np.uint64(0x7F7F7F7F7F7F7F7F)  # every limb +127
BOUND = 16320


@pytest.fixture(scope="module")
def m():
    import paper_2109_00984_amd as mod
    return mod


@pytest.fixture(scope="module")
def ctx(m):
    c = m.Context(device=0, seed=77)
    yield c
    c.close()


def test_limb_values():
    d = oracle.limbs(np.array([NEG, POS], dtype=np.uint64))
    assert (d[0] == -128).all() and (d[1] == 127).all()


def mixed(seed, shape):
    g = workloads.rng(seed)
    return np.where(g.integers(0, 2, size=shape) == 1, NEG, POS).astype(np.uint64)


def closed_form(K, v, w):
    return np.uint64((int(K) * int(v) * int(w)) % (1 << 64))


@pytest.mark.parametrize("M,N,K", [(2048, 2048, BOUND), (2048, 2048, BOUND + 1), (2048, 2048, 2 * BOUND + 1),
                                   (64, 64, 2 * BOUND + 1)])
def test_ring_gemm_all_minus128(m, ctx, M, N, K):
    say(f"chunk bound: ring GEMM {M}x{N}x{K}, every limb -128")
    A = torch.full((M, K), int(NEG.view(np.int64)), dtype=torch.int64, device=ctx.device)
    B = torch.full((K, N), int(NEG.view(np.int64)), dtype=torch.int64, device=ctx.device)
    C = host(ctx, ctx.ring_gemm(A, B, "limb8"))
    assert (C == closed_form(K, NEG, NEG)).all()


@pytest.mark.parametrize("M,N,K", [(2048, 2048, BOUND), (2048, 2048, BOUND + 1), (2048, 2048, 2 * BOUND + 1),
                                   (64, 64, 2 * BOUND + 1)])
def test_ring_gemm_mixed_extremes(m, ctx, M, N, K):
    say(f"chunk bound: ring GEMM {M}x{N}x{K}, limbs -128 and +127 mixed")
    Ah, Bh = mixed(11 + K, (M, K)), mixed(12 + K, (K, N))
    C = host(ctx, ctx.ring_gemm(dev(Ah), dev(Bh), "limb8"))
    g = workloads.rng(K)
    rows, cols = g.integers(0, M, size=64), g.integers(0, N, size=64)
    rows[:2], cols[:2] = [0, M - 1], [0, N - 1]
    assert np.array_equal(C[rows, cols], oracle.ring_gemm_at(Ah, Bh, rows, cols))


@pytest.mark.parametrize("M,N,K", [(2048, 2048, 8200), (2048, 2048, BOUND + 1), (64, 64, 8200)])
def test_beaver_matmul_worst_limbs(m, ctx, M, N, K):
    """A Beaver matmul whose concatenated 2K crosses the chunk bound, with
    shares and a hand-built triple chosen so that every packed operand of
    both parties' finish ([eps | a_0 + eps | a_1] and [b_0 | b_1 | delta])
    holds only -128 limbs: x_0 = 2v, x_1 = 0, a_0 = 0, a_1 = v give eps = v
    and a_0 + eps = v; y_0 = 3v, y_1 = 0, b_0 = b_1 = v give delta = v.
    The Beaver identity holds for any triple, so the oracle computes the same
    shares from the same inputs."""
    say(f"chunk bound: Beaver matmul {M}x{N}x{K}, every packed limb -128, truncation 16")
    v = int(NEG)
    enc = lambda u: np.uint64(u % (1 << 64))
    full = lambda shape, u: np.full(shape, enc(u), dtype=np.uint64)
    x = (full((M, K), 2 * v), full((M, K), 0))
    y = (full((K, N), 3 * v), full((K, N), 0))
    a = (full((M, K), 0), full((M, K), v))
    b = (full((K, N), v), full((K, N), v))
    g = workloads.rng(K + 5)
    cc = (workloads.uniform_u64(K + 6, (M, N)), workloads.uniform_u64(K + 7, (M, N)))
    t = m.TripleShares(dev(a[0]), dev(a[1]), dev(b[0]), dev(b[1]), dev(cc[0]), dev(cc[1]))
    xs, ys = m.SharedPair(dev(x[0]), dev(x[1])), m.SharedPair(dev(y[0]), dev(y[1]))
    z = ctx.beaver_matmul(xs, ys, t, 16, "limb8")
    got = (host(ctx, z.s0), host(ctx, z.s1))
    rows, cols = g.integers(0, M, size=64), g.integers(0, N, size=64)
    rows[:2], cols[:2] = [0, M - 1], [0, N - 1]
    c_at = (cc[0][rows, cols], cc[1][rows, cols])
    want = oracle.beaver_matmul_at(x, y, a, b, c_at, 16, rows, cols)
    assert np.array_equal(got[0][rows, cols], want[0]) and np.array_equal(got[1][rows, cols], want[1])


@pytest.mark.parametrize("sched", [14, 15])
def test_ring_gemm_chunked_with_edge_strips(m, sched):
    # the classes schedules split a product whose last rows and columns fill
    # at most half a 64-wide tile into a 64x64 interior, two strips and a
    # corner; with k past the chunk bound each region adds its second chunk
    # into its own part of the output: every limb -128 gives the closed form
    # at every output, strips and corner included
    M, N, K = 2056, 2056, BOUND + 1
    say(f"chunk bound with edge strips: schedule {sched}, ring GEMM {M}x{N}x{K}")
    assert len(m.limb_plan(M, N, sched)[1]) == 4
    c = m.Context(device=0, seed=79)
    try:
        c.set_default_tile_config(sched, 8, True)
        A = torch.full((M, K), int(NEG.view(np.int64)), dtype=torch.int64, device=c.device)
        B = torch.full((K, N), int(NEG.view(np.int64)), dtype=torch.int64, device=c.device)
        c.profile(True)
        c.profile_read()
        C = host(c, c.ring_gemm(A, B, "limb8"))
        assert c.profile_read()["limb8"]["launches"] == 2  # the two k chunks, one launch each
        assert (C == closed_form(K, NEG, NEG)).all()
    finally:
        c.close()
