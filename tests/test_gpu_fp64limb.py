"""GPU parity of the fp64 limb form (the paper's own GPU method, Section 5.3):
ring GEMM and Beaver matmul against the CPU oracle, bit for bit, on both limb
splits (three 22-bit limbs below 1024 summed k, four 16-bit limbs above), with
limb values at the extremes of each split; k = 0; replay from a HIP graph.
(Its convolution runs with the other forms' in test_gpu_parity.py.)"""
import numpy as np
import pytest

import oracle
import workloads
from tests.gpu_util import dev, host, pair, say

pytestmark = pytest.mark.gpu

SEED = 2025
FORM = "fp64limb"


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


# values whose limbs sit at the ends of their ranges:
#   16-bit split (bias 0x8000800080008000): all limbs -2^15, all limbs 2^15-1
#   22-bit split (bias 2^21 + 2^43): low limbs -2^21 with the top (20-bit) limb 0 or 2^20-1
EXTREMES16 = [0x7FFF7FFF7FFF8000, 0x7FFF7FFF7FFF7FFF]
B22 = (1 << 21) + (1 << 43)
EXTREMES22 = [(0 - B22) % (1 << 64), (((1 << 20) - 1) << 44) - B22, (1 << 64) - 1 - B22]


@pytest.mark.parametrize("M,N,K", [(1, 1, 1), (37, 53, 70), (129, 65, 1023), (64, 48, 1024),
                                   (100, 70, 3000), (5, 300, 17)])
def test_ring_gemm_fp64limb(m, ctx, M, N, K):
    say(f"ring gemm fp64limb {M}x{N}x{K}")
    A, B = rnd(M * 5 + K, (M, K)), rnd(N * 3 + K, (K, N))
    ext = EXTREMES22 if K < 1024 else EXTREMES16
    A.ravel()[: len(ext)] = ext[: A.size]
    B.ravel()[: len(ext)] = ext[: B.size]
    C = ctx.ring_gemm(dev(A), dev(B), form=FORM)
    assert np.array_equal(host(ctx, C), oracle.ring_gemm(A, B))


@pytest.mark.parametrize("K,vals", [(1023, EXTREMES22), (4096, EXTREMES16)])
def test_ring_gemm_fp64limb_worst_case_sums(m, ctx, K, vals):
    # every k contributes the largest products the split allows: the per-diagonal
    # float64 sums come closest to 2^53 here
    M = N = 32
    for va in vals:
        for vb in vals:
            say(f"ring gemm fp64limb extremes K={K} {va:#x} {vb:#x}")
            A = np.full((M, K), va, dtype=np.uint64)
            B = np.full((K, N), vb, dtype=np.uint64)
            C = ctx.ring_gemm(dev(A), dev(B), form=FORM)
            assert np.array_equal(host(ctx, C), oracle.ring_gemm(A, B))


@pytest.mark.parametrize("M,N,K", [(1, 1, 1), (64, 32, 128), (37, 53, 700), (129, 65, 600)])
@pytest.mark.parametrize("trunc", [0, 16])
def test_beaver_matmul_fp64limb(m, ctx, M, N, K, trunc):
    say(f"beaver matmul fp64limb {M}x{N}x{K} trunc={trunc}")
    X = oracle.encode(workloads.uniform(M + 7, (M, K), -4, 4))
    Y = oracle.encode(workloads.uniform(N + 8, (K, N), -4, 4))
    xs, ys = oracle.share(X, 0, SEED, 51), oracle.share(Y, 1, SEED, 52)
    t = ctx.dealer(m.TRIPLE_MATMUL, 3101, 60, (M, N, K))
    z = ctx.beaver_matmul(ctx.share(dev(X), 0, 51), ctx.share(dev(Y), 1, 52), t, trunc, FORM)
    want = oracle.beaver_matmul(xs, ys, oracle.dealer_matmul(3101, 60, M, N, K), trunc)
    g0, g1 = pair(ctx, z)
    assert np.array_equal(g0, want[0]) and np.array_equal(g1, want[1])


def test_fp64limb_matches_limb8_and_profiles(m, ctx):
    M, N, K = 96, 80, 2048
    A, B = rnd(11, (M, K)), rnd(12, (K, N))
    ctx.profile(True)
    ctx.profile_read()
    C1 = ctx.ring_gemm(dev(A), dev(B), form=FORM)
    C2 = ctx.ring_gemm(dev(A), dev(B), form="limb8")
    prof = ctx.profile_read()
    ctx.profile(False)
    assert np.array_equal(host(ctx, C1), host(ctx, C2))
    assert prof["fp64limb"]["launches"] == 1 and prof["fp64limb"]["ring_macs"] == M * N * K
    assert prof["limb8"]["launches"] == 1


def test_fp64limb_unsupported_cases(m, ctx):
    # summed k at the exactness bound of the 16-bit split
    K = 1 << 21
    A = dev(np.zeros((1, K), dtype=np.uint64))
    B = dev(np.zeros((K, 1), dtype=np.uint64))
    with pytest.raises(m.MPCError) as e:
        ctx.ring_gemm(A, B, form=FORM)
    assert e.value.status == -6


def test_fp64limb_k_zero(m, ctx):
    # an empty sum: the product is 0 and the epilogue still adds the triple share
    say("fp64limb k = 0")
    M, N = 7, 9
    t = ctx.dealer(m.TRIPLE_MATMUL, 3102, 61, (M, N, 0))
    x = ctx.share(dev(np.zeros((M, 0), dtype=np.uint64)), 0, 53)
    y = ctx.share(dev(np.zeros((0, N), dtype=np.uint64)), 1, 54)
    z = ctx.beaver_matmul(x, y, t, 16, FORM)
    want = oracle.beaver_matmul(oracle.share(np.zeros((M, 0), dtype=np.uint64), 0, SEED, 53),
                                oracle.share(np.zeros((0, N), dtype=np.uint64), 1, SEED, 54),
                                oracle.dealer_matmul(3102, 61, M, N, 0), 16)
    g0, g1 = pair(ctx, z)
    assert np.array_equal(g0, want[0]) and np.array_equal(g1, want[1])


def test_fp64limb_graph_replay(m):
    # the vendor BLAS GEMMs are recorded into a graph like the library's own
    # kernels once the context has created its BLAS handle eagerly; before
    # that, a captured fp64 call is refused and records nothing
    import torch
    with torch.cuda.stream(torch.cuda.Stream()):
        c = m.Context(device=0, seed=SEED)
        try:
            M, N, K = 72, 40, 300
            X = oracle.encode(workloads.uniform(81, (M, K), -4, 4))
            Y = oracle.encode(workloads.uniform(82, (K, N), -4, 4))
            x, y = c.share(dev(X), 0, 55), c.share(dev(Y), 1, 56)
            t = c.dealer(m.TRIPLE_MATMUL, 3103, 62, (M, N, K))
            out = m.SharedPair(c.empty((M, N)), c.empty((M, N)))
            c.sync()
            say("fp64limb capture before any eager fp64 call")
            c.graph_begin()
            with pytest.raises(m.MPCError) as e:
                c.beaver_matmul(x, y, t, 16, FORM, out=out)
            g = c.graph_end()
            g.destroy()
            assert e.value.status == -6
            eager = c.beaver_matmul(x, y, t, 16, FORM)
            c.sync()
            want = oracle.beaver_matmul(oracle.share(X, 0, SEED, 55), oracle.share(Y, 1, SEED, 56),
                                        oracle.dealer_matmul(3103, 62, M, N, K), 16)
            g0, g1 = pair(c, eager)
            assert np.array_equal(g0, want[0]) and np.array_equal(g1, want[1])
            say("fp64limb capture")
            c.graph_begin()
            c.beaver_matmul(x, y, t, 16, FORM, out=out)
            g = c.graph_end()
            try:
                for rep in range(3):
                    out.s0.fill_(-1)
                    out.s1.fill_(-1)
                    say(f"fp64limb replay {rep}")
                    c.graph_launch(g)
                    c.sync()
                    r0, r1 = pair(c, out)
                    assert np.array_equal(r0, want[0]) and np.array_equal(r1, want[1]), rep
                    c.ring_gemm(dev(X[:, :8]), dev(Y[:8, :]), form=FORM)  # eager work between replays
                    c.sync()
            finally:
                g.destroy()
        finally:
            c.close()
