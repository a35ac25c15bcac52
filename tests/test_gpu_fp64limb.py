"""GPU parity of the fp64 limb form (the paper's own GPU method, Section 5.3):
ring GEMM and Beaver matmul against the CPU oracle, bit for bit, on both limb
splits (three 22-bit limbs below 1024 summed k, four 16-bit limbs above), with
limb values at the extremes of each split."""
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
    # convolution has no fp64 limb path
    b, cin, L, cout, k = 1, 2, 8, 3, 3
    x = ctx.share(dev(rnd(1, (b, cin, L))), 0, 1)
    w = ctx.share(dev(rnd(2, (cout, cin, k))), 1, 2)
    t = ctx.dealer(m.TRIPLE_CONV1D, 7, 3, (b, cin, L, cout, k, 1))
    with pytest.raises(m.MPCError) as e:
        ctx.beaver_conv1d(x, w, t, 1, 0, FORM)
    assert e.value.status == -6
