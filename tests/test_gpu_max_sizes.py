"""GPU parity at the largest sizes: element counts past 2^31, where 32-bit
index arithmetic would wrap; a Beaver matmul whose left operand holds more
than 2^31 elements; and the longest k segment the limb form addresses, with
the next length up rejected by the limb form and taken by the plain one.
Large outputs are compared with the oracle on sampled elements and rows that
it computes one by one (sharing and triples are counter-based, section 5.1
and App. C.1.1, so any element can be drawn alone); the reveal of a sharing
is also checked over every element.

Inputs past 2^31 elements repeat a seeded vector of length 2^20 + 7, which
does not divide 2^32, so an index that wrapped would read another value."""
import numpy as np
import pytest
import torch

import oracle
import workloads
from tests.gpu_util import dev, say

pytestmark = pytest.mark.gpu

SEED = 4242
BIG = (1 << 31) + 37
PERIOD = (1 << 20) + 7
GIB = 1 << 30
LIMB_MAX_SEG_K = 65534 * 32  # longest k segment of the limb form (include/mpc.h)


@pytest.fixture(scope="module")
def m():
    import paper_2109_00984_amd as mod
    return mod


@pytest.fixture(scope="module")
def ctx(m):
    torch.cuda.empty_cache()
    c = m.Context(device=0, seed=SEED)
    yield c
    c.sync()
    c.close()
    torch.cuda.empty_cache()


def need(nbytes):
    torch.cuda.empty_cache()
    free, _ = torch.cuda.mem_get_info()
    if free < nbytes:
        pytest.skip(f"needs {nbytes / GIB:.0f} GiB of free device memory, {free / GIB:.0f} free")


def tiled(base, n):
    """Device vector of n elements whose element i is base[i % base.size]."""
    reps = -(-n // base.size)
    return dev(base).repeat(reps)[:n]


def sample_idx(n, seed, count=2000):
    fixed = [0, 1, (1 << 31) - 1, 1 << 31, (1 << 31) + 1, (1 << 32) - 1, n - 1]
    rnd = np.random.default_rng(seed).integers(0, n, size=count, dtype=np.int64)
    return np.unique(np.concatenate([np.array([i for i in fixed if i < n], dtype=np.int64), rnd]))


def gather(ctx, t, idx):
    """Elements idx of a device tensor (flat index), as uint64 on the host."""
    ctx.sync()
    return t.reshape(-1)[torch.from_numpy(idx).to(t.device)].cpu().numpy().view(np.uint64)


def same(ctx, got, idx, want, what):
    g = gather(ctx, got, idx)
    bad = np.flatnonzero(g != want)
    assert bad.size == 0, f"{what}: {bad.size} of {idx.size} sampled elements differ, first at {idx[bad[0]]}"


def test_share_reveal_square_truncate_past_2_31(m, ctx):
    n = BIG
    need(11 * n * 8)
    say(f"max size: share, reveal, Beaver square, truncate over n={n}")
    base = workloads.uniform_u64(SEED + 1, (PERIOD,))
    x = tiled(base, n)
    idx = sample_idx(n, 1)
    uidx = idx.astype(np.uint64)
    xs = oracle.share_at(base[idx % PERIOD], uidx, 0, SEED, 21)
    s = ctx.share(x, 0, 21)
    same(ctx, s.s0, idx, xs[0], "share, party 0")
    same(ctx, s.s1, idx, xs[1], "share, party 1")
    r = ctx.reveal(s)
    ctx.sync()
    assert torch.equal(r, x), "reveal differs from the shared vector"
    del r, x
    tp = ctx.dealer(m.TRIPLE_SQUARE, 3101, 22, (n,))
    wt = oracle.dealer_square_at(3101, 22, uidx)
    for name, got, want in (("a0", tp.a0, wt.a[0]), ("a1", tp.a1, wt.a[1]), ("b0", tp.b0, wt.b[0]),
                            ("b1", tp.b1, wt.b[1])):
        same(ctx, got, idx, want, f"square pair {name}")
    z = ctx.beaver_mul(s, None, tp, 16)
    wz = oracle.beaver_square(xs, wt, 16)
    same(ctx, z.s0, idx, wz[0], "Beaver square, party 0")
    same(ctx, z.s1, idx, wz[1], "Beaver square, party 1")
    ctx.truncate(z, 5)
    same(ctx, z.s0, idx, oracle.truncate(wz[0], 5), "truncate, party 0")
    same(ctx, z.s1, idx, oracle.truncate(wz[1], 5), "truncate, party 1")
    ctx.sync()
    del s, tp, z


def test_beaver_mul_past_2_31(m, ctx):
    n = BIG
    need(13 * n * 8)
    say(f"max size: Beaver product over n={n}")
    bx = workloads.uniform_u64(SEED + 2, (PERIOD,))
    by = workloads.uniform_u64(SEED + 3, (PERIOD,))
    idx = sample_idx(n, 2)
    uidx = idx.astype(np.uint64)
    x = tiled(bx, n)
    xs = ctx.share(x, 1, 23)
    ctx.sync()
    del x
    y = tiled(by, n)
    ys = ctx.share(y, 0, 24)
    ctx.sync()
    del y
    torch.cuda.empty_cache()
    t = ctx.dealer(m.TRIPLE_MUL, 3102, 25, (n,))
    z = ctx.beaver_mul(xs, ys, t, 16)
    want = oracle.beaver_mul(oracle.share_at(bx[idx % PERIOD], uidx, 1, SEED, 23),
                             oracle.share_at(by[idx % PERIOD], uidx, 0, SEED, 24),
                             oracle.dealer_mul_at(3102, 25, uidx), 16)
    same(ctx, z.s0, idx, want[0], "Beaver product, party 0")
    same(ctx, z.s1, idx, want[1], "Beaver product, party 1")
    ctx.sync()
    del xs, ys, t, z


def test_beaver_matmul_left_operand_past_2_31(m, ctx):
    # x is M x K with M * K > 2^31; row 65530 straddles flat index 2^31
    M, N, K = 65539, 8, 32771
    assert M * K > (1 << 31) and 65530 * K < (1 << 31) < 65531 * K
    need(10 * M * K * 8)
    say(f"max size: Beaver matmul {M}x{N}x{K} (left operand {M * K} elements)")
    base = workloads.uniform_u64(SEED + 4, (PERIOD,))
    Y = workloads.uniform_u64(SEED + 5, (K, N))
    X = tiled(base, M * K).view(M, K)
    xs = ctx.share(X, 0, 26)
    ctx.sync()
    del X
    torch.cuda.empty_cache()
    ys = ctx.share(dev(Y), 1, 27)
    t = ctx.dealer(m.TRIPLE_MATMUL, 3103, 28, (M, N, K))
    rows = np.array([0, 1, 4097, 65530, 65531, M - 1], dtype=np.int64)
    flat = (rows[:, None] * K + np.arange(K, dtype=np.int64)[None, :]).ravel()
    wx = oracle.share_at(base[flat % PERIOD], flat.astype(np.uint64), 0, SEED, 26)
    wx = (wx[0].reshape(rows.size, K), wx[1].reshape(rows.size, K))
    wy = oracle.share(Y, 1, SEED, 27)
    wt = oracle.dealer_matmul_rows(3103, 28, N, K, rows)
    same(ctx, xs.s0, flat, wx[0].ravel(), "share of x, party 0")
    same(ctx, xs.s1, flat, wx[1].ravel(), "share of x, party 1")
    same(ctx, t.a0, flat, wt.a[0].ravel(), "triple a0")
    same(ctx, t.a1, flat, wt.a[1].ravel(), "triple a1")
    cidx = (rows[:, None] * N + np.arange(N, dtype=np.int64)[None, :]).ravel()
    same(ctx, t.c0, cidx, wt.c[0].ravel(), "triple c0")
    same(ctx, t.c1, cidx, wt.c[1].ravel(), "triple c1")
    bidx = np.arange(K * N, dtype=np.int64)
    same(ctx, t.b0, bidx, wt.b[0].ravel(), "triple b0")
    same(ctx, t.b1, bidx, wt.b[1].ravel(), "triple b1")
    want = oracle.beaver_matmul(wx, wy, wt, 16)
    z = None
    for form in ("limb8", "plain"):
        say(f"  form {form}")
        z = ctx.beaver_matmul(xs, ys, t, 16, form=form, out=z)
        same(ctx, z.s0, cidx, want[0].ravel(), f"Beaver matmul ({form}), party 0")
        same(ctx, z.s1, cidx, want[1].ravel(), f"Beaver matmul ({form}), party 1")
    ctx.sync()
    del xs, ys, t, z


# ------------------------------------------------------------------ longest limb k segment
@pytest.fixture(scope="module")
def long_k():
    """Beaver matmul 3 x 5 with k at the limb form's limit, and its oracle result."""
    M, N, K = 3, 5, LIMB_MAX_SEG_K
    X = workloads.uniform_u64(SEED + 6, (M, K))
    Y = workloads.uniform_u64(SEED + 7, (K, N))
    xs, ys = oracle.share(X, 0, SEED, 31), oracle.share(Y, 1, SEED, 32)
    want = oracle.beaver_matmul(xs, ys, oracle.dealer_matmul(3104, 33, M, N, K), 16)
    return X, Y, want


@pytest.mark.parametrize("variant", [0, 3, 5, 7, 9, 10])
def test_longest_limb_k_segment(m, long_k, variant):
    X, Y, want = long_k
    M, K = X.shape
    N = Y.shape[1]
    say(f"max size: limb Beaver matmul {M}x{N}x{K}, tile variant {variant}")
    with m.Context(device=0, seed=SEED) as c:
        c.set_default_tile_config(variant, 8, True)
        xs, ys = c.share(dev(X), 0, 31), c.share(dev(Y), 1, 32)
        t = c.dealer(m.TRIPLE_MATMUL, 3104, 33, (M, N, K))
        z = c.beaver_matmul(xs, ys, t, 16, form="limb8")
        c.sync()
        assert np.array_equal(z.s0.cpu().numpy().view(np.uint64), want[0])
        assert np.array_equal(z.s1.cpu().numpy().view(np.uint64), want[1])


def test_limb_k_segment_past_limit(m, ctx):
    M, N, K = 2, 3, LIMB_MAX_SEG_K + 1
    say(f"max size: k = {K} past the limb form's limit")
    X = workloads.uniform_u64(SEED + 8, (M, K))
    Y = workloads.uniform_u64(SEED + 9, (K, N))
    xs, ys = ctx.share(dev(X), 0, 34), ctx.share(dev(Y), 1, 35)
    t = ctx.dealer(m.TRIPLE_MATMUL, 3105, 36, (M, N, K))
    for call in (lambda: ctx.beaver_matmul(xs, ys, t, 16, form="limb8"),
                 lambda: ctx.ring_gemm(xs.s0, ys.s0, form="limb8")):
        with pytest.raises(m.MPCError) as e:
            call()
        assert e.value.status == -6
    z = ctx.beaver_matmul(xs, ys, t, 16, form="auto")
    C = ctx.ring_gemm(xs.s0, ys.s0, form="auto")
    ctx.sync()
    wx, wy = oracle.share(X, 0, SEED, 34), oracle.share(Y, 1, SEED, 35)
    want = oracle.beaver_matmul(wx, wy, oracle.dealer_matmul(3105, 36, M, N, K), 16)
    assert np.array_equal(z.s0.cpu().numpy().view(np.uint64), want[0])
    assert np.array_equal(z.s1.cpu().numpy().view(np.uint64), want[1])
    assert np.array_equal(C.cpu().numpy().view(np.uint64), oracle.ring_gemm(wx[0], wy[0]))
