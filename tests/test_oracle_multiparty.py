"""CPU pins of the oracle's sharing among more than two parties (App. C.1.1,
arithmetic secret sharing for |P| parties) and of its wrap-count truncation
(Algorithm 1, with eta set to 0 as the paper does).  Every expectation is
computed independently of the oracle's own arithmetic: Python integers,
numpy's uint64 products, the definition of the wrap count."""
import numpy as np
import pytest

import oracle

Q = 1 << 64
PARTIES = [2, 3, 5, 8]


def s64(v):
    v = int(v)
    return v - Q if v >= 1 << 63 else v


def reveal_int(shares, i):
    return sum(int(s.ravel()[i]) for s in shares) % Q


def rand_u64(rng, shape):
    return rng.integers(0, Q, size=shape, dtype=np.uint64)


@pytest.mark.parametrize("P", PARTIES)
def test_mp_share_reveal_roundtrip(P):
    rng = np.random.default_rng(P)
    x = np.concatenate([rand_u64(rng, 200),
                        np.array([0, 1, Q - 1, 1 << 63, (1 << 63) - 1], dtype=np.uint64)])
    for src in (0, P - 1):
        s = oracle.mp_share(x, P, src, seed=11 + P, tag=5)
        assert len(s) == P
        assert np.array_equal(oracle.mp_reveal(s), x)
        # the zero-share alone: sharing 0 reveals 0, and no single share is 0-valued
        z = oracle.mp_share(np.zeros(64, dtype=np.uint64), P, src, seed=11 + P, tag=6)
        assert not oracle.mp_reveal(z).any()
        for p in range(P):
            assert np.count_nonzero(z[p]) == 64


@pytest.mark.parametrize("P", PARTIES)
def test_mp_shares_are_balanced_bits(P):
    # every share of a fixed secret looks uniform: each bit set about half the time
    s = oracle.mp_share(np.full(4096, 0x1234, dtype=np.uint64), P, 0, seed=3, tag=9)
    for p in range(P):
        bits = np.unpackbits(s[p].view(np.uint8)).reshape(-1, 64).mean(axis=0)
        assert np.all(np.abs(bits - 0.5) < 0.06)


@pytest.mark.parametrize("P", PARTIES)
@pytest.mark.parametrize("square", [False, True])
def test_mp_dealer_elementwise(P, square):
    n = 300
    t = oracle.mp_dealer_mul(77, 4, P, n, square=square)
    for i in range(0, n, 7):
        a = reveal_int(t.a, i)
        b = reveal_int(t.b, i)
        if square:
            assert b == a * a % Q
        else:
            assert reveal_int(t.c, i) == a * b % Q


@pytest.mark.parametrize("P", PARTIES)
def test_mp_dealer_matmul(P):
    M, N, K = 5, 4, 7
    t = oracle.mp_dealer_matmul(78, 2, P, M, N, K)
    a = oracle.mp_reveal(t.a)
    b = oracle.mp_reveal(t.b)
    with np.errstate(over="ignore"):
        want = a @ b  # numpy wraps uint64 products and sums mod 2^64
    assert np.array_equal(oracle.mp_reveal(t.c), want)


def random_sharing(rng, P, shape):
    return [rand_u64(rng, shape) for _ in range(P)]


@pytest.mark.parametrize("P", PARTIES)
def test_mp_beaver_identity_any_triple(P):
    # shares and triple shares drawn at random (not from the dealer): the
    # identity holds for any triple with c = a*b
    rng = np.random.default_rng(100 + P)
    n = 64
    x, y = random_sharing(rng, P, n), random_sharing(rng, P, n)
    a, b = random_sharing(rng, P, n), random_sharing(rng, P, n)
    c = random_sharing(rng, P, n)
    av = oracle.mp_reveal(a)
    bv = oracle.mp_reveal(b)
    cv = oracle.mp_reveal(c)
    with np.errstate(over="ignore"):
        c[P - 1] = c[P - 1] - cv + av * bv  # fix the triple: c = a * b
    z = oracle.mp_beaver_mul(x, y, oracle.Triple(a, b, c))
    for i in range(n):
        assert reveal_int(z, i) == reveal_int(x, i) * reveal_int(y, i) % Q
    # square with the pair (a, a^2)
    bb = random_sharing(rng, P, n)
    bsum = oracle.mp_reveal(bb)
    with np.errstate(over="ignore"):
        bb[0] = bb[0] - bsum + av * av
    z2 = oracle.mp_beaver_mul(x, None, oracle.Triple(a, bb, None))
    for i in range(n):
        assert reveal_int(z2, i) == reveal_int(x, i) ** 2 % Q


@pytest.mark.parametrize("P", PARTIES)
def test_mp_beaver_matmul_identity(P):
    rng = np.random.default_rng(200 + P)
    M, N, K = 6, 5, 9
    x, y = random_sharing(rng, P, (M, K)), random_sharing(rng, P, (K, N))
    t = oracle.mp_dealer_matmul(91, 1, P, M, N, K)
    z = oracle.mp_beaver_matmul(x, y, t)
    xv, yv = oracle.mp_reveal(x), oracle.mp_reveal(y)
    for i in range(M):
        for j in range(N):
            want = sum(int(xv[i, k]) * int(yv[k, j]) for k in range(K)) % Q
            assert reveal_int(z, i * N + j) == want


@pytest.mark.parametrize("P", PARTIES)
def test_mp_dealer_trunc_wrap_count(P):
    # theta_r, revealed from its shares, is the wrap count of r's shares:
    # sum_p s64(r_p) = s64(r) + theta_r * Q
    n = 500
    r, t = oracle.mp_dealer_trunc(5, 8, P, n)
    for i in range(n):
        rs = sum(s64(v.ravel()[i]) for v in r)
        theta = s64(reveal_int(t, i))
        assert rs == s64(reveal_int(r, i)) + theta * Q


def floor_div(v, bits):
    return v >> bits  # Python's >> on ints is floor division by 2^bits


@pytest.mark.parametrize("P", PARTIES)
def test_mp_truncate_error_law(P):
    # |x| < 2^40: x + r overflows the signed range with probability ~2^-23, so
    # every element must land in floor(x / 2^16) - {0, ..., P-1}
    rng = np.random.default_rng(300 + P)
    n, bits = 2000, 16
    xs = rng.integers(-(1 << 40), 1 << 40, size=n, dtype=np.int64)
    sh = oracle.mp_share(xs.view(np.uint64), P, 0, seed=12, tag=3)
    r, t = oracle.mp_dealer_trunc(6, 9, P, n)
    y = oracle.mp_truncate(sh, bits, r, t)
    for i in range(n):
        got = s64(reveal_int(y, i))
        err = got - floor_div(int(xs[i]), bits)
        assert -(P - 1) <= err <= 0, (i, err)


@pytest.mark.parametrize("P", [3, 5])
def test_mp_truncate_fails_exactly_when_eta_is_nonzero(P):
    # large |x|: the plaintext sum x + r leaves the signed range for a fraction
    # ~|x|/Q of the elements; with eta taken as 0 exactly those come out wrong
    # (off by a multiple of 2^48) and all others are within the error law
    rng = np.random.default_rng(400 + P)
    n, bits = 4000, 16
    xs = rng.integers(-(1 << 62), 1 << 62, size=n, dtype=np.int64)
    sh = oracle.mp_share(xs.view(np.uint64), P, 1, seed=13, tag=4)
    r, t = oracle.mp_dealer_trunc(7, 10, P, n)
    y = oracle.mp_truncate(sh, bits, r, t)
    bad = 0
    expect_rate = 0.0
    for i in range(n):
        x = int(xs[i])
        rv = s64(reveal_int(r, i))
        eta = (x + rv - s64((x + rv) % Q)) // Q
        got = s64(reveal_int(y, i))
        err = got - floor_div(x, bits)
        if eta == 0:
            assert -(P - 1) <= err <= 0, (i, err)
        else:
            bad += 1
            assert abs(err) >= (1 << 47), (i, err)
        expect_rate += abs(x) / Q
    assert bad > 0
    # the failure count matches the |x|/Q law within 5 sigma
    sigma = max(1.0, expect_rate ** 0.5)
    assert abs(bad - expect_rate) < 5 * sigma, (bad, expect_rate)
