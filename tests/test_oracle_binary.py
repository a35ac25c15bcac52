"""CPU pins of the oracle's binary sharing (App. C.1.1: binary secret sharing,
bitwise AND with Beaver triples, conversions between sharing types,
comparison and ReLU).  Expectations come from numpy's bitwise operators on
the revealed values, Python integers, and the definitions of sign and ReLU,
never from the oracle's own arithmetic."""
import numpy as np
import pytest

import oracle

Q = 1 << 64
EDGE = np.array([0, 1, 2, Q - 1, 1 << 63, (1 << 63) - 1, (1 << 63) + 1, 0x5555555555555555,
                 0xAAAAAAAAAAAAAAAA, 0x00000000FFFFFFFF], dtype=np.uint64)


def rand_u64(seed, n):
    return np.random.default_rng(seed).integers(0, Q, size=n, dtype=np.uint64)


@pytest.mark.parametrize("src", [0, 1])
def test_bin_share_reveal(src):
    x = np.concatenate([rand_u64(1, 500), EDGE])
    s0, s1 = oracle.bin_share(x, src, 3, 7)
    assert np.array_equal(s0 ^ s1, x)
    # the other party's share carries no information about x: sharing two
    # different secrets under the same (seed, tag) gives it the same share
    y = rand_u64(2, x.size)
    t0, t1 = oracle.bin_share(y, src, 3, 7)
    other = (s1, t1) if src == 0 else (s0, t0)
    assert np.array_equal(other[0], other[1])


def test_dealer_and_triple():
    t = oracle.dealer_and(11, 4, 2000)
    a = t.a[0] ^ t.a[1]
    b = t.b[0] ^ t.b[1]
    assert np.array_equal(t.c[0] ^ t.c[1], a & b)
    # a and b look uniform: each bit set about half the time
    bits = np.unpackbits(a.view(np.uint8)).mean()
    assert abs(bits - 0.5) < 0.01


def test_bin_and_identity_any_triple():
    # the identity holds for any triple with c = a & b, not only the dealer's
    n = 700
    x = np.concatenate([rand_u64(3, n - EDGE.size), EDGE])
    y = rand_u64(4, n)
    xs, ys = oracle.bin_share(x, 0, 5, 1), oracle.bin_share(y, 1, 5, 2)
    a0, a1, b0, b1, c0 = (rand_u64(10 + k, n) for k in range(5))
    t = oracle.Triple((a0, a1), (b0, b1), (c0, ((a0 ^ a1) & (b0 ^ b1)) ^ c0))
    z = oracle.bin_and(xs, ys, t)
    assert np.array_equal(z[0] ^ z[1], x & y)


def test_a2b_reveals_the_ring_value():
    n = 3000
    x = np.concatenate([rand_u64(20, n - EDGE.size), EDGE])
    xs = oracle.share(x, 0, 8, 3)  # arithmetic shares
    t = oracle.dealer_and(12, 5, oracle.A2B_TRIPLES * n)
    b = oracle.a2b(xs, 8, 9, t)
    assert np.array_equal(b[0] ^ b[1], x)


def test_a2b_carry_chains():
    # shares chosen so the sum carries through every bit position: y0 = 2^k - 1,
    # y1 = 1 (carry ripples k places), and y0 = all ones, y1 = 1 (wraps to 0)
    y0 = np.array([(1 << k) - 1 for k in range(1, 64)] + [Q - 1, Q - 1, 1 << 63], dtype=np.uint64)
    y1 = np.array([1] * 63 + [1, Q - 1, 1 << 63], dtype=np.uint64)
    want = np.array([(int(a) + int(b)) % Q for a, b in zip(y0, y1)], dtype=np.uint64)
    t = oracle.dealer_and(13, 6, oracle.A2B_TRIPLES * y0.size)
    b = oracle.a2b((y0, y1), 8, 10, t)
    assert np.array_equal(b[0] ^ b[1], want)


def test_b2a_bit_all_positions():
    n = 64 * 40
    x = rand_u64(30, n)
    bits = np.arange(n) % 64
    bs = oracle.bin_share(x, 1, 4, 4)
    rb, ra = oracle.dealer_b2a(14, 7, n)
    # the dealer's bit: the same r in both sharings, r in {0, 1}
    r = (rb[0] ^ rb[1]) & np.uint64(1)
    assert np.array_equal((ra[0] + ra[1]), r)
    for k in (0, 1, 31, 62, 63):
        sel = bits == k
        z = oracle.b2a_bit((bs[0][sel], bs[1][sel]), int(k), (rb[0][sel], rb[1][sel]), (ra[0][sel], ra[1][sel]))
        want = (x[sel] >> np.uint64(k)) & np.uint64(1)
        assert np.array_equal(z[0] + z[1], want)


def test_relu_and_sign_from_definition():
    n = 2000
    rng = np.random.default_rng(40)
    v = rng.integers(-(1 << 40), 1 << 40, size=n, dtype=np.int64)
    v[:4] = [0, 1, -1, -(1 << 40)]
    xs = oracle.share(v.view(np.uint64), 0, 8, 11)
    t = oracle.dealer_and(15, 8, oracle.A2B_TRIPLES * n)
    rb, ra = oracle.dealer_b2a(15, 9, n)
    tm = oracle.dealer_mul(15, 10, n)
    z = oracle.relu(xs, 8, 12, t, rb, ra, tm)
    got = (z[0] + z[1]).view(np.int64)
    assert np.array_equal(got, np.maximum(v, 0))
