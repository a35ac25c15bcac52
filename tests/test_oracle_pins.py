"""Pins for the CPU oracle: each test checks the oracle against a fact fixed
outside it (published PRG outputs, the paper's worked example, exact Python
integer arithmetic, numpy/library routines, closed-form laws).  CPU only."""
import json
import os

import numpy as np
import pytest

import oracle
from oracle import bigint
import workloads

Q = 1 << 64
GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
EDGE = [0, 1, 2, (1 << 63) - 1, 1 << 63, Q - 1, 0x7F7F7F7F7F7F7F80, 0x7F7F7F7F7F7F7F7F,
        0x8080808080808080, 12345678901234567]


def ring(vals):
    return np.array([v % Q for v in vals], dtype=np.uint64)


def rand_ring(seed, shape):
    return workloads.uniform_u64(seed, shape)


def pyints(a):
    return [int(v) for v in np.asarray(a, dtype=np.uint64).ravel()]


# ------------------------------------------------------------------ PRG
def test_splitmix64_published_outputs():
    lines = open(os.path.join(GOLDEN, "splitmix64_state1234567.txt")).read().split("\n")
    want = [int(l) for l in lines if l and not l.startswith("#")]
    got = [oracle.sm64_at(1234567, i) for i in range(5)]
    assert got == want
    # the Python twin, stepping the state, gives the same stream
    assert bigint.splitmix64_stream(1234567, 5) == want


def test_prg_domains_distinct_and_deterministic():
    a = oracle.prg_fill(7, 3, oracle.SLOT_A0, 1000)
    b = oracle.prg_fill(7, 3, oracle.SLOT_A1, 1000)
    c = oracle.prg_fill(7, 4, oracle.SLOT_A0, 1000)
    d = oracle.prg_fill(8, 3, oracle.SLOT_A0, 1000)
    assert np.array_equal(a, oracle.prg_fill(7, 3, oracle.SLOT_A0, 1000))
    for other in (b, c, d):
        assert np.count_nonzero(a == other) == 0
    assert len(set(pyints(a))) == 1000
    # the nested-stream definition: idx-th output of the (slot-th output of the
    # tag-th output of the seed stream) stream
    s = oracle.sm64_at(oracle.sm64_at(7, 3), oracle.SLOT_A0)
    assert int(a[17]) == bigint.splitmix64_stream(s, 18)[17]


# element indices past 2^31 and 2^32, where 32-bit index arithmetic would wrap
FAR = np.array([(1 << 31) - 1, 1 << 31, (1 << 31) + 37, (1 << 32) + 3, (1 << 40) + 11],
               dtype=np.uint64)


def test_prg_far_indices_jump_ahead():
    # a SplitMix64 stream's state only advances by the gamma, so output idx of
    # the stream with state s is the first output of the stream with state
    # s + idx * gamma: the Python twin reaches far indices in one step
    seed, tag = 2005, 7
    t = bigint.splitmix64_stream(seed, tag + 1)[tag]
    for slot in (oracle.SLOT_SHARE, oracle.SLOT_A0, oracle.SLOT_C0):
        s = bigint.splitmix64_stream(t, slot + 1)[slot]
        for i in pyints(FAR):
            want = bigint.splitmix64_stream((s + i * 0x9E3779B97F4A7C15) % Q, 1)[0]
            assert oracle.prg(seed, tag, slot, i) == want
    # the array form agrees element by element, at far and near indices
    idx = np.concatenate([FAR, np.arange(5, dtype=np.uint64)])
    got = oracle.prg_at(seed, tag, oracle.SLOT_B1, idx)
    assert pyints(got) == [oracle.prg(seed, tag, oracle.SLOT_B1, i) for i in pyints(idx)]
    assert np.array_equal(got[FAR.size:], oracle.prg_fill(seed, tag, oracle.SLOT_B1, 5))


@pytest.mark.parametrize("src", [0, 1])
def test_share_at_far_indices(src):
    x = rand_ring(61, FAR.size)
    s0, s1 = oracle.share_at(x, FAR, src, 2005, 7)
    # reveals x, and the non-source share is the PRG mask of that element
    assert pyints(s0 + s1) == pyints(x)
    other = s1 if src == 0 else s0
    assert pyints(other) == [oracle.prg(2005, 7, oracle.SLOT_SHARE, i) for i in pyints(FAR)]
    # near the start the selected elements are those of the whole vector
    idx = np.array([0, 3, 999, 500], dtype=np.uint64)
    full = oracle.share(rand_ring(62, 1000), src, 2005, 7)
    part = oracle.share_at(rand_ring(62, 1000)[idx.astype(np.int64)], idx, src, 2005, 7)
    for p in (0, 1):
        assert np.array_equal(full[p][idx.astype(np.int64)], part[p])


def test_dealer_at_far_indices():
    t = oracle.dealer_mul_at(3005, 9, FAR)
    sq = oracle.dealer_square_at(3005, 9, FAR)
    for k in range(FAR.size):
        a = (int(t.a[0][k]) + int(t.a[1][k])) % Q
        b = (int(t.b[0][k]) + int(t.b[1][k])) % Q
        assert (int(t.c[0][k]) + int(t.c[1][k])) % Q == a * b % Q
        a2 = (int(sq.a[0][k]) + int(sq.a[1][k])) % Q
        assert (int(sq.b[0][k]) + int(sq.b[1][k])) % Q == a2 * a2 % Q
    # the pair shares its a with the product triple of the same (seed, tag)
    assert np.array_equal(t.a[0], sq.a[0]) and np.array_equal(t.a[1], sq.a[1])
    idx = np.array([0, 7, 63], dtype=np.uint64)
    full, part = oracle.dealer_mul(3005, 9, 64), oracle.dealer_mul_at(3005, 9, idx)
    for k in "abc":
        for p in (0, 1):
            assert np.array_equal(getattr(full, k)[p][idx.astype(np.int64)], getattr(part, k)[p])


def test_dealer_matmul_rows():
    M, N, K = 9, 4, 13
    rows = np.array([0, 8, 3], dtype=np.int64)
    full, part = oracle.dealer_matmul(3006, 2, M, N, K), oracle.dealer_matmul_rows(3006, 2, N, K, rows)
    for p in (0, 1):
        assert np.array_equal(full.a[p][rows], part.a[p])
        assert np.array_equal(full.b[p], part.b[p])
        assert np.array_equal(full.c[p][rows], part.c[p])
    # far rows: c = a @ b, checked with Python integers on the revealed values
    far = np.array([(1 << 31) // K + 1, (1 << 33) // K], dtype=np.int64)
    t = oracle.dealer_matmul_rows(3006, 2, N, K, far)
    A = [[(int(t.a[0][r, k]) + int(t.a[1][r, k])) % Q for k in range(K)] for r in range(far.size)]
    B = [[(int(t.b[0][k, j]) + int(t.b[1][k, j])) % Q for j in range(N)] for k in range(K)]
    C = bigint.matmul(A, B)
    for r in range(far.size):
        for j in range(N):
            assert (int(t.c[0][r, j]) + int(t.c[1][r, j])) % Q == C[r][j]
        assert int(t.a[0][r, 5]) == oracle.prg(3006, 2, oracle.SLOT_A0, int(far[r]) * K + 5)
        assert int(t.c[0][r, 1]) == oracle.prg(3006, 2, oracle.SLOT_C0, int(far[r]) * N + 1)


def test_prg_bits_balanced():
    v = oracle.prg_fill(11, 1, 0, 1 << 16)
    bits = np.unpackbits(v.view(np.uint8)).reshape(-1, 64).mean(axis=0)
    assert np.all(np.abs(bits - 0.5) < 0.02)


# ------------------------------------------------------------------ encoding
def test_encode_values_and_ties_to_even():
    h = 2.0 ** -17  # half of one fixed-point unit at 16 fractional bits
    x = np.array([1.0, 2.0, 3.0, -1.5, h, 3 * h, -h, 5 * h, -3 * h, 0.0])
    want = [65536, 131072, 196608, -98304, 0, 2, 0, 2, -2, 0]
    assert oracle.encode(x, 16).tolist() == want
    assert oracle.encode(np.array([1.0]), 0).tolist() == [1]


def test_encode_range_and_decode():
    with pytest.raises(OverflowError):
        oracle.encode(np.array([2.0 ** 47]), 16)
    with pytest.raises(OverflowError):
        oracle.encode(np.array([np.nan]), 16)
    # the largest double below 2^47 is 2^47 - 2^-6, which encodes to 2^63 - 2^10
    ok = oracle.encode(np.array([np.nextafter(2.0 ** 47, 0), -(2.0 ** 47)]), 16)
    assert ok.tolist() == [(1 << 63) - 1024, -(1 << 63)]
    x = workloads.uniform(5, 1000, -100, 100)
    err = oracle.decode(oracle.as_ring(oracle.encode(x, 16)), 16) - x
    assert np.max(np.abs(err)) <= 2.0 ** -17


# ------------------------------------------------------------------ sharing
def test_figure2_example():
    ex = json.load(open(os.path.join(GOLDEN, "figure2_example.json")))
    f = ex["frac_bits"]
    xs = oracle.share(oracle.encode(np.array(ex["x"]), f), ex["src"], 2001, 1)
    ys = oracle.share(oracle.encode(np.array(ex["y"]), f), ex["src"], 2001, 2)
    assert oracle.decode(oracle.reveal(*xs), f).tolist() == ex["x"]
    zs = (oracle.add(xs[0], ys[0]), oracle.add(xs[1], ys[1]))
    assert oracle.decode(oracle.reveal(*zs), f).tolist() == ex["x_plus_y"]
    # the shares themselves do not show the value
    assert not np.array_equal(xs[0], oracle.as_ring(oracle.encode(np.array(ex["x"]), f)))
    # extension: the Beaver product is x*y within one fixed-point unit
    t = oracle.dealer_mul(3001, 9, 3)
    z = oracle.beaver_mul(xs, ys, t, f)
    prod = oracle.decode(oracle.reveal(*z), f)
    assert np.max(np.abs(prod - np.array([2.0, 6.0, 12.0]))) <= 2.0 ** -f


@pytest.mark.parametrize("src", [0, 1])
def test_reveal_share_roundtrip(src):
    x = np.concatenate([ring(EDGE), rand_ring(3, 500)])
    s0, s1 = oracle.share(x, src, 99, 5)
    assert np.array_equal(oracle.reveal(s0, s1), x)
    # exact big-int check of the sum
    assert [(a + b) % Q for a, b in zip(pyints(s0), pyints(s1))] == pyints(x)
    # the non-source party holds the raw mask; the zero-share sums to 0
    mask = oracle.prg_fill(99, 5, oracle.SLOT_SHARE, x.size)
    assert np.array_equal(s1 if src == 0 else s0, mask)
    zero = oracle.share(np.zeros_like(x), src, 99, 5)
    assert np.all(oracle.reveal(*zero) == 0)


# ------------------------------------------------------------------ Beaver element-wise
def test_beaver_mul_identity_bigint():
    n = 300
    x = np.concatenate([ring(EDGE), rand_ring(10, n - len(EDGE))])
    y = np.concatenate([ring(EDGE[::-1]), rand_ring(11, n - len(EDGE))])
    xs, ys = oracle.share(x, 0, 5, 1), oracle.share(y, 1, 5, 2)
    t = oracle.dealer_mul(77, 3, n)
    z = oracle.beaver_mul(xs, ys, t, 0)
    want = [(a * b) % Q for a, b in zip(pyints(x), pyints(y))]
    assert pyints(oracle.reveal(*z)) == want


def test_beaver_mul_any_valid_triple():
    # the identity must hold for any triple with c = a*b, not only dealer ones
    n = 64
    a = (rand_ring(1, n), rand_ring(2, n))
    b = (rand_ring(3, n), rand_ring(4, n))
    c_full = [(int(p) + int(q)) * (int(r) + int(s)) % Q
              for p, q, r, s in zip(a[0], a[1], b[0], b[1])]
    c0 = rand_ring(5, n)
    c1 = ring([(c - int(v)) for c, v in zip(c_full, c0)])
    t = oracle.Triple(a, b, (c0, c1))
    x, y = rand_ring(6, n), rand_ring(7, n)
    z = oracle.beaver_mul(oracle.share(x, 0, 1, 1), oracle.share(y, 0, 1, 2), t, 0)
    assert pyints(oracle.reveal(*z)) == [(p * q) % Q for p, q in zip(pyints(x), pyints(y))]


def test_beaver_square_identity_bigint():
    n = 200
    x = np.concatenate([ring(EDGE), rand_ring(12, n - len(EDGE))])
    xs = oracle.share(x, 0, 5, 3)
    t = oracle.dealer_square(78, 4, n)
    assert pyints(oracle.reveal(*t.b)) == [(v * v) % Q for v in pyints(oracle.reveal(*t.a))]
    z = oracle.beaver_square(xs, t, 0)
    assert pyints(oracle.reveal(*z)) == [(v * v) % Q for v in pyints(x)]


def test_dealer_mul_relation():
    t = oracle.dealer_mul(3, 1, 500)
    a, b, c = (pyints(oracle.reveal(*t.a)), pyints(oracle.reveal(*t.b)),
               pyints(oracle.reveal(*t.c)))
    assert c == [(p * q) % Q for p, q in zip(a, b)]
    assert len(set(a)) == 500 and len(set(b)) == 500


def test_triple_independence():
    # P11: the revealed product does not depend on the dealer's randomness
    x = oracle.encode(workloads.uniform(1, 256, -4, 4), 16)
    y = oracle.encode(workloads.uniform(2, 256, -4, 4), 16)
    xs, ys = oracle.share(x, 0, 1, 1), oracle.share(y, 0, 1, 2)
    r1 = oracle.reveal(*oracle.beaver_mul(xs, ys, oracle.dealer_mul(10, 1, 256), 0))
    r2 = oracle.reveal(*oracle.beaver_mul(xs, ys, oracle.dealer_mul(11, 1, 256), 0))
    assert np.array_equal(r1, r2)
    t1 = oracle.reveal(*oracle.beaver_mul(xs, ys, oracle.dealer_mul(10, 1, 256), 16))
    exact = [bigint.s64(p * q) >> 16 for p, q in zip(pyints(x), pyints(y))]
    d = np.array([bigint.s64(v) for v in pyints(t1)]) - np.array(exact)
    assert set(d.tolist()) <= {-1, 0}


# ------------------------------------------------------------------ ring GEMM and Beaver matmul
def test_numpy_uint64_matmul_wraps():
    A = ring([Q - 1, 1 << 63]).reshape(1, 2)
    B = ring([Q - 1, 3]).reshape(2, 1)
    assert int((A @ B)[0, 0]) == bigint.matmul([[Q - 1, 1 << 63]], [[Q - 1], [3]])[0][0]


@pytest.mark.parametrize("M,N,K", [(1, 1, 1), (3, 2, 5), (4, 7, 3), (2, 3, 9)])
def test_ring_gemm_bigint(M, N, K):
    A = rand_ring(M * 100 + K, (M, K))
    B = rand_ring(N * 100 + K, (K, N))
    A.ravel()[0] = Q - 1
    B.ravel()[-1] = 1 << 63
    want = bigint.matmul(A.tolist(), B.tolist())
    assert oracle.ring_gemm(A, B).tolist() == want


def test_ring_gemm_numpy_and_sampled():
    A, B = rand_ring(1, (37, 53)), rand_ring(2, (53, 29))
    C = oracle.ring_gemm(A, B)
    assert np.array_equal(C, A @ B)
    rows, cols = np.array([0, 36, 5, 17]), np.array([0, 28, 3, 11])
    assert np.array_equal(oracle.ring_gemm_at(A, B, rows, cols), C[rows, cols])


@pytest.mark.parametrize("M,N,K", [(1, 1, 1), (3, 2, 4), (2, 5, 3), (4, 3, 6)])
def test_beaver_matmul_identity_bigint(M, N, K):
    X, Y = rand_ring(M + 7, (M, K)), rand_ring(N + 9, (K, N))
    xs, ys = oracle.share(X, 0, 4, 1), oracle.share(Y, 1, 4, 2)
    t = oracle.dealer_matmul(33, 7, M, N, K)
    assert oracle.reveal(*t.c).tolist() == bigint.matmul(oracle.reveal(*t.a).tolist(),
                                                         oracle.reveal(*t.b).tolist())
    z = oracle.beaver_matmul(xs, ys, t, 0)
    assert oracle.reveal(*z).tolist() == bigint.matmul(X.tolist(), Y.tolist())


def test_beaver_matmul_numpy_medium_and_sampled():
    M, N, K = 40, 24, 70
    X, Y = rand_ring(1, (M, K)), rand_ring(2, (K, N))
    xs, ys = oracle.share(X, 0, 4, 1), oracle.share(Y, 0, 4, 2)
    t = oracle.dealer_matmul(5, 7, M, N, K)
    z = oracle.beaver_matmul(xs, ys, t, 16)
    zr = oracle.beaver_matmul(xs, ys, t, 0)
    assert np.array_equal(oracle.reveal(*zr), X @ Y)
    # the sampled evaluation agrees with the full one, shares and all
    rows, cols = np.array([0, 39, 13, 7]), np.array([0, 23, 5, 19])
    c_at = oracle.dealer_matmul_c_at(5, 7, M, N, K, t.a, t.b, rows, cols)
    assert np.array_equal(c_at[0], t.c[0][rows, cols]) and np.array_equal(c_at[1], t.c[1][rows, cols])
    z_at = oracle.beaver_matmul_at(xs, ys, t.a, t.b, c_at, 16, rows, cols)
    assert np.array_equal(z_at[0], z[0][rows, cols]) and np.array_equal(z_at[1], z[1][rows, cols])


def test_beaver_matmul_zero_triple_is_plain_gemm():
    # P6: with a zero triple and zero masks the protocol is a plain ring GEMM,
    # which must equal numpy's wrapping uint64 matmul and torch's int64 matmul.
    import torch
    M, N, K = 17, 9, 23
    X, Y = rand_ring(3, (M, K)), rand_ring(4, (K, N))
    zM = np.zeros((M, K), np.uint64)
    zK = np.zeros((K, N), np.uint64)
    zC = np.zeros((M, N), np.uint64)
    t = oracle.Triple((zM, zM), (zK, zK), (zC, zC))
    z = oracle.beaver_matmul((X, zM), (Y, zK), t, 0)
    assert np.array_equal(z[0], X @ Y) and np.all(z[1] == 0)
    tt = torch.from_numpy(X.view(np.int64)) @ torch.from_numpy(Y.view(np.int64))
    assert np.array_equal(z[0].view(np.int64), tt.numpy())


# ------------------------------------------------------------------ truncation
@pytest.mark.parametrize("bits", [1, 15, 16, 17, 32, 62, 63])
def test_truncate_floor_division(bits):
    v = np.concatenate([ring([0, 1, 65535, 65536, -1, -65536, -65537, (1 << 63) - 1,
                              -(1 << 63), 1 << 62, -(1 << 62)]), rand_ring(4, 200)])
    got = [bigint.s64(t) for t in pyints(oracle.truncate(v, bits))]
    assert got == [bigint.s64(x) // (1 << bits) for x in pyints(v)]
    assert np.array_equal(oracle.truncate(v, 0), v)


def test_truncation_error_law_forced():
    # P5: when the signed shares do not overflow, the truncated reveal is
    # floor(x / 2^16) or one less; when they do, the error is catastrophic.
    x = (1 << 40) + 12345
    good = (ring([x - 5]), ring([5]))
    r = bigint.s64(int(oracle.reveal(oracle.truncate(good[0], 16), oracle.truncate(good[1], 16))[0]))
    assert r - (x >> 16) in (-1, 0)
    m = (1 << 63) + 10  # s64(m) = -2^63 + 10, so s64(m) + s64(x - m) overflows int64
    bad = (ring([x - m]), ring([m]))
    assert bigint.s64(x - m) + bigint.s64(m) != x
    r = bigint.s64(int(oracle.reveal(oracle.truncate(bad[0], 16), oracle.truncate(bad[1], 16))[0]))
    assert abs(r - (x >> 16)) > 2 ** 40


@pytest.mark.parametrize("x", [1 << 60, -(1 << 61), 3 << 58])
def test_truncation_failure_rate(x):
    # the simple division fails with probability |x|/Q (App. C.1.1, Truncation)
    n = 40000
    s0, s1 = oracle.share(ring([x] * n), 0, 1234, 17)
    t = oracle.reveal(oracle.truncate(s0, 16), oracle.truncate(s1, 16))
    err = np.array([bigint.s64(v) for v in pyints(t)]) - (x >> 16)
    fail = np.mean(np.abs(err) > 1)
    assert np.all((np.abs(err) <= 1) | (np.abs(err) > 2 ** 40))
    p = abs(x) / Q
    assert abs(fail - p) < 5 * np.sqrt(p * (1 - p) / n)
    # the failures are exactly the signed-overflow events of the shares
    wrap = np.array([bigint.s64(a) + bigint.s64(b) != x for a, b in zip(pyints(s0), pyints(s1))])
    assert np.array_equal(wrap, np.abs(err) > 1)


# ------------------------------------------------------------------ conv1d
def _correlate_reference(x, w, stride):
    Bt, Cin, L = x.shape
    Cout, _, k = w.shape
    out = []
    for b in range(Bt):
        rows = []
        for o in range(Cout):
            acc = sum(np.correlate(x[b, c].astype(np.float64), w[o, c].astype(np.float64), "valid")
                      for c in range(Cin))
            rows.append(acc[::stride])
        out.append(rows)
    return np.rint(np.array(out)).astype(np.int64)


@pytest.mark.parametrize("Bt,Cin,L,Cout,k,s", [(1, 1, 10, 1, 3, 1), (2, 3, 17, 4, 5, 2),
                                                (1, 2, 9, 3, 9, 1), (3, 4, 20, 2, 1, 3)])
def test_conv1d_matches_numpy_correlate(Bt, Cin, L, Cout, k, s):
    g = workloads.rng(Bt * 1000 + L)
    x = g.integers(-8, 9, size=(Bt, Cin, L))
    w = g.integers(-8, 9, size=(Cout, Cin, k))
    y = oracle.conv1d(x.astype(np.int64).view(np.uint64), w.astype(np.int64).view(np.uint64), s)
    assert y.view(np.int64).tolist() == _correlate_reference(x, w, s).tolist()
    assert y.shape[2] == (L - k) // s + 1
    bs, os_, ls = np.array([0, Bt - 1]), np.array([0, Cout - 1]), np.array([0, y.shape[2] - 1])
    at = oracle.conv1d_at(x.astype(np.int64).view(np.uint64), w.astype(np.int64).view(np.uint64),
                          s, bs, os_, ls)
    assert np.array_equal(at, y[bs, os_, ls])


def test_beaver_conv_identity():
    Bt, Cin, L, Cout, k, s = 2, 3, 15, 4, 4, 2
    X, W = rand_ring(1, (Bt, Cin, L)), rand_ring(2, (Cout, Cin, k))
    t = oracle.dealer_conv1d(9, 1, Bt, Cin, L, Cout, k, s)
    assert np.array_equal(oracle.reveal(*t.c), oracle.conv1d(oracle.reveal(*t.a),
                                                             oracle.reveal(*t.b), s))
    z = oracle.beaver_conv1d(oracle.share(X, 0, 3, 1), oracle.share(W, 0, 3, 2), t, s, 0)
    assert np.array_equal(oracle.reveal(*z), oracle.conv1d(X, W, s))
    # with tiny integer values the ring conv is the integer conv of numpy
    g = workloads.rng(5)
    xi, wi = g.integers(-8, 9, size=(Bt, Cin, L)), g.integers(-8, 9, size=(Cout, Cin, k))
    z = oracle.beaver_conv1d(oracle.share(xi.view(np.uint64), 1, 3, 1),
                             oracle.share(wi.view(np.uint64), 0, 3, 2), t, s, 0)
    assert oracle.reveal(*z).view(np.int64).tolist() == _correlate_reference(xi, wi, s).tolist()


def test_beaver_conv_sampled_matches_full():
    shape = (2, 3, 20, 4, 5, 2)
    Bt, Cin, L, Cout, k, s = shape
    X, W = rand_ring(3, (Bt, Cin, L)), rand_ring(4, (Cout, Cin, k))
    xs, ws = oracle.share(X, 0, 3, 1), oracle.share(W, 1, 3, 2)
    t = oracle.dealer_conv1d(9, 2, *shape)
    z = oracle.beaver_conv1d(xs, ws, t, s, 16)
    a, b = oracle.dealer_conv1d_ab(9, 2, Bt, Cin, L, Cout, k)
    assert all(np.array_equal(u, v) for u, v in zip(a + b, t.a + t.b))
    Lout = z[0].shape[2]
    bs, os_, ls = np.array([0, 1, 1, 0]), np.array([0, 3, 1, 2]), np.array([0, Lout - 1, 3, 5])
    c_at = oracle.dealer_conv1d_c_at(9, 2, shape, a, b, bs, os_, ls)
    assert np.array_equal(c_at[0], t.c[0][bs, os_, ls]) and np.array_equal(c_at[1], t.c[1][bs, os_, ls])
    z_at = oracle.beaver_conv1d_at(xs, ws, a, b, c_at, s, 16, bs, os_, ls)
    assert np.array_equal(z_at[0], z[0][bs, os_, ls]) and np.array_equal(z_at[1], z[1][bs, os_, ls])


# ------------------------------------------------------------------ limbs
def test_limb_decomposition_identity():
    v = np.concatenate([ring(EDGE), rand_ring(8, 5000)])
    d = oracle.limbs(v)
    assert d.min() >= -128 and d.max() <= 127
    for val, row in zip(pyints(v), d.astype(np.int64).tolist()):
        assert sum(di << (8 * i) for i, di in enumerate(row)) % Q == val
    assert oracle.limbs(ring([0x7F7F7F7F7F7F7F80])).tolist() == [[-128] * 8]
    assert oracle.limbs(ring([0x7F7F7F7F7F7F7F7F])).tolist() == [[127] * 8]
    assert oracle.limbs(ring([0])).tolist() == [[0] * 8]


@pytest.mark.parametrize("kchunk", [1, 7, 64, 1 << 20])
def test_limb_gemm_equals_ring_gemm(kchunk):
    A, B = rand_ring(21, (9, 70)), rand_ring(22, (70, 6))
    A[0, :] = 0x7F7F7F7F7F7F7F80
    B[:, 0] = 0x7F7F7F7F7F7F7F80
    assert np.array_equal(oracle.limb_gemm(A, B, kchunk), A @ B)


def test_limb_gemm_int32_chunk_bound():
    # all limbs -128: each product is 2^14, so K = 2^17 + 1 terms overflow int32
    K = (1 << 17) + 1
    A = np.full((1, K), 0x7F7F7F7F7F7F7F80, dtype=np.uint64)
    B = np.full((K, 1), 0x7F7F7F7F7F7F7F80, dtype=np.uint64)
    with pytest.raises(OverflowError):
        oracle.limb_gemm(A, B, K)
    assert np.array_equal(oracle.limb_gemm(A, B, (1 << 17) - 1), A @ B)
