"""CPU oracle for two-party arithmetic secret sharing over Z/2^64.

TEST INFRASTRUCTURE ONLY: only the tests, the smoke check and the benchmark's
CPU-baseline leg may import this package.  It wraps ``liboracle.so`` (built
from ``oracle.c`` with gcc) through ctypes and takes/returns numpy arrays.
Ring elements are ``numpy.uint64``; signed fixed-point values ``numpy.int64``.

The C file holds every step of the method (section 5 and App. C.1.1 of the
paper); ``bigint`` holds an arbitrary-precision twin for tiny shapes.
"""
import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
# MPC_ORACLE_LIB may name another build of oracle.c (the sanitizer build)
_LIB_PATH = os.environ.get("MPC_ORACLE_LIB") or os.path.join(_HERE, "liboracle.so")
_lib = None

u64p = ctypes.POINTER(ctypes.c_uint64)
i64p = ctypes.POINTER(ctypes.c_int64)
i8p = ctypes.POINTER(ctypes.c_int8)
dblp = ctypes.POINTER(ctypes.c_double)
u64pp = ctypes.POINTER(u64p)
U64 = ctypes.c_uint64
I64 = ctypes.c_int64
SZ = ctypes.c_size_t
INT = ctypes.c_int

SLOT_SHARE, SLOT_A0, SLOT_A1, SLOT_B0, SLOT_B1, SLOT_C0 = range(6)


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            from . import build as _b
            _b.build()
        L = ctypes.CDLL(_LIB_PATH)
        sig = {
            "orc_num_threads": (INT, []),
            "orc_set_num_threads": (None, [INT]),
            "orc_sm64_mix": (U64, [U64]),
            "orc_sm64_at": (U64, [U64, U64]),
            "orc_prg": (U64, [U64, U64, U64, U64]),
            "orc_prg_fill": (None, [U64, U64, U64, SZ, u64p]),
            "orc_prg_at": (None, [U64, U64, U64, u64p, SZ, u64p]),
            "orc_encode": (SZ, [dblp, SZ, INT, i64p]),
            "orc_decode": (None, [u64p, SZ, INT, dblp]),
            "orc_share": (None, [u64p, SZ, INT, U64, U64, u64p, u64p]),
            "orc_share_at": (None, [u64p, u64p, SZ, INT, U64, U64, u64p, u64p]),
            "orc_reveal": (None, [u64p, u64p, SZ, u64p]),
            "orc_add": (None, [u64p, u64p, SZ, u64p]),
            "orc_truncate": (None, [u64p, SZ, INT]),
            "orc_ring_gemm": (None, [I64, I64, I64, u64p, u64p, u64p]),
            "orc_ring_gemm_at": (None, [I64, I64, I64, u64p, u64p, I64, i64p, i64p, u64p]),
            "orc_conv1d_lout": (I64, [I64, I64, I64]),
            "orc_conv1d": (None, [I64] * 6 + [u64p, u64p, u64p]),
            "orc_conv1d_at": (None, [I64] * 6 + [u64p, u64p, I64, i64p, i64p, i64p, u64p]),
            "orc_dealer_mul": (None, [U64, U64, SZ] + [u64p] * 6),
            "orc_dealer_square": (None, [U64, U64, SZ] + [u64p] * 4),
            "orc_dealer_mul_at": (None, [U64, U64, u64p, SZ] + [u64p] * 6),
            "orc_dealer_square_at": (None, [U64, U64, u64p, SZ] + [u64p] * 4),
            "orc_dealer_matmul": (None, [U64, U64, I64, I64, I64] + [u64p] * 6),
            "orc_dealer_matmul_c_at": (None, [U64, U64, I64, I64, I64] + [u64p] * 4
                                       + [I64, i64p, i64p, u64p, u64p]),
            "orc_dealer_conv1d": (None, [U64, U64] + [I64] * 6 + [u64p] * 6),
            "orc_dealer_matmul_rows": (None, [U64, U64, I64, I64, I64, i64p] + [u64p] * 6),
            "orc_beaver_mul": (None, [SZ] + [u64p] * 10 + [INT, u64p, u64p]),
            "orc_beaver_square": (None, [SZ] + [u64p] * 6 + [INT, u64p, u64p]),
            "orc_beaver_matmul": (None, [I64, I64, I64] + [u64p] * 10 + [INT, u64p, u64p]),
            "orc_beaver_matmul_at": (None, [I64, I64, I64] + [u64p] * 10
                                     + [INT, I64, i64p, i64p, u64p, u64p]),
            "orc_beaver_conv1d": (None, [I64] * 6 + [u64p] * 10 + [INT, u64p, u64p]),
            "orc_dealer_conv1d_c_at": (None, [U64, U64] + [I64] * 6 + [u64p] * 4
                                       + [I64, i64p, i64p, i64p, u64p, u64p]),
            "orc_beaver_conv1d_at": (None, [I64] * 6 + [u64p] * 10
                                     + [INT, I64, i64p, i64p, i64p, u64p, u64p]),
            "orc_limbs": (None, [u64p, SZ, i8p]),
            "orc_limb_gemm": (INT, [I64, I64, I64, u64p, u64p, I64, u64p]),
            "orc_bin_share": (None, [u64p, SZ, INT, U64, U64, u64p, u64p]),
            "orc_bin_reveal": (None, [u64p, u64p, SZ, u64p]),
            "orc_dealer_and": (None, [U64, U64, SZ] + [u64p] * 6),
            "orc_bin_and": (None, [SZ] + [u64p] * 12),
            "orc_a2b": (None, [SZ, u64p, u64p, U64, U64, u64pp, u64p, u64p]),
            "orc_dealer_b2a": (None, [U64, U64, SZ] + [u64p] * 4),
            "orc_b2a_bit": (None, [SZ, INT] + [u64p] * 8),
            "orc_relu": (None, [SZ, u64p, u64p, U64, U64, u64pp] + [u64p] * 12),
            "orc_mp_share": (None, [u64p, SZ, INT, INT, U64, U64, u64pp]),
            "orc_mp_reveal": (None, [INT, u64pp, SZ, u64p]),
            "orc_mp_dealer_mul": (None, [U64, U64, INT, SZ, INT, u64pp, u64pp, u64pp]),
            "orc_mp_dealer_matmul": (None, [U64, U64, INT, I64, I64, I64, u64pp, u64pp, u64pp]),
            "orc_mp_beaver_mul": (None, [INT, SZ, u64pp, u64pp, u64pp, u64pp, u64pp, u64pp]),
            "orc_mp_beaver_matmul": (None, [INT, I64, I64, I64] + [u64pp] * 6),
            "orc_mp_dealer_trunc": (None, [U64, U64, INT, SZ, u64pp, u64pp]),
            "orc_mp_truncate": (None, [INT, SZ, INT, u64pp, u64pp, u64pp]),
        }
        for name, (res, args) in sig.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def _u(a):
    a = np.ascontiguousarray(a, dtype=np.uint64)
    return a, a.ctypes.data_as(u64p)


def _i(a):
    a = np.ascontiguousarray(a, dtype=np.int64)
    return a, a.ctypes.data_as(i64p)


def _out(shape):
    a = np.zeros(shape, dtype=np.uint64)
    return a, a.ctypes.data_as(u64p)


def num_threads():
    return lib().orc_num_threads()


def set_num_threads(n):
    lib().orc_set_num_threads(int(n))


# ----------------------------------------------------------------- PRG
def sm64_mix(z):
    return int(lib().orc_sm64_mix(int(z) & (2**64 - 1)))


def sm64_at(s, i):
    return int(lib().orc_sm64_at(int(s) & (2**64 - 1), int(i)))


def prg(seed, tag, slot, idx):
    return int(lib().orc_prg(seed, tag, slot, idx))


def prg_fill(seed, tag, slot, n):
    out, p = _out(n)
    lib().orc_prg_fill(seed, tag, slot, n, p)
    return out


def prg_at(seed, tag, slot, idx):
    """G(seed, tag, slot, i) for each i of the index array idx (same shape)."""
    idx, pi = _u(idx)
    out, p = _out(idx.shape)
    lib().orc_prg_at(seed, tag, slot, pi, idx.size, p)
    return out


# ----------------------------------------------------------------- fixed point
def encode(x, frac_bits=16):
    x = np.ascontiguousarray(x, dtype=np.float64)
    out = np.zeros(x.shape, dtype=np.int64)
    bad = lib().orc_encode(x.ctypes.data_as(dblp), x.size, frac_bits, out.ctypes.data_as(i64p))
    if bad:
        raise OverflowError(f"element {bad - 1} does not fit the int64 fixed-point range")
    return out


def decode(v, frac_bits=16):
    v, p = _u(np.asarray(v).view(np.uint64) if np.asarray(v).dtype == np.int64 else v)
    out = np.zeros(v.shape, dtype=np.float64)
    lib().orc_decode(p, v.size, frac_bits, out.ctypes.data_as(dblp))
    return out


# ----------------------------------------------------------------- sharing
def as_ring(x):
    """int64 fixed-point values -> their ring elements (same bits)."""
    x = np.ascontiguousarray(x)
    return x.view(np.uint64) if x.dtype == np.int64 else x.astype(np.uint64)


def share(x, src, seed, tag):
    x, px = _u(as_ring(x))
    s0, p0 = _out(x.shape)
    s1, p1 = _out(x.shape)
    lib().orc_share(px, x.size, src, seed, tag, p0, p1)
    return s0, s1


def share_at(x, idx, src, seed, tag):
    """Shares of the elements idx of a shared vector, x holding their values:
    the same shares ``share`` gives those elements, for vectors of any length."""
    x, px = _u(as_ring(x))
    idx, pi = _u(idx)
    s0, p0 = _out(x.shape)
    s1, p1 = _out(x.shape)
    lib().orc_share_at(px, pi, x.size, src, seed, tag, p0, p1)
    return s0, s1


def reveal(s0, s1):
    s0, p0 = _u(s0)
    s1, p1 = _u(s1)
    out, po = _out(s0.shape)
    lib().orc_reveal(p0, p1, s0.size, po)
    return out


def add(x, y):
    x, px = _u(x)
    y, py = _u(y)
    out, po = _out(x.shape)
    lib().orc_add(px, py, x.size, po)
    return out


def truncate(s, bits):
    s = np.array(s, dtype=np.uint64, copy=True)
    lib().orc_truncate(s.ctypes.data_as(u64p), s.size, bits)
    return s


# ----------------------------------------------------------------- products
def ring_gemm(A, B):
    A, pa = _u(A)
    B, pb = _u(B)
    M, K = A.shape
    K2, N = B.shape
    assert K == K2
    C, pc = _out((M, N))
    lib().orc_ring_gemm(M, N, K, pa, pb, pc)
    return C


def ring_gemm_at(A, B, rows, cols):
    A, pa = _u(A)
    B, pb = _u(B)
    M, K = A.shape
    N = B.shape[1]
    rows, pr = _i(rows)
    cols, pcl = _i(cols)
    out, po = _out(rows.size)
    lib().orc_ring_gemm_at(M, N, K, pa, pb, rows.size, pr, pcl, po)
    return out


def conv1d_lout(L, ksz, stride):
    return int(lib().orc_conv1d_lout(L, ksz, stride))


def conv1d(x, w, stride):
    x, px = _u(x)
    w, pw = _u(w)
    Bt, Cin, L = x.shape
    Cout, Cin2, ksz = w.shape
    assert Cin == Cin2
    Lout = conv1d_lout(L, ksz, stride)
    y, py = _out((Bt, Cout, Lout))
    lib().orc_conv1d(Bt, Cin, L, Cout, ksz, stride, px, pw, py)
    return y


def conv1d_at(x, w, stride, bs, os_, ls):
    x, px = _u(x)
    w, pw = _u(w)
    Bt, Cin, L = x.shape
    Cout, _, ksz = w.shape
    bs, pb = _i(bs)
    os_, po_ = _i(os_)
    ls, pl = _i(ls)
    out, po = _out(bs.size)
    lib().orc_conv1d_at(Bt, Cin, L, Cout, ksz, stride, px, pw, bs.size, pb, po_, pl, po)
    return out


# ----------------------------------------------------------------- dealer
class Triple:
    """Shares of a Beaver triple (a, b, c): a[p], b[p], c[p] for p in {0, 1}.
    For a square pair c is None and b = a^2."""

    def __init__(self, a, b, c=None):
        self.a, self.b, self.c = a, b, c


def dealer_mul(dseed, tag, n):
    bufs = [_out(n) for _ in range(6)]
    lib().orc_dealer_mul(dseed, tag, n, *[p for _, p in bufs])
    a0, a1, b0, b1, c0, c1 = [b for b, _ in bufs]
    return Triple((a0, a1), (b0, b1), (c0, c1))


def dealer_square(dseed, tag, n):
    bufs = [_out(n) for _ in range(4)]
    lib().orc_dealer_square(dseed, tag, n, *[p for _, p in bufs])
    a0, a1, b0, b1 = [b for b, _ in bufs]
    return Triple((a0, a1), (b0, b1))


def dealer_mul_at(dseed, tag, idx):
    """Elements idx of the product triple ``dealer_mul`` draws (any length)."""
    idx, pi = _u(idx)
    bufs = [_out(idx.size) for _ in range(6)]
    lib().orc_dealer_mul_at(dseed, tag, pi, idx.size, *[p for _, p in bufs])
    a0, a1, b0, b1, c0, c1 = [b for b, _ in bufs]
    return Triple((a0, a1), (b0, b1), (c0, c1))


def dealer_square_at(dseed, tag, idx):
    """Elements idx of the square pair ``dealer_square`` draws (any length)."""
    idx, pi = _u(idx)
    bufs = [_out(idx.size) for _ in range(4)]
    lib().orc_dealer_square_at(dseed, tag, pi, idx.size, *[p for _, p in bufs])
    a0, a1, b0, b1 = [b for b, _ in bufs]
    return Triple((a0, a1), (b0, b1))


def dealer_matmul(dseed, tag, M, N, K):
    shapes = [(M, K), (M, K), (K, N), (K, N), (M, N), (M, N)]
    bufs = [_out(s) for s in shapes]
    lib().orc_dealer_matmul(dseed, tag, M, N, K, *[p for _, p in bufs])
    a0, a1, b0, b1, c0, c1 = [b for b, _ in bufs]
    return Triple((a0, a1), (b0, b1), (c0, c1))


def dealer_matmul_ab(dseed, tag, M, N, K):
    """a_p and b_p of a matrix triple (PRG fills only, no product)."""
    a0 = prg_fill(dseed, tag, SLOT_A0, M * K).reshape(M, K)
    a1 = prg_fill(dseed, tag, SLOT_A1, M * K).reshape(M, K)
    b0 = prg_fill(dseed, tag, SLOT_B0, K * N).reshape(K, N)
    b1 = prg_fill(dseed, tag, SLOT_B1, K * N).reshape(K, N)
    return (a0, a1), (b0, b1)


def dealer_matmul_c_at(dseed, tag, M, N, K, a, b, rows, cols):
    (a0, pa0), (a1, pa1) = _u(a[0]), _u(a[1])
    (b0, pb0), (b1, pb1) = _u(b[0]), _u(b[1])
    rows, pr = _i(rows)
    cols, pcl = _i(cols)
    c0, pc0 = _out(rows.size)
    c1, pc1 = _out(rows.size)
    lib().orc_dealer_matmul_c_at(dseed, tag, M, N, K, pa0, pa1, pb0, pb1, rows.size, pr, pcl,
                                 pc0, pc1)
    return c0, c1


def dealer_matmul_rows(dseed, tag, N, K, rows):
    """Rows `rows` of the matrix triple ``dealer_matmul`` draws, for any
    height: a_p and c_p restricted to those rows, and all of b_p."""
    rows, pr = _i(rows)
    R = rows.size
    shapes = [(R, K), (R, K), (K, N), (K, N), (R, N), (R, N)]
    bufs = [_out(s) for s in shapes]
    lib().orc_dealer_matmul_rows(dseed, tag, N, K, R, pr, *[p for _, p in bufs])
    a0, a1, b0, b1, c0, c1 = [b for b, _ in bufs]
    return Triple((a0, a1), (b0, b1), (c0, c1))


def dealer_conv1d(dseed, tag, Bt, Cin, L, Cout, ksz, stride):
    Lout = conv1d_lout(L, ksz, stride)
    shapes = [(Bt, Cin, L)] * 2 + [(Cout, Cin, ksz)] * 2 + [(Bt, Cout, Lout)] * 2
    bufs = [_out(s) for s in shapes]
    lib().orc_dealer_conv1d(dseed, tag, Bt, Cin, L, Cout, ksz, stride, *[p for _, p in bufs])
    a0, a1, b0, b1, c0, c1 = [b for b, _ in bufs]
    return Triple((a0, a1), (b0, b1), (c0, c1))


# ----------------------------------------------------------------- Beaver
def beaver_mul(x, y, t, trunc_bits):
    n = x[0].size
    args = [_u(v) for v in (x[0], x[1], y[0], y[1], t.a[0], t.a[1], t.b[0], t.b[1], t.c[0],
                            t.c[1])]
    z0, p0 = _out(x[0].shape)
    z1, p1 = _out(x[0].shape)
    lib().orc_beaver_mul(n, *[p for _, p in args], trunc_bits, p0, p1)
    return z0, z1


def beaver_square(x, t, trunc_bits):
    n = x[0].size
    args = [_u(v) for v in (x[0], x[1], t.a[0], t.a[1], t.b[0], t.b[1])]
    z0, p0 = _out(x[0].shape)
    z1, p1 = _out(x[0].shape)
    lib().orc_beaver_square(n, *[p for _, p in args], trunc_bits, p0, p1)
    return z0, z1


def beaver_matmul(x, y, t, trunc_bits):
    M, K = x[0].shape
    N = y[0].shape[1]
    args = [_u(v) for v in (x[0], x[1], y[0], y[1], t.a[0], t.a[1], t.b[0], t.b[1], t.c[0],
                            t.c[1])]
    z0, p0 = _out((M, N))
    z1, p1 = _out((M, N))
    lib().orc_beaver_matmul(M, N, K, *[p for _, p in args], trunc_bits, p0, p1)
    return z0, z1


def beaver_matmul_at(x, y, a, b, c_at, trunc_bits, rows, cols):
    M, K = x[0].shape
    N = y[0].shape[1]
    args = [_u(v) for v in (x[0], x[1], y[0], y[1], a[0], a[1], b[0], b[1], c_at[0], c_at[1])]
    rows, pr = _i(rows)
    cols, pcl = _i(cols)
    z0, p0 = _out(rows.size)
    z1, p1 = _out(rows.size)
    lib().orc_beaver_matmul_at(M, N, K, *[p for _, p in args], trunc_bits, rows.size, pr, pcl,
                               p0, p1)
    return z0, z1


def beaver_conv1d(x, w, t, stride, trunc_bits):
    Bt, Cin, L = x[0].shape
    Cout, _, ksz = w[0].shape
    Lout = conv1d_lout(L, ksz, stride)
    args = [_u(v) for v in (x[0], x[1], w[0], w[1], t.a[0], t.a[1], t.b[0], t.b[1], t.c[0],
                            t.c[1])]
    z0, p0 = _out((Bt, Cout, Lout))
    z1, p1 = _out((Bt, Cout, Lout))
    lib().orc_beaver_conv1d(Bt, Cin, L, Cout, ksz, stride, *[p for _, p in args], trunc_bits,
                            p0, p1)
    return z0, z1


def dealer_conv1d_ab(dseed, tag, Bt, Cin, L, Cout, ksz):
    """a_p (activation shape) and b_p (weight shape) of a conv triple (PRG fills)."""
    nx, nw = Bt * Cin * L, Cout * Cin * ksz
    a = tuple(prg_fill(dseed, tag, s, nx).reshape(Bt, Cin, L) for s in (SLOT_A0, SLOT_A1))
    b = tuple(prg_fill(dseed, tag, s, nw).reshape(Cout, Cin, ksz) for s in (SLOT_B0, SLOT_B1))
    return a, b


def dealer_conv1d_c_at(dseed, tag, shape, a, b, bs, os_, ls):
    Bt, Cin, L, Cout, ksz, stride = shape
    (a0, pa0), (a1, pa1) = _u(a[0]), _u(a[1])
    (b0, pb0), (b1, pb1) = _u(b[0]), _u(b[1])
    bs, pb = _i(bs)
    os_, po_ = _i(os_)
    ls, pl = _i(ls)
    c0, pc0 = _out(bs.size)
    c1, pc1 = _out(bs.size)
    lib().orc_dealer_conv1d_c_at(dseed, tag, Bt, Cin, L, Cout, ksz, stride, pa0, pa1, pb0, pb1,
                                 bs.size, pb, po_, pl, pc0, pc1)
    return c0, c1


def beaver_conv1d_at(x, w, a, b, c_at, stride, trunc_bits, bs, os_, ls):
    Bt, Cin, L = x[0].shape
    Cout, _, ksz = w[0].shape
    args = [_u(v) for v in (x[0], x[1], w[0], w[1], a[0], a[1], b[0], b[1], c_at[0], c_at[1])]
    bs, pb = _i(bs)
    os_, po_ = _i(os_)
    ls, pl = _i(ls)
    z0, p0 = _out(bs.size)
    z1, p1 = _out(bs.size)
    lib().orc_beaver_conv1d_at(Bt, Cin, L, Cout, ksz, stride, *[p for _, p in args], trunc_bits,
                               bs.size, pb, po_, pl, p0, p1)
    return z0, z1


# ----------------------------------------------------------------- limbs (test helpers)
def limbs(v):
    v, pv = _u(v)
    d = np.zeros(v.shape + (8,), dtype=np.int8)
    lib().orc_limbs(pv, v.size, d.ctypes.data_as(i8p))
    return d


def limb_gemm(A, B, kchunk):
    A, pa = _u(A)
    B, pb = _u(B)
    M, K = A.shape
    N = B.shape[1]
    C, pc = _out((M, N))
    rc = lib().orc_limb_gemm(M, N, K, pa, pb, kchunk, pc)
    if rc != 0:
        raise OverflowError("an int32 chunk sum overflowed")
    return C


# ----------------------------------------------------------------- more than two parties
# A sharing among P parties is a list of P numpy uint64 arrays of one shape.
def _pp(arrs):
    """C array of P pointers to contiguous uint64 arrays (kept alive by the caller)."""
    return (u64p * len(arrs))(*[a.ctypes.data_as(u64p) for a in arrs])


def _outs(P, shape):
    return [np.zeros(shape, dtype=np.uint64) for _ in range(P)]


def mp_share(x, P, src, seed, tag):
    x = np.ascontiguousarray(x).view(np.uint64) if np.asarray(x).dtype == np.int64 else np.ascontiguousarray(x, dtype=np.uint64)
    s = _outs(P, x.shape)
    lib().orc_mp_share(x.ctypes.data_as(u64p), x.size, P, src, seed, tag, _pp(s))
    return s


def mp_reveal(s):
    s = [np.ascontiguousarray(v, dtype=np.uint64) for v in s]
    out = np.zeros(s[0].shape, dtype=np.uint64)
    lib().orc_mp_reveal(len(s), _pp(s), s[0].size, out.ctypes.data_as(u64p))
    return out


def mp_dealer_mul(dseed, tag, P, n, square=False):
    a, b, c = _outs(P, n), _outs(P, n), _outs(P, n)
    lib().orc_mp_dealer_mul(dseed, tag, P, n, int(square), _pp(a), _pp(b), _pp(c))
    return Triple(a, b, None if square else c)


def mp_dealer_matmul(dseed, tag, P, M, N, K):
    a, b, c = _outs(P, (M, K)), _outs(P, (K, N)), _outs(P, (M, N))
    lib().orc_mp_dealer_matmul(dseed, tag, P, M, N, K, _pp(a), _pp(b), _pp(c))
    return Triple(a, b, c)


def mp_beaver_mul(x, y, t):
    """P-party Beaver product (y None: square with the pair t = (a, b = a^2))."""
    P = len(x)
    x = [np.ascontiguousarray(v, dtype=np.uint64) for v in x]
    a = [np.ascontiguousarray(v, dtype=np.uint64) for v in t.a]
    b = [np.ascontiguousarray(v, dtype=np.uint64) for v in t.b]
    z = _outs(P, x[0].shape)
    if y is None:
        lib().orc_mp_beaver_mul(P, x[0].size, _pp(x), None, _pp(a), _pp(b), None, _pp(z))
    else:
        y = [np.ascontiguousarray(v, dtype=np.uint64) for v in y]
        c = [np.ascontiguousarray(v, dtype=np.uint64) for v in t.c]
        lib().orc_mp_beaver_mul(P, x[0].size, _pp(x), _pp(y), _pp(a), _pp(b), _pp(c), _pp(z))
    return z


def mp_beaver_matmul(x, y, t):
    P = len(x)
    M, K = x[0].shape
    N = y[0].shape[1]
    arrs = [[np.ascontiguousarray(v, dtype=np.uint64) for v in g] for g in (x, y, t.a, t.b, t.c)]
    z = _outs(P, (M, N))
    lib().orc_mp_beaver_matmul(P, M, N, K, *[_pp(g) for g in arrs], _pp(z))
    return z


def mp_dealer_trunc(dseed, tag, P, n):
    """Algorithm 1's dealer inputs: shares of a uniform r and of its wrap count."""
    r, t = _outs(P, n), _outs(P, n)
    lib().orc_mp_dealer_trunc(dseed, tag, P, n, _pp(r), _pp(t))
    return r, t


def mp_truncate(x, bits, r, t):
    """Algorithm 1 truncation (eta = 0) of a P-party sharing; returns new shares."""
    P = len(x)
    out = [np.array(v, dtype=np.uint64, copy=True).ravel() for v in x]
    r = [np.ascontiguousarray(v, dtype=np.uint64).ravel() for v in r]
    t = [np.ascontiguousarray(v, dtype=np.uint64).ravel() for v in t]
    lib().orc_mp_truncate(P, out[0].size, bits, _pp(out), _pp(r), _pp(t))
    return [o.reshape(np.shape(x[0])) for o in out]


# ----------------------------------------------------------------- binary sharing (two parties)
A2B_TRIPLES = 12


def bin_share(x, src, seed, tag):
    x, px = _u(x)
    s0, p0 = _out(x.shape)
    s1, p1 = _out(x.shape)
    lib().orc_bin_share(px, x.size, src, seed, tag, p0, p1)
    return s0, s1


def bin_reveal(s0, s1):
    (a, pa), (b, pb) = _u(s0), _u(s1)
    out, po = _out(a.shape)
    lib().orc_bin_reveal(pa, pb, a.size, po)
    return out


def dealer_and(dseed, tag, n):
    """n bitwise AND triples (a, b, c = a & b), XOR-shared."""
    bufs = [_out(n) for _ in range(6)]
    lib().orc_dealer_and(dseed, tag, n, *[p for _, p in bufs])
    a0, a1, b0, b1, c0, c1 = [b for b, _ in bufs]
    return Triple((a0, a1), (b0, b1), (c0, c1))


def bin_and(x, y, t):
    args = [_u(v) for v in (x[0], x[1], y[0], y[1], t.a[0], t.a[1], t.b[0], t.b[1], t.c[0], t.c[1])]
    z0, p0 = _out(args[0][0].shape)
    z1, p1 = _out(args[0][0].shape)
    lib().orc_bin_and(args[0][0].size, *[p for _, p in args], p0, p1)
    return z0, z1


def _tr6(t):
    arrs = [np.ascontiguousarray(v, dtype=np.uint64) for v in (t.a[0], t.a[1], t.b[0], t.b[1], t.c[0], t.c[1])]
    return arrs, _pp(arrs)


def a2b(x, seed, tag, t):
    """Arithmetic to binary sharing; t holds A2B_TRIPLES * n AND triples ([12][n] layout)."""
    (x0, px0), (x1, px1) = _u(x[0]), _u(x[1])
    arrs, pp = _tr6(t)
    z0, p0 = _out(x0.shape)
    z1, p1 = _out(x0.shape)
    lib().orc_a2b(x0.size, px0, px1, seed, tag, pp, p0, p1)
    return z0, z1


def dealer_b2a(dseed, tag, n):
    """Algorithm 2's random bits: (<r>_0, <r>_1), ([r]_0, [r]_1)."""
    bufs = [_out(n) for _ in range(4)]
    lib().orc_dealer_b2a(dseed, tag, n, *[p for _, p in bufs])
    rb0, rb1, ra0, ra1 = [b for b, _ in bufs]
    return (rb0, rb1), (ra0, ra1)


def b2a_bit(b, bit, rb, ra):
    args = [_u(v) for v in (b[0], b[1], rb[0], rb[1], ra[0], ra[1])]
    z0, p0 = _out(args[0][0].shape)
    z1, p1 = _out(args[0][0].shape)
    lib().orc_b2a_bit(args[0][0].size, bit, *[p for _, p in args], p0, p1)
    return z0, z1


def relu(x, seed, tag, t, rb, ra, tm):
    (x0, px0), (x1, px1) = _u(x[0]), _u(x[1])
    arrs, pp = _tr6(t)
    rest = [_u(v) for v in (rb[0], rb[1], ra[0], ra[1], tm.a[0], tm.a[1], tm.b[0], tm.b[1], tm.c[0], tm.c[1])]
    z0, p0 = _out(x0.shape)
    z1, p1 = _out(x0.shape)
    lib().orc_relu(x0.size, px0, px1, seed, tag, pp, *[p for _, p in rest], p0, p1)
    return z0, z1
