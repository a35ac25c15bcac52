"""Python binding of libmpc: two-party arithmetic secret sharing over Z/2^64
on one MI355X.

Argument marshalling only: tensors are torch ``int64`` CUDA (HIP) tensors whose
bits are ring elements; their ``data_ptr()`` and the party streams' handles are
passed to the C ABI of ``include/mpc.h``, and every step runs in the library's
HIP kernels.  There is no fallback: if ``libmpc.so`` is missing or does not
load, importing this package raises.
"""
import ctypes
import os

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libmpc.so")

FORM_PLAIN, FORM_LIMB8, FORM_AUTO, FORM_FP64LIMB = 0, 1, 2, 3
TRIPLE_MUL, TRIPLE_SQUARE, TRIPLE_MATMUL, TRIPLE_CONV1D = 0, 1, 2, 3
FORMS = {"plain": FORM_PLAIN, "limb8": FORM_LIMB8, "auto": FORM_AUTO, "fp64limb": FORM_FP64LIMB}
# mpc_status values (include/mpc.h)
(MPC_OK, MPC_E_INVAL, MPC_E_SHAPE, MPC_E_ALIAS, MPC_E_NOMEM, MPC_E_HIP, MPC_E_UNSUPPORTED,
 MPC_E_RANGE) = 0, -1, -2, -3, -4, -5, -6, -7

if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is not built; run paper_2109_00984_amd/build.py "
                      "(or __graft_entry__.build())")
_lib = ctypes.CDLL(LIB_PATH)

VP = ctypes.c_void_p
I64 = ctypes.c_int64
U64 = ctypes.c_uint64
SZ = ctypes.c_size_t
INT = ctypes.c_int


class Triple(ctypes.Structure):
    _fields_ = [("a0", VP), ("a1", VP), ("b0", VP), ("b1", VP), ("c0", VP), ("c1", VP)]


class Conv1dShape(ctypes.Structure):
    _fields_ = [("batch", I64), ("cin", I64), ("length", I64), ("cout", I64), ("ksize", I64),
                ("stride", I64)]


class MatmulDesc(ctypes.Structure):
    _fields_ = [("M", I64), ("N", I64), ("K", I64), ("x0", VP), ("x1", VP), ("y0", VP),
                ("y1", VP), ("t", Triple), ("z0", VP), ("z1", VP)]


class MulDesc(ctypes.Structure):
    _fields_ = [("n", ctypes.c_size_t), ("x0", VP), ("x1", VP), ("y0", VP), ("y1", VP), ("t", Triple),
                ("z0", VP), ("z1", VP)]


MAX_PARTIES = 16


class MpTriple(ctypes.Structure):
    _fields_ = [("a", VP * MAX_PARTIES), ("b", VP * MAX_PARTIES), ("c", VP * MAX_PARTIES)]


class GemmTiming(ctypes.Structure):
    _fields_ = [("launches", U64), ("total_ms", ctypes.c_double), ("ring_macs", ctypes.c_double)]


class TileConfig(ctypes.Structure):
    _fields_ = [("variant", INT), ("group_m", INT), ("xcd_remap", INT), ("ms", ctypes.c_double)]


TILE_VARIANTS = {0: "128x64", 1: "64x128", 2: "64x64", 3: "lds128x64", 4: "lds64x128", 5: "lds64x64",
                 6: "lds64x128w8", 7: "lds128x64w8", 8: "lds64x128w8s", 9: "sh64x64", 10: "sh64x128",
                 11: "sh128x64", 12: "lds32x128", 13: "lds128x32", 14: "classes", 15: "classes_persistent"}


class Stats(ctypes.Structure):
    _fields_ = [("opens", U64), ("open_bytes_per_party", U64), ("truncations", U64),
                ("launches", U64), ("gemm_problems", U64)]


_SIGS = {
    "mpc_status_str": (ctypes.c_char_p, [INT]),
    "mpc_last_hip_error": (INT, []),
    "mpc_encode": (INT, [VP, SZ, INT, VP]),
    "mpc_decode": (INT, [VP, SZ, INT, VP]),
    "mpc_ctx_create": (INT, [INT, VP, VP, U64, ctypes.POINTER(VP)]),
    "mpc_ctx_destroy": (INT, [VP]),
    "mpc_sync": (INT, [VP]),
    "mpc_ctx_stats": (INT, [VP, ctypes.POINTER(Stats)]),
    "mpc_reserve": (INT, [VP, SZ]),
    "mpc_share": (INT, [VP, VP, SZ, INT, U64, VP, VP]),
    "mpc_reveal": (INT, [VP, VP, VP, SZ, VP]),
    "mpc_truncate": (INT, [VP, VP, VP, SZ, INT]),
    "mpc_dealer_triples": (INT, [VP, INT, U64, U64, ctypes.POINTER(I64), ctypes.POINTER(Triple)]),
    "mpc_beaver_mul": (INT, [VP, SZ, VP, VP, VP, VP, ctypes.POINTER(Triple), INT, VP, VP]),
    "mpc_beaver_matmul": (INT, [VP, I64, I64, I64, VP, VP, VP, VP, ctypes.POINTER(Triple), INT,
                                INT, VP, VP]),
    "mpc_packed_triple_bytes": (SZ, [I64, I64, I64]),
    "mpc_dealer_triples_packed": (INT, [VP, U64, U64, I64, I64, I64, ctypes.POINTER(Triple), VP]),
    "mpc_beaver_matmul_prepacked": (INT, [VP, I64, I64, I64, VP, VP, VP, VP, ctypes.POINTER(Triple), VP, INT,
                                          VP, VP]),
    "mpc_beaver_matmul_grouped_prepacked": (INT, [VP, SZ, ctypes.POINTER(MatmulDesc), ctypes.POINTER(VP), INT]),
    "mpc_beaver_matmul_noalloc": (INT, [VP, I64, I64, I64, VP, VP, VP, VP, ctypes.POINTER(Triple), INT,
                                        INT, VP, VP]),
    "mpc_beaver_conv1d": (INT, [VP, ctypes.POINTER(Conv1dShape), VP, VP, VP, VP,
                                ctypes.POINTER(Triple), INT, INT, VP, VP]),
    "mpc_ring_gemm": (INT, [VP, I64, I64, I64, VP, VP, VP, INT]),
    "mpc_beaver_matmul_grouped": (INT, [VP, SZ, ctypes.POINTER(MatmulDesc), INT, INT]),
    "mpc_profile_enable": (INT, [VP, INT]),
    "mpc_profile_read": (INT, [VP, ctypes.POINTER(GemmTiming), ctypes.POINTER(GemmTiming),
                             ctypes.POINTER(GemmTiming)]),
    "mpc_autotune_matmul": (INT, [VP, SZ, ctypes.POINTER(I64), ctypes.POINTER(TileConfig)]),
    "mpc_autotune_save": (INT, [VP, ctypes.c_char_p]),
    "mpc_autotune_load": (INT, [VP, ctypes.c_char_p]),
    "mpc_set_default_tile_config": (INT, [VP, ctypes.POINTER(TileConfig)]),
    "mpc_beaver_mul_grouped": (INT, [VP, ctypes.c_size_t, ctypes.POINTER(MulDesc), INT]),
    "mpc_get_default_tile_config": (INT, [VP, ctypes.POINTER(TileConfig)]),
    "mpc_limb_plan": (INT, [I64, I64, INT, ctypes.POINTER(INT), ctypes.POINTER(I64), ctypes.POINTER(INT),
                            ctypes.POINTER(I64)]),
    "mpc_graph_begin": (INT, [VP]),
    "mpc_graph_end": (INT, [VP, ctypes.POINTER(VP)]),
    "mpc_graph_launch": (INT, [VP, VP]),
    "mpc_graph_destroy": (INT, [VP]),
    "mpc_bin_share": (INT, [VP, VP, SZ, INT, U64, VP, VP]),
    "mpc_bin_reveal": (INT, [VP, VP, VP, SZ, VP]),
    "mpc_dealer_and_triples": (INT, [VP, U64, U64, SZ, ctypes.POINTER(Triple)]),
    "mpc_bin_and": (INT, [VP, SZ, VP, VP, VP, VP, ctypes.POINTER(Triple), VP, VP]),
    "mpc_a2b": (INT, [VP, SZ, VP, VP, U64, ctypes.POINTER(Triple), VP, VP]),
    "mpc_dealer_b2a": (INT, [VP, U64, U64, SZ, VP, VP, VP, VP]),
    "mpc_b2a_bit": (INT, [VP, SZ, INT, VP, VP, VP, VP, VP, VP, VP, VP]),
    "mpc_relu": (INT, [VP, SZ, VP, VP, U64, ctypes.POINTER(Triple), VP, VP, VP, VP,
                       ctypes.POINTER(Triple), VP, VP]),
    "mpc_mp_share": (INT, [VP, INT, VP, SZ, INT, U64, ctypes.POINTER(VP)]),
    "mpc_mp_reveal": (INT, [VP, INT, ctypes.POINTER(VP), SZ, VP]),
    "mpc_mp_dealer_triples": (INT, [VP, INT, INT, U64, U64, ctypes.POINTER(I64),
                                    ctypes.POINTER(MpTriple)]),
    "mpc_mp_dealer_trunc": (INT, [VP, INT, U64, U64, SZ, ctypes.POINTER(VP), ctypes.POINTER(VP)]),
    "mpc_mp_beaver_mul": (INT, [VP, INT, SZ, ctypes.POINTER(VP), ctypes.POINTER(VP),
                                ctypes.POINTER(MpTriple), ctypes.POINTER(VP)]),
    "mpc_mp_beaver_matmul": (INT, [VP, INT, I64, I64, I64, ctypes.POINTER(VP), ctypes.POINTER(VP),
                                   ctypes.POINTER(MpTriple), INT, ctypes.POINTER(VP)]),
    "mpc_mp_truncate": (INT, [VP, INT, SZ, INT, ctypes.POINTER(VP), ctypes.POINTER(VP),
                              ctypes.POINTER(VP)]),
}
for _name, (_res, _args) in _SIGS.items():
    _f = getattr(_lib, _name)
    _f.restype = _res
    _f.argtypes = _args


class MPCError(RuntimeError):
    def __init__(self, status, where):
        msg = _lib.mpc_status_str(status).decode()
        if status == -5:
            msg += f" (hip error {_lib.mpc_last_hip_error()})"
        super().__init__(f"{where}: {msg} [{status}]")
        self.status = status


def _check(status, where):
    if status != 0:
        raise MPCError(status, where)


def exported_symbols():
    return list(_SIGS)


# ------------------------------------------------------------------ host codec
def encode(x, frac_bits=16):
    """Host-side fixed-point encoding: round-half-even(x * 2^frac_bits) -> int64."""
    x = np.ascontiguousarray(x, dtype=np.float64)
    out = np.empty(x.shape, dtype=np.int64)
    _check(_lib.mpc_encode(x.ctypes.data, x.size, frac_bits, out.ctypes.data), "mpc_encode")
    return out


def decode(v, frac_bits=16):
    if isinstance(v, torch.Tensor):
        v = v.cpu().numpy()
    v = np.ascontiguousarray(v).view(np.int64)
    out = np.empty(v.shape, dtype=np.float64)
    _check(_lib.mpc_decode(v.ctypes.data, v.size, frac_bits, out.ctypes.data), "mpc_decode")
    return out


def limb_plan(M, N, variant):
    """Host-side planning query: how the limb GEMM tiles an M x N row-major
    output under tile schedule `variant`.  Returns (tile class, regions,
    tiles), each region (first row, first column, rows, columns, tile rows,
    tile columns)."""
    cls, count, tiles = ctypes.c_int(), ctypes.c_int(), ctypes.c_int64()
    reg = (ctypes.c_int64 * 24)()
    _check(_lib.mpc_limb_plan(M, N, variant, ctypes.byref(cls), reg, ctypes.byref(count), ctypes.byref(tiles)),
           "mpc_limb_plan")
    return cls.value, [tuple(reg[6 * i:6 * i + 6]) for i in range(count.value)], tiles.value


# ------------------------------------------------------------------ helpers
def _ptr(t):
    return VP(t.data_ptr()) if t is not None else VP(0)


class SharedPair:
    """Party 0's and party 1's shares of one secret tensor."""

    def __init__(self, s0, s1):
        self.s0, self.s1 = s0, s1

    @property
    def shape(self):
        return self.s0.shape

    def __iter__(self):
        return iter((self.s0, self.s1))


class Shared:
    """The P parties' shares of one secret tensor (P >= 2)."""

    def __init__(self, shares):
        self.shares = list(shares)

    @property
    def P(self):
        return len(self.shares)

    @property
    def shape(self):
        return self.shares[0].shape

    def __iter__(self):
        return iter(self.shares)

    def __getitem__(self, p):
        return self.shares[p]


class MpTripleShares:
    """Device buffers of a triple shared among P parties: lists a, b, c."""

    def __init__(self, a, b, c=None):
        self.a, self.b, self.c = list(a), list(b), (list(c) if c is not None else None)

    def struct(self):
        t = MpTriple()
        for p, v in enumerate(self.a):
            t.a[p] = v.data_ptr()
        for p, v in enumerate(self.b):
            t.b[p] = v.data_ptr()
        if self.c is not None:
            for p, v in enumerate(self.c):
                t.c[p] = v.data_ptr()
        return t


def _pptr(ts):
    return (VP * len(ts))(*[t.data_ptr() for t in ts])


class TripleShares:
    """Device buffers of a Beaver triple: a = (a0, a1), b = (b0, b1), c = (c0, c1)."""

    def __init__(self, a0, a1, b0, b1, c0=None, c1=None):
        self.a0, self.a1, self.b0, self.b1, self.c0, self.c1 = a0, a1, b0, b1, c0, c1

    def struct(self):
        return Triple(*[(VP(t.data_ptr()) if t is not None else VP(0))
                        for t in (self.a0, self.a1, self.b0, self.b1, self.c0, self.c1)])


class Context:
    """One library context: a device, two party streams and the parties' seed.

    Party 0's stream defaults to torch's current stream, so tensors torch
    allocates and frees on that stream are ordered with the library's work
    (torch's caching allocator may hand a freed block to the next allocation
    on that stream at once); party 1's stream is a new stream at the default
    priority, used only inside calls.  Pass ``streams`` to override; then the
    caller keeps every tensor alive (or calls ``record_stream``) until the
    work on those streams is done.
    """

    def __init__(self, device=0, seed=0, streams=None):
        self.device = torch.device("cuda", device)
        if streams is None:
            streams = (torch.cuda.current_stream(self.device),
                       torch.cuda.Stream(device=self.device))
        self.streams = streams
        h = VP()
        _check(_lib.mpc_ctx_create(device, VP(streams[0].cuda_stream),
                                   VP(streams[1].cuda_stream), seed, ctypes.byref(h)),
               "mpc_ctx_create")
        self._h = h
        self._graphs = set()

    def close(self):
        if getattr(self, "_h", None):
            for g in list(self._graphs):
                g.destroy()
            _check(_lib.mpc_ctx_destroy(self._h), "mpc_ctx_destroy")
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    # -------------------------------------------------------------- basics
    def _check_t(self, *ts, n=None, at_least=None):
        """Every tensor: contiguous int64 on this context's device; with n,
        exactly n elements; with at_least, at least that many.  The library
        takes bare pointers, so this is what keeps its kernels inside them."""
        for t in ts:
            if t is None:
                continue
            if t.device != self.device or t.dtype != torch.int64 or not t.is_contiguous():
                raise ValueError("expected contiguous int64 tensors on " + str(self.device))
            if n is not None and t.numel() != n:
                raise ValueError(f"expected {n} elements, got {t.numel()}")
            if at_least is not None and t.numel() < at_least:
                raise ValueError(f"expected at least {at_least} elements, got {t.numel()}")

    @staticmethod
    def _check_parties(P, *groups):
        for g in groups:
            if g is not None and len(g) != P:
                raise ValueError(f"expected the shares of {P} parties, got {len(g)}")

    def _check_triple(self, t, na, nb, nc):
        """A two-party triple holding at least na, nb, nc elements in a, b, c
        (nc None: a Beaver pair, whose c is not used)."""
        self._check_t(t.a0, t.a1, at_least=na)
        self._check_t(t.b0, t.b1, at_least=nb)
        if nc is not None:
            if t.c0 is None or t.c1 is None:
                raise ValueError("this product needs the triple's c shares")
            self._check_t(t.c0, t.c1, at_least=nc)

    def empty(self, shape):
        return torch.empty(shape, dtype=torch.int64, device=self.device)

    def sync(self):
        _check(_lib.mpc_sync(self._h), "mpc_sync")

    def stats(self):
        s = Stats()
        _check(_lib.mpc_ctx_stats(self._h, ctypes.byref(s)), "mpc_ctx_stats")
        return {k: int(getattr(s, k)) for k, _ in Stats._fields_}

    def profile(self, on=True):
        """Bracket every ring GEMM launch with HIP events (see mpc_profile_read)."""
        _check(_lib.mpc_profile_enable(self._h, 1 if on else 0), "mpc_profile_enable")

    def profile_read(self):
        lm, pl, fp = GemmTiming(), GemmTiming(), GemmTiming()
        _check(_lib.mpc_profile_read(self._h, ctypes.byref(lm), ctypes.byref(pl), ctypes.byref(fp)),
               "mpc_profile_read")
        as_dict = lambda g: {"launches": int(g.launches), "total_ms": float(g.total_ms),
                             "ring_macs": float(g.ring_macs)}
        return {"limb8": as_dict(lm), "plain": as_dict(pl), "fp64limb": as_dict(fp)}

    def reserve(self, nbytes):
        _check(_lib.mpc_reserve(self._h, int(nbytes)), "mpc_reserve")

    def share(self, x, src, tag, out=None):
        self._check_t(x)
        s0, s1 = (self.empty(x.shape), self.empty(x.shape)) if out is None else (out.s0, out.s1)
        self._check_t(s0, s1, n=x.numel())
        _check(_lib.mpc_share(self._h, _ptr(x), x.numel(), src, tag, _ptr(s0), _ptr(s1)),
               "mpc_share")
        return SharedPair(s0, s1)

    def reveal(self, x, out=None):
        self._check_t(x.s0, x.s1, out, n=x.s0.numel())
        out = self.empty(x.shape) if out is None else out
        _check(_lib.mpc_reveal(self._h, _ptr(x.s0), _ptr(x.s1), x.s0.numel(), _ptr(out)),
               "mpc_reveal")
        return out

    def truncate(self, x, bits):
        self._check_t(x.s0, x.s1, n=x.s0.numel())
        _check(_lib.mpc_truncate(self._h, _ptr(x.s0), _ptr(x.s1), x.s0.numel(), bits),
               "mpc_truncate")
        return x

    # -------------------------------------------------------------- dealer
    def dealer(self, kind, dseed, tag, dims):
        """Allocates and fills a triple of `kind` (TRIPLE_*) with shape `dims`."""
        if kind in (TRIPLE_MUL, TRIPLE_SQUARE):
            (n,) = dims
            sa = sb = sc = (n,)
        elif kind == TRIPLE_MATMUL:
            M, N, K = dims
            sa, sb, sc = (M, K), (K, N), (M, N)
        elif kind == TRIPLE_CONV1D:
            B, cin, L, cout, k, s = dims
            lout = (L - k) // s + 1 if L >= k else 0
            sa, sb, sc = (B, cin, L), (cout, cin, k), (B, cout, lout)
        else:
            raise ValueError("unknown triple kind")
        t = TripleShares(self.empty(sa), self.empty(sa), self.empty(sb), self.empty(sb),
                         None if kind == TRIPLE_SQUARE else self.empty(sc),
                         None if kind == TRIPLE_SQUARE else self.empty(sc))
        self.dealer_into(kind, dseed, tag, dims, t)
        return t

    def dealer_into(self, kind, dseed, tag, dims, t):
        if kind in (TRIPLE_MUL, TRIPLE_SQUARE):
            (n,) = dims
            self._check_triple(t, n, n, None if kind == TRIPLE_SQUARE else n)
        elif kind == TRIPLE_MATMUL:
            M, N, K = dims
            self._check_triple(t, M * K, K * N, M * N)
        elif kind == TRIPLE_CONV1D:
            B, cin, L, cout, k, s = dims
            lout = (L - k) // s + 1 if L >= k and s > 0 else 0
            self._check_triple(t, B * cin * L, cout * cin * k, B * cout * lout)
        d = (I64 * 6)(*list(dims) + [0] * (6 - len(dims)))
        st = t.struct()
        _check(_lib.mpc_dealer_triples(self._h, kind, dseed, tag, d, ctypes.byref(st)),
               "mpc_dealer_triples")
        return t

    # -------------------------------------------------------------- offline-packed triples
    @staticmethod
    def packed_triple_bytes(M, N, K):
        return int(_lib.mpc_packed_triple_bytes(M, N, K))

    def dealer_packed(self, dseed, tag, dims):
        """A matrix triple (the same as dealer(TRIPLE_MATMUL, ...)) and its
        offline-packed a1, b0, b1 (a uint8 device tensor)."""
        M, N, K = dims
        t = TripleShares(self.empty((M, K)), self.empty((M, K)), self.empty((K, N)), self.empty((K, N)),
                         self.empty((M, N)), self.empty((M, N)))
        packed = torch.empty(max(1, self.packed_triple_bytes(M, N, K)), dtype=torch.uint8, device=self.device)
        return self._dealer_packed_into(dseed, tag, dims, t, packed), packed

    def _dealer_packed_into(self, dseed, tag, dims, t, packed):
        M, N, K = dims
        self._check_triple(t, M * K, K * N, M * N)
        self._check_packed(packed, M, N, K)
        st = t.struct()
        _check(_lib.mpc_dealer_triples_packed(self._h, dseed, tag, M, N, K, ctypes.byref(st), _ptr(packed)),
               "mpc_dealer_triples_packed")
        return t

    def _check_packed(self, packed, M, N, K):
        if packed.device != self.device or packed.dtype != torch.uint8 or not packed.is_contiguous():
            raise ValueError("packed triple: a contiguous uint8 tensor on the context's device")
        if packed.numel() < self.packed_triple_bytes(M, N, K):
            raise ValueError("packed triple too small")

    def beaver_matmul_prepacked(self, x, y, t, packed, trunc_bits=0, out=None):
        M, K = x.s0.shape
        K2, N = y.s0.shape
        if K != K2:
            raise ValueError("inner dimensions differ")
        z = out if out is not None else SharedPair(self.empty((M, N)), self.empty((M, N)))
        self._check_t(x.s0, x.s1, n=M * K)
        self._check_t(y.s0, y.s1, n=K * N)
        self._check_t(z.s0, z.s1, n=M * N)
        self._check_triple(t, M * K, K * N, M * N)
        self._check_packed(packed, M, N, K)
        st = t.struct()
        _check(_lib.mpc_beaver_matmul_prepacked(self._h, M, N, K, _ptr(x.s0), _ptr(x.s1), _ptr(y.s0), _ptr(y.s1),
                                                ctypes.byref(st), _ptr(packed), trunc_bits, _ptr(z.s0),
                                                _ptr(z.s1)), "mpc_beaver_matmul_prepacked")
        return z

    def beaver_matmul_grouped_prepacked(self, problems, trunc_bits=0, outs=None):
        """problems: list of (x, y, triple, packed); returns the output pairs."""
        n = len(problems)
        descs = (MatmulDesc * max(1, n))()
        ptrs = (VP * max(1, n))()
        results = []
        for i, (x, y, t, packed) in enumerate(problems):
            M, K = x.s0.shape
            K2, N = y.s0.shape
            if K != K2:
                raise ValueError(f"problem {i}: inner dimensions differ")
            z = outs[i] if outs is not None else SharedPair(self.empty((M, N)), self.empty((M, N)))
            self._check_t(x.s0, x.s1, n=M * K)
            self._check_t(y.s0, y.s1, n=K * N)
            self._check_t(z.s0, z.s1, n=M * N)
            self._check_triple(t, M * K, K * N, M * N)
            self._check_packed(packed, M, N, K)
            results.append(z)
            descs[i] = MatmulDesc(M, N, K, x.s0.data_ptr(), x.s1.data_ptr(), y.s0.data_ptr(),
                                  y.s1.data_ptr(), t.struct(), z.s0.data_ptr(), z.s1.data_ptr())
            ptrs[i] = packed.data_ptr()
        _check(_lib.mpc_beaver_matmul_grouped_prepacked(self._h, n, descs, ptrs, trunc_bits),
               "mpc_beaver_matmul_grouped_prepacked")
        return results

    # -------------------------------------------------------------- binary sharing
    A2B_TRIPLES = 12

    def bin_share(self, x, src, tag, out=None):
        self._check_t(x)
        z = out if out is not None else SharedPair(self.empty(x.shape), self.empty(x.shape))
        self._check_t(z.s0, z.s1, n=x.numel())
        _check(_lib.mpc_bin_share(self._h, _ptr(x), x.numel(), src, tag, _ptr(z.s0), _ptr(z.s1)),
               "mpc_bin_share")
        return z

    def bin_reveal(self, s, out=None):
        n = s.s0.numel()
        self._check_t(s.s0, s.s1, out, n=n)
        out = out if out is not None else self.empty(s.shape)
        _check(_lib.mpc_bin_reveal(self._h, _ptr(s.s0), _ptr(s.s1), n, _ptr(out)),
               "mpc_bin_reveal")
        return out

    def dealer_and(self, dseed, tag, n):
        """n bitwise AND triples (XOR-shared words)."""
        t = TripleShares(*[self.empty((n,)) for _ in range(6)])
        st = t.struct()
        _check(_lib.mpc_dealer_and_triples(self._h, dseed, tag, n, ctypes.byref(st)),
               "mpc_dealer_and_triples")
        return t

    def bin_and(self, x, y, t, out=None):
        n = x.s0.numel()
        z = out if out is not None else SharedPair(self.empty(x.shape), self.empty(x.shape))
        self._check_t(x.s0, x.s1, y.s0, y.s1, z.s0, z.s1, n=n)
        self._check_triple(t, n, n, n)
        st = t.struct()
        _check(_lib.mpc_bin_and(self._h, x.s0.numel(), _ptr(x.s0), _ptr(x.s1), _ptr(y.s0), _ptr(y.s1),
                                ctypes.byref(st), _ptr(z.s0), _ptr(z.s1)), "mpc_bin_and")
        return z

    def a2b(self, x, tag, t, out=None):
        """Arithmetic to binary sharing; t holds 12 * n AND triples."""
        n = x.s0.numel()
        z = out if out is not None else SharedPair(self.empty(x.shape), self.empty(x.shape))
        self._check_t(x.s0, x.s1, z.s0, z.s1, n=n)
        self._check_triple(t, self.A2B_TRIPLES * n, self.A2B_TRIPLES * n, self.A2B_TRIPLES * n)
        st = t.struct()
        _check(_lib.mpc_a2b(self._h, x.s0.numel(), _ptr(x.s0), _ptr(x.s1), tag, ctypes.byref(st),
                            _ptr(z.s0), _ptr(z.s1)), "mpc_a2b")
        return z

    def dealer_b2a(self, dseed, tag, n):
        """Algorithm 2's random bits: (<r> shares, [r] shares)."""
        rb = SharedPair(self.empty((n,)), self.empty((n,)))
        ra = SharedPair(self.empty((n,)), self.empty((n,)))
        _check(_lib.mpc_dealer_b2a(self._h, dseed, tag, n, _ptr(rb.s0), _ptr(rb.s1), _ptr(ra.s0),
                                   _ptr(ra.s1)), "mpc_dealer_b2a")
        return rb, ra

    def b2a_bit(self, b, bit, rb, ra, out=None):
        n = b.s0.numel()
        z = out if out is not None else SharedPair(self.empty(b.shape), self.empty(b.shape))
        self._check_t(b.s0, b.s1, z.s0, z.s1, n=n)
        self._check_t(rb.s0, rb.s1, ra.s0, ra.s1, at_least=n)
        _check(_lib.mpc_b2a_bit(self._h, b.s0.numel(), bit, _ptr(b.s0), _ptr(b.s1), _ptr(rb.s0),
                                _ptr(rb.s1), _ptr(ra.s0), _ptr(ra.s1), _ptr(z.s0), _ptr(z.s1)),
               "mpc_b2a_bit")
        return z

    def relu(self, x, tag, t, rb, ra, m, out=None):
        """ReLU of a fixed-point sharing: t 12*n AND triples, (rb, ra) B2A bits, m MUL triple."""
        n = x.s0.numel()
        z = out if out is not None else SharedPair(self.empty(x.shape), self.empty(x.shape))
        self._check_t(x.s0, x.s1, z.s0, z.s1, n=n)
        self._check_triple(t, self.A2B_TRIPLES * n, self.A2B_TRIPLES * n, self.A2B_TRIPLES * n)
        self._check_t(rb.s0, rb.s1, ra.s0, ra.s1, at_least=n)
        self._check_triple(m, n, n, n)
        st, sm = t.struct(), m.struct()
        _check(_lib.mpc_relu(self._h, x.s0.numel(), _ptr(x.s0), _ptr(x.s1), tag, ctypes.byref(st),
                             _ptr(rb.s0), _ptr(rb.s1), _ptr(ra.s0), _ptr(ra.s1), ctypes.byref(sm),
                             _ptr(z.s0), _ptr(z.s1)), "mpc_relu")
        return z

    # -------------------------------------------------------------- more than two parties
    def mp_share(self, x, P, src, tag, out=None):
        """Shares x among P parties (pseudorandom zero-share; party src adds x)."""
        self._check_t(x)
        s = out if out is not None else Shared([self.empty(x.shape) for _ in range(P)])
        self._check_parties(P, s.shares)
        self._check_t(*s.shares, n=x.numel())
        _check(_lib.mpc_mp_share(self._h, P, _ptr(x), x.numel(), src, tag, _pptr(s.shares)),
               "mpc_mp_share")
        return s

    def mp_reveal(self, s, out=None):
        n = s.shares[0].numel()
        self._check_t(*s.shares, out, n=n)
        out = out if out is not None else self.empty(s.shape)
        _check(_lib.mpc_mp_reveal(self._h, s.P, _pptr(s.shares), n, _ptr(out)),
               "mpc_mp_reveal")
        return out

    def mp_dealer(self, P, kind, dseed, tag, dims):
        if kind in (TRIPLE_MUL, TRIPLE_SQUARE):
            (n,) = dims
            sa = sb = sc = (n,)
        elif kind == TRIPLE_MATMUL:
            M, N, K = dims
            sa, sb, sc = (M, K), (K, N), (M, N)
        else:
            raise ValueError("multi-party triples: MUL, SQUARE or MATMUL")
        t = MpTripleShares([self.empty(sa) for _ in range(P)], [self.empty(sb) for _ in range(P)],
                           None if kind == TRIPLE_SQUARE else [self.empty(sc) for _ in range(P)])
        d = (I64 * 3)(*(list(dims) + [0] * (3 - len(dims))))
        st = t.struct()
        _check(_lib.mpc_mp_dealer_triples(self._h, P, kind, dseed, tag, d, ctypes.byref(st)),
               "mpc_mp_dealer_triples")
        return t

    def mp_dealer_trunc(self, P, dseed, tag, n):
        """Algorithm 1's dealer inputs: (shares of r, shares of r's wrap count)."""
        r = Shared([self.empty((n,)) for _ in range(P)])
        th = Shared([self.empty((n,)) for _ in range(P)])
        _check(_lib.mpc_mp_dealer_trunc(self._h, P, dseed, tag, n, _pptr(r.shares), _pptr(th.shares)),
               "mpc_mp_dealer_trunc")
        return r, th

    def mp_beaver_mul(self, x, y, t, out=None):
        """P-party Beaver product; y=None selects the square with the pair t."""
        P = x.P
        n = x.shares[0].numel()
        z = out if out is not None else Shared([self.empty(x.shape) for _ in range(P)])
        self._check_parties(P, y.shares if y is not None else None, t.a, t.b, t.c if y is not None else None,
                            z.shares)
        self._check_t(*x.shares, *(y.shares if y is not None else []), *z.shares, n=n)
        self._check_t(*t.a, *t.b, at_least=n)
        if y is not None:
            if t.c is None:
                raise ValueError("a product needs the triple's c shares")
            self._check_t(*t.c, at_least=n)
        st = t.struct()
        _check(_lib.mpc_mp_beaver_mul(self._h, P, x.shares[0].numel(), _pptr(x.shares),
                                      _pptr(y.shares) if y is not None else None, ctypes.byref(st),
                                      _pptr(z.shares)), "mpc_mp_beaver_mul")
        return z

    def mp_beaver_matmul(self, x, y, t, form="auto", out=None):
        P = x.P
        M, K = x.shape
        K2, N = y.shape
        if K != K2:
            raise ValueError("inner dimensions differ")
        z = out if out is not None else Shared([self.empty((M, N)) for _ in range(P)])
        self._check_parties(P, y.shares, t.a, t.b, t.c, z.shares)
        self._check_t(*x.shares, n=M * K)
        self._check_t(*y.shares, n=K * N)
        self._check_t(*z.shares, n=M * N)
        self._check_t(*t.a, at_least=M * K)
        self._check_t(*t.b, at_least=K * N)
        self._check_t(*t.c, at_least=M * N)
        st = t.struct()
        _check(_lib.mpc_mp_beaver_matmul(self._h, P, M, N, K, _pptr(x.shares), _pptr(y.shares),
                                         ctypes.byref(st), FORMS[form], _pptr(z.shares)),
               "mpc_mp_beaver_matmul")
        return z

    def mp_truncate(self, x, bits, r, theta_r):
        """In-place truncation by 2^bits (Algorithm 1, eta = 0)."""
        n = x.shares[0].numel()
        self._check_parties(x.P, r.shares, theta_r.shares)
        self._check_t(*x.shares, n=n)
        self._check_t(*r.shares, *theta_r.shares, at_least=n)
        _check(_lib.mpc_mp_truncate(self._h, x.P, x.shares[0].numel(), bits, _pptr(x.shares),
                                    _pptr(r.shares), _pptr(theta_r.shares)), "mpc_mp_truncate")
        return x

    # -------------------------------------------------------------- Beaver
    def beaver_mul(self, x, y, t, trunc_bits=0, out=None):
        """y=None selects the square with a Beaver pair (t.a, t.b = a^2)."""
        n = x.s0.numel()
        z = out if out is not None else SharedPair(self.empty(x.shape), self.empty(x.shape))
        self._check_t(x.s0, x.s1, z.s0, z.s1, *((y.s0, y.s1) if y is not None else ()), n=n)
        self._check_triple(t, n, n, n if y is not None else None)
        st = t.struct()
        _check(_lib.mpc_beaver_mul(self._h, n, _ptr(x.s0), _ptr(x.s1),
                                   _ptr(y.s0 if y is not None else None),
                                   _ptr(y.s1 if y is not None else None), ctypes.byref(st),
                                   trunc_bits, _ptr(z.s0), _ptr(z.s1)), "mpc_beaver_mul")
        return z

    def beaver_matmul(self, x, y, t, trunc_bits=0, form="auto", out=None):
        M, K = x.s0.shape
        K2, N = y.s0.shape
        if K != K2:
            raise ValueError("inner dimensions differ")
        z = out if out is not None else SharedPair(self.empty((M, N)), self.empty((M, N)))
        self._check_t(x.s0, x.s1, n=M * K)
        self._check_t(y.s0, y.s1, n=K * N)
        self._check_t(z.s0, z.s1, n=M * N)
        self._check_triple(t, M * K, K * N, M * N)
        st = t.struct()
        _check(_lib.mpc_beaver_matmul(self._h, M, N, K, _ptr(x.s0), _ptr(x.s1), _ptr(y.s0),
                                      _ptr(y.s1), ctypes.byref(st), trunc_bits, FORMS[form],
                                      _ptr(z.s0), _ptr(z.s1)), "mpc_beaver_matmul")
        return z

    def beaver_matmul_noalloc(self, x, y, t, trunc_bits=0, form="auto", out=None):
        """beaver_matmul through the entry point that allocates nothing (its
        workspace is the library's static per-device array); `out` should be
        given by callers that must not allocate either."""
        M, K = x.s0.shape
        K2, N = y.s0.shape
        if K != K2:
            raise ValueError("inner dimensions differ")
        z = out if out is not None else SharedPair(self.empty((M, N)), self.empty((M, N)))
        self._check_t(x.s0, x.s1, n=M * K)
        self._check_t(y.s0, y.s1, n=K * N)
        self._check_t(z.s0, z.s1, n=M * N)
        self._check_triple(t, M * K, K * N, M * N)
        st = t.struct()
        _check(_lib.mpc_beaver_matmul_noalloc(self._h, M, N, K, _ptr(x.s0), _ptr(x.s1), _ptr(y.s0),
                                              _ptr(y.s1), ctypes.byref(st), trunc_bits, FORMS[form],
                                              _ptr(z.s0), _ptr(z.s1)), "mpc_beaver_matmul_noalloc")
        return z

    def beaver_conv1d(self, x, w, t, stride, trunc_bits=0, form="auto", out=None):
        B, cin, L = x.s0.shape
        cout, cin2, k = w.s0.shape
        if cin != cin2:
            raise ValueError("channel counts differ")
        lout = (L - k) // stride + 1 if L >= k and stride > 0 else 0
        shape = Conv1dShape(B, cin, L, cout, k, stride)
        z = out if out is not None else SharedPair(self.empty((B, cout, lout)),
                                                   self.empty((B, cout, lout)))
        self._check_t(x.s0, x.s1, n=B * cin * L)
        self._check_t(w.s0, w.s1, n=cout * cin * k)
        self._check_t(z.s0, z.s1, n=B * cout * lout)
        self._check_triple(t, B * cin * L, cout * cin * k, B * cout * lout)
        st = t.struct()
        _check(_lib.mpc_beaver_conv1d(self._h, ctypes.byref(shape), _ptr(x.s0), _ptr(x.s1),
                                      _ptr(w.s0), _ptr(w.s1), ctypes.byref(st), trunc_bits,
                                      FORMS[form], _ptr(z.s0), _ptr(z.s1)), "mpc_beaver_conv1d")
        return z

    def ring_gemm(self, A, B, form="auto", out=None):
        M, K = A.shape
        K2, N = B.shape
        if K != K2:
            raise ValueError("inner dimensions differ")
        C = out if out is not None else self.empty((M, N))
        self._check_t(A, n=M * K)
        self._check_t(B, n=K * N)
        self._check_t(C, n=M * N)
        _check(_lib.mpc_ring_gemm(self._h, M, N, K, _ptr(A), _ptr(B), _ptr(C), FORMS[form]),
               "mpc_ring_gemm")
        return C

    def beaver_matmul_grouped(self, problems, trunc_bits=0, form="auto", outs=None):
        """problems: list of (x, y, triple); returns the list of output pairs."""
        descs = (MatmulDesc * max(1, len(problems)))()
        results = []
        for i, (x, y, t) in enumerate(problems):
            M, K = x.s0.shape
            K2, N = y.s0.shape
            if K != K2:
                raise ValueError(f"problem {i}: inner dimensions differ")
            z = outs[i] if outs is not None else SharedPair(self.empty((M, N)),
                                                            self.empty((M, N)))
            self._check_t(x.s0, x.s1, n=M * K)
            self._check_t(y.s0, y.s1, n=K * N)
            self._check_t(z.s0, z.s1, n=M * N)
            self._check_triple(t, M * K, K * N, M * N)
            results.append(z)
            descs[i] = MatmulDesc(M, N, K, x.s0.data_ptr(), x.s1.data_ptr(), y.s0.data_ptr(),
                                  y.s1.data_ptr(), t.struct(), z.s0.data_ptr(), z.s1.data_ptr())
        _check(_lib.mpc_beaver_matmul_grouped(self._h, len(problems), descs, trunc_bits,
                                              FORMS[form]), "mpc_beaver_matmul_grouped")
        return results

    def beaver_mul_grouped(self, problems, trunc_bits=0, outs=None):
        """problems: list of (x, y or None, triple); one launch for all of them;
        returns the list of output pairs (y None: square with the pair a, a^2)."""
        descs = (MulDesc * max(1, len(problems)))()
        results = []
        for i, (x, y, t) in enumerate(problems):
            n = x.s0.numel()
            z = outs[i] if outs is not None else SharedPair(self.empty(x.shape), self.empty(x.shape))
            self._check_t(x.s0, x.s1, z.s0, z.s1, *((y.s0, y.s1) if y is not None else ()), n=n)
            self._check_triple(t, n, n, n if y is not None else None)
            results.append(z)
            descs[i] = MulDesc(x.s0.numel(), _ptr(x.s0), _ptr(x.s1), _ptr(y.s0 if y is not None else None),
                               _ptr(y.s1 if y is not None else None), t.struct(), _ptr(z.s0), _ptr(z.s1))
        _check(_lib.mpc_beaver_mul_grouped(self._h, len(problems), descs, trunc_bits),
               "mpc_beaver_mul_grouped")
        return results

    # -------------------------------------------------------------- autotuning
    def autotune_matmul(self, shapes):
        """Tune the limb GEMM schedule for a Beaver matmul (one shape) or a
        grouped call of these (M, N, K) shapes; returns the chosen schedule."""
        flat = [int(v) for s in shapes for v in s]
        dims = (I64 * max(1, len(flat)))(*flat)
        best = TileConfig()
        _check(_lib.mpc_autotune_matmul(self._h, len(shapes), dims, ctypes.byref(best)),
               "mpc_autotune_matmul")
        return {"variant": TILE_VARIANTS[best.variant], "group_m": best.group_m,
                "xcd_remap": bool(best.xcd_remap), "ms": best.ms}

    def autotune_save(self, path):
        _check(_lib.mpc_autotune_save(self._h, str(path).encode()), "mpc_autotune_save")

    def autotune_load(self, path):
        _check(_lib.mpc_autotune_load(self._h, str(path).encode()), "mpc_autotune_load")

    def set_default_tile_config(self, variant=0, group_m=8, xcd_remap=True):
        cfg = TileConfig(variant, group_m, 1 if xcd_remap else 0, 0.0)
        _check(_lib.mpc_set_default_tile_config(self._h, ctypes.byref(cfg)),
               "mpc_set_default_tile_config")

    def default_tile_config(self):
        cfg = TileConfig()
        _check(_lib.mpc_get_default_tile_config(self._h, ctypes.byref(cfg)), "mpc_get_default_tile_config")
        return {"variant": TILE_VARIANTS[cfg.variant], "variant_id": int(cfg.variant),
                "group_m": int(cfg.group_m), "xcd_remap": bool(cfg.xcd_remap)}

    # -------------------------------------------------------------- graphs
    def graph_begin(self):
        _check(_lib.mpc_graph_begin(self._h), "mpc_graph_begin")

    def graph_end(self):
        """Ends the capture; returns a Graph, which keeps this context alive
        until it is destroyed (the library refuses to destroy a context whose
        graphs still exist)."""
        h = VP()
        _check(_lib.mpc_graph_end(self._h, ctypes.byref(h)), "mpc_graph_end")
        g = Graph(self, h)
        self._graphs.add(g)
        return g

    def graph_launch(self, g):
        if not isinstance(g, Graph) or g.ctx is not self or not g._h:
            raise ValueError("not a live graph of this context")
        _check(_lib.mpc_graph_launch(self._h, g._h), "mpc_graph_launch")

    @staticmethod
    def graph_destroy(g):
        g.destroy()


class Graph:
    """An instantiated capture of a context's calls (see Context.graph_end)."""

    def __init__(self, ctx, h):
        self.ctx, self._h = ctx, h

    def destroy(self):
        if self._h:
            h, self._h = self._h, None
            self.ctx._graphs.discard(self)
            _check(_lib.mpc_graph_destroy(h), "mpc_graph_destroy")

    def __del__(self):
        try:
            self.destroy()
        except Exception:
            pass
