"""The C-ABI library loads and exports every entry point its header declares;
its host-only codec matches the oracle.  No GPU needed (no kernel is called)."""
import ctypes
import os
import re

import numpy as np

import oracle
import workloads

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "mpc.h")
LIB = os.path.join(ROOT, "paper_2109_00984_amd", "libmpc.so")


def declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(mpc_[a-z0-9_]+)\s*\(", text)))


def test_header_declares_the_boundary():
    names = declared()
    for required in ["mpc_share", "mpc_dealer_triples", "mpc_beaver_mul", "mpc_beaver_matmul",
                     "mpc_truncate", "mpc_reveal"]:
        assert required in names


def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(LIB)
    missing = [n for n in declared() if not hasattr(lib, n)]
    assert not missing, missing


def test_binding_covers_the_header():
    import paper_2109_00984_amd as m
    assert sorted(m.exported_symbols()) == declared()


def test_host_codec_matches_oracle():
    import paper_2109_00984_amd as m
    x = np.concatenate([workloads.uniform(1, 5000, -4, 4),
                        np.array([2.0 ** -17, 3 * 2.0 ** -17, -2.0 ** -17, 0.0, -1.5])])
    assert np.array_equal(m.encode(x, 16), oracle.encode(x, 16))
    v = m.encode(x, 16)
    assert np.array_equal(m.decode(v, 16), oracle.decode(v.view(np.uint64), 16))


def test_host_codec_rejects_out_of_range():
    import paper_2109_00984_amd as m
    import pytest
    with pytest.raises(m.MPCError):
        m.encode(np.array([2.0 ** 47]), 16)
    with pytest.raises(m.MPCError):
        m.encode(np.array([np.nan]), 16)
    with pytest.raises(m.MPCError):
        m.encode(np.array([1.0]), 63)


def test_bench_refuses_more_than_one_gpu():
    # the benchmark measures one GPU (both parties' shares live on it); it
    # says so and exits before touching any device
    import subprocess
    import sys
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "8"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""


def test_packed_triple_bytes():
    # host-only: the offline-packed a1 (M x K), b0 and b1 (K x N), each a grid
    # of 8 KiB blocks of 32 rows (columns) x 32 k, rows padded to 4 blocks and
    # k to an even number of blocks, every operand 256-byte aligned
    import paper_2109_00984_amd as m

    def packed(rows, K):
        rb = -(-(-(-rows // 32)) // 4) * 4
        kb = -(-K // 64) * 2
        return rb * kb * 8192

    for M, N, K in [(1, 1, 1), (64, 32, 128), (300, 17, 4097), (4096, 4096, 4096), (0, 5, 7)]:
        want = packed(M, K) + 2 * packed(N, K)
        assert m.Context.packed_triple_bytes(M, N, K) == want, (M, N, K)
    assert m.Context.packed_triple_bytes(-1, 2, 3) == 0
