"""Party streams: the one hand-off between them.

Every call is issued on party 0's stream.  Both parties' shares are on the
one GPU, so the Beaver kernels read and write both parties' buffers in one
pass on that stream; the only per-party work is truncation after a product
(Table 1: zero rounds for two parties), which mpc_truncate runs for party 1
on party 1's stream, after an event on party 0's stream, and joins back.
These tests queue slow work before the call on each stream and read the
result on party 0's stream without any host synchronisation in between, so
a missing wait in either direction shows up as a wrong value; the expected
values are the oracle's floor truncation (App. C.1.1, truncation)."""
import numpy as np
import pytest
import torch

import oracle
import workloads
from tests.gpu_util import dev, say

pytestmark = pytest.mark.gpu
N = 1 << 22
BITS = 16


@pytest.fixture(scope="module")
def m():
    import paper_2109_00984_amd as mod
    return mod


def busy(device):
    """About a few milliseconds of matrix work on the current stream."""
    a = torch.full((4096, 4096), 1.0 / 4096, device=device)
    for _ in range(6):
        a = a @ a
    return a


@pytest.mark.parametrize("writer", [0, 1])
def test_truncate_after_slow_writer(m, writer):
    """The share party 1 truncates is written, behind slow work, on party
    `writer`'s stream just before the call."""
    say(f"streams: truncate after slow work on party {writer}'s stream")
    s0h, s1h = workloads.uniform_u64(51, (N,)), workloads.uniform_u64(52, (N,))
    want0, want1 = oracle.truncate(s0h, BITS), oracle.truncate(s1h, BITS)
    side = torch.cuda.Stream()
    with torch.cuda.stream(side):
        c = m.Context(device=0, seed=5)
        try:
            src0, src1 = dev(s0h), dev(s1h)
            s0 = torch.empty_like(src0)
            s1 = torch.zeros_like(src1)
            torch.cuda.synchronize()
            s0.copy_(src0)
            w = c.streams[writer]
            w.wait_stream(side)
            with torch.cuda.stream(w):
                busy(c.device)
                s1.copy_(src1)
            c.truncate(m.SharedPair(s0, s1), BITS)
            # read back on party 0's stream, no host synchronisation before
            got0, got1 = s0.clone(), s1.clone()
            got0, got1 = got0.cpu().numpy().view(np.uint64), got1.cpu().numpy().view(np.uint64)
        finally:
            c.close()
    assert np.array_equal(got0, want0)
    assert np.array_equal(got1, want1)


def test_truncate_then_slow_reader_on_party1(m):
    """Work the caller queues on party 1's stream after the call sees party
    1's truncated share (the call leaves party 1's stream ordered after it)."""
    say("streams: party 1's stream reads after the call")
    s0h, s1h = workloads.uniform_u64(53, (N,)), workloads.uniform_u64(54, (N,))
    want1 = oracle.truncate(s1h, BITS)
    side = torch.cuda.Stream()
    with torch.cuda.stream(side):
        c = m.Context(device=0, seed=6)
        try:
            s0, s1 = dev(s0h), dev(s1h)
            torch.cuda.synchronize()
            busy(c.device)  # party 0's stream is still busy when the call is issued
            c.truncate(m.SharedPair(s0, s1), BITS)
            with torch.cuda.stream(c.streams[1]):
                got1 = s1.clone()
            torch.cuda.synchronize()
            got1 = got1.cpu().numpy().view(np.uint64)
        finally:
            c.close()
    assert np.array_equal(got1, want1)


def test_randomized_delays(m):
    """Seeded random schedules around the hand-off: slow work of random length
    on each party's stream, random host sleeps between enqueueing it and the
    call, party 1's share written on either stream and read back on either
    stream, ragged sizes.  Only stream order connects the steps."""
    import time
    g = workloads.rng(2109)
    side = torch.cuda.Stream()
    with torch.cuda.stream(side):
        c = m.Context(device=0, seed=7)
        try:
            for trial in range(8):
                n = int(g.choice([1, 4097, (1 << 20) + 3, N]))
                b0, b1 = int(g.integers(0, 4)), int(g.integers(0, 4))
                w1, r1 = int(g.integers(0, 2)), int(g.integers(0, 2))
                sleep_ms = float(g.uniform(0, 3))
                say(f"streams: trial {trial} n={n} busy=({b0},{b1}) writer1={w1} reader1={r1} sleep={sleep_ms:.1f}ms")
                s0h, s1h = workloads.uniform_u64(60 + 2 * trial, (n,)), workloads.uniform_u64(61 + 2 * trial, (n,))
                src0, src1 = dev(s0h), dev(s1h)
                s0, s1 = torch.zeros_like(src0), torch.zeros_like(src1)
                torch.cuda.synchronize()
                p0, p1 = c.streams
                p0.wait_stream(side)
                p1.wait_stream(side)
                with torch.cuda.stream(p0):
                    for _ in range(b0):
                        busy(c.device)
                    s0.copy_(src0)
                with torch.cuda.stream(c.streams[w1]):
                    for _ in range(b1):
                        busy(c.device)
                    s1.copy_(src1)
                time.sleep(sleep_ms / 1e3)
                c.truncate(m.SharedPair(s0, s1), BITS)
                with torch.cuda.stream(p0):
                    got0 = s0.clone()
                with torch.cuda.stream(c.streams[r1]):
                    got1 = s1.clone()
                torch.cuda.synchronize()
                assert np.array_equal(got0.cpu().numpy().view(np.uint64), oracle.truncate(s0h, BITS)), trial
                assert np.array_equal(got1.cpu().numpy().view(np.uint64), oracle.truncate(s1h, BITS)), trial
        finally:
            c.close()
