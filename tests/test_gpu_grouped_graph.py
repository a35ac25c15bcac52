"""The batching workload as specified: 256 Beaver matmuls of log-uniform
shapes (M in [16, 2048], N in [16, 1024], K in [32, 4096]) with 2^16
truncation, limb form, tile schedule chosen by the library's autotuner (or
the persistent grouped launch, schedule 15, set as the default), captured
once in a HIP graph and replayed.  Every replay is compared with the
eager call on every element of both parties' shares, and the eager call with
the oracle: in full where M*N*K <= 2^22, at sampled outputs of every other
problem (section 6.1: batching amortises rounds; App. C.1.1, multiplication
with a matrix triple)."""
import numpy as np
import pytest
import torch

import oracle
import workloads
from tests.gpu_util import dev, host, say

pytestmark = pytest.mark.gpu
FRAC = 16
FULL_MNK = 1 << 22


@pytest.fixture(scope="module")
def m():
    import paper_2109_00984_amd as mod
    return mod


def sample_positions(seed, M, N, count):
    g = workloads.rng(seed)
    rows = g.integers(0, M, size=count)
    cols = g.integers(0, N, size=count)
    rows[:2], cols[:2] = [0, M - 1], [0, N - 1]
    return rows, cols


@pytest.mark.parametrize("schedule", ["autotuned", "persistent"])
def test_grouped_256_graph_replay(m, schedule):
    # captured on a stream of its own: the null stream cannot be captured
    with torch.cuda.stream(torch.cuda.Stream()):
        _grouped_256_graph_replay(m, schedule)


def _grouped_256_graph_replay(m, schedule):
    data_seed, pseed, dseed = workloads.seeds(5)
    shapes = workloads.grouped_shapes(data_seed, **{k: v for k, v in workloads.GROUPED.items() if k != "count"})
    assert len(shapes) == 256
    c = m.Context(device=0, seed=pseed)
    try:
        say("grouped graph: building 256 problems")
        probs, host_in = [], []
        for i, (M, N, K) in enumerate(shapes):
            X = workloads.uniform_u64(data_seed * 1000 + 2 * i, (M, K))
            Y = workloads.uniform_u64(data_seed * 1000 + 2 * i + 1, (K, N))
            x, y = c.share(dev(X), 0, 2 * i), c.share(dev(Y), 1, 2 * i + 1)
            probs.append((x, y, c.dealer(m.TRIPLE_MATMUL, dseed, i, (M, N, K))))
            host_in.append((X, Y))
        if schedule == "autotuned":
            say("grouped graph: autotune")
            best = c.autotune_matmul(shapes)
            say(f"grouped graph: tuned schedule {best}")
        else:
            c.set_default_tile_config(15, 8, True)  # every problem in its own tile class, one persistent launch
            c.profile(True)
            c.profile_read()
            c.beaver_matmul_grouped(probs, FRAC, "limb8")
            c.sync()
            assert c.profile_read()["limb8"]["launches"] == 1
            c.profile(False)
        outs = [m.SharedPair(c.empty((M, N)), c.empty((M, N))) for (M, N, K) in shapes]
        eager = c.beaver_matmul_grouped(probs, FRAC, "limb8")  # also sizes the workspace
        c.sync()
        say("grouped graph: capture")
        c.graph_begin()
        c.beaver_matmul_grouped(probs, FRAC, "limb8", outs=outs)
        g = c.graph_end()
        try:
            for rep in range(3):
                for o in outs:
                    o.s0.fill_(-1)
                    o.s1.fill_(-1)
                say(f"grouped graph: replay {rep}")
                c.graph_launch(g)
                c.sync()
                for i, (o, e) in enumerate(zip(outs, eager)):
                    assert torch.equal(o.s0, e.s0) and torch.equal(o.s1, e.s1), \
                        f"replay {rep}: problem {i} {shapes[i]} differs from the eager call"
                # eager work of the same context between replays
                scratch = c.beaver_matmul(*probs[rep], FRAC, "limb8")
                c.sync()
                assert torch.equal(scratch.s0, eager[rep].s0) and torch.equal(scratch.s1, eager[rep].s1)
        finally:
            g.destroy()
        say("grouped graph: oracle")
        full = 0
        for i, ((M, N, K), (X, Y)) in enumerate(zip(shapes, host_in)):
            xs, ys = oracle.share(X, 0, pseed, 2 * i), oracle.share(Y, 1, pseed, 2 * i + 1)
            got = (host(c, eager[i].s0), host(c, eager[i].s1))
            if M * N * K <= FULL_MNK:
                full += 1
                want = oracle.beaver_matmul(xs, ys, oracle.dealer_matmul(dseed, i, M, N, K), FRAC)
                assert np.array_equal(got[0], want[0]) and np.array_equal(got[1], want[1]), \
                    f"problem {i} {shapes[i]}: differs from the oracle"
            else:
                rows, cols = sample_positions(i, M, N, 16)
                a, b = oracle.dealer_matmul_ab(dseed, i, M, N, K)
                c_at = oracle.dealer_matmul_c_at(dseed, i, M, N, K, a, b, rows, cols)
                want = oracle.beaver_matmul_at(xs, ys, a, b, c_at, FRAC, rows, cols)
                assert np.array_equal(got[0][rows, cols], want[0]) and np.array_equal(got[1][rows, cols], want[1]), \
                    f"problem {i} {shapes[i]}: differs from the oracle at sampled outputs"
        say(f"grouped graph: {full} problems compared in full, {256 - full} at sampled outputs")
        assert full > 0
    finally:
        c.close()
