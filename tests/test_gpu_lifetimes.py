"""Host-side contracts of the library on a live context: graph and context
lifetimes, and the bounds of a tile schedule (its raster group height)."""
import ctypes

import pytest
import torch

import workloads
from tests.gpu_util import say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def m():
    import paper_2109_00984_amd as mod
    return mod


def test_graph_begin_refuses_null_stream(m):
    # torch's default stream is the null stream, which cannot be captured
    c = m.Context(device=0, seed=1, streams=(torch.cuda.default_stream(0), torch.cuda.Stream(0)))
    try:
        if c.streams[0].cuda_stream == 0:
            with pytest.raises(m.MPCError) as ei:
                c.graph_begin()
            assert ei.value.status == m.MPC_E_INVAL
        # the context still works eagerly
        x = c.share(torch.arange(64, dtype=torch.int64, device=c.device), 0, 1)
        r = c.reveal(x)
        c.sync()
        assert torch.equal(r.cpu(), torch.arange(64, dtype=torch.int64))
    finally:
        c.close()


def test_context_refuses_destroy_with_live_graph(m):
    say("lifetimes: context destroy with a live graph")
    with torch.cuda.stream(torch.cuda.Stream()):
        _destroy_with_live_graph(m)


def _destroy_with_live_graph(m):
    c = m.Context(device=0, seed=1)
    x = c.share(torch.arange(1024, dtype=torch.int64, device=c.device), 0, 1)
    t = c.dealer(m.TRIPLE_SQUARE, 3, 4, (1024,))
    c.sync()
    c.graph_begin()
    c.beaver_mul(x, None, t, 16)
    g = c.graph_end()
    # the raw C ABI refuses while the graph exists
    st = m._lib.mpc_ctx_destroy(c._h)
    assert st == m.MPC_E_INVAL
    c.graph_launch(g)
    c.sync()
    # the binding destroys the context's graphs first
    c.close()
    assert g._h is None
    g.destroy()  # a second destroy is a no-op


def test_graph_of_other_context_refused(m):
    with torch.cuda.stream(torch.cuda.Stream()):
        _graph_of_other_context(m)


def _graph_of_other_context(m):
    a, b = m.Context(device=0, seed=1), m.Context(device=0, seed=2)
    try:
        x = a.share(torch.arange(64, dtype=torch.int64, device=a.device), 0, 1)
        a.sync()
        a.graph_begin()
        a.truncate(x, 3)
        g = a.graph_end()
        with pytest.raises(ValueError):
            b.graph_launch(g)
        g.destroy()
        with pytest.raises(ValueError):
            a.graph_launch(g)
    finally:
        a.close()
        b.close()


def test_tile_schedule_bounds(m, tmp_path):
    c = m.Context(device=0, seed=workloads.seeds(0)[1])
    try:
        before = c.default_tile_config()
        for gm in (0, 65, 1 << 20):
            with pytest.raises(m.MPCError):
                c.set_default_tile_config(variant=before["variant_id"], group_m=gm)
        assert c.default_tile_config() == before
        c.set_default_tile_config(variant=before["variant_id"], group_m=64)
        assert c.default_tile_config()["group_m"] == 64
        # a cache file (hash, then three classes' variant, group_m, remap) with
        # out-of-range entries in some class: those lines are ignored
        p = tmp_path / "tune.txt"
        p.write_text("00000000000000aa 5 8 1 5 100000 1 5 8 1\n"
                     "00000000000000bb 5 8 1 5 8 1 99 8 1\n"
                     "00000000000000dd 5 8 1 -1 8 1 5 8 1\n"
                     "00000000000000cc 5 8 1 12 4 0 14 16 1\n")
        c.autotune_load(p)
        out = tmp_path / "saved.txt"
        c.autotune_save(out)
        lines = out.read_text().split()
        assert lines == ["00000000000000cc", "5", "8", "1", "12", "4", "0", "14", "16", "1"]
    finally:
        c.close()
