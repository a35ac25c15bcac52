"""Host planning of the limb GEMM (no GPU): the tile class a product takes
and the output regions it runs as (edge strips under the classes schedules).
The regions are pointer offsets into the packed operands, the output and the
triple share, so they must cover the output exactly, start on 32-row and
32-column block boundaries and keep every tile inside the padded operands."""
import numpy as np
import pytest

import paper_2109_00984_amd as m

# documented tile shapes of the single-shape schedules 0..13 (rows, columns)
VARIANT_TILE = {0: (128, 64), 1: (64, 128), 2: (64, 64), 3: (128, 64), 4: (64, 128), 5: (64, 64),
                6: (64, 128), 7: (128, 64), 8: (64, 128), 9: (64, 64), 10: (64, 128), 11: (128, 64),
                12: (32, 128), 13: (128, 32)}
CLASS_TILE = {0: (64, 64), 1: (32, 128), 2: (128, 32)}
EDGES = [1, 2, 16, 31, 32, 33, 48, 63, 64, 65, 95, 96, 97, 127, 128, 129, 160, 191, 200, 255, 257, 1000,
         2047, 2049, 4095, 4096, 4097]


def cdiv(a, b):
    return -(-a // b)


def padded(v):
    return cdiv(v, 128) * 128


def expected_class(M, N):
    # the class rule as the header states it
    area = lambda bm, bn: cdiv(M, bm) * bm * cdiv(N, bn) * bn
    reg, tm, tn = area(64, 64), area(32, 128), area(128, 32)
    if M <= 32 and tm <= 0.9 * reg and tm <= tn:
        return 1
    if N <= 32 and tn <= 0.9 * reg:
        return 2
    return 0


def shapes():
    g = np.random.default_rng(2109)
    out = [(a, b) for a in EDGES for b in EDGES]
    out += [(int(a), int(b)) for a, b in zip(np.exp(g.uniform(0, np.log(8192), 300)).astype(int) + 1,
                                             np.exp(g.uniform(0, np.log(8192), 300)).astype(int) + 1)]
    return out


def check_plan(M, N, variant):
    cls, regs, tiles = m.limb_plan(M, N, variant)
    assert cls == expected_class(M, N), (M, N)
    cover = np.zeros((M, N), dtype=np.int8) if M * N <= 1 << 22 else None
    area, count = 0, 0
    for (r0, c0, rows, cols, bm, bn) in regs:
        assert rows >= 1 and cols >= 1 and r0 % 32 == 0 and c0 % 32 == 0, (M, N, variant, regs)
        assert r0 + rows <= M and c0 + cols <= N, (M, N, variant, regs)
        # every tile reads only row and column blocks inside the padded operands
        assert r0 + cdiv(rows, bm) * bm <= padded(M) and c0 + cdiv(cols, bn) * bn <= padded(N), \
            (M, N, variant, regs)
        if variant in (14, 15):
            assert (bm, bn) in CLASS_TILE.values()
        else:
            assert (bm, bn) == VARIANT_TILE[variant]
        if cover is not None:
            cover[r0:r0 + rows, c0:c0 + cols] += 1
        area += rows * cols
        count += cdiv(rows, bm) * cdiv(cols, bn)
    # the regions cover the output exactly once
    assert area == M * N, (M, N, variant, regs)
    if cover is not None:
        assert cover.min() == 1 and cover.max() == 1, (M, N, variant, regs)
    assert tiles == count
    return cls, regs, tiles


@pytest.mark.parametrize("variant", list(range(16)))
def test_plan_covers_output(variant):
    for (M, N) in shapes():
        cls, regs, _ = check_plan(M, N, variant)
        if variant not in (14, 15):
            assert regs == [(0, 0, M, N) + VARIANT_TILE[variant]]
        elif cls != 0:
            assert regs == [(0, 0, M, N) + CLASS_TILE[cls]]


def test_edge_strips():
    # 200 x 136: 64x64 interior, 8-row strip of 32x128 tiles, 8-column strip of
    # 128x32 tiles, one 64x64 corner tile
    for variant in (14, 15):
        cls, regs, tiles = m.limb_plan(200, 136, variant)
        assert cls == 0
        assert regs == [(0, 0, 192, 128, 64, 64), (192, 0, 8, 128, 32, 128), (0, 128, 192, 8, 128, 32),
                        (192, 128, 8, 8, 64, 64)]
        assert tiles == 6 + 1 + 2 + 1
    # leftovers past half a tile keep the whole 64x64 tiling
    assert m.limb_plan(300, 120, 14)[1] == [(0, 0, 300, 120, 64, 64)]
    # a strip on one side only
    assert m.limb_plan(520, 256, 14)[1] == [(0, 0, 512, 256, 64, 64), (512, 0, 8, 256, 32, 128)]
    assert m.limb_plan(256, 1041, 15)[1] == [(0, 0, 256, 1024, 64, 64), (0, 1024, 256, 17, 128, 32)]
    # under 64 rows or columns there is no interior: the product runs whole
    assert m.limb_plan(20, 500, 14)[1][0][:4] == (0, 0, 20, 500)


def test_strips_follow_the_edge_at_32():
    # with strips: a 64x64 interior over the 64-aligned part, strips at most
    # 32 deep along the edges that leave at most half a 64-wide tile, and
    # fewer issued outputs than the 64x64 tiling of the whole product
    for (M, N) in shapes():
        cls, regs, _ = m.limb_plan(M, N, 14)
        if len(regs) == 1:
            continue
        rm, rn = M % 64, N % 64
        m64 = M - rm if 0 < rm <= 32 else M
        n64 = N - rn if 0 < rn <= 32 else N
        assert cls == 0 and regs[0] == (0, 0, m64, n64, 64, 64), (M, N, regs)
        for (r0, c0, rows, cols, bm, bn) in regs[1:]:
            assert (r0 == m64 and rows == M - m64 <= 32) or (c0 == n64 and cols == N - n64 <= 32), (M, N, regs)
        issued = sum(cdiv(r, bm) * bm * cdiv(c, bn) * bn for (_, _, r, c, bm, bn) in regs)
        assert issued < cdiv(M, 64) * 64 * cdiv(N, 64) * 64, (M, N, regs)


def test_plan_errors():
    for bad in [(0, 5, 5), (5, 0, 5), (-1, 5, 5)]:
        with pytest.raises(m.MPCError) as e:
            m.limb_plan(*bad)
        assert "mpc_limb_plan" in str(e.value)
    for variant in (-1, 16):
        with pytest.raises(m.MPCError):
            m.limb_plan(64, 64, variant)
