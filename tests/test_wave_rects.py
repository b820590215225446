"""The generated table of per-wave output-block rectangles of the tile kernels (host logic)."""
import importlib.util
import os
import re

import pytest

CSRC = os.path.join(os.path.dirname(os.path.abspath(__file__)), "..", "paper_1504_05046_amd", "csrc")


def _gen():
    spec = importlib.util.spec_from_file_location("gen_wave_rects", os.path.join(CSRC, "gen_wave_rects.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def _tables(text):
    """{(pa, pb, nw): {(a, b): [rect words]}} parsed from the device tables of the .inc file."""
    out = {}
    for m in re.finditer(r"kWaveRects_(\d+)x(\d+)_(\d+)\[\d+\] = \{\n(.*?)\n\};", text, re.S):
        pa, pb, nw = int(m.group(1)), int(m.group(2)), int(m.group(3))
        rows = {}
        for line in m.group(4).splitlines():
            words, ab = line.split("//")
            a, b = (int(v) for v in ab.split("x"))
            rows[(a, b)] = [int(v.strip().rstrip("u"), 16) for v in words.split(",") if v.strip()]
        out[(pa, pb, nw)] = rows
    return out


def test_generated_file_is_current():
    gen = _gen()
    with open(os.path.join(CSRC, "wave_rects.inc")) as f:
        assert f.read() == gen.generate()


def test_rectangles_tile_every_subtile():
    gen = _gen()
    text = open(os.path.join(CSRC, "wave_rects.inc")).read()
    tables = _tables(text)
    assert set(tables) == {(tm // 16, tn // 16, nw) for tm, tn, nw in gen.variants(os.path.join(CSRC, "types.hpp"))}
    for (pa, pb, nw), rows in tables.items():
        assert set(rows) == {(a, b) for a in range(1, pa + 1) for b in range(1, pb + 1)}
        host = re.search(rf"kWaveRectMax_{pa}x{pb}_{nw}\[\d+\] = \{{\n(.*?)\n\}};", text, re.S).group(1)
        host_max = [int(v) for v in host.replace("\n", " ").split(",") if v.strip()]
        for (a, b), words in rows.items():
            assert len(words) == nw
            cover = [[0] * b for _ in range(a)]
            areas = []
            for wd in words:
                r0, c0, na, nb = wd & 0xFF, (wd >> 8) & 0xFF, (wd >> 16) & 0xFF, wd >> 24
                if wd == 0:
                    continue
                assert na >= 1 and nb >= 1 and r0 + na <= a and c0 + nb <= b
                for x in range(r0, r0 + na):
                    for y in range(c0, c0 + nb):
                        cover[x][y] += 1
                areas.append(na * nb)
            assert all(c == 1 for row in cover for c in row), (pa, pb, nw, a, b)
            fair = -(-a * b // nw)  # dealing the blocks out one by one
            assert max(areas) == host_max[(a - 1) * pb + (b - 1)]
            if nw == 8:
                assert max(areas) == fair
            else:
                assert max(areas) <= fair + 1


def test_fewer_fragment_reads_than_round_robin():
    gen = _gen()
    for a in range(1, 9):
        for b in range(1, 9):
            rects = gen.partition(a, b, 8)
            reads = sum(na + nb for _, _, na, nb in rects)
            assert reads <= 2 * a * b
    # a full 128 x 128 sub-tile: eight 2 x 4 (or 4 x 2) rectangles, 6 reads per 8 MFMAs
    assert sorted((na, nb) for _, _, na, nb in gen.partition(8, 8, 8)) in ([(2, 4)] * 8, [(4, 2)] * 8)


@pytest.mark.parametrize("a,b,nw", [(5, 5, 4), (7, 7, 4)])
def test_no_rectangle_tiling_reaches_fair_share(a, b, nw):
    # the few shapes where the busiest wave owns one block more than ceil(ab / nw): brute force
    # over all tilings confirms that no tiling into nw rectangles does better
    fair = -(-a * b // nw)

    def fits(cells, k):
        if not cells:
            return True
        if k == 0:
            return False
        x, y = min(cells)
        for na in range(1, a - x + 1):
            for nb in range(1, b - y + 1):
                if na * nb > fair:
                    break
                rect = {(x + i, y + j) for i in range(na) for j in range(nb)}
                if rect <= cells and fits(cells - rect, k - 1):
                    return True
        return False

    assert not fits({(x, y) for x in range(a) for y in range(b)}, nw)
