"""Host checks of the LDS tile layout of the 8-wave float64 passes at block width 128
(k_grad_wide, k_dir_wide, k_gram_wide): the layout constants and the address map are read
from the kernel source, then checked on the CPU for what the kernels rely on:

* every (row, column) of a 64 x 128 tile has its own slot inside the tile's allocation, and
  16-byte pairs stay aligned and adjacent;
* the product's 16-byte reads (16 rows of one lane group), the Gram's 8-byte reads (4
  consecutive rows x 16 columns, a half-wave at a time) and the staging stores hit 64 distinct
  banks (4-byte banks, 64 of them);
* the lane-base-plus-constant forms the kernels use for those addresses equal the map.
"""
import os
import re

import pytest

SRC = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))),
                   "paper_2306_10379_amd", "csrc", "gsi_kernels.hip")


@pytest.fixture(scope="module")
def layout():
    text = open(SRC).read()
    consts = {k: int(re.search(rf"constexpr int {k} = ([^;]+);", text).group(1).split("*")[-1].strip())
              for k in ("WLD", "WPP")}
    assert re.search(r"constexpr int WGW = 2 \* WG;", text)
    # the map itself, as written in the source
    assert "return row * WLD + (col ^ (2 * ((row >> 1) & 7)));" in text
    wld = consts["WLD"]

    def at(row, col):
        return row * wld + (col ^ (2 * ((row >> 1) & 7)))
    return wld, consts["WPP"], at


def banks(elem, nbytes):
    return [((elem * 8) // 4 + k) % 64 for k in range(nbytes // 4)]


def test_map_is_a_bijection_inside_the_tile(layout):
    wld, wpp, at = layout
    assert wpp == 128 and wld >= wpp
    seen = set()
    for r in range(64):
        for c in range(wpp):
            a = at(r, c)
            assert r * wld <= a < r * wld + wpp
            seen.add(a)
        for c in range(0, wpp, 2):
            assert at(r, c) % 2 == 0 and at(r, c + 1) == at(r, c) + 1
    assert len(seen) == 64 * wpp


def test_reads_and_stores_are_free_of_bank_conflicts(layout):
    _, _, at = layout
    for j in range(16):  # product: lane group g, lanes c = 0..15 read rows 16 rg + c
        for g in range(4):
            for rg in range(4):
                b = sum((banks(at(16 * rg + c, 8 * j + 2 * g), 16) for c in range(16)), [])
                assert len(set(b)) == 64
    for rg in range(4):  # Gram: rows 16 rg + 4 r + g, columns 16 ib + c, g in {0, 1} / {2, 3}
        for r in range(4):
            for ib in range(8):
                for g0 in (0, 2):
                    b = sum((banks(at(16 * rg + 4 * r + g, 16 * ib + c), 8)
                             for g in (g0, g0 + 1) for c in range(16)), [])
                    assert len(set(b)) == 64
    for base in range(0, 4096, 16):  # staging: granule i of the tile -> row i / 64
        b = sum((banks(at(i >> 6, 2 * (i & 63)), 16) for i in range(base, base + 16)), [])
        assert len(set(b)) == 64


def test_lane_bases_with_constant_offsets(layout):
    wld, _, at = layout
    for tid in range(512):
        g, c = (tid & 63) >> 4, tid & 15
        la0, la1 = at(c, 2 * g), at(c, 8 + 2 * g)
        for rg in range(4):
            for j in range(16):
                assert at(16 * rg + c, 8 * j + 2 * g) == (la1 if j & 1 else la0) + 16 * rg * wld + 16 * (j >> 1)
        lb = [at(g + 4 * r, c) for r in range(4)]
        for rg in range(4):
            for r in range(4):
                for ib in range(8):
                    assert at(16 * rg + g + 4 * r, 16 * ib + c) == lb[r] + 16 * rg * wld + 16 * ib
        b0, b1 = at(tid >> 6, 2 * (tid & 63)), at((tid >> 6) + 8, 2 * (tid & 63))
        for m in range(8):
            i = tid + 512 * m
            assert at(i >> 6, 2 * (i & 63)) == (b1 if m & 1 else b0) + 16 * (m >> 1) * wld


def test_lds_budget(layout):
    wld, _, _ = layout
    tile = 64 * wld * 8
    assert 2 * tile + 16 * 64 * 8 + 8 * 3 * 8 <= 160 * 1024  # gradient pass: two tiles, row sums, red
    assert 2 * tile <= 160 * 1024  # direction and Gram passes


def test_direction_pass_shares_out_each_block_of_the_symmetric_gram_once():
    """k_dir_wide: wave w forms blocks (w + d mod 8, w) for d < 5 when w < 4, d < 4 otherwise,
    and mirrors the off-diagonal ones; every block of P^T P is then written exactly once."""
    text = open(SRC).read()
    assert "const int nd = w < 4 ? 5 : 4;" in text and "const int ib = (w + d) & 7;" in text
    written = {}
    for w in range(8):
        for d in range(5 if w < 4 else 4):
            ib = (w + d) & 7
            for blk in {(ib, w), (w, ib)}:
                written[blk] = written.get(blk, 0) + 1
    assert sorted(written) == [(i, j) for i in range(8) for j in range(8)]
    assert set(written.values()) == {1}
    assert sum(5 if w < 4 else 4 for w in range(8)) == 36  # the upper blocks, diagonal included
