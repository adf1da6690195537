"""Host logic: the tile walks of the stencil's sub-banded and quadrant orders
(csrc/tile_walk.hpp), compiled with the host C++ compiler and checked on the
box shapes the library meets: every walk is a permutation of the tiles with
each XCD's share contiguous in xoff; on boxes that split, each XCD stays in
its region and walks its slices in the stated blocks; boxes that do not split
get the banded walk; and the quadrant regions of order 5 border on fewer
tiles of other XCDs than the x1 ranges of orders 2-4 (the reason for order 5).
"""
import os
import shutil
import subprocess

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HDR = os.path.join(ROOT, "paper_1601_04587_amd", "csrc")
NX, TILE = 8, 64

HARNESS = r"""
#include <cstdio>
#include <cstdlib>
#include "tile_walk.hpp"
int main(int argc, char** argv) {
  int L[4];
  for (int k = 0; k < 4; ++k) L[k] = atoi(argv[1 + k]);
  const int nrg = atoi(argv[5]), nsub = atoi(argv[6]), split = atoi(argv[7]), tblock = atoi(argv[8]);
  const long vh = (long)L[0] * L[1] * L[2] * L[3] / 2, v3h = (long)L[1] * L[2] * L[3] / 2;
  const int ntiles = (int)((vh + 63) / 64), tps = v3h % 64 == 0 ? (int)(v3h / 64) : 0;
  std::vector<int> walk;
  int xoff[9];
  const bool ok = ddml::tile_walk(L, ntiles, tps, 64, 8, nrg, nsub, split != 0, tblock, walk, xoff);
  printf("%d %d %d\n", ok ? 1 : 0, ntiles, tps);
  for (int x = 0; x <= 8; ++x) printf("%d ", xoff[x]);
  printf("\n");
  for (int t : walk) printf("%d ", t);
  printf("\n");
  return 0;
}
"""

# (nrg, nsub, split along x1, slices per block) of tile orders 2..5
ORDERS = {2: (1, 2, 0, 1), 3: (1, 4, 0, 1), 4: (1, 4, 0, 4), 5: (4, 4, 1, 4)}


@pytest.fixture(scope="module")
def walker(tmp_path_factory):
    cxx = shutil.which("g++") or shutil.which("c++")
    if cxx is None:
        pytest.skip("no host C++ compiler")
    d = tmp_path_factory.mktemp("walk")
    src = d / "walk.cpp"
    src.write_text(HARNESS)
    exe = d / "walk"
    subprocess.run([cxx, "-std=c++17", "-O1", "-I", HDR, str(src), "-o", str(exe)], check=True)

    def run(L, order):
        nrg, nsub, split, tb = ORDERS[order]
        out = subprocess.run([str(exe)] + [str(v) for v in L] + [str(nrg), str(nsub), str(split), str(tb)],
                             capture_output=True, text=True, check=True).stdout.split("\n")
        ok, ntiles, tps = map(int, out[0].split())
        xoff = np.array(out[1].split(), dtype=int)
        walk = np.array(out[2].split(), dtype=int)
        return bool(ok), ntiles, tps, xoff, walk
    return run


def _splits(L, order):
    """Whether the box gets the order's own walk (not the banded fallback)."""
    nrg, nsub, split, _ = ORDERS[order]
    plane = L[2] * L[3] // 2
    tps = (L[1] * plane) // TILE if (L[1] * plane) % TILE == 0 else 0
    tpp = plane // TILE if plane % TILE == 0 else 0
    if not (tps > 0 and tpp > 0 and L[1] >= NX):
        return False
    nrx = NX // nrg
    return nrg == 1 or (L[1] % nrx == 0 and tpp % nrg == 0 and (L[1] // nrx) % nsub == 0)


BOXES = [(16, 32, 32, 32), (4, 32, 32, 32), (8, 32, 32, 32), (40, 32, 32, 32), (16, 24, 24, 24),
         (4, 8, 16, 32), (8, 8, 16, 32), (16, 16, 16, 16), (6, 16, 16, 16), (6, 6, 6, 6), (16, 8, 8, 8),
         (4, 12, 16, 32)]


@pytest.mark.parametrize("order", [2, 3, 4, 5])
@pytest.mark.parametrize("L", BOXES)
def test_walk_is_a_permutation_with_contiguous_shares(walker, L, order):
    ok, ntiles, tps, xoff, walk = walker(L, order)
    assert ok
    assert len(walk) == ntiles and np.array_equal(np.sort(walk), np.arange(ntiles))
    assert xoff[0] == 0 and xoff[-1] == ntiles and np.all(np.diff(xoff) >= 0)


@pytest.mark.parametrize("order", [2, 3, 4, 5])
@pytest.mark.parametrize("L", [b for b in BOXES])
def test_regions_blocks_and_fallback(walker, L, order):
    ok, ntiles, tps, xoff, walk = walker(L, order)
    nrg, nsub, split, tb = ORDERS[order]
    if not _splits(L, order):
        # banded: XCD x owns tiles [x S / 8, (x+1) S / 8) of every slice of S tiles
        S = tps if tps > 0 else ntiles
        for x in range(NX):
            lo, hi = x * S // NX, (x + 1) * S // NX
            part = walk[xoff[x]:xoff[x + 1]]
            assert np.all((part % S >= lo) & (part % S < hi))
            assert len(part) == (hi - lo) * (ntiles // S)
        return
    tpp = L[2] * L[3] // 2 // TILE
    nrx = NX // nrg
    nslice = ntiles // tps
    shares = np.diff(xoff)
    assert shares.max() - shares.min() <= nslice * tpp   # at most one x1 row of difference
    for x in range(NX):
        part = walk[xoff[x]:xoff[x + 1]]
        t, rem = part // tps, part % tps
        x1, g = rem // tpp, rem % tpp
        if nrg == 1:
            a, b, g0, g1 = x * L[1] // NX, (x + 1) * L[1] // NX, 0, tpp
        else:
            ax, ag = x % nrx, x // nrx
            a, b = ax * (L[1] // nrx), (ax + 1) * (L[1] // nrx)
            g0, g1 = ag * (tpp // nrg), (ag + 1) * (tpp // nrg)
        assert np.all((x1 >= a) & (x1 < b) & (g >= g0) & (g < g1)), (L, order, x)
        # every tile of the region, each slice of a block innermost
        assert len(part) == (b - a) * (g1 - g0) * nslice
        # the sub-bands: the walk visits each sub-band's tiles in one stretch
        sub = ((x1 - a) * nsub // (b - a)) if split else ((g - g0) * nsub // (g1 - g0))
        assert np.all(np.diff(sub) >= 0)
        # inside a sub-band the blocks of tb slices come in order, and inside a
        # block each tile's slices are consecutive in the walk
        blk = t // tb
        for sb in np.unique(sub):
            assert np.all(np.diff(blk[sub == sb]) >= 0)
        for k in range(1, len(part)):
            if x1[k] == x1[k - 1] and g[k] == g[k - 1] and blk[k] == blk[k - 1]:
                assert t[k] == t[k - 1] + 1
            elif tb > 1 and t[k] % tb != 0 and t[k] != nslice:
                raise AssertionError("a block of slices is interrupted")


def test_quadrant_regions_have_fewer_border_tiles():
    """Per slice of a 32^3 box, the tiles of other XCDs that a region's hops
    reach (whole tiles across its x1 faces, one row of 16 of the 64 sites of
    a tile across its faces in the tile index of a plane): 2 x 8 = 16 tile
    equivalents for an x1 range of 4 rows (orders 2-4), 2 x 2 + 2 x 16 / 4 = 12
    for a quadrant of 16 rows x 2 tiles (order 5)."""
    L1, tpp = 32, 8

    def border(rows, tiles):
        x1_faces = 2 * tiles if rows < L1 else 0
        plane_faces = 2 * rows * 0.25 if tiles < tpp else 0
        return x1_faces + plane_faces
    assert border(L1 // NX, tpp) == 16
    assert border(L1 // 2, tpp // 4) == 12
    assert border(L1 // 2, tpp // 4) < border(L1 // NX, tpp)
