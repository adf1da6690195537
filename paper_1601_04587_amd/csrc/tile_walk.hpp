// Tile walks of the stencil's sub-banded and quadrant tile orders (host code,
// no HIP types, so that it also builds with a plain C++ compiler).
//
// A box of even-odd sites is stored as 64-site tiles, lexicographic with x3
// fastest and t slowest; tps tiles make one time slice and tpp tiles one
// (x2, x3) plane.  Workgroup b of a launch runs on XCD b % nxcd, and XCD x
// works through walk[xoff[x] .. xoff[x+1]).  XCD x owns a region of the
// (x1, tile-of-plane) cross-section over all slices: with nrg = 1 the x1 range
// [x L1 / nxcd, (x+1) L1 / nxcd) and every tile of its planes; with nrg > 1
// the x1 block x % (nxcd / nrg) (of L1 / (nxcd / nrg) rows) and the block
// x / (nxcd / nrg) of the tiles of each plane (tpp / nrg tiles).  The region
// is cut into nsub sub-bands (along the tiles of a plane, or along x1 with
// split_x1), each walked slice by slice (t outermost, then x1, then the tiles
// of the plane); with tblock > 1 the slices go in blocks of tblock, the slices
// of a block innermost.  A box whose planes are not a whole number of tiles,
// with fewer than nxcd x1 rows, or (nrg > 1) that does not split into the
// regions and sub-bands gets the banded walk instead: XCD x owns tiles
// [x S / nxcd, (x+1) S / nxcd) of every slice of S tiles (S = tps, or the whole
// box when a slice is not a whole number of tiles).
#pragma once

#include <algorithm>
#include <vector>

namespace ddml {

// L: box extents (t, x1, x2, x3); returns false unless the walk is a
// permutation of the ntiles tiles (xoff has nxcd + 1 entries).
inline bool tile_walk(const int L[4], int ntiles, int tps, int tile, int nxcd, int nrg, int nsub, bool split_x1,
                      int tblock, std::vector<int>& walk, int* xoff) {
  walk.clear();
  const int nt = ntiles;
  const long plane = (long)L[2] * L[3] / 2;
  const int nrx = nxcd / nrg;   // regions along x1
  const int tpp = plane % tile == 0 ? (int)(plane / tile) : 0;
  const bool fits = tps > 0 && tpp > 0 && L[1] >= nxcd &&
                    (nrg == 1 || (nxcd % nrg == 0 && L[1] % nrx == 0 && tpp % nrg == 0 && (L[1] / nrx) % nsub == 0));
  if (fits) {
    const int nslice = nt / tps;
    for (int x = 0; x < nxcd; ++x) {
      xoff[x] = (int)walk.size();
      const int ax = x % nrx, ag = x / nrx;
      const int a = nrg == 1 ? x * L[1] / nxcd : ax * (L[1] / nrx);
      const int b = nrg == 1 ? (x + 1) * L[1] / nxcd : (ax + 1) * (L[1] / nrx);
      const int g0 = ag * (tpp / nrg), g1 = (ag + 1) * (tpp / nrg);
      for (int sb = 0; sb < nsub; ++sb) {
        const int xlo = split_x1 ? a + sb * (b - a) / nsub : a, xhi = split_x1 ? a + (sb + 1) * (b - a) / nsub : b;
        const int glo = split_x1 ? g0 : g0 + sb * (g1 - g0) / nsub;
        const int ghi = split_x1 ? g1 : g0 + (sb + 1) * (g1 - g0) / nsub;
        for (int t0 = 0; t0 < nslice; t0 += tblock)
          for (int x1 = xlo; x1 < xhi; ++x1)
            for (int gg = glo; gg < ghi; ++gg)
              for (int t = t0; t < std::min(t0 + tblock, nslice); ++t) walk.push_back(t * tps + x1 * tpp + gg);
      }
    }
  } else {
    const int S = tps > 0 ? tps : nt;
    for (int x = 0; x < nxcd; ++x) {
      xoff[x] = (int)walk.size();
      const int lo = (int)((long)x * S / nxcd), bs = (int)((long)(x + 1) * S / nxcd) - lo;
      for (int v = 0; v < bs * (nt / S); ++v) walk.push_back((v / bs) * S + lo + v % bs);
    }
  }
  xoff[nxcd] = (int)walk.size();
  std::vector<char> seen(nt, 0);
  if ((int)walk.size() != nt) return false;
  for (int t : walk) {
    if (t < 0 || t >= nt || seen[t]) return false;
    seen[t] = 1;
  }
  return true;
}

}  // namespace ddml
