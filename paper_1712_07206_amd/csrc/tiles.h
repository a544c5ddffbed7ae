// Tile numbering shared by the contraction kernels: which 128 x 128 super-tile of
// the upper triangle a workgroup takes, and how the numbers are dealt to XCDs.
#pragma once

#include <hip/hip_runtime.h>

namespace hsb {

constexpr int kXcds = 8;

// Start and length of XCD x's contiguous share of `num` items (dispatch is
// round-robin over the XCDs, so giving each a contiguous range keeps the tiles
// it runs at one time next to each other).
__device__ inline void xcd_range(int x, int num, int& start, int& len) {
  const int per = num / kXcds, rem = num % kXcds;
  start = x < rem ? x * (per + 1) : rem * (per + 1) + (x - rem) * per;
  len = per + (x < rem ? 1 : 0);
}

// s -> (bi, bj), bj >= bi, row-major over the upper triangle of an nb x nb grid.
__device__ inline void tri_decode(int s, int nb, int& bi, int& bj) {
  const double b = 2.0 * nb + 1.0;
  int i = (int)((b - sqrt(b * b - 8.0 * s)) * 0.5);
  if (i < 0) i = 0;
  if (i > nb - 1) i = nb - 1;
  auto start = [nb](int r) { return r * nb - r * (r - 1) / 2; };
  while (i > 0 && start(i) > s) --i;
  while (i + 1 < nb && start(i + 1) <= s) ++i;
  bi = i;
  bj = i + (s - start(i));
}

// Super-tile s -> (bi, sj) when the super-rows are taken in groups of gr: group by
// group, and inside a group super-column by super-column, the group's rows with
// bi <= sj.  Consecutive numbers then cover a compact gr-row patch, so the tiles an
// XCD runs at one time share row strips and column strips.
__device__ inline void grouped_decode(int s, int nb, int gr, int& bi, int& sj) {
  int g0 = 0;
  int rows = min(gr, nb);
  for (;;) {
    rows = min(gr, nb - g0);
    const int ncol = nb - g0;
    const int cnt = rows * (rows + 1) / 2 + (ncol - rows) * rows;
    if (s < cnt || g0 + rows >= nb) break;
    s -= cnt;
    g0 += rows;
  }
  int c = 0;
  for (;;) {
    const int k = min(rows, c + 1);
    if (s < k || g0 + c + 1 >= nb) break;
    s -= k;
    ++c;
  }
  sj = g0 + c;
  bi = g0 + s;
}

// Tile w -> (row0, col0) of a 128 x 64 tile: two per 128 x 128 super-tile.
// gr = 0: row-major over the upper triangle; gr > 0: grouped order.
__device__ inline void tile_origin(int w, int nbr, int gr, int& row0, int& col0) {
  int bi, sj;
  if (gr > 0) grouped_decode(w >> 1, nbr, gr, bi, sj);
  else tri_decode(w >> 1, nbr, bi, sj);
  row0 = bi * 128;
  col0 = sj * 128 + (w & 1) * 64;
}

}  // namespace hsb
