// tilewalk.h -- assignment of tiles to the workgroups of a launch.
//
// The tile kernels (statistics, key generation, histograms, scatter, tile
// scan) walk the call's (trace, tile) queue.  A launch has G workgroups, G a
// multiple of 8; G may equal the tile count (one tile each) or be a
// persistent grid of a few workgroups per CU that loops over many tiles.
//
// MI355X dispatches the workgroups of a grid round-robin over its eight
// XCDs, so workgroup w runs on XCD w mod 8, and each XCD has its own L2.
// The walk gives every XCD one contiguous eighth of the queue, which its
// G / 8 workgroups visit with stride G / 8: tiles that run at the same time
// on one XCD are neighbours, so the cache lines that neighbouring tiles
// share (the ends of a digit run in the scatter, the edge keys the scan
// reads) meet in one L2.
//
// Functions are usable from host and device code.
#pragma once
#include <stdint.h>

#include "keys.h"

namespace sc {

constexpr uint32_t N_XCD = 8;

struct TileWalk {
  uint32_t first;  // first tile of the workgroup
  uint32_t end;    // one past the last tile of its XCD's range
  uint32_t step;   // workgroups per XCD
};

// Walk of workgroup `wg` in a grid of `grid` workgroups (a multiple of 8)
// over `n` tiles: tiles first, first + step, ... below end.
SC_HD TileWalk tile_walk(uint32_t n, uint32_t grid, uint32_t wg) {
  const uint32_t step = grid / N_XCD, xcd = wg % N_XCD, k = wg / N_XCD;
  const uint32_t chunk = (n + N_XCD - 1) / N_XCD;
  const uint64_t lo = (uint64_t)xcd * chunk;
  const uint32_t end = (uint32_t)(lo + chunk < n ? lo + chunk : n);
  TileWalk w;
  w.first = (uint32_t)(lo + k < end ? lo + k : end);
  w.end = end;
  w.step = step ? step : 1;
  return w;
}

// Grid of a tile kernel: `per_cu` workgroups per CU over `n_cu` CUs (0: one
// workgroup per tile), never more than the tiles, rounded up to a multiple
// of 8.
SC_HD uint32_t tile_grid(uint32_t n, uint32_t per_cu, uint32_t n_cu) {
  uint64_t g = n;
  if (per_cu) {
    const uint64_t cap = (uint64_t)per_cu * n_cu;
    if (cap < g) g = cap;
  }
  g = (g + N_XCD - 1) / N_XCD * N_XCD;
  return (uint32_t)(g ? g : N_XCD);
}

}  // namespace sc
