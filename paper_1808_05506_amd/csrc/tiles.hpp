// Chunk order of the one-row kernels in tiles of by x bz (y, z) rows: the
// chunks of a tile's rows at one t, then at the next t, tile after tile.  The
// XCD mapping (xcd_block) gives each XCD a contiguous range of this order, so
// the neighbour rows a chunk stages (+-y, +-z, +-t) are mostly the own rows of
// chunks that run shortly before or after it on the same XCD and are still in
// its L2; the t-band order of RowTraversal reaches the z neighbours a whole
// band of planes later.  The grid is the same (chunks x Ny x Nz x Nt).
#pragma once

#include "rows.hpp"

namespace dsl {

struct ChunkTiles {
  uint32_t on, chunks, by, bz, tiles_y;
};

// The largest by x bz rows (by | Ny, bz | Nz) whose rows at one t take at
// most `budget` bytes (row_bytes each), the squarer of equal sizes and the
// larger by of equally square ones; by = bz = 0 when no row fits.
inline void pick_tile(const Geom& g, long row_bytes, long budget, int& by, int& bz) {
  const long max_rows = row_bytes > 0 ? budget / row_bytes : 0;
  by = bz = 0;
  for (int y = 1; y <= g.n[1]; ++y) {
    if (g.n[1] % y) continue;
    for (int z = 1; z <= g.n[2]; ++z) {
      if (g.n[2] % z || long(y) * z > max_rows) continue;
      const int a = y * z, b = by * bz, d = y > z ? y - z : z - y, e = by > bz ? by - bz : bz - by;
      if (a > b || (a == b && (d < e || (d == e && y > by)))) {
        by = y;
        bz = z;
      }
    }
  }
}

// by | Ny and bz | Nz, both > 0, else the tiles are off (t-band order).
inline ChunkTiles make_chunk_tiles(const Geom& g, int R, int by, int bz) {
  ChunkTiles o{};
  if (by > 0 && bz > 0 && g.n[1] % by == 0 && g.n[2] % bz == 0) {
    o.on = 1;
    o.chunks = uint32_t((g.n[0] + R - 1) / R);
    o.by = uint32_t(by);
    o.bz = uint32_t(bz);
    o.tiles_y = uint32_t(g.n[1] / by);
  }
  return o;
}

DSL_HD RowChunk tile_chunk(const Geom& g, const ChunkTiles& o, uint32_t sb, uint32_t L) {
  const uint32_t per_row = o.chunks * o.by;
  const uint32_t per_t = per_row * o.bz;
  const uint32_t per_tile = per_t * uint32_t(g.n[3]);
  const uint32_t tile = L / per_tile;
  uint32_t r = L - tile * per_tile;
  const uint32_t t = r / per_t;
  r -= t * per_t;
  const uint32_t zz = r / per_row;
  r -= zz * per_row;
  const uint32_t yy = r / o.chunks;
  const uint32_t chunk = r - yy * o.chunks;
  const uint32_t tz = tile / o.tiles_y, ty = tile - tz * o.tiles_y;
  RowChunk c;
  c.x0 = int(chunk * sb);
  c.n = g.n[0] - c.x0 < int(sb) ? g.n[0] - c.x0 : int(sb);
  c.y = int(ty * o.by + yy);
  c.z = int(tz * o.bz + zz);
  c.t = int(t);
  c.row_base = uint32_t(g.n[0]) * (uint32_t(c.y) + uint32_t(g.n[1]) * (uint32_t(c.z) + uint32_t(g.n[2]) * t));
  return c;
}

// The chunk of logical block L: tiled order when o.on, else the t-band order.
DSL_HD RowChunk order_chunk(const Geom& g, const RowTraversal& tr, const ChunkTiles& o, uint32_t L) {
  return o.on ? tile_chunk(g, o, tr.sb, L) : row_chunk(g, tr, L);
}

// Workgroup order in tiles of by x bz (y, z) rows, every t segment of a tile
// before the next tile.  With eight tiles each XCD takes one whole tile (the
// XCD mapping deals contiguous eighths of the order), and its workgroups walk
// the tile's rows segment by segment, so the +-y and +-z rows a workgroup
// stages were mostly just staged by its neighbours on the same XCD.  The D_S
// march on 32^4 (N_v = 12, FP32) in 8 x 16 tiles read 1.11 GB per launch
// instead of 1.55 GB, and ran 286.6 against 296.6 us (N_v = 4: 138.6 / 142.9,
// N_v = 8: 203.6 / 210.7, N_v = 24: 521.8 / 528.4, FP64 N_v = 12: 511.1 /
// 526.2 us).
struct MarchTiles {
  uint32_t on, chunks, by, bz, tiles_y, nseg;
};

// by | Ny and bz | Nz, both > 0, else the tiles are off (plane order).
inline MarchTiles make_march_tiles(const Geom& g, uint32_t chunks, uint32_t nseg, int by, int bz) {
  MarchTiles o{};
  if (by > 0 && bz > 0 && g.n[1] % by == 0 && g.n[2] % bz == 0) {
    o.on = 1;
    o.chunks = chunks;
    o.by = uint32_t(by);
    o.bz = uint32_t(bz);
    o.tiles_y = uint32_t(g.n[1] / by);
    o.nseg = nseg;
  }
  return o;
}

DSL_HD uint32_t march_tile_id(const Geom& g, const MarchTiles& o, uint32_t L, uint32_t& seg) {
  const uint32_t per_row = o.chunks * o.by, per_seg = per_row * o.bz, per_tile = per_seg * o.nseg;
  const uint32_t tile = L / per_tile;
  uint32_t r = L - tile * per_tile;
  seg = r / per_seg;
  r -= seg * per_seg;
  const uint32_t zz = r / per_row;
  r -= zz * per_row;
  const uint32_t yy = r / o.chunks, chunk = r - yy * o.chunks;
  const uint32_t tz = tile / o.tiles_y, ty = tile - tz * o.tiles_y;
  return ((tz * o.bz + zz) * uint32_t(g.n[1]) + ty * o.by + yy) * o.chunks + chunk;
}

// Segment and chunk id of logical block L: tiled order when o.on, else plane
// order (segment-major).
DSL_HD uint32_t march_order_id(const Geom& g, const MarchTraversal& m, const MarchTiles& o, uint32_t L,
                               uint32_t& seg) {
  if (o.on) return march_tile_id(g, o, L, seg);
  seg = m.d_rows.div(L);
  return L - seg * m.rows;
}

// Eight tiles, the squarest with by <= bz (8 x 16 on 32^4); by = bz = 0 when
// Ny x Nz has no such split.
inline void march_tile_default(const Geom& g, int& by, int& bz) {
  by = bz = 0;
  for (int y = 1; y <= g.n[1]; ++y) {
    if (g.n[1] % y) continue;
    for (int z = y; z <= g.n[2]; ++z) {
      if (g.n[2] % z || (g.n[1] / y) * (g.n[2] / z) != 8) continue;
      if (by == 0 || z - y < bz - by) {
        by = y;
        bz = z;
      }
    }
  }
}

}  // namespace dsl
