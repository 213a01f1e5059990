// Row-staged execution of the one-hop stencils (D_W, D_S).
//
// A workgroup owns one chunk of R consecutive sites of an x-row and all N_v
// right-hand sides (thread (x, v), v fastest).  Every input the chunk needs is
// a contiguous run of memory in the site-slowest layout: the chunk's own row
// (plus one halo site on each side for the x-hops), and for each of the six
// y/z/t hops the same x-range of the neighbour row.  These runs are copied into
// LDS with 16-byte loads in which consecutive lanes read consecutive bytes, so
// each wave instruction touches the fewest cache lines possible; the stencil
// arithmetic then reads its operands from LDS.  Without the staging every
// lane fetches its own 8-byte pieces of nine different sites through L1, which
// costs about three times as many L1 accesses per byte and is what limits a
// direct-load kernel on this GPU.  The results go back to HBM the same way:
// through LDS, then coalesced 16-byte stores.
#pragma once

#include "stencils.hpp"

namespace dsl {

// Geometry of one row chunk.
struct RowChunk {
  int x0, n;           // first x, number of live sites in the chunk (<= R)
  int y, z, t;         // uniform row coordinates
  uint32_t row_base;   // site index of (0, y, z, t)
};

DSL_HD RowChunk row_chunk(const Geom& g, const RowTraversal& tr, uint32_t L) {
  uint32_t s;
  bool live;
  SiteNbr nb = row_site(g, tr, L, 0, s, live);
  RowChunk c;
  c.x0 = nb.c[0];
  c.y = nb.c[1];
  c.z = nb.c[2];
  c.t = nb.c[3];
  c.n = g.n[0] - c.x0 < int(tr.sb) ? g.n[0] - c.x0 : int(tr.sb);
  c.row_base = s - uint32_t(c.x0);
  return c;
}

// Site index of (x, y, z, t) + d for a single-axis step d (mu, +-1), periodic.
DSL_HD uint32_t row_base_shift(const Geom& g, const RowChunk& c, int mu, int sgn) {
  int q[4] = {0, c.y, c.z, c.t};
  q[mu] += sgn;
  if (q[mu] < 0) q[mu] += g.n[mu];
  if (q[mu] >= g.n[mu]) q[mu] -= g.n[mu];
  return uint32_t(g.stride[1] * q[1] + g.stride[2] * q[2] + g.stride[3] * q[3]);
}

// Default chunk length: split an x-row into the fewest chunks of at most 16
// sites, evenly (24 -> 12 + 12 rather than 16 + 8), but keep at least 128
// threads per workgroup.
inline int row_sites_default(int nx, int nv) {
  const int k = (nx + 15) / 16;
  int r = (nx + k - 1) / k;
  const int rmin = (128 + nv - 1) / nv;
  if (r < rmin) r = nx < rmin ? nx : rmin;
  return r;
}

DSL_HD int wrap_x(const Geom& g, int x) { return x < 0 ? x + g.n[0] : (x >= g.n[0] ? x - g.n[0] : x); }

}  // namespace dsl
