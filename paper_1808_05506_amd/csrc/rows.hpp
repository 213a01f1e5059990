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
// sites (more where fewer than 128 threads would result) and at most 256
// threads (R N_v), evenly (24 -> 12 + 12 rather than 16 + 8), but keep at least
// 128 threads per workgroup where the row and the 256-thread limit allow.
inline int row_sites_default(int nx, int nv) {
  const int want = (128 + nv - 1) / nv, lim = 256 / nv;
  const int cap = want > 16 ? (want < lim ? want : lim) : (16 < lim ? 16 : lim);
  const int k = (nx + cap - 1) / cap;
  int r = (nx + k - 1) / k;
  const int rmin = want < cap ? want : cap;
  if (r < rmin) r = nx < rmin ? nx : rmin;
  return r;
}

// Traversal of the t-marching kernels: a workgroup owns the x-row chunk at
// (y, z) for T consecutive t and steps through them.
struct MarchTraversal {
  uint32_t sb, chunks, rows;  // sites per chunk, chunks per x-row, chunks per t-plane
  uint32_t T;                 // t steps per workgroup
  FastDiv d_chunks, d_ny, d_rows;
};

inline MarchTraversal make_march_traversal(const Geom& g, uint32_t sb, uint32_t T) {
  MarchTraversal m;
  m.sb = sb;
  m.chunks = (uint32_t(g.n[0]) + sb - 1) / sb;
  m.rows = m.chunks * uint32_t(g.n[1]) * uint32_t(g.n[2]);
  if (T < 1) T = 1;
  if (T > uint32_t(g.n[3])) T = uint32_t(g.n[3]);
  m.T = T;
  m.d_chunks = FastDiv::make(m.chunks);
  m.d_ny = FastDiv::make(uint32_t(g.n[1]));
  m.d_rows = FastDiv::make(m.rows);
  return m;
}

// Chunk `id` = (z Ny + y) chunks + chunk of t-plane t.
DSL_HD RowChunk march_chunk(const Geom& g, const MarchTraversal& m, uint32_t id, int t) {
  const uint32_t yz = m.d_chunks.div(id);
  const uint32_t chunk = id - yz * m.chunks;
  const uint32_t z = m.d_ny.div(yz);
  const uint32_t y = yz - z * uint32_t(g.n[1]);
  RowChunk c;
  c.x0 = int(chunk * m.sb);
  c.n = g.n[0] - c.x0 < int(m.sb) ? g.n[0] - c.x0 : int(m.sb);
  c.y = int(y);
  c.z = int(z);
  c.t = t;
  c.row_base = uint32_t(g.stride[1] * c.y + g.stride[2] * c.z + g.stride[3] * t);
  return c;
}

DSL_HD int wrap_x(const Geom& g, int x) { return x < 0 ? x + g.n[0] : (x >= g.n[0] ? x - g.n[0] : x); }

// LDS stride of one site in the row buffer, in storage words.  For a fixed
// spin-colour component the lanes of one site read a window of N_v words;
// consecutive sites are placed so that their windows fall on consecutive LDS
// banks (stride = window mod 64 dwords), which makes the per-component reads
// of a wave conflict-free.  The unpadded stride (12 N_v words) is a multiple
// of 64 dwords for FP32 N_v = 12 and would put every site on the same banks.
// Padding is skipped when it would cost more than a quarter of the row.
template <int NV, class S>
struct SiteStride {
  static constexpr int WB = int(sizeof(typename S::word));
  static constexpr int SWD = 12 * NV * WB / 4;                // dwords per site, unpadded
  static constexpr int WIN = NV * WB / 4;                     // dwords per component window
  static constexpr int PAD = (((WIN - SWD) % 64) + 64) % 64;
  static constexpr int DW = (PAD <= SWD / 4 && (PAD * 4) % 16 == 0) ? SWD + PAD : SWD;
  static constexpr int WORDS = DW * 4 / WB;                   // site stride in storage words
  static constexpr int PIECES = DW * 4 / 16;                  // site stride in 16-byte pieces
};

// Empty register constraint on an accumulator: keeps a hop's arithmetic
// before the next barrier.  Without it the scheduler may sink all hops of a
// workgroup to its end, keeping every staged operand live in registers.
template <class T>
__device__ __forceinline__ void hold(cpx<T>& z) {
  asm volatile("" : "+v"(z.r), "+v"(z.i));
}

// ---------------------------------------------------------------- staging of
// fields with COMPS components per site (12 for Wilson spinors, 3 for
// staggered ones), N_v right-hand sides fastest.


// 16-, 8- or 4-byte pieces, the largest that divides a lane's share of a site
// (COMPS storage words: the lanes of a site are its N_v right-hand sides).
template <int BYTES> struct PieceT;
template <> struct PieceT<16> { typedef u32x4 type; };
template <> struct PieceT<8> { typedef u32x2 type; };
template <> struct PieceT<4> { typedef unsigned int type; };

template <int COMPS, int NV, class S>
struct Stage {
  static constexpr int WB = int(sizeof(typename S::word));
  static constexpr int LANE_BYTES = COMPS * WB;  // one lane's share of a site
  static constexpr int PB = LANE_BYTES % 16 == 0 ? 16 : (LANE_BYTES % 8 == 0 ? 8 : 4);
  typedef typename PieceT<PB>::type P;
  static constexpr int CH = LANE_BYTES / PB;     // pieces per lane per site
  static constexpr int SW = COMPS * NV;          // words per site
  static constexpr int SWD = SW * WB / 4;        // dwords per site
  static constexpr int WIN = NV * WB / 4;        // dwords of one component window
  static constexpr int PAD = (((WIN - SWD) % 64) + 64) % 64;
  static constexpr int DW = (PAD <= SWD / 4 && (PAD * 4) % PB == 0) ? SWD + PAD : SWD;
  static constexpr int SSW = DW * 4 / WB;        // padded LDS site stride in words
  static constexpr int SSP = DW * 4 / PB;        // ... in pieces
};

// lane (x, v) moves pieces j * N_v + v of site x of a run starting at `base`
// (clamped to the last live site); `halo` adds one piece of site `hs` into
// slot CH for the lanes tid < pieces-per-site.
template <int COMPS, int NV, class S, bool HALO>
__device__ __forceinline__ void stage_issue(const typename S::word* __restrict__ f, uint32_t base, int n, uint32_t hs,
                                            int xl, int v, int tid,
                                            typename Stage<COMPS, NV, S>::P (&r)[Stage<COMPS, NV, S>::CH + 1]) {
  typedef Stage<COMPS, NV, S> St;
  typedef typename St::P P;
  const int xc = xl < n ? xl : n - 1;
  const P* src = reinterpret_cast<const P*>(f + size_t(base + xc) * St::SW);
#pragma unroll
  for (int j = 0; j < St::CH; ++j) r[j] = src[j * NV + v];
  if (HALO) {
    constexpr int SP = St::CH * NV;
    const int h = tid < SP ? tid : SP - 1;
    r[St::CH] = reinterpret_cast<const P*>(f + size_t(hs) * St::SW)[h];
  }
}

template <int COMPS, int NV, class S, bool HALO>
__device__ __forceinline__ void stage_commit(const typename Stage<COMPS, NV, S>::P (&r)[Stage<COMPS, NV, S>::CH + 1],
                                             typename S::word* buf, int n, int xl, int v, int tid) {
  typedef Stage<COMPS, NV, S> St;
  typedef typename St::P P;
  const int xc = xl < n ? xl : n - 1;
  P* dst = reinterpret_cast<P*>(buf) + xc * St::SSP;
#pragma unroll
  for (int j = 0; j < St::CH; ++j) dst[j * NV + v] = r[j];
  if (HALO) {
    constexpr int SP = St::CH * NV;
    const int h = tid < SP ? tid : SP - 1;
    (reinterpret_cast<P*>(buf) + n * St::SSP)[h] = r[St::CH];
  }
}

template <int COMPS, int NV, class S, class T>
__device__ __forceinline__ void lds_column(const typename S::word* site, int v, cpx<T> (&p)[COMPS]) {
#pragma unroll
  for (int c = 0; c < COMPS; ++c) p[c] = S::template load<T>(site + c * NV + v);
}


// Copy `pieces` 16-byte pieces (both pointers 16-byte aligned) with the
// workgroup's threads; consecutive threads move consecutive pieces and each
// thread moves at most K.  Loads and stores are both unconditional: indices
// past the end are clamped to the last piece, so a surplus lane rewrites that
// piece with the value it already holds.  Predicated loads would be sunk by
// the compiler into their store's branch and waited for one at a time.
template <int K>
__device__ __forceinline__ void copy_pieces(void* __restrict__ dst, const void* __restrict__ src, int pieces,
                                            int tid, int nth) {
  const u32x4* s = static_cast<const u32x4*>(src);
  u32x4* d = static_cast<u32x4*>(dst);
  u32x4 r[K];
#pragma unroll
  for (int j = 0; j < K; ++j) {
    const int i = tid + j * nth;
    r[j] = s[i < pieces ? i : pieces - 1];
  }
#pragma unroll
  for (int j = 0; j < K; ++j) {
    const int i = tid + j * nth;
    d[i < pieces ? i : pieces - 1] = r[j];
  }
}

// ---------------------------------------------------------------- output epilogues
// Fused forms of a D_W application for the inner CG on D^dag D (the solver):
//   EPI_STORE  out = result
//   EPI_NORM   out = result, and per column v the sum of |out|^2 over the
//              workgroup's sites (of the stored, rounded values) goes to
//              partial[workgroup][v]
//   EPI_AXPY   out holds the residual r and is updated in place,
//              r -= alpha[v] result (result as stored, i.e. rounded to the
//              storage format first), and the sums of |r|^2 of the stored r
//              go to partial[workgroup][v]
// A lane's 16-byte output pieces always cover the same VW columns, so it keeps
// VW FP32 sums over its few sites and steps in a fixed order (registers are
// what bounds these kernels' occupancy); the workgroup adds them in FP64 in a
// fixed tree at the end.  The kernel reads the stencil input only, so
// r can be updated in place; the partials are summed over workgroups in a
// fixed order by the caller (bitwise reproducible).
// (EPI_* and EpiArgs are in dslash_common.hpp.)

template <class S>
struct EpiLane {
  using W = typename S::word;
  static constexpr int VW = 16 / int(sizeof(W));  // columns per 16-byte piece
  const double* alpha;                            // EPI_AXPY coefficients, read where used
  int col0;                                       // first of the lane's VW columns
  float sum[VW];                                  // the lane's |out|^2 sums, one per column

  template <int NV>
  __device__ __forceinline__ void init(const EpiArgs& e, int v, bool axpy) {
    static_assert(NV % VW == 0, "a piece holds whole columns");
    alpha = axpy ? e.alpha : nullptr;
    col0 = (v * VW) % NV;
#pragma unroll
    for (int k = 0; k < VW; ++k) sum[k] = 0.f;
  }
};

// The VW storage words of a 16-byte piece and back, element by element (a bit
// cast of a vector element is miscompiled by this compiler).
template <class S>
__device__ __forceinline__ void piece_unpack(u32x4 z, typename S::word (&w)[EpiLane<S>::VW]) {
  using W = typename S::word;
  constexpr int VW = EpiLane<S>::VW;
#pragma unroll
  for (int k = 0; k < VW; ++k) {
    if constexpr (VW == 1) {
      w[k] = __builtin_bit_cast(W, z);
    } else if constexpr (VW == 2) {
      w[k] = __builtin_bit_cast(W, u32x2{z[2 * k], z[2 * k + 1]});
    } else {
      static_assert(__is_same(W, uint32_t), "4-byte storage words are uint32_t");
      w[k] = z[k];
    }
  }
}

template <class S>
__device__ __forceinline__ u32x4 piece_pack(const typename S::word (&w)[EpiLane<S>::VW]) {
  constexpr int VW = EpiLane<S>::VW;
  u32x4 z;
#pragma unroll
  for (int k = 0; k < VW; ++k) {
    if constexpr (VW == 1) {
      z = __builtin_bit_cast(u32x4, w[k]);
    } else if constexpr (VW == 2) {
      const u32x2 a = __builtin_bit_cast(u32x2, w[k]);
      z[2 * k] = a[0];
      z[2 * k + 1] = a[1];
    } else {
      z[k] = w[k];
    }
  }
  return z;
}

// Copy-out of one site's CH pieces (lane v takes pieces j NV + v) from LDS to
// global memory with the epilogue EPI; `live` is false for lanes past a
// partial chunk's end, which then store and count nothing.
template <int EPI, int NV, class S, int CH>
__device__ __forceinline__ void epi_copy_out(const u32x4* src, u32x4* dst, int v, bool live, EpiLane<S>& e) {
  using W = typename S::word;
  constexpr int VW = EpiLane<S>::VW;
  u32x4 z[CH];
#pragma unroll
  for (int j = 0; j < CH; ++j) z[j] = src[j * NV + v];
  if constexpr (EPI == EPI_AXPY) {
    float al[VW];
#pragma unroll
    for (int k = 0; k < VW; ++k) al[k] = float(e.alpha[e.col0 + k]);
#pragma unroll
    for (int j = 0; j < CH; ++j) {
      W ws[VW], wr[VW];
      piece_unpack<S>(z[j], ws);
      piece_unpack<S>(live ? dst[j * NV + v] : u32x4{0u, 0u, 0u, 0u}, wr);
#pragma unroll
      for (int k = 0; k < VW; ++k)
        S::template store<float>(&wr[k], rmadd(S::template load<float>(&wr[k]), -al[k],
                                               S::template load<float>(&ws[k])));
      z[j] = piece_pack<S>(wr);
    }
  }
  if constexpr (EPI == EPI_STORE) {
    // lanes past a partial chunk's end repeat the last site: same data, same place
#pragma unroll
    for (int j = 0; j < CH; ++j) __builtin_nontemporal_store(z[j], &dst[j * NV + v]);
  } else if (live) {
#pragma unroll
    for (int j = 0; j < CH; ++j) __builtin_nontemporal_store(z[j], &dst[j * NV + v]);
#pragma unroll
    for (int j = 0; j < CH; ++j) {
      W w[VW];
      piece_unpack<S>(z[j], w);
#pragma unroll
      for (int k = 0; k < VW; ++k) {
        const cpx<float> q = S::template load<float>(&w[k]);
        e.sum[k] = fmaf(q.r, q.r, fmaf(q.i, q.i, e.sum[k]));
      }
    }
  }
}

// The workgroup's per-column sums into partial[blockIdx.x][0 .. NV): the
// lanes' sums go to LDS as [VW][R][NV] (lds: at least VW R NV doubles, free
// apart from a barrier), are added over the R sites in a fixed tree, and
// thread v < NV adds the lanes v' < NV whose pieces hold column v.
template <int EPI, int NV, class S>
__device__ __forceinline__ void epi_finish(const EpiArgs& ea, const EpiLane<S>& e, double* lds, int xl, int v,
                                           int R) {
  if constexpr (EPI != EPI_STORE) {
    constexpr int VW = EpiLane<S>::VW;
    __syncthreads();
#pragma unroll
    for (int k = 0; k < VW; ++k) lds[(k * R + xl) * NV + v] = double(e.sum[k]);
    __syncthreads();
    for (int w = 1; w < R; w <<= 1) {
      if ((xl & (2 * w - 1)) == 0 && xl + w < R) {
#pragma unroll
        for (int k = 0; k < VW; ++k) lds[(k * R + xl) * NV + v] += lds[(k * R + xl + w) * NV + v];
      }
      __syncthreads();
    }
    const int tid = xl * NV + v;
    if (tid < NV) {
      double s = 0.0;
      for (int lv = 0; lv < NV; ++lv) {
#pragma unroll
        for (int k = 0; k < VW; ++k)
          if ((lv * VW + k) % NV == tid) s += lds[k * R * NV + lv];
      }
      ea.partial[size_t(blockIdx.x) * NV + tid] = s;
    }
  }
}

}  // namespace dsl
