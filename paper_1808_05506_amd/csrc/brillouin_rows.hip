// Row-staged D_B (Sec. 5; see rows.hpp for the row staging).  A workgroup
// owns an x-row chunk of R sites and all N_v right-hand sides (thread (x, v)).
// The 80 hops of the 3^4 stencil reach the 27 rows (y + dy, z + dz, t + dt),
// dy, dz, dt in {-1, 0, 1}; each such row is staged once, with the halo sites
// x0 - 1 and x0 + n, through one LDS buffer with coalesced 16-byte loads, and
// serves the hops d = (dx, dy, dz, dt), dx in {-1, 0, 1}.  With each row come
// the three link columns those hops need: W_d(x) at the chunk's own sites when
// d is one of the 40 stored directions, else W_{-d}(x + d) at the neighbour
// row's sites, applied as its adjoint.  Thread (x, v) accumulates
//   out(x) = (m0 + 15/8) psi(x) + sum_d (-lambda_k / 2 + rho_k d.gamma) W_d(x) psi(x + d)
// (rho_k -> -rho_k for the adjoint) in registers over the 27 rows and writes
// its output once, through LDS with coalesced 16-byte stores.
#include <stdlib.h>

#include "launch.hpp"
#include "rows.hpp"
#include "tiles.hpp"

namespace dsl {

namespace {

constexpr int kBriRows = 27;  // (dy, dz, dt) in {-1, 0, 1}^3, row 13 is the own row

DSL_HD void bri_row_offset(int r, int& dy, int& dz, int& dt) {
  dy = r % 3 - 1;
  dz = (r / 3) % 3 - 1;
  dt = r / 9 - 1;
}

DSL_HD uint32_t bri_row_base(const Geom& g, const RowChunk& c, int dy, int dz, int dt) {
  int y = c.y + dy, z = c.z + dz, t = c.t + dt;
  y = y < 0 ? y + g.n[1] : (y >= g.n[1] ? y - g.n[1] : y);
  z = z < 0 ? z + g.n[2] : (z >= g.n[2] ? z - g.n[2] : z);
  t = t < 0 ? t + g.n[3] : (t >= g.n[3] ? t - g.n[3] : t);
  return uint32_t(g.stride[1] * y + g.stride[2] * z + g.stride[3] * t);
}

// base-3 code n(d) = sum_mu (d_mu + 1) 3^mu; d is stored (in slot n - 41) iff n > 40
DSL_HD int bri_code(int dx, int dy, int dz, int dt) { return (dx + 1) + 3 * (dy + 1) + 9 * (dz + 1) + 27 * (dt + 1); }

template <int NV, class S>
struct BriStage {
  using W = typename S::word;
  static constexpr int SW = 12 * NV;                  // words per site
  static constexpr int SP = SW * int(sizeof(W)) / 16; // 16-byte pieces per site
  static constexpr int CH = SP / NV;                  // pieces per lane
  static constexpr int KW = (27 + NV - 1) / NV;       // link words per thread (27 n words per row)
  // halo pieces per thread (2 SP = 12 N_v of them over R N_v threads): one
  // for chunks of at least 12 sites, two for the chunks of 6 .. 11 sites
  // taken at N_v > 16 (the launcher checks R HK >= 12)
  static constexpr int HK = NV > 16 ? 2 : 1;
};

// A staged row in flight: the lane's pieces of its site, one piece of the halo
// sites, and its words of the row's three link columns.
template <int NV, class S>
struct BriRowRegs {
  u32x4 p[BriStage<NV, S>::CH];
  u32x4 halo[BriStage<NV, S>::HK];
  typename S::word w[BriStage<NV, S>::KW];
};

template <bool FLY, int NV, class S>
__device__ __forceinline__ void bri_issue(const Geom& g, const RowChunk& c, const typename S::word* __restrict__ Wl,
                                          const typename S::word* __restrict__ in, int r, int xm, int xp, int xl,
                                          int v, int tid, int nth, BriRowRegs<NV, S>& q) {
  using St = BriStage<NV, S>;
  int dy, dz, dt;
  bri_row_offset(r, dy, dz, dt);
  const uint32_t nb = bri_row_base(g, c, dy, dz, dt);
  const int xc = xl < c.n ? xl : c.n - 1;
  const u32x4* src = reinterpret_cast<const u32x4*>(in + size_t(nb + c.x0) * St::SW);
#pragma unroll
  for (int j = 0; j < St::CH; ++j) q.p[j] = src[xc * St::SP + j * NV + v];
#pragma unroll
  for (int k = 0; k < St::HK; ++k) {
    int h = tid + k * nth;
    h = h < 2 * St::SP ? h : 2 * St::SP - 1;
    const int hs = h < St::SP ? xm : xp;
    q.halo[k] = reinterpret_cast<const u32x4*>(in + size_t(nb + hs) * St::SW)[h < St::SP ? h : h - St::SP];
  }
  // link columns dx = -1, 0, 1: 9 words per site of the chunk (built from V
  // in LDS instead when FLY)
  if constexpr (FLY) return;
  const int nw = 27 * c.n;
#pragma unroll
  for (int k = 0; k < St::KW; ++k) {
    int w = tid + k * nth;
    w = w < nw ? w : nw - 1;
    const int col = w / (9 * c.n), rem = w - col * 9 * c.n;
    const int site = rem / 9, e = rem - site * 9;
    const int dx = col - 1;
    const int code = bri_code(dx, dy, dz, dt);
    size_t idx;
    if (code > 40) {
      idx = (size_t(c.row_base + c.x0 + site) * 40 + (code - 41)) * 9 + e;  // W_d(x), stored
    } else {
      // W_{-d}(x + d), slot n(-d) - 41 = 39 - n(d); for d = 0 any valid word (unused)
      const int slot = code == 40 ? 0 : 39 - code;
      idx = (size_t(nb + wrap_x(g, c.x0 + site + dx)) * 40 + slot) * 9 + e;
    }
    q.w[k] = Wl[idx];
  }
}

template <bool FLY, int NV, class S>
__device__ __forceinline__ void bri_commit(const RowChunk& c, const BriRowRegs<NV, S>& q, typename S::word* buf,
                                           typename S::word* wbuf, int R, int xl, int v, int tid, int nth) {
  using St = BriStage<NV, S>;
  constexpr int SSP = SiteStride<NV, S>::PIECES;
  const int xc = xl < c.n ? xl : c.n - 1;
  u32x4* dst = reinterpret_cast<u32x4*>(buf) + (xc + 1) * SSP;
#pragma unroll
  for (int j = 0; j < St::CH; ++j) dst[j * NV + v] = q.p[j];
#pragma unroll
  for (int k = 0; k < St::HK; ++k) {
    int h = tid + k * nth;
    h = h < 2 * St::SP ? h : 2 * St::SP - 1;
    u32x4* hdst = reinterpret_cast<u32x4*>(buf) + (h < St::SP ? 0 : (c.n + 1) * SSP);
    hdst[h < St::SP ? h : h - St::SP] = q.halo[k];
  }
  if constexpr (FLY) return;
  const int nw = 27 * c.n;
#pragma unroll
  for (int k = 0; k < St::KW; ++k) {
    int w = tid + k * nth;
    w = w < nw ? w : nw - 1;
    const int col = w / (9 * c.n), rem = w - col * 9 * c.n;
    wbuf[col * R * 9 + rem] = q.w[k];
  }
}

// acc += (a + b d.gamma) chi for chi = W' psi, one hop of row (dy, dz, dt)
template <int NV, class S, class T>
__device__ __forceinline__ void bri_hop(const typename S::word* site, const typename S::word* link, bool dag, int v,
                                        T a, T B1, T B2, T B3, T B4, int d0, int d1, int d2, int d3,
                                        cpx<T> (&acc)[4][3]) {
  cpx<T> u[3][3], p[4][3];
  // W' = link or its adjoint (dag is the same for every lane)
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      const cpx<T> l = S::template load<T>(link + (dag ? j * 3 + i : i * 3 + j));
      u[i][j].r = l.r;
      u[i][j].i = dag ? -l.i : l.i;
    }
#pragma unroll
  for (int sp = 0; sp < 4; ++sp)
#pragma unroll
    for (int cc = 0; cc < 3; ++cc) p[sp][cc] = S::template load<T>(site + (sp * 3 + cc) * NV + v);
  // one colour row of chi = W' psi at a time (the spin factor does not mix
  // colours): upper spins += S chi_low, lower += S^dag chi_up with
  // S = sum_mu d_mu s_mu; d_mu is the same for every lane (uniform branches)
#pragma unroll
  for (int cc = 0; cc < 3; ++cc) {
    cpx<T> chi[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      cpx<T> t = zero<T>();
#pragma unroll
      for (int b = 0; b < 3; ++b) t = cmadd(t, u[cc][b], p[q][b]);
      chi[q] = t;
      acc[q][cc] = rmadd(acc[q][cc], a, t);
    }
    if (d3 != 0) {
      acc[0][cc] = rmadd(acc[0][cc], B4, chi[2]);
      acc[1][cc] = rmadd(acc[1][cc], B4, chi[3]);
      acc[2][cc] = rmadd(acc[2][cc], B4, chi[0]);
      acc[3][cc] = rmadd(acc[3][cc], B4, chi[1]);
    }
    if (d2 != 0) {
      acc[0][cc] = cmadd_i(acc[0][cc], -B3, chi[2]);
      acc[1][cc] = cmadd_i(acc[1][cc], B3, chi[3]);
      acc[2][cc] = cmadd_i(acc[2][cc], B3, chi[0]);
      acc[3][cc] = cmadd_i(acc[3][cc], -B3, chi[1]);
    }
    if (d1 != 0) {
      acc[0][cc] = rmadd(acc[0][cc], -B2, chi[3]);
      acc[1][cc] = rmadd(acc[1][cc], B2, chi[2]);
      acc[2][cc] = rmadd(acc[2][cc], B2, chi[1]);
      acc[3][cc] = rmadd(acc[3][cc], -B2, chi[0]);
    }
    if (d0 != 0) {
      acc[0][cc] = cmadd_i(acc[0][cc], -B1, chi[3]);
      acc[1][cc] = cmadd_i(acc[1][cc], -B1, chi[2]);
      acc[2][cc] = cmadd_i(acc[2][cc], B1, chi[1]);
      acc[3][cc] = cmadd_i(acc[3][cc], B1, chi[0]);
    }
  }
#pragma unroll
  for (int q = 0; q < 4; ++q)
#pragma unroll
    for (int cc = 0; cc < 3; ++cc) hold(acc[q][cc]);
}

// On-the-fly links: W_d(x) for the three hops (dx = -1, 0, 1; dy, dz, dt) of
// row r and the chunk's sites, built from V (Tab. 1) straight into the link
// columns, four lanes per (column, site) pair, one per first hop.  Every W_d(x) of the 80
// directions is built where it is used, so no adjoint relation is needed.
template <class S, class T>
__device__ __forceinline__ void bri_build(const Geom& g, const RowChunk& c, const typename S::word* __restrict__ V,
                                          int r, typename S::word* wbuf, int R, int tid, int nth) {
  // GL = 4 consecutive lanes share one (column, site) item: lane `part` sums
  // the orderings that begin with hop number `part` of d, and the partial
  // sums are added in a fixed butterfly (every lane of the group ends with
  // the same bits).  The nth / GL groups step through the 3 n items.
  constexpr int GL = 4;
  int dy, dz, dt;
  bri_row_offset(r, dy, dz, dt);
  const int part = tid % GL;
#pragma unroll 1
  for (int item = tid / GL; item < 3 * c.n; item += nth / GL) {  // uniform over a group
    const int col = item / c.n, site = item - col * c.n;
    const int d[4] = {col - 1, dy, dz, dt};
    if ((d[0] | dy | dz | dt) == 0) continue;  // no hop (a whole group)
    const int x[4] = {c.x0 + site, c.y, c.z, c.t};
    cpx<T> w[3][3];
    const int nperm = brillouin_path_tree_sum<S, T>(g, V, x, d, part, w);
#pragma unroll
    for (int off = 1; off < GL; off *= 2)
#pragma unroll
      for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int b = 0; b < 3; ++b) {
          w[a][b].r += __shfl_xor(w[a][b].r, off);
          w[a][b].i += __shfl_xor(w[a][b].i, off);
        }
    if (part == 0) {
      const T inv = T(1) / T(nperm);
      typename S::word* o = wbuf + col * R * 9 + site * 9;
#pragma unroll
      for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int b = 0; b < 3; ++b) S::template store<T>(o + a * 3 + b, inv * w[a][b]);
    }
  }
}

// The three hops of staged row r (and the diagonal term, with the clover term
// if CLOV, for the own row).  FLY: the link columns hold W_d(x) for all three
// hops (built in place), never an adjoint.
template <bool ADJ, bool CLOV, bool FLY, int NV, class S, class T>
__device__ __forceinline__ void bri_row_compute(int r, const typename S::word* buf, const typename S::word* wbuf,
                                                const typename S::word* lcl, int R, int xl, int v, T diag,
                                                cpx<T> (&acc)[4][3]) {
  constexpr int SSW = SiteStride<NV, S>::WORDS;
  int dy, dz, dt;
  bri_row_offset(r, dy, dz, dt);
#pragma unroll
  for (int dx = -1; dx <= 1; ++dx) {
    const int k = (dx != 0) + (dy != 0) + (dz != 0) + (dt != 0);
    const typename S::word* site = buf + (xl + 1 + dx) * SSW;
    if (k == 0) {
      // own site: the diagonal term
      if constexpr (CLOV) {
        cpx<T> p[4][3];
#pragma unroll
        for (int q = 0; q < 4; ++q)
#pragma unroll
          for (int cc = 0; cc < 3; ++cc) {
            p[q][cc] = S::template load<T>(site + (q * 3 + cc) * NV + v);
            acc[q][cc] = rmadd(acc[q][cc], diag, p[q][cc]);
          }
        clover_madd<S, T>(lcl + xl * 36, p, acc);
      } else {
#pragma unroll
        for (int q = 0; q < 4; ++q)
#pragma unroll
          for (int cc = 0; cc < 3; ++cc)
            acc[q][cc] = rmadd(acc[q][cc], diag, S::template load<T>(site + (q * 3 + cc) * NV + v));
      }
      continue;
    }
    const T a = T(-0.5) * bri_lambda<T>(k);
    const T b = (ADJ ? T(-1) : T(1)) * bri_rho<T>(k);
    const typename S::word* link = wbuf + (dx + 1) * R * 9 + xl * 9;
    bri_hop<NV, S, T>(site, link, !FLY && bri_code(dx, dy, dz, dt) <= 40, v, a, b * T(dx), b * T(dy), b * T(dz),
                      b * T(dt), dx, dy, dz, dt, acc);
  }
}


}  // namespace

// Waves per SIMD: three (168 VGPRs); two below N_v = 8, where a thread moves
// ceil(27 / N_v) link words of every staged row.
template <int NV> struct BriWaves { static constexpr int value = NV < 8 ? 2 : 3; };

// CLOV: adds the site-local clover term (packed, 36 words per site, staged
// in LDS after the link columns).  FLY: Wl holds the one-hop links V and the
// off-axis links are built on the fly for every row.
template <bool ADJ, bool CLOV, bool FLY, int NV, class S, class T>
__global__ void __launch_bounds__(256, BriWaves<NV>::value)
    brillouin_rows_kernel(Geom g, RowTraversal tr, ChunkTiles o, int xcd, const typename S::word* __restrict__ Wl,
                          const typename S::word* __restrict__ in, typename S::word* __restrict__ out,
                          const typename S::word* __restrict__ C, T diag) {
  using W = typename S::word;
  using St = BriStage<NV, S>;
  constexpr int SSW = SiteStride<NV, S>::WORDS, SSP = SiteStride<NV, S>::PIECES;
  extern __shared__ uint4 smem_bri[];
  const int R = int(tr.sb);
  W* buf = reinterpret_cast<W*>(smem_bri);
  W* wbuf = buf + (R + 2) * SSW;  // [3][R][9]
  W* lcl = wbuf + ((27 * R + 3) & ~3);  // [R][36] (CLOV), 16-byte aligned

  const uint32_t L = xcd_block(blockIdx.x, gridDim.x, xcd != 0);
  const RowChunk c = order_chunk(g, tr, o, L);
  const int v = threadIdx.x, xl = threadIdx.y;
  const int tid = xl * NV + v, nth = R * NV;
  const int xm = wrap_x(g, c.x0 - 1), xp = wrap_x(g, c.x0 + c.n);

  cpx<T> acc[4][3];
#pragma unroll
  for (int q = 0; q < 4; ++q)
#pragma unroll
    for (int cc = 0; cc < 3; ++cc) acc[q][cc] = zero<T>();

  // one row in flight while the previous one is applied (three hops of
  // about a thousand instructions per lane hide the load latency); the
  // request after the last row repeats it, unused, so every load is
  // unconditional and in bounds
  constexpr int CLP = 36 * int(sizeof(W)) / 16;  // 16-byte pieces of a site's clover term
  if constexpr (CLOV) copy_pieces<(CLP + NV - 1) / NV>(lcl, C + size_t(c.row_base + c.x0) * 36, c.n * CLP, tid, nth);
  BriRowRegs<NV, S> q;
  bri_issue<FLY, NV, S>(g, c, Wl, in, 0, xm, xp, xl, v, tid, nth, q);
#pragma nounroll
  for (int r = 0; r < kBriRows; ++r) {
    bri_commit<FLY, NV, S>(c, q, buf, wbuf, R, xl, v, tid, nth);
    if constexpr (FLY) bri_build<S, T>(g, c, Wl, r, wbuf, R, tid, nth);
    __syncthreads();
    bri_issue<FLY, NV, S>(g, c, Wl, in, r + 1 < kBriRows ? r + 1 : kBriRows - 1, xm, xp, xl, v, tid, nth, q);
    bri_row_compute<ADJ, CLOV, FLY, NV, S, T>(r, buf, wbuf, lcl, R, xl, v, diag, acc);
    __syncthreads();
  }
  // output through LDS, coalesced 16-byte stores
  {
    W* o = buf + xl * SSW;
#pragma unroll
    for (int q = 0; q < 4; ++q)
#pragma unroll
      for (int cc = 0; cc < 3; ++cc) S::template store<T>(o + (q * 3 + cc) * NV + v, acc[q][cc]);
  }
  __syncthreads();
  {
    const int xc = xl < c.n ? xl : c.n - 1;
    const u32x4* src = reinterpret_cast<const u32x4*>(buf) + xc * SSP;
    u32x4* dst = reinterpret_cast<u32x4*>(out + size_t(c.row_base + c.x0) * St::SW);
    u32x4 o[St::CH];
#pragma unroll
    for (int j = 0; j < St::CH; ++j) o[j] = src[j * NV + v];
#pragma unroll
    for (int j = 0; j < St::CH; ++j) __builtin_nontemporal_store(o[j], &dst[xc * St::SP + j * NV + v]);
  }
}

// Chunk tiles of the D_B row kernels: the largest by x bz rows (by | Ny,
// bz | Nz) whose spinor rows at one t take at most 1.25 MB, the squarer of
// equal sizes, by >= bz on a tie; DSLASH_BRI_TILE_Y, _Z override (0: t-band
// order).  Each output row stages the 27 rows around it, and in the t-band
// order its +-z rows were a band of planes away, gone from the XCD's L2.  On
// 32^4, N_v = 12: FP64 4 x 4, 16.72 against 17.77 ms (2 x 2: 18.00, 8 x 8:
// 17.03); FP32 8 x 4, 7.09 against 7.39 ms (4 x 4: 7.18, 8 x 8: 7.21); W on
// the fly 23.8 against 24.5 ms.  The W-gradient kernel gained nothing (6.96
// ms either way) and keeps the t-band order (tiled = false).
static ChunkTiles bri_tiles(const Geom& g, int R, long site_bytes, bool tiled = true) {
  int by, bz;
  pick_tile(g, long((g.n[0] + R - 1) / R) * R * site_bytes, tiled ? 1280L * 1024 : 0, by, bz);
  return make_chunk_tiles(g, R, knobs().bri_tile_y.get(by), knobs().bri_tile_z.get(bz));
}

// CLOVER_OK = false builds the form without the clover term only (C must be null).
template <int NV, class S, class T, bool FLY, bool CLOVER_OK = true>
static hipError_t brillouin_rows_t(bool adj, const Geom& g, int R, int bt, bool xcd, const void* Wl, const void* in,
                                   void* out, const void* C, double mass, hipStream_t st) {
  using W = typename S::word;
  const RowTraversal tr = make_row_traversal(g, uint32_t(R), uint32_t(bt));
  const ChunkTiles o = bri_tiles(g, R, 12L * NV * long(sizeof(W)));
  const dim3 block(NV, R), grid(tr.rows_plane * uint32_t(g.n[2]) * uint32_t(g.n[3]));
  const size_t lds =
      (size_t(R + 2) * SiteStride<NV, S>::WORDS + size_t(3 * R) * 9 + (C ? 3 + size_t(R) * 36 : 0)) * sizeof(W);
  const T diag = T(mass) + T(15.0 / 8.0);
#define DSL_BK(A, CL)                                                                                        \
  hipLaunchKernelGGL((brillouin_rows_kernel<A, CL, FLY, NV, S, T>), grid, block, lds, st, g, tr, o, int(xcd), (const W*)Wl, \
                     (const W*)in, (W*)out, (const W*)C, diag)
  if constexpr (CLOVER_OK) {
    if (C) {
      if (adj) DSL_BK(true, true); else DSL_BK(false, true);
    } else {
      if (adj) DSL_BK(true, false); else DSL_BK(false, false);
    }
  } else {
    if (C) return hipErrorInvalidValue;
    if (adj) DSL_BK(true, false); else DSL_BK(false, false);
  }
#undef DSL_BK
  return hipGetLastError();
}

// ---------------------------------------------------------------- gradient with respect to W
// G_{W_d}(x) for the 40 stored directions d (slot n(d) - 41): the derivative
// of L = Re sum conj(chi) (D_B psi) with each W taken as a free complex matrix.
// W_d(x) enters the hop of d into out(x) with the spin factor S_d =
// a_k + b_k d.gamma, and, as W_{-d}(x + d) = W_d(x)^dag, the hop of -d into
// out(x + d) with S_{-d} = a_k - b_k d.gamma (eqs. def_der, def_lap, Tab. 1).
// Both factors are Hermitian, so
//   G_{W_d}(x) = sum_v sum_s [ chi(x)_s (x) conj((S_d psi(x + d))_s)
//                            + psi(x)_s (x) conj((S_{-d} chi(x + d))_s) ].
// The stored d reach the 14 rows 13 .. 26 of the 27-row order (the own row
// for d = +x only, then every row with (dt, dz, dy) lexicographically
// positive, where all three dx are stored).  A workgroup owns an x-row chunk;
// each row's psi run, then its chi run, with the halo sites x0 - 1 and x0 + n,
// pass through one LDS buffer.  Lane (x, v) keeps chi(x), psi(x) of its
// right-hand side in registers; it forms the first term of each of the row's
// directions from the psi run and adds the second from the chi run, in its own
// LDS slots.  The N_v shares of a site are then summed in lane order
// (deterministic, no atomics) and written to G_W.  One run at a time keeps the
// kernel at 160 VGPRs, three waves per SIMD.

constexpr int kWgFirstRow = 13;  // the own row; rows 13 .. 26 hold every stored d

// out = (a + sum_mu B_mu gamma_mu) in, B_mu = b d_mu: the spin factor of a
// hop, in the chiral basis of bri_hop; the d_mu tests are uniform.
template <class T>
__device__ __forceinline__ void bri_spin(T a, T B1, T B2, T B3, T B4, int d0, int d1, int d2, int d3,
                                         const cpx<T> (&in)[4][3], cpx<T> (&out)[4][3]) {
#pragma unroll
  for (int q = 0; q < 4; ++q)
#pragma unroll
    for (int cc = 0; cc < 3; ++cc) out[q][cc] = mk(a * in[q][cc].r, a * in[q][cc].i);
#pragma unroll
  for (int cc = 0; cc < 3; ++cc) {
    if (__builtin_amdgcn_readfirstlane(d3) != 0) {
      out[0][cc] = rmadd(out[0][cc], B4, in[2][cc]);
      out[1][cc] = rmadd(out[1][cc], B4, in[3][cc]);
      out[2][cc] = rmadd(out[2][cc], B4, in[0][cc]);
      out[3][cc] = rmadd(out[3][cc], B4, in[1][cc]);
    }
    if (__builtin_amdgcn_readfirstlane(d2) != 0) {
      out[0][cc] = cmadd_i(out[0][cc], -B3, in[2][cc]);
      out[1][cc] = cmadd_i(out[1][cc], B3, in[3][cc]);
      out[2][cc] = cmadd_i(out[2][cc], B3, in[0][cc]);
      out[3][cc] = cmadd_i(out[3][cc], -B3, in[1][cc]);
    }
    if (__builtin_amdgcn_readfirstlane(d1) != 0) {
      out[0][cc] = rmadd(out[0][cc], -B2, in[3][cc]);
      out[1][cc] = rmadd(out[1][cc], B2, in[2][cc]);
      out[2][cc] = rmadd(out[2][cc], B2, in[1][cc]);
      out[3][cc] = rmadd(out[3][cc], -B2, in[0][cc]);
    }
    if (__builtin_amdgcn_readfirstlane(d0) != 0) {
      out[0][cc] = cmadd_i(out[0][cc], -B1, in[3][cc]);
      out[1][cc] = cmadd_i(out[1][cc], -B1, in[2][cc]);
      out[2][cc] = cmadd_i(out[2][cc], B1, in[1][cc]);
      out[3][cc] = cmadd_i(out[3][cc], B1, in[0][cc]);
    }
  }
}

// gm += sum_s l_s (x) conj(r_s)
template <class T>
__device__ __forceinline__ void bri_outer(const cpx<T> (&l)[4][3], const cpx<T> (&r)[4][3], cpx<T> (&gm)[3][3]) {
#pragma unroll
  for (int s = 0; s < 4; ++s)
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
      for (int b = 0; b < 3; ++b) gm[a][b] = cmaddj(gm[a][b], l[s][a], r[s][b]);
}

template <int NV, class S, class T>
__device__ __forceinline__ void bri_lds_spinor(const typename S::word* site, int v, cpx<T> (&p)[4][3]) {
#pragma unroll
  for (int q = 0; q < 4; ++q)
#pragma unroll
    for (int cc = 0; cc < 3; ++cc) p[q][cc] = S::template load<T>(site + (q * 3 + cc) * NV + v);
}

template <int NV, class S, class T>
__global__ void __launch_bounds__(256, 3)
    bri_wgrad_rows_kernel(Geom g, RowTraversal tr, ChunkTiles o, int xcd, const typename S::word* __restrict__ chi,
                          const typename S::word* __restrict__ psi, typename S::word* __restrict__ GW) {
  using W = typename S::word;
  constexpr int SSW = SiteStride<NV, S>::WORDS;
  extern __shared__ uint4 smem_wg[];
  const int R = int(tr.sb);
  W* bs = reinterpret_cast<W*>(smem_wg);              // one staged run, (R + 2) sites
  T* red = reinterpret_cast<T*>(bs + (R + 2) * SSW);  // [3][R][18][NV]

  const uint32_t L = xcd_block(blockIdx.x, gridDim.x, xcd != 0);
  const RowChunk c = order_chunk(g, tr, o, L);
  const int v = threadIdx.x, xl = threadIdx.y;
  const int tid = xl * NV + v, nth = R * NV;
  const int xm = wrap_x(g, c.x0 - 1), xp = wrap_x(g, c.x0 + c.n);
  const int xc = xl < c.n ? xl : c.n - 1;

  cpx<T> ox[4][3], op[4][3];  // chi(x), psi(x) of the lane, read once from global memory
  {
    const size_t base = size_t(c.row_base + c.x0 + xc) * 12 * NV + v;
#pragma unroll
    for (int q = 0; q < 4; ++q)
#pragma unroll
      for (int cc = 0; cc < 3; ++cc) {
        ox[q][cc] = S::template load<T>(chi + base + (q * 3 + cc) * NV);
        op[q][cc] = S::template load<T>(psi + base + (q * 3 + cc) * NV);
      }
  }
  BriRowRegs<NV, S> qr;
  bri_issue<true, NV, S>(g, c, nullptr, psi, kWgFirstRow, xm, xp, xl, v, tid, nth, qr);
#pragma nounroll
  for (int r = kWgFirstRow; r < kBriRows; ++r) {
    int dy, dz, dt;
    bri_row_offset(r, dy, dz, dt);
#pragma unroll
    for (int phase = 0; phase < 2; ++phase) {
      // phase 0 stages psi of the row, phase 1 chi; each requests the next run
      __syncthreads();  // the staged run and the sums of the previous phase or row are read
      bri_commit<true, NV, S>(c, qr, bs, nullptr, R, xl, v, tid, nth);
      __syncthreads();
      const int rn = phase == 0 ? r : (r + 1 < kBriRows ? r + 1 : kBriRows - 1);
      bri_issue<true, NV, S>(g, c, nullptr, phase == 0 ? chi : psi, rn, xm, xp, xl, v, tid, nth, qr);
#pragma unroll
      for (int dx = -1; dx <= 1; ++dx) {
        if (r == kWgFirstRow && dx != 1) continue;
        const int k = (dx != 0) + (dy != 0) + (dz != 0) + (dt != 0);
        const T a = T(-0.5) * bri_lambda<T>(k), b = (phase == 0 ? T(1) : T(-1)) * bri_rho<T>(k);
        cpx<T> gm[3][3];
#pragma unroll
        for (int i = 0; i < 3; ++i)
#pragma unroll
          for (int j = 0; j < 3; ++j) gm[i][j] = zero<T>();
        cpx<T> f[4][3], sf[4][3];
        bri_lds_spinor<NV, S, T>(bs + (xl + 1 + dx) * SSW, v, f);
        bri_spin<T>(a, b * T(dx), b * T(dy), b * T(dz), b * T(dt), dx, dy, dz, dt, f, sf);
        // phase 0: chi(x) (x) conj(S_d psi(x + d)); phase 1: psi(x) (x) conj(S_{-d} chi(x + d))
        if (phase == 0) bri_outer<T>(ox, sf, gm);
        else bri_outer<T>(op, sf, gm);
        // the lane's own slots of the row's sums: written in phase 0, added to in phase 1
        T* mine = red + ((dx + 1) * R + xl) * 18 * NV + v;
#pragma unroll
        for (int e = 0; e < 9; ++e) {
          if (phase == 0) {
            mine[(2 * e) * NV] = gm[e / 3][e % 3].r;
            mine[(2 * e + 1) * NV] = gm[e / 3][e % 3].i;
          } else {
            mine[(2 * e) * NV] += gm[e / 3][e % 3].r;
            mine[(2 * e + 1) * NV] += gm[e / 3][e % 3].i;
          }
        }
      }
    }
    __syncthreads();
    // sums over the N_v lanes of each (direction, site, element), in lane order
    const int k0 = r == kWgFirstRow ? 2 : 0;
    const int nout = (3 - k0) * c.n * 9;
    for (int o = tid; o < nout; o += nth) {
      const int k = k0 + o / (c.n * 9), rem = o - (k - k0) * c.n * 9;
      const int site = rem / 9, e = rem - site * 9;
      const T* src = red + ((k * R + site) * 18 + 2 * e) * NV;
      T re = T(0), im = T(0);
#pragma unroll
      for (int l = 0; l < NV; ++l) {
        re += src[l];
        im += src[NV + l];
      }
      const int slot = bri_code(k - 1, dy, dz, dt) - 41;
      S::template store<T>(GW + (size_t(c.row_base + c.x0 + site) * 40 + slot) * 9 + e, mk(re, im));
    }
  }
}

template <int NV, class S, class T>
static hipError_t brillouin_wgrad_rows_t(const Geom& g, int R, int bt, bool xcd, const void* chi, const void* psi,
                                         void* GW, hipStream_t st) {
  using W = typename S::word;
  const RowTraversal tr = make_row_traversal(g, uint32_t(R), uint32_t(bt));
  const ChunkTiles o = bri_tiles(g, R, 12L * NV * long(sizeof(W)), false);
  const dim3 block(NV, R), grid(tr.rows_plane * uint32_t(g.n[2]) * uint32_t(g.n[3]));
  const size_t lds = size_t(R + 2) * SiteStride<NV, S>::WORDS * sizeof(W) + size_t(3 * R) * 18 * NV * sizeof(T);
  hipLaunchKernelGGL((bri_wgrad_rows_kernel<NV, S, T>), grid, block, lds, st, g, tr, o, int(xcd), (const W*)chi,
                     (const W*)psi, (W*)GW);
  return hipGetLastError();
}

// ---------------------------------------------------------------- FP64, staged straight into LDS
// The FP64 D_B keeps the row staging of brillouin_rows_kernel, but its rows
// are copied from global memory into LDS by the direct-to-LDS load path
// (global_load_lds_dwordx4: lane l of a wave writes LDS bytes [b + 16 l,
// b + 16 l + 16) for a wave-uniform b), so no staged row passes through
// registers.  With the hop computed one colour row of the link at a time the
// kernel fits three waves per SIMD, where register staging of FP64 rows
// allowed one.  A row in LDS is [halo x0 - 1][the chunk's n sites][halo
// x0 + n] without padding (16-byte reads of consecutive lanes fall on
// consecutive banks), then its three link columns [dx + 1][site][9].
// Workgroup: 16 sites x N_v right-hand sides, a multiple of 64 threads, so
// every wave covers whole 64-piece LDS ranges; chunks of fewer live sites
// (the row's last, or rows shorter than 16) stage only their own.
constexpr int kDmaSites = 16;

__device__ __forceinline__ void lds_dma16(const void* src, void* lds_wave_base) {
  __builtin_amdgcn_global_load_lds(src, (__attribute__((address_space(3))) void*)lds_wave_base, 16, 0, 0);
}

// Stage row r (spinor run with halos, three link columns) of chunk c into buf
// and wbuf: LDS piece L of the row is loaded by lane L % 64 of wave
// (L / 64) % waves, instruction L / (64 waves).
template <int NV>
__device__ __forceinline__ void bri_dma_row(const Geom& g, const RowChunk& c, const C128::word* __restrict__ Wl,
                                            const C128::word* __restrict__ in, int r, int xm, int xp, int wave,
                                            int lane, int waves, char* buf, char* wbuf) {
  constexpr int SP = 12 * NV;  // 16-byte pieces (FP64 complex words) per site
  int dy, dz, dt;
  bri_row_offset(r, dy, dz, dt);
  const uint32_t nb = bri_row_base(g, c, dy, dz, dt);
  const int np = (c.n + 2) * SP;
  for (int base = wave * 64; base < np; base += waves * 64) {
    const int L = base + lane;
    if (L < np) {
      const int slot = L / SP, pp = L - slot * SP;
      const int site = slot == 0 ? xm : (slot == c.n + 1 ? xp : c.x0 + slot - 1);
      lds_dma16(in + size_t(nb + site) * SP + pp, buf + size_t(__builtin_amdgcn_readfirstlane(base)) * 16);
    }
  }
  const int nw = 27 * kDmaSites;
  for (int base = wave * 64; base < nw; base += waves * 64) {
    const int L = base + lane;
    if (L < nw) {
      const int col = L / (9 * kDmaSites), rem = L - col * 9 * kDmaSites;
      int site = rem / 9;
      const int e = rem - site * 9;
      site = site < c.n ? site : c.n - 1;
      const int code = bri_code(col - 1, dy, dz, dt);
      size_t idx;
      if (code > 40) {
        idx = (size_t(c.row_base + c.x0 + site) * 40 + (code - 41)) * 9 + e;  // W_d(x), stored
      } else {
        const int slot = code == 40 ? 0 : 39 - code;  // W_{-d}(x + d); d = 0: any valid word (unused)
        idx = (size_t(nb + wrap_x(g, c.x0 + site + col - 1)) * 40 + slot) * 9 + e;
      }
      lds_dma16(Wl + idx, wbuf + size_t(__builtin_amdgcn_readfirstlane(base)) * 16);
    }
  }
}

// acc += (a + b d.gamma) W' psi for one hop, W' = the link or its adjoint,
// taken one source spin at a time: chi_q = W' psi_q (one colour triple) goes
// to acc_q with weight a and, for every non-zero d_mu, to the spin that
// gamma_mu pairs with q (chiral basis, as in bri_hop), so only psi_q and chi_q
// are live beside the link.
template <int NV, class T>
__device__ __forceinline__ void bri_hop_lean(const C128::word* site, const C128::word* link, bool dag, int v, T a,
                                             T B1, T B2, T B3, T B4, int d0, int d1, int d2, int d3,
                                             cpx<T> (&acc)[4][3]) {
  cpx<T> u[3][3];
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      const cpx<T> l = C128::template load<T>(link + (dag ? j * 3 + i : i * 3 + j));
      u[i][j].r = l.r;
      u[i][j].i = dag ? -l.i : l.i;
    }
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    cpx<T> p[3], chi[3];
#pragma unroll
    for (int b = 0; b < 3; ++b) p[b] = C128::template load<T>(site + (q * 3 + b) * NV + v);
#pragma unroll
    for (int cc = 0; cc < 3; ++cc) {
      cpx<T> t = zero<T>();
#pragma unroll
      for (int b = 0; b < 3; ++b) t = cmadd(t, u[cc][b], p[b]);
      chi[cc] = t;
      acc[q][cc] = rmadd(acc[q][cc], a, t);
    }
    // partner spins: gamma_4 and gamma_3 pair q with q ^ 2, gamma_2 and gamma_1
    // with 3 - q; the factors, by source spin q = 0, 1, 2, 3:
    //   gamma_4: B4 (all)   gamma_3: i B3 (+, -, -, +)
    //   gamma_2: B2 (-, +, +, -)   gamma_1: i B1 (+, +, -, -)
    const int P43 = q ^ 2, P21 = 3 - q;
    const T s3 = (q == 1 || q == 2) ? T(-1) : T(1);
    const T s2 = (q == 1 || q == 2) ? T(1) : T(-1);
    const T s1 = q <= 1 ? T(1) : T(-1);
    // d is uniform over the workgroup: scalar branches skip the zero axes
    if (__builtin_amdgcn_readfirstlane(d3) != 0) {
#pragma unroll
      for (int cc = 0; cc < 3; ++cc) acc[P43][cc] = rmadd(acc[P43][cc], B4, chi[cc]);
    }
    if (__builtin_amdgcn_readfirstlane(d2) != 0) {
#pragma unroll
      for (int cc = 0; cc < 3; ++cc) acc[P43][cc] = cmadd_i(acc[P43][cc], s3 * B3, chi[cc]);
    }
    if (__builtin_amdgcn_readfirstlane(d1) != 0) {
#pragma unroll
      for (int cc = 0; cc < 3; ++cc) acc[P21][cc] = rmadd(acc[P21][cc], s2 * B2, chi[cc]);
    }
    if (__builtin_amdgcn_readfirstlane(d0) != 0) {
#pragma unroll
      for (int cc = 0; cc < 3; ++cc) acc[P21][cc] = cmadd_i(acc[P21][cc], s1 * B1, chi[cc]);
    }
  }
#pragma unroll
  for (int q = 0; q < 4; ++q)
#pragma unroll
    for (int cc = 0; cc < 3; ++cc) hold(acc[q][cc]);
}

constexpr size_t kDmaRowBytes = (size_t(kDmaSites + 2) * 12 * 12 + size_t(27) * kDmaSites) * 16;

// One row buffer, three workgroups per CU: each loads a row, then applies it,
// while the others do the same out of step.
template <bool ADJ, int NV>
__global__ void __launch_bounds__(kDmaSites * NV, 3)
    brillouin_rows_dma_kernel(Geom g, RowTraversal tr, ChunkTiles o, int xcd, const C128::word* __restrict__ Wl,
                              const C128::word* __restrict__ in, C128::word* __restrict__ out, double diag) {
  using T = double;
  constexpr int SW = 12 * NV;
  extern __shared__ uint4 smem_bdma[];
  char* const buf = reinterpret_cast<char*>(smem_bdma);       // [(16 + 2) SW] pieces: the row with its halos
  char* const wbuf = buf + size_t(kDmaSites + 2) * SW * 16;   // [3][16][9] pieces: its link columns

  const uint32_t L = xcd_block(blockIdx.x, gridDim.x, xcd != 0);
  const RowChunk c = order_chunk(g, tr, o, L);
  const int v = threadIdx.x, xl = threadIdx.y;
  const int tid = xl * NV + v;
  const int wave = tid >> 6, lane = tid & 63, waves = kDmaSites * NV / 64;
  const int xm = wrap_x(g, c.x0 - 1), xp = wrap_x(g, c.x0 + c.n);

  cpx<T> acc[4][3];
#pragma unroll
  for (int q = 0; q < 4; ++q)
#pragma unroll
    for (int cc = 0; cc < 3; ++cc) acc[q][cc] = zero<T>();

#pragma nounroll
  for (int r = 0; r < kBriRows; ++r) {
    __syncthreads();  // the previous row's hops are done with the buffers
    bri_dma_row<NV>(g, c, Wl, in, r, xm, xp, wave, lane, waves, buf, wbuf);
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
    const C128::word* lrow = reinterpret_cast<const C128::word*>(buf);
    const C128::word* lw = reinterpret_cast<const C128::word*>(wbuf);
    int dy, dz, dt;
    bri_row_offset(r, dy, dz, dt);
#pragma unroll
    for (int dx = -1; dx <= 1; ++dx) {
      const int k = (dx != 0) + (dy != 0) + (dz != 0) + (dt != 0);
      const C128::word* site = lrow + (xl + 1 + dx) * SW;
      if (k == 0) {
#pragma unroll
        for (int q = 0; q < 4; ++q)
#pragma unroll
          for (int cc = 0; cc < 3; ++cc)
            acc[q][cc] = rmadd(acc[q][cc], diag, C128::template load<T>(site + (q * 3 + cc) * NV + v));
        continue;
      }
      const T a = T(-0.5) * bri_lambda<T>(k);
      const T b = (ADJ ? T(-1) : T(1)) * bri_rho<T>(k);
      const C128::word* link = lw + ((dx + 1) * kDmaSites + xl) * 9;
      bri_hop_lean<NV, T>(site, link, bri_code(dx, dy, dz, dt) <= 40, v, a, b * T(dx), b * T(dy), b * T(dz),
                          b * T(dt), dx, dy, dz, dt, acc);
    }
  }
  // each lane writes its own 12 words: the N_v lanes of a site cover 16 N_v
  // contiguous bytes per component
  if (xl < c.n) {
    u32x4* o = reinterpret_cast<u32x4*>(out + size_t(c.row_base + c.x0 + xl) * SW + v);
#pragma unroll
    for (int q = 0; q < 4; ++q)
#pragma unroll
      for (int cc = 0; cc < 3; ++cc)
        __builtin_nontemporal_store(__builtin_bit_cast(u32x4, make_double2(acc[q][cc].r, acc[q][cc].i)),
                                    o + (q * 3 + cc) * NV);
  }
}

// Chunk length of the register-staged D_B (C64; N_v = 4, 8, 12, 16, 24), or 0
// when the configuration is not covered.
static int brillouin_rows_sites(int dtype, const Geom& g) {
  // FP32 only: the FP64 variant would not fit in registers
  const int nv = g.nv;
  if (dtype != DT_C64 || (nv != 4 && nv != 8 && nv != 12 && nv != 16 && nv != 24)) return 0;
  int R = row_sites_default(g.n[0], nv);
  R = knobs().row_sites.get(R);
  if (R > g.n[0]) R = g.n[0];
  // the halo sites (2 * 12 N_v words) take HK 16-byte pieces per thread:
  // R HK >= 12; 64 .. 256 threads
  const int hk = nv > 16 ? 2 : 1;
  if (R * hk < 12 || R * nv > 256 || R * nv < 64) return 0;
  return R;
}

// Row-staged D_B: FP32 storage for N_v = 4, 8, 12, 16, 24 (the clover term for
// N_v = 12 only), FP64 storage for N_v = 12.  Returns hipErrorNotSupported
// when the configuration is not covered (the caller then uses the direct
// kernel).  DSLASH_ROWS=0 disables it.
hipError_t launch_brillouin_rows(bool adj, int dtype, const Geom& g, const void* Wl, const void* in, void* out,
                                 double mass, hipStream_t st, const void* clover) {
  if (knobs().rows.get(1) == 0) return hipErrorNotSupported;
  if (!aligned16(Wl) || !aligned16(in) || !aligned16(out) || !aligned16(clover)) return hipErrorNotSupported;
  if (dtype == DT_C128 && g.nv == 12 && !clover) {
    // FP64: the direct-to-LDS staged kernel, chunks of 16 sites
    const RowTraversal tr = make_row_traversal(g, uint32_t(kDmaSites), uint32_t(knobs().tband.get(2)));
    const ChunkTiles o = bri_tiles(g, kDmaSites, 12L * 12 * long(sizeof(C128::word)));
    const dim3 block(12, kDmaSites), grid(tr.rows_plane * uint32_t(g.n[2]) * uint32_t(g.n[3]));
    const bool xcd = knobs().xcd.get(1) != 0;
    const double diag = mass + 15.0 / 8.0;
#define DSL_BD(A)                                                                                         \
  hipLaunchKernelGGL((brillouin_rows_dma_kernel<A, 12>), grid, block, kDmaRowBytes, st, g, tr, o, int(xcd), \
                     (const C128::word*)Wl, (const C128::word*)in, (C128::word*)out, diag)
    if (adj) DSL_BD(true); else DSL_BD(false);
#undef DSL_BD
    return hipGetLastError();
  }
  const int R = brillouin_rows_sites(dtype, g);
  if (R == 0 || (clover && g.nv != 12)) return hipErrorNotSupported;
  int bt = 2;
  bt = knobs().tband.get(bt);
  bool xcd = true;
  xcd = knobs().xcd.get(xcd) != 0;
  switch (g.nv) {
    case 4: return brillouin_rows_t<4, C64, float, false, false>(adj, g, R, bt, xcd, Wl, in, out, nullptr, mass, st);
    case 8: return brillouin_rows_t<8, C64, float, false, false>(adj, g, R, bt, xcd, Wl, in, out, nullptr, mass, st);
    case 16: return brillouin_rows_t<16, C64, float, false, false>(adj, g, R, bt, xcd, Wl, in, out, nullptr, mass, st);
    case 24: return brillouin_rows_t<24, C64, float, false, false>(adj, g, R, bt, xcd, Wl, in, out, nullptr, mass, st);
  }
  return brillouin_rows_t<12, C64, float, false>(adj, g, R, bt, xcd, Wl, in, out, clover, mass, st);
}

// D_B with the off-axis links built from V inside the row-staged kernel (no W
// array).  The FP32 configurations of launch_brillouin_rows (N_v = 4, 8, 12,
// 16, 24; the clover term at N_v = 12); hipErrorNotSupported otherwise.
hipError_t launch_brillouin_fly(bool adj, int dtype, const Geom& g, const void* V, const void* in, void* out,
                                double mass, hipStream_t st, const void* clover) {
  if (!aligned16(V) || !aligned16(in) || !aligned16(out) || !aligned16(clover)) return hipErrorNotSupported;
  const int R = brillouin_rows_sites(dtype, g);
  if (R == 0 || (clover && g.nv != 12)) return hipErrorNotSupported;
  int bt = 2;
  bt = knobs().tband.get(bt);
  bool xcd = true;
  xcd = knobs().xcd.get(xcd) != 0;
  switch (g.nv) {
    case 4: return brillouin_rows_t<4, C64, float, true, false>(adj, g, R, bt, xcd, V, in, out, nullptr, mass, st);
    case 8: return brillouin_rows_t<8, C64, float, true, false>(adj, g, R, bt, xcd, V, in, out, nullptr, mass, st);
    case 16: return brillouin_rows_t<16, C64, float, true, false>(adj, g, R, bt, xcd, V, in, out, nullptr, mass, st);
    case 24: return brillouin_rows_t<24, C64, float, true, false>(adj, g, R, bt, xcd, V, in, out, nullptr, mass, st);
  }
  return brillouin_rows_t<12, C64, float, true>(adj, g, R, bt, xcd, V, in, out, clover, mass, st);
}

// Row-staged gradient with respect to W (FP32 storage, N_v = 4, 8, 12, 16,
// 24, the chunks of brillouin_rows_sites); hipErrorNotSupported otherwise (the
// caller then uses the per-direction kernel).  DSLASH_ROWS=0 disables it.
hipError_t launch_brillouin_wgrad_rows(int dtype, const Geom& g, const void* chi, const void* psi, void* GW,
                                       hipStream_t st) {
  if (knobs().rows.get(1) == 0) return hipErrorNotSupported;
  if (!aligned16(chi) || !aligned16(psi) || !aligned16(GW)) return hipErrorNotSupported;
  if (dtype != DT_C64) return hipErrorNotSupported;
  const int R = brillouin_rows_sites(dtype, g);
  if (R == 0) return hipErrorNotSupported;
  int bt = 2;
  bt = knobs().tband.get(bt);
  const bool xcd = knobs().xcd.get(1) != 0;
  switch (g.nv) {
    case 4: return brillouin_wgrad_rows_t<4, C64, float>(g, R, bt, xcd, chi, psi, GW, st);
    case 8: return brillouin_wgrad_rows_t<8, C64, float>(g, R, bt, xcd, chi, psi, GW, st);
    case 16: return brillouin_wgrad_rows_t<16, C64, float>(g, R, bt, xcd, chi, psi, GW, st);
    case 24: return brillouin_wgrad_rows_t<24, C64, float>(g, R, bt, xcd, chi, psi, GW, st);
  }
  return brillouin_wgrad_rows_t<12, C64, float>(g, R, bt, xcd, chi, psi, GW, st);
}

}  // namespace dsl
