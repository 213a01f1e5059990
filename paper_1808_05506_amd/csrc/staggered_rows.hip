// Row-staged D_S (see rows.hpp): a workgroup owns an x-row chunk of R sites
// and all N_v right-hand sides.  The seven input rows (+y, -y, +z, -z, +t, -t
// and the chunk's own row with the halo sites x0 - 1 and x0 + n) pass one at a
// time through one LDS buffer; each is requested DEPTH rows before it is used,
// with coalesced loads of whole runs of memory.  The chunk's links and, per
// backward row, V_mu(x - mu) are staged as well.  Thread (x, v) accumulates
//   out(x) = m psi(x) +/- 1/2 sum_mu eta_mu(x) [V_mu(x) psi(x + mu) - V_mu(x - mu)^dag psi(x - mu)]
// (minus for the adjoint) and stores its three colour components directly:
// the N_v lanes of a site write consecutive words.
#include <stdlib.h>

#include "launch.hpp"
#include "rows.hpp"

namespace dsl {

namespace {

// LDS layout, in storage words:
//   buf  [(R + 2) * SSW]  the staged row (a neighbour row at index 1 .. n, the
//                         own row at 0 .. n + 1 with its halo sites)
//   lown [(R + 1) * 4 LW] links of sites x0 - 1 .. x0 + n - 1 (index x - x0 + 1)
//   lnb  [R * LW]         V_mu(x - mu) of the current backward row
// with LW = 9 words per link, or 6 for compressed links (first two rows).
template <int NV, class S, int LW>
size_t srows_lds_words(int R) {
  return size_t(R + 2) * Stage<3, NV, S>::SSW + size_t(R + 1) * 4 * LW + size_t(R) * LW;
}

template <int NV, class S>
using SPiece = typename Stage<3, NV, S>::P;
template <int NV, class S>
constexpr int kSCH = Stage<3, NV, S>::CH;

// Neighbour row (MU, SGN): lane (x, v) takes pieces j N_v + v of its site;
// slot CH carries one word of V_mu(x - mu) for a backward row.
template <int MU, int SGN, int NV, class S, int LW>
__device__ __forceinline__ void srow_issue(const Geom& g, const RowChunk& c, const typename S::word* __restrict__ U,
                                           const typename S::word* __restrict__ in, int xl, int v, int tid,
                                           SPiece<NV, S> (&r)[kSCH<NV, S> + 1]) {
  using W = typename S::word;
  using P = SPiece<NV, S>;
  static_assert(sizeof(P) == sizeof(W), "one link word per piece slot");
  constexpr int SW = 3 * NV, CH = kSCH<NV, S>;
  const uint32_t nrow = row_base_shift(g, c, MU, SGN) + uint32_t(c.x0);
  const int xc = xl < c.n ? xl : c.n - 1;
  const P* src = reinterpret_cast<const P*>(in + size_t(nrow + xc) * SW);
#pragma unroll
  for (int j = 0; j < CH; ++j) r[j] = src[j * NV + v];
  if (SGN < 0) {
    const int w = tid < c.n * LW ? tid : c.n * LW - 1;
    const int k = w / LW, e = w - k * LW;
    r[CH] = reinterpret_cast<const P*>(U)[(size_t(nrow + k) * 4 + MU) * LW + e];
  }
}

template <int SGN, int NV, class S, int LW>
__device__ __forceinline__ void srow_commit(const RowChunk& c, const SPiece<NV, S> (&r)[kSCH<NV, S> + 1],
                                            typename S::word* row, typename S::word* lnb, int xl, int v, int tid) {
  using P = SPiece<NV, S>;
  constexpr int CH = kSCH<NV, S>, SSP = Stage<3, NV, S>::SSP;
  const int xc = xl < c.n ? xl : c.n - 1;
  P* dst = reinterpret_cast<P*>(row) + xc * SSP;
#pragma unroll
  for (int j = 0; j < CH; ++j) dst[j * NV + v] = r[j];
  if (SGN < 0) reinterpret_cast<P*>(lnb)[tid < c.n * LW ? tid : c.n * LW - 1] = r[CH];
}

// Own row: CH pieces of site x and, in slot CH, one piece of the halo sites
// x0 - 1, x0 + n (2 * 3 N_v words; the launcher checks there are enough threads).
template <int NV, class S>
__device__ __forceinline__ void sown_issue(const RowChunk& c, const typename S::word* __restrict__ in, int xm, int xp,
                                           int xl, int v, int tid, SPiece<NV, S> (&r)[kSCH<NV, S> + 1]) {
  using P = SPiece<NV, S>;
  constexpr int SW = 3 * NV, CH = kSCH<NV, S>, SP = CH * NV;
  const int xc = xl < c.n ? xl : c.n - 1;
  const P* src = reinterpret_cast<const P*>(in + size_t(c.row_base + c.x0 + xc) * SW);
#pragma unroll
  for (int j = 0; j < CH; ++j) r[j] = src[j * NV + v];
  const int h = tid < 2 * SP ? tid : 2 * SP - 1;
  const int hs = h < SP ? xm : xp;
  r[CH] = reinterpret_cast<const P*>(in + size_t(c.row_base + hs) * SW)[h < SP ? h : h - SP];
}

template <int NV, class S>
__device__ __forceinline__ void sown_commit(const RowChunk& c, const SPiece<NV, S> (&r)[kSCH<NV, S> + 1],
                                            typename S::word* buf, int xl, int v, int tid) {
  using P = SPiece<NV, S>;
  constexpr int CH = kSCH<NV, S>, SP = CH * NV, SSP = Stage<3, NV, S>::SSP;
  const int xc = xl < c.n ? xl : c.n - 1;
  P* dst = reinterpret_cast<P*>(buf) + (xc + 1) * SSP;
#pragma unroll
  for (int j = 0; j < CH; ++j) dst[j * NV + v] = r[j];
  const int h = tid < 2 * SP ? tid : 2 * SP - 1;
  P* hdst = reinterpret_cast<P*>(buf) + (h < SP ? 0 : (c.n + 1) * SSP);
  hdst[h < SP ? h : h - SP] = r[CH];
}

// acc += eta V psi (forward) or acc -= eta V^dag psi (backward), operands in LDS
template <bool DAG, int NV, class S, class T, int LW>
__device__ __forceinline__ void shop(const typename S::word* site, const typename S::word* link, int v, T eta,
                                     cpx<T> (&acc)[3]) {
  cpx<T> p[3];
  lds_column<3, NV, S, T>(site, v, p);
  if constexpr (LW == 6) {
    // compressed link: complete the third row, then the same products
    cpx<T> u[3][3];
    load_link_lw<6, S, T>(link, u);
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      cpx<T> t = zero<T>();
#pragma unroll
      for (int b = 0; b < 3; ++b) t = DAG ? cjmadd(t, u[b][a], p[b]) : cmadd(t, u[a][b], p[b]);
      acc[a] = rmadd(acc[a], DAG ? -eta : eta, t);
      hold(acc[a]);
    }
  } else {
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      cpx<T> t = zero<T>();
#pragma unroll
      for (int b = 0; b < 3; ++b) {
        if (DAG)
          t = cjmadd(t, S::template load<T>(link + b * 3 + a), p[b]);
        else
          t = cmadd(t, S::template load<T>(link + a * 3 + b), p[b]);
      }
      acc[a] = rmadd(acc[a], DAG ? -eta : eta, t);
      hold(acc[a]);
    }
  }
}

template <int DEPTH> struct SRowsWaves { static constexpr int value = DEPTH <= 3 ? 4 : 3; };

}  // namespace

template <int DEPTH, bool ADJ, int NV, class S, class T, int LW>
__global__ void __launch_bounds__(256, SRowsWaves<DEPTH>::value)
    staggered_rows_kernel(Geom g, RowTraversal tr, int xcd, const typename S::word* __restrict__ U,
                          const typename S::word* __restrict__ in, typename S::word* __restrict__ out, T mass) {
  using W = typename S::word;
  using P = SPiece<NV, S>;
  constexpr int SW = 3 * NV, CH = kSCH<NV, S>;
  constexpr int SSW = Stage<3, NV, S>::SSW;
  extern __shared__ uint4 smem_srows[];
  const int R = int(tr.sb);
  W* buf = reinterpret_cast<W*>(smem_srows);
  W* lown = buf + (R + 2) * SSW;
  W* lnb = lown + (R + 1) * 4 * LW;

  const uint32_t L = xcd_block(blockIdx.x, gridDim.x, xcd != 0);
  const RowChunk c = row_chunk(g, tr, L);
  const int v = threadIdx.x, xl = threadIdx.y;
  const int tid = xl * NV + v, nth = R * NV;
  const int xm = wrap_x(g, c.x0 - 1), xp = wrap_x(g, c.x0 + c.n);

  P r0[CH + 1], r1[CH + 1], r2[CH + 1], r3[CH + 1], r4[CH + 1], r5[CH + 1], r6[CH + 1];
#define DSL_SISSUE(K)                                                                   \
  do {                                                                                  \
    if constexpr (K == 0) srow_issue<1, +1, NV, S, LW>(g, c, U, in, xl, v, tid, r0);        \
    if constexpr (K == 1) srow_issue<1, -1, NV, S, LW>(g, c, U, in, xl, v, tid, r1);        \
    if constexpr (K == 2) srow_issue<2, +1, NV, S, LW>(g, c, U, in, xl, v, tid, r2);        \
    if constexpr (K == 3) srow_issue<2, -1, NV, S, LW>(g, c, U, in, xl, v, tid, r3);        \
    if constexpr (K == 4) srow_issue<3, +1, NV, S, LW>(g, c, U, in, xl, v, tid, r4);        \
    if constexpr (K == 5) srow_issue<3, -1, NV, S, LW>(g, c, U, in, xl, v, tid, r5);        \
    if constexpr (K == 6) sown_issue<NV, S>(c, in, xm, xp, xl, v, tid, r6);             \
  } while (0)
  DSL_SISSUE(0);
  if constexpr (DEPTH > 1) DSL_SISSUE(1);
  if constexpr (DEPTH > 2) DSL_SISSUE(2);
  if constexpr (DEPTH > 3) DSL_SISSUE(3);
  if constexpr (DEPTH > 4) DSL_SISSUE(4);
  if constexpr (DEPTH > 5) DSL_SISSUE(5);
  if constexpr (DEPTH > 6) DSL_SISSUE(6);
  {
    // links of the chunk's sites (index 1 .. n) and of the halo site x0 - 1
    constexpr int LP = 4 * LW * int(sizeof(W)) / 16;  // 16-byte pieces per site
    constexpr int K = (LP + NV - 1) / NV;              // pieces per thread
    const u32x4* own = reinterpret_cast<const u32x4*>(U + size_t(c.row_base + c.x0) * 4 * LW);
    const u32x4* halo = reinterpret_cast<const u32x4*>(U + size_t(c.row_base + xm) * 4 * LW);
    const int pieces = c.n * LP;
    u32x4 lr[K], lh;
#pragma unroll
    for (int j = 0; j < K; ++j) {
      const int i = tid + j * nth;
      lr[j] = own[i < pieces ? i : pieces - 1];
    }
    lh = halo[tid < LP ? tid : LP - 1];
    u32x4* down = reinterpret_cast<u32x4*>(lown + 4 * LW);
#pragma unroll
    for (int j = 0; j < K; ++j) {
      const int i = tid + j * nth;
      down[i < pieces ? i : pieces - 1] = lr[j];
    }
    reinterpret_cast<u32x4*>(lown)[tid < LP ? tid : LP - 1] = lh;
  }

  // eta_mu(x) = (-1)^(x_1 + ... + x_{mu-1}) for the site of this lane
  const int x = c.x0 + xl;
  const T ey = (x & 1) ? T(-1) : T(1);
  const T ez = ((x + c.y) & 1) ? T(-1) : T(1);
  const T et = ((x + c.y + c.z) & 1) ? T(-1) : T(1);

  cpx<T> acc[3] = {zero<T>(), zero<T>(), zero<T>()};
  W* const row = buf + SSW;  // neighbour rows sit at index 1 .. n
  const int xc = xl < c.n ? xl : c.n - 1;
#define DSL_SROW_STEP(K, MU, SGN, CUR, ETA)                                                      \
  srow_commit<SGN, NV, S, LW>(c, CUR, row, lnb, xl, v, tid);                                     \
  __syncthreads();                                                                               \
  if constexpr (K + DEPTH < 7) DSL_SISSUE(K + DEPTH);                                            \
  if (SGN > 0)                                                                                   \
    shop<false, NV, S, T, LW>(row + xc * SSW, lown + (xc + 1) * 4 * LW + MU * LW, v, ETA, acc);  \
  else                                                                                           \
    shop<true, NV, S, T, LW>(row + xc * SSW, lnb + xc * LW, v, ETA, acc);                        \
  __syncthreads();
  DSL_SROW_STEP(0, 1, +1, r0, ey)
  DSL_SROW_STEP(1, 1, -1, r1, ey)
  DSL_SROW_STEP(2, 2, +1, r2, ez)
  DSL_SROW_STEP(3, 2, -1, r3, ez)
  DSL_SROW_STEP(4, 3, +1, r4, et)
  DSL_SROW_STEP(5, 3, -1, r5, et)
#undef DSL_SROW_STEP
#undef DSL_SISSUE

  sown_commit<NV, S>(c, r6, buf, xl, v, tid);
  __syncthreads();
  // x hops (eta_1 = 1): x + 1 at index xc + 2, x - 1 (and its link) at index xc
  shop<false, NV, S, T, LW>(buf + (xc + 2) * SSW, lown + (xc + 1) * 4 * LW, v, T(1), acc);
  shop<true, NV, S, T, LW>(buf + xc * SSW, lown + xc * 4 * LW, v, T(1), acc);
  cpx<T> self[3];
  lds_column<3, NV, S, T>(buf + (xc + 1) * SSW, v, self);
  const T half = ADJ ? T(-0.5) : T(0.5);
  if (xl < c.n) {
    W* o = out + size_t(c.row_base + c.x0 + xl) * SW + v;
#pragma unroll
    for (int cc = 0; cc < 3; ++cc) {
      cpx<T> z;
      z.r = fma(mass, self[cc].r, half * acc[cc].r);
      z.i = fma(mass, self[cc].i, half * acc[cc].i);
      S::template store<T>(o + cc * NV, z);
    }
  }
}

template <int DEPTH, int NV, class S, class T, int LW>
static hipError_t staggered_rows_t(bool adj, const Geom& g, int R, int bt, bool xcd, const void* U, const void* in,
                                   void* out, double mass, hipStream_t st) {
  using W = typename S::word;
  const RowTraversal tr = make_row_traversal(g, uint32_t(R), uint32_t(bt));
  const dim3 block(NV, R), grid(tr.rows_plane * uint32_t(g.n[2]) * uint32_t(g.n[3]));
  const size_t lds = srows_lds_words<NV, S, LW>(R) * sizeof(W);
  if (adj)
    hipLaunchKernelGGL((staggered_rows_kernel<DEPTH, true, NV, S, T, LW>), grid, block, lds, st, g, tr, int(xcd),
                       (const W*)U, (const W*)in, (W*)out, T(mass));
  else
    hipLaunchKernelGGL((staggered_rows_kernel<DEPTH, false, NV, S, T, LW>), grid, block, lds, st, g, tr, int(xcd),
                       (const W*)U, (const W*)in, (W*)out, T(mass));
  return hipGetLastError();
}

// Row-staged D_S for N_v = 12 in C64 and C128.  Returns hipErrorNotSupported
// when the configuration is not covered (the caller then uses the direct
// kernel).  DSLASH_ROWS=0 disables it.
hipError_t launch_staggered_rows(bool adj, int dtype, const Geom& g, const void* U, const void* in, void* out,
                                 double mass, hipStream_t st, bool compressed) {
  if (const char* e = getenv("DSLASH_ROWS"))
    if (atoi(e) == 0) return hipErrorNotSupported;
  if (g.nv != 12 || (dtype != DT_C64 && dtype != DT_C128)) return hipErrorNotSupported;
  int R = row_sites_default(g.n[0], g.nv);
  if (const char* e = getenv("DSLASH_ROW_SITES")) R = atoi(e);
  if (R > g.n[0]) R = g.n[0];
  // R >= 11 also gives every thread at most one piece of the own row's halo
  // (2 sites of 3 N_v words) and one word of a row's backward links (9 n words)
  if (R < 1 || R * g.nv > 256 || R * g.nv < 128) return hipErrorNotSupported;
  int bt = 4;
  if (const char* e = getenv("DSLASH_TBAND")) bt = atoi(e);
  bool xcd = true;
  if (const char* e = getenv("DSLASH_XCD")) xcd = atoi(e) != 0;
  int depth = 3;
  if (const char* e = getenv("DSLASH_ROW_DEPTH")) depth = atoi(e);
  if (compressed) {
    if (dtype == DT_C64) return staggered_rows_t<3, 12, C64, float, 6>(adj, g, R, bt, xcd, U, in, out, mass, st);
    return staggered_rows_t<3, 12, C128, double, 6>(adj, g, R, bt, xcd, U, in, out, mass, st);
  }
  if (dtype == DT_C64) {
    if (depth <= 3) return staggered_rows_t<3, 12, C64, float, 9>(adj, g, R, bt, xcd, U, in, out, mass, st);
    return staggered_rows_t<7, 12, C64, float, 9>(adj, g, R, bt, xcd, U, in, out, mass, st);
  }
  if (depth <= 3) return staggered_rows_t<3, 12, C128, double, 9>(adj, g, R, bt, xcd, U, in, out, mass, st);
  return staggered_rows_t<7, 12, C128, double, 9>(adj, g, R, bt, xcd, U, in, out, mass, st);
}

}  // namespace dsl
