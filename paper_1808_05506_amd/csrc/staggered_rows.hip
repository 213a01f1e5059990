// Row-staged D_S (see rows.hpp).  staggered_march_kernel (the default) steps
// a workgroup through consecutive t of one x-row chunk (below);
// staggered_rows_kernel computes one output row per workgroup: a workgroup
// owns an x-row chunk of R sites
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
#include "tiles.hpp"

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
// Slots after the CH spinor pieces of a staged row: the ceil(9 / N_v) words of
// the backward links a thread moves (one word per slot), or, on the own row,
// one piece of the halo sites.
template <int NV>
constexpr int kSE = (9 + NV - 1) / NV;
template <int NV, class S>
using SRowBuf = SPiece<NV, S>[kSCH<NV, S> + kSE<NV>];

// Neighbour row (MU, SGN): lane (x, v) takes pieces j N_v + v of its site;
// for a backward row, slots CH .. carry the thread's words tid + i nth of the
// row's V_mu(x - mu) (clamped to the last).
template <int MU, int SGN, int NV, class S, int LW>
__device__ __forceinline__ void srow_issue(const Geom& g, const RowChunk& c, const typename S::word* __restrict__ U,
                                           const typename S::word* __restrict__ in, int xl, int v, int tid,
                                           SRowBuf<NV, S>& r) {
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
    constexpr int KW = (LW + NV - 1) / NV;
    const int nth = KW > 1 ? int(blockDim.x * blockDim.y) : 0;
    const int lim = c.n * LW - 1;
#pragma unroll
    for (int i = 0; i < KW; ++i) {
      const int q = tid + i * nth, w = q < lim ? q : lim;
      const int k = w / LW, e = w - k * LW;
      r[CH + i] = reinterpret_cast<const P*>(U)[(size_t(nrow + k) * 4 + MU) * LW + e];
    }
  }
}

template <int SGN, int NV, class S, int LW>
__device__ __forceinline__ void srow_commit(const RowChunk& c, const SRowBuf<NV, S>& r,
                                            typename S::word* row, typename S::word* lnb, int xl, int v, int tid) {
  using P = SPiece<NV, S>;
  constexpr int CH = kSCH<NV, S>, SSP = Stage<3, NV, S>::SSP;
  const int xc = xl < c.n ? xl : c.n - 1;
  P* dst = reinterpret_cast<P*>(row) + xc * SSP;
#pragma unroll
  for (int j = 0; j < CH; ++j) dst[j * NV + v] = r[j];
  if (SGN < 0) {
    constexpr int KW = (LW + NV - 1) / NV;
    const int nth = KW > 1 ? int(blockDim.x * blockDim.y) : 0;
    const int lim = c.n * LW - 1;
#pragma unroll
    for (int i = 0; i < KW; ++i) {
      const int q = tid + i * nth;
      reinterpret_cast<P*>(lnb)[q < lim ? q : lim] = r[CH + i];
    }
  }
}

// Own row: CH pieces of site x and, in slot CH, one piece of the halo sites
// x0 - 1, x0 + n (2 * 3 N_v words; the launcher checks there are enough threads).
template <int NV, class S>
__device__ __forceinline__ void sown_issue(const RowChunk& c, const typename S::word* __restrict__ in, int xm, int xp,
                                           int xl, int v, int tid, SRowBuf<NV, S>& r) {
  using P = SPiece<NV, S>;
  constexpr int SW = 3 * NV, CH = kSCH<NV, S>, SP = CH * NV;
  const int xc = xl < c.n ? xl : c.n - 1;
  const P* src = reinterpret_cast<const P*>(in + size_t(c.row_base + c.x0 + xc) * SW);
#pragma unroll
  for (int j = 0; j < CH; ++j) r[j] = src[j * NV + v];
  const int h = tid < 2 * SP ? tid : 2 * SP - 1;
  const int hs = h < SP ? xm : xp;
  r[CH] = reinterpret_cast<const P*>(in + size_t(c.row_base + hs) * SW)[h < SP ? h : h - SP];
#pragma unroll
  for (int i = 1; i < kSE<NV>; ++i) r[CH + i] = P{};
}

template <int NV, class S>
__device__ __forceinline__ void sown_commit(const RowChunk& c, const SRowBuf<NV, S>& r,
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

// Only the halo sites of the own row (its interior is already in LDS), in slot
// CH; the other slots are cleared so every call site writes the whole array.
template <int NV, class S>
__device__ __forceinline__ void sown_halo_issue(const RowChunk& c, const typename S::word* __restrict__ in, int xm,
                                                int xp, int tid, SRowBuf<NV, S>& r) {
  using P = SPiece<NV, S>;
  constexpr int SW = 3 * NV, CH = kSCH<NV, S>, SP = CH * NV;
#pragma unroll
  for (int j = 0; j < CH; ++j) r[j] = P{};
  const int h = tid < 2 * SP ? tid : 2 * SP - 1;
  const int hs = h < SP ? xm : xp;
  r[CH] = reinterpret_cast<const P*>(in + size_t(c.row_base + hs) * SW)[h < SP ? h : h - SP];
#pragma unroll
  for (int i = 1; i < kSE<NV>; ++i) r[CH + i] = P{};
}

template <int NV, class S>
__device__ __forceinline__ void sown_halo_commit(const RowChunk& c, const SRowBuf<NV, S>& r,
                                                 typename S::word* buf, int tid) {
  using P = SPiece<NV, S>;
  constexpr int CH = kSCH<NV, S>, SP = CH * NV, SSP = Stage<3, NV, S>::SSP;
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

  SRowBuf<NV, S> r0, r1, r2, r3, r4, r5, r6;
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

// ---------------------------------------------------------------- t-marching D_S
// A workgroup owns the x-row chunk at (y, z) for T consecutive t.  The -t hop
// of step t + 1, -eta_t V_t(x, t)^dag psi(x, t), is formed at step t from the
// own row in LDS and carried in registers (eta_t does not depend on t).  The
// +t row of a step is staged into the own-row buffer and is the next step's
// own row, so a later step stages the own row's two halo sites, +y, -y, +z,
// -z and +t; the first step also stages the whole own row and -t.  The
// neighbour rows pass through two buffers in turn (one barrier per row).
// LDS: bo [(R + 2) SSW], ba, bb [R SSW], lown [(R + 1) 4 LW], lnba, lnbb [R LW].

// Staged rows of a step: K = 0 +y, 1 -y, 2 +z, 3 -z, 4 +t, 5 -t, 6 own row,
// 7 the own row's halo sites.
//   first step: own, +y, -y, +z, -z, -t, +t     later steps: halo, +y, -y, +z, -z, +t
template <bool FIRST> struct SMarchSeq {
  static constexpr int N = FIRST ? 7 : 6;
  static constexpr int at(int p) {
    return p == 0 ? (FIRST ? 6 : 7) : (p <= 4 ? p - 1 : (FIRST ? (p == 5 ? 5 : 4) : 4));
  }
};

template <int K, int NV, class S, int LW>
__device__ __forceinline__ void smarch_issue(const Geom& g, const RowChunk& c, const typename S::word* __restrict__ U,
                                             const typename S::word* __restrict__ in, int xm, int xp, int xl, int v,
                                             int tid, SRowBuf<NV, S>& r0,
                                             SRowBuf<NV, S>& r1, SRowBuf<NV, S>& r2,
                                             SRowBuf<NV, S>& r3, SRowBuf<NV, S>& r4,
                                             SRowBuf<NV, S>& r5, SRowBuf<NV, S>& r6) {
  if constexpr (K == 0) srow_issue<1, +1, NV, S, LW>(g, c, U, in, xl, v, tid, r0);
  if constexpr (K == 1) srow_issue<1, -1, NV, S, LW>(g, c, U, in, xl, v, tid, r1);
  if constexpr (K == 2) srow_issue<2, +1, NV, S, LW>(g, c, U, in, xl, v, tid, r2);
  if constexpr (K == 3) srow_issue<2, -1, NV, S, LW>(g, c, U, in, xl, v, tid, r3);
  if constexpr (K == 4) srow_issue<3, +1, NV, S, LW>(g, c, U, in, xl, v, tid, r4);
  if constexpr (K == 5) srow_issue<3, -1, NV, S, LW>(g, c, U, in, xl, v, tid, r5);
  if constexpr (K == 6) sown_issue<NV, S>(c, in, xm, xp, xl, v, tid, r6);
  if constexpr (K == 7) sown_halo_issue<NV, S>(c, in, xm, xp, tid, r6);
}

// Links of the own row's sites x0 .. x0 + n - 1 (K 16-byte pieces per thread)
// and of the halo site x0 - 1 (one piece).
template <class S, int NV, int LW>
struct SLinks {
  static constexpr int LP = 4 * LW * int(sizeof(typename S::word)) / 16;  // pieces per site
  static constexpr int K = (LP + NV - 1) / NV;
};

template <class S, int NV, int LW>
__device__ __forceinline__ void slinks_issue(const RowChunk& c, const typename S::word* __restrict__ U, int xm,
                                             int tid, int nth, u32x4 (&lr)[SLinks<S, NV, LW>::K + 1]) {
  constexpr int LP = SLinks<S, NV, LW>::LP, K = SLinks<S, NV, LW>::K;
  const u32x4* own = reinterpret_cast<const u32x4*>(U + size_t(c.row_base + c.x0) * 4 * LW);
  const u32x4* halo = reinterpret_cast<const u32x4*>(U + size_t(c.row_base + xm) * 4 * LW);
  const int pieces = c.n * LP;
#pragma unroll
  for (int j = 0; j < K; ++j) {
    const int i = tid + j * nth;
    lr[j] = own[i < pieces ? i : pieces - 1];
  }
  lr[K] = halo[tid < LP ? tid : LP - 1];
}

template <class S, int NV, int LW>
__device__ __forceinline__ void slinks_commit(const RowChunk& c, const u32x4 (&lr)[SLinks<S, NV, LW>::K + 1],
                                              typename S::word* lown, int tid, int nth) {
  constexpr int LP = SLinks<S, NV, LW>::LP, K = SLinks<S, NV, LW>::K;
  u32x4* down = reinterpret_cast<u32x4*>(lown + 4 * LW);
  const int pieces = c.n * LP;
#pragma unroll
  for (int j = 0; j < K; ++j) {
    const int i = tid + j * nth;
    down[i < pieces ? i : pieces - 1] = lr[j];
  }
  reinterpret_cast<u32x4*>(lown)[tid < LP ? tid : LP - 1] = lr[K];
}

// carry = V_t(x)^dag psi(x) for the -t hop of the next step
template <int NV, class S, class T, int LW>
__device__ __forceinline__ void scarry(const cpx<T> (&p)[3], const typename S::word* link, cpx<T> (&carry)[3]) {
  cpx<T> u[3][3];
  load_link_lw<LW, S, T>(link, u);
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    cpx<T> t = zero<T>();
#pragma unroll
    for (int b = 0; b < 3; ++b) t = cjmadd(t, u[b][a], p[b]);
    carry[a] = t;
  }
}

template <bool FIRST, int DEPTH, bool ADJ, int NV, class S, class T, int LW>
__device__ __forceinline__ void smarch_step(const Geom& g, const RowChunk& c, const typename S::word* __restrict__ U,
                                            const typename S::word* __restrict__ in, typename S::word* __restrict__ out,
                                            typename S::word* bo, typename S::word* ba, typename S::word* bb,
                                            typename S::word* lown, typename S::word* lnba, typename S::word* lnbb,
                                            int xm, int xp, int xl, int v, int tid, int nth, T mass, T ey, T ez, T et,
                                            SRowBuf<NV, S>& r0, SRowBuf<NV, S>& r1,
                                            SRowBuf<NV, S>& r2, SRowBuf<NV, S>& r3,
                                            SRowBuf<NV, S>& r4, SRowBuf<NV, S>& r5,
                                            SRowBuf<NV, S>& r6,
                                            u32x4 (&lr)[SLinks<S, NV, LW>::K + 1], cpx<T> (&carry)[3]) {
  using W = typename S::word;
  using Q = SMarchSeq<FIRST>;
  constexpr int SW = 3 * NV, SSW = Stage<3, NV, S>::SSW;
#define DSL_SMI(P) smarch_issue<Q::at(P), NV, S, LW>(g, c, U, in, xm, xp, xl, v, tid, r0, r1, r2, r3, r4, r5, r6)
  if constexpr (!FIRST) {
    DSL_SMI(0);
    if constexpr (DEPTH > 1) DSL_SMI(1);
    if constexpr (DEPTH > 2) DSL_SMI(2);
    if constexpr (DEPTH > 3) DSL_SMI(3);
    slinks_issue<S, NV, LW>(c, U, xm, tid, nth, lr);
  }
  slinks_commit<S, NV, LW>(c, lr, lown, tid, nth);
  if constexpr (FIRST)
    sown_commit<NV, S>(c, r6, bo, xl, v, tid);
  else
    sown_halo_commit<NV, S>(c, r6, bo, tid);
  __syncthreads();
  if constexpr (DEPTH < Q::N) DSL_SMI(DEPTH);
  const int xc = xl < c.n ? xl : c.n - 1;
  cpx<T> acc[3] = {zero<T>(), zero<T>(), zero<T>()};
  cpx<T> self[3];
  lds_column<3, NV, S, T>(bo + (xc + 1) * SSW, v, self);
  if constexpr (!FIRST) {
#pragma unroll
    for (int a = 0; a < 3; ++a) acc[a] = rmadd(acc[a], -et, carry[a]);
  }
  scarry<NV, S, T, LW>(self, lown + (xc + 1) * 4 * LW + 3 * LW, carry);
  // x hops (eta_1 = 1): x + 1 at index xc + 2, x - 1 (and its link) at index xc
  shop<false, NV, S, T, LW>(bo + (xc + 2) * SSW, lown + (xc + 1) * 4 * LW, v, T(1), acc);
  shop<true, NV, S, T, LW>(bo + xc * SSW, lown + xc * 4 * LW, v, T(1), acc);
  srow_commit<+1, NV, S, LW>(c, r0, ba, lnba, xl, v, tid);
  __syncthreads();
#define DSL_SMSTEP(P, MU, SGN, BUF, LNB, ETA)                                                           \
  if constexpr (P + DEPTH < Q::N) DSL_SMI(P + DEPTH);                                                   \
  if constexpr (SGN > 0)                                                                                \
    shop<false, NV, S, T, LW>(BUF + xc * SSW, lown + (xc + 1) * 4 * LW + MU * LW, v, ETA, acc);         \
  else                                                                                                  \
    shop<true, NV, S, T, LW>(BUF + xc * SSW, LNB + xc * LW, v, ETA, acc);
#define DSL_SMCOMMIT(SGN, CUR, BUF, LNB)                   \
  srow_commit<SGN, NV, S, LW>(c, CUR, BUF, LNB, xl, v, tid); \
  __syncthreads();
  DSL_SMSTEP(1, 1, +1, ba, lnba, ey)
  DSL_SMCOMMIT(-1, r1, bb, lnbb)
  DSL_SMSTEP(2, 1, -1, bb, lnbb, ey)
  DSL_SMCOMMIT(+1, r2, ba, lnba)
  DSL_SMSTEP(3, 2, +1, ba, lnba, ez)
  DSL_SMCOMMIT(-1, r3, bb, lnbb)
  if constexpr (FIRST) {
    DSL_SMSTEP(4, 2, -1, bb, lnbb, ez)
    DSL_SMCOMMIT(-1, r5, ba, lnba)
    DSL_SMSTEP(5, 3, -1, ba, lnba, et)
    DSL_SMCOMMIT(+1, r4, bo + SSW, lnbb)
    DSL_SMSTEP(6, 3, +1, bo + SSW, lnbb, et)
  } else {
    DSL_SMSTEP(4, 2, -1, bb, lnbb, ez)
    DSL_SMCOMMIT(+1, r4, bo + SSW, lnba)
    DSL_SMSTEP(5, 3, +1, bo + SSW, lnba, et)
  }
#undef DSL_SMSTEP
#undef DSL_SMCOMMIT
#undef DSL_SMI
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
  // the next step rewrites lown and the own row's halo sites
  __syncthreads();
}

template <int NV, class S, int LW>
size_t smarch_lds_words(int R) {
  return size_t(3 * R + 2) * Stage<3, NV, S>::SSW + size_t(R + 1) * 4 * LW + size_t(2 * R) * LW;
}

// Waves per SIMD: FP32 four (about 100 VGPRs), FP64 two.
template <class S> struct SMarchWaves { static constexpr int value = sizeof(typename S::word) == 16 ? 2 : 4; };

template <int DEPTH, bool ADJ, int NV, class S, class T, int LW>
__global__ void __launch_bounds__(256, SMarchWaves<S>::value)
    staggered_march_kernel(Geom g, MarchTraversal m, MarchTiles o, int xcd, const typename S::word* __restrict__ U,
                           const typename S::word* __restrict__ in, typename S::word* __restrict__ out, T mass) {
  using W = typename S::word;
  using P = SPiece<NV, S>;
  constexpr int CH = kSCH<NV, S>, SSW = Stage<3, NV, S>::SSW;
  extern __shared__ uint4 smem_smarch[];
  const int R = int(m.sb);
  W* bo = reinterpret_cast<W*>(smem_smarch);
  W* ba = bo + (R + 2) * SSW;
  W* bb = ba + R * SSW;
  W* lown = bb + R * SSW;
  W* lnba = lown + (R + 1) * 4 * LW;
  W* lnbb = lnba + R * LW;

  const uint32_t L = xcd_block(blockIdx.x, gridDim.x, xcd != 0);
  uint32_t seg;
  const uint32_t id = march_order_id(g, m, o, L, seg);
  const int t0 = int(seg * m.T);
  const int steps = g.n[3] - t0 < int(m.T) ? g.n[3] - t0 : int(m.T);
  RowChunk c = march_chunk(g, m, id, t0);
  const int v = threadIdx.x, xl = threadIdx.y;
  const int tid = xl * NV + v, nth = R * NV;
  const int xm = wrap_x(g, c.x0 - 1), xp = wrap_x(g, c.x0 + c.n);
  // eta_mu(x) = (-1)^(x_1 + ... + x_{mu-1}) for the site of this lane
  const int x = c.x0 + xl;
  const T ey = (x & 1) ? T(-1) : T(1);
  const T ez = ((x + c.y) & 1) ? T(-1) : T(1);
  const T et = ((x + c.y + c.z) & 1) ? T(-1) : T(1);

  SRowBuf<NV, S> r0, r1, r2, r3, r4, r5, r6;
  u32x4 lr[SLinks<S, NV, LW>::K + 1];
  cpx<T> carry[3];
  using Q0 = SMarchSeq<true>;
#define DSL_SMP(P) smarch_issue<Q0::at(P), NV, S, LW>(g, c, U, in, xm, xp, xl, v, tid, r0, r1, r2, r3, r4, r5, r6)
  DSL_SMP(0);
  if constexpr (DEPTH > 1) DSL_SMP(1);
  if constexpr (DEPTH > 2) DSL_SMP(2);
  if constexpr (DEPTH > 3) DSL_SMP(3);
#undef DSL_SMP
  slinks_issue<S, NV, LW>(c, U, xm, tid, nth, lr);
  smarch_step<true, DEPTH, ADJ, NV, S, T, LW>(g, c, U, in, out, bo, ba, bb, lown, lnba, lnbb, xm, xp, xl, v, tid, nth,
                                              mass, ey, ez, et, r0, r1, r2, r3, r4, r5, r6, lr, carry);
#pragma nounroll
  for (int k = 1; k < steps; ++k) {
    c.t += 1;
    c.row_base += uint32_t(g.stride[3]);
    smarch_step<false, DEPTH, ADJ, NV, S, T, LW>(g, c, U, in, out, bo, ba, bb, lown, lnba, lnbb, xm, xp, xl, v, tid,
                                                 nth, mass, ey, ez, et, r0, r1, r2, r3, r4, r5, r6, lr, carry);
  }
}

template <int DEPTH, int NV, class S, class T, int LW>
static hipError_t staggered_march_t(bool adj, const Geom& g, int R, int tsteps, bool xcd, const void* U,
                                    const void* in, void* out, double mass, hipStream_t st) {
  using W = typename S::word;
  const MarchTraversal m = make_march_traversal(g, uint32_t(R), uint32_t(tsteps));
  const uint32_t nseg = (uint32_t(g.n[3]) + m.T - 1) / m.T;
  const dim3 block(NV, R), grid(m.rows * nseg);
  size_t lds = smarch_lds_words<NV, S, LW>(R) * sizeof(W);
  lds += size_t(knobs().row_lds_extra.get(0));
  int by, bz;
  march_tile_default(g, by, bz);
  const MarchTiles o = make_march_tiles(g, m.chunks, nseg, knobs().march_tile_y.get(by), knobs().march_tile_z.get(bz));
  if (adj)
    hipLaunchKernelGGL((staggered_march_kernel<DEPTH, true, NV, S, T, LW>), grid, block, lds, st, g, m, o, int(xcd),
                       (const W*)U, (const W*)in, (W*)out, T(mass));
  else
    hipLaunchKernelGGL((staggered_march_kernel<DEPTH, false, NV, S, T, LW>), grid, block, lds, st, g, m, o, int(xcd),
                       (const W*)U, (const W*)in, (W*)out, T(mass));
  return hipGetLastError();
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

// Other block sizes than N_v = 12 take the t-marching kernel with three rows
// in flight and full links.
template <int NV>
static hipError_t staggered_march_nv(bool adj, int dtype, const Geom& g, int R, int tsteps, bool xcd, const void* U,
                                     const void* in, void* out, double mass, hipStream_t st) {
  if (dtype == DT_C64) return staggered_march_t<3, NV, C64, float, 9>(adj, g, R, tsteps, xcd, U, in, out, mass, st);
  return staggered_march_t<3, NV, C128, double, 9>(adj, g, R, tsteps, xcd, U, in, out, mass, st);
}

// Row-staged D_S in C64 and C128 for N_v = 4, 8, 12, 16, 24.  Returns
// hipErrorNotSupported when the configuration is not covered (the caller then
// uses the direct kernel).  DSLASH_ROWS=0 disables it.
hipError_t launch_staggered_rows(bool adj, int dtype, const Geom& g, const void* U, const void* in, void* out,
                                 double mass, hipStream_t st, bool compressed) {
  if (knobs().rows.get(1) == 0) return hipErrorNotSupported;
  if (!aligned16(U) || !aligned16(in) || !aligned16(out)) return hipErrorNotSupported;
  const int nv = g.nv;
  if (nv != 4 && nv != 8 && nv != 12 && nv != 16 && nv != 24) return hipErrorNotSupported;
  if (dtype != DT_C64 && dtype != DT_C128) return hipErrorNotSupported;
  if (nv != 12 && compressed) return hipErrorNotSupported;
  int R = row_sites_default(g.n[0], nv);
  R = knobs().row_sites.get(R);
  if (R > g.n[0]) R = g.n[0];
  // 64 .. 256 threads; R >= 6 gives every thread at most one piece of the own
  // row's halo (2 sites of 3 N_v words); a row's backward links (9 n words)
  // take ceil(9 / N_v) words a thread
  if (R < 6 || R * nv > 256 || R * nv < 64) return hipErrorNotSupported;
  int bt = 4;
  bt = knobs().tband.get(bt);
  bool xcd = true;
  xcd = knobs().xcd.get(xcd) != 0;
  int depth = 3;
  depth = knobs().row_depth.get(depth);
  // DSLASH_TSTEPS: t steps per workgroup of the t-marching kernel (default 8;
  // 0 selects the kernel with one output row per workgroup)
  int tsteps = 8;
  tsteps = knobs().tsteps.get(tsteps);
  if (nv != 12) {
    if (tsteps <= 0) return hipErrorNotSupported;
    switch (nv) {
      case 4: return staggered_march_nv<4>(adj, dtype, g, R, tsteps, xcd, U, in, out, mass, st);
      case 8: return staggered_march_nv<8>(adj, dtype, g, R, tsteps, xcd, U, in, out, mass, st);
      case 16: return staggered_march_nv<16>(adj, dtype, g, R, tsteps, xcd, U, in, out, mass, st);
      case 24: return staggered_march_nv<24>(adj, dtype, g, R, tsteps, xcd, U, in, out, mass, st);
    }
    return hipErrorNotSupported;
  }
  if (tsteps > 0) {
#define DSL_SMT(D, LW)                                                                                          \
  return dtype == DT_C64 ? staggered_march_t<D, 12, C64, float, LW>(adj, g, R, tsteps, xcd, U, in, out, mass, st) \
                         : staggered_march_t<D, 12, C128, double, LW>(adj, g, R, tsteps, xcd, U, in, out, mass, st);
    if (compressed) {
      DSL_SMT(3, 6)
    }
    if (depth <= 2) {
      DSL_SMT(2, 9)
    }
    if (depth <= 3) {
      DSL_SMT(3, 9)
    }
    DSL_SMT(4, 9)
#undef DSL_SMT
  }
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
