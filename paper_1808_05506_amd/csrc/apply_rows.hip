// Row-staged D_W kernels (see rows.hpp): a workgroup owns an x-row chunk of
// R sites and all N_v right-hand sides; its inputs are copied into LDS with
// coalesced 16-byte loads, the hops are evaluated from LDS, and the outputs
// leave through LDS with coalesced 16-byte stores.  wilson_rows_kernel
// computes one output row per workgroup; wilson_march_kernel (the default)
// steps one workgroup through several consecutive t of the same (y, z).
#include <stdlib.h>

#include <type_traits>

#include "launch.hpp"
#include "rows.hpp"
#include "tiles.hpp"

namespace dsl {

// LDS layout, in storage words (one complex number each):
//   buf  [(R + 2) * 12 NV]  one staged row at index x - x0 + 1: a neighbour row
//                           fills 1 .. n, the chunk's own row 0 .. n + 1 (with
//                           the halo sites x0 - 1 and x0 + n); reused for the output
//   lown [(R + 1) * 36]     links of sites x0 - 1 .. x0 + n - 1 (index x - x0 + 1)
//   lnb  [R * 9]            V_mu of the backward neighbour row (current mu)
template <int NV, class S, int LW = 9>
size_t rows_lds_words(int R);

template <class S, class T, int NV>
DSL_HD void lds_spinor(const typename S::word* __restrict__ site, int v, cpx<T> (&p)[4][3]) {
#pragma unroll
  for (int sp = 0; sp < 4; ++sp)
#pragma unroll
    for (int c = 0; c < 3; ++c) p[sp][c] = S::template load<T>(site + (sp * 3 + c) * NV + v);
}

// acc += (1 + C gamma_MU) U' psi with psi and U' read from LDS
template <int MU, int C, bool DAG, int NV, class S, class T, int LW = 9>
__device__ __forceinline__ void lds_hop(const typename S::word* __restrict__ site,
                                       const typename S::word* __restrict__ link, int v, cpx<T> (&acc)[4][3]) {
  cpx<T> p[4][3];
  lds_spinor<S, T, NV>(site, v, p);
  cpx<T> h[2][3];
  project<MU, C, T>(p, h);
  cpx<T> u[3][3];
  if constexpr (LW == 9) {
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
      for (int b = 0; b < 3; ++b) u[a][b] = S::template load<T>(link + a * 3 + b);
  } else {
    load_link_lw<LW, S, T>(link, u);
  }
  cpx<T> t[2][3];
  su3_mul2<DAG, T>(u, h, t);
  reconstruct_add<MU, C, T>(acc, t);
}

// A storage word (4, 8 or 16 bytes) in the low bytes of a 16-byte register
// group and back, by value (a memcpy through a local can leave the group in
// scratch memory).
template <class W>
__device__ __forceinline__ u32x4 word_to_piece(W w) {
  if constexpr (sizeof(W) == 16) {
    return __builtin_bit_cast(u32x4, w);
  } else if constexpr (sizeof(W) == 8) {
    const u32x2 t = __builtin_bit_cast(u32x2, w);
    return u32x4{t.x, t.y, 0u, 0u};
  } else {
    return u32x4{__builtin_bit_cast(unsigned, w), 0u, 0u, 0u};
  }
}

template <class W>
__device__ __forceinline__ W piece_to_word(u32x4 z) {
  if constexpr (sizeof(W) == 16) {
    return __builtin_bit_cast(W, z);
  } else if constexpr (sizeof(W) == 8) {
    return __builtin_bit_cast(W, u32x2{z.x, z.y});
  } else {
    // 4-byte words are uint32_t pairs of 16-bit halves: a plain conversion
    // (a bit cast of a vector element is miscompiled by this compiler)
    static_assert(__is_same(W, uint32_t), "4-byte storage words are uint32_t");
    return z.x;
  }
}

// One thread's share of a neighbour row in flight: CH 16-byte pieces of the
// spinor run (pieces tid, tid + nth, ...) plus E more 16-byte register groups
// (so that the whole row is one array) for, on a backward hop, the thread's
// ceil(9 / N_v) words of the row's V_mu links, packed, or, on the own row, its
// pieces of the two halo sites.  The piece count per thread does not depend on
// R: a row chunk is R * 12 NV words and the workgroup has R * NV threads.
template <class S>
struct RowPieces {
  static constexpr int CH = 12 * int(sizeof(typename S::word)) / 16;
};

// E for N_v right-hand sides and wb-byte storage words.  The halo needs
// 2 * 12 N_v words in R N_v threads, 24 wb / (16 R) groups a thread: one at
// the R >= 16 that a workgroup of at most 256 threads holds up to N_v = 16,
// two for the R = 8 taken at larger N_v with 8-byte words.
DSL_HD constexpr int row_extra_groups(int nv, int wb) {
  const int links = (((9 + nv - 1) / nv) * wb + 15) / 16;
  const int halo = nv > 16 ? (24 * wb / 16 + 7) / 8 : 1;
  return links > halo ? links : halo;
}

template <int NV, class S>
struct RowRegs {
  static constexpr int CH = RowPieces<S>::CH;
  static constexpr int E = row_extra_groups(NV, int(sizeof(typename S::word)));
  static constexpr int N = CH + E;
};

template <int NV, class S>
using RowBuf = u32x4[RowRegs<NV, S>::N];

// Word i of the thread's link words (i = 0 .. KW - 1) in group i / PER of the
// extra groups, PER = 16 / word bytes words to a group, and back.
template <class W, int KW>
__device__ __forceinline__ u32x4 pack_words(const W (&w)[KW], int i0) {
  constexpr int WB = int(sizeof(W));
  if constexpr (WB == 16) {
    return i0 < KW ? __builtin_bit_cast(u32x4, w[i0]) : u32x4{0u, 0u, 0u, 0u};
  } else if constexpr (WB == 8) {
    const u32x2 a = i0 < KW ? __builtin_bit_cast(u32x2, w[i0]) : u32x2{0u, 0u};
    const u32x2 b = i0 + 1 < KW ? __builtin_bit_cast(u32x2, w[i0 + 1]) : u32x2{0u, 0u};
    return u32x4{a.x, a.y, b.x, b.y};
  } else {
    static_assert(__is_same(W, uint32_t), "4-byte storage words are uint32_t");
    return u32x4{i0 < KW ? w[i0] : 0u, i0 + 1 < KW ? w[i0 + 1] : 0u, i0 + 2 < KW ? w[i0 + 2] : 0u,
                 i0 + 3 < KW ? w[i0 + 3] : 0u};
  }
}

template <class W>
__device__ __forceinline__ W unpack_word(u32x4 z, int k) {
  constexpr int WB = int(sizeof(W));
  if constexpr (WB == 16) {
    return __builtin_bit_cast(W, z);
  } else if constexpr (WB == 8) {
    return __builtin_bit_cast(W, k == 0 ? u32x2{z.x, z.y} : u32x2{z.z, z.w});
  } else {
    return k == 0 ? z.x : (k == 1 ? z.y : (k == 2 ? z.z : z.w));
  }
}

// The backward hop's links V_mu(x - mu) of the chunk's n sites (LW words at
// stride 4 LW in U, from row site nrow): the thread's word i is word
// tid + i nth of the run, clamped to its last word.
template <int MU, int NV, class S, int LW>
__device__ __forceinline__ void lnb_issue(const typename S::word* __restrict__ U, uint32_t nrow, int n, int tid,
                                          RowBuf<NV, S>& r) {
  using W = typename S::word;
  constexpr int CH = RowRegs<NV, S>::CH, E = RowRegs<NV, S>::E;
  constexpr int KW = (LW + NV - 1) / NV, PER = 16 / int(sizeof(W));
  static_assert((KW + PER - 1) / PER <= E, "the link words fit the extra groups");
  const int nth = KW > 1 ? int(blockDim.x * blockDim.y) : 0;
  const int lim = n * LW - 1;
  W w[KW];
#pragma unroll
  for (int i = 0; i < KW; ++i) {
    const int q = tid + i * nth, wi = q < lim ? q : lim;
    const int k = wi / LW, e = wi - k * LW;
    w[i] = U[(size_t(nrow + k) * 4 + MU) * LW + e];
  }
#pragma unroll
  for (int s = 0; s < E; ++s) r[CH + s] = pack_words<W, KW>(w, s * PER);
}

template <int NV, class S, int LW>
__device__ __forceinline__ void lnb_commit(const RowBuf<NV, S>& r, typename S::word* lnb, int n,
                                           int tid) {
  using W = typename S::word;
  constexpr int CH = RowRegs<NV, S>::CH, KW = (LW + NV - 1) / NV, PER = 16 / int(sizeof(W));
  const int nth = KW > 1 ? int(blockDim.x * blockDim.y) : 0;
  const int lim = n * LW - 1;
#pragma unroll
  for (int i = 0; i < KW; ++i) {
    const int q = tid + i * nth;
    lnb[q < lim ? q : lim] = unpack_word<W>(r[CH + i / PER], i % PER);
  }
}

template <int NV, class S>
__device__ __forceinline__ void extra_clear(RowBuf<NV, S>& r) {
  constexpr int CH = RowRegs<NV, S>::CH, E = RowRegs<NV, S>::E;
#pragma unroll
  for (int s = 0; s < E; ++s) r[CH + s] = u32x4{0u, 0u, 0u, 0u};
}

// The own row's halo sites x0 - 1 (xm) and x0 + n (xp), SP pieces each: the
// thread's group s holds piece tid + s nth of the 2 SP, clamped to the last.
template <int NV, class S>
__device__ __forceinline__ void halo_issue(const RowChunk& c, const typename S::word* __restrict__ in, int xm, int xp,
                                           int tid, RowBuf<NV, S>& r) {
  constexpr int SW = 12 * NV, CH = RowRegs<NV, S>::CH, E = RowRegs<NV, S>::E;
  constexpr int SP = SW * int(sizeof(typename S::word)) / 16;
  const int nth = E > 1 ? int(blockDim.x * blockDim.y) : 0;
#pragma unroll
  for (int s = 0; s < E; ++s) {
    const int q = tid + s * nth, h = q < 2 * SP ? q : 2 * SP - 1;
    const int hs = h < SP ? xm : xp;
    r[CH + s] = reinterpret_cast<const u32x4*>(in + size_t(c.row_base + hs) * SW)[h < SP ? h : h - SP];
  }
}

template <int NV, class S>
__device__ __forceinline__ void halo_commit(const RowChunk& c, const RowBuf<NV, S>& r,
                                            typename S::word* buf, int tid) {
  constexpr int SW = 12 * NV, CH = RowRegs<NV, S>::CH, E = RowRegs<NV, S>::E;
  constexpr int SP = SW * int(sizeof(typename S::word)) / 16, SSP = SiteStride<NV, S>::PIECES;
  const int nth = E > 1 ? int(blockDim.x * blockDim.y) : 0;
#pragma unroll
  for (int s = 0; s < E; ++s) {
    const int q = tid + s * nth, h = q < 2 * SP ? q : 2 * SP - 1;
    u32x4* hdst = reinterpret_cast<u32x4*>(buf) + (h < SP ? 0 : (c.n + 1) * SSP);
    hdst[h < SP ? h : h - SP] = r[CH + s];
  }
}

template <int NV, class S, int LW>
size_t rows_lds_words(int R) {
  return size_t(R + 2) * SiteStride<NV, S>::WORDS + size_t(R + 1) * 4 * LW + size_t(R) * LW;
}

// Piece assignment of a staged row: lane (x, v) of the workgroup moves the
// pieces j * N_v + v (j = 0 .. CH - 1) of site x of the run, so the N_v lanes
// of a site read N_v consecutive 16-byte pieces per instruction and the LDS
// position follows from the site without a division.  Lanes past a partial
// chunk's end repeat the last site (same data to the same place).
template <int MU, int SGN, int NV, class S, int LW = 9>
__device__ __forceinline__ void row_issue(const Geom& g, const RowChunk& c, const typename S::word* __restrict__ U,
                                          const typename S::word* __restrict__ in, int xl, int v, int tid,
                                          RowBuf<NV, S>& r) {
  using W = typename S::word;
  constexpr int SW = 12 * NV, CH = RowPieces<S>::CH;
  const uint32_t nrow = row_base_shift(g, c, MU, SGN) + uint32_t(c.x0);
  const int xc = xl < c.n ? xl : c.n - 1;
  const u32x4* src = reinterpret_cast<const u32x4*>(in + size_t(nrow + xc) * SW);
#pragma unroll
  for (int j = 0; j < CH; ++j) r[j] = src[j * NV + v];
  if (SGN < 0) {
    lnb_issue<MU, NV, S, LW>(U, nrow, c.n, tid, r);
  } else {
    // every row writes the whole array, so that call sites merged into one
    // array store the same elements (the compiler's store sinking would
    // otherwise make the array addressable and put it in scratch memory)
    extra_clear<NV, S>(r);
  }
}

template <int SGN, int NV, class S, int LW = 9>
__device__ __forceinline__ void row_commit(const RowChunk& c, const RowBuf<NV, S>& r,
                                           typename S::word* row, typename S::word* lnb, int xl, int v, int tid) {
  using W = typename S::word;
  constexpr int CH = RowPieces<S>::CH, SSP = SiteStride<NV, S>::PIECES;
  const int xc = xl < c.n ? xl : c.n - 1;
  u32x4* dst = reinterpret_cast<u32x4*>(row) + xc * SSP;
#pragma unroll
  for (int j = 0; j < CH; ++j) dst[j * NV + v] = r[j];
  if (SGN < 0) lnb_commit<NV, S, LW>(r, lnb, c.n, tid);
}

// The chunk's own row in the same register shape: CH pieces of site x and,
// in the extra groups, the thread's pieces of the two halo sites x0 - 1, x0 + n
// (2 * 12 N_v words; the launcher checks that the groups of the workgroup
// hold them).
template <int NV, class S>
__device__ __forceinline__ void own_issue(const RowChunk& c, const typename S::word* __restrict__ in, int xm,
                                          int xp, int xl, int v, int tid, RowBuf<NV, S>& r) {
  using W = typename S::word;
  constexpr int SW = 12 * NV, CH = RowPieces<S>::CH;
  const int xc = xl < c.n ? xl : c.n - 1;
  const u32x4* src = reinterpret_cast<const u32x4*>(in + size_t(c.row_base + c.x0 + xc) * SW);
#pragma unroll
  for (int j = 0; j < CH; ++j) r[j] = src[j * NV + v];
  halo_issue<NV, S>(c, in, xm, xp, tid, r);
}

template <int NV, class S>
__device__ __forceinline__ void own_commit(const RowChunk& c, const RowBuf<NV, S>& r,
                                           typename S::word* buf, int xl, int v, int tid) {
  constexpr int CH = RowPieces<S>::CH, SSP = SiteStride<NV, S>::PIECES;
  const int xc = xl < c.n ? xl : c.n - 1;
  u32x4* dst = reinterpret_cast<u32x4*>(buf) + (xc + 1) * SSP;
#pragma unroll
  for (int j = 0; j < CH; ++j) dst[j * NV + v] = r[j];
  halo_commit<NV, S>(c, r, buf, tid);
}

// Only the halo sites x0 - 1, x0 + n of the own row (its interior is already
// in LDS), in the extra groups; the spinor slots are cleared so that every
// call site writes the whole register array.
template <int NV, class S>
__device__ __forceinline__ void own_halo_issue(const RowChunk& c, const typename S::word* __restrict__ in, int xm,
                                               int xp, int tid, RowBuf<NV, S>& r) {
  constexpr int CH = RowPieces<S>::CH;
#pragma unroll
  for (int j = 0; j < CH; ++j) r[j] = u32x4{0u, 0u, 0u, 0u};
  halo_issue<NV, S>(c, in, xm, xp, tid, r);
}

template <int NV, class S>
__device__ __forceinline__ void own_halo_commit(const RowChunk& c, const RowBuf<NV, S>& r,
                                                typename S::word* buf, int tid) {
  halo_commit<NV, S>(c, r, buf, tid);
}

template <int MU, int SGN, bool ADJ, int NV, class S, class T, int LW = 9>
__device__ __forceinline__ void row_compute(const typename S::word* nbr, const typename S::word* lown,
                                            const typename S::word* lnb, int xl, int v, cpx<T> (&acc)[4][3]) {
  constexpr int SSW = SiteStride<NV, S>::WORDS;
  if (SGN > 0)
    lds_hop<MU, (ADJ ? 1 : -1), false, NV, S, T, LW>(nbr + xl * SSW, lown + (xl + 1) * 4 * LW + MU * LW, v, acc);
  else
    lds_hop<MU, (ADJ ? -1 : 1), true, NV, S, T, LW>(nbr + xl * SSW, lnb + xl * LW, v, acc);
}

// ---------------------------------------------------------------- half-spinor
// rows (FP32 complex storage).  A hop reads its neighbour only through the
// projection (1 + C gamma_mu) psi, two spin components per colour (eq. def_wils
// with the chiral gamma matrices).  Lane (x, v) of a site loads, for the
// right-hand-side pair q = v mod N_v/2, the two spins that form half-spin
// component s = v div N_v/2 of that projection (spin s and its partner under
// gamma_mu) in all three colours, projects them, and writes the half spinor
// [s][c][N_v] of the site to LDS: half the LDS writes, reads and space of a full
// row.  The projection is the same sum as in project(), so the results are
// bit-identical to staging the full spinor.

// Partner of spin 0 under gamma_mu (spin 1's partner is 5 minus it).
template <int MU> struct HalfPartner { static constexpr int value = MU <= 1 ? 3 : 2; };

// Site stride of a half-spinor row in LDS, padded like SiteStride.
template <int NV, class S>
struct HalfStride {
  static constexpr int WB = int(sizeof(typename S::word));
  static constexpr int SWD = 6 * NV * WB / 4;
  static constexpr int WIN = NV * WB / 4;
  static constexpr int PAD = (((WIN - SWD) % 64) + 64) % 64;
  static constexpr int DW = (PAD <= SWD / 4 && (PAD * 4) % 16 == 0) ? SWD + PAD : SWD;
  static constexpr int WORDS = DW * 4 / WB;
  static constexpr int PIECES = DW * 4 / 16;
};

template <int MU, int SGN, int NV, class S, int LW = 9>
__device__ __forceinline__ void half_issue(const Geom& g, const RowChunk& c, const typename S::word* __restrict__ U,
                                           const typename S::word* __restrict__ in, int xl, int v, int tid,
                                           RowBuf<NV, S>& r) {
  static_assert(sizeof(typename S::word) == 8 && NV % 2 == 0 && RowPieces<S>::CH == 6,
                "half-spinor rows take FP32 complex storage and an even N_v");
  constexpr int SW = 12 * NV, HP = NV / 2, P0 = HalfPartner<MU>::value;
  const uint32_t nrow = row_base_shift(g, c, MU, SGN) + uint32_t(c.x0);
  const int xc = xl < c.n ? xl : c.n - 1;
  const u32x4* src = reinterpret_cast<const u32x4*>(in + size_t(nrow + xc) * SW);
  const int hs = v >= HP ? 1 : 0, q = v - hs * HP;
  const int sa = hs, sb = hs ? 5 - P0 : P0;
#pragma unroll
  for (int cc = 0; cc < 3; ++cc) {
    r[cc] = src[(sa * 3 + cc) * HP + q];
    r[3 + cc] = src[(sb * 3 + cc) * HP + q];
  }
  if (SGN < 0)
    lnb_issue<MU, NV, S, LW>(U, nrow, c.n, tid, r);
  else
    extra_clear<NV, S>(r);
}

template <int MU, int SGN, bool ADJ, int NV, class S, int LW = 9>
__device__ __forceinline__ void half_commit(const RowChunk& c, const RowBuf<NV, S>& r,
                                            typename S::word* hrow, typename S::word* lnb, int xl, int v, int tid) {
  using W = typename S::word;
  constexpr int HP = NV / 2, HSP = HalfStride<NV, S>::PIECES;
  constexpr int C = SGN > 0 ? (ADJ ? 1 : -1) : (ADJ ? -1 : 1);
  const int xc = xl < c.n ? xl : c.n - 1;
  const int hs = v >= HP ? 1 : 0, q = v - hs * HP;
  // h_s = psi_s + sg X(psi_partner), X = C i (MU = 0, 2) or C (MU = 1, 3)
  const float sg = MU == 0 ? -1.f : (MU == 3 ? 1.f : (hs ? 1.f : -1.f));
  u32x4* dst = reinterpret_cast<u32x4*>(hrow) + xc * HSP + hs * 3 * HP + q;
#pragma unroll
  for (int cc = 0; cc < 3; ++cc) {
    // whole-vector bit casts (a bit cast of a vector element is miscompiled)
    const f32x4 a = __builtin_bit_cast(f32x4, r[cc]), b = __builtin_bit_cast(f32x4, r[3 + cc]);
    f32x4 x;
    if constexpr (MU == 0 || MU == 2) {
      x = f32x4{float(-C) * b.y, float(C) * b.x, float(-C) * b.w, float(C) * b.z};
    } else {
      x = f32x4{float(C) * b.x, float(C) * b.y, float(C) * b.z, float(C) * b.w};
    }
    const f32x4 h = f32x4{a.x + sg * x.x, a.y + sg * x.y, a.z + sg * x.z, a.w + sg * x.w};
    dst[cc * HP] = __builtin_bit_cast(u32x4, h);
  }
  if (SGN < 0) lnb_commit<NV, S, LW>(r, lnb, c.n, tid);
}

template <int MU, int SGN, bool ADJ, int NV, class S, class T, int LW = 9>
__device__ __forceinline__ void half_compute(const typename S::word* hrow, const typename S::word* lown,
                                             const typename S::word* lnb, int xl, int v, cpx<T> (&acc)[4][3]) {
  constexpr int HSW = HalfStride<NV, S>::WORDS;
  constexpr int C = SGN > 0 ? (ADJ ? 1 : -1) : (ADJ ? -1 : 1);
  const typename S::word* site = hrow + xl * HSW;
  cpx<T> h[2][3];
#pragma unroll
  for (int hs = 0; hs < 2; ++hs)
#pragma unroll
    for (int cc = 0; cc < 3; ++cc) h[hs][cc] = S::template load<T>(site + (hs * 3 + cc) * NV + v);
  const typename S::word* link = SGN > 0 ? lown + (xl + 1) * 4 * LW + MU * LW : lnb + xl * LW;
  cpx<T> u[3][3];
  if constexpr (LW == 9) {
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
      for (int b = 0; b < 3; ++b) u[a][b] = S::template load<T>(link + a * 3 + b);
  } else {
    load_link_lw<LW, S, T>(link, u);
  }
  cpx<T> t[2][3];
  su3_mul2<(SGN < 0), T>(u, h, t);
  reconstruct_add<MU, C, T>(acc, t);
}

// Full or half-spinor staging of a neighbour row, by HALF.
template <bool HALF, int MU, int SGN, bool ADJ, int NV, class S, int LW>
__device__ __forceinline__ void o_commit(const RowChunk& c, const RowBuf<NV, S>& r,
                                         typename S::word* row, typename S::word* lnb, int xl, int v, int tid) {
  if constexpr (HALF)
    half_commit<MU, SGN, ADJ, NV, S, LW>(c, r, row, lnb, xl, v, tid);
  else
    row_commit<SGN, NV, S, LW>(c, r, row, lnb, xl, v, tid);
}

template <bool HALF, int MU, int SGN, bool ADJ, int NV, class S, class T, int LW>
__device__ __forceinline__ void o_compute(const typename S::word* row, const typename S::word* lown,
                                          const typename S::word* lnb, int xl, int v, cpx<T> (&acc)[4][3]) {
  if constexpr (HALF)
    half_compute<MU, SGN, ADJ, NV, S, T, LW>(row, lown, lnb, xl, v, acc);
  else
    row_compute<MU, SGN, ADJ, NV, S, T, LW>(row, lown, lnb, xl, v, acc);
}

// Occupancy hint per prefetch depth: deeper prefetch holds more rows in
// registers (about 28 VGPRs per FP32 row) and runs fewer waves per SIMD.
template <int DEPTH> struct RowsWaves { static constexpr int value = DEPTH <= 2 ? 4 : (DEPTH <= 4 ? 3 : 2); };

// CLOV: adds the site-local clover term C(x) in(x) (packed, 36 words per
// site, staged in LDS after lnb).
template <int DEPTH, bool ADJ, bool CLOV, int NV, class S, class T>
__global__ void __launch_bounds__(256, RowsWaves<DEPTH>::value)
    wilson_rows_kernel(Geom g, RowTraversal tr, ChunkTiles o, int xcd, const typename S::word* __restrict__ U,
                       const typename S::word* __restrict__ in, typename S::word* __restrict__ out,
                       const typename S::word* __restrict__ C, T diag) {
  using W = typename S::word;
  constexpr int SW = 12 * NV, CH = RowPieces<S>::CH;
  constexpr int SSW = SiteStride<NV, S>::WORDS, SSP = SiteStride<NV, S>::PIECES;
  extern __shared__ uint4 smem_rows[];
  const int R = int(tr.sb);
  W* buf = reinterpret_cast<W*>(smem_rows);
  W* lown = buf + (R + 2) * SSW;
  W* lnb = lown + (R + 1) * 36;
  W* lcl = lnb + ((R * 9 + 3) & ~3);  // [R][36] clover words of the chunk's sites (CLOV), 16-byte aligned

  const uint32_t L = xcd_block(blockIdx.x, gridDim.x, xcd != 0);
  const RowChunk c = order_chunk(g, tr, o, L);
  const int v = threadIdx.x, xl = threadIdx.y;
  const int tid = xl * NV + v, nth = R * NV;
  const int xm = wrap_x(g, c.x0 - 1), xp = wrap_x(g, c.x0 + c.n);

  // Seven rows pass through the one LDS row buffer: +y, -y, +z, -z, +t, -t,
  // then the chunk's own row with its halo sites.  Row k is requested DEPTH
  // steps before it is consumed (DEPTH = 7: all at once), each into its own
  // register array.
  constexpr int RN = RowRegs<NV, S>::N;
  u32x4 r0[RN], r1[RN], r2[RN], r3[RN], r4[RN], r5[RN], r6[RN];
#define DSL_ISSUE(K)                                                                   \
  do {                                                                                 \
    if constexpr (K == 0) row_issue<1, +1, NV, S>(g, c, U, in, xl, v, tid, r0);        \
    if constexpr (K == 1) row_issue<1, -1, NV, S>(g, c, U, in, xl, v, tid, r1);        \
    if constexpr (K == 2) row_issue<2, +1, NV, S>(g, c, U, in, xl, v, tid, r2);        \
    if constexpr (K == 3) row_issue<2, -1, NV, S>(g, c, U, in, xl, v, tid, r3);        \
    if constexpr (K == 4) row_issue<3, +1, NV, S>(g, c, U, in, xl, v, tid, r4);        \
    if constexpr (K == 5) row_issue<3, -1, NV, S>(g, c, U, in, xl, v, tid, r5);        \
    if constexpr (K == 6) own_issue<NV, S>(c, in, xm, xp, xl, v, tid, r6);             \
  } while (0)
  DSL_ISSUE(0);
  if constexpr (DEPTH > 1) DSL_ISSUE(1);
  if constexpr (DEPTH > 2) DSL_ISSUE(2);
  if constexpr (DEPTH > 3) DSL_ISSUE(3);
  if constexpr (DEPTH > 4) DSL_ISSUE(4);
  if constexpr (DEPTH > 5) DSL_ISSUE(5);
  if constexpr (DEPTH > 6) DSL_ISSUE(6);
  // links of the chunk's sites and of the halo site x0 - 1: a site's links
  // are LINK_PIECES 16-byte pieces, so the R N_v threads move ceil(LINK_PIECES /
  // N_v) pieces each (the halo site's, one piece each)
  constexpr int LINK_PIECES = 36 * int(sizeof(W)) / 16, LK = (LINK_PIECES + NV - 1) / NV;
  copy_pieces<LK>(lown + 36, U + size_t(c.row_base + c.x0) * 36, c.n * LINK_PIECES, tid, nth);
  copy_pieces<1>(lown, U + size_t(c.row_base + xm) * 36, LINK_PIECES, tid, nth);
  if constexpr (CLOV) copy_pieces<LK>(lcl, C + size_t(c.row_base + c.x0) * 36, c.n * LINK_PIECES, tid, nth);

  cpx<T> acc[4][3];
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 3; ++b) acc[a][b] = zero<T>();

  // Lanes past a partial chunk's end (xl >= n) compute on stale but in-bounds
  // LDS data and their results are never copied out; keeping every lane on
  // the same straight-line path lets the compiler keep the prefetches in
  // flight across the hops.
  W* const row = buf + SSW;  // neighbour rows sit at index 1 .. n
#define DSL_ROW_STEP(K, MU, SGN, CUR)                                         \
  row_commit<SGN, NV, S>(c, CUR, row, lnb, xl, v, tid);                       \
  __syncthreads();                                                            \
  if constexpr (K + DEPTH < 7) DSL_ISSUE(K + DEPTH);                          \
  row_compute<MU, SGN, ADJ, NV, S, T>(row, lown, lnb, xl, v, acc);            \
  __syncthreads();
  DSL_ROW_STEP(0, 1, +1, r0)
  DSL_ROW_STEP(1, 1, -1, r1)
  DSL_ROW_STEP(2, 2, +1, r2)
  DSL_ROW_STEP(3, 2, -1, r3)
  DSL_ROW_STEP(4, 3, +1, r4)
  DSL_ROW_STEP(5, 3, -1, r5)
#undef DSL_ROW_STEP
#undef DSL_ISSUE

  own_commit<NV, S>(c, r6, buf, xl, v, tid);
  __syncthreads();
  cpx<T> res[4][3];
  {
    constexpr int CF = ADJ ? +1 : -1, CB = -CF;
    // x hops from the own row: x + 1 at index xl + 2, x - 1 (and its link) at index xl
    lds_hop<0, CF, false, NV, S, T>(buf + (xl + 2) * SSW, lown + (xl + 1) * 36, v, acc);
    lds_hop<0, CB, true, NV, S, T>(buf + xl * SSW, lown + xl * 36, v, acc);
    const W* self = buf + (xl + 1) * SSW;
    if constexpr (CLOV) {
      cpx<T> p[4][3];
      lds_spinor<S, T, NV>(self, v, p);
#pragma unroll
      for (int sp = 0; sp < 4; ++sp)
#pragma unroll
        for (int cc = 0; cc < 3; ++cc) {
          res[sp][cc].r = fma(diag, p[sp][cc].r, T(-0.5) * acc[sp][cc].r);
          res[sp][cc].i = fma(diag, p[sp][cc].i, T(-0.5) * acc[sp][cc].i);
        }
      clover_madd<S, T>(lcl + xl * 36, p, res);
    } else {
#pragma unroll
      for (int sp = 0; sp < 4; ++sp)
#pragma unroll
        for (int cc = 0; cc < 3; ++cc) {
          cpx<T> p = S::template load<T>(self + (sp * 3 + cc) * NV + v);
          res[sp][cc].r = fma(diag, p.r, T(-0.5) * acc[sp][cc].r);
          res[sp][cc].i = fma(diag, p.i, T(-0.5) * acc[sp][cc].i);
        }
    }
  }
  __syncthreads();
  {
    W* o = buf + xl * SSW;
#pragma unroll
    for (int sp = 0; sp < 4; ++sp)
#pragma unroll
      for (int cc = 0; cc < 3; ++cc) S::template store<T>(o + (sp * 3 + cc) * NV + v, res[sp][cc]);
  }
  __syncthreads();
  {
    // copy-out with the same site-local piece assignment as the staging
    const int xc = xl < c.n ? xl : c.n - 1;
    const u32x4* src = reinterpret_cast<const u32x4*>(buf) + xc * SSP;
    u32x4* dst = reinterpret_cast<u32x4*>(out + size_t(c.row_base + c.x0 + xc) * SW);
    u32x4 r[CH];
#pragma unroll
    for (int j = 0; j < CH; ++j) r[j] = src[j * NV + v];
    // outputs are never read again by this kernel: stream them past the L2
    // so its capacity stays with the input rows that neighbours reuse
#pragma unroll
    for (int j = 0; j < CH; ++j) __builtin_nontemporal_store(r[j], &dst[j * NV + v]);
  }
}

// ---------------------------------------------------------------- t-marching variant
// A workgroup owns the x-row chunk at (y, z) for T consecutive t and steps
// through them.  The -t hop of step t + 1 is U_t(x, t)^dag (1 -/+ gamma_t) psi(x, t),
// formed at step t from the own row already in LDS (a carry of one half
// spinor per lane), so after the first step only six rows are staged per
// output row: +y, -y, +z, -z, +t and the own row, and the +t row of one step
// is the own row of the next, read again while it is still in L2.
// (MarchTraversal, make_march_traversal and march_chunk are in rows.hpp.)

// Row K of a step's sequence (0 +y, 1 -y, 2 +z, 3 -z, 4 +t, 5 -t, 6 own, 7 the
// own row's halo sites only) into its register array.
template <int K, int NV, class S, int LW = 9>
__device__ __forceinline__ void march_issue(const Geom& g, const RowChunk& c, const typename S::word* __restrict__ U,
                                            const typename S::word* __restrict__ in, int xm, int xp, int xl, int v,
                                            int tid, RowBuf<NV, S>& r0,
                                            RowBuf<NV, S>& r1, RowBuf<NV, S>& r2,
                                            RowBuf<NV, S>& r3, RowBuf<NV, S>& r4,
                                            RowBuf<NV, S>& r5, RowBuf<NV, S>& r6) {
  if constexpr (K == 0) row_issue<1, +1, NV, S, LW>(g, c, U, in, xl, v, tid, r0);
  if constexpr (K == 1) row_issue<1, -1, NV, S, LW>(g, c, U, in, xl, v, tid, r1);
  if constexpr (K == 2) row_issue<2, +1, NV, S, LW>(g, c, U, in, xl, v, tid, r2);
  if constexpr (K == 3) row_issue<2, -1, NV, S, LW>(g, c, U, in, xl, v, tid, r3);
  if constexpr (K == 4) row_issue<3, +1, NV, S, LW>(g, c, U, in, xl, v, tid, r4);
  if constexpr (K == 5) row_issue<3, -1, NV, S, LW>(g, c, U, in, xl, v, tid, r5);
  if constexpr (K == 6) own_issue<NV, S>(c, in, xm, xp, xl, v, tid, r6);
  if constexpr (K == 7) own_halo_issue<NV, S>(c, in, xm, xp, tid, r6);
}

// march_issue with the neighbour rows (K = 0 .. 3 and 5) as half spinors.
template <bool HALF, int K, int NV, class S, int LW = 9>
__device__ __forceinline__ void march_issue_o(const Geom& g, const RowChunk& c, const typename S::word* __restrict__ U,
                                              const typename S::word* __restrict__ in, int xm, int xp, int xl, int v,
                                              int tid, RowBuf<NV, S>& r0,
                                              RowBuf<NV, S>& r1, RowBuf<NV, S>& r2,
                                              RowBuf<NV, S>& r3, RowBuf<NV, S>& r4,
                                              RowBuf<NV, S>& r5, RowBuf<NV, S>& r6) {
  if constexpr (HALF && K == 0) half_issue<1, +1, NV, S, LW>(g, c, U, in, xl, v, tid, r0);
  else if constexpr (HALF && K == 1) half_issue<1, -1, NV, S, LW>(g, c, U, in, xl, v, tid, r1);
  else if constexpr (HALF && K == 2) half_issue<2, +1, NV, S, LW>(g, c, U, in, xl, v, tid, r2);
  else if constexpr (HALF && K == 3) half_issue<2, -1, NV, S, LW>(g, c, U, in, xl, v, tid, r3);
  else if constexpr (HALF && K == 5) half_issue<3, -1, NV, S, LW>(g, c, U, in, xl, v, tid, r5);
  else march_issue<K, NV, S, LW>(g, c, U, in, xm, xp, xl, v, tid, r0, r1, r2, r3, r4, r5, r6);
}

// Sequence of staged rows in a step: all seven in the first step of a
// workgroup, without the -t row (K = 5) afterwards.
template <bool FIRST> struct MarchSeq {
  static constexpr int N = FIRST ? 7 : 6;
  static constexpr int at(int p) { return FIRST ? p : (p < 5 ? p : 6); }
};

// Sequence of the own-buffer step: the own row first and the +t row last, into
// the same buffer, so the +t row of step t is the own row of step t + 1 and a
// later step stages only its two halo sites (K = 7).
//   first step: own, +y, -y, +z, -z, -t, +t     later steps: halo, +y, -y, +z, -z, +t
template <bool FIRST> struct MarchSeqO {
  static constexpr int N = FIRST ? 7 : 6;
  static constexpr int at(int p) {
    return p == 0 ? (FIRST ? 6 : 7) : (p <= 4 ? p - 1 : (FIRST ? (p == 5 ? 5 : 4) : 4));
  }
};

// Links of sites x0 - 1 .. x0 + n - 1 of a row (36 words each): up to 3
// 16-byte pieces per thread for the chunk, one for the halo site.
template <class S, int LW = 9>
struct LinkPieces {
  static constexpr int PER_SITE = 4 * LW * int(sizeof(typename S::word)) / 16;
};

// Pieces of the chunk's links per thread: ceil(LP / threads per site).
template <class S, int THREADS_PER_SITE, int LW = 9>
struct LinkK {
  static constexpr int value = (LinkPieces<S, LW>::PER_SITE + THREADS_PER_SITE - 1) / THREADS_PER_SITE;
};

template <class S, int K, int LW = 9>
__device__ __forceinline__ void links_issue(const RowChunk& c, const typename S::word* __restrict__ U, int xm, int tid,
                                            int nth, u32x4 (&lr)[K + 1]) {
  constexpr int LP = LinkPieces<S, LW>::PER_SITE;
  const u32x4* own = reinterpret_cast<const u32x4*>(U + size_t(c.row_base + c.x0) * 4 * LW);
  const int pieces = c.n * LP;
#pragma unroll
  for (int j = 0; j < K; ++j) {
    const int i = tid + j * nth;
    lr[j] = own[i < pieces ? i : pieces - 1];
  }
  const u32x4* halo = reinterpret_cast<const u32x4*>(U + size_t(c.row_base + xm) * 4 * LW);
  lr[K] = halo[tid < LP ? tid : LP - 1];
}

template <class S, int K, int LW = 9>
__device__ __forceinline__ void links_commit(const RowChunk& c, const u32x4 (&lr)[K + 1], typename S::word* lown,
                                             int tid, int nth) {
  constexpr int LP = LinkPieces<S, LW>::PER_SITE;
  u32x4* own = reinterpret_cast<u32x4*>(lown + 4 * LW);
  const int pieces = c.n * LP;
#pragma unroll
  for (int j = 0; j < K; ++j) {
    const int i = tid + j * nth;
    own[i < pieces ? i : pieces - 1] = lr[j];
  }
  reinterpret_cast<u32x4*>(lown)[tid < LP ? tid : LP - 1] = lr[K];
}

template <class T>
__device__ __forceinline__ void hold_acc(cpx<T> (&acc)[4][3]) {
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 3; ++b) hold(acc[a][b]);
}

// Two or three rows in flight fit the 168 VGPRs of three waves per SIMD.
template <int DEPTH> struct MarchWaves { static constexpr int value = DEPTH <= 3 ? 3 : 2; };

template <bool FIRST, int DEPTH, bool ADJ, int NV, class S, class T, int LW, int EPI = EPI_STORE>
__device__ __forceinline__ void march_step(const Geom& g, const RowChunk& c,
                                           const typename S::word* __restrict__ U,
                                           const typename S::word* __restrict__ in, typename S::word* __restrict__ out,
                                           typename S::word* buf, typename S::word* lown, typename S::word* lnb,
                                           int xm, int xp, int xl, int v, int tid, int nth, T diag,
                                           RowBuf<NV, S>& r0, RowBuf<NV, S>& r1,
                                           RowBuf<NV, S>& r2, RowBuf<NV, S>& r3,
                                           RowBuf<NV, S>& r4, RowBuf<NV, S>& r5,
                                           RowBuf<NV, S>& r6, u32x4 (&lr)[LinkK<S, NV, LW>::value + 1],
                                           cpx<T> (&carry)[2][3], EpiLane<S>& ep) {
  using W = typename S::word;
  using Q = MarchSeq<FIRST>;
  constexpr int LK = LinkK<S, NV, LW>::value;
  constexpr int SW = 12 * NV, CH = RowPieces<S>::CH;
  constexpr int SSW = SiteStride<NV, S>::WORDS, SSP = SiteStride<NV, S>::PIECES;
  constexpr int CF = ADJ ? +1 : -1, CB = -CF;
  // the first step's leading rows and links were requested by the caller; a
  // later step requests them here, after the previous step's last barrier
  if constexpr (!FIRST) {
#define DSL_SISSUE(P) march_issue<Q::at(P), NV, S, LW>(g, c, U, in, xm, xp, xl, v, tid, r0, r1, r2, r3, r4, r5, r6)
    DSL_SISSUE(0);
    if constexpr (DEPTH > 1) DSL_SISSUE(1);
    if constexpr (DEPTH > 2) DSL_SISSUE(2);
    if constexpr (DEPTH > 3) DSL_SISSUE(3);
    if constexpr (DEPTH > 4) DSL_SISSUE(4);
    if constexpr (DEPTH > 5) DSL_SISSUE(5);
#undef DSL_SISSUE
    links_issue<S, LK, LW>(c, U, xm, tid, nth, lr);
  }
  links_commit<S, LK, LW>(c, lr, lown, tid, nth);

  cpx<T> acc[4][3];
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 3; ++b) acc[a][b] = zero<T>();

  W* const row = buf + SSW;
#define DSL_MISSUE(P, CH_)                                                                             \
  march_issue<Q::at(P), NV, S, LW>(g, CH_, U, in, xm, xp, xl, v, tid, r0, r1, r2, r3, r4, r5, r6)
#define DSL_MSTEP(P, MU, SGN, CUR)                                        \
  if constexpr (P < Q::N - 1) {                                           \
    row_commit<SGN, NV, S, LW>(c, CUR, row, lnb, xl, v, tid);                 \
    __syncthreads();                                                      \
    if constexpr (P + DEPTH < Q::N) DSL_MISSUE(P + DEPTH, c);             \
    row_compute<MU, SGN, ADJ, NV, S, T, LW>(row, lown, lnb, xl, v, acc);      \
    hold_acc<T>(acc);                                                     \
    __syncthreads();                                                      \
  }
  DSL_MSTEP(0, 1, +1, r0)
  DSL_MSTEP(1, 1, -1, r1)
  DSL_MSTEP(2, 2, +1, r2)
  DSL_MSTEP(3, 2, -1, r3)
  DSL_MSTEP(4, 3, +1, r4)
  DSL_MSTEP(5, 3, -1, r5)
#undef DSL_MSTEP

  own_commit<NV, S>(c, r6, buf, xl, v, tid);
  __syncthreads();
#undef DSL_MISSUE
  cpx<T> res[4][3];
  {
    lds_hop<0, CF, false, NV, S, T, LW>(buf + (xl + 2) * SSW, lown + (xl + 1) * 4 * LW, v, acc);
    lds_hop<0, CB, true, NV, S, T, LW>(buf + xl * SSW, lown + xl * 4 * LW, v, acc);
    if constexpr (!FIRST) reconstruct_add<3, CB, T>(acc, carry);
    const W* self = buf + (xl + 1) * SSW;
    cpx<T> p[4][3];
    lds_spinor<S, T, NV>(self, v, p);
#pragma unroll
    for (int sp = 0; sp < 4; ++sp)
#pragma unroll
      for (int cc = 0; cc < 3; ++cc) {
        res[sp][cc].r = fma(diag, p[sp][cc].r, T(-0.5) * acc[sp][cc].r);
        res[sp][cc].i = fma(diag, p[sp][cc].i, T(-0.5) * acc[sp][cc].i);
      }
    // carry for the next step: U_t(x, t)^dag (1 + CB gamma_t) psi(x, t), projected
    cpx<T> h[2][3];
    project<3, CB, T>(p, h);
    cpx<T> u[3][3];
    load_link_lw<LW, S, T>(lown + (xl + 1) * 4 * LW + 3 * LW, u);
    su3_mul2<true, T>(u, h, carry);
  }
  __syncthreads();
  {
    W* o = buf + xl * SSW;
#pragma unroll
    for (int sp = 0; sp < 4; ++sp)
#pragma unroll
      for (int cc = 0; cc < 3; ++cc) S::template store<T>(o + (sp * 3 + cc) * NV + v, res[sp][cc]);
  }
  __syncthreads();
  {
    const int xc = xl < c.n ? xl : c.n - 1;
    const u32x4* src = reinterpret_cast<const u32x4*>(buf) + xc * SSP;
    u32x4* dst = reinterpret_cast<u32x4*>(out + size_t(c.row_base + c.x0 + xc) * SW);
    epi_copy_out<EPI, NV, S, CH>(src, dst, v, xl < c.n, ep);
  }
  __syncthreads();
}

// The same step with two row buffers used in turn: row k + 1 is written to
// one buffer while row k is applied from the other, so each staged row costs
// one barrier instead of two.  LDS: buf0, buf1 [(R + 2) SSW], lown, lnb0, lnb1.
template <bool FIRST, int DEPTH, bool ADJ, int NV, class S, class T, int LW, int EPI = EPI_STORE>
__device__ __forceinline__ void march_step_pp(const Geom& g, const RowChunk& c,
                                              const typename S::word* __restrict__ U,
                                              const typename S::word* __restrict__ in,
                                              typename S::word* __restrict__ out, typename S::word* buf0,
                                              typename S::word* buf1, typename S::word* lown, typename S::word* lnb0,
                                              typename S::word* lnb1, int xm, int xp, int xl, int v, int tid, int nth,
                                              T diag, RowBuf<NV, S>& r0,
                                              RowBuf<NV, S>& r1, RowBuf<NV, S>& r2,
                                              RowBuf<NV, S>& r3, RowBuf<NV, S>& r4,
                                              RowBuf<NV, S>& r5, RowBuf<NV, S>& r6,
                                              u32x4 (&lr)[LinkK<S, NV, LW>::value + 1], cpx<T> (&carry)[2][3], EpiLane<S>& ep) {
  using W = typename S::word;
  using Q = MarchSeq<FIRST>;
  constexpr int LK = LinkK<S, NV, LW>::value;
  constexpr int SW = 12 * NV, CH = RowPieces<S>::CH;
  constexpr int SSW = SiteStride<NV, S>::WORDS, SSP = SiteStride<NV, S>::PIECES;
  constexpr int CF = ADJ ? +1 : -1, CB = -CF;
  if constexpr (!FIRST) {
#define DSL_SISSUE(P) march_issue<Q::at(P), NV, S, LW>(g, c, U, in, xm, xp, xl, v, tid, r0, r1, r2, r3, r4, r5, r6)
    DSL_SISSUE(0);
    if constexpr (DEPTH > 1) DSL_SISSUE(1);
    if constexpr (DEPTH > 2) DSL_SISSUE(2);
#undef DSL_SISSUE
    links_issue<S, LK, LW>(c, U, xm, tid, nth, lr);
  }
  links_commit<S, LK, LW>(c, lr, lown, tid, nth);

  cpx<T> acc[4][3];
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 3; ++b) acc[a][b] = zero<T>();

#define DSL_MISSUE(P) march_issue<Q::at(P), NV, S, LW>(g, c, U, in, xm, xp, xl, v, tid, r0, r1, r2, r3, r4, r5, r6)
  // row P of the sequence goes to buffer P % 2
#define DSL_BUF(P) ((P) % 2 == 0 ? buf0 : buf1)
#define DSL_LNB(P) ((P) % 2 == 0 ? lnb0 : lnb1)
#define DSL_COMMIT(P, SGN, CUR) row_commit<SGN, NV, S, LW>(c, CUR, DSL_BUF(P) + SSW, DSL_LNB(P), xl, v, tid)
  DSL_COMMIT(0, +1, r0);
  __syncthreads();
  // P: the row applied now; then P + 1 is written into the other buffer
#define DSL_PSTEP(P, MU, SGN, NSGN, NCUR)                                             \
  if constexpr (P + DEPTH < Q::N) DSL_MISSUE(P + DEPTH);                              \
  row_compute<MU, SGN, ADJ, NV, S, T, LW>(DSL_BUF(P) + SSW, lown, DSL_LNB(P), xl, v, acc); \
  hold_acc<T>(acc);                                                                   \
  if constexpr (P + 1 < Q::N - 1) DSL_COMMIT(P + 1, NSGN, NCUR);                      \
  if constexpr (P + 1 == Q::N - 1) own_commit<NV, S>(c, r6, DSL_BUF(P + 1), xl, v, tid); \
  __syncthreads();
  if constexpr (FIRST) {
    DSL_PSTEP(0, 1, +1, -1, r1)
    DSL_PSTEP(1, 1, -1, +1, r2)
    DSL_PSTEP(2, 2, +1, -1, r3)
    DSL_PSTEP(3, 2, -1, +1, r4)
    DSL_PSTEP(4, 3, +1, -1, r5)
    DSL_PSTEP(5, 3, -1, +1, r0)
  } else {
    DSL_PSTEP(0, 1, +1, -1, r1)
    DSL_PSTEP(1, 1, -1, +1, r2)
    DSL_PSTEP(2, 2, +1, -1, r3)
    DSL_PSTEP(3, 2, -1, +1, r4)
    DSL_PSTEP(4, 3, +1, +1, r0)
  }
#undef DSL_PSTEP
#undef DSL_COMMIT
#undef DSL_MISSUE
  W* const own = DSL_BUF(Q::N - 1);
#undef DSL_BUF
#undef DSL_LNB
  cpx<T> res[4][3];
  {
    lds_hop<0, CF, false, NV, S, T, LW>(own + (xl + 2) * SSW, lown + (xl + 1) * 4 * LW, v, acc);
    lds_hop<0, CB, true, NV, S, T, LW>(own + xl * SSW, lown + xl * 4 * LW, v, acc);
    if constexpr (!FIRST) reconstruct_add<3, CB, T>(acc, carry);
    cpx<T> p[4][3];
    lds_spinor<S, T, NV>(own + (xl + 1) * SSW, v, p);
#pragma unroll
    for (int sp = 0; sp < 4; ++sp)
#pragma unroll
      for (int cc = 0; cc < 3; ++cc) {
        res[sp][cc].r = fma(diag, p[sp][cc].r, T(-0.5) * acc[sp][cc].r);
        res[sp][cc].i = fma(diag, p[sp][cc].i, T(-0.5) * acc[sp][cc].i);
      }
    cpx<T> h[2][3];
    project<3, CB, T>(p, h);
    cpx<T> u[3][3];
    load_link_lw<LW, S, T>(lown + (xl + 1) * 4 * LW + 3 * LW, u);
    su3_mul2<true, T>(u, h, carry);
  }
  // the output leaves through the other buffer (free since the last barrier)
  W* const ob = own == buf0 ? buf1 : buf0;
  {
    W* o = ob + xl * SSW;
#pragma unroll
    for (int sp = 0; sp < 4; ++sp)
#pragma unroll
      for (int cc = 0; cc < 3; ++cc) S::template store<T>(o + (sp * 3 + cc) * NV + v, res[sp][cc]);
  }
  __syncthreads();
  {
    const int xc = xl < c.n ? xl : c.n - 1;
    const u32x4* src = reinterpret_cast<const u32x4*>(ob) + xc * SSP;
    u32x4* dst = reinterpret_cast<u32x4*>(out + size_t(c.row_base + c.x0 + xc) * SW);
    epi_copy_out<EPI, NV, S, CH>(src, dst, v, xl < c.n, ep);
  }
  __syncthreads();
}

// The step with three buffers: bo holds the own row (with its halo sites)
// and receives the +t row at the end of the step, which is then the next
// step's own row; ba and bb take the other rows in turn (one barrier per staged
// row) and the output.  The diagonal term is folded into acc as -2 diag psi at
// the start, since the own row is gone from bo when the output is formed.
// LDS: bo [(R + 2) SSW], ba, bb [R SSW], lown, lnba, lnbb [R LW].
// HALF: the +-y, +-z and first -t rows go through ba and bb as half spinors
// (ba, bb [R HSW], adjacent), and the output through ba and bb together.
template <bool FIRST, int DEPTH, bool ADJ, int NV, class S, class T, int LW, bool HALF = false, int EPI = EPI_STORE>
__device__ __forceinline__ void march_step_o(const Geom& g, const RowChunk& c, const typename S::word* __restrict__ U,
                                             const typename S::word* __restrict__ in,
                                             typename S::word* __restrict__ out, typename S::word* bo,
                                             typename S::word* ba, typename S::word* bb, typename S::word* lown,
                                             typename S::word* lnba, typename S::word* lnbb, int xm, int xp, int xl,
                                             int v, int tid, int nth, T diag, RowBuf<NV, S>& r0,
                                             RowBuf<NV, S>& r1, RowBuf<NV, S>& r2,
                                             RowBuf<NV, S>& r3, RowBuf<NV, S>& r4,
                                             RowBuf<NV, S>& r5, RowBuf<NV, S>& r6,
                                             u32x4 (&lr)[LinkK<S, NV, LW>::value + 1], cpx<T> (&carry)[2][3], EpiLane<S>& ep) {
  using W = typename S::word;
  using Q = MarchSeqO<FIRST>;
  constexpr int LK = LinkK<S, NV, LW>::value;
  constexpr int SW = 12 * NV, CH = RowPieces<S>::CH;
  constexpr int SSW = SiteStride<NV, S>::WORDS, SSP = SiteStride<NV, S>::PIECES;
  constexpr int CF = ADJ ? +1 : -1, CB = -CF;
#define DSL_OISSUE(P) \
  march_issue_o<HALF, Q::at(P), NV, S, LW>(g, c, U, in, xm, xp, xl, v, tid, r0, r1, r2, r3, r4, r5, r6)
  if constexpr (!FIRST) {
    DSL_OISSUE(0);
    if constexpr (DEPTH > 1) DSL_OISSUE(1);
    if constexpr (DEPTH > 2) DSL_OISSUE(2);
    links_issue<S, LK, LW>(c, U, xm, tid, nth, lr);
  }
  links_commit<S, LK, LW>(c, lr, lown, tid, nth);
  if constexpr (FIRST)
    own_commit<NV, S>(c, r6, bo, xl, v, tid);
  else
    own_halo_commit<NV, S>(c, r6, bo, tid);
  __syncthreads();
  if constexpr (DEPTH < Q::N) DSL_OISSUE(DEPTH);
  cpx<T> acc[4][3];
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 3; ++b) acc[a][b] = zero<T>();
  {
    if constexpr (!FIRST) reconstruct_add<3, CB, T>(acc, carry);
    cpx<T> p[4][3];
    lds_spinor<S, T, NV>(bo + (xl + 1) * SSW, v, p);
    const T m2d = T(-2) * diag;
#pragma unroll
    for (int sp = 0; sp < 4; ++sp)
#pragma unroll
      for (int cc = 0; cc < 3; ++cc) acc[sp][cc] = rmadd(acc[sp][cc], m2d, p[sp][cc]);
    // carry for the next step: U_t(x, t)^dag (1 + CB gamma_t) psi(x, t), projected
    cpx<T> h[2][3];
    project<3, CB, T>(p, h);
    cpx<T> u[3][3];
    load_link_lw<LW, S, T>(lown + (xl + 1) * 4 * LW + 3 * LW, u);
    su3_mul2<true, T>(u, h, carry);
  }
  hold_acc<T>(acc);
  lds_hop<0, CF, false, NV, S, T, LW>(bo + (xl + 2) * SSW, lown + (xl + 1) * 4 * LW, v, acc);
  lds_hop<0, CB, true, NV, S, T, LW>(bo + xl * SSW, lown + xl * 4 * LW, v, acc);
  hold_acc<T>(acc);
  o_commit<HALF, 1, +1, ADJ, NV, S, LW>(c, r0, ba, lnba, xl, v, tid);
  __syncthreads();
  // row P (in buffer BUF) applied, then row P + 1 written to NBUF
#define DSL_OSTEP(P, MU, SGN, H, BUF, LNB)                                     \
  if constexpr (P + DEPTH < Q::N) DSL_OISSUE(P + DEPTH);                       \
  o_compute<H, MU, SGN, ADJ, NV, S, T, LW>(BUF, lown, LNB, xl, v, acc);        \
  hold_acc<T>(acc);
#define DSL_OCOMMIT(MU, SGN, H, CUR, BUF, LNB)                  \
  o_commit<H, MU, SGN, ADJ, NV, S, LW>(c, CUR, BUF, LNB, xl, v, tid); \
  __syncthreads();
  DSL_OSTEP(1, 1, +1, HALF, ba, lnba)
  DSL_OCOMMIT(1, -1, HALF, r1, bb, lnbb)
  DSL_OSTEP(2, 1, -1, HALF, bb, lnbb)
  DSL_OCOMMIT(2, +1, HALF, r2, ba, lnba)
  DSL_OSTEP(3, 2, +1, HALF, ba, lnba)
  DSL_OCOMMIT(2, -1, HALF, r3, bb, lnbb)
  W* ob;
  if constexpr (FIRST) {
    DSL_OSTEP(4, 2, -1, HALF, bb, lnbb)
    DSL_OCOMMIT(3, -1, HALF, r5, ba, lnba)
    DSL_OSTEP(5, 3, -1, HALF, ba, lnba)
    DSL_OCOMMIT(3, +1, false, r4, bo + SSW, lnbb)
    DSL_OSTEP(6, 3, +1, false, bo + SSW, lnbb)
    ob = HALF ? ba : bb;
  } else {
    DSL_OSTEP(4, 2, -1, HALF, bb, lnbb)
    DSL_OCOMMIT(3, +1, false, r4, bo + SSW, lnba)
    DSL_OSTEP(5, 3, +1, false, bo + SSW, lnba)
    ob = ba;
  }
#undef DSL_OSTEP
#undef DSL_OCOMMIT
#undef DSL_OISSUE
  // out = diag psi - 1/2 (hops) = -1/2 acc, through a free buffer (HALF: ba
  // and bb together, with a site stride of 12 N_v + 4 words where that fits,
  // 12 N_v otherwise)
  constexpr int OSW = HALF ? (12 * NV + 4 <= 2 * HalfStride<NV, S>::WORDS ? 12 * NV + 4 : 12 * NV) : SSW;
  constexpr int OSP = OSW * int(sizeof(W)) / 16;
  static_assert(!HALF || OSW <= 2 * HalfStride<NV, S>::WORDS, "the output fits ba and bb");
  {
    W* o = ob + xl * OSW;
#pragma unroll
    for (int sp = 0; sp < 4; ++sp)
#pragma unroll
      for (int cc = 0; cc < 3; ++cc) {
        cpx<T> r;
        r.r = T(-0.5) * acc[sp][cc].r;
        r.i = T(-0.5) * acc[sp][cc].i;
        S::template store<T>(o + (sp * 3 + cc) * NV + v, r);
      }
  }
  __syncthreads();
  {
    const int xc = xl < c.n ? xl : c.n - 1;
    const u32x4* src = reinterpret_cast<const u32x4*>(ob) + xc * OSP;
    u32x4* dst = reinterpret_cast<u32x4*>(out + size_t(c.row_base + c.x0 + xc) * SW);
    epi_copy_out<EPI, NV, S, CH>(src, dst, v, xl < c.n, ep);
  }
  __syncthreads();
}

// PP: 0 the one-buffer step (march_step), 1 two buffers in turn
// (march_step_pp), 2 an own-row buffer plus two in turn (march_step_o), 3 the
// same with half-spinor neighbour rows (FP32 storage).
template <int PP, int DEPTH> struct MarchOcc { static constexpr int value = PP ? 2 : MarchWaves<DEPTH>::value; };

template <int DEPTH, bool ADJ, int NV, class S, class T, int LW, int PP = 0, int EPI = EPI_STORE>
__global__ void __launch_bounds__(256, (MarchOcc<PP, DEPTH>::value))
    wilson_march_kernel(Geom g, MarchTraversal m, MarchTiles o, int xcd, const typename S::word* __restrict__ U,
                        const typename S::word* __restrict__ in, typename S::word* __restrict__ out, T diag,
                        EpiArgs ea) {
  using W = typename S::word;
  constexpr int CH = RowPieces<S>::CH, LK = LinkK<S, NV, LW>::value;
  constexpr int SSW = SiteStride<NV, S>::WORDS;
  extern __shared__ uint4 smem_march[];
  const int R = int(m.sb);
  W* buf = reinterpret_cast<W*>(smem_march);
  constexpr int BSW = PP == 3 ? HalfStride<NV, S>::WORDS : SSW;  // ba, bb site stride
  W* buf1 = buf + (R + 2) * SSW;  // PP 1: the second buffer; PP 2, 3: ba
  W* buf2 = buf1 + R * BSW;       // PP 2, 3: bb
  W* lown = PP == 1 ? buf1 + (R + 2) * SSW : (PP >= 2 ? buf2 + R * BSW : buf + (R + 2) * SSW);
  W* lnb = lown + (R + 1) * 4 * LW;
  W* lnb1 = lnb + R * LW;  // PP only

  const uint32_t L = xcd_block(blockIdx.x, gridDim.x, xcd != 0);
  uint32_t seg;
  const uint32_t id = march_order_id(g, m, o, L, seg);
  const int t0 = int(seg * m.T);
  const int steps = g.n[3] - t0 < int(m.T) ? g.n[3] - t0 : int(m.T);
  RowChunk c = march_chunk(g, m, id, t0);
  const int v = threadIdx.x, xl = threadIdx.y;
  const int tid = xl * NV + v, nth = R * NV;
  const int xm = wrap_x(g, c.x0 - 1), xp = wrap_x(g, c.x0 + c.n);

  constexpr int RN = RowRegs<NV, S>::N;
  u32x4 r0[RN], r1[RN], r2[RN], r3[RN], r4[RN], r5[RN], r6[RN];
  u32x4 lr[LK + 1];
  cpx<T> carry[2][3];
  EpiLane<S> ep;
  ep.template init<NV>(ea, v, EPI == EPI_AXPY);
  using Q0 = typename std::conditional<PP >= 2, MarchSeqO<true>, MarchSeq<true>>::type;
#define DSL_PISSUE(P) \
  march_issue_o<PP == 3, Q0::at(P), NV, S, LW>(g, c, U, in, xm, xp, xl, v, tid, r0, r1, r2, r3, r4, r5, r6)
  DSL_PISSUE(0);
  if constexpr (DEPTH > 1) DSL_PISSUE(1);
  if constexpr (DEPTH > 2) DSL_PISSUE(2);
  if constexpr (DEPTH > 3) DSL_PISSUE(3);
  if constexpr (DEPTH > 4) DSL_PISSUE(4);
#undef DSL_PISSUE
  links_issue<S, LK, LW>(c, U, xm, tid, nth, lr);
  if constexpr (PP >= 2)
    march_step_o<true, DEPTH, ADJ, NV, S, T, LW, PP == 3, EPI>(g, c, U, in, out, buf, buf1, buf2, lown, lnb, lnb1, xm,
                                                               xp, xl, v, tid, nth, diag, r0, r1, r2, r3, r4, r5, r6,
                                                               lr, carry, ep);
  else if constexpr (PP == 1)
    march_step_pp<true, DEPTH, ADJ, NV, S, T, LW, EPI>(g, c, U, in, out, buf, buf1, lown, lnb, lnb1, xm, xp, xl, v,
                                                       tid, nth, diag, r0, r1, r2, r3, r4, r5, r6, lr, carry, ep);
  else
    march_step<true, DEPTH, ADJ, NV, S, T, LW, EPI>(g, c, U, in, out, buf, lown, lnb, xm, xp, xl, v, tid, nth, diag,
                                                    r0, r1, r2, r3, r4, r5, r6, lr, carry, ep);
#pragma nounroll
  for (int k = 1; k < steps; ++k) {
    c.t += 1;
    c.row_base += uint32_t(g.stride[3]);
    if constexpr (PP >= 2)
      march_step_o<false, DEPTH, ADJ, NV, S, T, LW, PP == 3, EPI>(g, c, U, in, out, buf, buf1, buf2, lown, lnb, lnb1,
                                                                  xm, xp, xl, v, tid, nth, diag, r0, r1, r2, r3, r4, r5,
                                                                  r6, lr, carry, ep);
    else if constexpr (PP == 1)
      march_step_pp<false, DEPTH, ADJ, NV, S, T, LW, EPI>(g, c, U, in, out, buf, buf1, lown, lnb, lnb1, xm, xp, xl,
                                                          v, tid, nth, diag, r0, r1, r2, r3, r4, r5, r6, lr, carry, ep);
    else
      march_step<false, DEPTH, ADJ, NV, S, T, LW, EPI>(g, c, U, in, out, buf, lown, lnb, xm, xp, xl, v, tid, nth,
                                                       diag, r0, r1, r2, r3, r4, r5, r6, lr, carry, ep);
  }
  epi_finish<EPI, NV, S>(ea, ep, reinterpret_cast<double*>(smem_march), xl, v, R);
}

// The fused epilogues are built for the solver's two forms only (D with
// EPI_NORM, D^dag with EPI_AXPY), on N_v = 12, full links and the default
// prefetch depth of each buffer scheme.
template <int PP, int DEPTH, int LW, int NV>
struct MarchEpiBuilt {
  static constexpr bool value = NV == 12 && LW == 9 && DEPTH == (PP == 3 ? 3 : 2);
};

template <int DEPTH, int NV, class S, class T, int LW, int PP>
static hipError_t march_launch(bool adj, int epi, dim3 grid, dim3 block, size_t lds, hipStream_t st, const Geom& g,
                               const MarchTraversal& m, const MarchTiles& o, bool xcd, const void* U, const void* in,
                               void* out, T diag, const EpiArgs& ea) {
  using W = typename S::word;
#define DSL_MK(A, E)                                                                                              \
  hipLaunchKernelGGL((wilson_march_kernel<DEPTH, A, NV, S, T, LW, PP, E>), grid, block, lds, st, g, m, o, int(xcd), \
                     (const W*)U, (const W*)in, (W*)out, diag, ea)
  if (epi == EPI_STORE) {
    if (adj) DSL_MK(true, EPI_STORE); else DSL_MK(false, EPI_STORE);
  } else if constexpr (MarchEpiBuilt<PP, DEPTH, LW, NV>::value) {
    if (epi == EPI_NORM && !adj) DSL_MK(false, EPI_NORM);
    else if (epi == EPI_AXPY && adj) DSL_MK(true, EPI_AXPY);
    else return hipErrorNotSupported;
  } else {
    return hipErrorNotSupported;
  }
#undef DSL_MK
  return hipGetLastError();
}

// Compute units of the current device (cached per device).
static int device_cus() {
  static int cus[64] = {0};
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return 256;
  if (cus[dev] == 0) {
    int n = 0;
    if (hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || n <= 0) n = 256;
    cus[dev] = n;
  }
  return cus[dev];
}

// ONLY_PP >= 0 builds that buffer scheme only (pp must equal it).
template <int DEPTH, int NV, class S, class T, int LW = 9, int ONLY_PP = -1>
static hipError_t wilson_march_t(bool adj, const Geom& g, int R, int tsteps, int pp, bool xcd, const void* U,
                                 const void* in, void* out, double mass, hipStream_t st, int epi, EpiArgs& ea) {
  if (ONLY_PP >= 0 && pp != ONLY_PP) return hipErrorInvalidValue;
  using W = typename S::word;
  const MarchTraversal m = make_march_traversal(g, uint32_t(R), uint32_t(tsteps));
  const uint32_t nseg = (uint32_t(g.n[3]) + m.T - 1) / m.T;
  const dim3 block(NV, R), grid(m.rows * nseg);
  if (epi != EPI_STORE && grid.x > ea.capacity) return hipErrorNotSupported;
  ea.blocks = grid.x;
  size_t lds = rows_lds_words<NV, S, LW>(R) * sizeof(W);
  if (pp == 1) lds += (size_t(R + 2) * SiteStride<NV, S>::WORDS + size_t(R) * LW) * sizeof(W);
  if (pp == 2) lds += (size_t(2 * R) * SiteStride<NV, S>::WORDS + size_t(R) * LW) * sizeof(W);
  if (pp == 3) lds += (size_t(2 * R) * HalfStride<NV, S>::WORDS + size_t(R) * LW) * sizeof(W);
  lds += size_t(knobs().row_lds_extra.get(0));
  const T diag = T(4) + T(mass);
  // Tiles of (y, z) rows, one per XCD, when the grid runs in more than one
  // round (more than two workgroups per CU); a grid resident at once keeps
  // the plane order.  DSLASH_WMARCH_TILE_Y, _Z override (0: plane order).
  int by = 0, bz = 0;
  if (grid.x > 2u * uint32_t(device_cus())) march_tile_default(g, by, bz);
  const MarchTiles o =
      make_march_tiles(g, m.chunks, nseg, knobs().wmarch_tile_y.get(by), knobs().wmarch_tile_z.get(bz));
  if constexpr (ONLY_PP >= 0) {
    if constexpr (ONLY_PP == 3 && !(sizeof(W) == 8 && NV % 2 == 0)) return hipErrorInvalidValue;
    else return march_launch<DEPTH, NV, S, T, LW, ONLY_PP>(adj, epi, grid, block, lds, st, g, m, o, xcd, U, in, out, diag, ea);
  } else {
    switch (pp) {
      case 3:
        if constexpr (sizeof(W) == 8 && NV % 2 == 0)
          return march_launch<DEPTH, NV, S, T, LW, 3>(adj, epi, grid, block, lds, st, g, m, o, xcd, U, in, out, diag, ea);
        else
          return hipErrorInvalidValue;
      case 2: return march_launch<DEPTH, NV, S, T, LW, 2>(adj, epi, grid, block, lds, st, g, m, o, xcd, U, in, out, diag, ea);
      case 1: return march_launch<DEPTH, NV, S, T, LW, 1>(adj, epi, grid, block, lds, st, g, m, o, xcd, U, in, out, diag, ea);
      default: return march_launch<DEPTH, NV, S, T, LW, 0>(adj, epi, grid, block, lds, st, g, m, o, xcd, U, in, out, diag, ea);
    }
  }
}

// ---------------------------------------------------------------- even-odd hop
// out = c_add add + c_hop H in on the packed sites of parity p (even-odd form
// of D_W, see eo.hip), staged like wilson_rows_kernel on the packed geometry
// (Nx/2 sites per row): the y, z, t neighbours of packed site i sit at packed
// index i of the neighbour rows of `in`; the x neighbours are in the same row
// of `in` at i + r (x + 1) and i - 1 + r (x - 1), r = (p + y + z + t) mod 2.
// Forward links come from Uo (parity p), backward ones from Ui (parity 1 - p).
template <int DEPTH, bool ADJ, int NV, class S, class T, int EPI = EPI_STORE>
__global__ void __launch_bounds__(256, RowsWaves<DEPTH>::value)
    wilson_eo_rows_kernel(Geom g, RowTraversal tr, ChunkTiles o, int xcd, int p, const typename S::word* __restrict__ Uo,
                          const typename S::word* __restrict__ Ui, const typename S::word* __restrict__ in,
                          typename S::word* __restrict__ out, const typename S::word* __restrict__ add, T c_add,
                          T c_hop, EpiArgs ea) {
  using W = typename S::word;
  constexpr int SW = 12 * NV, CH = RowPieces<S>::CH;
  constexpr int SSW = SiteStride<NV, S>::WORDS, SSP = SiteStride<NV, S>::PIECES;
  extern __shared__ uint4 smem_eo[];
  const int R = int(tr.sb);
  W* buf = reinterpret_cast<W*>(smem_eo);
  W* lown = buf + (R + 2) * SSW;  // [R + 1][36], index x - x0 + 1
  W* lnb = lown + (R + 1) * 36;   // [R][9]
  W* lxb = lnb + R * 9;           // [R][9]: V_x(x - 1) from Ui

  const uint32_t L = xcd_block(blockIdx.x, gridDim.x, xcd != 0);
  const RowChunk c = order_chunk(g, tr, o, L);
  const int v = threadIdx.x, xl = threadIdx.y;
  const int tid = xl * NV + v, nth = R * NV;
  const int xm = wrap_x(g, c.x0 - 1), xp = wrap_x(g, c.x0 + c.n);
  const int r = (p + c.y + c.z + c.t) & 1;

  constexpr int RN = RowRegs<NV, S>::N;
  u32x4 r0[RN], r1[RN], r2[RN], r3[RN], r4[RN], r5[RN], r6[RN];
#define DSL_ISSUE(K)                                                                   \
  do {                                                                                 \
    if constexpr (K == 0) row_issue<1, +1, NV, S>(g, c, Ui, in, xl, v, tid, r0);       \
    if constexpr (K == 1) row_issue<1, -1, NV, S>(g, c, Ui, in, xl, v, tid, r1);       \
    if constexpr (K == 2) row_issue<2, +1, NV, S>(g, c, Ui, in, xl, v, tid, r2);       \
    if constexpr (K == 3) row_issue<2, -1, NV, S>(g, c, Ui, in, xl, v, tid, r3);       \
    if constexpr (K == 4) row_issue<3, +1, NV, S>(g, c, Ui, in, xl, v, tid, r4);       \
    if constexpr (K == 5) row_issue<3, -1, NV, S>(g, c, Ui, in, xl, v, tid, r5);       \
    if constexpr (K == 6) own_issue<NV, S>(c, in, xm, xp, xl, v, tid, r6);             \
  } while (0)
  DSL_ISSUE(0);
  if constexpr (DEPTH > 1) DSL_ISSUE(1);
  if constexpr (DEPTH > 2) DSL_ISSUE(2);
  if constexpr (DEPTH > 3) DSL_ISSUE(3);
  if constexpr (DEPTH > 4) DSL_ISSUE(4);
  if constexpr (DEPTH > 5) DSL_ISSUE(5);
  if constexpr (DEPTH > 6) DSL_ISSUE(6);
  {
    // links of the chunk's own sites (forward hops) and V_x(x - 1) of the x - 1
    // neighbours, which live in the other parity's row
    constexpr int LINK_PIECES = 36 * int(sizeof(W)) / 16, LK = (LINK_PIECES + NV - 1) / NV;
    copy_pieces<LK>(lown + 36, Uo + size_t(c.row_base + c.x0) * 36, c.n * LINK_PIECES, tid, nth);
    constexpr int KX = (9 + NV - 1) / NV;  // words of V_x(x - 1) per thread
#pragma unroll
    for (int i = 0; i < KX; ++i) {
      const int q = tid + i * nth, w = q < c.n * 9 ? q : c.n * 9 - 1;
      const int k = w / 9, e = w - k * 9;
      lxb[w] = Ui[size_t(c.row_base + wrap_x(g, c.x0 + k - 1 + r)) * 36 + e];
    }
  }

  cpx<T> acc[4][3];
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 3; ++b) acc[a][b] = zero<T>();

  W* const row = buf + SSW;
#define DSL_ROW_STEP(K, MU, SGN, CUR)                                         \
  row_commit<SGN, NV, S>(c, CUR, row, lnb, xl, v, tid);                       \
  __syncthreads();                                                            \
  if constexpr (K + DEPTH < 7) DSL_ISSUE(K + DEPTH);                          \
  row_compute<MU, SGN, ADJ, NV, S, T>(row, lown, lnb, xl, v, acc);            \
  hold_acc<T>(acc);                                                           \
  __syncthreads();
  DSL_ROW_STEP(0, 1, +1, r0)
  DSL_ROW_STEP(1, 1, -1, r1)
  DSL_ROW_STEP(2, 2, +1, r2)
  DSL_ROW_STEP(3, 2, -1, r3)
  DSL_ROW_STEP(4, 3, +1, r4)
  DSL_ROW_STEP(5, 3, -1, r5)
#undef DSL_ROW_STEP
#undef DSL_ISSUE

  own_commit<NV, S>(c, r6, buf, xl, v, tid);
  __syncthreads();
  cpx<T> res[4][3];
  {
    constexpr int CF = ADJ ? +1 : -1, CB = -CF;
    // x + 1 at packed i + r (buffer index xl + 1 + r), x - 1 at i - 1 + r
    lds_hop<0, CF, false, NV, S, T>(buf + (xl + 1 + r) * SSW, lown + (xl + 1) * 36, v, acc);
    lds_hop<0, CB, true, NV, S, T>(buf + (xl + r) * SSW, lxb + xl * 9, v, acc);
    const T ch = T(-0.5) * c_hop;
    const int xc = xl < c.n ? xl : c.n - 1;
    const W* a = add + size_t(c.row_base + c.x0 + xc) * SW + v;
#pragma unroll
    for (int sp = 0; sp < 4; ++sp)
#pragma unroll
      for (int cc = 0; cc < 3; ++cc) {
        res[sp][cc].r = ch * acc[sp][cc].r;
        res[sp][cc].i = ch * acc[sp][cc].i;
        if (add) {
          const cpx<T> q = S::template load<T>(a + (sp * 3 + cc) * NV);
          res[sp][cc].r = fma(c_add, q.r, res[sp][cc].r);
          res[sp][cc].i = fma(c_add, q.i, res[sp][cc].i);
        }
      }
  }
  __syncthreads();
  {
    W* o = buf + xl * SSW;
#pragma unroll
    for (int sp = 0; sp < 4; ++sp)
#pragma unroll
      for (int cc = 0; cc < 3; ++cc) S::template store<T>(o + (sp * 3 + cc) * NV + v, res[sp][cc]);
  }
  __syncthreads();
  {
    const int xc = xl < c.n ? xl : c.n - 1;
    const u32x4* src = reinterpret_cast<const u32x4*>(buf) + xc * SSP;
    u32x4* dst = reinterpret_cast<u32x4*>(out + size_t(c.row_base + c.x0 + xc) * SW);
    EpiLane<S> ep;
    ep.template init<NV>(ea, v, EPI == EPI_AXPY);
    epi_copy_out<EPI, NV, S, CH>(src, dst, v, xl < c.n, ep);
    epi_finish<EPI, NV, S>(ea, ep, reinterpret_cast<double*>(smem_eo), xl, v, R);
  }
}

// Chunk tiles of the one-row D_W kernels: the largest by x bz rows (by | Ny,
// bz | Nz) whose spinor rows at one t take at most 1.25 MB, the squarer of
// equal sizes, by >= bz on a tie; DSLASH_ROWS_TILE_Y, _Z override (0: t-band
// order).  The even-odd hop on 32^3 x 64 (N_v = 12, 8 x 8 tiles) took 890
// against 948 us in FP32 and 547 against 557 us in BF16; the kernel with the
// clover term on 16^3 x 32 took 102 against 99 us and keeps the t-band order
// (tiled = false).
static ChunkTiles rows_tiles(const Geom& g, int R, long site_bytes, bool tiled) {
  int by, bz;
  pick_tile(g, long((g.n[0] + R - 1) / R) * R * site_bytes, tiled ? 1280L * 1024 : 0, by, bz);
  return make_chunk_tiles(g, R, knobs().rows_tile_y.get(by), knobs().rows_tile_z.get(bz));
}

template <int NV, class S, class T>
static hipError_t wilson_eo_rows_t(bool adj, const Geom& g, int R, int bt, bool xcd, int parity, const void* Uo,
                                   const void* Ui, const void* in, void* out, const void* add, double c_add,
                                   double c_hop, hipStream_t st, int epi, EpiArgs& ea) {
  using W = typename S::word;
  const RowTraversal tr = make_row_traversal(g, uint32_t(R), uint32_t(bt));
  const ChunkTiles o = rows_tiles(g, R, 12L * NV * long(sizeof(W)), true);
  const dim3 block(NV, R), grid(tr.rows_plane * uint32_t(g.n[2]) * uint32_t(g.n[3]));
  if (epi != EPI_STORE && grid.x > ea.capacity) return hipErrorNotSupported;
  ea.blocks = grid.x;
  const size_t lds = (rows_lds_words<NV, S>(R) + size_t(R) * 9) * sizeof(W);
#define DSL_EK(A, E)                                                                                          \
  hipLaunchKernelGGL((wilson_eo_rows_kernel<3, A, NV, S, T, E>), grid, block, lds, st, g, tr, o, int(xcd), parity, \
                     (const W*)Uo, (const W*)Ui, (const W*)in, (W*)out, (const W*)add, T(c_add), T(c_hop), ea)
  // fused epilogues: the Schur operator M with EPI_NORM, M^dag with EPI_AXPY
  if (epi == EPI_STORE) {
    if (adj) DSL_EK(true, EPI_STORE); else DSL_EK(false, EPI_STORE);
  } else if (epi == EPI_NORM && !adj) {
    DSL_EK(false, EPI_NORM);
  } else if (epi == EPI_AXPY && adj) {
    DSL_EK(true, EPI_AXPY);
  } else {
    return hipErrorNotSupported;
  }
#undef DSL_EK
  return hipGetLastError();
}

template <int NV>
static hipError_t wilson_eo_rows_nv(bool adj, int dtype, const Geom& g, int R, int bt, bool xcd, int parity,
                                    const void* Uo, const void* Ui, const void* in, void* out, const void* add,
                                    double c_add, double c_hop, hipStream_t st, int epi, EpiArgs& ep) {
  switch (dtype) {
    case DT_C64: return wilson_eo_rows_t<NV, C64, float>(adj, g, R, bt, xcd, parity, Uo, Ui, in, out, add, c_add, c_hop,
                                                      st, epi, ep);
    case DT_BF16: return wilson_eo_rows_t<NV, BF16, float>(adj, g, R, bt, xcd, parity, Uo, Ui, in, out, add, c_add,
                                                       c_hop, st, epi, ep);
    case DT_F16: return wilson_eo_rows_t<NV, F16, float>(adj, g, R, bt, xcd, parity, Uo, Ui, in, out, add, c_add, c_hop,
                                                      st, epi, ep);
  }
  return hipErrorNotSupported;
}

// Row-staged even-odd hop for N_v = 4, 8, 12, 16, 24 (C64, BF16, F16
// storage), with the chunk rule of the full-lattice kernels on the packed
// rows; hipErrorNotSupported otherwise (the caller then uses the direct
// kernel).  DSLASH_ROWS=0 disables it.
hipError_t launch_wilson_eo_rows(bool adj, int dtype, const EoGeom& e, int parity, const void* Uo, const void* Ui,
                                 const void* in, void* out, const void* add, double c_add, double c_hop,
                                 hipStream_t st, int epi, EpiArgs* ea) {
  if (knobs().rows.get(1) == 0) return hipErrorNotSupported;
  if (!aligned16(Uo) || !aligned16(Ui) || !aligned16(in) || !aligned16(out) || !aligned16(add))
    return hipErrorNotSupported;
  if (epi != EPI_STORE && !ea) return hipErrorNotSupported;
  EpiArgs none;
  EpiArgs& ep = ea ? *ea : none;
  const int nv = e.nv;
  if (nv != 4 && nv != 8 && nv != 12 && nv != 16 && nv != 24) return hipErrorNotSupported;
  const int pdims[4] = {e.nh, e.n[1], e.n[2], e.n[3]};
  const Geom g = make_geom(pdims, nv);
  int R = row_sites_default(g.n[0], nv);
  R = knobs().row_sites.get(R);
  if (R > g.n[0]) R = g.n[0];
  if (R < 1 || R * nv > 256 || R * nv < 64) return hipErrorNotSupported;
  // the own row's two halo sites in the extra register groups
  const int word_bytes = int(dtype_bytes(dtype));
  if (R * 16 * row_extra_groups(nv, word_bytes) < 2 * 12 * word_bytes) return hipErrorNotSupported;
  int bt = 2;
  bt = knobs().tband.get(bt);
  bool xcd = true;
  xcd = knobs().xcd.get(xcd) != 0;
  switch (nv) {
    case 4: return wilson_eo_rows_nv<4>(adj, dtype, g, R, bt, xcd, parity, Uo, Ui, in, out, add, c_add, c_hop, st, epi, ep);
    case 8: return wilson_eo_rows_nv<8>(adj, dtype, g, R, bt, xcd, parity, Uo, Ui, in, out, add, c_add, c_hop, st, epi, ep);
    case 16:
      return wilson_eo_rows_nv<16>(adj, dtype, g, R, bt, xcd, parity, Uo, Ui, in, out, add, c_add, c_hop, st, epi, ep);
    case 24:
      return wilson_eo_rows_nv<24>(adj, dtype, g, R, bt, xcd, parity, Uo, Ui, in, out, add, c_add, c_hop, st, epi, ep);
  }
  return wilson_eo_rows_nv<12>(adj, dtype, g, R, bt, xcd, parity, Uo, Ui, in, out, add, c_add, c_hop, st, epi, ep);
}

template <int DEPTH, int NV, class S, class T>
static hipError_t wilson_rows_t(bool adj, const Geom& g, int R, int bt, bool xcd, const void* U, const void* in,
                                void* out, const void* C, double mass, hipStream_t st) {
  using W = typename S::word;
  const RowTraversal tr = make_row_traversal(g, uint32_t(R), uint32_t(bt));
  const ChunkTiles o = rows_tiles(g, R, 12L * NV * long(sizeof(W)), false);
  const dim3 block(NV, R), grid(tr.rows_plane * uint32_t(g.n[2]) * uint32_t(g.n[3]));
  size_t lds = (rows_lds_words<NV, S>(R) + (C ? 3 + size_t(R) * 36 : 0)) * sizeof(W);
  // DSLASH_ROW_LDS_EXTRA (bytes) lowers the workgroups per CU (tuning).
  lds += size_t(knobs().row_lds_extra.get(0));
  const T diag = T(4) + T(mass);
#define DSL_RK(A, CL)                                                                                      \
  hipLaunchKernelGGL((wilson_rows_kernel<DEPTH, A, CL, NV, S, T>), grid, block, lds, st, g, tr, o, int(xcd), (const W*)U, \
                     (const W*)in, (W*)out, (const W*)C, diag)
  if (C) {
    if (adj) DSL_RK(true, true); else DSL_RK(false, true);
  } else {
    if (adj) DSL_RK(true, false); else DSL_RK(false, false);
  }
#undef DSL_RK
  return hipGetLastError();
}


// Row-staged D_W with FP32 arithmetic (C64, BF16, F16 storage) for N_v = 4, 8,
// 12, 16, 24.  Returns hipErrorNotSupported when the configuration is not
// covered (the caller then uses the direct-load kernel).  DSLASH_ROWS=0
// disables it.
//
// Other block sizes than 12 take the t-marching kernel in the
// default form of each storage: FP32 with half-spinor neighbour rows, BF16
// with the own-row buffer, FP16 with one buffer; full links, no fused epilogue.
template <int NV>
static hipError_t wilson_march_nv(bool adj, int dtype, const Geom& g, int R, int tsteps, bool xcd, const void* U,
                                  const void* in, void* out, double mass, hipStream_t st) {
  EpiArgs none;
  switch (dtype) {
    case DT_C64:
      return wilson_march_t<3, NV, C64, float, 9, 3>(adj, g, R, tsteps, 3, xcd, U, in, out, mass, st, EPI_STORE, none);
    case DT_BF16:
      return wilson_march_t<2, NV, BF16, float, 9, 2>(adj, g, R, tsteps, 2, xcd, U, in, out, mass, st, EPI_STORE, none);
    case DT_F16:
      return wilson_march_t<2, NV, F16, float, 9, 0>(adj, g, R, tsteps, 0, xcd, U, in, out, mass, st, EPI_STORE, none);
  }
  return hipErrorNotSupported;
}

hipError_t launch_wilson_rows(bool adj, int dtype, const Geom& g, const void* U, const void* in, void* out,
                              double mass, hipStream_t st, const void* clover, bool compressed, int epi,
                              EpiArgs* ea) {
  if (knobs().rows.get(1) == 0) return hipErrorNotSupported;
  if (!aligned16(U) || !aligned16(in) || !aligned16(out) || !aligned16(clover)) return hipErrorNotSupported;
  if (epi != EPI_STORE && (!ea || clover || compressed)) return hipErrorNotSupported;
  EpiArgs none;
  EpiArgs& e = ea ? *ea : none;
  const int nv = g.nv;
  if (nv != 4 && nv != 8 && nv != 12 && nv != 16 && nv != 24) return hipErrorNotSupported;
  if (nv != 12 && (clover || compressed || epi != EPI_STORE)) return hipErrorNotSupported;
  int R = row_sites_default(g.n[0], nv);
  R = knobs().row_sites.get(R);
  if (R > g.n[0]) R = g.n[0];
  if (R < 1 || R * nv > 256 || R * nv < 64) return hipErrorNotSupported;
  // the own row's two halo sites (2 * 12 N_v words) must fit the extra
  // register groups of the workgroup's R N_v threads
  const int word_bytes = int(dtype_bytes(dtype));
  if (R * 16 * row_extra_groups(nv, word_bytes) < 2 * 12 * word_bytes) return hipErrorNotSupported;
  int bt = 2;
  bt = knobs().tband.get(bt);
  bool xcd = true;
  xcd = knobs().xcd.get(xcd) != 0;
  // DSLASH_TSTEPS: t steps per workgroup of the t-marching kernel (default 8;
  // 0 selects the kernel with one output row per workgroup).
  // DSLASH_ROW_DEPTH: rows in flight per workgroup (default 3 with half-spinor
  // rows, 2 otherwise when marching, 3 for the one-row kernel).
  // DSLASH_MARCH_PP: 0 = one row buffer, 1 = two used in turn (one barrier per
  // staged row), 2 = an own-row buffer that keeps the +t row for the next step
  // plus two used in turn, 3 = the same with half-spinor neighbour rows (FP32
  // storage only; others fall back to 2).
  // Default: FP32 storage takes 3 (full or compressed links), BF16 storage 2,
  // FP16 storage and other compressed links one buffer; with FP32 storage, a
  // lattice whose 16-step grid fits at two workgroups per CU (all its
  // workgroups resident at once) and still gives every SIMD 1.5 waves marches
  // 16 steps, otherwise 8.  On 16^3 x 32: N_v = 12 and 16 take 16 steps
  // (1536 and 2048 waves); N_v = 4 and 8 (512 and 1024 waves at 16 steps)
  // took 44.4 and 65.6 us at 8 steps against 64.8 and 74.6 us at 16.
  int tsteps = 8;
  int pp = 0;
  if (knobs().tsteps.set) {
    tsteps = knobs().tsteps.value;
  } else if (!clover) {
    if (dtype == DT_C64) pp = 3;
    if (dtype == DT_BF16 && !compressed) pp = 2;
    if (dtype == DT_C64 && g.n[3] >= 16) {
      const MarchTraversal m16 = make_march_traversal(g, uint32_t(R), 16u);
      const uint32_t wgs = m16.rows * ((uint32_t(g.n[3]) + 15u) / 16u);
      const uint32_t waves = wgs * uint32_t((R * nv + 63) / 64);
      if (wgs <= 2u * uint32_t(device_cus()) && 2u * waves >= 3u * 4u * uint32_t(device_cus())) tsteps = 16;
    }
  }
  if (nv != 12) {
    if (tsteps <= 0 || clover) return hipErrorNotSupported;
    switch (nv) {
      case 4: return wilson_march_nv<4>(adj, dtype, g, R, tsteps, xcd, U, in, out, mass, st);
      case 8: return wilson_march_nv<8>(adj, dtype, g, R, tsteps, xcd, U, in, out, mass, st);
      case 16: return wilson_march_nv<16>(adj, dtype, g, R, tsteps, xcd, U, in, out, mass, st);
      case 24: return wilson_march_nv<24>(adj, dtype, g, R, tsteps, xcd, U, in, out, mass, st);
    }
    return hipErrorNotSupported;
  }
  pp = knobs().march_pp.get(pp);
  if (pp == 3 && dtype != DT_C64) pp = 2;
  if (pp < 0 || pp > 3 || (compressed && pp != 3)) pp = 0;
  // the clover term is fused into the one-row-per-workgroup kernel only;
  // compressed links are read by the t-marching kernel only
  if (compressed && (tsteps <= 0 || clover)) return hipErrorNotSupported;
  if (tsteps > 0 && !clover) {
    // the fused epilogues take the default depth of the buffer scheme
    const int depth = epi != EPI_STORE ? (pp == 3 ? 3 : 2) : knobs().row_depth.get(pp == 3 ? 3 : 2);
#define DSL_MT(D, LW)                                                                                               \
  switch (dtype) {                                                                                                  \
    case DT_C64: return wilson_march_t<D, 12, C64, float, LW>(adj, g, R, tsteps, pp, xcd, U, in, out, mass, st, epi, e); \
    case DT_BF16:                                                                                                   \
      return wilson_march_t<D, 12, BF16, float, LW>(adj, g, R, tsteps, pp, xcd, U, in, out, mass, st, epi, e);       \
    case DT_F16: return wilson_march_t<D, 12, F16, float, LW>(adj, g, R, tsteps, pp, xcd, U, in, out, mass, st, epi, e); \
  }
    if (compressed) {
      if (depth <= 2) {
        DSL_MT(2, 6)
      } else {
        DSL_MT(3, 6)
      }
    } else if (depth <= 2) {
      DSL_MT(2, 9)
    } else {
      DSL_MT(3, 9)
    }
#undef DSL_MT
    return hipErrorNotSupported;
  }
  if (epi != EPI_STORE) return hipErrorNotSupported;
  const int depth = knobs().row_depth.get(3);
#define DSL_RT(D)                                                                               \
  switch (dtype) {                                                                              \
    case DT_C64: return wilson_rows_t<D, 12, C64, float>(adj, g, R, bt, xcd, U, in, out, clover, mass, st);   \
    case DT_BF16: return wilson_rows_t<D, 12, BF16, float>(adj, g, R, bt, xcd, U, in, out, clover, mass, st); \
    case DT_F16: return wilson_rows_t<D, 12, F16, float>(adj, g, R, bt, xcd, U, in, out, clover, mass, st);   \
  }
  if (depth <= 2) { DSL_RT(2) } else if (depth <= 3) { DSL_RT(3) } else { DSL_RT(7) }
#undef DSL_RT
  return hipErrorNotSupported;
}

}  // namespace dsl
