// Row-staged D_W kernel (see rows.hpp): a workgroup owns an x-row chunk of
// R sites and all N_v right-hand sides; its inputs are copied into LDS with
// coalesced 16-byte loads, the hops are evaluated from LDS, and the outputs
// leave through LDS with coalesced 16-byte stores.
#include <stdlib.h>

#include "launch.hpp"
#include "rows.hpp"

namespace dsl {

// 16 bytes as a native vector (HIP's uint4 is a class around a union, which
// keeps arrays of it in scratch memory instead of registers).
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

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

// LDS layout, in storage words (one complex number each):
//   own  [(R + 2) * 12 NV]  sites x0 - 1 .. x0 + n of the chunk's row (index x - x0 + 1)
//   nbr  [R * 12 NV]        the current neighbour row's x0 .. x0 + n - 1; reused for the output
//   lown [(R + 1) * 36]     links of sites x0 - 1 .. x0 + n - 1 (index x - x0 + 1)
//   lnb  [R * 9]            V_mu of the backward neighbour row (current mu)
template <int NV>
DSL_HD size_t rows_lds_words(int R) {
  return size_t(R + 2) * 12 * NV + size_t(R) * 12 * NV + size_t(R + 1) * 36 + size_t(R) * 9;
}

template <class S, class T, int NV>
DSL_HD void lds_spinor(const typename S::word* __restrict__ site, int v, cpx<T> (&p)[4][3]) {
#pragma unroll
  for (int sp = 0; sp < 4; ++sp)
#pragma unroll
    for (int c = 0; c < 3; ++c) p[sp][c] = S::template load<T>(site + (sp * 3 + c) * NV + v);
}

// acc += (1 + C gamma_MU) U' psi with psi and U' read from LDS
template <int MU, int C, bool DAG, int NV, class S, class T>
__device__ __forceinline__ void lds_hop(const typename S::word* __restrict__ site,
                                       const typename S::word* __restrict__ link, int v, cpx<T> (&acc)[4][3]) {
  cpx<T> p[4][3];
  lds_spinor<S, T, NV>(site, v, p);
  cpx<T> h[2][3];
  project<MU, C, T>(p, h);
  cpx<T> u[3][3];
#pragma unroll
  for (int a = 0; a < 3; ++a)
#pragma unroll
    for (int b = 0; b < 3; ++b) u[a][b] = S::template load<T>(link + a * 3 + b);
  cpx<T> t[2][3];
  su3_mul2<DAG, T>(u, h, t);
  reconstruct_add<MU, C, T>(acc, t);
}

// One thread's share of a neighbour row in flight: CH 16-byte pieces of the
// spinor run (pieces tid, tid + nth, ...) plus, for a backward hop, one word of
// the V_mu piece of the row's links (held as a 16-byte register group so the
// whole row is one array).  The piece count per thread does not depend on R:
// a row chunk is R * 12 NV words and the workgroup has R * NV threads.
template <class S>
struct RowPieces {
  static constexpr int CH = 12 * int(sizeof(typename S::word)) / 16;
};

template <int MU, int SGN, int NV, class S>
__device__ __forceinline__ void row_issue(const Geom& g, const RowChunk& c, const typename S::word* __restrict__ U,
                                          const typename S::word* __restrict__ in, int tid, int nth,
                                          u32x4 (&r)[RowPieces<S>::CH + 1]) {
  using W = typename S::word;
  constexpr int SW = 12 * NV, CH = RowPieces<S>::CH;
  const uint32_t nrow = row_base_shift(g, c, MU, SGN) + uint32_t(c.x0);
  const u32x4* src = reinterpret_cast<const u32x4*>(in + size_t(nrow) * SW);
  const int pieces = c.n * SW * int(sizeof(W)) / 16;
#pragma unroll
  for (int j = 0; j < CH; ++j) {
    const int i = tid + j * nth;
    r[j] = src[i < pieces ? i : pieces - 1];
  }
  if (SGN < 0) {
    const int w = tid < c.n * 9 ? tid : c.n * 9 - 1;
    const int k = w / 9, e = w - k * 9;
    const W lk = U[(size_t(nrow + k) * 4 + MU) * 9 + e];
    u32x4 z = {0u, 0u, 0u, 0u};
    __builtin_memcpy(&z, &lk, sizeof(W));
    r[CH] = z;
  }
}

template <int SGN, int NV, class S>
__device__ __forceinline__ void row_commit(const RowChunk& c, const u32x4 (&r)[RowPieces<S>::CH + 1],
                                           typename S::word* nbr, typename S::word* lnb, int tid, int nth) {
  using W = typename S::word;
  constexpr int SW = 12 * NV, CH = RowPieces<S>::CH;
  u32x4* dst = reinterpret_cast<u32x4*>(nbr);
  const int pieces = c.n * SW * int(sizeof(W)) / 16;
#pragma unroll
  for (int j = 0; j < CH; ++j) {
    const int i = tid + j * nth;
    dst[i < pieces ? i : pieces - 1] = r[j];
  }
  if (SGN < 0) {
    W lk;
    const u32x4 z = r[CH];
    __builtin_memcpy(&lk, &z, sizeof(W));
    lnb[tid < c.n * 9 ? tid : c.n * 9 - 1] = lk;
  }
}

template <int MU, int SGN, bool ADJ, int NV, class S, class T>
__device__ __forceinline__ void row_compute(const typename S::word* nbr, const typename S::word* lown,
                                            const typename S::word* lnb, int xl, int v, cpx<T> (&acc)[4][3]) {
  constexpr int SW = 12 * NV;
  if (SGN > 0)
    lds_hop<MU, (ADJ ? 1 : -1), false, NV, S, T>(nbr + xl * SW, lown + (xl + 1) * 36 + MU * 9, v, acc);
  else
    lds_hop<MU, (ADJ ? -1 : 1), true, NV, S, T>(nbr + xl * SW, lnb + xl * 9, v, acc);
}

template <bool ADJ, int NV, class S, class T>
__global__ void __launch_bounds__(256) wilson_rows_kernel(Geom g, RowTraversal tr, int xcd,
                                                         const typename S::word* __restrict__ U,
                                                         const typename S::word* __restrict__ in,
                                                         typename S::word* __restrict__ out, T diag) {
  using W = typename S::word;
  constexpr int SW = 12 * NV;
  extern __shared__ uint4 smem_rows[];
  const int R = int(tr.sb);
  W* own = reinterpret_cast<W*>(smem_rows);
  W* nbr = own + (R + 2) * SW;
  W* lown = nbr + R * SW;
  W* lnb = lown + (R + 1) * 36;

  const uint32_t L = xcd_block(blockIdx.x, gridDim.x, xcd != 0);
  const RowChunk c = row_chunk(g, tr, L);
  const int v = threadIdx.x, xl = threadIdx.y;
  const int tid = xl * NV + v, nth = R * NV;
  const int xm = wrap_x(g, c.x0 - 1), xp = wrap_x(g, c.x0 + c.n);

  // Three neighbour rows in flight at a time: row k + 2 is requested while
  // hop k is evaluated.  Order: +y, -y, +z, -z, +t, -t.
  u32x4 ra[RowPieces<S>::CH + 1], rb[RowPieces<S>::CH + 1], rc[RowPieces<S>::CH + 1];
  row_issue<1, +1, NV, S>(g, c, U, in, tid, nth, ra);
  row_issue<1, -1, NV, S>(g, c, U, in, tid, nth, rb);

  // own row with one halo site on each side, and its links
  // (piece counts: a site's spinor is 12 NV words = RowPieces::CH pieces per
  // right-hand side, so the row needs CH pieces per thread and a halo site at
  // most one; a site's links are 36 words, at most 3 pieces per thread)
  constexpr int CH = RowPieces<S>::CH;
  constexpr int SITE_PIECES = SW * int(sizeof(W)) / 16, LINK_PIECES = 36 * int(sizeof(W)) / 16;
  copy_pieces<CH>(own + SW, in + size_t(c.row_base + c.x0) * SW, c.n * SITE_PIECES, tid, nth);
  copy_pieces<1>(own, in + size_t(c.row_base + xm) * SW, SITE_PIECES, tid, nth);
  copy_pieces<1>(own + (c.n + 1) * SW, in + size_t(c.row_base + xp) * SW, SITE_PIECES, tid, nth);
  copy_pieces<3>(lown + 36, U + size_t(c.row_base + c.x0) * 36, c.n * LINK_PIECES, tid, nth);
  copy_pieces<1>(lown, U + size_t(c.row_base + xm) * 36, LINK_PIECES, tid, nth);

  cpx<T> acc[4][3];
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 3; ++b) acc[a][b] = zero<T>();

#define DSL_ROW_STEP(MU, SGN, CUR, NMU, NSGN, NEXT)                            \
  row_commit<SGN, NV, S>(c, CUR, nbr, lnb, tid, nth);                          \
  __syncthreads();                                                             \
  if (NMU > 0) row_issue<(NMU > 0 ? NMU : 1), NSGN, NV, S>(g, c, U, in, tid, nth, NEXT); \
  row_compute<MU, SGN, ADJ, NV, S, T>(nbr, lown, lnb, xl, v, acc);             \
  __syncthreads();
  DSL_ROW_STEP(1, +1, ra, 2, +1, rc)
  DSL_ROW_STEP(1, -1, rb, 2, -1, ra)
  DSL_ROW_STEP(2, +1, rc, 3, +1, rb)
  DSL_ROW_STEP(2, -1, ra, 3, -1, rc)
  DSL_ROW_STEP(3, +1, rb, 0, +1, ra)
  DSL_ROW_STEP(3, -1, rc, 0, +1, rb)
#undef DSL_ROW_STEP

  // Lanes past a partial chunk's end (xl >= n) compute on stale but in-bounds
  // LDS data and their results are never copied out; keeping every lane on
  // the same straight-line path lets the compiler keep the prefetches in
  // flight across the hops.
  {
    constexpr int CF = ADJ ? +1 : -1, CB = -CF;
    // x hops from the own row: x + 1 at index xl + 2, x - 1 (and its link) at index xl
    lds_hop<0, CF, false, NV, S, T>(own + (xl + 2) * SW, lown + (xl + 1) * 36, v, acc);
    lds_hop<0, CB, true, NV, S, T>(own + xl * SW, lown + xl * 36, v, acc);
    const W* self = own + (xl + 1) * SW;
    W* o = nbr + xl * SW;
#pragma unroll
    for (int sp = 0; sp < 4; ++sp)
#pragma unroll
      for (int cc = 0; cc < 3; ++cc) {
        const int e = (sp * 3 + cc) * NV + v;
        cpx<T> p = S::template load<T>(self + e);
        cpx<T> r;
        r.r = fma(diag, p.r, T(-0.5) * acc[sp][cc].r);
        r.i = fma(diag, p.i, T(-0.5) * acc[sp][cc].i);
        S::template store<T>(o + e, r);
      }
  }
  __syncthreads();
  copy_pieces<CH>(out + size_t(c.row_base + c.x0) * SW, nbr, c.n * SITE_PIECES, tid, nth);
}

template <int NV, class S, class T>
static hipError_t wilson_rows_t(bool adj, const Geom& g, int R, int bt, bool xcd, const void* U, const void* in,
                                void* out, double mass, hipStream_t st) {
  using W = typename S::word;
  const RowTraversal tr = make_row_traversal(g, uint32_t(R), uint32_t(bt));
  const dim3 block(NV, R), grid(tr.rows_plane * uint32_t(g.n[2]) * uint32_t(g.n[3]));
  const size_t lds = rows_lds_words<NV>(R) * sizeof(W);
  const T diag = T(4) + T(mass);
  if (adj)
    hipLaunchKernelGGL((wilson_rows_kernel<true, NV, S, T>), grid, block, lds, st, g, tr, int(xcd), (const W*)U,
                       (const W*)in, (W*)out, diag);
  else
    hipLaunchKernelGGL((wilson_rows_kernel<false, NV, S, T>), grid, block, lds, st, g, tr, int(xcd), (const W*)U,
                       (const W*)in, (W*)out, diag);
  return hipGetLastError();
}

// Row-staged D_W for N_v = 12 with FP32 arithmetic (C64, BF16, F16 storage).
// Returns hipErrorNotSupported when the configuration is not covered (the
// caller then uses the direct-load kernel).  DSLASH_ROWS=0 disables it.
hipError_t launch_wilson_rows(bool adj, int dtype, const Geom& g, const void* U, const void* in, void* out,
                              double mass, hipStream_t st) {
  if (const char* e = getenv("DSLASH_ROWS"))
    if (atoi(e) == 0) return hipErrorNotSupported;
  if (g.nv != 12) return hipErrorNotSupported;
  int R = 16;
  if (const char* e = getenv("DSLASH_ROW_SITES")) R = atoi(e);
  if (R > g.n[0]) R = g.n[0];
  if (R < 1 || R * g.nv > 256 || R * g.nv < 128) return hipErrorNotSupported;
  int bt = 8;
  if (const char* e = getenv("DSLASH_TBAND")) bt = atoi(e);
  bool xcd = true;
  if (const char* e = getenv("DSLASH_XCD")) xcd = atoi(e) != 0;
  switch (dtype) {
    case DT_C64: return wilson_rows_t<12, C64, float>(adj, g, R, bt, xcd, U, in, out, mass, st);
    case DT_BF16: return wilson_rows_t<12, BF16, float>(adj, g, R, bt, xcd, U, in, out, mass, st);
    case DT_F16: return wilson_rows_t<12, F16, float>(adj, g, R, bt, xcd, U, in, out, mass, st);
  }
  return hipErrorNotSupported;
}

}  // namespace dsl
