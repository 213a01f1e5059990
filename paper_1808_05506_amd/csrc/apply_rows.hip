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
//   buf  [(R + 2) * 12 NV]  one staged row at index x - x0 + 1: a neighbour row
//                           fills 1 .. n, the chunk's own row 0 .. n + 1 (with
//                           the halo sites x0 - 1 and x0 + n); reused for the output
//   lown [(R + 1) * 36]     links of sites x0 - 1 .. x0 + n - 1 (index x - x0 + 1)
//   lnb  [R * 9]            V_mu of the backward neighbour row (current mu)
template <int NV, class S>
size_t rows_lds_words(int R);

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

template <int NV, class S>
size_t rows_lds_words(int R) {
  return size_t(R + 2) * SiteStride<NV, S>::WORDS + size_t(R + 1) * 36 + size_t(R) * 9;
}

// Piece assignment of a staged row: lane (x, v) of the workgroup moves the
// pieces j * N_v + v (j = 0 .. CH - 1) of site x of the run, so the N_v lanes
// of a site read N_v consecutive 16-byte pieces per instruction and the LDS
// position follows from the site without a division.  Lanes past a partial
// chunk's end repeat the last site (same data to the same place).
template <int MU, int SGN, int NV, class S>
__device__ __forceinline__ void row_issue(const Geom& g, const RowChunk& c, const typename S::word* __restrict__ U,
                                          const typename S::word* __restrict__ in, int xl, int v, int tid,
                                          u32x4 (&r)[RowPieces<S>::CH + 1]) {
  using W = typename S::word;
  constexpr int SW = 12 * NV, CH = RowPieces<S>::CH;
  const uint32_t nrow = row_base_shift(g, c, MU, SGN) + uint32_t(c.x0);
  const int xc = xl < c.n ? xl : c.n - 1;
  const u32x4* src = reinterpret_cast<const u32x4*>(in + size_t(nrow + xc) * SW);
#pragma unroll
  for (int j = 0; j < CH; ++j) r[j] = src[j * NV + v];
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
                                           typename S::word* row, typename S::word* lnb, int xl, int v, int tid) {
  using W = typename S::word;
  constexpr int CH = RowPieces<S>::CH, SSP = SiteStride<NV, S>::PIECES;
  const int xc = xl < c.n ? xl : c.n - 1;
  u32x4* dst = reinterpret_cast<u32x4*>(row) + xc * SSP;
#pragma unroll
  for (int j = 0; j < CH; ++j) dst[j * NV + v] = r[j];
  if (SGN < 0) {
    W lk;
    const u32x4 z = r[CH];
    __builtin_memcpy(&lk, &z, sizeof(W));
    lnb[tid < c.n * 9 ? tid : c.n * 9 - 1] = lk;
  }
}

// The chunk's own row in the same register shape: CH pieces of site x and,
// in slot CH, at most one piece of the two halo sites x0 - 1, x0 + n (2 * 12 N_v
// words, never more pieces than threads; the launcher checks this).
template <int NV, class S>
__device__ __forceinline__ void own_issue(const RowChunk& c, const typename S::word* __restrict__ in, int xm,
                                          int xp, int xl, int v, int tid, u32x4 (&r)[RowPieces<S>::CH + 1]) {
  using W = typename S::word;
  constexpr int SW = 12 * NV, CH = RowPieces<S>::CH, SP = SW * int(sizeof(W)) / 16;
  const int xc = xl < c.n ? xl : c.n - 1;
  const u32x4* src = reinterpret_cast<const u32x4*>(in + size_t(c.row_base + c.x0 + xc) * SW);
#pragma unroll
  for (int j = 0; j < CH; ++j) r[j] = src[j * NV + v];
  const int h = tid < 2 * SP ? tid : 2 * SP - 1;
  const int hs = h < SP ? xm : xp;
  r[CH] = reinterpret_cast<const u32x4*>(in + size_t(c.row_base + hs) * SW)[h < SP ? h : h - SP];
}

template <int NV, class S>
__device__ __forceinline__ void own_commit(const RowChunk& c, const u32x4 (&r)[RowPieces<S>::CH + 1],
                                           typename S::word* buf, int xl, int v, int tid) {
  using W = typename S::word;
  constexpr int SW = 12 * NV, CH = RowPieces<S>::CH, SP = SW * int(sizeof(W)) / 16;
  constexpr int SSP = SiteStride<NV, S>::PIECES;
  const int xc = xl < c.n ? xl : c.n - 1;
  u32x4* dst = reinterpret_cast<u32x4*>(buf) + (xc + 1) * SSP;
#pragma unroll
  for (int j = 0; j < CH; ++j) dst[j * NV + v] = r[j];
  const int h = tid < 2 * SP ? tid : 2 * SP - 1;
  u32x4* hdst = reinterpret_cast<u32x4*>(buf) + (h < SP ? 0 : (c.n + 1) * SSP);
  hdst[h < SP ? h : h - SP] = r[CH];
}

template <int MU, int SGN, bool ADJ, int NV, class S, class T>
__device__ __forceinline__ void row_compute(const typename S::word* nbr, const typename S::word* lown,
                                            const typename S::word* lnb, int xl, int v, cpx<T> (&acc)[4][3]) {
  constexpr int SSW = SiteStride<NV, S>::WORDS;
  if (SGN > 0)
    lds_hop<MU, (ADJ ? 1 : -1), false, NV, S, T>(nbr + xl * SSW, lown + (xl + 1) * 36 + MU * 9, v, acc);
  else
    lds_hop<MU, (ADJ ? -1 : 1), true, NV, S, T>(nbr + xl * SSW, lnb + xl * 9, v, acc);
}

// Occupancy hint per prefetch depth: deeper prefetch holds more rows in
// registers (about 28 VGPRs per FP32 row) and runs fewer waves per SIMD.
template <int DEPTH> struct RowsWaves { static constexpr int value = DEPTH <= 2 ? 4 : (DEPTH <= 4 ? 3 : 2); };

template <int DEPTH, bool ADJ, int NV, class S, class T>
__global__ void __launch_bounds__(256, RowsWaves<DEPTH>::value)
    wilson_rows_kernel(Geom g, RowTraversal tr, int xcd, const typename S::word* __restrict__ U,
                       const typename S::word* __restrict__ in, typename S::word* __restrict__ out, T diag) {
  using W = typename S::word;
  constexpr int SW = 12 * NV, CH = RowPieces<S>::CH;
  constexpr int SSW = SiteStride<NV, S>::WORDS, SSP = SiteStride<NV, S>::PIECES;
  extern __shared__ uint4 smem_rows[];
  const int R = int(tr.sb);
  W* buf = reinterpret_cast<W*>(smem_rows);
  W* lown = buf + (R + 2) * SSW;
  W* lnb = lown + (R + 1) * 36;

  const uint32_t L = xcd_block(blockIdx.x, gridDim.x, xcd != 0);
  const RowChunk c = row_chunk(g, tr, L);
  const int v = threadIdx.x, xl = threadIdx.y;
  const int tid = xl * NV + v, nth = R * NV;
  const int xm = wrap_x(g, c.x0 - 1), xp = wrap_x(g, c.x0 + c.n);

  // Seven rows pass through the one LDS row buffer: +y, -y, +z, -z, +t, -t,
  // then the chunk's own row with its halo sites.  Row k is requested DEPTH
  // steps before it is consumed (DEPTH = 7: all at once), each into its own
  // register array.
  u32x4 r0[CH + 1], r1[CH + 1], r2[CH + 1], r3[CH + 1], r4[CH + 1], r5[CH + 1], r6[CH + 1];
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
  // links of the chunk's sites and of the halo site x0 - 1 (at most 3 pieces
  // per thread: a site's links are 36 words)
  constexpr int LINK_PIECES = 36 * int(sizeof(W)) / 16;
  copy_pieces<3>(lown + 36, U + size_t(c.row_base + c.x0) * 36, c.n * LINK_PIECES, tid, nth);
  copy_pieces<1>(lown, U + size_t(c.row_base + xm) * 36, LINK_PIECES, tid, nth);

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
#pragma unroll
    for (int sp = 0; sp < 4; ++sp)
#pragma unroll
      for (int cc = 0; cc < 3; ++cc) {
        cpx<T> p = S::template load<T>(self + (sp * 3 + cc) * NV + v);
        res[sp][cc].r = fma(diag, p.r, T(-0.5) * acc[sp][cc].r);
        res[sp][cc].i = fma(diag, p.i, T(-0.5) * acc[sp][cc].i);
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

template <int DEPTH, int NV, class S, class T>
static hipError_t wilson_rows_t(bool adj, const Geom& g, int R, int bt, bool xcd, const void* U, const void* in,
                                void* out, double mass, hipStream_t st) {
  using W = typename S::word;
  const RowTraversal tr = make_row_traversal(g, uint32_t(R), uint32_t(bt));
  const dim3 block(NV, R), grid(tr.rows_plane * uint32_t(g.n[2]) * uint32_t(g.n[3]));
  size_t lds = rows_lds_words<NV, S>(R) * sizeof(W);
  // DSLASH_ROW_LDS_EXTRA (bytes) lowers the workgroups per CU (tuning).
  if (const char* e = getenv("DSLASH_ROW_LDS_EXTRA")) lds += size_t(atoi(e));
  const T diag = T(4) + T(mass);
  if (adj)
    hipLaunchKernelGGL((wilson_rows_kernel<DEPTH, true, NV, S, T>), grid, block, lds, st, g, tr, int(xcd), (const W*)U,
                       (const W*)in, (W*)out, diag);
  else
    hipLaunchKernelGGL((wilson_rows_kernel<DEPTH, false, NV, S, T>), grid, block, lds, st, g, tr, int(xcd), (const W*)U,
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
  int R = row_sites_default(g.n[0], g.nv);
  if (const char* e = getenv("DSLASH_ROW_SITES")) R = atoi(e);
  if (R > g.n[0]) R = g.n[0];
  if (R < 1 || R * g.nv > 256 || R * g.nv < 128) return hipErrorNotSupported;
  // the own row's two halo sites (2 * 12 N_v words) must be at most one
  // 16-byte piece per thread
  const int word_bytes = int(dtype_bytes(dtype));
  if (R * g.nv * 16 < 2 * 12 * g.nv * word_bytes) return hipErrorNotSupported;
  int bt = 2;
  if (const char* e = getenv("DSLASH_TBAND")) bt = atoi(e);
  bool xcd = true;
  if (const char* e = getenv("DSLASH_XCD")) xcd = atoi(e) != 0;
  int depth = 3;
  if (const char* e = getenv("DSLASH_ROW_DEPTH")) depth = atoi(e);
#define DSL_RT(D)                                                                               \
  switch (dtype) {                                                                              \
    case DT_C64: return wilson_rows_t<D, 12, C64, float>(adj, g, R, bt, xcd, U, in, out, mass, st);   \
    case DT_BF16: return wilson_rows_t<D, 12, BF16, float>(adj, g, R, bt, xcd, U, in, out, mass, st); \
    case DT_F16: return wilson_rows_t<D, 12, F16, float>(adj, g, R, bt, xcd, U, in, out, mass, st);   \
  }
  if (depth <= 2) { DSL_RT(2) } else if (depth <= 3) { DSL_RT(3) } else { DSL_RT(7) }
#undef DSL_RT
  return hipErrorNotSupported;
}

}  // namespace dsl
