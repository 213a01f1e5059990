// Row-staged link gradients of D_W and D_S (see rows.hpp for the row
// staging).  A workgroup owns an x-row chunk of R sites and all N_v
// right-hand sides.  For G_mu(x) each site needs chi and psi at x and at
// x + mu; every such input is a contiguous run (the chunk's own row with one
// halo site at x0 + n, or the same x-range of the +y, +z, +t row), staged one
// field at a time through one LDS buffer with coalesced loads.  A thread keeps
// the chi and psi of its own (site, rhs) in registers; the two halves of each
// term use one neighbour field each:
//   Wilson     G_mu(x) = -1/2 sum_v sum_t [ (P_- chi(x))_t (x) conj((P_- psi(x+mu))_t)
//                                        + (P_+ psi(x))_t (x) conj((P_+ chi(x+mu))_t) ]
//   staggered  G_mu(x) = eta_mu(x)/2 sum_v [ chi(x) (x) conj(psi(x+mu)) - psi(x) (x) conj(chi(x+mu)) ]
// The per-rhs shares are summed over v through LDS; G leaves through LDS with
// coalesced stores, written once.
#include <stdlib.h>

#include "launch.hpp"
#include "rows.hpp"
#include "tiles.hpp"

namespace dsl {

namespace {

// G_mu share: gm[a][b] += sum_t l[t][a] conj(r[t][b])
template <int K, class T>
__device__ __forceinline__ void outer_add(cpx<T> (&gm)[3][3], const cpx<T> (&l)[K][3], const cpx<T> (&r)[K][3]) {
#pragma unroll
  for (int a = 0; a < 3; ++a)
#pragma unroll
    for (int b = 0; b < 3; ++b)
#pragma unroll
      for (int t = 0; t < K; ++t) gm[a][b] = cmaddj(gm[a][b], l[t][a], r[t][b]);
}

template <int MU, int C, class T>
__device__ __forceinline__ void proj12(const cpx<T> (&p)[12], cpx<T> (&h)[2][3]) {
  cpx<T> q[4][3];
#pragma unroll
  for (int s = 0; s < 4; ++s)
#pragma unroll
    for (int c = 0; c < 3; ++c) q[s][c] = p[s * 3 + c];
  project<MU, C, T>(q, h);
}

// One term of G_mu from the neighbour field in LDS.  TERM 0 pairs the own chi
// with the neighbour psi, TERM 1 the own psi with the neighbour chi.
template <int OP, int MU, int TERM, int NV, class S, class T>
__device__ __forceinline__ void grad_term(const typename S::word* nb, const cpx<T>* own_chi, const cpx<T>* own_psi,
                                          int v, cpx<T> (&gm)[3][3]) {
  if constexpr (OP == OP_WILSON) {
    cpx<T> f[12];
    lds_column<12, NV, S, T>(nb, v, f);
    cpx<T> hl[2][3], hr[2][3];
    cpx<T> own[12];
#pragma unroll
    for (int c = 0; c < 12; ++c) own[c] = TERM == 0 ? own_chi[c] : own_psi[c];
    // TERM 0: (1 - gamma) projections, TERM 1: (1 + gamma) projections
    proj12<MU, (TERM == 0 ? -1 : +1), T>(own, hl);
    proj12<MU, (TERM == 0 ? -1 : +1), T>(f, hr);
    outer_add<2, T>(gm, hl, hr);
  } else {
    cpx<T> f[3];
    lds_column<3, NV, S, T>(nb, v, f);
    cpx<T> l[1][3], r[1][3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      l[0][c] = TERM == 0 ? own_chi[c] : -own_psi[c];
      r[0][c] = f[c];
    }
    outer_add<1, T>(gm, l, r);
  }
}

}  // namespace

template <int OP, int NV, class S, class T>
__global__ void __launch_bounds__(256, 3) grad_rows_kernel(Geom g, RowTraversal tr, ChunkTiles o, int xcd,
                                                          const typename S::word* __restrict__ chi,
                                                          const typename S::word* __restrict__ psi,
                                                          typename S::word* __restrict__ G) {
  constexpr int COMPS = OP == OP_WILSON ? 12 : 3;
  typedef Stage<COMPS, NV, S> St;
  typedef typename St::P P;
  using W = typename S::word;
  extern __shared__ uint4 smem_grad[];
  const int R = int(tr.sb);
  W* buf = reinterpret_cast<W*>(smem_grad);                         // (R + 1) padded sites
  cpx<T>* red = reinterpret_cast<cpx<T>*>(buf + (R + 1) * St::SSW);  // [R][9][NV]
  W* gout = reinterpret_cast<W*>(red + R * 9 * NV);                  // [R][36]

  const uint32_t L = xcd_block(blockIdx.x, gridDim.x, xcd != 0);
  const RowChunk c = order_chunk(g, tr, o, L);
  const int v = threadIdx.x, xl = threadIdx.y;
  const int tid = xl * NV + v, nth = R * NV;
  const uint32_t own_base = c.row_base + uint32_t(c.x0);
  const uint32_t xp = c.row_base + uint32_t(wrap_x(g, c.x0 + c.n));
  const int xc = xl < c.n ? xl : c.n - 1;

  cpx<T> oc[COMPS], op[COMPS];  // own chi and psi of (x, v)
  P ra[St::CH + 1], rb[St::CH + 1];
  stage_issue<COMPS, NV, S, true>(psi, own_base, c.n, xp, xl, v, tid, ra);
  stage_issue<COMPS, NV, S, true>(chi, own_base, c.n, xp, xl, v, tid, rb);

  // mu = 0: psi row, then chi row (both with the x0 + n halo)
  cpx<T> gm[3][3];
#pragma unroll
  for (int a = 0; a < 3; ++a)
#pragma unroll
    for (int b = 0; b < 3; ++b) gm[a][b] = zero<T>();
  cpx<T> pnext[COMPS];
  stage_commit<COMPS, NV, S, true>(ra, buf, c.n, xl, v, tid);
  __syncthreads();
  stage_issue<COMPS, NV, S, false>(psi, row_base_shift(g, c, 1, +1) + uint32_t(c.x0), c.n, 0, xl, v, tid, ra);
  lds_column<COMPS, NV, S, T>(buf + xc * St::SSW, v, op);
  lds_column<COMPS, NV, S, T>(buf + (xc + 1) * St::SSW, v, pnext);
  __syncthreads();
  stage_commit<COMPS, NV, S, true>(rb, buf, c.n, xl, v, tid);
  __syncthreads();
  stage_issue<COMPS, NV, S, false>(chi, row_base_shift(g, c, 1, +1) + uint32_t(c.x0), c.n, 0, xl, v, tid, rb);
  lds_column<COMPS, NV, S, T>(buf + xc * St::SSW, v, oc);
  {
    // term 0 with psi(x + 1) from registers, term 1 with chi(x + 1) from LDS
    if constexpr (OP == OP_WILSON) {
      cpx<T> hl[2][3], hr[2][3];
      proj12<0, -1, T>(oc, hl);
      proj12<0, -1, T>(pnext, hr);
      outer_add<2, T>(gm, hl, hr);
    } else {
      cpx<T> l[1][3], r[1][3];
#pragma unroll
      for (int cc = 0; cc < 3; ++cc) {
        l[0][cc] = oc[cc];
        r[0][cc] = pnext[cc];
      }
      outer_add<1, T>(gm, l, r);
    }
    grad_term<OP, 0, 1, NV, S, T>(buf + (xc + 1) * St::SSW, oc, op, v, gm);
  }

  // reduce the mu share over the right-hand sides and stage it in gout
  auto reduce_mu = [&](int mu) {
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
      for (int b = 0; b < 3; ++b) red[(xl * 9 + a * 3 + b) * NV + v] = gm[a][b];
    __syncthreads();
    for (int o = tid; o < R * 9; o += nth) {
      const int sl = o / 9, e = o - sl * 9;
      cpx<T> z = zero<T>();
#pragma unroll
      for (int l = 0; l < NV; ++l) z += red[(sl * 9 + e) * NV + l];
      T f;
      if (OP == OP_WILSON) {
        f = T(-0.5);
      } else {
        int pp = 0;
        const int coord[4] = {c.x0 + sl, c.y, c.z, c.t};
        for (int nu = 0; nu < mu; ++nu) pp += coord[nu];
        f = (pp & 1) ? T(-0.5) : T(0.5);
      }
      S::template store<T>(gout + sl * 36 + mu * 9 + e, f * z);
    }
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
      for (int b = 0; b < 3; ++b) gm[a][b] = zero<T>();
  };
  reduce_mu(0);
  __syncthreads();

  // mu = 1, 2, 3: the psi row of x + mu, then the chi row; the next row is
  // requested while the current one is used
#define DSL_GRAD_MU(MU, NEXT_MU)                                                                        \
  stage_commit<COMPS, NV, S, false>(ra, buf, c.n, xl, v, tid);                                          \
  __syncthreads();                                                                                      \
  if (NEXT_MU > 0)                                                                                      \
    stage_issue<COMPS, NV, S, false>(psi, row_base_shift(g, c, (NEXT_MU > 0 ? NEXT_MU : 1), +1) +       \
                                              uint32_t(c.x0), c.n, 0, xl, v, tid, ra);                  \
  grad_term<OP, MU, 0, NV, S, T>(buf + xc * St::SSW, oc, op, v, gm);                                    \
  __syncthreads();                                                                                      \
  stage_commit<COMPS, NV, S, false>(rb, buf, c.n, xl, v, tid);                                          \
  __syncthreads();                                                                                      \
  if (NEXT_MU > 0)                                                                                      \
    stage_issue<COMPS, NV, S, false>(chi, row_base_shift(g, c, (NEXT_MU > 0 ? NEXT_MU : 1), +1) +       \
                                              uint32_t(c.x0), c.n, 0, xl, v, tid, rb);                  \
  grad_term<OP, MU, 1, NV, S, T>(buf + xc * St::SSW, oc, op, v, gm);                                    \
  reduce_mu(MU);                                                                                        \
  __syncthreads();
  DSL_GRAD_MU(1, 2)
  DSL_GRAD_MU(2, 3)
  DSL_GRAD_MU(3, 0)
#undef DSL_GRAD_MU

  // G of the chunk: c.n * 36 words, contiguous
  {
    constexpr int GP = 36 * int(sizeof(W)) / 16;  // 16-byte pieces per site
    const int pieces = c.n * GP;
    const u32x4* src = reinterpret_cast<const u32x4*>(gout);
    u32x4* dst = reinterpret_cast<u32x4*>(G + size_t(own_base) * 36);
    for (int i = tid; i < pieces; i += nth) __builtin_nontemporal_store(src[i], &dst[i]);
  }
}

template <int OP, int NV, class S, class T>
static hipError_t grad_rows_t(const Geom& g, int R, int bt, const ChunkTiles& o, bool xcd, const void* chi,
                              const void* psi, void* G, hipStream_t st) {
  using W = typename S::word;
  constexpr int COMPS = OP == OP_WILSON ? 12 : 3;
  const RowTraversal tr = make_row_traversal(g, uint32_t(R), uint32_t(bt));
  const dim3 block(NV, R), grid(tr.rows_plane * uint32_t(g.n[2]) * uint32_t(g.n[3]));
  const size_t lds = size_t(R + 1) * Stage<COMPS, NV, S>::SSW * sizeof(W) + size_t(R) * 9 * NV * sizeof(cpx<T>) +
                     size_t(R) * 36 * sizeof(W);
  hipLaunchKernelGGL((grad_rows_kernel<OP, NV, S, T>), grid, block, lds, st, g, tr, o, int(xcd), (const W*)chi,
                     (const W*)psi, (W*)G);
  return hipGetLastError();
}

template <int NV>
static hipError_t grad_rows_nv(int op, int dtype, const Geom& g, int R, int bt, const ChunkTiles& o, bool xcd,
                               const void* chi, const void* psi, void* G, hipStream_t st) {
  if (op == OP_WILSON) return grad_rows_t<OP_WILSON, NV, C64, float>(g, R, bt, o, xcd, chi, psi, G, st);
  if (dtype == DT_C64) return grad_rows_t<OP_STAGGERED, NV, C64, float>(g, R, bt, o, xcd, chi, psi, G, st);
  return grad_rows_t<OP_STAGGERED, NV, C128, double>(g, R, bt, o, xcd, chi, psi, G, st);
}

// Default tile of the D_W gradient: the largest by x bz rows (by | Ny,
// bz | Nz) whose chi and psi at one t take at most 2 MB, the squarer of equal
// sizes.  At 24^3 x 48, N_v = 12 that is 6 x 6: reads 2.1 instead of 3.5 GB
// per launch, 562 against 581-587 us (8 x 3: 2.3 GB, 560 us; 4 x 6: 2.2 GB,
// 569 us; 12 x 2: 2.5 GB, 590 us).  D_S, whose rows are a quarter of the
// size, gained nothing (212 against 206 us) and keeps the t-band order.
static void grad_tile_default(const Geom& g, int R, int nv, int& by, int& bz) {
  pick_tile(g, long((g.n[0] + R - 1) / R) * R * 2L * 12 * nv * 8, 2048L * 1024, by, bz);
}

// Row-staged link gradient for N_v = 4, 8, 12, 16, 24: D_W in C64, D_S in C64
// and C128 (the D_W C128 variant would not fit in registers).  Returns
// hipErrorNotSupported when the configuration is not covered (the caller then
// uses the direct kernel).  DSLASH_ROWS=0 disables it.
hipError_t launch_grad_rows(int op, int dtype, const Geom& g, const void* chi, const void* psi, void* G,
                            hipStream_t st) {
  if (knobs().rows.get(1) == 0) return hipErrorNotSupported;
  if (!aligned16(chi) || !aligned16(psi) || !aligned16(G)) return hipErrorNotSupported;
  const int nv = g.nv;
  if (nv != 4 && nv != 8 && nv != 12 && nv != 16 && nv != 24) return hipErrorNotSupported;
  if (op != OP_WILSON && op != OP_STAGGERED) return hipErrorNotSupported;
  if (dtype != DT_C64 && !(dtype == DT_C128 && op == OP_STAGGERED)) return hipErrorNotSupported;
  int R = row_sites_default(g.n[0], nv);
  R = knobs().row_sites.get(R);
  if (R > g.n[0]) R = g.n[0];
  // 64 .. 256 threads; the +x halo site (CH N_v pieces, CH <= 6) takes one
  // piece per thread at R >= 6
  if (R < 6 || R * nv > 256 || R * nv < 64) return hipErrorNotSupported;
  // t-band of the row traversal: 4 (2: 587 against 578 us for D_W at 24^3 x 48)
  int bt = 4;
  bt = knobs().tband.get(bt);
  bool xcd = true;
  xcd = knobs().xcd.get(xcd) != 0;
  int by = 0, bz = 0;
  if (op == OP_WILSON) grad_tile_default(g, R, nv, by, bz);
  const ChunkTiles o = make_chunk_tiles(g, R, knobs().grad_tile_y.get(by), knobs().grad_tile_z.get(bz));
  switch (nv) {
    case 4: return grad_rows_nv<4>(op, dtype, g, R, bt, o, xcd, chi, psi, G, st);
    case 8: return grad_rows_nv<8>(op, dtype, g, R, bt, o, xcd, chi, psi, G, st);
    case 16: return grad_rows_nv<16>(op, dtype, g, R, bt, o, xcd, chi, psi, G, st);
    case 24: return grad_rows_nv<24>(op, dtype, g, R, bt, o, xcd, chi, psi, G, st);
  }
  return grad_rows_nv<12>(op, dtype, g, R, bt, o, xcd, chi, psi, G, st);
}

}  // namespace dsl
