// Dirac-operator application kernels: D_S, D_W, D_B and their adjoints, in
// every storage type.  One thread per (site, right-hand side); see stencils.hpp.
#include <stdlib.h>

#include "launch.hpp"
#include "stencils.hpp"

namespace dsl {

Geom make_geom(const int dims[4], int nv) {
  Geom g;
  for (int i = 0; i < 4; ++i) g.n[i] = dims[i];
  g.stride[0] = 1;
  g.stride[1] = dims[0];
  g.stride[2] = dims[0] * dims[1];
  g.stride[3] = dims[0] * dims[1] * dims[2];
  g.vol = uint32_t(dims[0]) * dims[1] * dims[2] * dims[3];
  g.nv = nv;
  g.dx = FastDiv::make(dims[0]);
  g.dy = FastDiv::make(dims[1]);
  g.dz = FastDiv::make(dims[2]);
  return g;
}

static int gcd_int(int a, int b) {
  while (b) {
    int t = a % b;
    a = b;
    b = t;
  }
  return a;
}

// Lanes: right-hand sides fastest (blockDim.x = min(nv, 64)), sites along
// blockDim.y.  The block holds whole waves when lcm(vc, 64) <= 256 and at
// most 256 threads.  DSLASH_SITES_PER_BLOCK overrides the site count (tuning).
Shape site_v_shape(uint32_t vol, int nv) {
  const int vc = nv < 64 ? nv : 64;
  const int l = vc / gcd_int(vc, 64) * 64;
  int sb = l <= 256 ? l / vc : (256 / vc > 0 ? 256 / vc : 1);
  while (vc * sb * 2 <= 256 && l <= 256) sb *= 2;
  if (knobs().sites_per_block.set) {
    const int v = knobs().sites_per_block.value;
    if (v > 0 && v * vc <= 256) sb = v;  // kernels are built for at most 256 threads
  }
  Shape sh;
  sh.block = dim3(vc, sb, 1);
  sh.grid = dim3((vol + sb - 1) / sb, (nv + vc - 1) / vc, 1);
  return sh;
}

// Launch configuration of the (site, right-hand side) kernels: thread shape,
// row-chunk traversal (used when one x-row chunk fills at least two waves),
// and whether workgroups are regrouped per XCD.  DSLASH_TBAND (t-band width,
// default 8) and DSLASH_XCD (0/1, default 1) are tuning overrides.
struct Launch {
  Shape sh;
  bool rows;
  bool xcd;
  RowTraversal tr;
};

static Launch make_launch(const Geom& g) {
  Launch L;
  L.sh = site_v_shape(g.vol, g.nv);
  const uint32_t vc = L.sh.block.x;
  uint32_t sb = L.sh.block.y;
  if (sb > uint32_t(g.n[0])) sb = g.n[0];
  L.rows = sb * vc >= 128;
  int bt = 8;
  bt = knobs().tband.get(bt);
  L.xcd = true;
  L.xcd = knobs().xcd.get(1) != 0;
  if (L.rows) {
    L.tr = make_row_traversal(g, sb, uint32_t(bt > 0 ? bt : 1));
    L.sh.block.y = sb;
    L.sh.grid.x = L.tr.rows_plane * uint32_t(g.n[2]) * uint32_t(g.n[3]);
  }
  return L;
}

// NV1: N_v = 1 known at compile time, with 16-byte aligned fields (the
// launcher checks), so a site's spinor (12 words) and links are contiguous
// runs that the compiler loads as 16-byte pieces.
template <int OP, bool ADJ, class S, class T, int LW, bool NV1 = false>
__global__ void __launch_bounds__(256) apply_kernel(Geom g, RowTraversal tr, int rows, int xcd,
                                                   const typename S::word* __restrict__ U,
                                                   const typename S::word* __restrict__ in,
                                                   typename S::word* __restrict__ out,
                                                   const typename S::word* __restrict__ C, T mass) {
  using W = typename S::word;
  if constexpr (NV1) {
    U = static_cast<const W*>(__builtin_assume_aligned(U, 16));
    in = static_cast<const W*>(__builtin_assume_aligned(in, 16));
    out = static_cast<W*>(__builtin_assume_aligned(out, 16));
  }
  const uint32_t lb = xcd_block(blockIdx.x, gridDim.x, xcd != 0);
  const int v = NV1 ? 0 : int(blockIdx.y * blockDim.x + threadIdx.x);
  uint32_t s;
  bool live;
  SiteNbr nb;
  if (rows) {
    nb = row_site(g, tr, lb, threadIdx.y, s, live);
  } else {
    s = lb * blockDim.y + threadIdx.y;
    live = s < g.vol;
    if (live) nb = site_nbr(g, s);
  }
  if (!live || v >= g.nv) return;
  if (OP == OP_STAGGERED)
    staggered_site<ADJ, S, T, LW, NV1 ? 1 : 0>(g, U, in, out, s, nb, v, mass);
  else if (OP == OP_WILSON)
    wilson_site<ADJ, S, T, LW, NV1 ? 1 : 0>(g, U, in, out, C, s, nb, v, T(4) + mass);
  else
    brillouin_site<ADJ, S, T>(g, U, in, out, C, s, nb, v, mass + T(15.0 / 8.0));
}

template <int OP, class S, class T>
static hipError_t apply_t(bool adj, const Geom& g, const void* U, const void* in, void* out, const void* C,
                          double mass, bool compressed, hipStream_t st) {
  using W = typename S::word;
  const Launch L = make_launch(g);
#define DSL_AK(A, LW, V1)                                                                                        \
  hipLaunchKernelGGL((apply_kernel<OP, A, S, T, LW, V1>), L.sh.grid, L.sh.block, 0, st, g, L.tr, int(L.rows), \
                     int(L.xcd), (const W*)U, (const W*)in, (W*)out, (const W*)C, T(mass))
  if constexpr (OP == OP_WILSON) {
    // N_v = 1 with 16-byte aligned fields: the contiguous-load form of D_W
    // (32^4: 261 against 598 us).  D_S keeps the per-word form, which its
    // 3-word spinors do not let the compiler merge (231 against 216 us).
    if (g.nv == 1 && !C && aligned16(U) && aligned16(in) && aligned16(out)) {
      if (compressed) {
        if (adj) DSL_AK(true, 6, true); else DSL_AK(false, 6, true);
      } else {
        if (adj) DSL_AK(true, 9, true); else DSL_AK(false, 9, true);
      }
      return hipGetLastError();
    }
  }
  if constexpr (OP != OP_BRILLOUIN) {
    if (compressed) {
      if (adj) DSL_AK(true, 6, false); else DSL_AK(false, 6, false);
      return hipGetLastError();
    }
  }
  if (adj) DSL_AK(true, 9, false); else DSL_AK(false, 9, false);
#undef DSL_AK
  return hipGetLastError();
}

template <int OP>
static hipError_t apply_op(bool adj, int dtype, const Geom& g, const void* U, const void* in, void* out,
                           const void* C, double mass, bool compressed, hipStream_t st) {
  switch (dtype) {
    case DT_C64: return apply_t<OP, C64, float>(adj, g, U, in, out, C, mass, compressed, st);
    case DT_C128: return apply_t<OP, C128, double>(adj, g, U, in, out, C, mass, compressed, st);
    case DT_BF16: return apply_t<OP, BF16, float>(adj, g, U, in, out, C, mass, compressed, st);
    case DT_F16: return apply_t<OP, F16, float>(adj, g, U, in, out, C, mass, compressed, st);
  }
  return hipErrorInvalidValue;
}

// DSLASH_ROWS: 0 the direct kernels only, 1 (default) the row-staged kernel
// where it covers the configuration and the direct one elsewhere, 2 the
// row-staged kernel or hipErrorNotSupported (to test that a configuration
// takes it).
hipError_t launch_apply(int op, bool adj, int dtype, const Geom& g, const void* U, const void* in, void* out,
                        double mass, hipStream_t st, const void* clover, bool compressed) {
  const bool rows_only = knobs().rows.get(1) == 2;
  switch (op) {
    case OP_STAGGERED: {
      if (clover) return hipErrorInvalidValue;
      const hipError_t e = launch_staggered_rows(adj, dtype, g, U, in, out, mass, st, compressed);
      if (e != hipErrorNotSupported || rows_only) return e;
      return apply_op<OP_STAGGERED>(adj, dtype, g, U, in, out, nullptr, mass, compressed, st);
    }
    case OP_WILSON: {
      if (clover && compressed) return hipErrorInvalidValue;
      const hipError_t e = launch_wilson_rows(adj, dtype, g, U, in, out, mass, st, clover, compressed);
      if (e != hipErrorNotSupported || rows_only) return e;
      return apply_op<OP_WILSON>(adj, dtype, g, U, in, out, clover, mass, compressed, st);
    }
    case OP_BRILLOUIN: {
      if (compressed) return hipErrorInvalidValue;
      const hipError_t e = launch_brillouin_rows(adj, dtype, g, U, in, out, mass, st, clover);
      if (e != hipErrorNotSupported || rows_only) return e;
      return apply_op<OP_BRILLOUIN>(adj, dtype, g, U, in, out, clover, mass, false, st);
    }
  }
  return hipErrorInvalidValue;
}

}  // namespace dsl
