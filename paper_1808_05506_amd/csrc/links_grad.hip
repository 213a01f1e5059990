// Off-axis link construction (Tab. 1) and link gradients of D_S and D_W.
#include "launch.hpp"
#include "stencils.hpp"

namespace dsl {

// ---------------------------------------------------------------- W build
// Level by level through the first-hop recursion of the path averages (the
// kernels sit with the adjoint of the same recursion).
hipError_t launch_brillouin_links(int dtype, const Geom& g, const void* V, void* W, hipStream_t st) {
  return launch_brillouin_links_levels(dtype, g, V, W, st);
}

// ---------------------------------------------------------------- link gradient
// Thread (site, v) builds its right-hand sides' share of all four G_mu(x) in
// registers; the shares are summed over v through LDS, one mu at a time, and
// G is written once.  No atomics: every output element has one writer.
//
// Wilson, with the rank-2 projections h = P psi of stencils.hpp:
//   G_mu(x) = -1/2 sum_v sum_{t=0,1} [ (P_- chi(x))_t (x) conj((P_- psi(x+mu))_t)
//                                    + (P_+ psi(x))_t (x) conj((P_+ chi(x+mu))_t) ]
// where P_-/P_+ are the c = -1 / c = +1 projections of (1 -/+ gamma_mu): for
// a (1 + c gamma) factor sum_s a_s conj(((1 + c gamma) b)_s) collapses to
// sum_t (P_c a)_t conj((P_c b)_t).
template <int MU, class T>
DSL_HD void wilson_grad_mu(const cpx<T> (&chi)[4][3], const cpx<T> (&psi)[4][3], const cpx<T> (&chif)[4][3],
                           const cpx<T> (&psif)[4][3], cpx<T> (&gm)[3][3]) {
  cpx<T> p1[2][3], q1[2][3], p2[2][3], q2[2][3];
  project<MU, -1, T>(chi, p1);
  project<MU, -1, T>(psif, q1);
  project<MU, +1, T>(psi, p2);
  project<MU, +1, T>(chif, q2);
#pragma unroll
  for (int a = 0; a < 3; ++a)
#pragma unroll
    for (int b = 0; b < 3; ++b) {
      cpx<T> z = gm[a][b];
#pragma unroll
      for (int t = 0; t < 2; ++t) {
        z = cmaddj(z, p1[t][a], q1[t][b]);
        z = cmaddj(z, p2[t][a], q2[t][b]);
      }
      gm[a][b] = z;
    }
}

// This thread's share (right-hand sides v, v + vc, ...) of G_mu(x), all mu,
// before the overall factor (-1/2 for Wilson, eta_mu(x)/2 for staggered).
template <int OP, class S, class T>
DSL_HD void link_grad_partial(const Geom& g, const typename S::word* __restrict__ chi,
                              const typename S::word* __restrict__ psi, uint32_t s, int v0, int vstep,
                              cpx<T> (&gm)[4][3][3]) {
#pragma unroll
  for (int m = 0; m < 4; ++m)
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
      for (int b = 0; b < 3; ++b) gm[m][a][b] = zero<T>();
  const SiteNbr nb = site_nbr(g, s);
  const int nv = g.nv;
  if (OP == OP_WILSON) {
    const size_t sps = size_t(12) * nv;
    for (int v = v0; v < nv; v += vstep) {
      cpx<T> c0[4][3], p0[4][3];
      load_wspinor<S, T>(chi, size_t(s) * sps + v, nv, c0);
      load_wspinor<S, T>(psi, size_t(s) * sps + v, nv, p0);
#define DSL_WGRAD(MU)                                                          \
  {                                                                            \
    cpx<T> cf[4][3], pf[4][3];                                                 \
    const size_t nbase = size_t(s + nb.fwd[MU]) * sps + v;                     \
    load_wspinor<S, T>(chi, nbase, nv, cf);                                    \
    load_wspinor<S, T>(psi, nbase, nv, pf);                                    \
    wilson_grad_mu<MU, T>(c0, p0, cf, pf, gm[MU]);                             \
  }
      DSL_WGRAD(0) DSL_WGRAD(1) DSL_WGRAD(2) DSL_WGRAD(3)
#undef DSL_WGRAD
    }
  } else {
    // D_S: G_mu(x) = eta_mu(x)/2 sum_v [chi(x) (x) conj(psi(x+mu)) - psi(x) (x) conj(chi(x+mu))]
    // (eta_mu(x + mu) = eta_mu(x): eta_mu depends only on x_1..x_{mu-1})
    const size_t sps = size_t(3) * nv;
    for (int v = v0; v < nv; v += vstep) {
      cpx<T> c0[3], p0[3];
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        c0[c] = S::template load<T>(chi + size_t(s) * sps + size_t(c) * nv + v);
        p0[c] = S::template load<T>(psi + size_t(s) * sps + size_t(c) * nv + v);
      }
#pragma unroll
      for (int mu = 0; mu < 4; ++mu) {
        const size_t nbase = size_t(s + nb.fwd[mu]) * sps + v;
        cpx<T> cf[3], pf[3];
#pragma unroll
        for (int c = 0; c < 3; ++c) {
          cf[c] = S::template load<T>(chi + nbase + size_t(c) * nv);
          pf[c] = S::template load<T>(psi + nbase + size_t(c) * nv);
        }
#pragma unroll
        for (int a = 0; a < 3; ++a)
#pragma unroll
          for (int b = 0; b < 3; ++b) {
            gm[mu][a][b] = cmaddj(gm[mu][a][b], c0[a], pf[b]);
            gm[mu][a][b] = cmaddj(gm[mu][a][b], -p0[a], cf[b]);
          }
      }
    }
  }
}

// Overall factor of G_mu at site s.
template <int OP, class T>
DSL_HD T link_grad_factor(const Geom& g, uint32_t s, int mu) {
  if (OP == OP_WILSON) return T(-0.5);
  const SiteNbr nb = site_nbr(g, s);
  int pp = 0;
  for (int nu = 0; nu < mu; ++nu) pp += nb.c[nu];
  return (pp & 1) ? T(-0.5) : T(0.5);
}

template <int OP, class S, class T>
__global__ void __launch_bounds__(256) link_grad_kernel(Geom g, const typename S::word* __restrict__ chi,
                                                        const typename S::word* __restrict__ psi,
                                                        typename S::word* __restrict__ G) {
  extern __shared__ unsigned char smem_raw[];
  cpx<T>* red = reinterpret_cast<cpx<T>*>(smem_raw);  // [sites][9][vc]
  const int vc = blockDim.x, sb = blockDim.y;
  const uint32_t lb = xcd_block(blockIdx.x, gridDim.x);
  const uint32_t s = lb * sb + threadIdx.y;
  cpx<T> gm[4][3][3];
  if (s < g.vol) {
    link_grad_partial<OP, S, T>(g, chi, psi, s, threadIdx.x, vc, gm);
  } else {
#pragma unroll
    for (int m = 0; m < 4; ++m)
#pragma unroll
      for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int b = 0; b < 3; ++b) gm[m][a][b] = zero<T>();
  }

  const int tid = threadIdx.y * vc + threadIdx.x;
  const int nthr = vc * sb;
#pragma unroll
  for (int mu = 0; mu < 4; ++mu) {
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
      for (int b = 0; b < 3; ++b) red[(threadIdx.y * 9 + a * 3 + b) * vc + threadIdx.x] = gm[mu][a][b];
    __syncthreads();
    for (int o = tid; o < sb * 9; o += nthr) {
      const int sl = o / 9, e = o - sl * 9;
      const uint32_t so = lb * sb + sl;
      if (so < g.vol) {
        cpx<T> z = zero<T>();
        for (int l = 0; l < vc; ++l) z += red[(sl * 9 + e) * vc + l];
        const T f = link_grad_factor<OP, T>(g, so, mu);
        S::template store<T>(G + (size_t(so) * 4 + mu) * 9 + e, f * z);
      }
    }
    __syncthreads();
  }
}

hipError_t launch_link_grad(int op, int dtype, const Geom& g, const void* chi, const void* psi, void* G,
                            hipStream_t st) {
  const hipError_t rows = launch_grad_rows(op, dtype, g, chi, psi, G, st);
  if (rows != hipErrorNotSupported || knobs().rows.get(1) == 2) return rows;
  Shape sh = site_v_shape(g.vol, g.nv);
  sh.grid.y = 1;  // one block covers every right-hand side of its sites
  const size_t csz = dtype == DT_C128 ? 16 : 8;
  const size_t lds = size_t(sh.block.x) * sh.block.y * 9 * csz;
  if (op == OP_WILSON && dtype == DT_C64)
    hipLaunchKernelGGL((link_grad_kernel<OP_WILSON, C64, float>), sh.grid, sh.block, lds, st, g,
                       (const float2*)chi, (const float2*)psi, (float2*)G);
  else if (op == OP_WILSON && dtype == DT_C128)
    hipLaunchKernelGGL((link_grad_kernel<OP_WILSON, C128, double>), sh.grid, sh.block, lds, st, g,
                       (const double2*)chi, (const double2*)psi, (double2*)G);
  else if (op == OP_STAGGERED && dtype == DT_C64)
    hipLaunchKernelGGL((link_grad_kernel<OP_STAGGERED, C64, float>), sh.grid, sh.block, lds, st, g,
                       (const float2*)chi, (const float2*)psi, (float2*)G);
  else if (op == OP_STAGGERED && dtype == DT_C128)
    hipLaunchKernelGGL((link_grad_kernel<OP_STAGGERED, C128, double>), sh.grid, sh.block, lds, st, g,
                       (const double2*)chi, (const double2*)psi, (double2*)G);
  else
    return hipErrorInvalidValue;
  return hipGetLastError();
}

}  // namespace dsl
