// Link gradients of the Brillouin operator.
//
// bri_wgrad_kernel: gradient of L = Re sum conj(chi) (D_B psi) with respect to
// the 40 stored W, taken as free complex matrices.  W_d(x) (d stored) enters
// the hop of d into out(x) with spin factor S_d = a_k + b_k d.gamma
// (a_k = -lambda_k / 2, b_k = rho_k; eqs. def_der, def_lap) and, as
// W_{-d}(x + d) = W_d(x)^dag (Tab. 1 caption), the hop of -d into out(x + d)
// with S_{-d} = a_k - b_k d.gamma.  S_d is Hermitian, so
//   G_{W_d}(x) = sum_v sum_s [ (S_d chi(x))_s (x) conj(psi(x+d)_s)
//                            + psi(x)_s (x) conj((S_{-d} chi(x+d))_s) ].
// A block handles one stored direction for a run of sites; the N_v lanes of a
// site each take their right-hand sides and the shares are summed through LDS.
//
// bri_links_backward_kernel: the adjoint of the construction of W from V
// (Tab. 1).  W_d(x) is the mean over the k! hop orderings of the path product
// M = A_1 ... A_k (A_i = V_mu(y) for a hop +mu from y, V_mu(y - mu)^dag for a
// hop -mu); for the gradient G of a path product, hop i receives
// P^dag G Q^dag with P, Q the products before and after it, or the adjoint of
// that when the hop runs against the link.  One thread per link (y, mu) gathers
// every (d, ordering, hop) that uses it, in a fixed order: the sum is
// deterministic and needs no atomics.  bri_links_backward_w_kernel sums the
// orderings that share the hops around the link through the path averages of
// W instead.
//
// bri_wlevel_*: the same adjoint through the recursion of the path averages
// by their first hop, level by level (the default when W is given), and
// bri_links_level_kernel: the construction of W itself by that recursion.
#include "launch.hpp"
#include "stencils.hpp"

namespace dsl {
namespace {

// out = (d.gamma) y in the chiral basis: d.gamma = [[0, S], [S^dag, 0]],
// S = [[d4 - i d3, -d2 - i d1], [d2 - i d1, d4 + i d3]].
template <class T>
DSL_HD void dgamma(const int (&d)[4], const cpx<T> (&y)[4][3], cpx<T> (&out)[4][3]) {
  const T d1 = T(d[0]), d2 = T(d[1]), d3 = T(d[2]), d4 = T(d[3]);
  const cpx<T> s00 = mk(d4, -d3), s01 = mk(-d2, -d1), s10 = mk(d2, -d1), s11 = mk(d4, d3);
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    out[0][c] = cmadd(cmadd(zero<T>(), s00, y[2][c]), s01, y[3][c]);
    out[1][c] = cmadd(cmadd(zero<T>(), s10, y[2][c]), s11, y[3][c]);
    // S^dag: rows (conj s00, conj s10), (conj s01, conj s11)
    out[2][c] = cjmadd(cjmadd(zero<T>(), s00, y[0][c]), s10, y[1][c]);
    out[3][c] = cjmadd(cjmadd(zero<T>(), s01, y[0][c]), s11, y[1][c]);
  }
}

// r = a^dag b
template <class T>
DSL_HD void m3_adj_mul(const cpx<T> (&a)[3][3], const cpx<T> (&b)[3][3], cpx<T> (&r)[3][3]) {
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      cpx<T> z = zero<T>();
#pragma unroll
      for (int k = 0; k < 3; ++k) z = cjmadd(z, a[k][i], b[k][j]);
      r[i][j] = z;
    }
}

// r = a b^dag
template <class T>
DSL_HD void m3_mul_adj(const cpx<T> (&a)[3][3], const cpx<T> (&b)[3][3], cpx<T> (&r)[3][3]) {
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      cpx<T> z = zero<T>();
#pragma unroll
      for (int k = 0; k < 3; ++k) z = cmaddj(z, a[i][k], b[j][k]);
      r[i][j] = z;
    }
}

template <class T>
DSL_HD void m3_identity(cpx<T> (&m)[3][3]) {
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) m[i][j] = i == j ? mk(T(1), T(0)) : zero<T>();
}

DSL_HD uint32_t site_of(const Geom& g, const int (&p)[4]) {
  return uint32_t(p[0] + g.stride[1] * p[1] + g.stride[2] * p[2] + g.stride[3] * p[3]);
}

DSL_HD int wrap(int x, int n) { return x < 0 ? x + n : (x >= n ? x - n : x); }

// Permutation `code` (0 .. 23, factorial number system) of {0, 1, 2, 3}.
DSL_HD void decode_perm(int code, int (&perm)[4]) {
  int avail[4] = {0, 1, 2, 3};
  int rem = code;
  const int fact[4] = {6, 2, 1, 1};
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int q = rem / fact[i];
    rem -= q * fact[i];
    perm[i] = avail[q];
#pragma unroll
    for (int t = 0; t < 3; ++t)
      if (t >= q) avail[t] = avail[t + 1];
  }
}

}  // namespace

// Block (VB, SB): lane x takes the right-hand sides v = x, x + VB, ... of
// site y (so the VB lanes of a site read consecutive words of every spinor
// component), accumulates its share of G_{W_d}, and the shares are summed over
// the lanes through LDS in a fixed order.  blockIdx.y = stored slot.
template <class S, class T>
__global__ void __launch_bounds__(256) bri_wgrad_kernel(Geom g, const typename S::word* __restrict__ chi,
                                                       const typename S::word* __restrict__ psi,
                                                       typename S::word* __restrict__ GW) {
  extern __shared__ unsigned char smem_wgrad[];
  T* red = reinterpret_cast<T*>(smem_wgrad);  // [SB][18][VB]
  const int VB = int(blockDim.x), SB = int(blockDim.y);
  const int lane = int(threadIdx.x), sl = int(threadIdx.y);
  const uint32_t s0 = blockIdx.x * uint32_t(SB);
  const uint32_t s = s0 + uint32_t(sl);
  const int j = int(blockIdx.y);  // stored slot, uniform over the block
  int d[4];
  stored_direction(j, d);
  const int k = (d[0] != 0) + (d[1] != 0) + (d[2] != 0) + (d[3] != 0);
  const T a = T(-0.5) * bri_lambda<T>(k), b = bri_rho<T>(k);
  const int nv = g.nv;
  const size_t sps = size_t(12) * nv;

  cpx<T> G[3][3];
#pragma unroll
  for (int r = 0; r < 3; ++r)
#pragma unroll
    for (int c = 0; c < 3; ++c) G[r][c] = zero<T>();
  if (s < g.vol) {
    const SiteNbr nb = site_nbr(g, s);
    int q[4] = {nb.c[0], nb.c[1], nb.c[2], nb.c[3]};
#pragma unroll
    for (int mu = 0; mu < 4; ++mu) q[mu] = wrap(q[mu] + d[mu], g.n[mu]);
    const uint32_t sd = site_of(g, q);
#pragma unroll 1
    for (int v = lane; v < nv; v += VB) {
      cpx<T> cx[4][3], cd[4][3], px[4][3], pd[4][3];
      load_wspinor<S, T>(chi, size_t(s) * sps + v, nv, cx);
      load_wspinor<S, T>(chi, size_t(sd) * sps + v, nv, cd);
      load_wspinor<S, T>(psi, size_t(s) * sps + v, nv, px);
      load_wspinor<S, T>(psi, size_t(sd) * sps + v, nv, pd);
      // af = S_d chi(x) = a chi(x) + b (d.gamma) chi(x); ab = S_{-d} chi(x+d) = a chi(x+d) - b (d.gamma) chi(x+d)
      cpx<T> af[4][3], ab[4][3];
      dgamma<T>(d, cx, af);
      dgamma<T>(d, cd, ab);
#pragma unroll
      for (int sp = 0; sp < 4; ++sp)
#pragma unroll
        for (int c = 0; c < 3; ++c) {
          af[sp][c] = rmadd(b * af[sp][c], a, cx[sp][c]);
          ab[sp][c] = rmadd((-b) * ab[sp][c], a, cd[sp][c]);
        }
#pragma unroll
      for (int sp = 0; sp < 4; ++sp)
#pragma unroll
        for (int r = 0; r < 3; ++r)
#pragma unroll
          for (int c = 0; c < 3; ++c) {
            G[r][c] = cmaddj(G[r][c], af[sp][r], pd[sp][c]);
            G[r][c] = cmaddj(G[r][c], px[sp][r], ab[sp][c]);
          }
    }
  }
  // shares of the VB lanes of each site, summed in lane order
  T* mine = red + size_t(sl) * 18 * VB + lane;
#pragma unroll
  for (int r = 0; r < 3; ++r)
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      mine[(2 * (r * 3 + c)) * VB] = G[r][c].r;
      mine[(2 * (r * 3 + c) + 1) * VB] = G[r][c].i;
    }
  __syncthreads();
  const int nthr = VB * SB;
  for (int t = sl * VB + lane; t < SB * 9; t += nthr) {
    const int site = t / 9, e = t - site * 9;
    if (s0 + uint32_t(site) >= g.vol) continue;
    const T* src = red + size_t(site) * 18 * VB;
    T re = T(0), im = T(0);
    for (int l = 0; l < VB; ++l) {
      re += src[(2 * e) * VB + l];
      im += src[(2 * e + 1) * VB + l];
    }
    S::template store<T>(GW + ((size_t(s0) + site) * 40 + j) * 9 + e, mk(re, im));
  }
}

template <class S, class T>
__global__ void __launch_bounds__(128) bri_links_backward_kernel(Geom g, const typename S::word* __restrict__ V,
                                                                const typename S::word* __restrict__ GW,
                                                                typename S::word* __restrict__ GV) {
  const uint32_t y = blockIdx.x * blockDim.x + threadIdx.x;
  const int mu = int(blockIdx.y);  // link direction, uniform over the block
  if (y >= g.vol) return;
  const SiteNbr nb = site_nbr(g, y);
  cpx<T> acc[3][3];
#pragma unroll
  for (int r = 0; r < 3; ++r)
#pragma unroll
    for (int c = 0; c < 3; ++c) acc[r][c] = zero<T>();

#pragma unroll 1
  for (int j = 0; j < 40; ++j) {
    int d[4];
    stored_direction(j, d);
    if (d[mu] == 0) continue;  // uniform: j and mu are the same for the whole wave
    int axes[4], k = 0;
#pragma unroll
    for (int nu = 0; nu < 4; ++nu)
      if (d[nu] != 0) axes[k++] = nu;
    const int nperm = k == 1 ? 1 : (k == 2 ? 2 : (k == 3 ? 6 : 24));
    const T inv = T(1) / T(nperm);
    const int sg = d[mu];
#pragma unroll 1
    for (int code = 0; code < 24; ++code) {
      int perm[4];
      decode_perm(code, perm);
      bool keep = true;
#pragma unroll
      for (int i = 0; i < 4; ++i)
        if (i >= k && perm[i] != i) keep = false;
      if (!keep) continue;
      // position of the mu hop in this ordering
      int ih = 0;
#pragma unroll
      for (int i = 0; i < 4; ++i)
        if (i < k && axes[perm[i]] == mu) ih = i;
      // the hop starts at y (forward) or at y + mu (backward); the path starts
      // at x = start - (hops before it)
      int x[4] = {nb.c[0], nb.c[1], nb.c[2], nb.c[3]};
      if (sg < 0) x[mu] = wrap(x[mu] + 1, g.n[mu]);
#pragma unroll
      for (int i = 0; i < 4; ++i)
        if (i < ih) {
          const int nu = axes[perm[i]];
          x[nu] = wrap(x[nu] - d[nu], g.n[nu]);
        }
      const uint32_t xs = site_of(g, x);
      // P = product of the hops before ih, walked from x
      int pos[4] = {x[0], x[1], x[2], x[3]};
      cpx<T> P[3][3], L[3][3], Tm[3][3];
      m3_identity(P);
#pragma unroll 1
      for (int i = 0; i < ih; ++i) {
        const int nu = axes[perm[i]];
        path_hop<S, T>(g, V, pos, nu, d[nu], L);
        path_mul(P, L, Tm);
#pragma unroll
        for (int r = 0; r < 3; ++r)
#pragma unroll
          for (int c = 0; c < 3; ++c) P[r][c] = Tm[r][c];
      }
      // step over the mu hop itself
      pos[mu] = wrap(pos[mu] + sg, g.n[mu]);
      // Q = product of the hops after ih
      cpx<T> Q[3][3];
      m3_identity(Q);
#pragma unroll 1
      for (int i = ih + 1; i < k; ++i) {
        const int nu = axes[perm[i]];
        path_hop<S, T>(g, V, pos, nu, d[nu], L);
        path_mul(Q, L, Tm);
#pragma unroll
        for (int r = 0; r < 3; ++r)
#pragma unroll
          for (int c = 0; c < 3; ++c) Q[r][c] = Tm[r][c];
      }
      // X = P^dag G Q^dag
      cpx<T> Gm[3][3];
      load_link<S, T>(GW, (size_t(xs) * 40 + j) * 9, Gm);
      m3_adj_mul(P, Gm, Tm);
      m3_mul_adj(Tm, Q, L);
      if (sg > 0) {
#pragma unroll
        for (int r = 0; r < 3; ++r)
#pragma unroll
          for (int c = 0; c < 3; ++c) acc[r][c] = rmadd(acc[r][c], inv, L[r][c]);
      } else {
#pragma unroll
        for (int r = 0; r < 3; ++r)
#pragma unroll
          for (int c = 0; c < 3; ++c) acc[r][c] = rmadd(acc[r][c], inv, conj(L[c][r]));
      }
    }
  }
  typename S::word* o = GV + (size_t(y) * 4 + mu) * 9;
#pragma unroll
  for (int r = 0; r < 3; ++r)
#pragma unroll
    for (int c = 0; c < 3; ++c) S::template store<T>(o + r * 3 + c, acc[r][c]);
}

// W_{dd}(x) for any displacement dd in {-1, 0, 1}^4: the stored W_dd(x), or
// W_{-dd}(x + dd)^dag (Tab. 1 caption) for the other 40, or 1 for dd = 0.
template <class S, class T>
DSL_HD void load_w_any(const Geom& g, const typename S::word* __restrict__ W, const int (&x)[4], const int (&dd)[4],
                       cpx<T> (&w)[3][3]) {
  const int n = (dd[0] + 1) + 3 * (dd[1] + 1) + 9 * (dd[2] + 1) + 27 * (dd[3] + 1);
  if (n == 40) {
    m3_identity(w);
  } else if (n > 40) {
    load_link<S, T>(W, (size_t(site_of(g, x)) * 40 + (n - 41)) * 9, w);
  } else {
    int y[4];
#pragma unroll
    for (int mu = 0; mu < 4; ++mu) y[mu] = wrap(x[mu] + dd[mu], g.n[mu]);
    cpx<T> t[3][3];
    load_link<S, T>(W, (size_t(site_of(g, y)) * 40 + (39 - n)) * 9, t);
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
      for (int b = 0; b < 3; ++b) w[a][b] = conj(t[b][a]);
  }
}

// The adjoint of the W construction with the path averages of W itself.  The
// hop along mu sits in the k! orderings of d behind the hops of a subset S of
// d's other axes (in any order) and before the rest R; summed over those
// orderings the products before and after it are |S|! W_{e_S}(x) and
// |R|! W_{e_R}(z), the path averages of the sub-displacements (x the path's
// start, z the site after the hop).  So
//   G_V = sum_d sum_S |S|! |R|! / k! W_{e_S}(x)^dag G_{W_d}(x) W_{e_R}(z)^dag,
// adjoint for a hop against the link: 2^(k-1) terms per direction instead of
// k! walks of up to k - 1 links.  W: the stored off-axis links of V.
template <class S, class T>
__global__ void __launch_bounds__(128) bri_links_backward_w_kernel(Geom g, const typename S::word* __restrict__ W,
                                                                  const typename S::word* __restrict__ GW,
                                                                  typename S::word* __restrict__ GV) {
  const uint32_t y = blockIdx.x * blockDim.x + threadIdx.x;
  const int mu = int(blockIdx.y);  // link direction, uniform over the block
  if (y >= g.vol) return;
  const SiteNbr nb = site_nbr(g, y);
  cpx<T> acc[3][3];
#pragma unroll
  for (int r = 0; r < 3; ++r)
#pragma unroll
    for (int c = 0; c < 3; ++c) acc[r][c] = zero<T>();
  const int fact[5] = {1, 1, 2, 6, 24};

#pragma unroll 1
  for (int j = 0; j < 40; ++j) {
    int d[4];
    stored_direction(j, d);
    if (d[mu] == 0) continue;  // uniform: j and mu are the same for the whole wave
    const int sg = d[mu];
    int other[3], no = 0;
#pragma unroll
    for (int nu = 0; nu < 4; ++nu)
      if (nu != mu && d[nu] != 0) other[no++] = nu;
    const int k = no + 1;
    // the hop starts at y (forward) or at y + mu (against the link); it ends at z
    int h[4] = {nb.c[0], nb.c[1], nb.c[2], nb.c[3]}, z[4] = {nb.c[0], nb.c[1], nb.c[2], nb.c[3]};
    if (sg < 0) h[mu] = wrap(h[mu] + 1, g.n[mu]);
    else z[mu] = wrap(z[mu] + 1, g.n[mu]);
#pragma unroll 1
    for (int mask = 0; mask < (1 << no); ++mask) {
      int eS[4] = {0, 0, 0, 0}, eR[4] = {0, 0, 0, 0}, ns = 0;
#pragma unroll
      for (int i = 0; i < 3; ++i) {
        if (i >= no) continue;
        const int nu = other[i];
        if (mask & (1 << i)) {
          eS[nu] = d[nu];
          ++ns;
        } else {
          eR[nu] = d[nu];
        }
      }
      int x[4];
#pragma unroll
      for (int nu = 0; nu < 4; ++nu) x[nu] = wrap(h[nu] - eS[nu], g.n[nu]);
      const T coef = T(fact[ns] * fact[no - ns]) / T(fact[k]);
      // an empty S or R is the identity: its product is skipped (mask is
      // uniform over the wave)
      cpx<T> X[3][3], Tm[3][3];
      load_link<S, T>(GW, (size_t(site_of(g, x)) * 40 + j) * 9, X);
      if (ns > 0) {
        cpx<T> WS[3][3];
        load_w_any<S, T>(g, W, x, eS, WS);
        m3_adj_mul(WS, X, Tm);
#pragma unroll
        for (int r = 0; r < 3; ++r)
#pragma unroll
          for (int c = 0; c < 3; ++c) X[r][c] = Tm[r][c];
      }
      if (ns < no) {
        cpx<T> WR[3][3];
        load_w_any<S, T>(g, W, z, eR, WR);
        m3_mul_adj(X, WR, Tm);
#pragma unroll
        for (int r = 0; r < 3; ++r)
#pragma unroll
          for (int c = 0; c < 3; ++c) X[r][c] = Tm[r][c];
      }
      if (sg > 0) {
#pragma unroll
        for (int r = 0; r < 3; ++r)
#pragma unroll
          for (int c = 0; c < 3; ++c) acc[r][c] = rmadd(acc[r][c], coef, X[r][c]);
      } else {
#pragma unroll
        for (int r = 0; r < 3; ++r)
#pragma unroll
          for (int c = 0; c < 3; ++c) acc[r][c] = rmadd(acc[r][c], coef, conj(X[c][r]));
      }
    }
  }
  typename S::word* o = GV + (size_t(y) * 4 + mu) * 9;
#pragma unroll
  for (int r = 0; r < 3; ++r)
#pragma unroll
    for (int c = 0; c < 3; ++c) S::template store<T>(o + r * 3 + c, acc[r][c]);
}

// ---------------------------------------------------------------- adjoint of the W construction by levels
// Grouping the k! orderings of a path by their first hop gives the recursion
//   W_d(x) = (1/k) sum_{mu: d_mu != 0} A_{s mu}(x) W_{d - s mu}(x + s mu),   s = d_mu,
// with W_0 = 1 and A_{+mu}(x) = V_mu(x), A_{-mu}(x) = V_mu(x - mu)^dag (Tab. 1).
// Reverse mode through it, from the four-hop directions down: the total
// gradient T_e of a stored direction e (k hops) is its operator gradient plus
// what the stored (k + 1)-hop directions pass down to it:
//   d = e + s mu stored, at x = x' - s mu:   (1/(k+1)) A_{s mu}(x)^dag T_d(x)
//   d = -e + s mu stored, at x = x' - d:     (1/(k+1)) T_d(x)^dag A_{s mu}(x)
// (the second because d's sub-direction -e is not stored: W_{-e}(x' + e) =
// W_e(x')^dag).  Then
//   G_V(y, mu) = sum_{stored d, d_mu = +1} (1/k) T_d(y) W_{d - mu}(y + mu)^dag
//              + sum_{stored d, d_mu = -1} [(1/k) T_d(y + mu) W_{d + mu}(y)^dag]^dag.
// Every sum is a gather in a fixed order (deterministic, no atomics); about
// 210 matrix products per site against about 1000 for the sums over orderings.

namespace {

// The workspace holds the totals, W and V as structures of arrays: word e of
// slot j at site x sits at [(j * 9 + e) * vol + x], so the lanes of a wave
// (consecutive sites) read consecutive words and the shifted gathers of the
// recursion stay contiguous; the inputs' [site][slot][9] layout would put each
// lane's matrix in other cache lines.

// The stored slots j of one level k (number of non-zero components).
struct LevelSlots {
  int n;
  int j[16];
};

constexpr int kSoaBlock = 256;

// dst[w * vol + x] = src[x * wps + w] for the wps words of every site: a block
// reads the contiguous words of its sites (16-byte loads, four in flight per
// lane, when VEC) and writes runs of consecutive sites through LDS (row stride
// wps + 1 words against bank conflicts).
template <class S, bool VEC>
__global__ void __launch_bounds__(kSoaBlock) bri_aos_to_soa_kernel(const typename S::word* __restrict__ src,
                                                                   typename S::word* __restrict__ dst, uint32_t vol,
                                                                   int wps, int sb) {
  using W = typename S::word;
  constexpr int WPC = VEC ? 16 / int(sizeof(W)) : 1;  // words a load
  extern __shared__ unsigned char smem_soa[];
  W* tile = reinterpret_cast<W*>(smem_soa);
  const uint32_t x0 = blockIdx.x * uint32_t(sb);
  const int ns = int(min(uint32_t(sb), vol - x0));
  const int tid = int(threadIdx.x);
  const W* in = src + size_t(x0) * wps;
  const int nch = ns * wps / WPC;  // wps * sizeof(W) is a multiple of 16 when VEC
  for (int t0 = 0; t0 < nch; t0 += 4 * kSoaBlock) {
    W r[4][WPC];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int t = t0 + u * kSoaBlock + tid;
      if (t < nch) {
        if constexpr (VEC) {
          const uint4 q = reinterpret_cast<const uint4*>(in)[t];
          __builtin_memcpy(&r[u][0], &q, 16);
        } else {
          r[u][0] = in[t];
        }
      }
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int t = t0 + u * kSoaBlock + tid;
      if (t < nch) {
#pragma unroll
        for (int h = 0; h < WPC; ++h) {
          const int wi = t * WPC + h, xl = wi / wps, w = wi - xl * wps;
          tile[xl * (wps + 1) + w] = r[u][h];
        }
      }
    }
  }
  __syncthreads();
#pragma unroll 4
  for (int t = tid; t < sb * wps; t += kSoaBlock) {
    const int w = t / sb, xl = t - w * sb;
    if (xl < ns) dst[size_t(w) * vol + x0 + xl] = tile[xl * (wps + 1) + w];
  }
}

template <class S, class T>
__device__ __forceinline__ void soa_load(const typename S::word* __restrict__ p, uint32_t vol, uint32_t x,
                                         cpx<T> (&m)[3][3]) {
#pragma unroll
  for (int r = 0; r < 3; ++r)
#pragma unroll
    for (int c = 0; c < 3; ++c) m[r][c] = S::template load<T>(p + size_t(r * 3 + c) * vol + x);
}

template <class T>
__device__ __forceinline__ void dagger_in_place(cpx<T> (&m)[3][3]) {
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    m[a][a] = conj(m[a][a]);
#pragma unroll
    for (int b = a + 1; b < 3; ++b) {
      const cpx<T> u = m[a][b], v = m[b][a];
      m[a][b] = conj(v);
      m[b][a] = conj(u);
    }
  }
}

// A_{s mu}(x): V_mu(x) for s = +1, V_mu(x - mu)^dag for s = -1 (Vs: V as
// structure of arrays, word mu * 9 + e)
template <class S, class T>
__device__ __forceinline__ void hop_link(const Geom& g, const typename S::word* __restrict__ Vs, const int (&x)[4],
                                         int mu, int s, cpx<T> (&a)[3][3]) {
  int p[4] = {x[0], x[1], x[2], x[3]};
  if (s < 0) p[mu] = wrap(p[mu] - 1, g.n[mu]);
  soa_load<S, T>(Vs + size_t(mu) * 9 * g.vol, g.vol, site_of(g, p), a);
  if (s < 0) dagger_in_place(a);
}

// W_{dd}(x) for any dd != 0 from W as structure of arrays (stored, or
// W_{-dd}(x + dd)^dag), 1 for dd = 0
template <class S, class T>
__device__ __forceinline__ void soa_w_any(const Geom& g, const typename S::word* __restrict__ Ws, const int (&x)[4],
                                          const int (&dd)[4], cpx<T> (&w)[3][3]) {
  const int n = (dd[0] + 1) + 3 * (dd[1] + 1) + 9 * (dd[2] + 1) + 27 * (dd[3] + 1);
  if (n == 40) {
    m3_identity(w);
  } else if (n > 40) {
    soa_load<S, T>(Ws + size_t(n - 41) * 9 * g.vol, g.vol, site_of(g, x), w);
  } else {
    int y[4];
#pragma unroll
    for (int mu = 0; mu < 4; ++mu) y[mu] = wrap(x[mu] + dd[mu], g.n[mu]);
    soa_load<S, T>(Ws + size_t(39 - n) * 9 * g.vol, g.vol, site_of(g, y), w);
    dagger_in_place(w);
  }
}

// blockIdx.x -> (unit u in [0, n), site block sb in [0, nsb8)), nsb8 the
// number of site blocks rounded up to a multiple of 8.  Workgroups go to the
// eight XCDs in turn, so the n units of one site block are placed on the same
// XCD one after another and share its L2 (the neighbours they gather).
DSL_HD void xcd_units(uint32_t b, int n, uint32_t& u, uint32_t& sb) {
  const uint32_t xcd = b & 7u, q = b >> 3;
  u = q % uint32_t(n);
  sb = (q / uint32_t(n)) * 8u + xcd;
}

DSL_HD int dir_code(const int (&d)[4]) { return (d[0] + 1) + 3 * (d[1] + 1) + 9 * (d[2] + 1) + 27 * (d[3] + 1); }

// T_e for the stored directions of level L < 4 (thread per (site, slot of
// the level)), in place in Ts: the slot starts as grad_W and receives the
// level-(L + 1) totals, which no thread of this launch writes.
template <class S, class T>
__global__ void __launch_bounds__(128) bri_wlevel_kernel(Geom g, LevelSlots ls, int L,
                                                         const typename S::word* __restrict__ Vs,
                                                         typename S::word* Ts) {
  uint32_t u, sbk;
  xcd_units(blockIdx.x, ls.n, u, sbk);
  const uint32_t xs = sbk * blockDim.x + threadIdx.x;
  if (xs >= g.vol) return;
  const int jt = ls.j[u];  // uniform over the block
  const uint32_t vol = g.vol;
  int e[4];
  stored_direction(jt, e);
  const SiteNbr nb = site_nbr(g, xs);
  const int xp[4] = {nb.c[0], nb.c[1], nb.c[2], nb.c[3]};
  const T w = T(1) / T(L + 1);
  cpx<T> h[3][3];
  soa_load<S, T>(Ts + size_t(jt) * 9 * vol, vol, xs, h);
#pragma unroll 1
  for (int mu = 0; mu < 4; ++mu) {
    if (e[mu] != 0) continue;
#pragma unroll 1
    for (int s = 1; s >= -1; s -= 2) {
      cpx<T> a[3][3], tm[3][3], r[3][3];
      int d[4] = {e[0], e[1], e[2], e[3]};
      d[mu] = s;
      int n = dir_code(d);
      if (n > 40) {  // d = e + s mu stored, at x = x' - s mu
        int x[4] = {xp[0], xp[1], xp[2], xp[3]};
        x[mu] = wrap(x[mu] - s, g.n[mu]);
        hop_link<S, T>(g, Vs, x, mu, s, a);
        soa_load<S, T>(Ts + size_t(n - 41) * 9 * vol, vol, site_of(g, x), tm);
        m3_adj_mul(a, tm, r);  // A^dag T_d
#pragma unroll
        for (int i = 0; i < 3; ++i)
#pragma unroll
          for (int c = 0; c < 3; ++c) h[i][c] = rmadd(h[i][c], w, r[i][c]);
      }
#pragma unroll
      for (int nu = 0; nu < 4; ++nu) d[nu] = nu == mu ? s : -e[nu];
      n = dir_code(d);
      if (n > 40) {  // d = -e + s mu stored, at x = x' - d
        int x[4];
#pragma unroll
        for (int nu = 0; nu < 4; ++nu) x[nu] = wrap(xp[nu] - d[nu], g.n[nu]);
        hop_link<S, T>(g, Vs, x, mu, s, a);
        soa_load<S, T>(Ts + size_t(n - 41) * 9 * vol, vol, site_of(g, x), tm);
        m3_adj_mul(tm, a, r);  // T_d^dag A
#pragma unroll
        for (int i = 0; i < 3; ++i)
#pragma unroll
          for (int c = 0; c < 3; ++c) h[i][c] = rmadd(h[i][c], w, r[i][c]);
      }
    }
  }
  typename S::word* o = Ts + size_t(jt) * 9 * vol + xs;
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int c = 0; c < 3; ++c) S::template store<T>(o + size_t(i * 3 + c) * vol, h[i][c]);
}

// G_V from the totals Ts (all 40 slots) and W as structure of arrays
template <class S, class T>
__global__ void __launch_bounds__(128) bri_wlevel_gv_kernel(Geom g, const typename S::word* __restrict__ Ws,
                                                            const typename S::word* __restrict__ Ts,
                                                            typename S::word* __restrict__ GV) {
  uint32_t u, sbk;
  xcd_units(blockIdx.x, 4, u, sbk);
  const uint32_t y = sbk * blockDim.x + threadIdx.x;
  const int mu = int(u);  // uniform over the block
  if (y >= g.vol) return;
  const uint32_t vol = g.vol;
  const SiteNbr nb = site_nbr(g, y);
  const int yc[4] = {nb.c[0], nb.c[1], nb.c[2], nb.c[3]};
  int yp[4] = {yc[0], yc[1], yc[2], yc[3]};
  yp[mu] = wrap(yp[mu] + 1, g.n[mu]);
  const uint32_t syp = site_of(g, yp);
  cpx<T> acc[3][3];
#pragma unroll
  for (int r = 0; r < 3; ++r)
#pragma unroll
    for (int c = 0; c < 3; ++c) acc[r][c] = zero<T>();
#pragma unroll 1
  for (int j = 0; j < 40; ++j) {
    int d[4];
    stored_direction(j, d);
    const int s = d[mu];
    if (s == 0) continue;  // uniform: j and mu are the same for the whole wave
    const int k = (d[0] != 0) + (d[1] != 0) + (d[2] != 0) + (d[3] != 0);
    const T w = T(1) / T(k);
    cpx<T> tm[3][3], ws[3][3], r[3][3];
    int sub[4] = {d[0], d[1], d[2], d[3]};
    sub[mu] = 0;
    if (s > 0) {
      // A = V_mu(y), the rest of the path from y + mu
      soa_load<S, T>(Ts + size_t(j) * 9 * vol, vol, y, tm);
      soa_w_any<S, T>(g, Ws, yp, sub, ws);
      m3_mul_adj(tm, ws, r);
#pragma unroll
      for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int c = 0; c < 3; ++c) acc[i][c] = rmadd(acc[i][c], w, r[i][c]);
    } else {
      // A = V_mu(y)^dag as the first hop from y + mu, the rest from y
      soa_load<S, T>(Ts + size_t(j) * 9 * vol, vol, syp, tm);
      soa_w_any<S, T>(g, Ws, yc, sub, ws);
      m3_mul_adj(tm, ws, r);
#pragma unroll
      for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int c = 0; c < 3; ++c) acc[i][c] = rmadd(acc[i][c], w, conj(r[c][i]));
    }
  }
  typename S::word* o = GV + (size_t(y) * 4 + mu) * 9;
#pragma unroll
  for (int r = 0; r < 3; ++r)
#pragma unroll
    for (int c = 0; c < 3; ++c) S::template store<T>(o + r * 3 + c, acc[r][c]);
}

// ---------------------------------------------------------------- W by levels
// The same first-hop recursion builds W (Tab. 1) level by level: the stored
// directions with k hops read those with k - 1 hops, stored or as the adjoint
// of a stored one at the shifted site, from W itself (one launch per level),
// so a k-hop direction costs k products instead of k! (k - 1) for the walks
// over every ordering.  Level 1 is V_mu itself.
template <class S, class T>
__global__ void __launch_bounds__(128) bri_links_level_kernel(Geom g, LevelSlots ls, int L,
                                                              const typename S::word* __restrict__ V,
                                                              typename S::word* W) {
  uint32_t u, sbk;
  xcd_units(blockIdx.x, ls.n, u, sbk);
  const uint32_t xs = sbk * blockDim.x + threadIdx.x;
  if (xs >= g.vol) return;
  const int jt = ls.j[u];  // uniform over the block
  int d[4];
  stored_direction(jt, d);
  const SiteNbr nb = site_nbr(g, xs);
  const int x[4] = {nb.c[0], nb.c[1], nb.c[2], nb.c[3]};
  cpx<T> acc[3][3];
#pragma unroll
  for (int r = 0; r < 3; ++r)
#pragma unroll
    for (int c = 0; c < 3; ++c) acc[r][c] = zero<T>();
#pragma unroll 1
  for (int mu = 0; mu < 4; ++mu) {
    const int s = d[mu];
    if (s == 0) continue;  // uniform over the block
    // A_{s mu}(x); path_hop leaves p at x + s mu, where the rest of the path starts
    int p[4] = {x[0], x[1], x[2], x[3]};
    cpx<T> a[3][3];
    path_hop<S, T>(g, V, p, mu, s, a);
    if (L == 1) {
#pragma unroll
      for (int r = 0; r < 3; ++r)
#pragma unroll
        for (int c = 0; c < 3; ++c) acc[r][c] = acc[r][c] + a[r][c];
    } else {
      int sub[4] = {d[0], d[1], d[2], d[3]};
      sub[mu] = 0;
      cpx<T> w[3][3], r3[3][3];
      load_w_any<S, T>(g, W, p, sub, w);
      path_mul(a, w, r3);
#pragma unroll
      for (int r = 0; r < 3; ++r)
#pragma unroll
        for (int c = 0; c < 3; ++c) acc[r][c] = acc[r][c] + r3[r][c];
    }
  }
  const T inv = T(1) / T(L);
  typename S::word* o = W + (size_t(xs) * 40 + jt) * 9;
#pragma unroll
  for (int r = 0; r < 3; ++r)
#pragma unroll
    for (int c = 0; c < 3; ++c) S::template store<T>(o + r * 3 + c, inv * acc[r][c]);
}

}  // namespace

namespace {

template <class S, class T>
hipError_t wgrad_t(const Geom& g, const void* chi, const void* psi, void* GW, hipStream_t st) {
  using W = typename S::word;
  const int vb = g.nv < 16 ? g.nv : 16;
  const int sb = 256 / vb;
  const dim3 block(vb, sb), grid((g.vol + sb - 1) / sb, 40);
  const size_t lds = size_t(sb) * 18 * vb * sizeof(T);
  hipLaunchKernelGGL((bri_wgrad_kernel<S, T>), grid, block, lds, st, g, (const W*)chi, (const W*)psi, (W*)GW);
  return hipGetLastError();
}

template <class S, class T>
hipError_t links_backward_t(const Geom& g, const void* V, const void* Wl, const void* GW, void* GV, hipStream_t st) {
  using W = typename S::word;
  const dim3 block(128), grid((g.vol + 127) / 128, 4);
  if (Wl)
    hipLaunchKernelGGL((bri_links_backward_w_kernel<S, T>), grid, block, 0, st, g, (const W*)Wl, (const W*)GW,
                       (W*)GV);
  else
    hipLaunchKernelGGL((bri_links_backward_kernel<S, T>), grid, block, 0, st, g, (const W*)V, (const W*)GW, (W*)GV);
  return hipGetLastError();
}

}  // namespace

hipError_t launch_brillouin_wgrad(int dtype, const Geom& g, const void* chi, const void* psi, void* GW,
                                  hipStream_t st) {
  const hipError_t e = launch_brillouin_wgrad_rows(dtype, g, chi, psi, GW, st);
  if (e != hipErrorNotSupported || knobs().rows.get(1) == 2) return e;
  switch (dtype) {
    case DT_C64: return wgrad_t<C64, float>(g, chi, psi, GW, st);
    case DT_C128: return wgrad_t<C128, double>(g, chi, psi, GW, st);
  }
  return hipErrorInvalidValue;
}

namespace {

template <class S, class T>
hipError_t links_backward_levels_t(const Geom& g, const void* V, const void* Wl, const void* GW, void* GV, void* ws,
                                   hipStream_t st) {
  using W = typename S::word;
  const uint32_t vol = g.vol;
  W* Ts = (W*)ws;                      // totals, 40 slots
  W* Ws = Ts + size_t(360) * vol;      // W, 40 slots
  W* Vs = Ws + size_t(360) * vol;      // V, 4 links
  // G_W, W and V as structures of arrays
  const int tile_words = 5760 * 8 / int(sizeof(W));
  const struct { const void* src; W* dst; int wps; } cp[3] = {{GW, Ts, 360}, {Wl, Ws, 360}, {V, Vs, 36}};
  for (const auto& c : cp) {
    const int sb = tile_words / c.wps;
    const size_t lds = size_t(sb) * (c.wps + 1) * sizeof(W);
    if (aligned16(c.src))
      hipLaunchKernelGGL((bri_aos_to_soa_kernel<S, true>), dim3((vol + sb - 1) / sb), dim3(kSoaBlock), lds, st,
                         (const W*)c.src, c.dst, vol, c.wps, sb);
    else
      hipLaunchKernelGGL((bri_aos_to_soa_kernel<S, false>), dim3((vol + sb - 1) / sb), dim3(kSoaBlock), lds, st,
                         (const W*)c.src, c.dst, vol, c.wps, sb);
    if (hipError_t e = hipGetLastError()) return e;
  }
  const uint32_t blocks8 = ((vol + 127) / 128 + 7) / 8 * 8;
  // levels 3, 2, 1: each adds what the level above passes down to its slots
  for (int L = 3; L >= 1; --L) {
    LevelSlots ls{};
    for (int j = 0; j < 40; ++j) {
      int d[4];
      stored_direction(j, d);
      if ((d[0] != 0) + (d[1] != 0) + (d[2] != 0) + (d[3] != 0) == L) ls.j[ls.n++] = j;
    }
    hipLaunchKernelGGL((bri_wlevel_kernel<S, T>), dim3(blocks8 * uint32_t(ls.n)), dim3(128), 0, st, g, ls, L,
                       (const W*)Vs, Ts);
    if (hipError_t e = hipGetLastError()) return e;
  }
  hipLaunchKernelGGL((bri_wlevel_gv_kernel<S, T>), dim3(blocks8 * 4), dim3(128), 0, st, g, (const W*)Ws, (const W*)Ts,
                     (W*)GV);
  return hipGetLastError();
}

}  // namespace

namespace {

template <class S, class T>
hipError_t links_levels_t(const Geom& g, const void* V, void* Wout, hipStream_t st) {
  using W = typename S::word;
  const uint32_t blocks8 = ((g.vol + 127) / 128 + 7) / 8 * 8;
  for (int L = 1; L <= 4; ++L) {
    LevelSlots ls{};
    for (int j = 0; j < 40; ++j) {
      int d[4];
      stored_direction(j, d);
      if ((d[0] != 0) + (d[1] != 0) + (d[2] != 0) + (d[3] != 0) == L) ls.j[ls.n++] = j;
    }
    hipLaunchKernelGGL((bri_links_level_kernel<S, T>), dim3(blocks8 * uint32_t(ls.n)), dim3(128), 0, st, g, ls, L,
                       (const W*)V, (W*)Wout);
    if (hipError_t e = hipGetLastError()) return e;
  }
  return hipSuccess;
}

}  // namespace

hipError_t launch_brillouin_links_levels(int dtype, const Geom& g, const void* V, void* W, hipStream_t st) {
  switch (dtype) {
    case DT_C64: return links_levels_t<C64, float>(g, V, W, st);
    case DT_C128: return links_levels_t<C128, double>(g, V, W, st);
  }
  return hipErrorInvalidValue;
}

hipError_t launch_brillouin_links_backward_levels(int dtype, const Geom& g, const void* V, const void* W,
                                                  const void* GW, void* GV, void* Tw, hipStream_t st) {
  switch (dtype) {
    case DT_C64: return links_backward_levels_t<C64, float>(g, V, W, GW, GV, Tw, st);
    case DT_C128: return links_backward_levels_t<C128, double>(g, V, W, GW, GV, Tw, st);
  }
  return hipErrorInvalidValue;
}

hipError_t launch_brillouin_links_backward(int dtype, const Geom& g, const void* V, const void* W, const void* GW,
                                           void* GV, hipStream_t st) {
  switch (dtype) {
    case DT_C64: return links_backward_t<C64, float>(g, V, W, GW, GV, st);
    case DT_C128: return links_backward_t<C128, double>(g, V, W, GW, GV, st);
  }
  return hipErrorInvalidValue;
}

}  // namespace dsl
