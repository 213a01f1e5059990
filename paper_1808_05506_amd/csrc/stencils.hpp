// Per-thread bodies of the three Dirac stencils.
//
// One thread owns one (site, right-hand side) pair and accumulates every
// contribution to that output in registers, then writes it once -- the
// thread-private "site" accumulator of Sec. 2, here one per GPU lane.  The
// right-hand-side index is the fastest lane index, so for a fixed spin and
// colour the lanes of one site read N_v consecutive complex numbers and every
// lane of a site reads the same link (one cache line serves them all).
//
// Spin structure uses the chiral basis gamma_mu = [[0, A_mu], [A_mu^dag, 0]]
// with A_k = -i sigma_k and A_4 = 1.  For c = +-1,
//   (1 + c gamma_mu) psi = [h ; c A_mu^dag h],  h = psi_up + c A_mu psi_low,
// so a hop needs only the 2-spinor h (rank-2 projector of eq. def_wils).
#pragma once

#include "dslash_common.hpp"

namespace dsl {

template <int C, class T> DSL_HD cpx<T> cs(cpx<T> a) { return C > 0 ? a : -a; }            // c * a
template <int C, class T> DSL_HD cpx<T> ci(cpx<T> a) { return C > 0 ? times_i(a) : times_mi(a); }  // c i a

template <class S, class T>
DSL_HD void load_link(const typename S::word* __restrict__ U, size_t base, cpx<T> (&u)[3][3]) {
#pragma unroll
  for (int a = 0; a < 3; ++a)
#pragma unroll
    for (int b = 0; b < 3; ++b) u[a][b] = S::template load<T>(U + base + a * 3 + b);
}

// Third row of an SU(3) matrix from its first two (unitarity and det u = 1):
// u_2j = conj(u_0k u_1l - u_0l u_1k), (j, k, l) a cyclic permutation of (0, 1, 2).
template <class T>
DSL_HD void complete_su3(cpx<T> (&u)[3][3]) {
#pragma unroll
  for (int j = 0; j < 3; ++j) {
    const int k = (j + 1) % 3, l = (j + 2) % 3;
    cpx<T> z = cmadd(zero<T>(), u[0][k], u[1][l]);
    z = cmadd(z, -u[0][l], u[1][k]);
    u[2][j] = conj(z);
  }
}

// A link of LW storage words at p: 9 (the full matrix) or 6 (gauge
// compression: its first two rows, the third completed as above).
template <int LW, class S, class T>
DSL_HD void load_link_lw(const typename S::word* p, cpx<T> (&u)[3][3]) {
  static_assert(LW == 9 || LW == 6, "a link is stored in 9 or 6 words");
#pragma unroll
  for (int a = 0; a < LW / 3; ++a)
#pragma unroll
    for (int b = 0; b < 3; ++b) u[a][b] = S::template load<T>(p + a * 3 + b);
  if constexpr (LW == 6) complete_su3(u);
}

template <class S, class T>
DSL_HD void load_wspinor(const typename S::word* __restrict__ in, size_t base, int nv, cpx<T> (&p)[4][3]) {
#pragma unroll
  for (int sp = 0; sp < 4; ++sp)
#pragma unroll
    for (int c = 0; c < 3; ++c) p[sp][c] = S::template load<T>(in + base + size_t(sp * 3 + c) * nv);
}

// ---------------------------------------------------------------- clover term
// res += C(x) p for the site-local clover term -(c_SW/2) sum_{mu<nu} sigma_{mu nu}
// F_{mu nu}(x) of eqs. def_wils / def_bril.  In the chiral basis it is block
// diagonal: block b acts on spins 2b, 2b+1, row index 3 s' + c.  Each block is
// Hermitian and stored in 18 complex words: words 0..2 hold the real diagonal
// pairwise, (H_00, H_11), (H_22, H_33), (H_44, H_55); words 3..17 the upper
// triangle H_ij (i < j) row by row.  C points at the site's 36 words.
template <class S, class T>
DSL_HD void clover_madd(const typename S::word* C, const cpx<T> (&p)[4][3], cpx<T> (&res)[4][3]) {
#pragma unroll
  for (int b = 0; b < 2; ++b) {
    const typename S::word* h = C + 18 * b;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      const cpx<T> d = S::template load<T>(h + k);
      const int i0 = 2 * k, i1 = 2 * k + 1;
      res[2 * b + i0 / 3][i0 % 3] = rmadd(res[2 * b + i0 / 3][i0 % 3], d.r, p[2 * b + i0 / 3][i0 % 3]);
      res[2 * b + i1 / 3][i1 % 3] = rmadd(res[2 * b + i1 / 3][i1 % 3], d.i, p[2 * b + i1 / 3][i1 % 3]);
    }
    int w = 3;
#pragma unroll
    for (int i = 0; i < 6; ++i)
#pragma unroll
      for (int j = i + 1; j < 6; ++j, ++w) {
        const cpx<T> hij = S::template load<T>(h + w);
        cpx<T>& ri = res[2 * b + i / 3][i % 3];
        cpx<T>& rj = res[2 * b + j / 3][j % 3];
        ri = cmadd(ri, hij, p[2 * b + j / 3][j % 3]);
        rj = cjmadd(rj, hij, p[2 * b + i / 3][i % 3]);
      }
  }
}

// out(x) = diag in(x) + ca acc (+ C(x) in(x) if C is given) for one (site, rhs)
// of the direct kernels.
template <class S, class T>
DSL_HD void site_finish(const typename S::word* __restrict__ in, typename S::word* __restrict__ out,
                        const typename S::word* __restrict__ C, uint32_t s, size_t base, int nv, T diag, T ca,
                        const cpx<T> (&acc)[4][3]) {
  cpx<T> p[4][3], res[4][3];
#pragma unroll
  for (int sp = 0; sp < 4; ++sp)
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      p[sp][c] = S::template load<T>(in + base + size_t(sp * 3 + c) * nv);
      res[sp][c].r = fma(diag, p[sp][c].r, ca * acc[sp][c].r);
      res[sp][c].i = fma(diag, p[sp][c].i, ca * acc[sp][c].i);
    }
  if (C) clover_madd<S, T>(C + size_t(s) * 36, p, res);
#pragma unroll
  for (int sp = 0; sp < 4; ++sp)
#pragma unroll
    for (int c = 0; c < 3; ++c) S::template store<T>(out + base + size_t(sp * 3 + c) * nv, res[sp][c]);
}

// h = psi_up + c A_mu psi_low
template <int MU, int C, class T>
DSL_HD void project(const cpx<T> (&p)[4][3], cpx<T> (&h)[2][3]) {
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    if (MU == 0) {        // A_1 = [[0,-i],[-i,0]]
      h[0][c] = p[0][c] - ci<C>(p[3][c]);
      h[1][c] = p[1][c] - ci<C>(p[2][c]);
    } else if (MU == 1) { // A_2 = [[0,-1],[1,0]]
      h[0][c] = p[0][c] - cs<C>(p[3][c]);
      h[1][c] = p[1][c] + cs<C>(p[2][c]);
    } else if (MU == 2) { // A_3 = [[-i,0],[0,i]]
      h[0][c] = p[0][c] - ci<C>(p[2][c]);
      h[1][c] = p[1][c] + ci<C>(p[3][c]);
    } else {              // A_4 = 1
      h[0][c] = p[0][c] + cs<C>(p[2][c]);
      h[1][c] = p[1][c] + cs<C>(p[3][c]);
    }
  }
}

// acc += [t ; c A_mu^dag t]
template <int MU, int C, class T>
DSL_HD void reconstruct_add(cpx<T> (&acc)[4][3], const cpx<T> (&t)[2][3]) {
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    acc[0][c] += t[0][c];
    acc[1][c] += t[1][c];
    if (MU == 0) {        // A_1^dag = [[0,i],[i,0]]
      acc[2][c] += ci<C>(t[1][c]);
      acc[3][c] += ci<C>(t[0][c]);
    } else if (MU == 1) { // A_2^dag = [[0,1],[-1,0]]
      acc[2][c] += cs<C>(t[1][c]);
      acc[3][c] -= cs<C>(t[0][c]);
    } else if (MU == 2) { // A_3^dag = [[i,0],[0,-i]]
      acc[2][c] += ci<C>(t[0][c]);
      acc[3][c] -= ci<C>(t[1][c]);
    } else {              // A_4^dag = 1
      acc[2][c] += cs<C>(t[0][c]);
      acc[3][c] += cs<C>(t[1][c]);
    }
  }
}

// t[s] = u h[s]  (DAG = false)  or  u^dag h[s]  (DAG = true), s = 0, 1
template <bool DAG, class T>
DSL_HD void su3_mul2(const cpx<T> (&u)[3][3], const cpx<T> (&h)[2][3], cpx<T> (&t)[2][3]) {
#pragma unroll
  for (int s = 0; s < 2; ++s)
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      cpx<T> r = zero<T>();
#pragma unroll
      for (int b = 0; b < 3; ++b) r = DAG ? cjmadd(r, u[b][a], h[s][b]) : cmadd(r, u[a][b], h[s][b]);
      t[s][a] = r;
    }
}

// One Wilson hop: acc += (1 + c gamma_mu) U' psi(n), U' = U or U^dag.
template <int MU, int C, bool DAG, class S, class T, int LW = 9>
DSL_HD void wilson_hop(const typename S::word* __restrict__ U, const typename S::word* __restrict__ in,
                       size_t link_base, size_t spin_base, int nv, cpx<T> (&acc)[4][3]) {
  cpx<T> p[4][3];
  load_wspinor<S, T>(in, spin_base, nv, p);
  cpx<T> h[2][3];
  project<MU, C, T>(p, h);
  cpx<T> u[3][3];
  load_link_lw<LW, S, T>(U + link_base, u);
  cpx<T> t[2][3];
  su3_mul2<DAG, T>(u, h, t);
  reconstruct_add<MU, C, T>(acc, t);
}

// D_W at c_SW = 0 (eq. def_wils) in hop form:
//   out(x) = (4 + m0) in(x) - 1/2 sum_mu [(1 - gamma_mu) V_mu(x) in(x+mu)
//                                       + (1 + gamma_mu) V_mu(x-mu)^dag in(x-mu)]
// ADJ: gamma_5 D_W gamma_5, i.e. gamma_mu -> -gamma_mu.  LW: words per stored
// link (9, or 6 for compressed links).
template <bool ADJ, class S, class T, int LW = 9, int NVC = 0>
DSL_HD void wilson_site(const Geom& g, const typename S::word* __restrict__ U,
                        const typename S::word* __restrict__ in, typename S::word* __restrict__ out,
                        const typename S::word* __restrict__ C, uint32_t s, const SiteNbr& nb, int v, T diag) {
  constexpr int CF = ADJ ? +1 : -1;  // forward projector 1 + CF gamma
  constexpr int CB = -CF;            // backward projector 1 + CB gamma
  const int nv = NVC ? NVC : g.nv;   // NVC: N_v known at compile time
  const size_t sps = size_t(12) * nv;  // complex numbers per site of a spinor block
  cpx<T> acc[4][3];
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int c = 0; c < 3; ++c) acc[a][c] = zero<T>();

  const uint32_t sf0 = s + nb.fwd[0], sb0 = s + nb.bwd[0];
  const uint32_t sf1 = s + nb.fwd[1], sb1 = s + nb.bwd[1];
  const uint32_t sf2 = s + nb.fwd[2], sb2 = s + nb.bwd[2];
  const uint32_t sf3 = s + nb.fwd[3], sb3 = s + nb.bwd[3];
  wilson_hop<0, CF, false, S, T, LW>(U, in, (size_t(s) * 4 + 0) * LW, sf0 * sps + v, nv, acc);
  wilson_hop<0, CB, true, S, T, LW>(U, in, (size_t(sb0) * 4 + 0) * LW, sb0 * sps + v, nv, acc);
  wilson_hop<1, CF, false, S, T, LW>(U, in, (size_t(s) * 4 + 1) * LW, sf1 * sps + v, nv, acc);
  wilson_hop<1, CB, true, S, T, LW>(U, in, (size_t(sb1) * 4 + 1) * LW, sb1 * sps + v, nv, acc);
  wilson_hop<2, CF, false, S, T, LW>(U, in, (size_t(s) * 4 + 2) * LW, sf2 * sps + v, nv, acc);
  wilson_hop<2, CB, true, S, T, LW>(U, in, (size_t(sb2) * 4 + 2) * LW, sb2 * sps + v, nv, acc);
  wilson_hop<3, CF, false, S, T, LW>(U, in, (size_t(s) * 4 + 3) * LW, sf3 * sps + v, nv, acc);
  wilson_hop<3, CB, true, S, T, LW>(U, in, (size_t(sb3) * 4 + 3) * LW, sb3 * sps + v, nv, acc);

  site_finish<S, T>(in, out, C, s, size_t(s) * sps + v, nv, diag, T(-0.5), acc);
}

// D_S (Sec. 3): out(x) = m in(x) + sum_mu eta_mu(x)/2 [V_mu(x) in(x+mu) - V_mu(x-mu)^dag in(x-mu)],
// eta_1 = 1, eta_2 = (-1)^x, eta_3 = (-1)^(x+y), eta_4 = (-1)^(x+y+z).  ADJ negates the hop term.
template <bool ADJ, class S, class T, int LW = 9, int NVC = 0>
DSL_HD void staggered_site(const Geom& g, const typename S::word* __restrict__ U,
                           const typename S::word* __restrict__ in, typename S::word* __restrict__ out,
                           uint32_t s, const SiteNbr& nb, int v, T mass) {
  const int nv = NVC ? NVC : g.nv;  // NVC: N_v known at compile time
  const size_t sps = size_t(3) * nv;
  cpx<T> acc[3] = {zero<T>(), zero<T>(), zero<T>()};
  int par = 0;  // x_1 + ... + x_{mu-1}
#pragma unroll
  for (int mu = 0; mu < 4; ++mu) {
    const T eta = (par & 1) ? T(-1) : T(1);
    par += nb.c[mu];
    const uint32_t sf = s + nb.fwd[mu], sb = s + nb.bwd[mu];
    cpx<T> u[3][3], ub[3][3], pf[3], pb[3];
    load_link_lw<LW, S, T>(U + (size_t(s) * 4 + mu) * LW, u);
    load_link_lw<LW, S, T>(U + (size_t(sb) * 4 + mu) * LW, ub);
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      pf[c] = S::template load<T>(in + size_t(sf) * sps + size_t(c) * nv + v);
      pb[c] = S::template load<T>(in + size_t(sb) * sps + size_t(c) * nv + v);
    }
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      cpx<T> t = zero<T>();
#pragma unroll
      for (int b = 0; b < 3; ++b) t = cmadd(t, u[a][b], pf[b]);
      cpx<T> tb = zero<T>();
#pragma unroll
      for (int b = 0; b < 3; ++b) tb = cjmadd(tb, ub[b][a], pb[b]);
      acc[a] = rmadd(acc[a], eta, t - tb);
    }
  }
  const T half = ADJ ? T(-0.5) : T(0.5);
  const size_t base = size_t(s) * sps + v;
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    const size_t e = base + size_t(c) * nv;
    cpx<T> p = S::template load<T>(in + e);
    cpx<T> o;
    o.r = fma(mass, p.r, half * acc[c].r);
    o.i = fma(mass, p.i, half * acc[c].i);
    S::template store<T>(out + e, o);
  }
}

// ---------------------------------------------------------------- Brillouin
// Direction of stored slot j (Tab. 1 caption): n = j + 41 = sum_mu (d_mu + 1) 3^mu.
DSL_HD void stored_direction(int j, int (&d)[4]) {
  int n = j + 41;
  d[0] = n % 3 - 1;
  d[1] = (n / 3) % 3 - 1;
  d[2] = (n / 9) % 3 - 1;
  d[3] = n / 27 - 1;
}

// Coefficients printed after eq. def_lap: rho_k = (64,16,4,1)/432, lambda_k = (-240,8,4,2,1)/64.
template <class T> DSL_HD T bri_rho(int k) {
  return k == 1 ? T(64.0 / 432.0) : k == 2 ? T(16.0 / 432.0) : k == 3 ? T(4.0 / 432.0) : T(1.0 / 432.0);
}
template <class T> DSL_HD T bri_lambda(int k) {
  return k == 0 ? T(-240.0 / 64.0) : k == 1 ? T(8.0 / 64.0) : k == 2 ? T(4.0 / 64.0) : k == 3 ? T(2.0 / 64.0) : T(1.0 / 64.0);
}

// t[s] = w p[s] (DAG false) or w^dag p[s] (DAG true), all four spins
template <bool DAG, class T>
DSL_HD void su3_mul4(const cpx<T> (&w)[3][3], const cpx<T> (&p)[4][3], cpx<T> (&t)[4][3]) {
#pragma unroll
  for (int s = 0; s < 4; ++s)
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      cpx<T> r = zero<T>();
#pragma unroll
      for (int b = 0; b < 3; ++b) r = DAG ? cjmadd(r, w[b][a], p[s][b]) : cmadd(r, w[a][b], p[s][b]);
      t[s][a] = r;
    }
}

// (alpha + i beta) * y added to acc
// acc + i beta y
template <class T> DSL_HD cpx<T> cmadd_i(cpx<T> acc, T beta, cpx<T> y) {
  acc.r = fma(-beta, y.i, acc.r);
  acc.i = fma(beta, y.r, acc.i);
  return acc;
}

template <class T> DSL_HD cpx<T> cmadd_ab(cpx<T> acc, T alpha, T beta, cpx<T> y) {
  acc.r = fma(alpha, y.r, acc.r);
  acc.r = fma(-beta, y.i, acc.r);
  acc.i = fma(alpha, y.i, acc.i);
  acc.i = fma(beta, y.r, acc.i);
  return acc;
}

// D_B at c_SW = 0 (eqs. def_bril, def_der, def_lap), hop form:
//   out(x) = (m0 - lambda_0/2) in(x) + sum_{d != 0} [-lambda_k/2 + rho_k d.gamma] W_d(x) in(x+d)
// taken over pairs (d, -d) of one stored slot j:  W_d(x) is stored at x,
// W_{-d}(x) = W_d(x-d)^dag is read at x-d.  With chi_+- the two products,
//   a (chi_+ + chi_-) + b (d.gamma)(chi_+ - chi_-),  a = -lambda_k/2, b = rho_k,
// and d.gamma = [[0, S], [S^dag, 0]], S = sum_mu d_mu A_mu
//   = [[d4 - i d3, -d2 - i d1], [d2 - i d1, d4 + i d3]].
// ADJ: gamma_5 D_B gamma_5, i.e. b -> -b.
template <bool ADJ, class S, class T>
DSL_HD void brillouin_site(const Geom& g, const typename S::word* __restrict__ W,
                           const typename S::word* __restrict__ in, typename S::word* __restrict__ out,
                           const typename S::word* __restrict__ C, uint32_t s, const SiteNbr& nb, int v, T diag) {
  const int nv = g.nv;
  const size_t sps = size_t(12) * nv;
  cpx<T> acc[4][3];
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int c = 0; c < 3; ++c) acc[a][c] = zero<T>();

#pragma unroll 1
  for (int j = 0; j < 40; ++j) {
    int d[4];
    stored_direction(j, d);
    int offp = 0, offm = 0, k = 0;
#pragma unroll
    for (int mu = 0; mu < 4; ++mu) {
      offp += d[mu] > 0 ? nb.fwd[mu] : (d[mu] < 0 ? nb.bwd[mu] : 0);
      offm += d[mu] > 0 ? nb.bwd[mu] : (d[mu] < 0 ? nb.fwd[mu] : 0);
      k += d[mu] != 0;
    }
    const uint32_t sp = s + offp, sm = s + offm;
    const T a = T(-0.5) * bri_lambda<T>(k);
    const T b = (ADJ ? T(-1) : T(1)) * bri_rho<T>(k);
    const T B1 = b * T(d[0]), B2 = b * T(d[1]), B3 = b * T(d[2]), B4 = b * T(d[3]);

    cpx<T> chi_p[4][3], chi_m[4][3];
    {
      cpx<T> w[3][3], p[4][3];
      load_link<S, T>(W, (size_t(s) * 40 + j) * 9, w);
      load_wspinor<S, T>(in, size_t(sp) * sps + v, nv, p);
      su3_mul4<false, T>(w, p, chi_p);
    }
    {
      cpx<T> w[3][3], p[4][3];
      load_link<S, T>(W, (size_t(sm) * 40 + j) * 9, w);
      load_wspinor<S, T>(in, size_t(sm) * sps + v, nv, p);
      su3_mul4<true, T>(w, p, chi_m);
    }
    // a (chi_+ + chi_-) + b (d.gamma)(chi_+ - chi_-); with S = sum_mu d_mu s_mu
    // (s_k = -i sigma_k, s_4 = 1) the upper spins take S y_low and the lower
    // ones S^dag y_up.  Each axis contributes only if d_mu != 0: the test is
    // uniform over the wave (one direction per iteration for every lane), so
    // the k-hop directions pay for k axes, not four.
    cpx<T> y[4][3];
#pragma unroll
    for (int q = 0; q < 4; ++q)
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        acc[q][c] = rmadd(acc[q][c], a, chi_p[q][c] + chi_m[q][c]);
        y[q][c] = chi_p[q][c] - chi_m[q][c];
      }
    if (d[3] != 0) {  // s_4 = 1
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        acc[0][c] = rmadd(acc[0][c], B4, y[2][c]);
        acc[1][c] = rmadd(acc[1][c], B4, y[3][c]);
        acc[2][c] = rmadd(acc[2][c], B4, y[0][c]);
        acc[3][c] = rmadd(acc[3][c], B4, y[1][c]);
      }
    }
    if (d[2] != 0) {  // s_3 = diag(-i, i)
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        acc[0][c] = cmadd_i(acc[0][c], -B3, y[2][c]);
        acc[1][c] = cmadd_i(acc[1][c], B3, y[3][c]);
        acc[2][c] = cmadd_i(acc[2][c], B3, y[0][c]);
        acc[3][c] = cmadd_i(acc[3][c], -B3, y[1][c]);
      }
    }
    if (d[1] != 0) {  // s_2 = [[0, -1], [1, 0]]
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        acc[0][c] = rmadd(acc[0][c], -B2, y[3][c]);
        acc[1][c] = rmadd(acc[1][c], B2, y[2][c]);
        acc[2][c] = rmadd(acc[2][c], B2, y[1][c]);
        acc[3][c] = rmadd(acc[3][c], -B2, y[0][c]);
      }
    }
    if (d[0] != 0) {  // s_1 = [[0, -i], [-i, 0]]
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        acc[0][c] = cmadd_i(acc[0][c], -B1, y[3][c]);
        acc[1][c] = cmadd_i(acc[1][c], -B1, y[2][c]);
        acc[2][c] = cmadd_i(acc[2][c], B1, y[1][c]);
        acc[3][c] = cmadd_i(acc[3][c], B1, y[0][c]);
      }
    }
  }
  site_finish<S, T>(in, out, C, s, size_t(s) * sps + v, nv, diag, T(1), acc);
}

// ---------------------------------------------------------------- W build
// W_d(x) (Tab. 1) is the mean over the k! orderings of the hops of d of the
// ordered product V_{e1}(x) V_{e2}(x+e1) ..., V_{-mu}(y) = V_mu(y-mu)^dag.

// Link of the hop sg * mu from pos (V_mu(pos), or V_mu(pos - mu)^dag); pos
// moves to the end of the hop.
template <class S, class T>
DSL_HD void path_hop(const Geom& g, const typename S::word* __restrict__ V, int (&pos)[4], int mu, int sg,
                     cpx<T> (&l)[3][3]) {
  if (sg < 0) pos[mu] = pos[mu] == 0 ? g.n[mu] - 1 : pos[mu] - 1;
  const uint32_t ls = uint32_t(pos[0] + g.stride[1] * pos[1] + g.stride[2] * pos[2] + g.stride[3] * pos[3]);
  load_link<S, T>(V, (size_t(ls) * 4 + mu) * 9, l);
  if (sg < 0) {
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
      for (int b = a; b < 3; ++b) {
        const cpx<T> x1 = l[a][b], y1 = l[b][a];
        l[a][b] = conj(y1);
        l[b][a] = conj(x1);
      }
  } else {
    pos[mu] = pos[mu] + 1 == g.n[mu] ? 0 : pos[mu] + 1;
  }
}

template <class T>
DSL_HD void path_mul(const cpx<T> (&a)[3][3], const cpx<T> (&b)[3][3], cpx<T> (&r)[3][3]) {
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      cpx<T> z = zero<T>();
#pragma unroll
      for (int c = 0; c < 3; ++c) z = cmadd(z, a[i][c], b[c][j]);
      r[i][j] = z;
    }
}

// The sum of the path products of W_d(x) over the (k - 1)! orderings that
// begin with hop number `first` of d (0 <= first < k; nothing otherwise),
// each shared prefix multiplied once (15 products for k = 4 instead of 18),
// in the fixed order of the remaining hops; returns k!.
template <class S, class T>
DSL_HD int brillouin_path_tree_sum(const Geom& g, const typename S::word* __restrict__ V, const int (&x)[4],
                                   const int (&d)[4], int first, cpx<T> (&acc)[3][3]) {
  int mus[4], sgn[4], k = 0;
#pragma unroll
  for (int mu = 0; mu < 4; ++mu)
    if (d[mu] != 0) {
      mus[k] = mu;
      sgn[k] = d[mu];
      ++k;
    }
#pragma unroll
  for (int a = 0; a < 3; ++a)
#pragma unroll
    for (int b = 0; b < 3; ++b) acc[a][b] = zero<T>();
  const int kfact = k == 4 ? 24 : (k == 3 ? 6 : (k == 2 ? 2 : 1));
  if (first >= k) return kfact;
  int p1[4] = {x[0], x[1], x[2], x[3]};
  cpx<T> a1[3][3];
  path_hop<S, T>(g, V, p1, mus[first], sgn[first], a1);
  if (k == 1) {
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
      for (int b = 0; b < 3; ++b) acc[a][b] = a1[a][b];
    return kfact;
  }
#pragma unroll 1
  for (int i2 = 0; i2 < k; ++i2) {
    if (i2 == first) continue;
    int p2[4] = {p1[0], p1[1], p1[2], p1[3]};
    cpx<T> l[3][3], m2[3][3];
    path_hop<S, T>(g, V, p2, mus[i2], sgn[i2], l);
    path_mul(a1, l, m2);
    if (k == 2) {
#pragma unroll
      for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int b = 0; b < 3; ++b) acc[a][b] += m2[a][b];
      continue;
    }
#pragma unroll 1
    for (int i3 = 0; i3 < k; ++i3) {
      if (i3 == first || i3 == i2) continue;
      int p3[4] = {p2[0], p2[1], p2[2], p2[3]};
      cpx<T> m3[3][3];
      path_hop<S, T>(g, V, p3, mus[i3], sgn[i3], l);
      path_mul(m2, l, m3);
      if (k == 4) {
        // the one hop left: 0 + 1 + 2 + 3 = 6
        const int i4 = 6 - first - i2 - i3;
        cpx<T> m4[3][3];
        path_hop<S, T>(g, V, p3, mus[i4], sgn[i4], l);
        path_mul(m3, l, m4);
#pragma unroll
        for (int a = 0; a < 3; ++a)
#pragma unroll
          for (int b = 0; b < 3; ++b) acc[a][b] += m4[a][b];
      } else {
#pragma unroll
        for (int a = 0; a < 3; ++a)
#pragma unroll
          for (int b = 0; b < 3; ++b) acc[a][b] += m3[a][b];
      }
    }
  }
  return kfact;
}

}  // namespace dsl
