// Clover term of D_W and D_B (setup kernel): per site the packed Hermitian
// blocks of -(c_SW/2) sum_{mu<nu} sigma_{mu nu} F_{mu nu}(x) (eqs. def_wils,
// def_bril), with the clover-leaf field strength
//   F_{mu nu}(x) = (Q_{mu nu}(x) - Q_{mu nu}(x)^dag) / (8 i),
// Q the sum of the four plaquettes of the (mu, nu) plane that start and end at
// x, all run in the same sense, and sigma_{mu nu} = (i/2) [gamma_mu, gamma_nu].
//
// In the chiral basis gamma_k = [[0, -i s_k], [i s_k, 0]], gamma_4 = [[0, 1], [1, 0]]
// (s_k the Pauli matrices; index 0..3 = the paper's 1..4):
//   sigma_{jk} = -eps_{jkl} diag(s_l, s_l),  sigma_{k4} = diag(s_k, -s_k),
// so block b (spins 2b, 2b+1; + for b = 0, - for b = 1) of the sum is
//   s_1 (x) E_1 + s_2 (x) E_2 + s_3 (x) E_3 = [[E_3, E_1 - i E_2], [E_1 + i E_2, -E_3]]
// with E_1 = -F_23 +- F_14, E_2 = F_13 +- F_24, E_3 = -F_12 +- F_34 (1-based).
// The storage of a block (18 complex words: the real diagonal pairwise, then
// the upper triangle row by row) is the one clover_madd reads.
#include "launch.hpp"
#include "stencils.hpp"

namespace dsl {
namespace {

template <class T>
DSL_HD void m3_mul(const cpx<T> (&a)[3][3], const cpx<T> (&b)[3][3], cpx<T> (&r)[3][3]) {
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      cpx<T> z = zero<T>();
#pragma unroll
      for (int k = 0; k < 3; ++k) z = cmadd(z, a[i][k], b[k][j]);
      r[i][j] = z;
    }
}

// Link of the hop from pos to pos + sg mu (V_mu(pos), or V_mu(pos - mu)^dag
// for sg < 0); pos moves along.
template <class S, class T>
DSL_HD void hop_link(const Geom& g, const typename S::word* __restrict__ V, int (&pos)[4], int mu, int sg,
                     cpx<T> (&l)[3][3]) {
  if (sg < 0) pos[mu] = pos[mu] == 0 ? g.n[mu] - 1 : pos[mu] - 1;
  const uint32_t s = uint32_t(pos[0] + g.stride[1] * pos[1] + g.stride[2] * pos[2] + g.stride[3] * pos[3]);
  load_link<S, T>(V, (size_t(s) * 4 + mu) * 9, l);
  if (sg < 0) {
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
      for (int b = a; b < 3; ++b) {
        const cpx<T> x = l[a][b], y = l[b][a];
        l[a][b] = conj(y);
        l[b][a] = conj(x);
      }
  } else {
    pos[mu] = pos[mu] + 1 == g.n[mu] ? 0 : pos[mu] + 1;
  }
}

// q += product of the links along x -> x+a -> x+a+b -> x+b -> x, a = sa mu, b = sb nu
template <class S, class T>
DSL_HD void add_plaquette(const Geom& g, const typename S::word* __restrict__ V, const int (&x)[4], int mu, int sa,
                          int nu, int sb, cpx<T> (&q)[3][3]) {
  int pos[4] = {x[0], x[1], x[2], x[3]};
  cpx<T> m[3][3], l[3][3], r[3][3];
  hop_link<S, T>(g, V, pos, mu, sa, m);
  hop_link<S, T>(g, V, pos, nu, sb, l);
  m3_mul(m, l, r);
  hop_link<S, T>(g, V, pos, mu, -sa, l);
  m3_mul(r, l, m);
  hop_link<S, T>(g, V, pos, nu, -sb, l);
  m3_mul(m, l, r);
#pragma unroll
  for (int a = 0; a < 3; ++a)
#pragma unroll
    for (int b = 0; b < 3; ++b) q[a][b] += r[a][b];
}

// dst += c F for a complex factor c in {+-1, +-i} (CR, CI: real and imaginary part)
template <int CR, int CI, class T>
DSL_HD void add_scaled(cpx<T> (&dst)[3][3], const cpx<T> (&f)[3][3]) {
#pragma unroll
  for (int a = 0; a < 3; ++a)
#pragma unroll
    for (int b = 0; b < 3; ++b) {
      if (CR > 0) dst[a][b] += f[a][b];
      if (CR < 0) dst[a][b] -= f[a][b];
      if (CI > 0) dst[a][b] += times_i(f[a][b]);
      if (CI < 0) dst[a][b] += times_mi(f[a][b]);
    }
}

}  // namespace

template <class S, class T>
__global__ void __launch_bounds__(128) clover_field_kernel(Geom g, const typename S::word* __restrict__ V,
                                                          typename S::word* __restrict__ C, T coef) {
  const uint32_t s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= g.vol) return;
  const SiteNbr nb = site_nbr(g, s);
  const int x[4] = {nb.c[0], nb.c[1], nb.c[2], nb.c[3]};
  // E3[b] and K[b] = E1 - i E2 of block b
  cpx<T> E3[2][3][3], K[2][3][3];
#pragma unroll
  for (int b = 0; b < 2; ++b)
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
      for (int j = 0; j < 3; ++j) E3[b][i][j] = K[b][i][j] = zero<T>();

#pragma unroll 1
  for (int p = 0; p < 6; ++p) {
    // planes (0,1) (0,2) (0,3) (1,2) (1,3) (2,3)
    const int mu = p < 3 ? 0 : (p < 5 ? 1 : 2);
    const int nu = p < 3 ? p + 1 : (p < 5 ? p - 1 : 3);
    cpx<T> q[3][3];
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
      for (int b = 0; b < 3; ++b) q[a][b] = zero<T>();
    add_plaquette<S, T>(g, V, x, mu, +1, nu, +1, q);
    add_plaquette<S, T>(g, V, x, nu, +1, mu, -1, q);
    add_plaquette<S, T>(g, V, x, mu, -1, nu, -1, q);
    add_plaquette<S, T>(g, V, x, nu, -1, mu, +1, q);
    // F = (q - q^dag) / (8 i) = -i (q - q^dag) / 8
    cpx<T> f[3][3];
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
      for (int b = 0; b < 3; ++b) f[a][b] = T(0.125) * times_mi(q[a][b] - conj(q[b][a]));
    switch (p) {
      case 0:  // F_12: E3 -= F in both blocks
        add_scaled<-1, 0>(E3[0], f);
        add_scaled<-1, 0>(E3[1], f);
        break;
      case 1:  // F_13: E2 += F in both blocks, K -= i F
        add_scaled<0, -1>(K[0], f);
        add_scaled<0, -1>(K[1], f);
        break;
      case 2:  // F_14: E1 +- F
        add_scaled<1, 0>(K[0], f);
        add_scaled<-1, 0>(K[1], f);
        break;
      case 3:  // F_23: E1 -= F in both blocks
        add_scaled<-1, 0>(K[0], f);
        add_scaled<-1, 0>(K[1], f);
        break;
      case 4:  // F_24: E2 +- F, K -+ i F
        add_scaled<0, -1>(K[0], f);
        add_scaled<0, 1>(K[1], f);
        break;
      default:  // F_34: E3 +- F
        add_scaled<1, 0>(E3[0], f);
        add_scaled<-1, 0>(E3[1], f);
        break;
    }
  }

  typename S::word* out = C + size_t(s) * 36;
#pragma unroll
  for (int b = 0; b < 2; ++b) {
    typename S::word* h = out + 18 * b;
    S::template store<T>(h + 0, mk(coef * E3[b][0][0].r, coef * E3[b][1][1].r));
    S::template store<T>(h + 1, mk(coef * E3[b][2][2].r, -coef * E3[b][0][0].r));
    S::template store<T>(h + 2, mk(-coef * E3[b][1][1].r, -coef * E3[b][2][2].r));
    int w = 3;
#pragma unroll
    for (int i = 0; i < 6; ++i)
#pragma unroll
      for (int j = i + 1; j < 6; ++j, ++w) {
        cpx<T> z;
        if (j < 3)
          z = E3[b][i][j];
        else if (i < 3)
          z = K[b][i][j - 3];
        else
          z = -E3[b][i - 3][j - 3];
        S::template store<T>(h + w, coef * z);
      }
  }
}

namespace {

template <class S, class T>
hipError_t clover_field_t(const Geom& g, const void* V, void* C, double c_sw, hipStream_t st) {
  using W = typename S::word;
  const dim3 block(128), grid((g.vol + 127) / 128);
  hipLaunchKernelGGL((clover_field_kernel<S, T>), grid, block, 0, st, g, (const W*)V, (W*)C, T(-0.5 * c_sw));
  return hipGetLastError();
}

}  // namespace

hipError_t launch_clover_field(int dtype, const Geom& g, const void* V, void* C, double c_sw, hipStream_t st) {
  switch (dtype) {
    case DT_C64: return clover_field_t<C64, float>(g, V, C, c_sw, st);
    case DT_C128: return clover_field_t<C128, double>(g, V, C, c_sw, st);
    case DT_BF16: return clover_field_t<BF16, float>(g, V, C, c_sw, st);
    case DT_F16: return clover_field_t<F16, float>(g, V, C, c_sw, st);
  }
  return hipErrorInvalidValue;
}

}  // namespace dsl
